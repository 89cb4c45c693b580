"""MI355X-native partial-assembly finite element library (HIP, gfx950)."""
