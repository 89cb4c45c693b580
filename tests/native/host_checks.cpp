// Host-code checks run under AddressSanitizer and UndefinedBehaviorSanitizer
// (built with g++ by tests/test_host_sanitizers.py; no GPU): the 1D node,
// quadrature and basis tables, the lattice maps, the multiply-high division
// and the x-interleaved E-vector layout, over every order and a set of mesh
// shapes.  Any out-of-bounds access or undefined operation aborts; a failed
// invariant returns 1.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../paper_2402_15940_amd/csrc/internal.h"

using namespace pafem;

static int failures = 0;
#define CHECK(cond)                                                            \
  do {                                                                         \
    if (!(cond)) {                                                             \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
      ++failures;                                                              \
    }                                                                          \
  } while (0)

static void tables() {
  for (int p = 1; p <= kMaxP; ++p) {
    const int n = p + 1;
    std::vector<double> nd(n);
    gll_nodes(p, nd.data());
    CHECK(std::fabs(nd[0]) < 1e-15 && std::fabs(nd[n - 1] - 1.0) < 1e-15);
    for (int i = 0; i + 1 < n; ++i) CHECK(nd[i] < nd[i + 1]);
    for (int i = 0; i < n; ++i) CHECK(std::fabs(nd[i] + nd[n - 1 - i] - 1.0) < 1e-14);
    for (int q = 1; q <= 12; ++q) {
      std::vector<double> x(q), w(q), B(q * n), G(q * n);
      gauss_legendre(q, x.data(), w.data());
      double sw = 0.0;
      for (int i = 0; i < q; ++i) sw += w[i];
      CHECK(std::fabs(sw - 1.0) < 1e-14);
      lagrange_tables(n, nd.data(), q, x.data(), B.data(), G.data());
      for (int i = 0; i < q; ++i) {
        double sb = 0.0, sg = 0.0;
        for (int a = 0; a < n; ++a) {
          sb += B[i * n + a];
          sg += G[i * n + a];
        }
        CHECK(std::fabs(sb - 1.0) < 1e-12 && std::fabs(sg) < 1e-9);
      }
    }
  }
}

static void maps(int nx, int ny, int nz, int p) {
  const int n = p + 1;
  const int64_t ne = (int64_t)nx * ny * nz;
  const int64_t nd = ((int64_t)nx * p + 1) * ((int64_t)ny * p + 1) * ((int64_t)nz * p + 1);
  std::vector<int32_t> E, off, idx, ess;
  std::vector<uint8_t> mask;
  build_restriction(nx, ny, nz, p, E);
  CHECK((int64_t)E.size() == ne * n * n * n);
  std::vector<int> count(nd, 0);
  for (int32_t g : E) {
    CHECK(g >= 0 && g < nd);
    if (g >= 0 && g < nd) ++count[g];
  }
  for (int64_t i = 0; i < nd; ++i) CHECK(count[i] >= 1 && count[i] <= 8);
  build_restriction_transpose(E, nd, off, idx);
  CHECK((int64_t)off.size() == nd + 1 && off[0] == 0 && off[nd] == (int32_t)E.size());
  for (int64_t i = 0; i < nd; ++i) {
    CHECK(off[i + 1] - off[i] == count[i]);
    for (int32_t k = off[i]; k < off[i + 1]; ++k) {
      CHECK(idx[k] >= 0 && idx[k] < (int32_t)E.size());
      if (idx[k] >= 0 && idx[k] < (int32_t)E.size()) CHECK(E[idx[k]] == i);
      if (k > off[i]) CHECK(idx[k - 1] < idx[k]);
    }
  }
  build_essential(nx, ny, nz, p, ess, mask);
  const int64_t interior = ((int64_t)nx * p - 1) * ((int64_t)ny * p - 1) * ((int64_t)nz * p - 1);
  CHECK((int64_t)ess.size() == nd - interior && (int64_t)mask.size() == nd);
  for (size_t k = 0; k < ess.size(); ++k) {
    CHECK(ess[k] >= 0 && ess[k] < nd && mask[ess[k]] == 1);
    if (k) CHECK(ess[k - 1] < ess[k]);
  }
  // x-interleaved layout: a bijection onto [0, evec_words) when unpadded
  const int64_t words = evec_words(ne, n);
  std::vector<uint8_t> seen(words, 0);
  for (int ez = 0; ez < nz; ++ez)
    for (int ey = 0; ey < ny; ++ey)
      for (int ex = 0; ex < nx; ++ex)
        for (int c = 0; c < n; ++c)
          for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) {
              const int o = xrows_index(nx, ny, n, ex, ey, ez, a, b, c);
              CHECK(o >= 0 && o < words);
              if (o >= 0 && o < words) {
                CHECK(seen[o] == 0);
                seen[o] = 1;
              }
            }
}

static void division() {
  const int ns[] = {0, 1, 2, 3, 7, 255, 256, 65535, 65536, 1 << 20, 123456789, 0x3fffffff,
                    0x7ffffffe, 0x7fffffff};
  for (int d = 2; d <= 4096; ++d) {
    const FastDiv f(d);
    for (int v : ns) CHECK(f.div(v) == v / d);
    for (int k = 1; k < 64; ++k) {
      const long long v = (long long)d * (k * 33331 % 65521) - 1;
      if (v >= 0 && v <= 0x7fffffff) CHECK(f.div((int)v) == (int)(v / d));
    }
  }
  const int big[] = {100001, 1 << 24, 536870913, 0x7fffffff};
  for (int d : big) {
    const FastDiv f(d);
    for (int v : ns) CHECK(f.div(v) == v / d);
  }
}

int main() {
  tables();
  const int meshes[][3] = {{1, 1, 1}, {3, 2, 1}, {2, 3, 4}, {5, 1, 2}};
  for (int p = 1; p <= kMaxP; ++p)
    for (const auto& m : meshes) maps(m[0], m[1], m[2], p);
  division();
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("host checks passed\n");
  return 0;
}
