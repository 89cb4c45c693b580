// Device helpers shared by the vector kernels and the batched serving kernels:
// wavefront/workgroup reductions and the lattice E^T sum at one node.
#pragma once

#include "internal.h"

namespace pafem {
namespace vec {

constexpr int kThreads = 256;
constexpr int kWave = 64;
constexpr int kMaxBlocks = 2048;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Sum over the workgroup of NV values per thread; results valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (&out)[NV]) {
  __shared__ double s[NV][kThreads / kWave];
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double w = wave_sum(v[k]);
    if (lane == 0) s[k][wid] = w;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double acc = 0;
      for (int i = 0; i < kThreads / kWave; ++i) acc += s[k][i];
      out[k] = acc;
    }
  }
}

// Elements (and local index) containing lattice coordinate I along one
// direction with n elements of order p: two at an interior element face.
__device__ __forceinline__ int lattice_cands(int I, int n, int p, int (&e)[2], int (&l)[2]) {
  if (I % p == 0 && I > 0 && I < n * p) {
    e[0] = I / p - 1;
    l[0] = p;
    e[1] = I / p;
    l[1] = 0;
    return 2;
  }
  int ee = I / p;
  if (ee > n - 1) ee = n - 1;
  e[0] = e[1] = ee;  // the second entry repeats the first (always a valid position)
  l[0] = l[1] = I - ee * p;
  return 1;
}

// Sum `ncols` (at most 4) interleaved columns of partials[nb][ncols] in a
// fixed order; a workgroup of kThreads threads calls it, results in thread 0.
// Each thread keeps four independent running sums over its fixed strided
// subset (so several loads are in flight), then wavefront shuffles and one
// pass over the per-wavefront sums combine them.
__device__ __forceinline__ void final_sums(const double* partials, int nb, int ncols,
                                           double* out) {
  __shared__ double s[4][kThreads / kWave];
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  for (int c = 0; c < ncols; ++c) {
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    int i = threadIdx.x;
    for (; i + 3 * kThreads < nb; i += 4 * kThreads) {
      a0 += partials[(int64_t)i * ncols + c];
      a1 += partials[(int64_t)(i + kThreads) * ncols + c];
      a2 += partials[(int64_t)(i + 2 * kThreads) * ncols + c];
      a3 += partials[(int64_t)(i + 3 * kThreads) * ncols + c];
    }
    for (; i < nb; i += kThreads) a0 += partials[(int64_t)i * ncols + c];
    const double w = wave_sum((a0 + a1) + (a2 + a3));
    if (lane == 0) s[c][wid] = w;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int c = 0; c < ncols; ++c) {
      double acc = 0;
      for (int k = 0; k < kThreads / kWave; ++k) acc += s[c][k];
      out[c] = acc;
    }
}

// E^T at lattice node (I, J, K): the sum of its element contributions in the
// E-vector (element-major, or x-interleaved when XROWS) in ascending
// (element, local node) order (the order of the stored map's CSR sum, so the
// forms agree bitwise); constrained essential rows take x[i] (or 0).  The up
// to eight contributions are loaded together.
// PC > 0 fixes the order at compile time (divisions by a constant).
template <typename T, bool XROWS = false, int PC = 0>
__device__ __forceinline__ void gather_lattice_ijk(const T* __restrict__ yE, int nx, int ny,
                                                   int nz, int p_rt, int constrained,
                                                   int accumulate, const T* __restrict__ x,
                                                   T* __restrict__ y, int I, int J, int K) {
  const int p = PC > 0 ? PC : p_rt;
  const int Lx = nx * p + 1, Ly = ny * p + 1, Lz = nz * p + 1;
  const int64_t i = I + (int64_t)Lx * (J + (int64_t)Ly * K);
  T acc = 0;
  const bool ess = I == 0 || I == Lx - 1 || J == 0 || J == Ly - 1 || K == 0 || K == Lz - 1;
  if (constrained && ess) {
    acc = x ? x[i] : T(0);
  } else {
    const int n = p + 1, nloc = n * n * n;  // ne (p+1)^3 < 2^31
    int ex[2], lx[2], ey[2], ly[2], ez[2], lz[2];
    const int cx = lattice_cands(I, nx, p, ex, lx);
    const int cy = lattice_cands(J, ny, p, ey, ly);
    const int cz = lattice_cands(K, nz, p, ez, lz);
    T v[8];
    // ascending element number: z outermost, x innermost
#pragma unroll
    for (int kz = 0; kz < 2; ++kz)
#pragma unroll
      for (int ky = 0; ky < 2; ++ky)
#pragma unroll
        for (int kx = 0; kx < 2; ++kx) {
          const int k = 4 * kz + 2 * ky + kx;
          const bool on = kz < cz && ky < cy && kx < cx;
          const int off = XROWS ? xrows_index(nx, ny, n, ex[kx], ey[ky], ez[kz], lx[kx], ly[ky], lz[kz])
                                : (ex[kx] + nx * (ey[ky] + ny * ez[kz])) * nloc + lx[kx] +
                                      n * (ly[ky] + n * lz[kz]);
          v[k] = on ? yE[off] : T(0);
        }
#pragma unroll
    for (int kz = 0; kz < 2; ++kz)
#pragma unroll
      for (int ky = 0; ky < 2; ++ky)
#pragma unroll
        for (int kx = 0; kx < 2; ++kx)
          if (kz < cz && ky < cy && kx < cx) acc += v[4 * kz + 2 * ky + kx];
  }
  y[i] = accumulate ? y[i] + acc : acc;
}

// The same at linear lattice index i (below the node count, < 2^31).
template <typename T, bool XROWS = false, int PC = 0>
__device__ __forceinline__ void gather_lattice_node(const T* __restrict__ yE, int nx, int ny,
                                                    int nz, int p_rt, int constrained,
                                                    int accumulate, const T* __restrict__ x,
                                                    T* __restrict__ y, int64_t i) {
  const int p = PC > 0 ? PC : p_rt;
  const int Lx = nx * p + 1, Ly = ny * p + 1;
  const int ii = (int)i, r = ii / Lx;
  gather_lattice_ijk<T, XROWS, PC>(yE, nx, ny, nz, p, constrained, accumulate, x, y,
                                   ii - r * Lx, r % Ly, r / Ly);
}

}  // namespace vec
}  // namespace pafem
