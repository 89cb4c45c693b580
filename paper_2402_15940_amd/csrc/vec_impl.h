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

// E^T from the x-interleaved E-vector, one thread per kXRowsNodes nodes:
// workgroup b takes the kXRowsNodes * kThreads consecutive lattice nodes from
// b kXRowsNodes kThreads on (lane t: nodes base + q kThreads + t), so every
// lane is busy and a wavefront may span the end of a lattice row.  Node
// I = ex p + a of row (J, K) reads word ex w + a of each (y, z) candidate's
// run (neighbouring lanes: neighbouring words) and, on an x face (a = 0,
// ex > 0), also the word of element ex-1's local p.  All loads of a thread
// are issued before its first sum.  Each node's sum runs in ascending
// (element, local node) order: for every (z, y) candidate in ascending order,
// element ex-1 before element ex (the order of the stored map's CSR sum, so
// the lattice and map forms agree bitwise).
//
// The row and plane of a node come from divisions by the lattice extents,
// fixed at launch (FastDiv: a multiply-high and a shift).  Along y (and z)
// the candidates of lattice coordinate J are the element ey = min(J / p,
// ny - 1) at local index ly = J - ey p and, when ly = 0 and ey > 0, also
// element ey - 1 at local index p; their runs sit N^2 - p runs apart (N (ny N
// - p) along z for the planes), so one base offset and two strides address
// all four (y, z) runs.  The y/z branches are uniform over a wavefront except
// where it crosses a row; the x-face word is loaded by every lane (the node's
// own word when it is not on an x face) and selected.
constexpr int kXRowsNodes = 2;

struct XRowsGeom {
  int nx, ny, nz;
  int Lx, Ly, Lz;
  FastDiv fLx, fLy;
  int64_t n;
};

inline XRowsGeom xrows_geom(int nx, int ny, int nz, int p) {
  XRowsGeom g;
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.Lx = nx * p + 1;
  g.Ly = ny * p + 1;
  g.Lz = nz * p + 1;
  g.fLx = FastDiv(g.Lx);
  g.fLy = FastDiv(g.Ly);
  g.n = (int64_t)g.Lx * g.Ly * g.Lz;
  return g;
}

// The loaded contributions of one node and what decides its sum.
template <typename T>
struct XRowsLoads {
  T v[4], w[4];  // (z, y) candidates 0: (right, right) 1: (right, left) 2: (left, right) 3: (left, left)
  bool hy, hz, xf, ess;
};

// One E-vector word: an ordinary or a non-temporal load (NT), as measured
// per operator and order.
template <bool NT, typename T>
__device__ __forceinline__ T evec_word(const T* __restrict__ p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

template <typename T, int P, bool NT = false>
__device__ __forceinline__ void xrows_load(const T* __restrict__ yX, const XRowsGeom& g, int i,
                                           XRowsLoads<T>& L) {
  constexpr int N = P + 1, W = xrows_width(N);
  const int row = g.fLx.div(i), I = i - row * g.Lx;
  const int K = g.fLy.div(row), J = row - K * g.Ly;
  int ex = I / P, a = I - ex * P;
  if (ex == g.nx) {  // the row's last node
    ex = g.nx - 1;
    a = P;
  }
  int ey = J / P, ez = K / P;
  ey = ey < g.ny - 1 ? ey : g.ny - 1;
  ez = ez < g.nz - 1 ? ez : g.nz - 1;
  const int ly = J - ey * P, lz = K - ez * P;
  L.hy = ly == 0 && ey > 0;
  L.hz = lz == 0 && ez > 0;
  L.xf = a == 0 && ex > 0;
  L.ess = I == 0 || I == g.Lx - 1 || J == 0 || J == g.Ly - 1 || K == 0 || K == g.Lz - 1;
  const int rowlen = g.nx * W;
  const int o = (((ez * g.ny + ey) * N + lz) * N + ly) * rowlen + ex * W + a;
  const int dy = (N * N - P) * rowlen, dz = N * (g.ny * N - P) * rowlen;
  const int left = L.xf ? P - W : 0;
  L.v[0] = evec_word<NT>(yX + o);
  L.w[0] = evec_word<NT>(yX + o + left);
  if (L.hy) {
    L.v[1] = evec_word<NT>(yX + o - dy);
    L.w[1] = evec_word<NT>(yX + o - dy + left);
  }
  if (L.hz) {
    L.v[2] = evec_word<NT>(yX + o - dz);
    L.w[2] = evec_word<NT>(yX + o - dz + left);
    if (L.hy) {
      L.v[3] = evec_word<NT>(yX + o - dz - dy);
      L.w[3] = evec_word<NT>(yX + o - dz - dy + left);
    }
  }
}

// Sum of the loaded contributions in ascending (element, local node) order.
template <typename T>
__device__ __forceinline__ T xrows_sum(const XRowsLoads<T>& L) {
  T acc = 0;
  if (L.hz) {
    if (L.hy) {
      if (L.xf) acc += L.w[3];
      acc += L.v[3];
    }
    if (L.xf) acc += L.w[2];
    acc += L.v[2];
  }
  if (L.hy) {
    if (L.xf) acc += L.w[1];
    acc += L.v[1];
  }
  if (L.xf) acc += L.w[0];
  acc += L.v[0];
  return acc;
}


}  // namespace vec
}  // namespace pafem
