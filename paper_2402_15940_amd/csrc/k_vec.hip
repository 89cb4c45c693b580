// Vector kernels of the Jacobi-PCG solve, the deterministic E^T gather and
// fixed-order reductions.
//
// Reductions are two-stage and bitwise reproducible for a given length: a
// fixed grid of `reduce_blocks(n)` workgroups each folds a grid-stride slice,
// reduces across the 64-lane wavefront with cross-lane shuffles and across the
// workgroup's wavefronts through LDS, and writes one partial; a one-workgroup
// kernel then sums the partials in a fixed tree order.  CG scalars (alpha,
// beta, residual norms) never leave the device.
#include "vec_impl.h"

namespace pafem {

namespace {

using vec::kThreads;
using vec::kWave;
using vec::kMaxBlocks;
using vec::block_sum;
using vec::final_sums;

template <typename T>
__global__ __launch_bounds__(kThreads) void k_gather_et(const T* __restrict__ yE,
                                                        const int32_t* __restrict__ off,
                                                        const int32_t* __restrict__ idx,
                                                        const uint8_t* __restrict__ ess_mask,
                                                        int constrained, int accumulate,
                                                        const T* __restrict__ x,
                                                        T* __restrict__ y, int64_t n,
                                                        const int* skip) {
  if (skip != nullptr && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T acc = 0;
  if (constrained && ess_mask[i]) {
    acc = x ? x[i] : T(0);
  } else {
    const int32_t b = off[i], en = off[i + 1];
    for (int32_t k = b; k < en; ++k) acc += yE[idx[k]];
  }
  y[i] = accumulate ? y[i] + acc : acc;
}

// E^T of a full E-vector (element-major, or x-interleaved when XROWS) on the
// lattice numbering: one workgroup per (slice of a) lattice row (J, K), 32-bit
// index arithmetic (extents < 2^31).
template <typename T, bool XROWS>
__global__ __launch_bounds__(kThreads) void k_gather_lattice(const T* __restrict__ yE, int nx,
                                                             int ny, int nz, int p,
                                                             int constrained, int accumulate,
                                                             const T* __restrict__ x,
                                                             T* __restrict__ y, const int* skip) {
  if (skip != nullptr && *skip) return;
  const int Lx = nx * p + 1, Ly = ny * p + 1, rows = Ly * (nz * p + 1);
  const int I = blockIdx.x * kThreads + threadIdx.x;
  if (I >= Lx) return;
  for (int row = blockIdx.y; row < rows; row += gridDim.y)
    vec::gather_lattice_ijk<T, XROWS>(yE, nx, ny, nz, p, constrained, accumulate, x, y, I,
                                      row % Ly, row / Ly);
}

// E^T from the x-interleaved E-vector (node mapping, loads and summation
// order in vec_impl.h: xrows_load, xrows_sum).
using vec::kXRowsNodes;
using vec::XRowsGeom;
using vec::XRowsLoads;
using vec::xrows_geom;
using vec::xrows_load;
using vec::xrows_sum;

template <typename T, int P, bool NT, bool NTY>
__global__ __launch_bounds__(kThreads) void k_gather_xrows(const T* __restrict__ yX, XRowsGeom g,
                                                           int constrained, int accumulate,
                                                           const T* __restrict__ x,
                                                           T* __restrict__ y, const int* skip) {
  constexpr int R = kXRowsNodes;
  if (skip != nullptr && *skip) return;
  const int64_t base = (int64_t)blockIdx.x * (kThreads * R) + threadIdx.x;
  XRowsLoads<T> L[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int64_t iq = base + q * kThreads;
    xrows_load<T, P, NT>(yX, g, (int)(iq < g.n ? iq : g.n - 1), L[q]);
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int64_t i = base + q * kThreads;
    if (i >= g.n) break;
    T acc;
    if (constrained && L[q].ess)
      acc = x ? x[i] : T(0);
    else
      acc = xrows_sum(L[q]);
    const T yi = accumulate ? y[i] + acc : acc;
    if constexpr (NTY)
      __builtin_nontemporal_store(yi, y + i);
    else
      y[i] = yi;
  }
}

// One CG step fused into the ordered E^T sum of the x-interleaved E-vector
// of A p (the node mapping and summation order of k_gather_xrows, p_i on
// essential rows): x_i += alpha p_i, r_i -= alpha (A p)_i, z_i = dinv_i r_i,
// and each workgroup's partials of (r . z, r . r).  A p never goes through
// memory.  A capped grid strides over the chunks of nodes; TX is the type of
// the solution (FP64 for mixed CG).
template <typename T, typename TX, int P, bool NT>
__global__ __launch_bounds__(kThreads) void k_gather_xrows_cg(
    const T* __restrict__ yX, XRowsGeom g, const T* __restrict__ p, TX* __restrict__ x,
    T* __restrict__ r, const T* __restrict__ dinv, double* __restrict__ partials,
    const CgState* __restrict__ st) {
  constexpr int R = kXRowsNodes;
  if (st->done) return;
  const T alpha = (T)st->alpha;
  const double alpha_x = st->alpha;
  double v2[2] = {0.0, 0.0}, out[2];
  for (int64_t base = (int64_t)blockIdx.x * (kThreads * R) + threadIdx.x; base - threadIdx.x < g.n;
       base += (int64_t)gridDim.x * (kThreads * R)) {
    XRowsLoads<T> L[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int64_t iq = base + q * kThreads;
      xrows_load<T, P, NT>(yX, g, (int)(iq < g.n ? iq : g.n - 1), L[q]);
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int64_t i = base + q * kThreads;
      if (i >= g.n) break;
      const T pi = p[i];
      const T acc = L[q].ess ? pi : xrows_sum(L[q]);
      if constexpr (sizeof(TX) == sizeof(T))
        x[i] += alpha * pi;
      else
        x[i] += alpha_x * (TX)pi;
      const T ri = r[i] - alpha * acc;
      r[i] = ri;
      const T zi = dinv[i] * ri;
      v2[0] += (double)ri * (double)zi;
      v2[1] += (double)ri * (double)ri;
    }
  }
  block_sum<2>(v2, out);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = out[0];
    partials[2 * blockIdx.x + 1] = out[1];
  }
}

// alpha = r . z / p . Ap from many partials of p . Ap (one workgroup of 1024
// threads, fixed order: four running sums per thread, wavefront shuffles, one
// pass over the wavefront sums).
constexpr int kWideThreads = 1024;
__global__ __launch_bounds__(kWideThreads) void k_cg_alpha_wide(const double* __restrict__ partials,
                                                                 int nb, CgState* st) {
  if (st->done) return;
  __shared__ double sh[kWideThreads / 64];
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  int i = threadIdx.x;
  for (; i + 3 * kWideThreads < nb; i += 4 * kWideThreads) {
    a0 += partials[i];
    a1 += partials[i + kWideThreads];
    a2 += partials[i + 2 * kWideThreads];
    a3 += partials[i + 3 * kWideThreads];
  }
  for (; i < nb; i += kWideThreads) a0 += partials[i];
  const double w = vec::wave_sum((a0 + a1) + (a2 + a3));
  if (threadIdx.x % 64 == 0) sh[threadIdx.x / 64] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < kWideThreads / 64; ++k) t += sh[k];
    st->pAp = t;
    st->alpha = st->rz / t;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_set_ess(const int32_t* __restrict__ ess, int64_t n,
                                                      const T* __restrict__ x, T value,
                                                      int accumulate, T* __restrict__ y,
                                                      const int* skip) {
  if (skip != nullptr && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t g = ess[i];
  const T v = x ? x[g] : value;
  y[g] = accumulate ? y[g] + v : v;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_fill(T* __restrict__ y, int64_t n, T value,
                                                   const int* skip) {
  if (skip != nullptr && *skip) return;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    y[i] = value;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_dot_partial(const T* __restrict__ x,
                                                          const T* __restrict__ y, int64_t n,
                                                          double* __restrict__ partials,
                                                          const int* skip) {
  if (skip != nullptr && *skip) return;
  double v[1] = {0.0}, out[1];
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    v[0] += (double)x[i] * (double)y[i];
  block_sum<1>(v, out);
  if (threadIdx.x == 0) partials[blockIdx.x] = out[0];
}

__global__ __launch_bounds__(kThreads) void k_sum_final(const double* __restrict__ partials,
                                                        int nb, int ncols,
                                                        double* __restrict__ out) {
  double r[4];
  final_sums(partials, nb, ncols, r);
  if (threadIdx.x == 0)
    for (int c = 0; c < ncols; ++c) out[c] = r[c];
}

// ---- CG ------------------------------------------------------------------------

// p = dinv .* r; partials of (r . p, r . r)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cg_init(const T* __restrict__ r,
                                                      const T* __restrict__ dinv,
                                                      T* __restrict__ p, int64_t n,
                                                      double* __restrict__ partials) {
  double v[2] = {0.0, 0.0}, out[2];
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const T ri = r[i];
    const T zi = dinv[i] * ri;
    p[i] = zi;
    v[0] += (double)ri * (double)zi;
    v[1] += (double)ri * (double)ri;
  }
  block_sum<2>(v, out);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = out[0];
    partials[2 * blockIdx.x + 1] = out[1];
  }
}

__global__ void k_cg_init_final(const double* __restrict__ partials, int nb, double bb_host,
                                const double* __restrict__ bb_dev, double rtol, int maxit,
                                double delta2, CgState* st) {
  double r[4];
  final_sums(partials, nb, 2, r);
  if (threadIdx.x == 0) {
    const double bb = bb_dev != nullptr ? *bb_dev : bb_host;
    st->rz = r[0];
    st->rr = r[1];
    st->bb = bb;
    st->rr_stop = rtol * rtol * bb;
    st->pAp = st->alpha = st->beta = 0.0;
    st->iter = 0;
    st->maxit = maxit;
    st->done = (r[1] <= st->rr_stop) || maxit <= 0;
    st->rr_ref = r[1];
    st->delta2 = delta2;
    st->rz_prev = 0.0;
  }
}

__global__ void k_cg_alpha(const double* __restrict__ partials, int nb, CgState* st) {
  if (st->done) return;
  double r[4];
  final_sums(partials, nb, 1, r);
  if (threadIdx.x == 0) {
    st->pAp = r[0];
    st->alpha = st->rz / r[0];
  }
}

// x += alpha p; r -= alpha Ap; partials of (r . z, r . r) with z = dinv .* r.
// With a wider solution type TX (FP64 x, FP32 Krylov vectors) the solution is
// accumulated in TX with the FP64 alpha.
template <typename TX, typename T>
__global__ __launch_bounds__(kThreads) void k_cg_update(TX* __restrict__ x, T* __restrict__ r,
                                                        const T* __restrict__ p,
                                                        const T* __restrict__ Ap,
                                                        const T* __restrict__ dinv, int64_t n,
                                                        double* __restrict__ partials,
                                                        const CgState* __restrict__ st) {
  if (st->done) return;
  const T alpha = (T)st->alpha;
  const double alpha_x = st->alpha;
  double v[2] = {0.0, 0.0}, out[2];
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    if constexpr (sizeof(TX) == sizeof(T))
      x[i] += alpha * p[i];
    else
      x[i] += alpha_x * (TX)p[i];
    const T ri = r[i] - alpha * Ap[i];
    r[i] = ri;
    const T zi = dinv[i] * ri;
    v[0] += (double)ri * (double)zi;
    v[1] += (double)ri * (double)ri;
  }
  block_sum<2>(v, out);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = out[0];
    partials[2 * blockIdx.x + 1] = out[1];
  }
}

__global__ void k_cg_beta(const double* __restrict__ partials, int nb, CgState* st) {
  if (st->done) return;
  double r[4];
  final_sums(partials, nb, 2, r);
  if (threadIdx.x == 0) {
    st->rz_prev = st->rz;
    st->beta = r[0] / st->rz;
    st->rz = r[0];
    st->rr = r[1];
    st->iter += 1;
    // a residual that overflowed or became NaN ends the iteration (not converged)
    if (r[1] <= st->rr_stop || st->iter >= st->maxit || !isfinite(r[1]))
      st->done = 1;
    else if (st->delta2 > 0.0 && r[1] <= st->delta2 * st->rr_ref)
      st->done = 2;  // the recursive residual fell by delta: replace it by the true one
  }
}

// p = dinv .* r + beta p
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cg_pupdate(T* __restrict__ p,
                                                         const T* __restrict__ r,
                                                         const T* __restrict__ dinv, int64_t n,
                                                         const CgState* __restrict__ st) {
  if (st->done) return;
  const T beta = (T)st->beta;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    p[i] = dinv[i] * r[i] + beta * p[i];
}

// ---- mixed precision ------------------------------------------------------------

// Residual replacement of the mixed-precision CG: rs = (float) r64 with r64 =
// b - A x computed in FP64; partials of (rs . z, r64 . r64), z = dinv .* rs.
__global__ __launch_bounds__(kThreads) void k_replace_residual(const double* __restrict__ r64,
                                                               const float* __restrict__ dinv,
                                                               float* __restrict__ rs, int64_t n,
                                                               double* __restrict__ partials) {
  double v[2] = {0.0, 0.0}, out[2];
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const double ri = r64[i];
    const float rsi = (float)ri;
    rs[i] = rsi;
    v[0] += (double)rsi * (double)(dinv[i] * rsi);
    v[1] += ri * ri;
  }
  block_sum<2>(v, out);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = out[0];
    partials[2 * blockIdx.x + 1] = out[1];
  }
}

// After a replacement: beta from the new r . z and the r . z before the
// paused iteration, the true FP64 residual norm as rr and as the new
// reference; done when the true residual meets the tolerance (or maxit).
__global__ void k_replace_final(const double* __restrict__ partials, int nb, CgState* st) {
  double r[4];
  final_sums(partials, nb, 2, r);
  if (threadIdx.x == 0) {
    st->beta = st->rz_prev != 0.0 ? r[0] / st->rz_prev : 0.0;
    st->rz = r[0];
    st->rr = r[1];
    st->rr_ref = r[1];
    st->done = (r[1] <= st->rr_stop || st->iter >= st->maxit || !isfinite(r[1])) ? 1 : 0;
  }
}

__global__ __launch_bounds__(kThreads) void k_residual(const double* __restrict__ b,
                                                       const double* __restrict__ Ax,
                                                       double* __restrict__ r, int64_t n,
                                                       const int* __restrict__ skip) {
  if (skip != nullptr && *skip) return;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    r[i] = b[i] - Ax[i];
}

// r32 = r / ||r||  (norm2 holds ||r||^2)
__global__ __launch_bounds__(kThreads) void k_scale_to_f32(const double* __restrict__ r,
                                                           const double* __restrict__ norm2,
                                                           float* __restrict__ r32, int64_t n) {
  const double nr = sqrt(*norm2);
  const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    r32[i] = (float)(r[i] * inv);
}

// x += ||r|| d32
__global__ __launch_bounds__(kThreads) void k_axpy_from_f32(double* __restrict__ x,
                                                            const double* __restrict__ norm2,
                                                            const float* __restrict__ d32,
                                                            int64_t n) {
  const double nr = sqrt(*norm2);
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    x[i] += nr * (double)d32[i];
}

__global__ __launch_bounds__(kThreads) void k_recip(const double* __restrict__ d,
                                                    double* __restrict__ dinv64,
                                                    float* __restrict__ dinv32, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const double v = 1.0 / d[i];
    if (dinv64) dinv64[i] = v;
    if (dinv32) dinv32[i] = (float)v;
  }
}

inline int grid_for(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

int reduce_blocks(int64_t n) {
  int64_t b = (n + kThreads * 4 - 1) / (kThreads * 4);
  if (b > kMaxBlocks) b = kMaxBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

template <typename T>
hipError_t launch_gather_et(const T* yE, const int32_t* off, const int32_t* idx,
                            const uint8_t* ess_mask, int constrained, int accumulate, const T* x,
                            T* y, int64_t ndofs, const int* skip, hipStream_t s) {
  if (ndofs == 0) return hipSuccess;
  hipLaunchKernelGGL((k_gather_et<T>), dim3((ndofs + kThreads - 1) / kThreads), dim3(kThreads), 0,
                     s, yE, off, idx, ess_mask, constrained, accumulate, x, y, ndofs, skip);
  return hipGetLastError();
}
template hipError_t launch_gather_et<double>(const double*, const int32_t*, const int32_t*,
                                             const uint8_t*, int, int, const double*, double*,
                                             int64_t, const int*, hipStream_t);
template hipError_t launch_gather_et<float>(const float*, const int32_t*, const int32_t*,
                                            const uint8_t*, int, int, const float*, float*,
                                            int64_t, const int*, hipStream_t);

template <typename T, bool XROWS>
hipError_t gather_rows(const T* yE, int nx, int ny, int nz, int p, int constrained, int accumulate,
                       const T* x, T* y, const int* skip, hipStream_t s) {
  const int64_t Lx = (int64_t)nx * p + 1, Ly = (int64_t)ny * p + 1, Lz = (int64_t)nz * p + 1;
  if (nx <= 0 || ny <= 0 || nz <= 0) return hipSuccess;
  if (Lx * Ly * Lz > 0x7fffffff) return hipErrorInvalidValue;
  const int64_t rows = Ly * Lz;
  const dim3 grid((unsigned)((Lx + kThreads - 1) / kThreads),
                  (unsigned)(rows < 65535 ? rows : 65535));
  hipLaunchKernelGGL((k_gather_lattice<T, XROWS>), grid, dim3(kThreads), 0, s, yE, nx, ny, nz, p,
                     constrained, accumulate, x, y, skip);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather_lattice(const T* yE, int nx, int ny, int nz, int p, int constrained,
                                 int accumulate, const T* x, T* y, const int* skip,
                                 hipStream_t s) {
  return gather_rows<T, false>(yE, nx, ny, nz, p, constrained, accumulate, x, y, skip, s);
}
template <typename T, int P>
hipError_t gather_xrows_p(const T* yX, int nx, int ny, int nz, int constrained, int accumulate,
                          const T* x, T* y, const int* skip, hipStream_t s, bool nt, bool nt_y) {
  const int64_t nodes = ((int64_t)nx * P + 1) * ((int64_t)ny * P + 1) * ((int64_t)nz * P + 1);
  const int64_t per = (int64_t)kThreads * kXRowsNodes;
  const dim3 grid((unsigned)((nodes + per - 1) / per));
  const XRowsGeom g = xrows_geom(nx, ny, nz, P);
  if (nt && nt_y)
    hipLaunchKernelGGL((k_gather_xrows<T, P, true, true>), grid, dim3(kThreads), 0, s, yX, g,
                       constrained, accumulate, x, y, skip);
  else if (nt)
    hipLaunchKernelGGL((k_gather_xrows<T, P, true, false>), grid, dim3(kThreads), 0, s, yX, g,
                       constrained, accumulate, x, y, skip);
  else if (nt_y)
    hipLaunchKernelGGL((k_gather_xrows<T, P, false, true>), grid, dim3(kThreads), 0, s, yX, g,
                       constrained, accumulate, x, y, skip);
  else
    hipLaunchKernelGGL((k_gather_xrows<T, P, false, false>), grid, dim3(kThreads), 0, s, yX, g,
                       constrained, accumulate, x, y, skip);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather_xrows(const T* yX, int nx, int ny, int nz, int p, int constrained,
                               int accumulate, const T* x, T* y, const int* skip, hipStream_t s,
                               bool nt, bool nt_y) {
  const int64_t Lx = (int64_t)nx * p + 1, Ly = (int64_t)ny * p + 1, Lz = (int64_t)nz * p + 1;
  if (nx <= 0 || ny <= 0 || nz <= 0) return hipSuccess;
  if (Lx * Ly * Lz > 0x7fffffff) return hipErrorInvalidValue;
  switch (p) {
    case 1:
      return gather_xrows_p<T, 1>(yX, nx, ny, nz, constrained, accumulate, x, y, skip, s, nt,
                                   nt_y);
    case 2:
      return gather_xrows_p<T, 2>(yX, nx, ny, nz, constrained, accumulate, x, y, skip, s, nt,
                                   nt_y);
    case 3:
      return gather_xrows_p<T, 3>(yX, nx, ny, nz, constrained, accumulate, x, y, skip, s, nt,
                                   nt_y);
    case 4:
      return gather_xrows_p<T, 4>(yX, nx, ny, nz, constrained, accumulate, x, y, skip, s, nt,
                                   nt_y);
    case 5:
      return gather_xrows_p<T, 5>(yX, nx, ny, nz, constrained, accumulate, x, y, skip, s, nt,
                                   nt_y);
    case 6:
      return gather_xrows_p<T, 6>(yX, nx, ny, nz, constrained, accumulate, x, y, skip, s, nt,
                                   nt_y);
    case 7:
      return gather_xrows_p<T, 7>(yX, nx, ny, nz, constrained, accumulate, x, y, skip, s, nt,
                                   nt_y);
    case 8:
      return gather_xrows_p<T, 8>(yX, nx, ny, nz, constrained, accumulate, x, y, skip, s, nt,
                                   nt_y);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_gather_xrows<double>(const double*, int, int, int, int, int, int,
                                                const double*, double*, const int*, hipStream_t,
                                                bool, bool);
template hipError_t launch_gather_xrows<float>(const float*, int, int, int, int, int, int,
                                               const float*, float*, const int*, hipStream_t,
                                               bool, bool);
template hipError_t launch_gather_lattice<double>(const double*, int, int, int, int, int, int,
                                                  const double*, double*, const int*, hipStream_t);
template hipError_t launch_gather_lattice<float>(const float*, int, int, int, int, int, int,
                                                 const float*, float*, const int*, hipStream_t);

template <typename T>
hipError_t launch_set_ess(const int32_t* ess, int64_t n_ess, const T* x, T value, int accumulate,
                          T* y, const int* skip, hipStream_t s) {
  if (n_ess == 0) return hipSuccess;
  hipLaunchKernelGGL((k_set_ess<T>), dim3((n_ess + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                     ess, n_ess, x, value, accumulate, y, skip);
  return hipGetLastError();
}
template hipError_t launch_set_ess<double>(const int32_t*, int64_t, const double*, double, int,
                                           double*, const int*, hipStream_t);
template hipError_t launch_set_ess<float>(const int32_t*, int64_t, const float*, float, int, float*,
                                          const int*, hipStream_t);

template <typename T>
hipError_t launch_fill(T* y, int64_t n, T value, const int* skip, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(n)), dim3(kThreads), 0, s, y, n, value, skip);
  return hipGetLastError();
}
template hipError_t launch_fill<double>(double*, int64_t, double, const int*, hipStream_t);
template hipError_t launch_fill<float>(float*, int64_t, float, const int*, hipStream_t);

template <typename T>
hipError_t launch_dot_partial(const T* x, const T* y, int64_t n, double* partials, int nb,
                              const int* skip, hipStream_t s) {
  hipLaunchKernelGGL((k_dot_partial<T>), dim3(nb), dim3(kThreads), 0, s, x, y, n, partials, skip);
  return hipGetLastError();
}
template hipError_t launch_dot_partial<double>(const double*, const double*, int64_t, double*, int,
                                               const int*, hipStream_t);
template hipError_t launch_dot_partial<float>(const float*, const float*, int64_t, double*, int,
                                              const int*, hipStream_t);

hipError_t launch_sum_final(const double* partials, int nb, int ncols, double* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kThreads), 0, s, partials, nb, ncols, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_init(const T* r, const T* dinv, T* p, int64_t n, double* partials, int nb,
                          hipStream_t s) {
  hipLaunchKernelGGL((k_cg_init<T>), dim3(nb), dim3(kThreads), 0, s, r, dinv, p, n, partials);
  return hipGetLastError();
}
template hipError_t launch_cg_init<double>(const double*, const double*, double*, int64_t,
                                           double*, int, hipStream_t);
template hipError_t launch_cg_init<float>(const float*, const float*, float*, int64_t, double*,
                                          int, hipStream_t);

hipError_t launch_cg_init_final(const double* partials, int nb, double bb, double rtol,
                                int maxit, CgState* st, hipStream_t s, double delta2,
                                const double* bb_dev) {
  hipLaunchKernelGGL(k_cg_init_final, dim3(1), dim3(kThreads), 0, s, partials, nb, bb, bb_dev,
                     rtol, maxit, delta2, st);
  return hipGetLastError();
}

hipError_t launch_replace_residual(const double* r64, const float* dinv, float* rs, int64_t n,
                                   double* partials, int nb, CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_replace_residual, dim3(nb), dim3(kThreads), 0, s, r64, dinv, rs, n,
                     partials);
  if (st != nullptr)
    hipLaunchKernelGGL(k_replace_final, dim3(1), dim3(kThreads), 0, s, partials, nb, st);
  return hipGetLastError();
}

hipError_t launch_cg_alpha(const double* partials, int nb, CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(kThreads), 0, s, partials, nb, st);
  return hipGetLastError();
}

template <typename TX, typename T>
hipError_t launch_cg_update(TX* x, T* r, const T* p, const T* Ap, const T* dinv, int64_t n,
                            double* partials, int nb, const CgState* st, hipStream_t s) {
  hipLaunchKernelGGL((k_cg_update<TX, T>), dim3(nb), dim3(kThreads), 0, s, x, r, p, Ap, dinv, n,
                     partials, st);
  return hipGetLastError();
}
template hipError_t launch_cg_update<double, double>(double*, double*, const double*,
                                                     const double*, const double*, int64_t,
                                                     double*, int, const CgState*, hipStream_t);
template hipError_t launch_cg_update<float, float>(float*, float*, const float*, const float*,
                                                   const float*, int64_t, double*, int,
                                                   const CgState*, hipStream_t);
template hipError_t launch_cg_update<double, float>(double*, float*, const float*, const float*,
                                                    const float*, int64_t, double*, int,
                                                    const CgState*, hipStream_t);

hipError_t launch_cg_beta(const double* partials, int nb, CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(kThreads), 0, s, partials, nb, st);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_pupdate(T* p, const T* r, const T* dinv, int64_t n, const CgState* st,
                             hipStream_t s) {
  hipLaunchKernelGGL((k_cg_pupdate<T>), dim3(grid_for(n)), dim3(kThreads), 0, s, p, r, dinv, n,
                     st);
  return hipGetLastError();
}
template hipError_t launch_cg_pupdate<double>(double*, const double*, const double*, int64_t,
                                              const CgState*, hipStream_t);
template hipError_t launch_cg_pupdate<float>(float*, const float*, const float*, int64_t,
                                             const CgState*, hipStream_t);

hipError_t launch_residual(const double* b, const double* Ax, double* r, int64_t n,
                           hipStream_t s, const int* skip) {
  hipLaunchKernelGGL(k_residual, dim3(grid_for(n)), dim3(kThreads), 0, s, b, Ax, r, n, skip);
  return hipGetLastError();
}

// *flag = 1 while the CG of st is still running, 0 once it is done (the skip
// flag of work that only a finished CG needs)
__global__ void k_running_flag(const CgState* __restrict__ st, int* __restrict__ flag) {
  *flag = st->done ? 0 : 1;
}

hipError_t launch_running_flag(const CgState* st, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_running_flag, dim3(1), dim3(1), 0, s, st, flag);
  return hipGetLastError();
}

hipError_t launch_scale_to_f32(const double* r, const double* norm2, float* r32, int64_t n,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_scale_to_f32, dim3(grid_for(n)), dim3(kThreads), 0, s, r, norm2, r32, n);
  return hipGetLastError();
}

hipError_t launch_axpy_from_f32(double* x, const double* norm2, const float* d32, int64_t n,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_from_f32, dim3(grid_for(n)), dim3(kThreads), 0, s, x, norm2, d32, n);
  return hipGetLastError();
}

hipError_t launch_recip(const double* d, double* dinv64, float* dinv32, int64_t n,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_recip, dim3(grid_for(n)), dim3(kThreads), 0, s, d, dinv64, dinv32, n);
  return hipGetLastError();
}

template <typename T, typename TX, int P>
hipError_t gather_xrows_cg_p(const T* yX, int nx, int ny, int nz, const T* p, TX* x, T* r,
                             const T* dinv, double* partials, int* nparts, const CgState* st,
                             hipStream_t s, bool nt) {
  const int64_t nodes = ((int64_t)nx * P + 1) * ((int64_t)ny * P + 1) * ((int64_t)nz * P + 1);
  const int64_t per = (int64_t)kThreads * kXRowsNodes;
  int64_t nblk = (nodes + per - 1) / per;
  if (nblk > kMaxCgParts) nblk = kMaxCgParts;  // the workgroups stride over the rest
  *nparts = (int)nblk;
  if (nt)
    hipLaunchKernelGGL((k_gather_xrows_cg<T, TX, P, true>), dim3((unsigned)nblk), dim3(kThreads), 0,
                       s, yX, xrows_geom(nx, ny, nz, P), p, x, r, dinv, partials, st);
  else
    hipLaunchKernelGGL((k_gather_xrows_cg<T, TX, P, false>), dim3((unsigned)nblk), dim3(kThreads),
                       0, s, yX, xrows_geom(nx, ny, nz, P), p, x, r, dinv, partials, st);
  return hipGetLastError();
}

template <typename T, typename TX>
hipError_t launch_gather_xrows_cg(const T* yX, int nx, int ny, int nz, int pdeg, const T* p,
                                  TX* x, T* r, const T* dinv, double* partials, int* nparts,
                                  const CgState* st, hipStream_t s, bool nt) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || pdeg < 1) return hipErrorInvalidValue;
  const int64_t nodes = ((int64_t)nx * pdeg + 1) * ((int64_t)ny * pdeg + 1) *
                        ((int64_t)nz * pdeg + 1);
  if (nodes > 0x7fffffff) return hipErrorInvalidValue;  // 32-bit node indices
  switch (pdeg) {
#define PAFEM_CASE(PP) \
  case PP:             \
    return gather_xrows_cg_p<T, TX, PP>(yX, nx, ny, nz, p, x, r, dinv, partials, nparts, st, s, \
                                        nt);
    PAFEM_CASE(1) PAFEM_CASE(2) PAFEM_CASE(3) PAFEM_CASE(4)
    PAFEM_CASE(5) PAFEM_CASE(6) PAFEM_CASE(7) PAFEM_CASE(8)
#undef PAFEM_CASE
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_gather_xrows_cg<double, double>(const double*, int, int, int, int,
                                                           const double*, double*, double*,
                                                           const double*, double*, int*,
                                                           const CgState*, hipStream_t, bool);
template hipError_t launch_gather_xrows_cg<float, float>(const float*, int, int, int, int,
                                                         const float*, float*, float*,
                                                         const float*, double*, int*,
                                                         const CgState*, hipStream_t, bool);
template hipError_t launch_gather_xrows_cg<float, double>(const float*, int, int, int, int,
                                                          const float*, double*, float*,
                                                          const float*, double*, int*,
                                                          const CgState*, hipStream_t, bool);

hipError_t launch_cg_alpha_wide(const double* partials, int nb, CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_alpha_wide, dim3(1), dim3(kWideThreads), 0, s, partials, nb, st);
  return hipGetLastError();
}

}  // namespace pafem
