// Kernels of the p-multigrid preconditioner: transfer between two orders of
// the hierarchy on the same mesh, the Chebyshev smoother's vector updates and
// the scalars of the flexible CG around it.
//
// The spaces are nested, so the prolongation P of a coarse function is its
// value at the fine nodes: on every element, the coarse element values are
// interpolated at the fine GLL nodes by the 1D matrix I[f][c] = l^c_c(x^f_f)
// applied one direction at a time (sum factorization, three contractions of
// (pc+1) -> (pf+1) lines).  Each fine node is written by exactly one element
// (the one with the lowest index containing it: local index below pf in each
// direction, the last element keeping its far face), so P needs no sum.  The
// restriction is P^T: every element contracts the fine values of the nodes it
// owns (the same ownership, so every fine node enters once) with I^T in the
// three directions, and the coarse element results are summed per coarse node
// by the ordered E^T of the x-interleaved E-vector, which also sets the
// essential coarse rows to zero.
#include "vec_impl.h"

namespace pafem {

namespace {

using vec::kThreads;
using vec::block_sum;

template <int PC, int PF>
struct Xfer {
  static constexpr int NC = PC + 1, NF = PF + 1;
  static constexpr int NE = (kThreads / (NF * NF)) > 0 ? kThreads / (NF * NF) : 1;  // elements per workgroup
  static constexpr int THREADS = ((NE * NF * NF + 63) / 64) * 64;
  static constexpr int S1 = NC * NC * NF;  // after the first contraction
  static constexpr int S2 = NC * NF * NF;  // after the second
};

struct LatticeElem {
  int ex, ey, ez;
  __device__ __forceinline__ void init(int64_t e, int nx, int ny) {
    const int64_t t = e / nx;
    ex = (int)(e - t * nx);
    ey = (int)(t % ny);
    ez = (int)(t / ny);
  }
};

// uf (+)= P uc: coarse order PC to fine order PF.  I1 is [PF+1][PC+1].
template <int PC, int PF>
__global__ __launch_bounds__((Xfer<PC, PF>::THREADS)) void k_prolong(
    const double* __restrict__ uc, double* __restrict__ uf, int nx, int ny, int nz, int64_t ne,
    const double* __restrict__ I1, int accumulate, const int* skip) {
  using X = Xfer<PC, PF>;
  constexpr int NC = X::NC, NF = X::NF, NE = X::NE;
  __shared__ double s1[NE * X::S1];  // [s][c][b][af]
  __shared__ double s2[NE * X::S2];  // [s][c][bf][af]
  if (skip != nullptr && *skip) return;
  const int tid = threadIdx.x, s = tid / (NF * NF), r = tid - s * (NF * NF);
  const int64_t e = (int64_t)blockIdx.x * NE + s;
  const bool act = s < NE && e < ne;
  LatticeElem L;
  L.init(act ? e : 0, nx, ny);
  const int Lxc = nx * PC + 1, Lyc = ny * PC + 1;
  const int Lxf = nx * PF + 1, Lyf = ny * PF + 1;
  // x contraction, line (b, c) of the coarse element
  if (act && r < NC * NC) {
    const int b = r % NC, c = r / NC;
    const double* src = uc + (L.ex * PC) + (int64_t)Lxc * ((L.ey * PC + b) + (int64_t)Lyc * (L.ez * PC + c));
    double u[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) u[a] = src[a];
#pragma unroll
    for (int af = 0; af < NF; ++af) {
      double v = 0.0;
#pragma unroll
      for (int a = 0; a < NC; ++a) v = fma(I1[af * NC + a], u[a], v);
      s1[s * X::S1 + (c * NC + b) * NF + af] = v;
    }
  }
  __syncthreads();
  // y contraction, line (af, c)
  if (act && r < NF * NC) {
    const int af = r % NF, c = r / NF;
    double u[NC];
#pragma unroll
    for (int b = 0; b < NC; ++b) u[b] = s1[s * X::S1 + (c * NC + b) * NF + af];
#pragma unroll
    for (int bf = 0; bf < NF; ++bf) {
      double v = 0.0;
#pragma unroll
      for (int b = 0; b < NC; ++b) v = fma(I1[bf * NC + b], u[b], v);
      s2[s * X::S2 + (c * NF + bf) * NF + af] = v;
    }
  }
  __syncthreads();
  // z contraction, line (af, bf); owned fine nodes only
  if (act) {
    const int af = r % NF, bf = r / NF;
    double u[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) u[c] = s2[s * X::S2 + (c * NF + bf) * NF + af];
    const bool own_xy = (af < PF || L.ex == nx - 1) && (bf < PF || L.ey == ny - 1);
    double* dst = uf + (L.ex * PF + af) + (int64_t)Lxf * ((L.ey * PF + bf) + (int64_t)Lyf * (L.ez * PF));
#pragma unroll
    for (int cf = 0; cf < NF; ++cf) {
      double v = 0.0;
#pragma unroll
      for (int c = 0; c < NC; ++c) v = fma(I1[cf * NC + c], u[c], v);
      if (own_xy && (cf < PF || L.ez == nz - 1)) {
        double* o = dst + (int64_t)Lxf * Lyf * cf;
        *o = accumulate ? *o + v : v;
      }
    }
  }
}

// rcX = per-element P_e^T of the owned fine values of rf, into the coarse
// x-interleaved E-vector (summed per coarse node afterwards).
template <int PC, int PF>
__global__ __launch_bounds__((Xfer<PC, PF>::THREADS)) void k_restrict_elem(
    const double* __restrict__ rf, double* __restrict__ rcX, int nx, int ny, int nz, int64_t ne,
    const double* __restrict__ I1, const int* skip) {
  using X = Xfer<PC, PF>;
  constexpr int NC = X::NC, NF = X::NF, NE = X::NE;
  __shared__ double s1[NE * X::S1];  // [s][c][b][af]
  __shared__ double s2[NE * X::S2];  // [s][c][bf][af]
  if (skip != nullptr && *skip) return;
  const int tid = threadIdx.x, s = tid / (NF * NF), r = tid - s * (NF * NF);
  const int64_t e = (int64_t)blockIdx.x * NE + s;
  const bool act = s < NE && e < ne;
  LatticeElem L;
  L.init(act ? e : 0, nx, ny);
  const int Lxf = nx * PF + 1, Lyf = ny * PF + 1;
  // transposed z contraction, fine line (af, bf)
  if (act) {
    const int af = r % NF, bf = r / NF;
    const bool own_xy = (af < PF || L.ex == nx - 1) && (bf < PF || L.ey == ny - 1);
    const double* src = rf + (L.ex * PF + af) + (int64_t)Lxf * ((L.ey * PF + bf) + (int64_t)Lyf * (L.ez * PF));
    double u[NF];
#pragma unroll
    for (int cf = 0; cf < NF; ++cf) {
      const double v = src[(int64_t)Lxf * Lyf * cf];
      u[cf] = (own_xy && (cf < PF || L.ez == nz - 1)) ? v : 0.0;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double v = 0.0;
#pragma unroll
      for (int cf = 0; cf < NF; ++cf) v = fma(I1[cf * NC + c], u[cf], v);
      s2[s * X::S2 + (c * NF + bf) * NF + af] = v;
    }
  }
  __syncthreads();
  // transposed y contraction, line (af, c)
  if (act && r < NF * NC) {
    const int af = r % NF, c = r / NF;
    double u[NF];
#pragma unroll
    for (int bf = 0; bf < NF; ++bf) u[bf] = s2[s * X::S2 + (c * NF + bf) * NF + af];
#pragma unroll
    for (int b = 0; b < NC; ++b) {
      double v = 0.0;
#pragma unroll
      for (int bf = 0; bf < NF; ++bf) v = fma(I1[bf * NC + b], u[bf], v);
      s1[s * X::S1 + (c * NC + b) * NF + af] = v;
    }
  }
  __syncthreads();
  // transposed x contraction, coarse line (b, c)
  if (act && r < NC * NC) {
    const int b = r % NC, c = r / NC;
    double u[NF];
#pragma unroll
    for (int af = 0; af < NF; ++af) u[af] = s1[s * X::S1 + (c * NC + b) * NF + af];
    double* dst = rcX + xrows_index(nx, ny, NC, L.ex, L.ey, L.ez, 0, b, c);
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      double v = 0.0;
#pragma unroll
      for (int af = 0; af < NF; ++af) v = fma(I1[af * NC + a], u[af], v);
      dst[a] = v;
    }
  }
}

// ---- Chebyshev smoother ----------------------------------------------------------
// d = c0 dinv b, t = b
__global__ __launch_bounds__(kThreads) void k_cheb_init(const double* __restrict__ b,
                                                        const double* __restrict__ dinv,
                                                        double* __restrict__ d,
                                                        double* __restrict__ t, double c0,
                                                        int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const double bi = b[i];
    d[i] = c0 * (dinv[i] * bi);
    if (t != b) t[i] = bi;
  }
}

// x (+)= d, t -= w (= A d), d = c1 d + c2 dinv t
__global__ __launch_bounds__(kThreads) void k_cheb_step(double* __restrict__ x,
                                                        double* __restrict__ t,
                                                        double* __restrict__ d,
                                                        const double* __restrict__ w,
                                                        const double* __restrict__ dinv,
                                                        double c1, double c2, int first,
                                                        int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const double di = d[i];
    x[i] = first ? di : x[i] + di;
    const double ti = t[i] - w[i];
    t[i] = ti;
    d[i] = c1 * di + c2 * (dinv[i] * ti);
  }
}

// ---- flexible CG ------------------------------------------------------------------
// x += alpha p, r -= alpha w; partials of r . r
__global__ __launch_bounds__(kThreads) void k_fcg_update(double* __restrict__ x,
                                                         double* __restrict__ r,
                                                         const double* __restrict__ p,
                                                         const double* __restrict__ w,
                                                         const FcgState* __restrict__ st,
                                                         int64_t n, double* __restrict__ part) {
  const double alpha = st->alpha;
  double v[1] = {0.0}, out[1];
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * w[i];
    r[i] = ri;
    v[0] += ri * ri;
  }
  block_sum<1>(v, out);
  if (threadIdx.x == 0) part[blockIdx.x] = out[0];
}

// partials of (z . w, r . z)
__global__ __launch_bounds__(kThreads) void k_fcg_dots(const double* __restrict__ z,
                                                       const double* __restrict__ w,
                                                       const double* __restrict__ r, int64_t n,
                                                       double* __restrict__ part) {
  double v[2] = {0.0, 0.0}, out[2];
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const double zi = z[i];
    v[0] += zi * w[i];
    v[1] += r[i] * zi;
  }
  block_sum<2>(v, out);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = out[0];
    part[2 * blockIdx.x + 1] = out[1];
  }
}

// stage: 0 alpha from p . w; 1 rr (and the stopping test); 2 beta from (z . w, r . z);
// 3 initial r . z and r . r
__global__ void k_fcg_scalars(const double* __restrict__ part, int nb, int stage,
                              FcgState* st) {
  double r[4];
  vec::final_sums(part, nb, stage == 2 || stage == 3 ? 2 : 1, r);
  if (threadIdx.x != 0) return;
  if (stage == 0) {
    st->pw = r[0];
    st->alpha = st->rz / r[0];
  } else if (stage == 1) {
    st->rr = r[0];
    st->iter += 1;
    st->done = r[0] <= st->rr_stop ? 1 : (st->iter >= st->maxit ? 2 : 0);
  } else if (stage == 2) {
    // flexible (Polak-Ribiere) beta: z_new . (r_new - r_old) / (z_old . r_old)
    // with r_new - r_old = -alpha w
    st->beta = -st->alpha * r[0] / st->rz;
    st->rz = r[1];
  } else {
    st->rz = r[1];
    st->rr = r[0];
    st->beta = 0.0;
  }
}

// p = z + beta p
__global__ __launch_bounds__(kThreads) void k_fcg_pupdate(double* __restrict__ p,
                                                          const double* __restrict__ z,
                                                          const FcgState* __restrict__ st,
                                                          int64_t n) {
  const double beta = st->beta;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    p[i] = z[i] + beta * p[i];
}

// partials of (r . r, r . z) for the first direction (stage 3 reads them as (rr, rz))
__global__ __launch_bounds__(kThreads) void k_fcg_init_dots(const double* __restrict__ r,
                                                            const double* __restrict__ z,
                                                            int64_t n, double* __restrict__ part) {
  double v[2] = {0.0, 0.0}, out[2];
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const double ri = r[i];
    v[0] += ri * ri;
    v[1] += ri * z[i];
  }
  block_sum<2>(v, out);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = out[0];
    part[2 * blockIdx.x + 1] = out[1];
  }
}

// ---- power iteration for the largest eigenvalue of D^-1 A -------------------------
// splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", 2014) of seed + i, top 53 bits to [-1, 1)
__device__ __forceinline__ double hash_uniform(uint64_t z) {
  z += 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ __launch_bounds__(kThreads) void k_hash_fill(double* __restrict__ v, int64_t n,
                                                        uint64_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    v[i] = hash_uniform(seed + (uint64_t)i);
}

__global__ __launch_bounds__(kThreads) void k_power_dots(const double* __restrict__ v,
                                                         const double* __restrict__ w,
                                                         const double* __restrict__ dinv,
                                                         int64_t n, double* __restrict__ part) {
  double a[3] = {0.0, 0.0, 0.0}, out[3];
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const double vi = v[i], wi = w[i], di = dinv[i], ui = di * wi;
    a[0] += vi * wi;
    a[1] += vi * vi / di;
    a[2] += ui * ui;
  }
  block_sum<3>(a, out);
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) part[3 * blockIdx.x + c] = out[c];
}

__global__ __launch_bounds__(kThreads) void k_power_next(double* __restrict__ v,
                                                         const double* __restrict__ w,
                                                         const double* __restrict__ dinv,
                                                         double scale, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    v[i] = scale * (dinv[i] * w[i]);
}

inline int grid_for(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

template <int PC, int PF>
hipError_t transfer_pair(bool prolong, const double* src, double* dst, int nx, int ny, int nz,
                         const double* I1, int accumulate, const int* skip, hipStream_t s) {
  using X = Xfer<PC, PF>;
  const int64_t ne = (int64_t)nx * ny * nz;
  const int64_t nb = (ne + X::NE - 1) / X::NE;
  if (prolong)
    hipLaunchKernelGGL((k_prolong<PC, PF>), dim3((unsigned)nb), dim3(X::THREADS), 0, s, src, dst,
                       nx, ny, nz, ne, I1, accumulate, skip);
  else
    hipLaunchKernelGGL((k_restrict_elem<PC, PF>), dim3((unsigned)nb), dim3(X::THREADS), 0, s, src,
                       dst, nx, ny, nz, ne, I1, skip);
  return hipGetLastError();
}

hipError_t transfer(bool prolong, int pc, int pf, const double* src, double* dst, int nx, int ny,
                    int nz, const double* I1, int accumulate, const int* skip, hipStream_t s) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || I1 == nullptr || src == nullptr || dst == nullptr)
    return hipErrorInvalidValue;
  if (pc != pf / 2) return hipErrorInvalidValue;
  switch (pf) {
    case 2: return transfer_pair<1, 2>(prolong, src, dst, nx, ny, nz, I1, accumulate, skip, s);
    case 3: return transfer_pair<1, 3>(prolong, src, dst, nx, ny, nz, I1, accumulate, skip, s);
    case 4: return transfer_pair<2, 4>(prolong, src, dst, nx, ny, nz, I1, accumulate, skip, s);
    case 5: return transfer_pair<2, 5>(prolong, src, dst, nx, ny, nz, I1, accumulate, skip, s);
    case 6: return transfer_pair<3, 6>(prolong, src, dst, nx, ny, nz, I1, accumulate, skip, s);
    case 7: return transfer_pair<3, 7>(prolong, src, dst, nx, ny, nz, I1, accumulate, skip, s);
    case 8: return transfer_pair<4, 8>(prolong, src, dst, nx, ny, nz, I1, accumulate, skip, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_prolong(int pc, int pf, const double* uc, double* uf, int nx, int ny, int nz,
                          const double* I1, int accumulate, const int* skip, hipStream_t s) {
  return transfer(true, pc, pf, uc, uf, nx, ny, nz, I1, accumulate, skip, s);
}

hipError_t launch_restrict_elem(int pc, int pf, const double* rf, double* rcX, int nx, int ny,
                                int nz, const double* I1, const int* skip, hipStream_t s) {
  return transfer(false, pc, pf, rf, rcX, nx, ny, nz, I1, 0, skip, s);
}

hipError_t launch_cheb_init(const double* b, const double* dinv, double* d, double* t, double c0,
                            int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cheb_init, dim3(grid_for(n)), dim3(kThreads), 0, s, b, dinv, d, t, c0, n);
  return hipGetLastError();
}

hipError_t launch_cheb_step(double* x, double* t, double* d, const double* w, const double* dinv,
                            double c1, double c2, int first, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cheb_step, dim3(grid_for(n)), dim3(kThreads), 0, s, x, t, d, w, dinv, c1,
                     c2, first, n);
  return hipGetLastError();
}

hipError_t launch_fcg_update(double* x, double* r, const double* p, const double* w,
                             const FcgState* st, int64_t n, double* part, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_fcg_update, dim3(nb), dim3(kThreads), 0, s, x, r, p, w, st, n, part);
  return hipGetLastError();
}

hipError_t launch_fcg_dots(const double* z, const double* w, const double* r, int64_t n,
                           double* part, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_fcg_dots, dim3(nb), dim3(kThreads), 0, s, z, w, r, n, part);
  return hipGetLastError();
}

hipError_t launch_fcg_init_dots(const double* r, const double* z, int64_t n, double* part, int nb,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_fcg_init_dots, dim3(nb), dim3(kThreads), 0, s, r, z, n, part);
  return hipGetLastError();
}

hipError_t launch_fcg_scalars(const double* part, int nb, int stage, FcgState* st,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_fcg_scalars, dim3(1), dim3(kThreads), 0, s, part, nb, stage, st);
  return hipGetLastError();
}

hipError_t launch_fcg_pupdate(double* p, const double* z, const FcgState* st, int64_t n,
                              hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fcg_pupdate, dim3(grid_for(n)), dim3(kThreads), 0, s, p, z, st, n);
  return hipGetLastError();
}

hipError_t launch_hash_fill(double* v, int64_t n, uint64_t seed, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_hash_fill, dim3(grid_for(n)), dim3(kThreads), 0, s, v, n, seed);
  return hipGetLastError();
}

hipError_t launch_power_dots(const double* v, const double* w, const double* dinv, int64_t n,
                             double* part, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_power_dots, dim3(nb), dim3(kThreads), 0, s, v, w, dinv, n, part);
  return hipGetLastError();
}

hipError_t launch_power_next(double* v, const double* w, const double* dinv, double scale,
                             int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_power_next, dim3(grid_for(n)), dim3(kThreads), 0, s, v, w, dinv, scale, n);
  return hipGetLastError();
}

}  // namespace pafem
