// Fused partial-assembly operator kernels for gfx950.
//
// One element is handled by a q x q slice of threads (tx, ty) of a workgroup;
// a workgroup holds NE such slices.  Per element the operator
// E^T B^T D B E of the paper's operator decomposition runs as
//   gather (E)  ->  x, y 1D contractions through LDS  ->  z contraction in
//   registers (each thread owns a z-pencil)  ->  pointwise D  ->  transposed z
//   in registers  ->  transposed y, x through LDS  ->  scatter (E^T).
// Only the quadrature data D is streamed from HBM besides the two vectors;
// the E-vector and Q-vector never leave LDS/registers.
#include "geom.h"
#include "internal.h"

namespace pafem {

namespace {

constexpr int kBlockTarget = 256;    // threads per workgroup aimed for
constexpr int kLdsBudget = 64 * 1024;  // bytes of LDS per workgroup

template <int P, int Q, typename T, int KIND>
struct Cfg {
  static constexpr int N = P + 1;
  static constexpr int QQ = Q * Q;
  // LDS words per element: forward buffers (u, x-contracted) and backward
  // buffers (z-contracted components, y-contracted components).
  static constexpr int L_DIFF_F = N * N * N + 2 * N * N * Q;
  static constexpr int L_DIFF_B = 3 * N * Q * Q + 2 * N * N * Q;
  static constexpr int L_MASS_F = N * N * N + N * N * Q;
  static constexpr int L_MASS_B = N * Q * Q + N * N * Q;
  static constexpr int L_F = KIND == PAFEM_DIFFUSION ? L_DIFF_F : L_MASS_F;
  static constexpr int L_B = KIND == PAFEM_DIFFUSION ? L_DIFF_B : L_MASS_B;
  static constexpr int L = L_F > L_B ? L_F : L_B;
  static constexpr int NE_T = kBlockTarget / QQ > 0 ? kBlockTarget / QQ : 1;
  static constexpr int NE_L = kLdsBudget / (L * (int)sizeof(T)) > 0 ? kLdsBudget / (L * (int)sizeof(T)) : 1;
  static constexpr int NE = NE_T < NE_L ? NE_T : NE_L;
  static constexpr int THREADS = QQ * NE;
};

template <typename T>
__device__ __forceinline__ void scatter_add(T* p, T v) {
  atomicAdd(p, v);
}

// ---------------------------------------------------------------------------
// diffusion:  y_e = sum_{i,j} G_i^T S_ij G_j x_e  with S the stored symmetric
// w k adj(J) adj(J)^T / detJ (6 entries per quadrature point).
// ---------------------------------------------------------------------------
template <int P, int Q, typename T, int SCATTER>
__global__ __launch_bounds__((Cfg<P, Q, T, PAFEM_DIFFUSION>::THREADS)) void k_apply_diff(
    ApplyArgs<T> a) {
  using C = Cfg<P, Q, T, PAFEM_DIFFUSION>;
  constexpr int N = C::N, QQ = C::QQ, NE = C::NE, L = C::L;
  constexpr int QQQ = Q * Q * Q;
  __shared__ T smem[NE * L];
  if (a.skip != nullptr && *a.skip) return;

  const int tid = threadIdx.x;
  const int slot = tid / QQ;
  const int t = tid - slot * QQ;
  const int tx = t % Q, ty = t / Q;
  const int64_t e = (int64_t)blockIdx.x * NE + slot;
  const bool active = e < a.ne;
  T* s = smem + slot * L;
  T* s_u = s;                     // [c][b][a]
  T* s_tb = s + N * N * N;        // [c][b][qx]  B-contracted in x
  T* s_tg = s_tb + N * N * Q;     // [c][b][qx]  G-contracted in x
  T* s_w = s;                     // [3][c][qy][qx] (reuses the forward region)
  T* s_W1 = s + 3 * N * QQ;       // [c][b][qx]
  T* s_W23 = s_W1 + N * N * Q;    // [c][b][qx]

  // Issue the quadrature-data loads for this thread's z-pencil first; they are
  // the dominant HBM stream and their latency hides behind the contractions.
  T dq[6][Q];
  if (active) {
    const T* qd = a.qd + (e * 6) * QQQ + ty * Q + tx;
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
      for (int qz = 0; qz < Q; ++qz) dq[k][qz] = __builtin_nontemporal_load(qd + k * QQQ + qz * QQ);
  }

  // gather x_e = E x
  if (active) {
    const int32_t* Ee = a.E + e * (N * N * N);
    for (int i = t; i < N * N * N; i += QQ) {
      int g = Ee[i];
      T v = a.x[g];
      if (a.constrained && a.ess_mask[g]) v = T(0);
      s_u[i] = v;
    }
  }
  __syncthreads();

  // x contraction: thread (qx = tx, b = ty)
  if (active && ty < N) {
    T bx[N], gx[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      bx[i] = a.B[tx * N + i];
      gx[i] = a.G[tx * N + i];
    }
#pragma unroll
    for (int c = 0; c < N; ++c) {
      T sb = 0, sg = 0;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        T u = s_u[(c * N + ty) * N + i];
        sb += bx[i] * u;
        sg += gx[i] * u;
      }
      s_tb[(c * N + ty) * Q + tx] = sb;
      s_tg[(c * N + ty) * Q + tx] = sg;
    }
  }
  __syncthreads();

  // y contraction: thread (qx = tx, qy = ty); results stay in registers (z-pencil over c)
  T rbb[N], rgb[N], rbg[N];  // (x,y) factors: (B,B), (G,B), (B,G)
  if (active) {
    T by[N], gy[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      by[i] = a.B[ty * N + i];
      gy[i] = a.G[ty * N + i];
    }
#pragma unroll
    for (int c = 0; c < N; ++c) {
      T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
      for (int b = 0; b < N; ++b) {
        T tb = s_tb[(c * N + b) * Q + tx];
        T tg = s_tg[(c * N + b) * Q + tx];
        s0 += by[b] * tb;
        s1 += by[b] * tg;
        s2 += gy[b] * tb;
      }
      rbb[c] = s0;
      rgb[c] = s1;
      rbg[c] = s2;
    }
  }
  __syncthreads();  // forward LDS region is reused below

  // z contraction, pointwise D, transposed z contraction -- all in registers
  T w1[N], w2[N], w3[N];
#pragma unroll
  for (int c = 0; c < N; ++c) w1[c] = w2[c] = w3[c] = 0;
  if (active) {
#pragma unroll
    for (int qz = 0; qz < Q; ++qz) {
      T gxq = 0, gyq = 0, gzq = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) {
        const T bz = a.B[qz * N + c], gz = a.G[qz * N + c];
        gxq += bz * rgb[c];
        gyq += bz * rbg[c];
        gzq += gz * rbb[c];
      }
      const T vx = dq[0][qz] * gxq + dq[1][qz] * gyq + dq[2][qz] * gzq;
      const T vy = dq[1][qz] * gxq + dq[3][qz] * gyq + dq[4][qz] * gzq;
      const T vz = dq[2][qz] * gxq + dq[4][qz] * gyq + dq[5][qz] * gzq;
#pragma unroll
      for (int c = 0; c < N; ++c) {
        const T bz = a.B[qz * N + c], gz = a.G[qz * N + c];
        w1[c] += bz * vx;
        w2[c] += bz * vy;
        w3[c] += gz * vz;
      }
    }
#pragma unroll
    for (int c = 0; c < N; ++c) {
      s_w[(0 * N + c) * QQ + t] = w1[c];
      s_w[(1 * N + c) * QQ + t] = w2[c];
      s_w[(2 * N + c) * QQ + t] = w3[c];
    }
  }
  __syncthreads();

  // transposed y contraction: thread (qx = tx, b = ty)
  if (active && ty < N) {
    T byc[Q], gyc[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      byc[i] = a.B[i * N + ty];
      gyc[i] = a.G[i * N + ty];
    }
#pragma unroll
    for (int c = 0; c < N; ++c) {
      T s1 = 0, s23 = 0;
#pragma unroll
      for (int qy = 0; qy < Q; ++qy) {
        s1 += byc[qy] * s_w[(0 * N + c) * QQ + qy * Q + tx];
        s23 += gyc[qy] * s_w[(1 * N + c) * QQ + qy * Q + tx] +
               byc[qy] * s_w[(2 * N + c) * QQ + qy * Q + tx];
      }
      s_W1[(c * N + ty) * Q + tx] = s1;
      s_W23[(c * N + ty) * Q + tx] = s23;
    }
  }
  __syncthreads();

  // transposed x contraction and scatter: thread (a = tx, b = ty)
  if (active && tx < N && ty < N) {
    T bxc[Q], gxc[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      bxc[i] = a.B[i * N + tx];
      gxc[i] = a.G[i * N + tx];
    }
    const int32_t* Ee = a.E + e * (N * N * N);
#pragma unroll
    for (int c = 0; c < N; ++c) {
      T acc = 0;
#pragma unroll
      for (int qx = 0; qx < Q; ++qx)
        acc += gxc[qx] * s_W1[(c * N + ty) * Q + qx] + bxc[qx] * s_W23[(c * N + ty) * Q + qx];
      const int l = (c * N + ty) * N + tx;
      if (SCATTER == PAFEM_SCATTER_DETERMINISTIC) {
        a.yE[e * (N * N * N) + l] = acc;
      } else {
        const int g = Ee[l];
        if (!(a.constrained && a.ess_mask[g])) scatter_add(a.y + g, acc);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// mass:  y_e = B^T D B x_e  with D = w rho detJ.
// ---------------------------------------------------------------------------
template <int P, int Q, typename T, int SCATTER>
__global__ __launch_bounds__((Cfg<P, Q, T, PAFEM_MASS>::THREADS)) void k_apply_mass(ApplyArgs<T> a) {
  using C = Cfg<P, Q, T, PAFEM_MASS>;
  constexpr int N = C::N, QQ = C::QQ, NE = C::NE, L = C::L;
  constexpr int QQQ = Q * Q * Q;
  __shared__ T smem[NE * L];
  if (a.skip != nullptr && *a.skip) return;

  const int tid = threadIdx.x;
  const int slot = tid / QQ;
  const int t = tid - slot * QQ;
  const int tx = t % Q, ty = t / Q;
  const int64_t e = (int64_t)blockIdx.x * NE + slot;
  const bool active = e < a.ne;
  T* s = smem + slot * L;
  T* s_u = s;                  // [c][b][a]
  T* s_t = s + N * N * N;      // [c][b][qx]
  T* s_w = s;                  // [c][qy][qx]
  T* s_W = s + N * QQ;         // [c][b][qx]

  T dq[Q];
  if (active) {
    const T* qd = a.qd + e * QQQ + ty * Q + tx;
#pragma unroll
    for (int qz = 0; qz < Q; ++qz) dq[qz] = __builtin_nontemporal_load(qd + qz * QQ);
  }

  if (active) {
    const int32_t* Ee = a.E + e * (N * N * N);
    for (int i = t; i < N * N * N; i += QQ) {
      int g = Ee[i];
      T v = a.x[g];
      if (a.constrained && a.ess_mask[g]) v = T(0);
      s_u[i] = v;
    }
  }
  __syncthreads();

  if (active && ty < N) {
    T bx[N];
#pragma unroll
    for (int i = 0; i < N; ++i) bx[i] = a.B[tx * N + i];
#pragma unroll
    for (int c = 0; c < N; ++c) {
      T sb = 0;
#pragma unroll
      for (int i = 0; i < N; ++i) sb += bx[i] * s_u[(c * N + ty) * N + i];
      s_t[(c * N + ty) * Q + tx] = sb;
    }
  }
  __syncthreads();

  T r[N];
  if (active) {
    T by[N];
#pragma unroll
    for (int i = 0; i < N; ++i) by[i] = a.B[ty * N + i];
#pragma unroll
    for (int c = 0; c < N; ++c) {
      T s0 = 0;
#pragma unroll
      for (int b = 0; b < N; ++b) s0 += by[b] * s_t[(c * N + b) * Q + tx];
      r[c] = s0;
    }
  }
  __syncthreads();

  T w[N];
#pragma unroll
  for (int c = 0; c < N; ++c) w[c] = 0;
  if (active) {
#pragma unroll
    for (int qz = 0; qz < Q; ++qz) {
      T uq = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) uq += a.B[qz * N + c] * r[c];
      const T v = dq[qz] * uq;
#pragma unroll
      for (int c = 0; c < N; ++c) w[c] += a.B[qz * N + c] * v;
    }
#pragma unroll
    for (int c = 0; c < N; ++c) s_w[c * QQ + t] = w[c];
  }
  __syncthreads();

  if (active && ty < N) {
    T byc[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) byc[i] = a.B[i * N + ty];
#pragma unroll
    for (int c = 0; c < N; ++c) {
      T s1 = 0;
#pragma unroll
      for (int qy = 0; qy < Q; ++qy) s1 += byc[qy] * s_w[c * QQ + qy * Q + tx];
      s_W[(c * N + ty) * Q + tx] = s1;
    }
  }
  __syncthreads();

  if (active && tx < N && ty < N) {
    T bxc[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) bxc[i] = a.B[i * N + tx];
    const int32_t* Ee = a.E + e * (N * N * N);
#pragma unroll
    for (int c = 0; c < N; ++c) {
      T acc = 0;
#pragma unroll
      for (int qx = 0; qx < Q; ++qx) acc += bxc[qx] * s_W[(c * N + ty) * Q + qx];
      const int l = (c * N + ty) * N + tx;
      if (SCATTER == PAFEM_SCATTER_DETERMINISTIC) {
        a.yE[e * (N * N * N) + l] = acc;
      } else {
        const int g = Ee[l];
        if (!(a.constrained && a.ess_mask[g])) scatter_add(a.y + g, acc);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Element diagonal by sum factorization.
//   diffusion: d[a,b,c] = sum_q sum_ij S_ij(q) Ghat_i(q;a,b,c) Ghat_j(q;a,b,c)
// where Ghat_x = G(qx,a) B(qy,b) B(qz,c) etc.  With the 1D tables
//   B2 = B.*B, G2 = G.*G, BG = B.*G  (elementwise, [q][n])
// the six terms factor direction by direction:
//   xx: G2 B2 B2   yy: B2 G2 B2   zz: B2 B2 G2
//   xy: 2 BG BG B2  xz: 2 BG B2 BG  yz: 2 B2 BG BG   (factors for x, y, z)
// and are contracted z, then y, then x.
// ---------------------------------------------------------------------------
template <int P, int Q, int KIND>
__global__ __launch_bounds__(Q * Q) void k_diag_elem(const double* __restrict__ qd,
                                                     const double* __restrict__ B,
                                                     const double* __restrict__ G, int64_t ne,
                                                     double* __restrict__ dE) {
  constexpr int N = P + 1, QQ = Q * Q, QQQ = Q * Q * Q;
  constexpr int NC = KIND == PAFEM_DIFFUSION ? 6 : 1;
  __shared__ double s_z[NC * N * QQ];   // z-contracted terms [term][c][qy][qx]
  __shared__ double s_y[3 * N * N * Q]; // y-contracted, grouped by x factor [grp][c][b][qx]
  __shared__ double s_b2[Q * N], s_g2[Q * N], s_bg[Q * N];
  const int t = threadIdx.x;
  const int tx = t % Q, ty = t / Q;
  const int64_t e = blockIdx.x;
  for (int i = t; i < Q * N; i += QQ) {
    s_b2[i] = B[i] * B[i];
    s_g2[i] = G[i] * G[i];
    s_bg[i] = B[i] * G[i];
  }
  __syncthreads();
  // z contraction: thread (qx, qy)
  {
    double d[NC][Q];
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
      for (int qz = 0; qz < Q; ++qz) d[k][qz] = qd[(e * NC + k) * QQQ + qz * QQ + t];
#pragma unroll
    for (int c = 0; c < N; ++c) {
      if (KIND == PAFEM_DIFFUSION) {
        double z00 = 0, z11 = 0, z22 = 0, z01 = 0, z02 = 0, z12 = 0;
#pragma unroll
        for (int qz = 0; qz < Q; ++qz) {
          const double b2 = s_b2[qz * N + c], g2 = s_g2[qz * N + c], bg = s_bg[qz * N + c];
          z00 += b2 * d[0][qz];
          z11 += b2 * d[3][qz];
          z22 += g2 * d[5][qz];
          z01 += b2 * d[1][qz];
          z02 += bg * d[2][qz];
          z12 += bg * d[4][qz];
        }
        s_z[(0 * N + c) * QQ + t] = z00;
        s_z[(1 * N + c) * QQ + t] = z11;
        s_z[(2 * N + c) * QQ + t] = z22;
        s_z[(3 * N + c) * QQ + t] = z01;
        s_z[(4 * N + c) * QQ + t] = z02;
        s_z[(5 * N + c) * QQ + t] = z12;
      } else {
        double z = 0;
#pragma unroll
        for (int qz = 0; qz < Q; ++qz) z += s_b2[qz * N + c] * d[0][qz];
        s_z[c * QQ + t] = z;
      }
    }
  }
  __syncthreads();
  // y contraction: thread (qx, b)
  if (ty < N) {
    const int b = ty;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      if (KIND == PAFEM_DIFFUSION) {
        double yg2 = 0, yb2 = 0, ybg = 0;
#pragma unroll
        for (int qy = 0; qy < Q; ++qy) {
          const double b2 = s_b2[qy * N + b], g2 = s_g2[qy * N + b], bg = s_bg[qy * N + b];
          const int o = qy * Q + tx;
          yg2 += b2 * s_z[(0 * N + c) * QQ + o];                                    // xx
          yb2 += g2 * s_z[(1 * N + c) * QQ + o] + b2 * s_z[(2 * N + c) * QQ + o]    // yy, zz
                 + 2.0 * bg * s_z[(5 * N + c) * QQ + o];                            // yz
          ybg += 2.0 * bg * s_z[(3 * N + c) * QQ + o] + 2.0 * b2 * s_z[(4 * N + c) * QQ + o];  // xy, xz
        }
        s_y[((0 * N + c) * N + b) * Q + tx] = yg2;
        s_y[((1 * N + c) * N + b) * Q + tx] = yb2;
        s_y[((2 * N + c) * N + b) * Q + tx] = ybg;
      } else {
        double yb2 = 0;
#pragma unroll
        for (int qy = 0; qy < Q; ++qy) yb2 += s_b2[qy * N + b] * s_z[c * QQ + qy * Q + tx];
        s_y[(c * N + b) * Q + tx] = yb2;
      }
    }
  }
  __syncthreads();
  // x contraction: thread (a, b)
  if (tx < N && ty < N) {
    const int aa = tx, b = ty;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      double acc = 0;
#pragma unroll
      for (int qx = 0; qx < Q; ++qx) {
        if (KIND == PAFEM_DIFFUSION) {
          acc += s_g2[qx * N + aa] * s_y[((0 * N + c) * N + b) * Q + qx] +
                 s_b2[qx * N + aa] * s_y[((1 * N + c) * N + b) * Q + qx] +
                 s_bg[qx * N + aa] * s_y[((2 * N + c) * N + b) * Q + qx];
        } else {
          acc += s_b2[qx * N + aa] * s_y[(c * N + b) * Q + qx];
        }
      }
      dE[e * (N * N * N) + (c * N + b) * N + aa] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// Right-hand side element vectors b_e[a,b,c] = sum_q B B B (w detJ f(x_q)).
// ---------------------------------------------------------------------------
template <int P, int Q>
__global__ __launch_bounds__(Q * Q) void k_rhs_elem(GeomArgs g, const double* __restrict__ B,
                                                    const double* __restrict__ f_q,
                                                    double* __restrict__ bE) {
  constexpr int N = P + 1, QQ = Q * Q, QQQ = Q * Q * Q;
  __shared__ double s_w[N * QQ];
  __shared__ double s_W[N * N * Q];
  const int t = threadIdx.x;
  const int tx = t % Q, ty = t / Q;
  const int64_t e = blockIdx.x;
  double v[8][3];
  load_corners(g, e, v);
  double w[N];
#pragma unroll
  for (int c = 0; c < N; ++c) w[c] = 0;
  for (int qz = 0; qz < Q; ++qz) {
    double X[3], J[3][3];
    trilinear_at(v, g.pts[tx], g.pts[ty], g.pts[qz], X, J);
    const double wq = g.wts[tx] * g.wts[ty] * g.wts[qz];
    double f;
    if (f_q != nullptr) {
      f = f_q[e * QQQ + qz * QQ + t];
    } else {
      f = 3.0 * M_PI * M_PI * sin(M_PI * X[0]) * sin(M_PI * X[1]) * sin(M_PI * X[2]);
    }
    const double val = wq * det3(J) * f;
#pragma unroll
    for (int c = 0; c < N; ++c) w[c] += B[qz * N + c] * val;
  }
#pragma unroll
  for (int c = 0; c < N; ++c) s_w[c * QQ + t] = w[c];
  __syncthreads();
  if (ty < N) {
#pragma unroll
    for (int c = 0; c < N; ++c) {
      double s1 = 0;
      for (int qy = 0; qy < Q; ++qy) s1 += B[qy * N + ty] * s_w[c * QQ + qy * Q + tx];
      s_W[(c * N + ty) * Q + tx] = s1;
    }
  }
  __syncthreads();
  if (tx < N && ty < N) {
#pragma unroll
    for (int c = 0; c < N; ++c) {
      double acc = 0;
      for (int qx = 0; qx < Q; ++qx) acc += B[qx * N + tx] * s_W[(c * N + ty) * Q + qx];
      bE[e * (N * N * N) + (c * N + ty) * N + tx] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
template <int P, typename T>
hipError_t apply_p(int kind, int scatter, const ApplyArgs<T>& a, hipStream_t s) {
  constexpr int Q = P + 2;
  if (a.ne == 0) return hipSuccess;
  if (kind == PAFEM_DIFFUSION) {
    using C = Cfg<P, Q, T, PAFEM_DIFFUSION>;
    const int64_t nb = (a.ne + C::NE - 1) / C::NE;
    if (scatter == PAFEM_SCATTER_DETERMINISTIC)
      hipLaunchKernelGGL((k_apply_diff<P, Q, T, PAFEM_SCATTER_DETERMINISTIC>), dim3(nb),
                         dim3(C::THREADS), 0, s, a);
    else
      hipLaunchKernelGGL((k_apply_diff<P, Q, T, PAFEM_SCATTER_ATOMIC>), dim3(nb),
                         dim3(C::THREADS), 0, s, a);
  } else {
    using C = Cfg<P, Q, T, PAFEM_MASS>;
    const int64_t nb = (a.ne + C::NE - 1) / C::NE;
    if (scatter == PAFEM_SCATTER_DETERMINISTIC)
      hipLaunchKernelGGL((k_apply_mass<P, Q, T, PAFEM_SCATTER_DETERMINISTIC>), dim3(nb),
                         dim3(C::THREADS), 0, s, a);
    else
      hipLaunchKernelGGL((k_apply_mass<P, Q, T, PAFEM_SCATTER_ATOMIC>), dim3(nb),
                         dim3(C::THREADS), 0, s, a);
  }
  return hipGetLastError();
}

template <int P>
hipError_t diag_p(int kind, const double* qd, const double* B, const double* G, int64_t ne,
                  double* dE, hipStream_t s) {
  constexpr int Q = P + 2;
  if (ne == 0) return hipSuccess;
  if (kind == PAFEM_DIFFUSION)
    hipLaunchKernelGGL((k_diag_elem<P, Q, PAFEM_DIFFUSION>), dim3(ne), dim3(Q * Q), 0, s, qd, B,
                       G, ne, dE);
  else
    hipLaunchKernelGGL((k_diag_elem<P, Q, PAFEM_MASS>), dim3(ne), dim3(Q * Q), 0, s, qd, B, G,
                       ne, dE);
  return hipGetLastError();
}

template <int P>
hipError_t rhs_p(const GeomArgs& g, const double* B, const double* f_q, double* bE,
                 hipStream_t s) {
  constexpr int Q = P + 2;
  if (g.ne == 0) return hipSuccess;
  hipLaunchKernelGGL((k_rhs_elem<P, Q>), dim3(g.ne), dim3(Q * Q), 0, s, g, B, f_q, bE);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_apply(int kind, int p, int q, int scatter_mode, const ApplyArgs<T>& a,
                        hipStream_t s) {
  if (q != p + 2) return hipErrorInvalidValue;
  switch (p) {
    case 1: return apply_p<1, T>(kind, scatter_mode, a, s);
    case 2: return apply_p<2, T>(kind, scatter_mode, a, s);
    case 3: return apply_p<3, T>(kind, scatter_mode, a, s);
    case 4: return apply_p<4, T>(kind, scatter_mode, a, s);
    case 5: return apply_p<5, T>(kind, scatter_mode, a, s);
    case 6: return apply_p<6, T>(kind, scatter_mode, a, s);
    case 7: return apply_p<7, T>(kind, scatter_mode, a, s);
    case 8: return apply_p<8, T>(kind, scatter_mode, a, s);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_apply<double>(int, int, int, int, const ApplyArgs<double>&, hipStream_t);
template hipError_t launch_apply<float>(int, int, int, int, const ApplyArgs<float>&, hipStream_t);

hipError_t launch_diag_elem(int kind, int p, int q, const double* qd, const double* B,
                            const double* G, int64_t ne, double* dE, hipStream_t s) {
  if (q != p + 2) return hipErrorInvalidValue;
  switch (p) {
    case 1: return diag_p<1>(kind, qd, B, G, ne, dE, s);
    case 2: return diag_p<2>(kind, qd, B, G, ne, dE, s);
    case 3: return diag_p<3>(kind, qd, B, G, ne, dE, s);
    case 4: return diag_p<4>(kind, qd, B, G, ne, dE, s);
    case 5: return diag_p<5>(kind, qd, B, G, ne, dE, s);
    case 6: return diag_p<6>(kind, qd, B, G, ne, dE, s);
    case 7: return diag_p<7>(kind, qd, B, G, ne, dE, s);
    case 8: return diag_p<8>(kind, qd, B, G, ne, dE, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rhs_elem(const GeomArgs& g, int p, const double* B, const double* f_q,
                           double* bE, hipStream_t s) {
  if (g.q != p + 2) return hipErrorInvalidValue;
  switch (p) {
    case 1: return rhs_p<1>(g, B, f_q, bE, s);
    case 2: return rhs_p<2>(g, B, f_q, bE, s);
    case 3: return rhs_p<3>(g, B, f_q, bE, s);
    case 4: return rhs_p<4>(g, B, f_q, bE, s);
    case 5: return rhs_p<5>(g, B, f_q, bE, s);
    case 6: return rhs_p<6>(g, B, f_q, bE, s);
    case 7: return rhs_p<7>(g, B, f_q, bE, s);
    case 8: return rhs_p<8>(g, B, f_q, bE, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pafem
