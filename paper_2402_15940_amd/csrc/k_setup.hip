// Setup kernels: quadrature-data assembly (the data partial assembly stores),
// quadrature point coordinates, the sum-factorized element diagonal and the
// right-hand side element vectors.
#include "geom.h"
#include "internal.h"

namespace pafem {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ void qpoint_of(const GeomArgs& g, int64_t idx, int64_t& e, int& qp,
                                          double& s, double& t, double& u, double& w) {
  const int q = g.q;
  const int qqq = q * q * q;
  e = idx / qqq;
  qp = (int)(idx - e * qqq);
  const int qx = qp % q, qy = (qp / q) % q, qz = qp / (q * q);
  s = g.pts[qx];
  t = g.pts[qy];
  u = g.pts[qz];
  w = g.wts[qx] * g.wts[qy] * g.wts[qz];
}

// Round a (finite) float to the nearest bfloat16, ties to even.
__device__ __forceinline__ uint16_t float_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// MASS:       D = w rho detJ
// DIFFUSION:  D = w k adj(J) adj(J)^T / detJ, upper triangle xx xy xz yy yz zz
// adj(J) is the adjugate (transposed cofactor matrix), so adj(J)/detJ = J^-1.
__global__ __launch_bounds__(kThreads) void k_qdata(GeomArgs g, int kind, int coef_kind,
                                                    double coef_value,
                                                    const double* __restrict__ coef_q,
                                                    double* __restrict__ qd64,
                                                    float* __restrict__ qd32,
                                                    uint16_t* __restrict__ qd16,
                                                    int* __restrict__ err_flag) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int qqq = g.q * g.q * g.q;
  if (idx >= g.ne * qqq) return;
  int64_t e;
  int qp;
  double s, t, u, w;
  qpoint_of(g, idx, e, qp, s, t, u, w);
  double v[8][3];
  load_corners(g, e, v);
  double X[3], J[3][3];
  trilinear_at(v, s, t, u, X, J);
  const double det = det3(J);
  if (!(det > 0.0)) atomicOr(err_flag, 1);
  double k;
  if (coef_kind == COEF_QPTS)
    k = coef_q[idx];
  else if (coef_kind == COEF_SINX)
    k = 1.0 + coef_value * sin(2.0 * M_PI * X[0]);
  else
    k = coef_value;
  if (qd64 == nullptr) return;  // Jacobian check only (matrix-free operators)
  if (kind == PAFEM_MASS) {
    const double d = w * k * det;
    qd64[e * qqq + qp] = d;
    if (qd32) qd32[e * qqq + qp] = (float)d;
    if (qd16) qd16[e * qqq + qp] = float_to_bf16((float)d);
    return;
  }
  // adjugate A = adj(J): A[i][j] = cofactor C[j][i]
  double A[3][3];
  A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const double f = w * k / det;
  double S[6];
  int m = 0;
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) S[m++] = f * (A[i][0] * A[j][0] + A[i][1] * A[j][1] + A[i][2] * A[j][2]);
  const int64_t base = e * 6 * (int64_t)qqq + qp;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    qd64[base + (int64_t)c * qqq] = S[c];
    if (qd32) qd32[base + (int64_t)c * qqq] = (float)S[c];
    if (qd16) qd16[base + (int64_t)c * qqq] = float_to_bf16((float)S[c]);
  }
}

__global__ __launch_bounds__(kThreads) void k_qpoint_coords(GeomArgs g, double* __restrict__ xyz) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int qqq = g.q * g.q * g.q;
  if (idx >= g.ne * qqq) return;
  int64_t e;
  int qp;
  double s, t, u, w;
  qpoint_of(g, idx, e, qp, s, t, u, w);
  double v[8][3];
  load_corners(g, e, v);
  double X[3], J[3][3];
  trilinear_at(v, s, t, u, X, J);
  for (int r = 0; r < 3; ++r) xyz[(e * 3 + r) * qqq + qp] = X[r];
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


// Launches for order P and quadrature size q (P + 1 <= q <= kMaxQ1d), one
// instantiation per q.
template <int P, int Q = P + 1>
hipError_t diag_p(int q, int kind, const double* qd, const double* B, const double* G, int64_t ne,
                  double* dE, hipStream_t s) {
  if constexpr (Q > kMaxQ1d) {
    return hipErrorInvalidValue;
  } else {
    if (q != Q) return diag_p<P, Q + 1>(q, kind, qd, B, G, ne, dE, s);
    if (ne == 0) return hipSuccess;
    if (kind == PAFEM_DIFFUSION)
      hipLaunchKernelGGL((k_diag_elem<P, Q, PAFEM_DIFFUSION>), dim3(ne), dim3(Q * Q), 0, s, qd, B,
                         G, ne, dE);
    else
      hipLaunchKernelGGL((k_diag_elem<P, Q, PAFEM_MASS>), dim3(ne), dim3(Q * Q), 0, s, qd, B, G,
                         ne, dE);
    return hipGetLastError();
  }
}

template <int P, int Q = P + 1>
hipError_t rhs_p(int q, const GeomArgs& g, const double* B, const double* f_q, double* bE,
                 hipStream_t s) {
  if constexpr (Q > kMaxQ1d) {
    return hipErrorInvalidValue;
  } else {
    if (q != Q) return rhs_p<P, Q + 1>(q, g, B, f_q, bE, s);
    if (g.ne == 0) return hipSuccess;
    hipLaunchKernelGGL((k_rhs_elem<P, Q>), dim3(g.ne), dim3(Q * Q), 0, s, g, B, f_q, bE);
    return hipGetLastError();
  }
}

}  // namespace

hipError_t launch_qdata(const GeomArgs& g, int kind, int coef_kind, double coef_value,
                        const double* coef_q, double* qd64, float* qd32, uint16_t* qd16,
                        int* err_flag, hipStream_t s) {
  const int64_t n = g.ne * g.q * g.q * g.q;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_qdata, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, s, g, kind,
                     coef_kind, coef_value, coef_q, qd64, qd32, qd16, err_flag);
  return hipGetLastError();
}

hipError_t launch_qpoint_coords(const GeomArgs& g, double* xyz, hipStream_t s) {
  const int64_t n = g.ne * g.q * g.q * g.q;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_qpoint_coords, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, s, g,
                     xyz);
  return hipGetLastError();
}

hipError_t launch_diag_elem(int kind, int p, int q, const double* qd, const double* B,
                            const double* G, int64_t ne, double* dE, hipStream_t s) {
  switch (p) {
    case 1: return diag_p<1>(q, kind, qd, B, G, ne, dE, s);
    case 2: return diag_p<2>(q, kind, qd, B, G, ne, dE, s);
    case 3: return diag_p<3>(q, kind, qd, B, G, ne, dE, s);
    case 4: return diag_p<4>(q, kind, qd, B, G, ne, dE, s);
    case 5: return diag_p<5>(q, kind, qd, B, G, ne, dE, s);
    case 6: return diag_p<6>(q, kind, qd, B, G, ne, dE, s);
    case 7: return diag_p<7>(q, kind, qd, B, G, ne, dE, s);
    case 8: return diag_p<8>(q, kind, qd, B, G, ne, dE, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rhs_elem(const GeomArgs& g, int p, const double* B, const double* f_q,
                           double* bE, hipStream_t s) {
  switch (p) {
    case 1: return rhs_p<1>(g.q, g, B, f_q, bE, s);
    case 2: return rhs_p<2>(g.q, g, B, f_q, bE, s);
    case 3: return rhs_p<3>(g.q, g, B, f_q, bE, s);
    case 4: return rhs_p<4>(g.q, g, B, f_q, bE, s);
    case 5: return rhs_p<5>(g.q, g, B, f_q, bE, s);
    case 6: return rhs_p<6>(g.q, g, B, f_q, bE, s);
    case 7: return rhs_p<7>(g.q, g, B, f_q, bE, s);
    case 8: return rhs_p<8>(g.q, g, B, f_q, bE, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pafem
