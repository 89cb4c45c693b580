// Quadrature-data assembly (the data partial assembly stores) and quadrature
// point coordinates.  One thread per (element, quadrature point).
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

// MASS:       D = w rho detJ
// DIFFUSION:  D = w k adj(J) adj(J)^T / detJ, upper triangle xx xy xz yy yz zz
// adj(J) is the adjugate (transposed cofactor matrix), so adj(J)/detJ = J^-1.
__global__ __launch_bounds__(kThreads) void k_qdata(GeomArgs g, int kind, int coef_kind,
                                                    double coef_value,
                                                    const double* __restrict__ coef_q,
                                                    double* __restrict__ qd64,
                                                    float* __restrict__ qd32,
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
  if (kind == PAFEM_MASS) {
    const double d = w * k * det;
    qd64[e * qqq + qp] = d;
    if (qd32) qd32[e * qqq + qp] = (float)d;
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

}  // namespace

hipError_t launch_qdata(const GeomArgs& g, int kind, int coef_kind, double coef_value,
                        const double* coef_q, double* qd64, float* qd32, int* err_flag,
                        hipStream_t s) {
  const int64_t n = g.ne * g.q * g.q * g.q;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_qdata, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, s, g, kind,
                     coef_kind, coef_value, coef_q, qd64, qd32, err_flag);
  return hipGetLastError();
}

hipError_t launch_qpoint_coords(const GeomArgs& g, double* xyz, hipStream_t s) {
  const int64_t n = g.ne * g.q * g.q * g.q;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_qpoint_coords, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, s, g,
                     xyz);
  return hipGetLastError();
}

}  // namespace pafem
