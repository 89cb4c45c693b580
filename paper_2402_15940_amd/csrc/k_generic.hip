// Element kernel for a quadrature size other than the default q = p + 2
// (p + 1 <= q <= 10), with p and q taken at run time: the same operator
// decomposition A = P^T G^T B^T D B G P (the paper's operator decomposition
// figure, partial assembly) as the tuned kernels of apply_impl.h, evaluated by
// plain sum factorization through LDS, one workgroup per element.  It serves
// operators created with a non-default q1d; the tuned kernels, their tables
// and launch shapes are specialised for q = p + 2.
//
// Stages (x fastest in every array; "B"/"G" the 1D value/derivative tables
// [q][n] of the operator, staged in LDS):
//   gather u[c][b][a] from x on the lattice numbering (essential dofs zero
//   for the constrained operator), then
//   1. along x:  Bu, Gu            [c][b][qx]
//   2. along y:  BBu, BGu, GBu     [c][qy][qx]
//   3. along z:  the reference gradient (or value) at every point, times D
//   3T, 2T, 1T: the transposed contractions back to [c][b][a], written to the
//   E-vector (element-major or x-interleaved) or added to y with atomics.
#include "internal.h"

namespace pafem {

namespace {

constexpr int kGenThreads = 256;
constexpr int kGenMaxN = kMaxP + 1;
// LDS words: tables, stage-1 (2 N^2 Q), stage-2 (3 N Q^2) and stage-3 (3 Q^3)
// regions at the largest sizes
constexpr int kGenLds = 2 * kMaxQ1d * kGenMaxN + 2 * kGenMaxN * kGenMaxN * kMaxQ1d +
                        3 * kGenMaxN * kMaxQ1d * kMaxQ1d + 3 * kMaxQ1d * kMaxQ1d * kMaxQ1d;

template <typename T>
__global__ __launch_bounds__(kGenThreads) void k_apply_generic(ApplyArgs<T> a, int p, int q,
                                                               int kind, int out_mode) {
  __shared__ T smem[kGenLds];
  if (a.skip != nullptr && *a.skip) return;
  const int N = p + 1, Q = q;
  const int NN = N * N, NNN = N * N * N, QQ = Q * Q, QQQ = Q * Q * Q;
  const bool diff = kind == PAFEM_DIFFUSION;
  T* sB = smem;                 // [Q][N]
  T* sG = sB + Q * N;           // [Q][N]
  T* r1 = sG + Q * N;           // 2 x [c][b][qx]
  T* r2 = r1 + 2 * NN * Q;      // 3 x [c][qy][qx]
  T* r3 = r2 + 3 * N * QQ;      // 3 x [qz][qy][qx]; also holds u before stage 1
  const int64_t e = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t t1 = e / a.nx;
  const int ex = (int)(e - t1 * a.nx), ey = (int)(t1 % a.ny), ez = (int)(t1 / a.ny);
  const int Lx = a.nx * p + 1, Ly = a.ny * p + 1, Lz = a.nz * p + 1;
  const int I0 = ex * p, J0 = ey * p, K0 = ez * p;
  for (int i = tid; i < Q * N; i += kGenThreads) {
    sB[i] = a.B[i];
    sG[i] = a.G[i];
  }
  T* u = r3;
  for (int i = tid; i < NNN; i += kGenThreads) {
    const int aa = i % N, b = (i / N) % N, c = i / NN;
    const int I = I0 + aa, J = J0 + b, K = K0 + c;
    const int64_t g = I + (int64_t)Lx * (J + (int64_t)Ly * K);
    const bool ess = I == 0 || I == Lx - 1 || J == 0 || J == Ly - 1 || K == 0 || K == Lz - 1;
    u[i] = (a.constrained && ess) ? T(0) : a.x[g];
  }
  __syncthreads();
  // 1: along x
  for (int i = tid; i < NN * Q; i += kGenThreads) {
    const int qx = i % Q, cb = i / Q;
    T sb = 0, sg = 0;
    for (int aa = 0; aa < N; ++aa) {
      const T v = u[cb * N + aa];
      sb = fma(sB[qx * N + aa], v, sb);
      sg = fma(sG[qx * N + aa], v, sg);
    }
    r1[i] = sb;
    if (diff) r1[NN * Q + i] = sg;
  }
  __syncthreads();
  // 2: along y
  for (int i = tid; i < N * QQ; i += kGenThreads) {
    const int qx = i % Q, qy = (i / Q) % Q, c = i / QQ;
    T bb = 0, bg = 0, gb = 0;
    for (int b = 0; b < N; ++b) {
      const T vb = r1[(c * N + b) * Q + qx];
      bb = fma(sB[qy * N + b], vb, bb);
      if (diff) {
        const T vg = r1[NN * Q + (c * N + b) * Q + qx];
        bg = fma(sB[qy * N + b], vg, bg);
        gb = fma(sG[qy * N + b], vb, gb);
      }
    }
    r2[i] = bb;
    if (diff) {
      r2[N * QQ + i] = bg;  // G along x, B along y
      r2[2 * N * QQ + i] = gb;
    }
  }
  __syncthreads();
  // 3: along z, then D at the point
  for (int i = tid; i < QQQ; i += kGenThreads) {
    const int qxy = i % QQ, qz = i / QQ;
    if (diff) {
      T gx = 0, gy = 0, gz = 0;
      for (int c = 0; c < N; ++c) {
        gx = fma(sB[qz * N + c], r2[N * QQ + c * QQ + qxy], gx);
        gy = fma(sB[qz * N + c], r2[2 * N * QQ + c * QQ + qxy], gy);
        gz = fma(sG[qz * N + c], r2[c * QQ + qxy], gz);
      }
      const T* d = a.qd + e * (6 * (int64_t)QQQ) + i;
      const T d0 = d[0], d1 = d[QQQ], d2 = d[2 * QQQ], d3 = d[3 * QQQ], d4 = d[4 * QQQ],
              d5 = d[5 * QQQ];
      r3[i] = fma(d0, gx, fma(d1, gy, d2 * gz));
      r3[QQQ + i] = fma(d1, gx, fma(d3, gy, d4 * gz));
      r3[2 * QQQ + i] = fma(d2, gx, fma(d4, gy, d5 * gz));
    } else {
      T v = 0;
      for (int c = 0; c < N; ++c) v = fma(sB[qz * N + c], r2[c * QQ + qxy], v);
      r3[i] = v * a.qd[e * (int64_t)QQQ + i];
    }
  }
  __syncthreads();
  // 3T: along z (G for the z-derivative path)
  for (int i = tid; i < N * QQ; i += kGenThreads) {
    const int qxy = i % QQ, c = i / QQ;
    T tx = 0, ty = 0, tz = 0;
    for (int qz = 0; qz < Q; ++qz) {
      tx = fma(sB[qz * N + c], r3[qz * QQ + qxy], tx);
      if (diff) {
        ty = fma(sB[qz * N + c], r3[QQQ + qz * QQ + qxy], ty);
        tz = fma(sG[qz * N + c], r3[2 * QQQ + qz * QQ + qxy], tz);
      }
    }
    r2[i] = tx;
    if (diff) {
      r2[N * QQ + i] = ty;
      r2[2 * N * QQ + i] = tz;
    }
  }
  __syncthreads();
  // 2T: along y; the x path (G along x later) and the sum of the y and z
  // paths (B along x later)
  for (int i = tid; i < NN * Q; i += kGenThreads) {
    const int qx = i % Q, b = (i / Q) % N, c = i / (N * Q);
    T sx = 0, syz = 0;
    for (int qy = 0; qy < Q; ++qy) {
      const int o = c * QQ + qy * Q + qx;
      sx = fma(sB[qy * N + b], r2[o], sx);
      if (diff) {
        syz = fma(sG[qy * N + b], r2[N * QQ + o], syz);
        syz = fma(sB[qy * N + b], r2[2 * N * QQ + o], syz);
      }
    }
    r1[i] = sx;
    if (diff) r1[NN * Q + i] = syz;
  }
  __syncthreads();
  // 1T: along x, and the output
  for (int i = tid; i < NNN; i += kGenThreads) {
    const int aa = i % N, cb = i / N;
    T y = 0;
    for (int qx = 0; qx < Q; ++qx) {
      if (diff) {
        y = fma(sG[qx * N + aa], r1[cb * Q + qx], y);
        y = fma(sB[qx * N + aa], r1[NN * Q + cb * Q + qx], y);
      } else {
        y = fma(sB[qx * N + aa], r1[cb * Q + qx], y);
      }
    }
    const int b = cb % N, c = cb / N;
    if (out_mode == kScatterEvector) {
      a.yE[e * NNN + i] = y;
    } else if (out_mode == kScatterXRows) {
      a.yE[xrows_index(a.nx, a.ny, N, ex, ey, ez, aa, b, c)] = y;
    } else {
      const int I = I0 + aa, J = J0 + b, K = K0 + c;
      const bool ess = I == 0 || I == Lx - 1 || J == 0 || J == Ly - 1 || K == 0 || K == Lz - 1;
      if (!(a.constrained && ess))
        atomicAdd(a.y + (I + (int64_t)Lx * (J + (int64_t)Ly * K)), y);
    }
  }
}

}  // namespace

template <typename T>
hipError_t launch_apply_generic(int kind, int p, int q, int scatter_mode, const ApplyArgs<T>& a,
                                hipStream_t s) {
  if (p < 1 || p > kMaxP || q < p + 1 || q > kMaxQ1d) return hipErrorInvalidValue;
  if (scatter_mode != PAFEM_SCATTER_ATOMIC && scatter_mode != kScatterEvector &&
      scatter_mode != kScatterXRows)
    return hipErrorInvalidValue;
  if (a.mf || a.qd16 != nullptr || a.qd == nullptr || a.x == nullptr || a.B == nullptr ||
      a.G == nullptr)
    return hipErrorInvalidValue;
  if (scatter_mode == PAFEM_SCATTER_ATOMIC ? a.y == nullptr : a.yE == nullptr)
    return hipErrorInvalidValue;
  if (a.ne == 0) return hipSuccess;
  hipLaunchKernelGGL((k_apply_generic<T>), dim3((unsigned)a.ne), dim3(kGenThreads), 0, s, a, p,
                     q, kind, scatter_mode);
  return hipGetLastError();
}
template hipError_t launch_apply_generic<double>(int, int, int, int, const ApplyArgs<double>&,
                                                 hipStream_t);
template hipError_t launch_apply_generic<float>(int, int, int, int, const ApplyArgs<float>&,
                                                hipStream_t);

}  // namespace pafem
