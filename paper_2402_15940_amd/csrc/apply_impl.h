// Device bodies of the fused partial-assembly element kernels (shared by the
// per-operator launches and the batched serving launch).
//
// y = E^T B^T D B E x, per element:
//
// Each element runs through five stages; every stage gives one thread one 1D
// line of the element and the full 1D table, so the tables are wave-uniform
// (scalar-register operands) and LDS carries each intermediate exactly once:
//
//   A   y contraction   line (a, c):   gather x_e(a, :, c)  -> B x, G x      (per qy)
//   B   x contraction   line (qy, c):  -> (B,B) (G,B) (B,G) factors         (per qx)
//   C   z contraction   line (qx, qy): -> reference gradient at every qz,
//                                         pointwise D (6 stored factors),
//                                         transposed z contraction
//   B^T x contraction   line (qy, c)
//   A^T y contraction   line (a, c):   -> y_e(a, :, c)  -> scatter (E^T)
//
// Lanes of stages A/A^T run along x, so the gather and the scatter-add touch
// consecutive dofs; lanes of stage C run along qx, so the quadrature-data
// stream is read in contiguous runs.
//
// LDS holds, per element, one private region of R words for every (c, qy)
// pair; each stage reads its line's inputs from the regions it owns and
// writes its outputs back into the same regions, so one buffer of N*Q*R words
// serves every stage (R = max(2N, 3Q) rounded up to an odd count, which keeps
// 64-bit LDS accesses with a line stride of R conflict-free).
//
// The element restriction E is either the stored int32 map or computed from
// the lattice coordinates of the structured mesh (no index traffic, and the x
// loads can be issued at kernel start together with the quadrature data).
#pragma once

#include "internal.h"

namespace pafem {

namespace apply {

constexpr int kXcds = 8;  // MI355X: 8 accelerator complex dies, one L2 each

// Launch tuning, measured on MI355X (overridable at build time for sweeps):
// elements per workgroup by q, and the waves per SIMD the register allocation
// must leave room for, by p, for the FP64 diffusion kernel.
#ifndef PAFEM_NE_BY_Q
#define PAFEM_NE_BY_Q 1, 1, 1, 7, 4, 5, 7, 5, 1, 3, 2
#endif
#ifndef PAFEM_WAVES_DIFF_F64
#define PAFEM_WAVES_DIFF_F64 1, 1, 1, 1, 4, 1, 1, 1, 1
#endif
constexpr int kNeByQ[] = {PAFEM_NE_BY_Q};
constexpr int kWavesDiff64[] = {PAFEM_WAVES_DIFF_F64};

// The 1D tables B[q][n], G[q][n] (q = p+2 Gauss-Legendre points, n = p+1 GLL
// nodes) depend on p alone, so every element kernel reads them from constant
// memory, [p = 1..8][B then G]: scalar loads the compiler may repeat anywhere
// (no store can clobber them), whatever the origin of the other pointers.
// Each translation unit that includes this header holds its own copy, filled
// by its upload_tables_* function when a context is created.
constexpr int kTabWords = tab_words();
static __constant__ double c_tab64[kTabWords];
static __constant__ float c_tab32[kTabWords];
template <typename T>
__device__ __forceinline__ const T* ctab(int p);
template <>
__device__ __forceinline__ const double* ctab<double>(int p) { return c_tab64 + tab_off(p); }
template <>
__device__ __forceinline__ const float* ctab<float>(int p) { return c_tab32 + tab_off(p); }

__host__ __device__ constexpr int odd_up(int v) { return (v % 2 == 0) ? v + 1 : v; }
__host__ __device__ constexpr int cmax(int a, int b) { return a > b ? a : b; }


template <int P, int Q, typename T, int KIND>
struct Cfg {
  static constexpr int N = P + 1;
  static constexpr int QQ = Q * Q;
  static constexpr int R = KIND == PAFEM_DIFFUSION ? odd_up(cmax(2 * N, 3 * Q)) : odd_up(cmax(N, Q));
  static constexpr int L = N * Q * R;  // LDS words per element
  static constexpr int NE = kNeByQ[Q];
  static constexpr int THREADS = ((NE * QQ + 63) / 64) * 64;
  // waves per SIMD the register allocation must allow (occupancy floor)
  static constexpr int MIN_WAVES =
      (KIND == PAFEM_DIFFUSION && sizeof(T) == 8) ? kWavesDiff64[P] : 1;
  static_assert(NE * L * (int)sizeof(T) <= 64 * 1024, "LDS budget");
};

// Workgroups are dealt to the XCDs round-robin; renumber them so that each XCD
// works on one contiguous run of elements (neighbours share face dofs in the
// XCD's L2 for both the x gather and the y scatter).
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t x = b % kXcds, k = b / kXcds;
  const int64_t q = nb / kXcds, r = nb % kXcds;
  return x * q + (x < r ? x : r) + k;
}

// Element restriction E of one element: the stored map row, or the lattice
// numbering of the structured mesh computed on the fly.
template <int P, int IDX, typename T>
struct Restrict {
  const int32_t* Ee;
  int ex, ey, ez;  // lattice element coordinates
  int I0, J0, K0;
  int Lx, Ly, Lz;
  __device__ __forceinline__ void init(const ApplyArgs<T>& a, int64_t e) {
    constexpr int N = P + 1;
    Lx = a.nx * P + 1;
    Ly = a.ny * P + 1;
    Lz = a.nz * P + 1;
    if (IDX == PAFEM_INDEX_MAP) {
      Ee = a.E + e * (N * N * N);
    } else {
      const int64_t t = e / a.nx;
      ex = (int)(e - t * a.nx);
      ey = (int)(t % a.ny);
      ez = (int)(t / a.ny);
      I0 = ex * P;
      J0 = ey * P;
      K0 = ez * P;
    }
  }
  __device__ __forceinline__ int32_t dof(int aa, int b, int c) const {
    constexpr int N = P + 1;
    if (IDX == PAFEM_INDEX_MAP) return Ee[(c * N + b) * N + aa];
    return (I0 + aa) + Lx * ((J0 + b) + Ly * (K0 + c));
  }
  __device__ __forceinline__ bool ess(const ApplyArgs<T>& a, int32_t g, int aa, int b,
                                      int c) const {
    if (IDX == PAFEM_INDEX_MAP) return a.ess_mask[g] != 0;
    const int I = I0 + aa, J = J0 + b, K = K0 + c;
    return I == 0 || I == Lx - 1 || J == 0 || J == Ly - 1 || K == 0 || K == Lz - 1;
  }
};

// bfloat16 bits (the upper half of an IEEE binary32) to float
__device__ __forceinline__ float bf16_to_float(uint16_t h) {
  return __uint_as_float((uint32_t)h << 16);
}

template <typename T>
__device__ __forceinline__ void scatter_add(T* p, T v) {
  atomicAdd(p, v);
}

// Where the element results of one y-line (a, :, c) go: the E-vector, as
// the output of the element pass itself or for the ordered per-node sum of
// the deterministic E^T (element-major with a stored map, x-interleaved with
// the lattice numbering), or global atomic adds into y (memory-side on MI355X).
template <int P, int SCATTER, int IDX, typename T>
__device__ __forceinline__ void store_line(const ApplyArgs<T>& a, const Restrict<P, IDX, T>& E,
                                           int64_t e, int aa, int c, const T (&acc)[P + 1]) {
  constexpr int N = P + 1;
  if constexpr (SCATTER == kScatterXRows) {
    static_assert(IDX == PAFEM_INDEX_LATTICE, "x-interleaved rows need the lattice numbering");
    T* out = a.yE + xrows_index(a.nx, a.ny, N, E.ex, E.ey, E.ez, aa, 0, c);
    const int stride = a.nx * xrows_width(N);
#pragma unroll
    for (int b = 0; b < N; ++b) out[b * stride] = acc[b];
  } else if constexpr (SCATTER != PAFEM_SCATTER_ATOMIC) {
    T* out = a.yE + e * (N * N * N) + c * N * N + aa;
#pragma unroll
    for (int b = 0; b < N; ++b) out[b * N] = acc[b];
  } else {
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const int32_t g = E.dof(aa, b, c);
      if (!(a.constrained && E.ess(a, g, aa, b, c))) scatter_add(a.y + g, acc[b]);
    }
  }
}

// ---------------------------------------------------------------------------
// diffusion: y_e = sum_ij G_i^T S_ij G_j x_e, S = w k adj(J) adj(J)^T / detJ
// stored as the 6 upper-triangle entries per quadrature point.
// ---------------------------------------------------------------------------
// Elements e0 .. e0+NE-1 (those below a.ne) with the workgroup's threads;
// smem holds NE * L words.  Every thread of the workgroup must call it.
// QD16: the quadrature data is stored in bfloat16 (a.qd16; FP32 arithmetic).
template <int P, int Q, typename T, int SCATTER, int IDX, int NE, bool QD16 = false>
__device__ __forceinline__ void diff_elements(const ApplyArgs<T>& a, int64_t e0, T* smem,
                                              int tid) {
  using C = Cfg<P, Q, T, PAFEM_DIFFUSION>;
  constexpr int N = C::N, QQ = C::QQ, L = C::L, R = C::R;
  constexpr int QQQ = Q * Q * Q;
  const T* __restrict__ Bt = ctab<T>(P);
  const T* __restrict__ Gt = ctab<T>(P) + Q * N;

  // stage-C role of this thread: z-line (qx, qy) of element slot sC
  const int sC = tid / QQ, rC = tid - sC * QQ;
  const int64_t eC = e0 + sC;
  const bool actC = sC < NE && eC < a.ne;
  const int qxC = rC % Q, qyC = rC / Q;

  // stage-A role: y-line (a, c); lanes run along x so gather and scatter coalesce
  const int sA = tid / (N * N), rA = tid - sA * (N * N);
  const int64_t eA = e0 + sA;
  const bool actA = sA < NE && eA < a.ne;
  const int aA = rA % N, cA = rA / N;

  // x gather of this thread's y-line, issued first and all at once: stage A
  // waits for it alone (vector loads complete in order); the essential-dof
  // mask is applied only after the quadrature-data loads are on their way
  // All loads are unconditional (idle threads read element 0): a branch around
  // them would make the compiler wait for every load before stage A.
  T u[N];
  Restrict<P, IDX, T> EA;
  EA.init(a, actA ? eA : 0);
#pragma unroll
  for (int b = 0; b < N; ++b) u[b] = a.x[EA.dof(aA, b, cA)];
  __builtin_amdgcn_sched_barrier(0);

  // Quadrature data of this thread's z-line: the dominant HBM stream, consumed
  // only in stage C, so it streams in while stages A and B run.
  T dq[6][Q];
  {
    const int64_t off = (actC ? eC : 0) * (6 * QQQ) + qyC * Q + qxC;
    if constexpr (QD16) {  // BF16 storage, FP32 arithmetic
      const uint16_t* qd = a.qd16 + off;
#pragma unroll
      for (int qz = 0; qz < Q; ++qz)
#pragma unroll
        for (int k = 0; k < 6; ++k)
          dq[k][qz] = (T)bf16_to_float(__builtin_nontemporal_load(qd + k * QQQ + qz * QQ));
    } else {
      // issued in the order stage C consumes them (qz outer), so it can start
      // on the first points while the rest are still arriving
      const T* qd = a.qd + off;
#pragma unroll
      for (int qz = 0; qz < Q; ++qz) {
#pragma unroll
        for (int k = 0; k < 6; ++k) dq[k][qz] = __builtin_nontemporal_load(qd + k * QQQ + qz * QQ);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  __builtin_amdgcn_sched_barrier(0);

  // ---- stage A: y contraction ----
  if (actA) {
#pragma unroll
    for (int b = 0; b < N; ++b)  // a select, not a branch: no early wait on the loads
      u[b] = (a.constrained && EA.ess(a, EA.dof(aA, b, cA), aA, b, cA)) ? T(0) : u[b];
    T* reg = smem + sA * L + (cA * Q) * R + aA;  // region (c, qy) at + qy*R
#pragma unroll
    for (int qy = 0; qy < Q; ++qy) {
      T tb = 0, tg = 0;
#pragma unroll
      for (int b = 0; b < N; ++b) {
        tb = fma(Bt[qy * N + b], u[b], tb);
        tg = fma(Gt[qy * N + b], u[b], tg);
      }
      reg[qy * R] = tb;
      reg[qy * R + N] = tg;
    }
  }
  __syncthreads();

  // ---- stage B: x contraction, x-line (qy, c) ----
  const int sB = tid / (Q * N), rB = tid - sB * (Q * N);
  const bool actB = sB < NE && e0 + sB < a.ne;
  const int qyB = rB % Q, cB = rB / Q;
  if (actB) {
    T* reg = smem + sB * L + (cB * Q + qyB) * R;
    T tb[N], tg[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      tb[i] = reg[i];
      tg[i] = reg[N + i];
    }
#pragma unroll
    for (int qx = 0; qx < Q; ++qx) {
      T bb = 0, gb = 0, bg = 0;  // factors (x, y): (B,B) (G,B) (B,G)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        bb = fma(Bt[qx * N + i], tb[i], bb);
        gb = fma(Gt[qx * N + i], tb[i], gb);
        bg = fma(Bt[qx * N + i], tg[i], bg);
      }
      reg[qx] = bb;
      reg[Q + qx] = gb;
      reg[2 * Q + qx] = bg;
    }
  }
  __syncthreads();

  // ---- stage C: z contraction, pointwise D, transposed z contraction ----
  if (actC) {
    T* reg0 = smem + sC * L + qyC * R + qxC;  // + c*Q*R + k*Q
    T ibb[N], igb[N], ibg[N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
      ibb[c] = reg0[c * Q * R];
      igb[c] = reg0[c * Q * R + Q];
      ibg[c] = reg0[c * Q * R + 2 * Q];
    }
    T w1[N], w2[N], w3[N];
#pragma unroll
    for (int c = 0; c < N; ++c) w1[c] = w2[c] = w3[c] = 0;
#pragma unroll
    for (int qz = 0; qz < Q; ++qz) {
      T gx = 0, gy = 0, gz = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) {
        gx = fma(Bt[qz * N + c], igb[c], gx);
        gy = fma(Bt[qz * N + c], ibg[c], gy);
        gz = fma(Gt[qz * N + c], ibb[c], gz);
      }
      const T vx = fma(dq[0][qz], gx, fma(dq[1][qz], gy, dq[2][qz] * gz));
      const T vy = fma(dq[1][qz], gx, fma(dq[3][qz], gy, dq[4][qz] * gz));
      const T vz = fma(dq[2][qz], gx, fma(dq[4][qz], gy, dq[5][qz] * gz));
#pragma unroll
      for (int c = 0; c < N; ++c) {
        w1[c] = fma(Bt[qz * N + c], vx, w1[c]);
        w2[c] = fma(Bt[qz * N + c], vy, w2[c]);
        w3[c] = fma(Gt[qz * N + c], vz, w3[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < N; ++c) {
      reg0[c * Q * R] = w1[c];
      reg0[c * Q * R + Q] = w2[c];
      reg0[c * Q * R + 2 * Q] = w3[c];
    }
  }
  __syncthreads();

  // ---- stage B^T: transposed x contraction, x-line (qy, c) ----
  // x-path needs G in x, the y- and z-paths B in x; afterwards the x- and
  // z-paths share B in y, so they are summed here.
  if (actB) {
    T* reg = smem + sB * L + (cB * Q + qyB) * R;
    T w1[Q], w2[Q], w3[Q];
#pragma unroll
    for (int qx = 0; qx < Q; ++qx) {
      w1[qx] = reg[qx];
      w2[qx] = reg[Q + qx];
      w3[qx] = reg[2 * Q + qx];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T s13 = 0, s2 = 0;
#pragma unroll
      for (int qx = 0; qx < Q; ++qx) {
        s13 = fma(Gt[qx * N + i], w1[qx], fma(Bt[qx * N + i], w3[qx], s13));
        s2 = fma(Bt[qx * N + i], w2[qx], s2);
      }
      reg[i] = s13;
      reg[N + i] = s2;
    }
  }
  __syncthreads();

  // ---- stage A^T: transposed y contraction + scatter, y-line (a, c) ----
  if (actA) {
    const T* reg = smem + sA * L + (cA * Q) * R + aA;
    T X13[Q], X2[Q];
#pragma unroll
    for (int qy = 0; qy < Q; ++qy) {
      X13[qy] = reg[qy * R];
      X2[qy] = reg[qy * R + N];
    }
    // the whole line is contracted before the first store: a global store
    // may alias the tables as far as the compiler can tell, and would force
    // every later table read onto the vector memory path
    T acc[N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
      acc[b] = 0;
#pragma unroll
      for (int qy = 0; qy < Q; ++qy)
        acc[b] = fma(Bt[qy * N + b], X13[qy], fma(Gt[qy * N + b], X2[qy], acc[b]));
    }
    Restrict<P, IDX, T> E;
    E.init(a, eA);
    store_line<P, SCATTER, IDX>(a, E, eA, aA, cA, acc);
  }
}

// ---------------------------------------------------------------------------
// mass: y_e = B^T D B x_e with D = w rho detJ.
// ---------------------------------------------------------------------------
template <int P, int Q, typename T, int SCATTER, int IDX, int NE, bool QD16 = false>
__device__ __forceinline__ void mass_elements(const ApplyArgs<T>& a, int64_t e0, T* smem,
                                              int tid) {
  using C = Cfg<P, Q, T, PAFEM_MASS>;
  constexpr int N = C::N, QQ = C::QQ, L = C::L, R = C::R;
  constexpr int QQQ = Q * Q * Q;
  const T* __restrict__ Bt = ctab<T>(P);

  const int sC = tid / QQ, rC = tid - sC * QQ;
  const int64_t eC = e0 + sC;
  const bool actC = sC < NE && eC < a.ne;
  const int qxC = rC % Q, qyC = rC / Q;
  const int sA = tid / (N * N), rA = tid - sA * (N * N);
  const int64_t eA = e0 + sA;
  const bool actA = sA < NE && eA < a.ne;
  const int aA = rA % N, cA = rA / N;
  T u[N];  // x gather first, unconditional, masked later (see diff_elements)
  Restrict<P, IDX, T> EA;
  EA.init(a, actA ? eA : 0);
#pragma unroll
  for (int b = 0; b < N; ++b) u[b] = a.x[EA.dof(aA, b, cA)];
  __builtin_amdgcn_sched_barrier(0);

  T dq[Q];
  {
    const int64_t off = (actC ? eC : 0) * QQQ + qyC * Q + qxC;
    if constexpr (QD16) {
      const uint16_t* qd = a.qd16 + off;
#pragma unroll
      for (int qz = 0; qz < Q; ++qz) dq[qz] = (T)bf16_to_float(__builtin_nontemporal_load(qd + qz * QQ));
    } else {
      const T* qd = a.qd + off;
#pragma unroll
      for (int qz = 0; qz < Q; ++qz) dq[qz] = __builtin_nontemporal_load(qd + qz * QQ);
    }
  }
  __builtin_amdgcn_sched_barrier(0);

  if (actA) {
#pragma unroll
    for (int b = 0; b < N; ++b)
      u[b] = (a.constrained && EA.ess(a, EA.dof(aA, b, cA), aA, b, cA)) ? T(0) : u[b];
    T* reg = smem + sA * L + (cA * Q) * R + aA;
#pragma unroll
    for (int qy = 0; qy < Q; ++qy) {
      T tb = 0;
#pragma unroll
      for (int b = 0; b < N; ++b) tb = fma(Bt[qy * N + b], u[b], tb);
      reg[qy * R] = tb;
    }
  }
  __syncthreads();

  const int sB = tid / (Q * N), rB = tid - sB * (Q * N);
  const bool actB = sB < NE && e0 + sB < a.ne;
  const int qyB = rB % Q, cB = rB / Q;
  if (actB) {
    T* reg = smem + sB * L + (cB * Q + qyB) * R;
    T tb[N];
#pragma unroll
    for (int i = 0; i < N; ++i) tb[i] = reg[i];
#pragma unroll
    for (int qx = 0; qx < Q; ++qx) {
      T bb = 0;
#pragma unroll
      for (int i = 0; i < N; ++i) bb = fma(Bt[qx * N + i], tb[i], bb);
      reg[qx] = bb;
    }
  }
  __syncthreads();

  if (actC) {
    T* reg0 = smem + sC * L + qyC * R + qxC;
    T in[N], w[N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
      in[c] = reg0[c * Q * R];
      w[c] = 0;
    }
#pragma unroll
    for (int qz = 0; qz < Q; ++qz) {
      T uq = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) uq = fma(Bt[qz * N + c], in[c], uq);
      const T v = dq[qz] * uq;
#pragma unroll
      for (int c = 0; c < N; ++c) w[c] = fma(Bt[qz * N + c], v, w[c]);
    }
#pragma unroll
    for (int c = 0; c < N; ++c) reg0[c * Q * R] = w[c];
  }
  __syncthreads();

  if (actB) {
    T* reg = smem + sB * L + (cB * Q + qyB) * R;
    T w[Q];
#pragma unroll
    for (int qx = 0; qx < Q; ++qx) w[qx] = reg[qx];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T s1 = 0;
#pragma unroll
      for (int qx = 0; qx < Q; ++qx) s1 = fma(Bt[qx * N + i], w[qx], s1);
      reg[i] = s1;
    }
  }
  __syncthreads();

  if (actA) {
    const T* reg = smem + sA * L + (cA * Q) * R + aA;
    T W[Q];
#pragma unroll
    for (int qy = 0; qy < Q; ++qy) W[qy] = reg[qy * R];
    T acc[N];  // contracted before the first store (see diff_elements)
#pragma unroll
    for (int b = 0; b < N; ++b) {
      acc[b] = 0;
#pragma unroll
      for (int qy = 0; qy < Q; ++qy) acc[b] = fma(Bt[qy * N + b], W[qy], acc[b]);
    }
    Restrict<P, IDX, T> E;
    E.init(a, eA);
    store_line<P, SCATTER, IDX>(a, E, eA, aA, cA, acc);
  }
}

}  // namespace apply
}  // namespace pafem
