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
#define PAFEM_NE_BY_Q 1, 1, 1, 7, 4, 5, 7, 5, 1, 3, 1
#endif
#ifndef PAFEM_WAVES_DIFF_F64
#define PAFEM_WAVES_DIFF_F64 1, 1, 1, 1, 3, 1, 1, 1, 1
#endif
constexpr int kNeByQ[] = {PAFEM_NE_BY_Q};
// quadrature-data loads by p: 1 = non-temporal (streamed past the caches),
// 0 = ordinary
#ifndef PAFEM_NT_QD_BY_P
#define PAFEM_NT_QD_BY_P 1, 1, 1, 0, 0, 0, 1, 0, 1
#endif
constexpr int kNtQd[] = {PAFEM_NT_QD_BY_P};
constexpr int kWavesDiff64[] = {PAFEM_WAVES_DIFF_F64};
// the mass kernel's own tables, measured separately (8M dofs, p = 1..8):
// elements per workgroup by q and the quadrature-data load type by p
#ifndef PAFEM_NE_MASS_BY_Q
#define PAFEM_NE_MASS_BY_Q 1, 1, 1, 7, 4, 8, 7, 5, 4, 3, 4
#endif
#ifndef PAFEM_NT_QD_MASS_BY_P
#define PAFEM_NT_QD_MASS_BY_P 1, 1, 1, 0, 1, 1, 1, 1, 1
#endif
constexpr int kNeMassByQ[] = {PAFEM_NE_MASS_BY_Q};
constexpr int kNtQdMass[] = {PAFEM_NT_QD_MASS_BY_P};
// the same for the element pass that also forms the CG dot product
#ifndef PAFEM_WAVES_DIFF_F64_DOT
#define PAFEM_WAVES_DIFF_F64_DOT 1, 1, 1, 1, 3, 3, 1, 1, 1
#endif
constexpr int kWavesDiff64Dot[] = {PAFEM_WAVES_DIFF_F64_DOT};

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

// ---- mirror split of the 1D contractions ----------------------------------
// The GLL nodes and the Gauss points lie symmetrically about the element
// centre, so T[Q-1-q][N-1-i] = S T[q][i] with S = +1 for B and -1 for G.
// With e_i = u_i + u_{N-1-i}, o_i = u_i - u_{N-1-i} (i < N/2; for odd N, e
// also carries the middle value), a contraction y_q = sum_i T[q][i] u_i is
//   E_q = sum_i P[q][i] e_i,  O_q = sum_i M[q][i] o_i   (q < ceil(Q/2))
//   y_q = E_q + O_q,  y_{Q-1-q} = S (E_q - O_q)          (q < Q/2)
// with P, M the halved sums and differences of mirrored table entries: about
// half the multiply-adds of the plain contraction.  The transposed
// contraction (over the points, to the nodes) has the same form with the
// roles of N and Q exchanged.
template <int N>
struct Mir {
  static constexpr int H = N / 2;        // mirror pairs
  static constexpr int HE = N - N / 2;   // pairs, and the middle when N is odd
};

// The split tables of order P for table t (0: B, 1: G), in constant memory.
template <typename T, int P>
struct SplitTab {
  static constexpr int N = P + 1, Q = P + 2;
  static constexpr int NH = Mir<N>::H, NHE = Mir<N>::HE, QH = Mir<Q>::H, QHE = Mir<Q>::HE;
  __device__ static const T* Pf(int t) { return ctab<T>(P) + 2 * Q * N + t * mir_words(P); }
  __device__ static const T* Mf(int t) { return Pf(t) + QHE * NHE; }
  __device__ static const T* Pt(int t) { return Mf(t) + QHE * NH; }
  __device__ static const T* Mt(int t) { return Pt(t) + NHE * QHE; }
};

template <int N, typename T>
__device__ __forceinline__ void mirror(const T (&u)[N], T (&e)[Mir<N>::HE], T (&o)[Mir<N>::H]) {
#pragma unroll
  for (int i = 0; i < Mir<N>::H; ++i) {
    e[i] = u[i] + u[N - 1 - i];
    o[i] = u[i] - u[N - 1 - i];
  }
  if (N % 2) e[Mir<N>::H] = u[Mir<N>::H];
}

// y[NO] from the split (e, o) of a vector of length NI; Pt [OHE][IHE], Mt [OHE][IH].
template <int NI, int NO, int S, typename T>
__device__ __forceinline__ void contract(const T* __restrict__ Ptab, const T* __restrict__ Mtab,
                                         const T (&e)[Mir<NI>::HE], const T (&o)[Mir<NI>::H],
                                         T (&y)[NO]) {
  constexpr int IH = Mir<NI>::H, IHE = Mir<NI>::HE, OH = Mir<NO>::H, OHE = Mir<NO>::HE;
#pragma unroll
  for (int j = 0; j < OHE; ++j) {
    T E = 0, O = 0;
#pragma unroll
    for (int i = 0; i < IHE; ++i) E = fma(Ptab[j * IHE + i], e[i], E);
#pragma unroll
    for (int i = 0; i < IH; ++i) O = fma(Mtab[j * IH + i], o[i], O);
    y[j] = E + O;
    if (j < OH) y[NO - 1 - j] = S > 0 ? E - O : O - E;
  }
}

__host__ __device__ constexpr int odd_up(int v) { return (v % 2 == 0) ? v + 1 : v; }
__host__ __device__ constexpr int cmax(int a, int b) { return a > b ? a : b; }


template <int P, int Q, typename T, int KIND>
struct Cfg {
  static constexpr int N = P + 1;
  static constexpr int QQ = Q * Q;
  static constexpr int R = KIND == PAFEM_DIFFUSION ? odd_up(cmax(2 * N, 3 * Q)) : odd_up(cmax(N, Q));
  static constexpr int L = N * Q * R;  // LDS words per element
  static constexpr int NE = KIND == PAFEM_DIFFUSION ? kNeByQ[Q] : kNeMassByQ[Q];
  static constexpr int THREADS = ((NE * QQ + 63) / 64) * 64;
  // waves per SIMD the register allocation must allow (occupancy floor)
  static constexpr int MIN_WAVES =
      (KIND == PAFEM_DIFFUSION && sizeof(T) == 8) ? kWavesDiff64[P] : 1;
  static constexpr int MIN_WAVES_DOT =
      (KIND == PAFEM_DIFFUSION && sizeof(T) == 8) ? kWavesDiff64Dot[P] : 1;
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
  if constexpr (SCATTER == kScatterXRows || SCATTER == kScatterXRowsDot) {
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

// Partials of x . (A x) for CG (kScatterXRowsDot).  With u = B x_e at the
// quadrature points of an element (x masked on the essential dofs) and D the
// pointwise data, x_e . (A_e x_e) = sum_q u_q . (D_q u_q): stage C has both
// factors in registers, so the dot product needs no pass over A x.  The
// constrained operator is the identity on essential rows, which adds x_i^2
// for each of them; stage A sees x_i before the mask, and the element that
// owns the node counts it (lowest local index in each direction, the last
// element keeping its far face).
template <int P, typename T>
__device__ __forceinline__ bool owns_node(const Restrict<P, PAFEM_INDEX_LATTICE, T>& E,
                                          const ApplyArgs<T>& a, int aa, int b, int c) {
  return (aa < P || E.ex == a.nx - 1) && (b < P || E.ey == a.ny - 1) &&
         (c < P || E.ez == a.nz - 1);
}

// Sum of v over the workgroup into a.dot_part[block]; every thread calls it.
__device__ __forceinline__ void workgroup_dot(double* dot_part, double v, int64_t block) {
  __shared__ double red[16];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x % 64, wid = threadIdx.x / 64, nw = (blockDim.x + 63) / 64;
  if (nw == 1) {
    if (lane == 0) dot_part[block] = v;
    return;
  }
  if (lane == 0) red[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[w];
    dot_part[block] = t;
  }
}

// ---------------------------------------------------------------------------
// Fully matrix-free D along one stage-C line (qx, qy) of an element.  The
// trilinear map is linear in each reference coordinate, so the Jacobian
// column d x / d s does not depend on s (likewise for t and u): along the line
// (s, t fixed) c1(u) = E0 + dE u, c2(u) = F0 + dF u and c3 is constant.  With
// the adjugate rows r0 = c2 x c3, r1 = c3 x c1, r2 = c1 x c2 and
// detJ = c1 . r0, diffusion needs w k (r_a . r_b) / detJ and mass w k detJ.
// ---------------------------------------------------------------------------
template <typename T>
struct MfLine {
  T E0[3], dE[3], F0[3], dF[3], C3[3];
  T X0, dX, wxy;
  __device__ __forceinline__ void init(const ApplyArgs<T>& a, int64_t e, int qx, int qy) {
    const int64_t t1 = e / a.nx;
    const int ex = (int)(e - t1 * a.nx), ey = (int)(t1 % a.ny), ez = (int)(t1 / a.ny);
    const int64_t sy = a.nx + 1, sz = (int64_t)(a.nx + 1) * (a.ny + 1);
    T v[2][2][2][3];  // [k (u)][j (t)][i (s)][coordinate]
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int d = 0; d < 3; ++d)
            v[k][j][i][d] = (T)a.verts[((ex + i) + (ey + j) * sy + (ez + k) * sz) * 3 + d];
    const T s = (T)a.qpts[qx], t = (T)a.qpts[qy], s1 = T(1) - s, t1m = T(1) - t;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const T a0 = (v[0][0][1][d] - v[0][0][0][d]) * t1m + (v[0][1][1][d] - v[0][1][0][d]) * t;
      const T a1 = (v[1][0][1][d] - v[1][0][0][d]) * t1m + (v[1][1][1][d] - v[1][1][0][d]) * t;
      E0[d] = a0;
      dE[d] = a1 - a0;
      const T b0 = (v[0][1][0][d] - v[0][0][0][d]) * s1 + (v[0][1][1][d] - v[0][0][1][d]) * s;
      const T b1 = (v[1][1][0][d] - v[1][0][0][d]) * s1 + (v[1][1][1][d] - v[1][0][1][d]) * s;
      F0[d] = b0;
      dF[d] = b1 - b0;
      const T c00 = v[1][0][0][d] - v[0][0][0][d], c10 = v[1][0][1][d] - v[0][0][1][d];
      const T c01 = v[1][1][0][d] - v[0][1][0][d], c11 = v[1][1][1][d] - v[0][1][1][d];
      C3[d] = (c00 * s1 + c10 * s) * t1m + (c01 * s1 + c11 * s) * t;
    }
    const T f0 = (v[0][0][0][0] * s1 + v[0][0][1][0] * s) * t1m + (v[0][1][0][0] * s1 + v[0][1][1][0] * s) * t;
    const T f1 = (v[1][0][0][0] * s1 + v[1][0][1][0] * s) * t1m + (v[1][1][0][0] * s1 + v[1][1][1][0] * s) * t;
    X0 = f0;
    dX = f1 - f0;
    wxy = (T)(a.qwts[qx] * a.qwts[qy]);
  }
  // weight times coefficient, adjugate rows and detJ at point u = qpts[qz]
  __device__ __forceinline__ void at(const ApplyArgs<T>& a, int qz, T& wk, T (&r)[3][3],
                                     T& det) const {
    const T u = (T)a.qpts[qz];
    T c1[3], c2[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      c1[d] = E0[d] + dE[d] * u;
      c2[d] = F0[d] + dF[d] * u;
    }
    const T* c3 = C3;
    r[0][0] = c2[1] * c3[2] - c2[2] * c3[1];
    r[0][1] = c2[2] * c3[0] - c2[0] * c3[2];
    r[0][2] = c2[0] * c3[1] - c2[1] * c3[0];
    r[1][0] = c3[1] * c1[2] - c3[2] * c1[1];
    r[1][1] = c3[2] * c1[0] - c3[0] * c1[2];
    r[1][2] = c3[0] * c1[1] - c3[1] * c1[0];
    r[2][0] = c1[1] * c2[2] - c1[2] * c2[1];
    r[2][1] = c1[2] * c2[0] - c1[0] * c2[2];
    r[2][2] = c1[0] * c2[1] - c1[1] * c2[0];
    det = c1[0] * r[0][0] + c1[1] * r[0][1] + c1[2] * r[0][2];
    T k = (T)a.coef_value;
    if (a.coef_kind == COEF_SINX) k = T(1) + (T)a.coef_value * sin(T(2.0 * M_PI) * (X0 + dX * u));
    wk = wxy * (T)a.qwts[qz] * k;
  }
};

template <typename T, int Q>
__device__ __forceinline__ void mf_fill_diffusion(const ApplyArgs<T>& a, int64_t e, int qx, int qy,
                                                  T (&dq)[6][Q]) {
  MfLine<T> L;
  L.init(a, e, qx, qy);
#pragma unroll
  for (int qz = 0; qz < Q; ++qz) {
    T wk, r[3][3], det;
    L.at(a, qz, wk, r, det);
    const T f = wk / det;
    int m = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j)
        dq[m++][qz] = f * (r[i][0] * r[j][0] + r[i][1] * r[j][1] + r[i][2] * r[j][2]);
  }
}

template <typename T, int Q>
__device__ __forceinline__ void mf_fill_mass(const ApplyArgs<T>& a, int64_t e, int qx, int qy,
                                             T (&dq)[Q]) {
  MfLine<T> L;
  L.init(a, e, qx, qy);
#pragma unroll
  for (int qz = 0; qz < Q; ++qz) {
    T wk, r[3][3], det;
    L.at(a, qz, wk, r, det);
    dq[qz] = wk * det;
  }
}

// ---------------------------------------------------------------------------
// diffusion: y_e = sum_ij G_i^T S_ij G_j x_e, S = w k adj(J) adj(J)^T / detJ
// stored as the 6 upper-triangle entries per quadrature point.
// ---------------------------------------------------------------------------
// Elements e0 .. e0+NE-1 (those below a.ne) with the workgroup's threads;
// smem holds NE * L words.  Every thread of the workgroup must call it.
// QD16: the quadrature data is stored in bfloat16 (a.qd16; FP32 arithmetic).
template <int P, int Q, typename T, int SCATTER, int IDX, int NE, bool QD16 = false,
          bool MF = false, bool DIR = false>
__device__ __forceinline__ void diff_elements(const ApplyArgs<T>& a, int64_t e0, T* smem,
                                              int tid, T dir_beta = T(0)) {
  using C = Cfg<P, Q, T, PAFEM_DIFFUSION>;
  constexpr int N = C::N, QQ = C::QQ, L = C::L, R = C::R;
  constexpr int QQQ = Q * Q * Q;
  using ST = SplitTab<T, P>;
  constexpr int HN = Mir<N>::HE, LN = Mir<N>::H, HQ = Mir<Q>::HE, LQ = Mir<Q>::H;

  constexpr bool DOT = SCATTER == kScatterXRowsDot;
  double vd = 0.0;  // this thread's share of x . (A x) (DOT only)

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
  for (int b = 0; b < N; ++b) {
    const int32_t g = EA.dof(aA, b, cA);
    // DIR: the CG direction formed on the fly, dinv r + beta p (a.x = p)
    if constexpr (DIR)
      u[b] = a.dir_dinv[g] * a.dir_r[g] + dir_beta * a.x[g];
    else
      u[b] = a.x[g];
  }
  __builtin_amdgcn_sched_barrier(0);

  // Quadrature data of this thread's z-line: the dominant HBM stream, consumed
  // only in stage C, so it streams in while stages A and B run.
  T dq[6][Q];
  if constexpr (!MF) {
    const int64_t off = (actC ? eC : 0) * (6 * QQQ) + qyC * Q + qxC;
    if constexpr (QD16) {  // BF16 storage, FP32 arithmetic
      const uint16_t* qd = a.qd16 + off;
#pragma unroll
      for (int qz = 0; qz < Q; ++qz)
#pragma unroll
        for (int k = 0; k < 6; ++k)
          dq[k][qz] = (T)bf16_to_float(__builtin_nontemporal_load(qd + k * QQQ + qz * QQ));
    } else {
      // component-major issue order (each component's z-line is one run of
      // addresses); ordinary or non-temporal loads by p, as measured
      const T* qd = a.qd + off;
#pragma unroll
      for (int k = 0; k < 6; ++k) {
#pragma unroll
        for (int qz = 0; qz < Q; ++qz) {
          if constexpr (kNtQd[P] != 0)
            dq[k][qz] = __builtin_nontemporal_load(qd + k * QQQ + qz * QQ);
          else
            dq[k][qz] = qd[k * QQQ + qz * QQ];
        }
      }
    }
  }
  __builtin_amdgcn_sched_barrier(0);

  // ---- stage A: y contraction ----
  if (actA) {
#pragma unroll
    for (int b = 0; b < N; ++b) {  // a select, not a branch: no early wait on the loads
      const bool es = a.constrained && EA.ess(a, EA.dof(aA, b, cA), aA, b, cA);
      if constexpr (DOT) {
        const double ub = (es && owns_node<P>(EA, a, aA, b, cA)) ? (double)u[b] : 0.0;
        vd = fma(ub, ub, vd);
      }
      u[b] = es ? T(0) : u[b];
    }
    T* reg = smem + sA * L + (cA * Q) * R + aA;  // region (c, qy) at + qy*R
    T ue[HN], uo[LN], tb[Q], tg[Q];
    mirror<N>(u, ue, uo);
    contract<N, Q, 1>(ST::Pf(0), ST::Mf(0), ue, uo, tb);
    contract<N, Q, -1>(ST::Pf(1), ST::Mf(1), ue, uo, tg);
#pragma unroll
    for (int qy = 0; qy < Q; ++qy) {
      reg[qy * R] = tb[qy];
      reg[qy * R + N] = tg[qy];
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
    T be[HN], bo[LN], ge[HN], go[LN], bb[Q], gb[Q], bg[Q];  // factors (x, y): (B,B) (G,B) (B,G)
    mirror<N>(tb, be, bo);
    mirror<N>(tg, ge, go);
    contract<N, Q, 1>(ST::Pf(0), ST::Mf(0), be, bo, bb);
    contract<N, Q, -1>(ST::Pf(1), ST::Mf(1), be, bo, gb);
    contract<N, Q, 1>(ST::Pf(0), ST::Mf(0), ge, go, bg);
#pragma unroll
    for (int qx = 0; qx < Q; ++qx) {
      reg[qx] = bb[qx];
      reg[Q + qx] = gb[qx];
      reg[2 * Q + qx] = bg[qx];
    }
  }
  __syncthreads();

  // ---- stage C: z contraction, pointwise D, transposed z contraction ----
  if (actC) {
    if constexpr (MF) mf_fill_diffusion<T, Q>(a, eC, qxC, qyC, dq);
    T* reg0 = smem + sC * L + qyC * R + qxC;  // + c*Q*R + k*Q
    T ibb[N], igb[N], ibg[N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
      ibb[c] = reg0[c * Q * R];
      igb[c] = reg0[c * Q * R + Q];
      ibg[c] = reg0[c * Q * R + 2 * Q];
    }
    // mirror pairs of points (qz, Q-1-qz) are handled together: the split
    // forward contraction gives the reference gradient at both, D is applied
    // at both, and their sum and difference feed the split transposed one
    T bbe[HN], bbo[LN], gbe[HN], gbo[LN], bge[HN], bgo[LN];
    mirror<N>(ibb, bbe, bbo);
    mirror<N>(igb, gbe, gbo);
    mirror<N>(ibg, bge, bgo);
    const T* PfB = ST::Pf(0);
    const T* MfB = ST::Mf(0);
    const T* PfG = ST::Pf(1);
    const T* MfG = ST::Mf(1);
    const T* PtB = ST::Pt(0);
    const T* MtB = ST::Mt(0);
    const T* PtG = ST::Pt(1);
    const T* MtG = ST::Mt(1);
    T E1[HN], O1[HN], E2[HN], O2[HN], E3[HN], O3[HN];
#pragma unroll
    for (int i = 0; i < HN; ++i) E1[i] = O1[i] = E2[i] = O2[i] = E3[i] = O3[i] = 0;
    T vq = 0;  // sum over this z-line of grad . (D grad) (DOT only)
#pragma unroll
    for (int k = 0; k < HQ; ++k) {
      T ex = 0, ox = 0, ey = 0, oy = 0, ez = 0, oz = 0;
#pragma unroll
      for (int i = 0; i < HN; ++i) {
        ex = fma(PfB[k * HN + i], gbe[i], ex);
        ey = fma(PfB[k * HN + i], bge[i], ey);
        ez = fma(PfG[k * HN + i], bbe[i], ez);
      }
#pragma unroll
      for (int i = 0; i < LN; ++i) {
        ox = fma(MfB[k * LN + i], gbo[i], ox);
        oy = fma(MfB[k * LN + i], bgo[i], oy);
        oz = fma(MfG[k * LN + i], bbo[i], oz);
      }
      // point k
      const T gx0 = ex + ox, gy0 = ey + oy, gz0 = ez + oz;
      const T vx0 = fma(dq[0][k], gx0, fma(dq[1][k], gy0, dq[2][k] * gz0));
      const T vy0 = fma(dq[1][k], gx0, fma(dq[3][k], gy0, dq[4][k] * gz0));
      const T vz0 = fma(dq[2][k], gx0, fma(dq[4][k], gy0, dq[5][k] * gz0));
      if constexpr (DOT) vq = fma(gx0, vx0, fma(gy0, vy0, fma(gz0, vz0, vq)));
      if (k < LQ) {
        // its mirror Q-1-k
        const int m = Q - 1 - k;
        const T gx1 = ex - ox, gy1 = ey - oy, gz1 = oz - ez;
        const T vx1 = fma(dq[0][m], gx1, fma(dq[1][m], gy1, dq[2][m] * gz1));
        const T vy1 = fma(dq[1][m], gx1, fma(dq[3][m], gy1, dq[4][m] * gz1));
        const T vz1 = fma(dq[2][m], gx1, fma(dq[4][m], gy1, dq[5][m] * gz1));
        if constexpr (DOT) vq = fma(gx1, vx1, fma(gy1, vy1, fma(gz1, vz1, vq)));
        const T fx = vx0 + vx1, gxd = vx0 - vx1, fy = vy0 + vy1, gyd = vy0 - vy1;
        const T fz = vz0 + vz1, gzd = vz0 - vz1;
#pragma unroll
        for (int i = 0; i < HN; ++i) {
          E1[i] = fma(PtB[i * HQ + k], fx, E1[i]);
          O1[i] = fma(MtB[i * LQ + k], gxd, O1[i]);
          E2[i] = fma(PtB[i * HQ + k], fy, E2[i]);
          O2[i] = fma(MtB[i * LQ + k], gyd, O2[i]);
          E3[i] = fma(PtG[i * HQ + k], fz, E3[i]);
          O3[i] = fma(MtG[i * LQ + k], gzd, O3[i]);
        }
      } else {  // the middle point of an odd Q
#pragma unroll
        for (int i = 0; i < HN; ++i) {
          E1[i] = fma(PtB[i * HQ + k], vx0, E1[i]);
          E2[i] = fma(PtB[i * HQ + k], vy0, E2[i]);
          E3[i] = fma(PtG[i * HQ + k], vz0, E3[i]);
        }
      }
    }
    if constexpr (DOT) vd += (double)vq;
#pragma unroll
    for (int i = 0; i < HN; ++i) {
      reg0[i * Q * R] = E1[i] + O1[i];
      reg0[i * Q * R + Q] = E2[i] + O2[i];
      reg0[i * Q * R + 2 * Q] = E3[i] + O3[i];
      if (i < LN) {
        const int m = N - 1 - i;
        reg0[m * Q * R] = E1[i] - O1[i];
        reg0[m * Q * R + Q] = E2[i] - O2[i];
        reg0[m * Q * R + 2 * Q] = O3[i] - E3[i];
      }
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
    T f1[HQ], g1[LQ], f2[HQ], g2[LQ], f3[HQ], g3[LQ], s1[N], s3[N], s2[N];
    mirror<Q>(w1, f1, g1);
    mirror<Q>(w2, f2, g2);
    mirror<Q>(w3, f3, g3);
    contract<Q, N, -1>(ST::Pt(1), ST::Mt(1), f1, g1, s1);
    contract<Q, N, 1>(ST::Pt(0), ST::Mt(0), f3, g3, s3);
    contract<Q, N, 1>(ST::Pt(0), ST::Mt(0), f2, g2, s2);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      reg[i] = s1[i] + s3[i];
      reg[N + i] = s2[i];
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
    T f13[HQ], g13[LQ], f2[HQ], g2[LQ], a13[N], a2[N], acc[N];
    mirror<Q>(X13, f13, g13);
    mirror<Q>(X2, f2, g2);
    contract<Q, N, 1>(ST::Pt(0), ST::Mt(0), f13, g13, a13);
    contract<Q, N, -1>(ST::Pt(1), ST::Mt(1), f2, g2, a2);
#pragma unroll
    for (int b = 0; b < N; ++b) acc[b] = a13[b] + a2[b];
    Restrict<P, IDX, T> E;
    E.init(a, eA);
    store_line<P, SCATTER, IDX>(a, E, eA, aA, cA, acc);
  }
  if constexpr (DOT) workgroup_dot(a.dot_part, vd, e0 / NE);
}

// ---------------------------------------------------------------------------
// mass: y_e = B^T D B x_e with D = w rho detJ.
// ---------------------------------------------------------------------------
template <int P, int Q, typename T, int SCATTER, int IDX, int NE, bool QD16 = false,
          bool MF = false, bool DIR = false>
__device__ __forceinline__ void mass_elements(const ApplyArgs<T>& a, int64_t e0, T* smem,
                                              int tid, T dir_beta = T(0)) {
  using C = Cfg<P, Q, T, PAFEM_MASS>;
  constexpr int N = C::N, QQ = C::QQ, L = C::L, R = C::R;
  constexpr int QQQ = Q * Q * Q;
  using ST = SplitTab<T, P>;
  constexpr int HN = Mir<N>::HE, LN = Mir<N>::H, HQ = Mir<Q>::HE, LQ = Mir<Q>::H;

  constexpr bool DOT = SCATTER == kScatterXRowsDot;
  double vd = 0.0;  // this thread's share of x . (A x) (DOT only)

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
  for (int b = 0; b < N; ++b) {
    const int32_t g = EA.dof(aA, b, cA);
    // DIR: the CG direction formed on the fly, dinv r + beta p (a.x = p)
    if constexpr (DIR)
      u[b] = a.dir_dinv[g] * a.dir_r[g] + dir_beta * a.x[g];
    else
      u[b] = a.x[g];
  }
  __builtin_amdgcn_sched_barrier(0);

  T dq[Q];
  if constexpr (!MF) {
    const int64_t off = (actC ? eC : 0) * QQQ + qyC * Q + qxC;
    if constexpr (QD16) {
      const uint16_t* qd = a.qd16 + off;
#pragma unroll
      for (int qz = 0; qz < Q; ++qz) dq[qz] = (T)bf16_to_float(__builtin_nontemporal_load(qd + qz * QQ));
    } else {
      const T* qd = a.qd + off;
#pragma unroll
      for (int qz = 0; qz < Q; ++qz) {
        if constexpr (kNtQdMass[P] != 0)
          dq[qz] = __builtin_nontemporal_load(qd + qz * QQ);
        else
          dq[qz] = qd[qz * QQ];
      }
    }
  }
  __builtin_amdgcn_sched_barrier(0);

  if (actA) {
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const bool es = a.constrained && EA.ess(a, EA.dof(aA, b, cA), aA, b, cA);
      if constexpr (DOT) {
        const double ub = (es && owns_node<P>(EA, a, aA, b, cA)) ? (double)u[b] : 0.0;
        vd = fma(ub, ub, vd);
      }
      u[b] = es ? T(0) : u[b];
    }
    T* reg = smem + sA * L + (cA * Q) * R + aA;
    T ue[HN], uo[LN], tb[Q];
    mirror<N>(u, ue, uo);
    contract<N, Q, 1>(ST::Pf(0), ST::Mf(0), ue, uo, tb);
#pragma unroll
    for (int qy = 0; qy < Q; ++qy) reg[qy * R] = tb[qy];
  }
  __syncthreads();

  const int sB = tid / (Q * N), rB = tid - sB * (Q * N);
  const bool actB = sB < NE && e0 + sB < a.ne;
  const int qyB = rB % Q, cB = rB / Q;
  if (actB) {
    T* reg = smem + sB * L + (cB * Q + qyB) * R;
    T tb[N], be[HN], bo[LN], bb[Q];
#pragma unroll
    for (int i = 0; i < N; ++i) tb[i] = reg[i];
    mirror<N>(tb, be, bo);
    contract<N, Q, 1>(ST::Pf(0), ST::Mf(0), be, bo, bb);
#pragma unroll
    for (int qx = 0; qx < Q; ++qx) reg[qx] = bb[qx];
  }
  __syncthreads();

  if (actC) {
    if constexpr (MF) mf_fill_mass<T, Q>(a, eC, qxC, qyC, dq);
    T* reg0 = smem + sC * L + qyC * R + qxC;
    T in[N], ie[HN], io[LN], E[HN], O[HN];
#pragma unroll
    for (int c = 0; c < N; ++c) in[c] = reg0[c * Q * R];
    mirror<N>(in, ie, io);
    const T* PfB = ST::Pf(0);
    const T* MfB = ST::Mf(0);
    const T* PtB = ST::Pt(0);
    const T* MtB = ST::Mt(0);
#pragma unroll
    for (int i = 0; i < HN; ++i) E[i] = O[i] = 0;
    T vq = 0;  // sum over this z-line of u . (D u) (DOT only)
#pragma unroll
    for (int k = 0; k < HQ; ++k) {  // mirror pairs of points (see diff_elements)
      T e = 0, o = 0;
#pragma unroll
      for (int i = 0; i < HN; ++i) e = fma(PfB[k * HN + i], ie[i], e);
#pragma unroll
      for (int i = 0; i < LN; ++i) o = fma(MfB[k * LN + i], io[i], o);
      const T v0 = dq[k] * (e + o);
      if constexpr (DOT) vq = fma(e + o, v0, vq);
      if (k < LQ) {
        const T v1 = dq[Q - 1 - k] * (e - o);
        if constexpr (DOT) vq = fma(e - o, v1, vq);
        const T f = v0 + v1, g = v0 - v1;
#pragma unroll
        for (int i = 0; i < HN; ++i) {
          E[i] = fma(PtB[i * HQ + k], f, E[i]);
          O[i] = fma(MtB[i * LQ + k], g, O[i]);
        }
      } else {
#pragma unroll
        for (int i = 0; i < HN; ++i) E[i] = fma(PtB[i * HQ + k], v0, E[i]);
      }
    }
    if constexpr (DOT) vd += (double)vq;
#pragma unroll
    for (int i = 0; i < HN; ++i) {
      reg0[i * Q * R] = E[i] + O[i];
      if (i < LN) reg0[(N - 1 - i) * Q * R] = E[i] - O[i];
    }
  }
  __syncthreads();

  if (actB) {
    T* reg = smem + sB * L + (cB * Q + qyB) * R;
    T w[Q], f[HQ], g[LQ], s1[N];
#pragma unroll
    for (int qx = 0; qx < Q; ++qx) w[qx] = reg[qx];
    mirror<Q>(w, f, g);
    contract<Q, N, 1>(ST::Pt(0), ST::Mt(0), f, g, s1);
#pragma unroll
    for (int i = 0; i < N; ++i) reg[i] = s1[i];
  }
  __syncthreads();

  if (actA) {
    const T* reg = smem + sA * L + (cA * Q) * R + aA;
    T W[Q];
#pragma unroll
    for (int qy = 0; qy < Q; ++qy) W[qy] = reg[qy * R];
    T f[HQ], g[LQ], acc[N];  // contracted before the first store (see diff_elements)
    mirror<Q>(W, f, g);
    contract<Q, N, 1>(ST::Pt(0), ST::Mt(0), f, g, acc);
    Restrict<P, IDX, T> E;
    E.init(a, eA);
    store_line<P, SCATTER, IDX>(a, E, eA, aA, cA, acc);
  }
  if constexpr (DOT) workgroup_dot(a.dot_part, vd, e0 / NE);
}

}  // namespace apply
}  // namespace pafem
