// Internal declarations of the pafem library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pafem.h"

namespace pafem {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
void clear_error();

// Status carrying a pafem error code; converted to the C return value.
#define PAFEM_TRY_HIP(expr)                                                             \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess) {                                                             \
      ::pafem::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));            \
      return _e == hipErrorOutOfMemory ? PAFEM_ERR_OUT_OF_MEMORY : PAFEM_ERR_HIP;       \
    }                                                                                   \
  } while (0)

#define PAFEM_TRY(expr)          \
  do {                           \
    int _rc = (expr);            \
    if (_rc != PAFEM_OK) return _rc; \
  } while (0)

// Device allocation owned by a library object.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
  // (Re)allocate at least `n` bytes; keeps the buffer if it is already large enough.
  int ensure(size_t n) {
    if (n <= bytes && ptr) return PAFEM_OK;
    release();
    if (n == 0) return PAFEM_OK;
    hipError_t e = hipMalloc(&ptr, n);
    if (e != hipSuccess) {
      ptr = nullptr;
      set_error("hipMalloc(" + std::to_string(n) + " bytes): " + hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? PAFEM_ERR_OUT_OF_MEMORY : PAFEM_ERR_HIP;
    }
    bytes = n;
    return PAFEM_OK;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(ptr); }
};

// ---------------------------------------------------------------------------
// host-side setup (basis.cpp, mesh.cpp)
// ---------------------------------------------------------------------------
constexpr int kMaxP = 8;
constexpr int kMaxQ1d = 10;  // largest quadrature size per direction
constexpr int kMaxQ = 12;

// Gauss-Lobatto-Legendre nodes on [0,1] (p+1 of them), by Newton's method on the
// Legendre three-term recurrence.
void gll_nodes(int p, double* x);
// Gauss-Legendre points and weights on [0,1] (weights sum to 1), Newton on P_q.
void gauss_legendre(int q, double* x, double* w);
// B[i][a] = l_a(x_i), G[i][a] = l_a'(x_i) for the Lagrange basis on `nodes`,
// evaluated with the barycentric form.
void lagrange_tables(int n, const double* nodes, int m, const double* x, double* B, double* G);

// Structured-lattice element restriction and friends.
void build_restriction(int nx, int ny, int nz, int p, std::vector<int32_t>& E);
void build_restriction_transpose(const std::vector<int32_t>& E, int64_t ndofs,
                                 std::vector<int32_t>& off, std::vector<int32_t>& idx);
void build_essential(int nx, int ny, int nz, int p, std::vector<int32_t>& ess,
                     std::vector<uint8_t>& mask);

// ---------------------------------------------------------------------------
// library objects
// ---------------------------------------------------------------------------
// Library objects are reference counted: the caller's handle holds one
// reference and every child (mesh of a context, space of a mesh, operator of a
// space) holds one on its parent, so handles may be destroyed in any order.
struct RefCounted {
  std::atomic<int> refs{1};
};

struct Ctx : RefCounted {
  int device = -1;
  bool host_only = true;
  DevBuf scratch;  // reduction partials for pafem_dot
};

struct Mesh : RefCounted {
  Ctx* ctx = nullptr;
  int nx = 0, ny = 0, nz = 0;
  std::vector<double> verts;
  DevBuf d_verts;
};

struct Space : RefCounted {
  Mesh* mesh = nullptr;
  int p = 0;
  int64_t ndofs = 0, ne = 0;
  // Integer maps, built on first use: the kernels compute the lattice
  // numbering themselves, so large meshes never pay for the stored maps
  // unless a caller asks for them.
  bool have_maps = false, have_dev_maps = false;  // E, E^T, essential mask
  bool have_ess = false, have_dev_ess = false;    // essential list
  std::vector<int32_t> E, et_off, et_idx, ess;
  std::vector<uint8_t> ess_mask;
  DevBuf d_E, d_et_off, d_et_idx, d_ess, d_ess_mask;
};

enum CoefKind { COEF_CONST = 0, COEF_QPTS = 1, COEF_SINX = 2 };

// Device-resident state of one Jacobi-PCG solve; all scalars live on the GPU so
// an iteration needs no host round trip.
struct CgState {
  double rz;       // r . z
  double pAp;      // p . A p
  double rr;       // r . r
  double alpha, beta;
  double rr_stop;  // stop when rr <= rr_stop
  double bb;       // b . b
  int iter;
  int done;        // 1: converged or out of iterations; 2: paused for a residual replacement
  int maxit;
  int pad;
  double rr_ref;   // r . r at the last residual replacement
  double delta2;   // pause when rr <= delta2 rr_ref (0: never)
  double rz_prev;  // r . z before the iteration that paused
};

// Device-resident scalars of the flexible CG of the p-multigrid solve.
struct FcgState {
  double rz;       // r . z
  double pw;       // p . A p
  double alpha, beta;
  double rr;       // r . r
  double rr_stop;  // converged when rr <= rr_stop
  int iter;
  int done;        // 1: converged on the recursive residual; 2: out of iterations
  int maxit;
  int pad;
};

struct Op : RefCounted {
  Space* space = nullptr;
  int kind = PAFEM_DIFFUSION;
  int level = PAFEM_ASSEMBLY_PARTIAL;  // or PAFEM_ASSEMBLY_MATRIX_FREE
  int q = 0;
  int ncomp = 6;
  int coef_kind = COEF_CONST;
  double coef_value = 1.0;
  DevBuf d_coef;                // [ne][q^3] when coef_kind == COEF_QPTS
  DevBuf d_tab64, d_tab32;      // B[q][n], G[q][n], pts[q], wts[q]
  DevBuf d_qd64, d_qd32, d_qd16; // quadrature data (FP64, rounded FP32 and bfloat16 copies)
  bool have64 = false, have32 = false, have16 = false;
  int scatter_mode = PAFEM_SCATTER_DETERMINISTIC;
  int index_mode = PAFEM_INDEX_LATTICE;
  DevBuf d_evec;                // E-vector workspace (deterministic scatter, diagonal, rhs)
  DevBuf d_flag;                // int error flag for assembly
  // solver workspace
  DevBuf d_cg;                  // vectors
  DevBuf d_part;                // reduction partials
  DevBuf d_gpart;               // per-workgroup partials of the element pass (fused CG)
  DevBuf d_state;               // CgState
  DevBuf d_dinv64, d_dinv32;
  bool have_dinv = false;
  // captured CG iterations (PAFEM_LAUNCH_GRAPH): the graph, the stream it was
  // captured on and what it was captured for
  hipGraphExec_t cg_graph = nullptr;
  hipStream_t cap_stream = nullptr;
  const void* cg_graph_key[10] = {};
  // persistent CG (PAFEM_LAUNCH_PERSISTENT): workgroup partials, barrier, error flag
  DevBuf d_pers;
  ~Op() {
    if (cg_graph) (void)hipGraphExecDestroy(cg_graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

// Shared host helpers (api.cpp).
int ensure_host_maps(Space* sp);
int ensure_device_maps(Space* sp);
int ensure_ess(Space* sp, bool device);
// qprec selects the stored quadrature data for float vectors: PAFEM_FP32 or PAFEM_BF16.
// With `work` (at least apply_work_bytes) the deterministic E^T on the lattice
// numbering runs with that E-vector workspace and nothing is allocated;
// otherwise the op's scatter and restriction modes apply.
template <typename T>
int apply_impl(Op* op, const T* x, T* y, int flags, const int* skip, hipStream_t s,
               int qprec = 0, void* work = nullptr);
int diagonal_impl(Op* op, double* d, int constrained, hipStream_t s);
// Device address of the allocation-free apply's workspace on `device` (current),
// looked up once per device (noalloc.hip).
int noalloc_init(int device);

// ---------------------------------------------------------------------------
// kernel launchers (k_*.hip)
// ---------------------------------------------------------------------------
struct GeomArgs {
  const double* verts;  // [(nx+1)(ny+1)(nz+1)][3]
  int nx, ny, nz;
  int64_t ne;
  int q;
  const double* pts;  // [q]
  const double* wts;  // [q]
};

// Quadrature data (and optionally physical qpoint coordinates).
hipError_t launch_qdata(const GeomArgs& g, int kind, int coef_kind, double coef_value,
                        const double* coef_q, double* qd64, float* qd32, uint16_t* qd16,
                        int* err_flag, hipStream_t s);
hipError_t launch_qpoint_coords(const GeomArgs& g, double* xyz, hipStream_t s);

template <typename T>
struct ApplyArgs {
  const T* x;
  T* y;               // L-vector output (atomic mode)
  T* yE;              // E-vector output (deterministic mode)
  const int32_t* E;
  const uint8_t* ess_mask;
  const T* qd;
  const uint16_t* qd16;  // bfloat16 quadrature data instead of qd (float kernels), or null
  const T* B;         // [q][n]
  const T* G;         // [q][n]
  int64_t ne;
  int nx, ny, nz;     // element lattice (lattice-computed restriction)
  int constrained;
  int accumulate;     // atomic mode: y holds a previous result to add to
  const int* skip;    // if non-null and *skip != 0, the kernel does nothing
  double* dot_part;   // if non-null: per workgroup, sum over its elements of x_e . y_e
  // fully matrix-free form (mf != 0): D recomputed at every quadrature point
  // from the corner vertices instead of read from qd
  int mf;
  int coef_kind;      // COEF_CONST or COEF_SINX
  double coef_value;
  const double* verts;  // [(nx+1)(ny+1)(nz+1)][3]
  const double* qpts;   // [q] Gauss points on [0,1]
  const double* qwts;   // [q] their weights
  // element pass on a CG direction formed on the fly (persistent CG):
  // the input is dir_dinv .* dir_r + beta x
  const T* dir_r;
  const T* dir_dinv;
};

// Tables of the element kernels for order p (n = p+1 nodes, q = p+2 points):
// B and G [q][n], then, for B and for G, the mirror-split tables of the
// contractions (see apply_impl.h), with nh = n/2, nhe = n - n/2 and the same
// for q:  Pf [qhe][nhe], Mf [qhe][nh]   (over the nodes, to the points)
//         Pt [nhe][qhe], Mt [nhe][qh]   (over the points, to the nodes)
__host__ __device__ constexpr int mir_words(int p) {
  const int n = p + 1, q = p + 2, nh = n / 2, nhe = n - n / 2, qh = q / 2, qhe = q - q / 2;
  return qhe * nhe + qhe * nh + nhe * qhe + nhe * qh;
}
__host__ __device__ constexpr int tab_len(int p) { return 2 * (p + 2) * (p + 1) + 2 * mir_words(p); }
// Offset of order p's tables in the concatenation over p = 1..8, and its length.
__host__ __device__ constexpr int tab_off(int p) {
  int o = 0;
  for (int k = 1; k < p; ++k) o += tab_len(k);
  return o;
}
__host__ __device__ constexpr int tab_words() { return tab_off(kMaxP + 1); }

// Fill the constant-memory tables of the element kernels (one copy per
// translation unit) on the current device: t64/t32 hold the tables of
// p = 1..8 at tab_off(p).
hipError_t upload_tables_apply(const double* t64, const float* t32, size_t words);
hipError_t upload_tables_batched(const double* t64, const float* t32, size_t words);

// Internal output modes of the element pass: the full E-vector
// [ne][(p+1)^3] (element results before assembly, pafem_op_apply_evector and
// the stored-map deterministic E^T), and the same values with element rows
// interleaved along x, [ez][ey][c][b][ex][a] (lattice numbering only), so that
// the ordered per-node sum reads consecutive words for consecutive nodes.
constexpr int kScatterEvector = 2;
constexpr int kScatterXRows = 3;
// kScatterXRows plus per-workgroup partials of x . (A x) for CG (a.dot_part).
constexpr int kScatterXRowsDot = 4;

// Words per element run of the x-interleaved layout (runs may be padded so
// that they fill whole memory sectors).
#ifndef PAFEM_XROWS_PAD7
#define PAFEM_XROWS_PAD7 7
#endif
__host__ __device__ constexpr int xrows_width(int n) { return n == 7 ? PAFEM_XROWS_PAD7 : n; }

// Division of a non-negative 31-bit integer by a divisor d >= 2 fixed at
// launch, as a multiply-high and a shift (no integer divide instruction on
// the GPU): with s = ceil(log2 d) and m = ceil(2^(31+s) / d) < 2^32,
// floor(n / d) = floor(n m / 2^(31+s)) exactly for 0 <= n < 2^31, since
// m d - 2^(31+s) < d <= 2^s makes the excess of n m / 2^(31+s) over n / d
// smaller than 1/d.
struct FastDiv {
  uint32_t m = 0;
  int s = 1;
  int d = 2;
  FastDiv() = default;
  explicit FastDiv(int divisor) : d(divisor) {
    s = 0;
    while ((1LL << s) < (long long)divisor) ++s;
    const unsigned long long num = 1ULL << (31 + s);
    m = (uint32_t)((num + (unsigned long long)divisor - 1) / (unsigned long long)divisor);
  }
  __host__ __device__ __forceinline__ int div(int n) const {
    return (int)((uint32_t)(((uint64_t)(uint32_t)n * m) >> 32) >> (s - 1));
  }
};

// Words of an E-vector buffer for either layout: ne (p+1)^2 max(p+1, width).
inline int64_t evec_words(int64_t ne, int n) { return ne * n * n * xrows_width(n); }

// Bytes of E-vector workspace one apply with elements of type T needs.
template <typename T>
inline int64_t apply_work_bytes(const Op* op) {
  return evec_words(op->space->ne, op->space->p + 1) * (int64_t)sizeof(T);
}

// Offset of local node (a, b, c) of element (ex, ey, ez) in the x-interleaved
// layout (< evec_words < 2^31).
__host__ __device__ __forceinline__ int xrows_index(int nx, int ny, int n, int ex, int ey, int ez,
                                                    int a, int b, int c) {
  const int w = xrows_width(n);
  return (((ez * ny + ey) * n + c) * n + b) * (nx * w) + ex * w + a;
}

// y (atomic) or yE (deterministic) from one fused sum-factorized element pass.
// q = p + 2 runs the tuned kernels; p + 1 <= q <= kMaxQ1d otherwise runs the
// run-time-sized kernel (k_generic.hip: atomic, element-major or
// x-interleaved output; no bfloat16 data, no matrix-free level, no CG dot).
template <typename T>
hipError_t launch_apply(int kind, int p, int q, int scatter_mode, int index_mode,
                        const ApplyArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_apply_generic(int kind, int p, int q, int scatter_mode, const ApplyArgs<T>& a,
                                hipStream_t s);

// Element-diagonal (E-vector) by sum factorization.
hipError_t launch_diag_elem(int kind, int p, int q, const double* qd, const double* B,
                            const double* G, int64_t ne, double* dE, hipStream_t s);
// RHS element vectors b_e = B^T (w detJ f) with the geometry recomputed.
hipError_t launch_rhs_elem(const GeomArgs& g, int p, const double* B, const double* f_q,
                           double* bE, hipStream_t s);

// Deterministic E^T: y[i] (+)= sum over E^T row i of yE (fixed order);
// constrained rows take x[i] (or 0 when x == nullptr) instead of the sum.
template <typename T>
hipError_t launch_gather_et(const T* yE, const int32_t* off, const int32_t* idx,
                            const uint8_t* ess_mask, int constrained, int accumulate, const T* x,
                            T* y, int64_t ndofs, const int* skip, hipStream_t s);
// The same sum with the E-vector positions of each dof computed from the
// lattice (same ascending (e, l) order, so bitwise equal to the CSR form).
template <typename T>
hipError_t launch_gather_lattice(const T* yE, int nx, int ny, int nz, int p, int constrained,
                                 int accumulate, const T* x, T* y, const int* skip,
                                 hipStream_t s);
// The same sum from the x-interleaved layout.
// nt: non-temporal E-vector loads (see evec_nt_loads); nt_y: non-temporal
// stores of y (see y_nt_stores).
template <typename T>
hipError_t launch_gather_xrows(const T* yX, int nx, int ny, int nz, int p, int constrained,
                               int accumulate, const T* x, T* y, const int* skip, hipStream_t s,
                               bool nt = false, bool nt_y = false);

// E-vector loads of the ordered sums, by p, for FP64 diffusion operators:
// 1 = non-temporal, 0 = ordinary.  Measured on MI355X: non-temporal loads
// shorten the p=6 FP64 diffusion apply by 5% and lengthen every other order,
// the FP32 applies and the mass applies by 1-10%.  The p=6 gain needs other
// device memory to have been written before the first apply (other
// quadrature data, the FP32 copy, any application data); in a process whose
// only device writes were this operator's assembly they cost 4% instead.
#ifndef PAFEM_NT_EVEC_DIFF64_BY_P
#define PAFEM_NT_EVEC_DIFF64_BY_P 0, 0, 0, 0, 0, 0, 1, 0, 0
#endif
inline bool evec_nt_loads(int kind, int p, bool f64) {
  constexpr int by_p[] = {PAFEM_NT_EVEC_DIFF64_BY_P};
  return kind == PAFEM_DIFFUSION && f64 && p >= 1 && p <= 8 && by_p[p] != 0;
}
// Stores of y in the ordered sum of an apply, by p, for the FP64 diffusion
// and mass operators: 1 = non-temporal, 0 = ordinary; FP32 applies always
// store non-temporally.  Measured on MI355X: non-temporal stores shorten the
// applies by 1-4% except FP64 diffusion at p = 6, 8 and FP64 mass at p >= 6,
// where they cost up to 1%.
#ifndef PAFEM_NT_Y_DIFF64_BY_P
#define PAFEM_NT_Y_DIFF64_BY_P 0, 1, 1, 1, 1, 1, 0, 1, 0
#endif
#ifndef PAFEM_NT_Y_MASS64_BY_P
#define PAFEM_NT_Y_MASS64_BY_P 0, 1, 1, 1, 1, 1, 0, 0, 0
#endif
inline bool y_nt_stores(int kind, int p, bool f64) {
  constexpr int diff[] = {PAFEM_NT_Y_DIFF64_BY_P};
  constexpr int mass[] = {PAFEM_NT_Y_MASS64_BY_P};
  if (p < 1 || p > 8) return false;
  if (!f64) return true;
  return (kind == PAFEM_DIFFUSION ? diff[p] : mass[p]) != 0;
}

// Essential-dof fix-up: y[ess[i]] (+)= x ? x[ess[i]] : value.
template <typename T>
hipError_t launch_set_ess(const int32_t* ess, int64_t n_ess, const T* x, T value, int accumulate,
                          T* y, const int* skip, hipStream_t s);
// y[0..n) = value (a kernel, so it may be recorded in a graph).
template <typename T>
hipError_t launch_fill(T* y, int64_t n, T value, const int* skip, hipStream_t s);

// Reductions: fixed grid, per-block partials, then one-block fixed-order finish.
int reduce_blocks(int64_t n);
template <typename T>
hipError_t launch_dot_partial(const T* x, const T* y, int64_t n, double* partials, int nb,
                              const int* skip, hipStream_t s);
hipError_t launch_sum_final(const double* partials, int nb, int ncols, double* out,
                            hipStream_t s);

// CG building blocks.
template <typename T>
hipError_t launch_cg_init(const T* r, const T* dinv, T* p, int64_t n, double* partials, int nb,
                          hipStream_t s);
// bb_dev, when given, is read on the device in place of bb (b . b stays there).
hipError_t launch_cg_init_final(const double* partials, int nb, double bb, double rtol,
                                int maxit, CgState* st, hipStream_t s, double delta2 = 0.0,
                                const double* bb_dev = nullptr);
// One CG step fused into the ordered E^T sum of the x-interleaved E-vector
// yX of A p: x += alpha p, r -= alpha A p, and fixed-partition partials of
// (r . dinv r, r . r) (*nparts pairs, at most kMaxCgParts).  A p is not stored.
constexpr int kMaxCgParts = 4096;
template <typename T, typename TX>
hipError_t launch_gather_xrows_cg(const T* yX, int nx, int ny, int nz, int p, const T* pvec,
                                  TX* x, T* r, const T* dinv, double* partials, int* nparts,
                                  const CgState* st, hipStream_t s, bool nt = false);
// alpha from nb partials of p . A p (one 1024-thread workgroup).
hipError_t launch_cg_alpha_wide(const double* partials, int nb, CgState* st, hipStream_t s);
// Element pass of A p for CG (deterministic E^T, lattice numbering): writes the
// x-interleaved E-vector and per-workgroup partials of p_e . (A p)_e to
// op->d_gpart; returns their count in *nparts.
template <typename T>
int apply_elements_dot(Op* op, const T* p, const int* skip, hipStream_t s, int qprec,
                       int* nparts);
// Argument block of the FP64 CG element pass of A p (constrained, x-interleaved
// E-vector, one partial of p . A p per element group) and the group count.
int cg_element_args(Op* op, const double* p, ApplyArgs<double>* out, int64_t* groups);
// Workgroups of the element pass of `kind`, order p, over ne elements.
int64_t element_blocks(int kind, int p, int64_t ne, bool f32);

// Mixed-precision CG: replace the FP32 recursive residual by rs = (float) r64
// (r64 = b - A x in FP64), leaving partials of (rs . dinv rs, r64 . r64), and
// (st non-null) finish the paused iteration's scalars from them.
hipError_t launch_replace_residual(const double* r64, const float* dinv, float* rs, int64_t n,
                                   double* partials, int nb, CgState* st, hipStream_t s);
hipError_t launch_cg_alpha(const double* partials, int nb, CgState* st, hipStream_t s);
template <typename TX, typename T>
hipError_t launch_cg_update(TX* x, T* r, const T* p, const T* Ap, const T* dinv, int64_t n,
                            double* partials, int nb, const CgState* st, hipStream_t s);
hipError_t launch_cg_beta(const double* partials, int nb, CgState* st, hipStream_t s);
template <typename T>
hipError_t launch_cg_pupdate(T* p, const T* r, const T* dinv, int64_t n, const CgState* st,
                             hipStream_t s);

// ---------------------------------------------------------------------------
// batched kernels of the serving engine (k_batched.hip)
// ---------------------------------------------------------------------------
constexpr int kBatchThreads = 256;   // workgroup size of every batched kernel
constexpr int kBatchChunk = 2048;    // dofs per vector chunk (8 per thread)

// One active request of a batch: the CG vectors of one Poisson solve in
// precision T and where its work items sit in the batch's index spaces.
template <typename T>
struct BatchEntry {
  ApplyArgs<T> a;           // x = CG direction, y = A dir, yE = E-vector workspace
  int p;
  int nchunks;
  int64_t ndofs;
  int64_t work_begin, work_end;    // element work items [begin, end) of the batched apply
  int64_t chunk_begin, chunk_end;  // vector chunks [begin, end)
  T* x;
  T* r;
  T* dir;
  T* Ad;
  const T* dinv;
  CgState* st;
  double* partials;         // [nchunks][2]
  double* x64;              // non-null: the solution is accumulated here in FP64 (mixed CG)
};

struct BatchHeader {
  int n;                    // active entries (sorted by work_begin / chunk_begin)
  int pad;
  int64_t total_work;
  int64_t total_chunks;
  int64_t p_begin[kMaxP + 1], p_end[kMaxP + 1];  // work items of the entries of order p
};

// Elements per work item of the batched apply for order p in precision T (the
// tuned elements-per-workgroup of the single-operator kernel).
template <typename T>
int batch_elems(int p);

// K CG iterations for every active entry of the batch; grids are fixed so the
// sequence can be captured once and replayed while the membership changes.
template <typename T>
hipError_t launch_batch_iterations(const BatchEntry<T>* ents, const BatchHeader* hdr,
                                   int max_entries, int iters, hipStream_t s);

// Mixed-precision helpers.
hipError_t launch_residual(const double* b, const double* Ax, double* r, int64_t n,
                           hipStream_t s, const int* skip = nullptr);
// *flag = 1 while the CG of st runs, 0 once it is done.
hipError_t launch_running_flag(const CgState* st, int* flag, hipStream_t s);
hipError_t launch_scale_to_f32(const double* r, const double* norm2, float* r32, int64_t n,
                               hipStream_t s);
hipError_t launch_axpy_from_f32(double* x, const double* norm2, const float* d32, int64_t n,
                                hipStream_t s);
hipError_t launch_recip(const double* d, double* dinv64, float* dinv32, int64_t n,
                        hipStream_t s);

// p-multigrid kernels (k_transfer.hip).  Orders pc = pf / 2; I1 is the
// [pf+1][pc+1] interpolation table from the coarse to the fine GLL nodes.
hipError_t launch_prolong(int pc, int pf, const double* uc, double* uf, int nx, int ny, int nz,
                          const double* I1, int accumulate, const int* skip, hipStream_t s);
// Per-element P^T of the fine values each element owns, into the coarse
// x-interleaved E-vector (then summed per coarse node by launch_gather_xrows).
hipError_t launch_restrict_elem(int pc, int pf, const double* rf, double* rcX, int nx, int ny,
                                int nz, const double* I1, const int* skip, hipStream_t s);
hipError_t launch_cheb_init(const double* b, const double* dinv, double* d, double* t, double c0,
                            int64_t n, hipStream_t s);
hipError_t launch_cheb_step(double* x, double* t, double* d, const double* w, const double* dinv,
                            double c1, double c2, int first, int64_t n, hipStream_t s);
hipError_t launch_fcg_update(double* x, double* r, const double* p, const double* w,
                             const FcgState* st, int64_t n, double* part, int nb, hipStream_t s);
hipError_t launch_fcg_dots(const double* z, const double* w, const double* r, int64_t n,
                           double* part, int nb, hipStream_t s);
hipError_t launch_fcg_init_dots(const double* r, const double* z, int64_t n, double* part, int nb,
                                hipStream_t s);
hipError_t launch_fcg_scalars(const double* part, int nb, int stage, FcgState* st, hipStream_t s);
hipError_t launch_fcg_pupdate(double* p, const double* z, const FcgState* st, int64_t n,
                              hipStream_t s);
// Power iteration helpers: v = pseudo-random in [-1, 1) (counter-based hash
// of the index); partials of (v . w, v . v / dinv, (dinv w) . (dinv w)); and
// v = scale dinv w.
hipError_t launch_hash_fill(double* v, int64_t n, uint64_t seed, hipStream_t s);
hipError_t launch_power_dots(const double* v, const double* w, const double* dinv, int64_t n,
                             double* part, int nb, hipStream_t s);
hipError_t launch_power_next(double* v, const double* w, const double* dinv, double scale,
                             int64_t n, hipStream_t s);

// Up to `iters` FP64 Jacobi-PCG iterations in one cooperative persistent
// launch (k_persistent.hip); *grid receives the workgroup count (<= max_blocks).
// bar points to kPersistentBarrierBytes of barrier words whose arrival
// counters are zero on entry (and again on return; the generations may hold
// anything).
constexpr size_t kPersistentBarrierBytes = 18 * 128;
hipError_t launch_pcg_persistent(int kind, int p, const ApplyArgs<double>& a, int64_t groups,
                                 double* xs, double* r, const double* dinv, double* bpart,
                                 double* npart, CgState* st, void* bar, int* err,
                                 long long spin_limit, int iters, int max_blocks, int* grid,
                                 hipStream_t s);
hipError_t upload_tables_persistent(const double* t64, const float* t32, size_t words);

// Solver helpers (solver.cpp).
int ensure_dinv(Op* op, hipStream_t s, bool want32);
// Exactly `iters` Jacobi-PCG steps (fewer only if the residual vanishes) on
// the constrained FP64 operator from x = 0, with no host synchronization:
// r holds the right-hand side on entry and is overwritten; p and Ap are work
// vectors of length ndofs.
int pcg_fixed(Op* op, double* r, double* x, double* p, double* Ap, int iters, hipStream_t s);
// ||b - A x||_2 / ||b||_2 in FP64 (synchronous; Ax and r are scratch vectors).
int relative_residual(Op* op, const double* b, const double* x, double* Ax, double* r,
                      hipStream_t s, double& out);

}  // namespace pafem

// The C handles are the library objects themselves.
struct pafem_ctx : pafem::Ctx {};
struct pafem_mesh : pafem::Mesh {};
struct pafem_space : pafem::Space {};
struct pafem_op : pafem::Op {};
