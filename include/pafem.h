/*
 * pafem -- partial-assembly (sum-factorized) H1 mass and diffusion operators on
 * tensor-product hexahedral meshes, and the Jacobi-preconditioned CG solve
 * built on them, for AMD Instinct MI355X (gfx950).
 *
 * The operator follows the finite element operator decomposition of the paper
 * (figure "finite element operator decomposition": A = P^T G^T B^T D B G P).
 * On one GPU P is the identity; G is the element restriction (called E here,
 * to keep G free for the basis-gradient table), B/G are 1D basis value and
 * derivative tables applied by sum factorization, and D is the pointwise
 * quadrature data that partial assembly stores (section "State-of-the-art
 * performance on exascale platforms and AMD GPUs", the partial assembly
 * level).  The diagonal for Jacobi is computed by sum factorization (section
 * "Matrix-free solvers for high-order finite elements").
 *
 * Discretization fixed by this library (the paper does not state them):
 *   - reference element [0,1]^3, trilinear geometry from the 8 element corners;
 *   - nodal Lagrange basis of order p (1..8) on the p+1 Gauss-Lobatto-Legendre
 *     points per direction;
 *   - q Gauss-Legendre points per direction, q = p+2 (the only value accepted);
 *   - global dofs numbered lattice-lexicographically, x fastest: dof (I,J,K) of
 *     the (nx p+1) x (ny p+1) x (nz p+1) node lattice has number
 *     I + (nx p+1) (J + (ny p+1) K); elements e = ex + nx (ey + ny ez); local
 *     element dof l = a + (p+1) (b + (p+1) c); quadrature point
 *     qx + q (qy + q qz);
 *   - essential (Dirichlet) dofs: every node on the boundary of the mesh block.
 *
 * Conventions
 *   - Every call returns int: PAFEM_OK (0) or a negative PAFEM_ERR_* code;
 *     pafem_last_error() then holds a message (per calling thread).
 *   - Handles are opaque, owned by the library, released by *_destroy.  Objects
 *     are reference counted: a mesh keeps its context alive, a space its mesh
 *     and an operator its space, so handles may be destroyed in any order.
 *   - Vectors passed as "_dev" are device pointers owned by the caller,
 *     contiguous, of the element type stated; the library never frees them.
 *     "_host" pointers are host memory, copied before the call returns.
 *   - `stream` is a hipStream_t passed as void* (NULL = the legacy default
 *     stream).  Calls that take a stream only enqueue work on it unless the
 *     comment says "synchronous".
 *   - A context created with device = -1 is host-only: mesh, space and map
 *     queries work without a GPU; anything that touches device memory returns
 *     PAFEM_ERR_UNSUPPORTED.
 */
#ifndef PAFEM_H
#define PAFEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------------- */
#define PAFEM_OK 0
#define PAFEM_ERR_INVALID_ARG (-1)
#define PAFEM_ERR_OUT_OF_MEMORY (-2)
#define PAFEM_ERR_HIP (-3)
#define PAFEM_ERR_NOT_CONVERGED (-4)
#define PAFEM_ERR_UNSUPPORTED (-5)
#define PAFEM_ERR_NO_DEVICE (-6)

/* ---- operator kinds, precisions, modes ------------------------------------ */
#define PAFEM_MASS 0      /* M_ij = sum_q w rho detJ phi_i phi_j            */
#define PAFEM_DIFFUSION 1 /* K_ij = sum_q w k detJ (J^-T dphi_i).(J^-T dphi_j) */

#define PAFEM_FP64 1 /* vectors double, FP64 quadrature data and contractions */
#define PAFEM_FP32 2 /* vectors float, FP32 quadrature data (rounded copy)     */
#define PAFEM_BF16 4 /* vectors float, bfloat16 quadrature data, FP32 arithmetic */

#define PAFEM_SCATTER_ATOMIC 0        /* E^T by global atomic adds (run-to-run rounding differences) */
#define PAFEM_SCATTER_DETERMINISTIC 1 /* E^T by an E-vector and a per-dof sum in fixed (e, l) order:
                                         bitwise reproducible; the default */

#define PAFEM_INDEX_LATTICE 0 /* E computed from the lattice numbering in the kernels */
#define PAFEM_INDEX_MAP 1     /* E and E^T read from the stored int32 maps            */

#define PAFEM_APPLY_CONSTRAINED 1 /* flag: identity rows/columns on essential dofs */
#define PAFEM_APPLY_ACCUMULATE 2  /* flag: y += A x instead of y = A x */

#define PAFEM_SOLVE_PLAIN_FP64 0 /* Jacobi-PCG entirely in FP64 */
#define PAFEM_SOLVE_IR_FP32 1    /* FP64 defect correction around an FP32 Jacobi-PCG */
#define PAFEM_SOLVE_IR_BF16 2    /* the same with bfloat16 quadrature data in the inner operator */
#define PAFEM_SOLVE_MIXED_FP32 3 /* one Jacobi-PCG with an FP32 operator and Krylov vectors, the
                                    solution accumulated in FP64 and the residual replaced by the
                                    FP64 residual b - A x whenever it has fallen by inner_rtol */
#define PAFEM_SOLVE_MIXED_BF16 4 /* the same with bfloat16 quadrature data in the FP32 operator */

/* ---- opaque handles -------------------------------------------------------- */
typedef struct pafem_ctx pafem_ctx;
typedef struct pafem_mesh pafem_mesh;
typedef struct pafem_space pafem_space;
typedef struct pafem_op pafem_op;

/* Message of the last failed call on this thread ("" if none).  The pointer
 * stays valid until the next pafem call on the same thread. */
const char* pafem_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int pafem_version(void);

/* ---- context ---------------------------------------------------------------- */
/* Bind to HIP device `device` (>= 0), or host-only with device = -1.  (No
 * counterpart in the paper: the device binding of everything below.)
 * Errors: NO_DEVICE if the device does not exist, HIP on runtime failure. */
int pafem_ctx_create(int device, pafem_ctx** out);
int pafem_ctx_destroy(pafem_ctx* ctx);

/* ---- mesh -------------------------------------------------------------------- */
/* Structured hexahedral mesh of nx*ny*nz elements (each >= 1) whose corner
 * vertices are given, x index fastest: vert_xyz_host[((k (ny+1) + j) (nx+1) + i) * 3 + d].
 * Element (ex,ey,ez) has corners (ex+i, ey+j, ez+k), i,j,k in {0,1}; the map
 * from [0,1]^3 is trilinear.  The array is copied (to the device too, for a
 * GPU context).  Orientation is checked later, at operator assembly.
 * Defined by: the mesh layer of the paper (section "Meshing"), whose element
 * maps carry the local Jacobian used in "High-order mesh optimization"; here
 * that Jacobian is the one of the trilinear map, evaluated at every
 * quadrature point by pafem_op_assemble. */
int pafem_mesh_create_structured(pafem_ctx* ctx, int nx, int ny, int nz,
                                 const double* vert_xyz_host, pafem_mesh** out);
int pafem_mesh_destroy(pafem_mesh* mesh);

/* ---- order p: H1 space and its integer maps ----------------------------------- */
/* Defined by: the operator decomposition figure ("finite element operator
 * decomposition"), whose G takes the L-vector of global dofs to the E-vector
 * of element dofs; it is topological, so here it is the lattice numbering.
 * Order p in 1..8 (INVALID_ARG otherwise).  Builds the element restriction E
 * (int32, [ne][(p+1)^3]), its transpose in CSR form and the essential-dof list;
 * ne*(p+1)^3 and the dof count must each fit in int32 (INVALID_ARG otherwise). */
int pafem_space_create(pafem_mesh* mesh, int p, pafem_space** out);
int pafem_space_destroy(pafem_space* space);
int64_t pafem_space_ndofs(const pafem_space* space);   /* (nx p+1)(ny p+1)(nz p+1), or -1 */
int64_t pafem_space_nelems(const pafem_space* space);  /* nx ny nz, or -1 */
int64_t pafem_space_num_ess(const pafem_space* space); /* number of essential dofs, or -1 */
/* Copy E (row e = element, column l = local dof) into E_host[ne*(p+1)^3]. */
int pafem_space_get_restriction(const pafem_space* space, int32_t* E_host);
/* Copy E^T as CSR: offsets_host[ndofs+1], indices_host[ne*(p+1)^3]; the
 * indices of dof i are the E-vector positions e*(p+1)^3+l with E[e][l] = i,
 * ascending. */
int pafem_space_get_restriction_transpose(const pafem_space* space, int32_t* offsets_host,
                                          int32_t* indices_host);
/* Copy the ascending essential-dof list into out_host[num_ess]. */
int pafem_space_get_ess_dofs(const pafem_space* space, int32_t* out_host);

/* ---- quadrature: 1D tables (host, no GPU needed) ------------------------------ */
/* Defined by: the B of the operator decomposition figure (element dofs to
 * quadrature-point values), applied one direction at a time (sum
 * factorization, section "Matrix-free solvers for high-order finite elements").
 * Gauss-Lobatto-Legendre nodes (p+1), Gauss-Legendre points and weights (q) on
 * [0,1], and B[qq][a] = l_a(x_qq), G[qq][a] = l_a'(x_qq) (row-major [q][p+1]).
 * Any output pointer may be NULL.  1 <= p <= 8, 1 <= q <= 12. */
int pafem_basis_tables(int p, int q, double* gll_nodes, double* gl_points, double* gl_weights,
                       double* B, double* G);

/* ---- operator --------------------------------------------------------------- */
/* Defined by: the operator decomposition figure (A = P^T G^T B^T D B G P) for
 * the mass and diffusion forms (the paper's BP1 and BP3 benchmarks, section
 * "State-of-the-art performance on exascale platforms and AMD GPUs").
 * Create a MASS or DIFFUSION operator on `space` with q1d Gauss-Legendre
 * points per direction: 0 = the default p+2, or any p+1 <= q1d <= 10
 * (others give UNSUPPORTED).  The default runs the tuned element kernels and
 * every solve and launch form; another q1d runs a run-time-sized element
 * kernel (plain sum factorization through LDS, one workgroup per element),
 * and then bfloat16 quadrature data, the matrix-free level and the persistent
 * launch form give UNSUPPORTED, and CG runs its separate-kernel iteration.
 * The coefficient defaults to the constant 1.  Nothing is computed until
 * pafem_op_assemble. */
int pafem_op_create(pafem_space* space, int kind, int q1d, pafem_op** out);
int pafem_op_destroy(pafem_op* op);
int pafem_op_q1d(const pafem_op* op);
/* Physical coordinates of the quadrature points, xyz_dev[ne][3][q^3] (double). */
int pafem_op_qpoint_coords(pafem_op* op, double* xyz_dev, void* stream);
/* Defined by: the pointwise D of the operator decomposition figure, which
 * holds the coefficient at the quadrature points; user-supplied variable
 * coefficients follow section "Python interface (PyMFEM)", evaluated here by
 * the caller at the points pafem_op_qpoint_coords returns (no callbacks).
 * Coefficient (rho for MASS, k for DIFFUSION): a constant, values at the
 * quadrature points k_dev[ne][q^3] (copied into library memory on `stream`),
 * or the built-in k = 1 + amp sin(2 pi x) evaluated on the device. Takes effect
 * at the next pafem_op_assemble. */
int pafem_op_set_coefficient_const(pafem_op* op, double c);
int pafem_op_set_coefficient_qpts(pafem_op* op, const double* k_dev, void* stream);
int pafem_op_set_coefficient_sinx(pafem_op* op, double amp);
/* Defined by: the partial assembly level of section "State-of-the-art
 * performance on exascale platforms and AMD GPUs" (only the data at the
 * quadrature points is precomputed and stored).
 * Compute the quadrature data D on the device (synchronous).
 * MASS: D[e][0][qpt] = w rho detJ.  DIFFUSION: D[e][0..5][qpt] = the upper
 * triangle xx,xy,xz,yy,yz,zz of w k adj(J) adj(J)^T / detJ.  FP64 is always
 * built; prec_mask | PAFEM_FP32 also keeps an FP32 rounded copy and
 * prec_mask | PAFEM_BF16 a bfloat16 one (round to nearest even of the FP32 value).
 * INVALID_ARG if detJ <= 0 at any quadrature point (inverted element). */
int pafem_op_assemble(pafem_op* op, int prec_mask, void* stream);
/* Device bytes the quadrature data occupies for prec_mask (or -1). */
int64_t pafem_op_qdata_bytes(const pafem_op* op, int prec_mask);
/* Device bytes the operator holds once assembled for prec_mask and used for
 * applies and solves in those precisions: quadrature data, the E-vector
 * workspace, the inverse diagonal (FP64, and FP32 when prec_mask asks for
 * FP32 or BF16), the CG work vectors (three FP64, four FP32 for the
 * mixed-precision modes, one FP64 copy of x for the graph launch form) and
 * the reduction partials; the mesh vertices and the caller's vectors are not
 * included (or -1). */
int64_t pafem_op_footprint_bytes(const pafem_op* op, int prec_mask);
/* Copy the stored quadrature data of precision `prec` into dst_dev
 * ([ne][C][q^3], C = 1 or 6, double or float). */
int pafem_op_get_qdata(pafem_op* op, int prec, void* dst_dev, void* stream);
/* Defined by: the assembly levels of section "State-of-the-art performance on
 * exascale platforms and AMD GPUs" (fully matrix-free: everything the apply
 * needs is computed on the fly; partial assembly: only the data at the
 * quadrature points is stored).
 * PAFEM_ASSEMBLY_PARTIAL (the default) stores D at pafem_op_assemble;
 * PAFEM_ASSEMBLY_MATRIX_FREE stores nothing per quadrature point: every apply
 * recomputes the geometric factors (and the coefficient) from the element
 * corners, so its HBM stream is the vectors alone.  Matrix-free operators take
 * a constant or the built-in sin x coefficient (INVALID_ARG at assembly for
 * values at quadrature points), FP64 and FP32 (not BF16), and compute their
 * diagonal from a temporary copy of D.  Takes effect at the next
 * pafem_op_assemble (which then only checks the Jacobian sign). */
#define PAFEM_ASSEMBLY_PARTIAL 0
#define PAFEM_ASSEMBLY_MATRIX_FREE 1
int pafem_op_set_assembly_level(pafem_op* op, int level);
/* Choose how E^T sums element contributions (default DETERMINISTIC). */
int pafem_op_set_scatter_mode(pafem_op* op, int mode);
/* Choose where the kernels take E (and, in deterministic mode, E^T) from:
 * PAFEM_INDEX_LATTICE (default) computes the lattice numbering in the kernel;
 * PAFEM_INDEX_MAP reads the stored maps (the ones pafem_space_get_restriction*
 * return).  Both give identical results. */
int pafem_op_set_restriction_mode(pafem_op* op, int mode);

/* Defined by: the operator decomposition figure, y = G^T B^T D B G x (P is
 * the identity on one GPU), at the partial assembly level.
 * y = A x.  prec selects double (PAFEM_FP64) or float vectors of length ndofs
 * with the FP32 (PAFEM_FP32) or bfloat16 (PAFEM_BF16) quadrature data; the
 * contractions then run in FP32.  x and y must not alias.  flags:
 *   0: the plain assembled operator;
 *   PAFEM_APPLY_CONSTRAINED: rows and columns of essential dofs replaced by
 *     the identity (y_ess = x_ess, free rows see x with essential entries 0);
 *   PAFEM_APPLY_ACCUMULATE: add the result to y instead of overwriting it (in
 *     the default atomic E^T mode this launches the element kernel alone). */
int pafem_op_apply(pafem_op* op, int prec, const void* x_dev, void* y_dev, int flags,
                   void* stream);
/* Defined by: the E-vector of the operator decomposition figure (before G^T).
 * The element results before assembly: yE_dev[e][l] = (B^T D B E x)_e at local
 * node l = a + (p+1)(b + (p+1)c), an E-vector of ne*(p+1)^3 entries of the
 * precision `prec` (one element kernel, no E^T).  flags: 0 or
 * PAFEM_APPLY_CONSTRAINED (essential entries of x read as 0). */
int pafem_op_apply_evector(pafem_op* op, int prec, const void* x_dev, void* yE_dev, int flags,
                           void* stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): pafem_op_apply
 * with the same arguments, flags and results, always with the deterministic
 * E^T on the lattice numbering (bitwise equal to pafem_op_apply in the default
 * modes), whose E-vector workspace is a fixed device array of
 * PAFEM_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends.  Nothing is allocated and no library routine that
 * allocates is called.  INVALID_ARG, before anything is enqueued, when the
 * workspace the operator needs (ne (p+1)^3 words of the vector type) exceeds
 * the array.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams, other threads) race. */
#define PAFEM_NOALLOC_SCRATCH_BYTES (32 * 1024 * 1024)
int pafem_op_apply_noalloc(pafem_op* op, int prec, const void* x_dev, void* y_dev, int flags,
                           void* stream);
/* Defined by: section "Matrix-free solvers for high-order finite elements"
 * (the diagonal of the operator computed by sum factorization without
 * assembling the matrix, for diagonal smoothers and Jacobi).
 * d = diag(A) by sum factorization (double, ndofs); constrained = 1 puts 1 on
 * essential dofs.  Bitwise reproducible. */
int pafem_op_diagonal(pafem_op* op, double* d_dev, int constrained, void* stream);

/* ---- right-hand side ------------------------------------------------------------ */
/* (The paper states no right-hand side; this is the load of the manufactured
 * Poisson problem, integrated with the operator's own quadrature.)
 * b_i = sum_e sum_q w detJ f(x_q) phi_i(x_q) with the op's quadrature rule and
 * geometry; f_qpts_dev[ne][q^3] holds f at the quadrature points (as returned
 * by pafem_op_qpoint_coords), or NULL for the built-in f = 3 pi^2
 * sin(pi x) sin(pi y) sin(pi z).  Essential entries of b are set to 0.
 * Bitwise reproducible. */
int pafem_rhs_assemble(pafem_op* op, const double* f_qpts_dev, double* b_dev, void* stream);

/* ---- solve ------------------------------------------------------------------- */
typedef struct {
  int mode;          /* PAFEM_SOLVE_* */
  double rtol;       /* stop when ||b - A x||_2 <= rtol ||b||_2, confirmed in every mode on the
                        residual recomputed in FP64 (plain CG restarts from x with that
                        residual when the recursive one meets rtol first) */
  double inner_rtol; /* IR: relative tolerance of each FP32 inner solve (e.g. 1e-4);
                        MIXED: residual drop that triggers a replacement, in (0, 1) (e.g. 0.1) */
  int maxit;         /* plain, MIXED: max CG iterations; IR: max inner iterations per solve */
  int max_outer;     /* IR: max refinement steps (MIXED: unused) */
  int check_every;   /* host reads the residual every this many iterations (>= 1) */
  int launch;        /* PAFEM_LAUNCH_*: how the iterations between two reads are issued */
} pafem_solve_opts;

/* Launch forms of the CG iterations (the same arithmetic; kernels and graph
 * give bitwise equal results, the persistent kernel sums its reductions in
 * another fixed order).  The fully fused form follows the paper's section on
 * kernel fusion. */
#define PAFEM_LAUNCH_KERNELS 0    /* one launch per kernel of every iteration */
#define PAFEM_LAUNCH_GRAPH 1      /* the check_every iterations captured once in a HIP graph
                                     (kept by the operator and reused while the vectors are
                                     the same) and replayed; PLAIN_FP64 and the IR inner solves */
#define PAFEM_LAUNCH_PERSISTENT 2 /* check_every whole iterations in one cooperative persistent
                                     kernel with grid-wide barriers (bounded waits); PLAIN_FP64
                                     with the deterministic E^T on the lattice numbering, partial
                                     assembly level */

typedef struct {
  int iterations;       /* plain, MIXED: CG iterations; IR: total inner iterations */
  int outer_iterations; /* IR: refinement steps; MIXED: residual replacements; plain: restarts
                           from the FP64 residual */
  double rel_res;       /* final relative residual of the last CG recursion */
  double true_rel_res;  /* ||b - A x||_2 / ||b||_2 recomputed in FP64 after the solve */
  double seconds;       /* wall time of the solve on the host clock */
  int fp64_inner_solves; /* IR: inner solves run in FP64 because a reduced-precision one gave
                            a non-finite result or cut the FP64 residual by less than a tenth
                            (such a solve then continues in FP64) */
} pafem_solve_stats;

/* Defined by: section "Matrix-free solvers for high-order finite elements"
 * (a Krylov method with a preconditioner built without the assembled matrix,
 * here CG with the sum-factorized diagonal); the fused iteration follows
 * section "Kernel fusion".  The mixed-precision modes are not in the paper.
 * Solve A x = b for the constrained operator of `op` (DIFFUSION or MASS) with
 * Jacobi preconditioning; x_dev holds the initial guess on entry (its
 * essential entries must equal b's) and the solution on return.
 * Synchronous.  NOT_CONVERGED if the iteration limit is hit (x then holds the
 * last iterate and stats are filled).  IR_FP32 and MIXED_FP32 need the FP32
 * quadrature copy, IR_BF16 and MIXED_BF16 the bfloat16 one. */
int pafem_solve_cg(pafem_op* op, const double* b_dev, double* x_dev, const pafem_solve_opts* opts,
                   pafem_solve_stats* stats, void* stream);

/* ---- p-multigrid preconditioned CG ---------------------------------------------- */
/* Defined by: section "Matrix-free solvers for high-order finite elements" of
 * the paper (p-multigrid: a hierarchy of polynomial degrees on the same mesh,
 * transfer between the nested spaces by sum factorization, smoothers built on
 * the sum-factorized diagonal with Chebyshev acceleration).  The readings
 * fixed here:
 *   - orders p, p/2, p/4, ..., 1 (integer halving) on the operator's mesh, each
 *     level a partial-assembly operator of the same kind and coefficient with
 *     its own q = p_level + 2 quadrature data (FP64);
 *   - prolongation: the fine nodal values of the coarse function (sum-factorized
 *     interpolation from the coarse to the fine GLL nodes); restriction: its
 *     transpose, with the essential coarse rows set to zero;
 *   - smoother: `cheb_degree` steps of Chebyshev-accelerated Jacobi for
 *     D^-1 A on [cheb_lower lmax, lmax], before and after the coarse
 *     correction (a symmetric V-cycle); lmax = lmax_safety times a
 *     power-iteration estimate (power_iters steps from a fixed pseudo-random
 *     vector) unless set with pafem_mg_set_lmax;
 *   - order-1 level: exactly coarse_iters Jacobi-PCG steps from zero;
 *   - outer solver: flexible CG (beta = z_new . (r_new - r_old) / z_old . r_old)
 *     with one V-cycle as preconditioner, stopping like pafem_solve_cg.
 * Levels are numbered from 0 (the operator's order) to num_levels - 1 (order 1). */
typedef struct pafem_mg pafem_mg;

typedef struct {
  int cheb_degree;    /* smoothing steps before and after the coarse correction, 1..16 (3) */
  double cheb_lower;  /* lower end of the smoothing interval as a fraction of lmax, (0, 1) (0.1) */
  double lmax_safety; /* factor on the power-iteration estimate, [1, 4] (1.1) */
  int power_iters;    /* power iterations per smoothed level, >= 1 (10) */
  int coarse_iters;   /* Jacobi-PCG steps on the order-1 level per V-cycle, >= 1 (20) */
} pafem_mg_opts;

/* Fill *opts with the defaults given in parentheses above. */
void pafem_mg_default_opts(pafem_mg_opts* opts);
/* Build the hierarchy for an operator assembled in FP64 whose coefficient is a
 * constant or the built-in sin x one (INVALID_ARG for values at quadrature
 * points): coarse spaces and operators, their quadrature data and diagonals,
 * the transfer tables and the eigenvalue estimates (synchronous, on the
 * legacy default stream).  opts may be NULL (defaults).  The hierarchy keeps
 * a reference to `op`; results follow later re-assembly of `op` only through
 * its quadrature data, not through the coarse levels. */
int pafem_mg_create(pafem_op* op, const pafem_mg_opts* opts, pafem_mg** out);
int pafem_mg_destroy(pafem_mg* mg);
int pafem_mg_num_levels(const pafem_mg* mg);
/* Order, dof count and lmax (0 on the order-1 level) of a level; any output may be NULL. */
int pafem_mg_level_info(const pafem_mg* mg, int level, int* p, int64_t* ndofs, double* lmax);
/* Replace the eigenvalue bound of a smoothed level (0 <= level < num_levels - 1). */
int pafem_mg_set_lmax(pafem_mg* mg, int level, double lmax);
/* uf = P uc from level + 1 to level (double vectors of the two levels' dof counts). */
int pafem_mg_prolong(pafem_mg* mg, int level, const double* uc_dev, double* uf_dev, void* stream);
/* rc = P^T rf from level to level + 1, essential coarse entries 0. */
int pafem_mg_restrict(pafem_mg* mg, int level, const double* rf_dev, double* rc_dev, void* stream);
/* x = the Chebyshev smoother applied to b from x = 0 on a smoothed level. */
int pafem_mg_smooth(pafem_mg* mg, int level, const double* b_dev, double* x_dev, void* stream);
/* z = one V-cycle applied to r on level 0 (r's essential entries should be 0). */
int pafem_mg_vcycle(pafem_mg* mg, const double* r_dev, double* z_dev, void* stream);
/* Solve A x = b (constrained operator of level 0) by flexible CG with one
 * V-cycle per iteration; x holds the initial guess (essential entries equal
 * to b's) and the solution.  opts->mode must be PAFEM_SOLVE_PLAIN_FP64; rtol
 * and maxit as for pafem_solve_cg (convergence is confirmed on the FP64
 * residual b - A x, restarting from x if needed; outer_iterations counts the
 * restarts).  Synchronous.  NOT_CONVERGED if maxit is reached. */
int pafem_mg_solve(pafem_mg* mg, const double* b_dev, double* x_dev, const pafem_solve_opts* opts,
                   pafem_solve_stats* stats, void* stream);

/* ---- reductions (exposed for testing the CG building blocks) --------------------- */
/* Defined by: section "Kernel fusion" (dot products reduced with wavefront-
 * level instructions).
 * result_dev[0] = sum_i x[i] y[i] over n doubles, fixed-order two-stage
 * reduction (bitwise reproducible for a given n); x, y may be NULL when n = 0. */
int pafem_dot(pafem_ctx* ctx, int64_t n, const double* x_dev, const double* y_dev,
              double* result_dev, void* stream);

/* ---- serving: continuous batching of Poisson solves --------------------------- */
/* A server owns one engine thread on the context's GPU.  Submitted requests
 * (each a Dirichlet Poisson problem -div(k grad u) = f, f = 3 pi^2
 * sin(pi x) sin(pi y) sin(pi z), on its own structured mesh and order) are
 * admitted first-in first-out while a slot is free and their estimated
 * device footprint fits the HBM budget; admitted requests keep their
 * quadrature data resident, and all of them advance together: each round
 * replays one HIP graph holding `iters_per_round` CG iterations whose kernels
 * (the element pass over every active request's elements, whatever its
 * order, then the E^T sums, reductions and vector updates) each cover the
 * whole batch.  Requests finish independently; their memory returns to the
 * budget at once and waiting requests are admitted in the next round.
 * Results are bitwise independent of which other requests share the batch.
 * IR_FP32 requests run their inner solves in the FP32 batch and their FP64
 * refinement steps between rounds. */
#define PAFEM_REQ_QUEUED 0
#define PAFEM_REQ_RUNNING 1
#define PAFEM_REQ_DONE 2
#define PAFEM_REQ_FAILED 3

#define PAFEM_COEF_CONST 0 /* k = coef_value */
#define PAFEM_COEF_SINX 1  /* k = 1 + coef_value sin(2 pi x) */

typedef struct pafem_server pafem_server;

typedef struct {
  int nx, ny, nz;           /* element lattice, each >= 1 */
  int p;                    /* order 1..8 (q = p + 2) */
  const double* verts_host; /* [(nx+1)(ny+1)(nz+1)][3], copied by pafem_server_submit */
  int coef_kind;            /* PAFEM_COEF_CONST or PAFEM_COEF_SINX */
  double coef_value;
  int mode;                 /* PAFEM_SOLVE_PLAIN_FP64, PAFEM_SOLVE_IR_FP32 or PAFEM_SOLVE_MIXED_FP32 */
  double rtol;              /* relative residual target (FP64) */
  double inner_rtol;        /* IR: inner FP32 relative tolerance; MIXED: replacement factor in (0, 1) */
  int maxit;                /* CG iteration limit (per inner solve for IR) */
  int max_outer;            /* IR: refinement step limit */
} pafem_request;

typedef struct {
  int status;               /* PAFEM_REQ_* */
  int error;                /* PAFEM_ERR_* when status is FAILED (NOT_CONVERGED keeps x) */
  int64_t ndofs;
  int64_t footprint_bytes;  /* device bytes reserved while admitted */
  int iterations;           /* CG iterations (inner total for IR) */
  int outer_iterations;     /* IR: refinement steps; MIXED: residual replacements */
  double rel_res;           /* final ||b - A x|| / ||b|| in FP64 */
  double t_arrive, t_admit, t_done; /* seconds on the server clock (-1 if not yet) */
} pafem_result;

typedef struct {
  int64_t submitted, completed, failed, rounds;
  int64_t peak_bytes;       /* largest sum of admitted footprints */
  int max_active;           /* most requests admitted at once */
  double dof_iterations;    /* sum over finished requests of ndofs * iterations */
  double seconds;           /* server clock now */
} pafem_server_counters;

/* Device bytes a request reserves while admitted (quadrature data, E-vector,
 * vectors, geometry), or -1 for an invalid request. */
int64_t pafem_request_footprint(const pafem_request* req);

/* Start a server on a GPU context with an HBM budget (bytes), at most
 * max_slots requests admitted at once (1..64) and iters_per_round CG
 * iterations per replayed graph (>= 1). */
int pafem_server_create(pafem_ctx* ctx, int64_t hbm_budget_bytes, int max_slots,
                        int iters_per_round, pafem_server** out);
/* Queue a request (thread-safe, returns at once).  INVALID_ARG for a
 * malformed request; a request larger than the whole budget is accepted and
 * then fails with OUT_OF_MEMORY. */
int pafem_server_submit(pafem_server* srv, const pafem_request* req, uint64_t* ticket);
int pafem_server_poll(pafem_server* srv, uint64_t ticket, pafem_result* out);
/* Copy the solution (ndofs doubles) of a finished request to x_host and
 * release it.  INVALID_ARG if the request has not finished or n differs. */
int pafem_server_get_solution(pafem_server* srv, uint64_t ticket, double* x_host, int64_t n);
/* Block until every request submitted so far has finished. */
int pafem_server_drain(pafem_server* srv);
int pafem_server_stats(pafem_server* srv, pafem_server_counters* out);
/* Drain, stop the engine and free everything. */
int pafem_server_destroy(pafem_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* PAFEM_H */
