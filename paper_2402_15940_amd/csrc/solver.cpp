// Jacobi-preconditioned conjugate gradient on the partially assembled
// operator: plain FP64, FP64 defect correction around an FP32 inner PCG, and
// one mixed-precision PCG with FP64 residual replacement.
//
// All CG scalars live in a device-resident CgState; one iteration is a fixed
// sequence of kernels with no host round trip: on the lattice numbering with
// the deterministic E^T, five (element pass + p.Ap partials, alpha, E^T sum +
// x and r updates + (r.z, r.r) partials, beta, direction update), otherwise
// seven (apply as element pass and E^T, p.Ap partial dot, alpha, update +
// partials, beta, direction update).  The host reads the state
// every `check_every` iterations; kernels of iterations enqueued after
// convergence see state.done and return at once.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "internal.h"

namespace pafem {

namespace {

inline hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

struct CgResult {
  int iterations = 0;
  double rr = 0.0, bb = 0.0;
  bool converged = false;
  double true_rr = -1.0;  // ||b - A x||^2 in FP64 when the check was enqueued (else -1)
};

// Reduction partials: pairs for the vector kernels (reduce_blocks) and for the
// fused CG step (at most kMaxCgParts), then 8 scalar slots.  Sized once for
// both, so that no caller's pointers into it go stale.
int partial_pairs(int64_t n) {
  const int nb = reduce_blocks(n);
  return nb > kMaxCgParts ? nb : kMaxCgParts;
}
int ensure_partials(Op* op, int64_t n) {
  return op->d_part.ensure(((size_t)partial_pairs(n) * 2 + 8) * sizeof(double));
}

// The deterministic E^T on the lattice numbering lets one CG step run as
// three passes over memory instead of five: the element pass of A p also
// forms p . A p per workgroup, and the ordered E^T sum applies the updates of
// x and r and forms (r . z, r . r) without storing A p.
bool fused_cg(const Op* op) {
  return op->scatter_mode == PAFEM_SCATTER_DETERMINISTIC &&
         op->index_mode == PAFEM_INDEX_LATTICE && op->q == op->space->p + 2;
}

// alpha, x += alpha p, r -= alpha A p, beta (the direction update follows).
// part holds at least kMaxCgParts pairs.
template <typename TX, typename T>
int cg_step_fused(Op* op, TX* x, T* r, const T* p, const T* dinv, double* part, CgState* st,
                  hipStream_t s, int qprec) {
  Space* sp = op->space;
  int ne_parts = 0, g_parts = 0;
  PAFEM_TRY(apply_elements_dot<T>(op, p, &st->done, s, qprec, &ne_parts));
  PAFEM_TRY_HIP(launch_cg_alpha_wide(op->d_gpart.as<double>(), ne_parts, st, s));
  const bool nt = op->level == PAFEM_ASSEMBLY_PARTIAL &&
                  evec_nt_loads(op->kind, sp->p, sizeof(T) == sizeof(double));
  PAFEM_TRY_HIP((launch_gather_xrows_cg<T, TX>(op->d_evec.as<T>(), sp->mesh->nx, sp->mesh->ny,
                                               sp->mesh->nz, sp->p, p, x, r, dinv, part,
                                               &g_parts, st, s, nt)));
  PAFEM_TRY_HIP(launch_cg_beta(part, g_parts, st, s));
  return PAFEM_OK;
}

// Solve A x = rhs for the constrained operator in precision T.  On entry x is
// the initial guess unless x0_zero.  r, p, Ap are work vectors of length n.
// The check_every iterations of one CG loop pass (the separate-kernel or the
// fused step, then the direction update), enqueued on s.
template <typename T>
int enqueue_iterations(Op* op, T* x, T* r, T* p, T* Ap, const T* dinv, double* part,
                       CgState* st, int check_every, hipStream_t s, int qprec) {
  const int64_t n = op->space->ndofs;
  const int nb = reduce_blocks(n);
  const int* done = &st->done;
  for (int k = 0; k < check_every; ++k) {
    if (fused_cg(op)) {
      PAFEM_TRY((cg_step_fused<T, T>(op, x, r, p, dinv, part, st, s, qprec)));
    } else {
      PAFEM_TRY(apply_impl<T>(op, p, Ap, PAFEM_APPLY_CONSTRAINED, done, s, qprec));
      PAFEM_TRY_HIP(launch_dot_partial<T>(p, Ap, n, part, nb, done, s));
      PAFEM_TRY_HIP(launch_cg_alpha(part, nb, st, s));
      PAFEM_TRY_HIP((launch_cg_update<T, T>(x, r, p, Ap, dinv, n, part, nb, st, s)));
      PAFEM_TRY_HIP(launch_cg_beta(part, nb, st, s));
    }
    PAFEM_TRY_HIP(launch_cg_pupdate<T>(p, r, dinv, n, st, s));
  }
  return PAFEM_OK;
}

// The op's captured graph of check_every iterations for these vectors,
// captured now unless the cached one was captured for the same ones.  Every
// buffer the kernels touch is allocated before the capture.
template <typename T>
int cg_graph(Op* op, T* x, T* r, T* p, T* Ap, const T* dinv, double* part, CgState* st,
             int check_every, int qprec, hipGraphExec_t* out) {
  const void* key[10] = {x, r, p, Ap, dinv, part, st, (const void*)(intptr_t)check_every,
                         (const void*)(intptr_t)qprec, (const void*)(intptr_t)sizeof(T)};
  bool same = op->cg_graph != nullptr;
  for (int i = 0; i < 10 && same; ++i) same = op->cg_graph_key[i] == key[i];
  if (same) {
    *out = op->cg_graph;
    return PAFEM_OK;
  }
  if (op->cg_graph) {
    PAFEM_TRY_HIP(hipGraphExecDestroy(op->cg_graph));
    op->cg_graph = nullptr;
  }
  Space* sp = op->space;
  PAFEM_TRY(op->d_evec.ensure((size_t)evec_words(sp->ne, sp->p + 1) * sizeof(double)));
  if (fused_cg(op)) {
    PAFEM_TRY(op->d_gpart.ensure(
        (size_t)element_blocks(op->kind, sp->p, sp->ne, !std::is_same<T, double>::value) *
        sizeof(double)));
  } else {
    if (op->index_mode == PAFEM_INDEX_MAP) PAFEM_TRY(ensure_device_maps(sp));
    if (op->scatter_mode == PAFEM_SCATTER_ATOMIC) PAFEM_TRY(ensure_ess(sp, true));
  }
  if (!op->cap_stream)
    PAFEM_TRY_HIP(hipStreamCreateWithFlags(&op->cap_stream, hipStreamNonBlocking));
  hipStream_t cs = op->cap_stream;
  PAFEM_TRY_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
  const int rc = enqueue_iterations<T>(op, x, r, p, Ap, dinv, part, st, check_every, cs, qprec);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(cs, &g);
  if (rc != PAFEM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  PAFEM_TRY_HIP(ec);
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  PAFEM_TRY_HIP(ei);
  op->cg_graph = exec;
  for (int i = 0; i < 10; ++i) op->cg_graph_key[i] = key[i];
  *out = exec;
  return PAFEM_OK;
}

// Spin limit of the persistent kernel's barrier waits (each poll sleeps
// briefly): far beyond any legitimate wait, so that a stall ends the launch.
constexpr long long kSpinLimit = 1LL << 24;

// Defect correction: an FP32/BF16 correction must bring the FP64 residual
// below this fraction of its value before it, or the inner solves switch to FP64.
constexpr double kIrStagnation = 0.9;

// The FP64 residual check of a finished CG, enqueued behind a batch of
// iterations: once the CG is done, r = b - A x and its squared norm go to
// true_rr (the kernels skip while it still runs), so the host reads the state
// and the check with one synchronization.
int enqueue_true_residual(Op* op, const double* b, const double* x, double* r, double* Ax,
                          double* part, int* running, double* true_rr, const CgState* st,
                          hipStream_t s) {
  const int64_t n = op->space->ndofs;
  const int nb = reduce_blocks(n);
  PAFEM_TRY_HIP(launch_running_flag(st, running, s));
  PAFEM_TRY(apply_impl<double>(op, x, Ax, PAFEM_APPLY_CONSTRAINED, running, s));
  PAFEM_TRY_HIP(launch_residual(b, Ax, r, n, s, running));
  PAFEM_TRY_HIP(launch_dot_partial<double>(r, r, n, part, nb, running, s));
  PAFEM_TRY_HIP(launch_sum_final(part, nb, 1, true_rr, s));
  return PAFEM_OK;
}

// true_b: when given (T = double), the FP64 residual check of the finished CG
// is enqueued behind every batch of iterations (res.true_rr).
template <typename T>
int run_pcg(Op* op, const T* rhs, T* x, bool x0_zero, T* r, T* p, T* Ap, const T* dinv,
            double rtol, int maxit, int check_every, hipStream_t s, CgResult& res,
            int qprec = 0, int launch = PAFEM_LAUNCH_KERNELS, const double* true_b = nullptr) {
  Space* sp = op->space;
  const int64_t n = sp->ndofs;
  const int nb = reduce_blocks(n);
  PAFEM_TRY(ensure_partials(op, n));
  PAFEM_TRY(op->d_state.ensure(sizeof(CgState)));
  double* part = op->d_part.as<double>();
  // scalar slots after the partials: 0 b.b, 2 the IR outer ||r||^2, 4 the
  // residual check, 6 the running flag
  double* bbdev = part + 2 * partial_pairs(n);
  double* true_rr_dev = bbdev + 4;
  int* running = reinterpret_cast<int*>(bbdev + 6);
  CgState* st = op->d_state.as<CgState>();

  // b.b for the stopping test, kept on the device
  PAFEM_TRY_HIP(launch_dot_partial<T>(rhs, rhs, n, part, nb, nullptr, s));
  PAFEM_TRY_HIP(launch_sum_final(part, nb, 1, bbdev, s));

  // r = rhs - A x
  if (x0_zero) {
    PAFEM_TRY_HIP(launch_fill<T>(x, n, T(0), nullptr, s));
    if (r != rhs)
      PAFEM_TRY_HIP(hipMemcpyAsync(r, rhs, n * sizeof(T), hipMemcpyDeviceToDevice, s));
  } else {
    PAFEM_TRY(apply_impl<T>(op, x, Ap, PAFEM_APPLY_CONSTRAINED, nullptr, s));
    if (std::is_same<T, double>::value) {
      PAFEM_TRY_HIP(launch_residual((const double*)rhs, (const double*)Ap, (double*)r, n, s));
    } else {
      set_error("internal: FP32 PCG needs a zero initial guess");
      return PAFEM_ERR_INVALID_ARG;
    }
  }
  PAFEM_TRY_HIP(launch_cg_init<T>(r, dinv, p, n, part, nb, s));
  PAFEM_TRY_HIP(launch_cg_init_final(part, nb, 0.0, rtol, maxit, st, s, 0.0, bbdev));

  CgState hs{};
  double hrr = -1.0;
  // behind each batch: the residual check (plain FP64 solves), then one read
  auto check = [&]() -> int {
    if constexpr (std::is_same<T, double>::value) {
      if (true_b != nullptr) {
        PAFEM_TRY(enqueue_true_residual(op, true_b, x, r, Ap, part, running, true_rr_dev, st, s));
        PAFEM_TRY_HIP(
            hipMemcpyAsync(&hrr, true_rr_dev, sizeof(double), hipMemcpyDeviceToHost, s));
      }
    }
    PAFEM_TRY_HIP(hipMemcpyAsync(&hs, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    return PAFEM_OK;
  };
  if (launch == PAFEM_LAUNCH_PERSISTENT) {
    if constexpr (std::is_same<T, double>::value) {
      ApplyArgs<double> a{};
      int64_t groups = 0;
      PAFEM_TRY(cg_element_args(op, p, &a, &groups));
      constexpr int kMaxPersistentBlocks = 8192;
      // partials, then the barrier words and the error flag (zero on entry)
      constexpr size_t kBarDoubles = kPersistentBarrierBytes / sizeof(double) + 16;
      PAFEM_TRY(op->d_pers.ensure((3 * (size_t)kMaxPersistentBlocks + kBarDoubles) *
                                  sizeof(double)));
      double* bpart = op->d_pers.as<double>();
      double* npart = bpart + kMaxPersistentBlocks;
      void* bar = npart + 2 * kMaxPersistentBlocks;
      int* err = reinterpret_cast<int*>(static_cast<double*>(bar) + kBarDoubles - 16);
      PAFEM_TRY_HIP(hipMemsetAsync(bar, 0, kBarDoubles * sizeof(double), s));
      for (;;) {
        int grid = 0;
        PAFEM_TRY_HIP(launch_pcg_persistent(op->kind, sp->p, a, groups, x, r, dinv, bpart, npart,
                                            st, bar, err, kSpinLimit, check_every,
                                            kMaxPersistentBlocks, &grid, s));
        int herr = 0;
        PAFEM_TRY(check());
        PAFEM_TRY_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
        PAFEM_TRY_HIP(hipStreamSynchronize(s));
        if (herr) {
          set_error("persistent CG: a grid barrier wait exceeded its bound");
          return PAFEM_ERR_HIP;
        }
        if (hs.done) break;
      }
    } else {
      set_error("internal: the persistent CG runs in FP64");
      return PAFEM_ERR_INVALID_ARG;
    }
  } else if (launch == PAFEM_LAUNCH_GRAPH) {
    hipGraphExec_t g = nullptr;
    PAFEM_TRY((cg_graph<T>(op, x, r, p, Ap, dinv, part, st, check_every, qprec, &g)));
    for (;;) {
      PAFEM_TRY_HIP(hipGraphLaunch(g, s));
      PAFEM_TRY(check());
      PAFEM_TRY_HIP(hipStreamSynchronize(s));
      if (hs.done) break;
    }
  } else {
    for (;;) {
      PAFEM_TRY((enqueue_iterations<T>(op, x, r, p, Ap, dinv, part, st, check_every, s, qprec)));
      PAFEM_TRY(check());
      PAFEM_TRY_HIP(hipStreamSynchronize(s));
      if (hs.done) break;
    }
  }
  res.iterations = hs.iter;
  res.rr = hs.rr;
  res.bb = hs.bb;
  res.converged = hs.rr <= hs.rr_stop;
  res.true_rr = hrr;
  return PAFEM_OK;
}

// Mixed-precision Jacobi-PCG with residual replacement: the operator, the
// residual, direction and preconditioned vectors are FP32 (rs, p, Ap), the
// solution is accumulated in FP64 with the FP64 alpha, all dot products
// accumulate in FP64, and whenever the recursive residual has fallen by delta
// since the last replacement (or meets the tolerance) it is replaced by the
// FP64 residual b - A x (FP64 operator), keeping the search direction.
// r64 and Ax are FP64 work vectors.
int run_mixed(Op* op, const double* b, double* x, double* r64, double* Ax, float* rs, float* p,
              float* Ap, const float* dinv, double rtol, double delta, int maxit,
              int check_every, int qprec, hipStream_t s, CgResult& res, int& replacements) {
  Space* sp = op->space;
  const int64_t n = sp->ndofs;
  const int nb = reduce_blocks(n);
  PAFEM_TRY(ensure_partials(op, n));
  PAFEM_TRY(op->d_state.ensure(sizeof(CgState)));
  double* part = op->d_part.as<double>();
  double* bbdev = part + 2 * partial_pairs(n);
  CgState* st = op->d_state.as<CgState>();

  PAFEM_TRY_HIP(launch_dot_partial<double>(b, b, n, part, nb, nullptr, s));
  PAFEM_TRY_HIP(launch_sum_final(part, nb, 1, bbdev, s));  // b.b stays on the device

  // r64 = b - A x, rs = (float) r64, p = dinv .* rs
  PAFEM_TRY(apply_impl<double>(op, x, Ax, PAFEM_APPLY_CONSTRAINED, nullptr, s));
  PAFEM_TRY_HIP(launch_residual(b, Ax, r64, n, s));
  PAFEM_TRY_HIP(launch_replace_residual(r64, dinv, rs, n, part, nb, nullptr, s));
  PAFEM_TRY_HIP(launch_cg_init_final(part, nb, 0.0, rtol, maxit, st, s, delta * delta, bbdev));
  PAFEM_TRY_HIP(launch_fill<float>(p, n, 0.0f, nullptr, s));
  PAFEM_TRY_HIP(launch_cg_pupdate<float>(p, rs, dinv, n, st, s));  // beta = 0 here: p = z

  const int* done = &st->done;
  CgState hs{};
  replacements = 0;
  for (;;) {
    for (int k = 0; k < check_every; ++k) {
      if (fused_cg(op)) {
        PAFEM_TRY((cg_step_fused<double, float>(op, x, rs, p, dinv, part, st, s, qprec)));
      } else {
        PAFEM_TRY(apply_impl<float>(op, p, Ap, PAFEM_APPLY_CONSTRAINED, done, s, qprec));
        PAFEM_TRY_HIP(launch_dot_partial<float>(p, Ap, n, part, nb, done, s));
        PAFEM_TRY_HIP(launch_cg_alpha(part, nb, st, s));
        PAFEM_TRY_HIP((launch_cg_update<double, float>(x, rs, p, Ap, dinv, n, part, nb, st, s)));
        PAFEM_TRY_HIP(launch_cg_beta(part, nb, st, s));
      }
      PAFEM_TRY_HIP(launch_cg_pupdate<float>(p, rs, dinv, n, st, s));
    }
    PAFEM_TRY_HIP(hipMemcpyAsync(&hs, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    PAFEM_TRY_HIP(hipStreamSynchronize(s));
    if (hs.done == 0) continue;
    // paused, converged on the recursive residual, or out of iterations:
    // replace the residual by the FP64 one, which also decides convergence
    PAFEM_TRY(apply_impl<double>(op, x, Ax, PAFEM_APPLY_CONSTRAINED, nullptr, s));
    PAFEM_TRY_HIP(launch_residual(b, Ax, r64, n, s));
    PAFEM_TRY_HIP(launch_replace_residual(r64, dinv, rs, n, part, nb, st, s));
    ++replacements;
    PAFEM_TRY_HIP(hipMemcpyAsync(&hs, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    PAFEM_TRY_HIP(hipStreamSynchronize(s));
    if (hs.done) break;
    PAFEM_TRY_HIP(launch_cg_pupdate<float>(p, rs, dinv, n, st, s));  // p = z + beta p
  }
  res.iterations = hs.iter;
  res.rr = hs.rr;
  res.bb = hs.bb;
  res.converged = hs.rr <= hs.rr_stop;
  return PAFEM_OK;
}

// ||b - A x|| / ||b|| in FP64 (uses the vectors r and Ax as scratch).
int true_residual(Op* op, const double* b, const double* x, double* Ax, double* r, double bb,
                  hipStream_t s, double& out) {
  const int64_t n = op->space->ndofs;
  const int nb = reduce_blocks(n);
  double* part = op->d_part.as<double>();
  double* dev = part + 2 * nb + 1;
  PAFEM_TRY(apply_impl<double>(op, x, Ax, PAFEM_APPLY_CONSTRAINED, nullptr, s));
  PAFEM_TRY_HIP(launch_residual(b, Ax, r, n, s));
  PAFEM_TRY_HIP(launch_dot_partial<double>(r, r, n, part, nb, nullptr, s));
  PAFEM_TRY_HIP(launch_sum_final(part, nb, 1, dev, s));
  double rr = 0.0;
  PAFEM_TRY_HIP(hipMemcpyAsync(&rr, dev, sizeof(double), hipMemcpyDeviceToHost, s));
  PAFEM_TRY_HIP(hipStreamSynchronize(s));
  out = bb > 0.0 ? std::sqrt(rr / bb) : std::sqrt(rr);
  return PAFEM_OK;
}

}  // namespace

int pcg_fixed(Op* op, double* r, double* x, double* p, double* Ap, int iters, hipStream_t s) {
  const int64_t n = op->space->ndofs;
  const int nb = reduce_blocks(n);
  PAFEM_TRY(ensure_dinv(op, s, false));
  PAFEM_TRY(ensure_partials(op, n));
  PAFEM_TRY(op->d_state.ensure(sizeof(CgState)));
  double* part = op->d_part.as<double>();
  CgState* st = op->d_state.as<CgState>();
  const double* dinv = op->d_dinv64.as<double>();
  PAFEM_TRY_HIP(launch_fill<double>(x, n, 0.0, nullptr, s));
  PAFEM_TRY_HIP(launch_cg_init<double>(r, dinv, p, n, part, nb, s));
  // rtol = 0: the state is done only when the residual vanishes or after iters steps
  PAFEM_TRY_HIP(launch_cg_init_final(part, nb, 1.0, 0.0, iters, st, s));
  for (int k = 0; k < iters; ++k) {
    if (fused_cg(op)) {
      PAFEM_TRY((cg_step_fused<double, double>(op, x, r, p, dinv, part, st, s, 0)));
    } else {
      PAFEM_TRY(apply_impl<double>(op, p, Ap, PAFEM_APPLY_CONSTRAINED, &st->done, s));
      PAFEM_TRY_HIP(launch_dot_partial<double>(p, Ap, n, part, nb, &st->done, s));
      PAFEM_TRY_HIP(launch_cg_alpha(part, nb, st, s));
      PAFEM_TRY_HIP((launch_cg_update<double, double>(x, r, p, Ap, dinv, n, part, nb, st, s)));
      PAFEM_TRY_HIP(launch_cg_beta(part, nb, st, s));
    }
    PAFEM_TRY_HIP(launch_cg_pupdate<double>(p, r, dinv, n, st, s));
  }
  return PAFEM_OK;
}

int relative_residual(Op* op, const double* b, const double* x, double* Ax, double* r,
                      hipStream_t s, double& out) {
  const int64_t n = op->space->ndofs;
  const int nb = reduce_blocks(n);
  PAFEM_TRY(ensure_partials(op, n));
  double* part = op->d_part.as<double>();
  double* dev = part + 2 * partial_pairs(n);
  PAFEM_TRY_HIP(launch_dot_partial<double>(b, b, n, part, nb, nullptr, s));
  PAFEM_TRY_HIP(launch_sum_final(part, nb, 1, dev + 1, s));
  PAFEM_TRY(apply_impl<double>(op, x, Ax, PAFEM_APPLY_CONSTRAINED, nullptr, s));
  PAFEM_TRY_HIP(launch_residual(b, Ax, r, n, s));
  PAFEM_TRY_HIP(launch_dot_partial<double>(r, r, n, part, nb, nullptr, s));
  PAFEM_TRY_HIP(launch_sum_final(part, nb, 1, dev, s));
  double v[2] = {0.0, 0.0};
  PAFEM_TRY_HIP(hipMemcpyAsync(v, dev, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  PAFEM_TRY_HIP(hipStreamSynchronize(s));
  out = v[1] > 0.0 ? std::sqrt(v[0] / v[1]) : std::sqrt(v[0]);
  return PAFEM_OK;
}

int ensure_dinv(Op* op, hipStream_t s, bool want32) {
  Space* sp = op->space;
  const int64_t n = sp->ndofs;
  if (!op->have_dinv || (want32 && !op->d_dinv32.ptr)) {
    PAFEM_TRY(op->d_dinv64.ensure(n * sizeof(double)));
    PAFEM_TRY(op->d_dinv32.ensure(n * sizeof(float)));
    double* d = op->d_dinv64.as<double>();
    PAFEM_TRY(diagonal_impl(op, d, 1, s));
    PAFEM_TRY(ensure_ess(sp, true));
    PAFEM_TRY_HIP(launch_set_ess<double>(sp->d_ess.as<int32_t>(), (int64_t)sp->ess.size(), nullptr,
                                         1.0, 0, d, nullptr, s));
    PAFEM_TRY_HIP(launch_recip(d, d, op->d_dinv32.as<float>(), n, s));
    op->have_dinv = true;
  }
  return PAFEM_OK;
}

}  // namespace pafem

using namespace pafem;

extern "C" int pafem_solve_cg(pafem_op* op_, const double* b, double* x,
                              const pafem_solve_opts* o, pafem_solve_stats* stats,
                              void* stream) {
  clear_error();
  Op* op = op_;
  if (!op || !b || !x || !o || !stats) {
    set_error("NULL argument");
    return PAFEM_ERR_INVALID_ARG;
  }
  if (!(o->rtol > 0.0) || o->maxit < 1 || o->check_every < 1) {
    set_error("need rtol > 0, maxit >= 1, check_every >= 1");
    return PAFEM_ERR_INVALID_ARG;
  }
  if (o->mode < PAFEM_SOLVE_PLAIN_FP64 || o->mode > PAFEM_SOLVE_MIXED_BF16) {
    set_error("unknown solve mode");
    return PAFEM_ERR_INVALID_ARG;
  }
  const bool mixed = o->mode == PAFEM_SOLVE_MIXED_FP32 || o->mode == PAFEM_SOLVE_MIXED_BF16;
  if (o->launch < PAFEM_LAUNCH_KERNELS || o->launch > PAFEM_LAUNCH_PERSISTENT) {
    set_error("unknown launch form");
    return PAFEM_ERR_INVALID_ARG;
  }
  if ((mixed && o->launch != PAFEM_LAUNCH_KERNELS) ||
      (o->launch == PAFEM_LAUNCH_PERSISTENT &&
       (o->mode != PAFEM_SOLVE_PLAIN_FP64 || !fused_cg(op) ||
        op->level != PAFEM_ASSEMBLY_PARTIAL))) {
    set_error("launch form not available for this mode (graph: PLAIN_FP64 and IR; persistent: "
              "PLAIN_FP64 with the deterministic E^T on the lattice numbering, stored "
              "quadrature data and q = p + 2)");
    return PAFEM_ERR_INVALID_ARG;
  }
  if (mixed && !(o->inner_rtol > 0.0 && o->inner_rtol < 1.0)) {
    set_error("MIXED modes need inner_rtol (the replacement factor) in (0, 1)");
    return PAFEM_ERR_INVALID_ARG;
  }
  const bool ir = o->mode != PAFEM_SOLVE_PLAIN_FP64;
  const bool bf16 = o->mode == PAFEM_SOLVE_IR_BF16 || o->mode == PAFEM_SOLVE_MIXED_BF16;
  if (!op->have64 || (ir && !bf16 && !op->have32) || (bf16 && !op->have16)) {
    set_error("operator not assembled in the precision the mode needs");
    return PAFEM_ERR_INVALID_ARG;
  }
  if (op->space->mesh->ctx->host_only) {
    set_error("solve needs a GPU context");
    return PAFEM_ERR_UNSUPPORTED;
  }
  PAFEM_TRY_HIP(hipSetDevice(op->space->mesh->ctx->device));
  hipStream_t s = S(stream);
  const auto t0 = std::chrono::steady_clock::now();
  Space* sp = op->space;
  const int64_t n = sp->ndofs;
  *stats = pafem_solve_stats{};

  PAFEM_TRY(ensure_dinv(op, s, ir));
  // workspace: 3 FP64 vectors, plus 4 FP32 vectors for IR, plus the solution
  // for the graph form (so that the captured iterations outlive one call)
  const size_t need = 3 * n * sizeof(double) + (ir ? 4 * n * sizeof(float) : 0);
  PAFEM_TRY(op->d_cg.ensure(need + n * sizeof(double)));
  double* r = op->d_cg.as<double>();
  double* p = r + n;
  double* Ap = p + n;
  double* x_graph = reinterpret_cast<double*>(reinterpret_cast<char*>(op->d_cg.ptr) + need);

  int rc = PAFEM_OK;
  if (mixed) {
    float* rs = reinterpret_cast<float*>(Ap + n);
    float* p32 = rs + n;
    float* Ap32 = p32 + n;
    CgResult res;
    int repl = 0;
    PAFEM_TRY(run_mixed(op, b, x, r, p, rs, p32, Ap32, op->d_dinv32.as<float>(), o->rtol,
                        o->inner_rtol, o->maxit, o->check_every, bf16 ? PAFEM_BF16 : PAFEM_FP32,
                        s, res, repl));
    stats->iterations = res.iterations;
    stats->outer_iterations = repl;
    stats->rel_res = res.bb > 0 ? std::sqrt(res.rr / res.bb) : std::sqrt(res.rr);
    PAFEM_TRY(true_residual(op, b, x, Ap, r, res.bb, s, stats->true_rel_res));
    if (!res.converged) rc = PAFEM_ERR_NOT_CONVERGED;
  } else if (o->mode == PAFEM_SOLVE_PLAIN_FP64) {
    // Convergence is confirmed on the FP64 residual b - A x: the recursively
    // updated residual drifts from it by rounding over many iterations, so
    // when the recursive one meets rtol but the true one does not, CG restarts
    // from the current x with r = b - A x, until the true residual meets rtol
    // or the iteration budget is spent.
    int total = 0, restarts = 0;
    bool ok = false;
    double rel = 0.0, true_rel = 0.0;
    double* xs = x;
    if (o->launch == PAFEM_LAUNCH_GRAPH) {
      xs = x_graph;
      PAFEM_TRY_HIP(hipMemcpyAsync(xs, x, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    for (;;) {
      CgResult res;
      // with more than one iteration per host check, the FP64 residual check
      // rides behind each batch (no separate round trip)
      PAFEM_TRY(run_pcg<double>(op, b, xs, false, r, p, Ap, op->d_dinv64.as<double>(), o->rtol,
                                o->maxit - total, o->check_every, s, res, 0, o->launch,
                                o->check_every > 1 ? b : nullptr));
      total += res.iterations;
      rel = res.bb > 0 ? std::sqrt(res.rr / res.bb) : 0.0;
      if (res.true_rr >= 0.0)
        true_rel = res.bb > 0.0 ? std::sqrt(res.true_rr / res.bb) : std::sqrt(res.true_rr);
      else
        PAFEM_TRY(true_residual(op, b, xs, Ap, r, res.bb, s, true_rel));
      if (true_rel <= o->rtol) {
        ok = true;
        break;
      }
      if (!res.converged || total >= o->maxit || res.iterations == 0) break;
      ++restarts;
    }
    if (xs != x)
      PAFEM_TRY_HIP(hipMemcpyAsync(x, xs, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    stats->iterations = total;
    stats->outer_iterations = restarts;
    stats->rel_res = rel;
    stats->true_rel_res = true_rel;
    if (!ok) rc = PAFEM_ERR_NOT_CONVERGED;
  } else {
    float* d32 = reinterpret_cast<float*>(Ap + n);
    float* r32 = d32 + n;
    float* p32 = r32 + n;
    float* Ap32 = p32 + n;
    const int nb = reduce_blocks(n);
    PAFEM_TRY(ensure_partials(op, n));
    double* part = op->d_part.as<double>();
    double* rr_dev = part + 2 * partial_pairs(n) + 2;  // ||r||^2 of the current outer residual
    // bb
    PAFEM_TRY_HIP(launch_dot_partial<double>(b, b, n, part, nb, nullptr, s));
    PAFEM_TRY_HIP(launch_sum_final(part, nb, 1, rr_dev, s));
    double bb = 0.0;
    PAFEM_TRY_HIP(hipMemcpyAsync(&bb, rr_dev, sizeof(double), hipMemcpyDeviceToHost, s));
    PAFEM_TRY_HIP(hipStreamSynchronize(s));
    // r = b - A x (FP64)
    PAFEM_TRY(apply_impl<double>(op, x, Ap, PAFEM_APPLY_CONSTRAINED, nullptr, s));
    PAFEM_TRY_HIP(launch_residual(b, Ap, r, n, s));
    int total_inner = 0, outer = 0, n64 = 0;
    double rel = 0.0, rel_prev = 0.0;
    bool ok = false, use64 = false, after32 = false;
    const double inner_rtol = o->inner_rtol > 0 ? o->inner_rtol : 1e-4;
    for (;;) {
      PAFEM_TRY_HIP(launch_dot_partial<double>(r, r, n, part, nb, nullptr, s));
      PAFEM_TRY_HIP(launch_sum_final(part, nb, 1, rr_dev, s));
      double rr = 0.0;
      PAFEM_TRY_HIP(hipMemcpyAsync(&rr, rr_dev, sizeof(double), hipMemcpyDeviceToHost, s));
      PAFEM_TRY_HIP(hipStreamSynchronize(s));
      rel = bb > 0.0 ? std::sqrt(rr / bb) : std::sqrt(rr);
      if (rel <= o->rtol) {
        ok = true;
        break;
      }
      if (!std::isfinite(rel) || outer >= o->max_outer) break;
      // a reduced-precision correction that did not reduce the FP64 residual
      // by a tenth: the inner solves continue in FP64
      if (after32 && !(rel <= kIrStagnation * rel_prev)) use64 = true;
      rel_prev = rel;
      after32 = false;
      if (!use64) {
        // inner FP32 solve of A d = r / ||r||
        PAFEM_TRY_HIP(launch_scale_to_f32(r, rr_dev, r32, n, s));
        CgResult res;
        // the inner solve overwrites the partials; keep ||r||^2 in its own slot
        PAFEM_TRY(run_pcg<float>(op, r32, d32, true, r32, p32, Ap32, op->d_dinv32.as<float>(),
                                 inner_rtol, o->maxit, o->check_every, s, res,
                                 o->mode == PAFEM_SOLVE_IR_BF16 ? PAFEM_BF16 : PAFEM_FP32,
                                 o->launch));
        total_inner += res.iterations;
        if (std::isfinite(res.rr)) {
          PAFEM_TRY_HIP(launch_axpy_from_f32(x, rr_dev, d32, n, s));
          after32 = true;
        } else {
          use64 = true;  // overflow or NaN in reduced precision: discard the correction
        }
      }
      if (use64) {
        // FP64 inner solve: CG from the current x, reducing the residual by
        // inner_rtol (not beyond rtol / 2)
        CgResult res;
        const double target = std::max(rel * inner_rtol, 0.5 * o->rtol);
        PAFEM_TRY(run_pcg<double>(op, b, x, false, r, p, Ap, op->d_dinv64.as<double>(), target,
                                  o->maxit, o->check_every, s, res));
        total_inner += res.iterations;
        ++n64;
      }
      PAFEM_TRY(apply_impl<double>(op, x, Ap, PAFEM_APPLY_CONSTRAINED, nullptr, s));
      PAFEM_TRY_HIP(launch_residual(b, Ap, r, n, s));
      ++outer;
    }
    stats->fp64_inner_solves = n64;
    stats->iterations = total_inner;
    stats->outer_iterations = outer;
    stats->rel_res = rel;
    stats->true_rel_res = rel;
    if (!ok) rc = PAFEM_ERR_NOT_CONVERGED;
  }
  PAFEM_TRY_HIP(hipStreamSynchronize(s));
  stats->seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (rc == PAFEM_ERR_NOT_CONVERGED) set_error("iteration limit reached before rtol");
  return rc;
}
