// Serving engine: continuous batching of Poisson solves on one GPU.
//
// Host side: a request queue (thread-safe submit/poll), FIFO admission while a
// slot is free and the request's device footprint fits the budget, an engine
// thread that runs the rounds, and a setup thread that builds each admitted
// request's operator, diagonal and right-hand side on its own stream while
// the rounds of the others go on; a request joins its batch at the first
// round boundary after its setup has completed.  Device side: two batches
// (FP64 CG for plain requests; FP32-operator CG for the inner solves of
// refined requests and for mixed requests, whose solution is kept in FP64 and
// whose residual is replaced by the FP64 one between rounds), each replaying
// one captured HIP graph per round on its own stream.  The graph's kernels
// read the batch membership from a device table, so admission and retirement
// only rewrite that table between replays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"

namespace pafem {

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
  uint64_t ticket = 0;
  pafem_request spec{};
  std::vector<double> verts;
  int64_t ndofs = 0, ne = 0, footprint = 0;
  // reported (guarded by the server mutex)
  int status = PAFEM_REQ_QUEUED;
  int error = 0;
  int iterations = 0, outer = 0;
  double rel_res = 0.0;
  double t_arrive = -1.0, t_admit = -1.0, t_done = -1.0;
  std::vector<double> solution;
  bool has_solution = false;
  // device side (engine thread only)
  pafem_mesh* mesh = nullptr;
  pafem_space* space = nullptr;
  pafem_op* op = nullptr;
  int slot = -1;
  DevBuf v64;   // b, x, r, dir, Ad
  DevBuf v32;   // d, r, dir, Ad (inner FP32 solve)
  DevBuf part;  // reduction partials + device scalars
  double bb = 0.0;
  bool ir = false;     // FP64 defect correction around FP32 inner solves
  bool mixed = false;  // one FP32 CG with FP64 solution and residual replacement
  double* b() const { return v64.as<double>(); }
  double* x() const { return v64.as<double>() + ndofs; }
  double* r() const { return v64.as<double>() + 2 * ndofs; }
  double* dir() const { return v64.as<double>() + 3 * ndofs; }
  double* Ad() const { return v64.as<double>() + 4 * ndofs; }
  float* d32() const { return v32.as<float>(); }
  float* r32() const { return v32.as<float>() + ndofs; }
  float* dir32() const { return v32.as<float>() + 2 * ndofs; }
  float* Ad32() const { return v32.as<float>() + 3 * ndofs; }
  int nchunks() const { return (int)((ndofs + kBatchChunk - 1) / kBatchChunk); }
  int nparts() const { return std::max(2 * reduce_blocks(ndofs), 2 * nchunks()); }
  double* partials() const { return part.as<double>(); }
  double* rr_dev() const { return part.as<double>() + nparts(); }   // ||r||^2 of the outer residual
  double* tmp_dev() const { return part.as<double>() + nparts() + 1; }
};

template <typename T>
struct Batch {
  std::vector<Req*> members;
  DevBuf d_entries, d_hdr;
  BatchEntry<T>* h_entries = nullptr;  // pinned staging
  BatchHeader* h_hdr = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool dirty = true;
};

}  // namespace

struct Server {
  pafem_ctx* ctx = nullptr;
  int device = 0;
  int64_t budget = 0;
  int max_slots = 0;
  int iters = 1;
  Clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> queue;
  std::map<uint64_t, std::unique_ptr<Req>> reqs;
  uint64_t next_ticket = 1;
  bool stopping = false;
  int64_t n_submitted = 0, n_completed = 0, n_failed = 0, n_rounds = 0;
  int64_t used = 0, peak = 0;
  int max_active = 0;
  double dof_iters = 0.0;
  int startup_error = 0;
  std::string startup_message;

  // engine thread; the FP64 batch and the per-request work between rounds run
  // on `stream`, the FP32 batch on `stream32`
  std::thread th;
  hipStream_t stream = nullptr;
  hipStream_t stream32 = nullptr;
  hipEvent_t main_done = nullptr;  // orders the FP32 batch after the work between rounds
  // setup worker: admitted requests build their operator, diagonal and
  // right-hand side on `setup_stream` while the rounds of the others go on
  std::thread setup_th;
  hipStream_t setup_stream = nullptr;
  std::deque<Req*> to_setup;                 // guarded by mu
  std::vector<std::pair<Req*, int>> ready;   // set up (or failed), guarded by mu
  int setting_up = 0;                        // admitted, not yet in a batch (engine only)
  std::condition_variable cv_setup;
  DevBuf d_states;                 // CgState[max_slots]
  CgState* h_states = nullptr;     // pinned mirror
  std::vector<int> free_slots;
  std::vector<Req*> active;
  Batch<double> b64;
  Batch<float> b32;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

int64_t footprint_of(const pafem_request& r) {
  if (r.nx < 1 || r.ny < 1 || r.nz < 1 || r.p < 1 || r.p > kMaxP) return -1;
  const int64_t p = r.p, n = p + 1, q = p + 2;
  const int64_t ne = (int64_t)r.nx * r.ny * r.nz;
  const int64_t nd = ((int64_t)r.nx * p + 1) * ((int64_t)r.ny * p + 1) * ((int64_t)r.nz * p + 1);
  const bool ir = r.mode == PAFEM_SOLVE_IR_FP32 || r.mode == PAFEM_SOLVE_MIXED_FP32;
  int64_t b = ne * q * q * q * 6 * 8;              // FP64 quadrature data
  if (ir) b += ne * q * q * q * 6 * 4;             // FP32 copy
  b += evec_words(ne, (int)n) * 8;                 // E-vector workspace
  b += nd * (5 * 8 + 8 + 4);                       // FP64 vectors, dinv (64 + 32)
  if (ir) b += nd * 4 * 4;                         // FP32 vectors
  b += (int64_t)(r.nx + 1) * (r.ny + 1) * (r.nz + 1) * 24;  // vertices
  b += 2 * (2 * 2048 + nd / kBatchChunk + 64) * 8 + 4096;    // partials, tables
  return b;
}

int request_valid(const pafem_request& r) {
  if (footprint_of(r) < 0) return 0;
  if (r.verts_host == nullptr) return 0;
  if (r.mode != PAFEM_SOLVE_PLAIN_FP64 && r.mode != PAFEM_SOLVE_IR_FP32 &&
      r.mode != PAFEM_SOLVE_MIXED_FP32)
    return 0;
  if (r.mode == PAFEM_SOLVE_MIXED_FP32 && !(r.inner_rtol > 0.0 && r.inner_rtol < 1.0)) return 0;
  if (r.coef_kind != PAFEM_COEF_CONST && r.coef_kind != PAFEM_COEF_SINX) return 0;
  if (!(r.rtol > 0.0) || r.maxit < 1) return 0;
  if (r.mode == PAFEM_SOLVE_IR_FP32 && (!(r.inner_rtol > 0.0) || r.max_outer < 1)) return 0;
  const int64_t ne = (int64_t)r.nx * r.ny * r.nz, n = r.p + 1;
  const int64_t nd = ((int64_t)r.nx * r.p + 1) * ((int64_t)r.ny * r.p + 1) * ((int64_t)r.nz * r.p + 1);
  if (evec_words(ne, (int)n) >= INT32_MAX || nd >= INT32_MAX) return 0;
  return 1;
}

template <typename T>
int batch_init(Batch<T>& b, int max_slots) {
  PAFEM_TRY(b.d_entries.ensure(sizeof(BatchEntry<T>) * max_slots));
  PAFEM_TRY(b.d_hdr.ensure(sizeof(BatchHeader)));
  PAFEM_TRY_HIP(hipHostMalloc((void**)&b.h_entries, sizeof(BatchEntry<T>) * max_slots));
  PAFEM_TRY_HIP(hipHostMalloc((void**)&b.h_hdr, sizeof(BatchHeader)));
  std::memset(b.h_entries, 0, sizeof(BatchEntry<T>) * max_slots);
  std::memset(b.h_hdr, 0, sizeof(BatchHeader));
  return PAFEM_OK;
}

template <typename T>
void batch_free(Batch<T>& b) {
  if (b.exec) (void)hipGraphExecDestroy(b.exec);
  if (b.graph) (void)hipGraphDestroy(b.graph);
  if (b.h_entries) (void)hipHostFree(b.h_entries);
  if (b.h_hdr) (void)hipHostFree(b.h_hdr);
  b.exec = nullptr;
  b.graph = nullptr;
  b.h_entries = nullptr;
  b.h_hdr = nullptr;
}

template <typename T>
BatchEntry<T> make_entry(Server& S, Req* r, int64_t work_begin, int64_t chunk_begin) {
  Op* op = r->op;
  Space* sp = op->space;
  const int n = sp->p + 1, q = op->q;
  const bool f32 = std::is_same<T, float>::value;
  const DevBuf& tab = f32 ? op->d_tab32 : op->d_tab64;
  BatchEntry<T> e{};
  e.p = sp->p;
  e.ndofs = sp->ndofs;
  e.nchunks = r->nchunks();
  e.work_begin = work_begin;
  const int ne_item = batch_elems<T>(sp->p);
  e.work_end = work_begin + (sp->ne + ne_item - 1) / ne_item;
  e.chunk_begin = chunk_begin;
  e.chunk_end = chunk_begin + e.nchunks;
  e.st = S.d_states.as<CgState>() + r->slot;
  e.partials = r->partials();
  e.x64 = r->mixed ? r->x() : nullptr;
  if (f32) {
    e.x = (T*)r->d32();
    e.r = (T*)r->r32();
    e.dir = (T*)r->dir32();
    e.Ad = (T*)r->Ad32();
    e.dinv = (const T*)op->d_dinv32.ptr;
  } else {
    e.x = (T*)r->x();
    e.r = (T*)r->r();
    e.dir = (T*)r->dir();
    e.Ad = (T*)r->Ad();
    e.dinv = (const T*)op->d_dinv64.ptr;
  }
  ApplyArgs<T>& a = e.a;
  a.x = e.dir;
  a.y = e.Ad;
  a.yE = op->d_evec.as<T>();
  a.qd = f32 ? (const T*)op->d_qd32.ptr : (const T*)op->d_qd64.ptr;
  a.B = tab.as<T>();
  a.G = tab.as<T>() + q * n;
  a.ne = sp->ne;
  a.nx = sp->mesh->nx;
  a.ny = sp->mesh->ny;
  a.nz = sp->mesh->nz;
  a.constrained = 1;
  a.accumulate = 0;
  a.skip = &e.st->done;
  return e;
}

// Device pointers of an entry as byte offsets from the device table `base`
// (the batched kernels rebuild them from their table argument).
template <typename P>
P* offset_from(const void* base, P* p) {
  return p == nullptr ? nullptr
                      : (P*)(intptr_t)((const char*)p - (const char*)base);
}
template <typename T>
BatchEntry<T> as_offsets(const void* base, BatchEntry<T> e) {
  e.a.x = offset_from(base, e.a.x);
  e.a.y = offset_from(base, e.a.y);
  e.a.yE = offset_from(base, e.a.yE);
  e.a.qd = offset_from(base, e.a.qd);
  e.a.qd16 = offset_from(base, e.a.qd16);
  e.a.E = offset_from(base, e.a.E);
  e.a.ess_mask = offset_from(base, e.a.ess_mask);
  e.a.B = offset_from(base, e.a.B);
  e.a.G = offset_from(base, e.a.G);
  e.a.skip = offset_from(base, e.a.skip);
  e.x = offset_from(base, e.x);
  e.r = offset_from(base, e.r);
  e.dir = offset_from(base, e.dir);
  e.Ad = offset_from(base, e.Ad);
  e.dinv = offset_from(base, e.dinv);
  e.st = offset_from(base, e.st);
  e.partials = offset_from(base, e.partials);
  e.x64 = offset_from(base, e.x64);
  return e;
}

// Rewrite the device table of a batch: entries grouped by order p (each
// order's element pass is its own launch over its range of work items), in
// admission order within an order.
template <typename T>
hipStream_t batch_stream(const Server& S) {
  return std::is_same<T, float>::value ? S.stream32 : S.stream;
}

template <typename T>
int batch_upload(Server& S, Batch<T>& b) {
  const hipStream_t bs = batch_stream<T>(S);
  int64_t w = 0, c = 0;
  size_t i = 0;
  for (int p = 1; p <= kMaxP; ++p) {
    b.h_hdr->p_begin[p] = w;
    for (Req* r : b.members) {
      if (r->spec.p != p) continue;
      b.h_entries[i] = as_offsets(b.d_entries.ptr, make_entry<T>(S, r, w, c));
      w = b.h_entries[i].work_end;
      c = b.h_entries[i].chunk_end;
      ++i;
    }
    b.h_hdr->p_end[p] = w;
  }
  b.h_hdr->p_begin[0] = b.h_hdr->p_end[0] = 0;
  b.h_hdr->n = (int)b.members.size();
  b.h_hdr->total_work = w;
  b.h_hdr->total_chunks = c;
  if (!b.members.empty())
    PAFEM_TRY_HIP(hipMemcpyAsync(b.d_entries.ptr, b.h_entries,
                                 sizeof(BatchEntry<T>) * b.members.size(),
                                 hipMemcpyHostToDevice, bs));
  PAFEM_TRY_HIP(hipMemcpyAsync(b.d_hdr.ptr, b.h_hdr, sizeof(BatchHeader), hipMemcpyHostToDevice,
                               bs));
  // the pinned staging is reused next round: wait for the copies to leave it
  PAFEM_TRY_HIP(hipStreamSynchronize(bs));
  b.dirty = false;
  return PAFEM_OK;
}

// The K iterations of a batch as one graph.  Its launch shapes do not depend
// on the members (the kernels read the table), so it is captured once, when
// the server is created and before its threads start: no capture is ever in
// progress while the setup thread makes synchronous calls.
template <typename T>
int batch_capture(Server& S, Batch<T>& b) {
  const hipStream_t bs = batch_stream<T>(S);
  PAFEM_TRY_HIP(hipStreamBeginCapture(bs, hipStreamCaptureModeThreadLocal));
  hipError_t le = launch_batch_iterations<T>(b.d_entries.template as<BatchEntry<T>>(),
                                             b.d_hdr.template as<BatchHeader>(), S.max_slots,
                                             S.iters, bs);
  hipError_t ce = hipStreamEndCapture(bs, &b.graph);
  PAFEM_TRY_HIP(le);
  PAFEM_TRY_HIP(ce);
  PAFEM_TRY_HIP(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
  return PAFEM_OK;
}

template <typename T>
int batch_round(Server& S, Batch<T>& b) {
  if (b.members.empty()) return PAFEM_OK;
  const hipStream_t bs = batch_stream<T>(S);
  if (b.dirty) PAFEM_TRY(batch_upload(S, b));
  PAFEM_TRY_HIP(hipGraphLaunch(b.exec, bs));
  return PAFEM_OK;
}

// CG start on the request's slot: r holds the right-hand side of this solve,
// x its zero initial guess; bb scales the stopping test.
template <typename T>
int cg_start(Server& S, Req* r, T* rr, T* dir, const T* dinv, double bb, double rtol,
             hipStream_t s) {
  const int nb = reduce_blocks(r->ndofs);
  PAFEM_TRY_HIP(launch_cg_init<T>(rr, dinv, dir, r->ndofs, r->partials(), nb, s));
  PAFEM_TRY_HIP(launch_cg_init_final(r->partials(), nb, bb, rtol, r->spec.maxit,
                                     S.d_states.as<CgState>() + r->slot, s));
  return PAFEM_OK;
}

int dot_to_host(Req* r, const double* a, const double* b, double* dev, double& out,
                hipStream_t s) {
  const int nb = reduce_blocks(r->ndofs);
  PAFEM_TRY_HIP(launch_dot_partial<double>(a, b, r->ndofs, r->partials(), nb, nullptr, s));
  PAFEM_TRY_HIP(launch_sum_final(r->partials(), nb, 1, dev, s));
  PAFEM_TRY_HIP(hipMemcpyAsync(&out, dev, sizeof(double), hipMemcpyDeviceToHost, s));
  PAFEM_TRY_HIP(hipStreamSynchronize(s));
  return PAFEM_OK;
}

// Inner FP32 solve of A d = r / ||r|| with d = 0 to start.
int start_inner(Server& S, Req* r, hipStream_t s) {
  const int64_t n = r->ndofs;
  PAFEM_TRY_HIP(launch_scale_to_f32(r->r(), r->rr_dev(), r->r32(), n, s));
  PAFEM_TRY_HIP(launch_fill<float>(r->d32(), n, 0.0f, nullptr, s));
  return cg_start<float>(S, r, r->r32(), r->dir32(), r->op->d_dinv32.as<float>(), 1.0,
                         r->spec.inner_rtol, s);
}

// Build a request's operator, diagonal, right-hand side and CG start on
// stream s (synchronous on s only).
int setup(Server& S, Req* r, hipStream_t s) {
  const pafem_request& q = r->spec;
  PAFEM_TRY(pafem_mesh_create_structured(S.ctx, q.nx, q.ny, q.nz, r->verts.data(), &r->mesh));
  PAFEM_TRY(pafem_space_create(r->mesh, q.p, &r->space));
  PAFEM_TRY(pafem_op_create(r->space, PAFEM_DIFFUSION, 0, &r->op));
  if (q.coef_kind == PAFEM_COEF_SINX)
    PAFEM_TRY(pafem_op_set_coefficient_sinx(r->op, q.coef_value));
  else
    PAFEM_TRY(pafem_op_set_coefficient_const(r->op, q.coef_value));
  const bool f32 = r->ir || r->mixed;
  PAFEM_TRY(pafem_op_assemble(r->op, PAFEM_FP64 | (f32 ? PAFEM_FP32 : 0), s));
  const int64_t n = r->ndofs;
  PAFEM_TRY(r->v64.ensure(5 * n * sizeof(double)));
  if (f32) PAFEM_TRY(r->v32.ensure(4 * n * sizeof(float)));
  PAFEM_TRY(r->part.ensure((r->nparts() + 8) * sizeof(double)));
  PAFEM_TRY(pafem_rhs_assemble(r->op, nullptr, r->b(), s));
  PAFEM_TRY(ensure_dinv(r->op, s, f32));
  PAFEM_TRY_HIP(launch_fill<double>(r->x(), n, 0.0, nullptr, s));
  PAFEM_TRY_HIP(hipMemcpyAsync(r->r(), r->b(), n * sizeof(double), hipMemcpyDeviceToDevice,
                               s));
  PAFEM_TRY(dot_to_host(r, r->b(), r->b(), r->rr_dev(), r->bb, s));
  if (r->mixed) {
    // x = 0: the FP64 residual is b; rs = (float) b, dir = dinv .* rs
    const int nb = reduce_blocks(n);
    CgState* st = S.d_states.as<CgState>() + r->slot;
    const float* dinv32 = r->op->d_dinv32.as<float>();
    PAFEM_TRY_HIP(launch_replace_residual(r->r(), dinv32, r->r32(), n, r->partials(), nb, nullptr,
                                          s));
    PAFEM_TRY_HIP(launch_cg_init_final(r->partials(), nb, r->bb, q.rtol, q.maxit, st, s,
                                       q.inner_rtol * q.inner_rtol));
    PAFEM_TRY_HIP(launch_fill<float>(r->dir32(), n, 0.0f, nullptr, s));
    PAFEM_TRY_HIP(launch_cg_pupdate<float>(r->dir32(), r->r32(), dinv32, n, st, s));
    return PAFEM_OK;
  }
  if (r->ir) return start_inner(S, r, s);  // rr_dev holds ||r||^2 = ||b||^2
  return cg_start<double>(S, r, r->r(), r->dir(), r->op->d_dinv64.as<double>(), r->bb,
                          q.rtol, s);
}

void release_device(Server& S, Req* r) {
  (void)S;
  r->v64.release();
  r->v32.release();
  r->part.release();
  if (r->op) pafem_op_destroy(r->op);
  if (r->space) pafem_space_destroy(r->space);
  if (r->mesh) pafem_mesh_destroy(r->mesh);
  r->op = nullptr;
  r->space = nullptr;
  r->mesh = nullptr;
}

template <typename T>
void batch_remove(Batch<T>& b, Req* r) {
  auto it = std::find(b.members.begin(), b.members.end(), r);
  if (it != b.members.end()) {
    b.members.erase(it);
    b.dirty = true;
  }
}

// Finish a request: record the outcome, copy x to the host, free its memory.
void finish(Server& S, Req* r, int err, bool keep_x) {
  std::vector<double> x;
  if (keep_x && r->op) {
    x.resize(r->ndofs);
    if (hipMemcpyAsync(x.data(), r->x(), r->ndofs * sizeof(double), hipMemcpyDeviceToHost,
                       S.stream) != hipSuccess ||
        hipStreamSynchronize(S.stream) != hipSuccess) {
      err = PAFEM_ERR_HIP;
      x.clear();
    }
  }
  batch_remove(S.b64, r);
  batch_remove(S.b32, r);
  auto it = std::find(S.active.begin(), S.active.end(), r);
  if (it != S.active.end()) S.active.erase(it);
  if (r->slot >= 0) S.free_slots.push_back(r->slot);
  r->slot = -1;
  release_device(S, r);
  std::lock_guard<std::mutex> g(S.mu);
  S.used -= r->footprint;
  r->error = err;
  r->status = (err == PAFEM_OK) ? PAFEM_REQ_DONE : PAFEM_REQ_FAILED;
  r->t_done = S.now();
  if (!x.empty()) {
    r->solution.swap(x);
    r->has_solution = true;
  }
  if (err == PAFEM_OK) {
    ++S.n_completed;
    S.dof_iters += (double)r->ndofs * r->iterations;
  } else {
    ++S.n_failed;
  }
  S.cv_done.notify_all();
}

// Relative FP64 residual ||b - A x|| / ||b|| (uses r and Ad as scratch).
int true_residual(Server& S, Req* r, double& rel) {
  PAFEM_TRY(apply_impl<double>(r->op, r->x(), r->Ad(), PAFEM_APPLY_CONSTRAINED, nullptr,
                               S.stream));
  PAFEM_TRY_HIP(launch_residual(r->b(), r->Ad(), r->r(), r->ndofs, S.stream));
  double rr = 0.0;
  PAFEM_TRY(dot_to_host(r, r->r(), r->r(), r->rr_dev(), rr, S.stream));
  rel = r->bb > 0.0 ? std::sqrt(rr / r->bb) : std::sqrt(rr);
  return PAFEM_OK;
}

// Mixed CGs paused (or stopped on their recursive residual): replace each
// FP32 residual by the FP64 one (all requests' work enqueued, then one read of
// the states); finish a request when that meets the tolerance (or maxit),
// else complete its paused iteration's direction update and continue.
void replace_residuals(Server& S, std::vector<Req*> reqs) {
  std::vector<Req*> ok;
  for (Req* r : reqs) {
    const int64_t n = r->ndofs;
    CgState* st = S.d_states.as<CgState>() + r->slot;
    int rc = apply_impl<double>(r->op, r->x(), r->Ad(), PAFEM_APPLY_CONSTRAINED, nullptr,
                                S.stream);
    if (rc == PAFEM_OK &&
        (launch_residual(r->b(), r->Ad(), r->r(), n, S.stream) != hipSuccess ||
         launch_replace_residual(r->r(), r->op->d_dinv32.as<float>(), r->r32(), n,
                                 r->partials(), reduce_blocks(n), st, S.stream) != hipSuccess))
      rc = PAFEM_ERR_HIP;
    if (rc != PAFEM_OK)
      finish(S, r, rc, false);
    else
      ok.push_back(r);
  }
  if (ok.empty()) return;
  if (hipMemcpyAsync(S.h_states, S.d_states.ptr, sizeof(CgState) * S.max_slots,
                     hipMemcpyDeviceToHost, S.stream) != hipSuccess ||
      hipStreamSynchronize(S.stream) != hipSuccess) {
    for (Req* r : ok) finish(S, r, PAFEM_ERR_HIP, false);
    return;
  }
  for (Req* r : ok) {
    const CgState hs = S.h_states[r->slot];
    {
      std::lock_guard<std::mutex> g(S.mu);
      r->iterations = hs.iter;
      r->outer += 1;
      r->rel_res = r->bb > 0.0 ? std::sqrt(hs.rr / r->bb) : std::sqrt(hs.rr);
    }
    if (hs.done) {
      finish(S, r, hs.rr <= hs.rr_stop ? PAFEM_OK : PAFEM_ERR_NOT_CONVERGED, true);
    } else if (launch_cg_pupdate<float>(r->dir32(), r->r32(), r->op->d_dinv32.as<float>(),
                                        r->ndofs, S.d_states.as<CgState>() + r->slot,
                                        S.stream) != hipSuccess) {
      finish(S, r, PAFEM_ERR_HIP, false);
    }
  }
}

// A request whose current CG has stopped: finish it, or take a refinement step.
void on_cg_done(Server& S, Req* r, const CgState& st) {
  if (!r->ir) {
    double rel = 0.0;
    int rc = true_residual(S, r, rel);
    {
      std::lock_guard<std::mutex> g(S.mu);
      r->iterations = st.iter;
      r->rel_res = rel;
    }
    if (rc != PAFEM_OK) return finish(S, r, rc, false);
    const bool conv = st.rr <= st.rr_stop;
    return finish(S, r, conv ? PAFEM_OK : PAFEM_ERR_NOT_CONVERGED, true);
  }
  // x += ||r|| d ; r = b - A x (FP64) ; test ; next inner solve
  int rc = PAFEM_OK;
  double rel = 0.0;
  {
    std::lock_guard<std::mutex> g(S.mu);
    r->iterations += st.iter;
    r->outer += 1;
  }
  if (launch_axpy_from_f32(r->x(), r->rr_dev(), r->d32(), r->ndofs, S.stream) != hipSuccess)
    rc = PAFEM_ERR_HIP;
  if (rc == PAFEM_OK) rc = true_residual(S, r, rel);  // leaves ||r||^2 in rr_dev
  if (rc != PAFEM_OK) return finish(S, r, rc, false);
  {
    std::lock_guard<std::mutex> g(S.mu);
    r->rel_res = rel;
  }
  if (rel <= r->spec.rtol) return finish(S, r, PAFEM_OK, true);
  if (r->outer >= r->spec.max_outer) return finish(S, r, PAFEM_ERR_NOT_CONVERGED, true);
  rc = start_inner(S, r, S.stream);
  if (rc != PAFEM_OK) finish(S, r, rc, false);
}

// Setup worker: admitted requests are set up here, one at a time, while the
// engine keeps replaying rounds for the others.
void setup_worker(Server& S) {
  (void)hipSetDevice(S.device);
  for (;;) {
    Req* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(S.mu);
      S.cv_setup.wait(lk, [&] { return S.stopping || !S.to_setup.empty(); });
      if (S.to_setup.empty()) return;  // stopping and nothing left
      r = S.to_setup.front();
      S.to_setup.pop_front();
    }
    int rc = setup(S, r, S.setup_stream);
    // the batches run on other streams: the setup must be complete first
    if (hipStreamSynchronize(S.setup_stream) != hipSuccess && rc == PAFEM_OK) rc = PAFEM_ERR_HIP;
    {
      std::lock_guard<std::mutex> g(S.mu);
      S.ready.emplace_back(r, rc);
    }
    S.cv_work.notify_all();
  }
}

void engine(Server& S) {
  (void)hipSetDevice(S.device);
  for (;;) {
    // ---- admission (FIFO while a slot is free and the footprint fits) ----
    std::vector<Req*> admit;
    std::vector<Req*> reject;
    std::vector<std::pair<Req*, int>> ready;
    {
      std::unique_lock<std::mutex> lk(S.mu);
      while (!S.queue.empty()) {
        Req* r = S.queue.front();
        if (r->footprint > S.budget) {
          S.queue.pop_front();
          reject.push_back(r);
          continue;
        }
        if ((int)(S.active.size() + S.setting_up + admit.size()) >= S.max_slots) break;
        if (S.used + r->footprint > S.budget) break;
        S.queue.pop_front();
        S.used += r->footprint;
        S.peak = std::max(S.peak, S.used);
        r->status = PAFEM_REQ_RUNNING;
        r->t_admit = S.now();
        admit.push_back(r);
      }
      // the slot is reserved before the setup thread can see the request: the
      // setup writes that slot's CG state
      for (Req* r : admit) {
        r->slot = S.free_slots.back();
        S.free_slots.pop_back();
        ++S.setting_up;
        S.to_setup.push_back(r);
      }
      ready.swap(S.ready);
      if (S.active.empty() && admit.empty() && reject.empty() && ready.empty()) {
        if (S.stopping && S.setting_up == 0) break;
        S.cv_work.wait_for(lk, std::chrono::milliseconds(20));
        continue;
      }
    }
    for (Req* r : reject) {
      r->footprint = 0;  // nothing was reserved
      finish(S, r, PAFEM_ERR_OUT_OF_MEMORY, false);
    }
    if (!admit.empty()) S.cv_setup.notify_all();
    for (auto& rr : ready) {
      Req* r = rr.first;
      --S.setting_up;
      S.active.push_back(r);
      if (rr.second != PAFEM_OK) {
        finish(S, r, rr.second, false);
        continue;
      }
      if (r->ir || r->mixed) {
        S.b32.members.push_back(r);
        S.b32.dirty = true;
      } else {
        S.b64.members.push_back(r);
        S.b64.dirty = true;
      }
    }
    {
      std::lock_guard<std::mutex> g(S.mu);
      S.max_active = std::max(S.max_active, (int)S.active.size());
    }
    if (S.active.empty()) continue;
    // ---- one round: K CG iterations for every batch member, the FP64 and
    // the FP32 batch on their own streams ----
    int rc = batch_round(S, S.b64);
    // the FP32 batch follows the work enqueued on the main stream between rounds
    if (rc == PAFEM_OK && (hipEventRecord(S.main_done, S.stream) != hipSuccess ||
                           hipStreamWaitEvent(S.stream32, S.main_done, 0) != hipSuccess))
      rc = PAFEM_ERR_HIP;
    if (rc == PAFEM_OK) rc = batch_round(S, S.b32);
    if (rc == PAFEM_OK && hipStreamSynchronize(S.stream32) != hipSuccess) rc = PAFEM_ERR_HIP;
    if (rc == PAFEM_OK &&
        (hipMemcpyAsync(S.h_states, S.d_states.ptr, sizeof(CgState) * S.max_slots,
                        hipMemcpyDeviceToHost, S.stream) != hipSuccess ||
         hipStreamSynchronize(S.stream) != hipSuccess))
      rc = PAFEM_ERR_HIP;
    {
      std::lock_guard<std::mutex> g(S.mu);
      ++S.n_rounds;
    }
    if (rc != PAFEM_OK) {
      std::vector<Req*> all = S.active;
      for (Req* r : all) finish(S, r, rc, false);
      continue;
    }
    std::vector<Req*> cur = S.active, paused;
    for (Req* r : cur) {
      const CgState st = S.h_states[r->slot];
      if (!st.done) continue;
      if (r->mixed)
        paused.push_back(r);
      else
        on_cg_done(S, r, st);
    }
    if (!paused.empty()) replace_residuals(S, paused);
  }
}

}  // namespace

}  // namespace pafem

using namespace pafem;

struct pafem_server : pafem::Server {};

extern "C" {

int64_t pafem_request_footprint(const pafem_request* req) {
  return req ? footprint_of(*req) : -1;
}

int pafem_server_create(pafem_ctx* ctx, int64_t budget, int max_slots, int iters,
                        pafem_server** out) {
  clear_error();
  if (!ctx || !out) {
    set_error("NULL argument");
    return PAFEM_ERR_INVALID_ARG;
  }
  *out = nullptr;
  if (ctx->host_only) {
    set_error("a server needs a GPU context");
    return PAFEM_ERR_UNSUPPORTED;
  }
  if (budget <= 0 || max_slots < 1 || max_slots > 64 || iters < 1) {
    set_error("need budget > 0, 1 <= max_slots <= 64, iters_per_round >= 1");
    return PAFEM_ERR_INVALID_ARG;
  }
  PAFEM_TRY_HIP(hipSetDevice(ctx->device));
  auto* S = new pafem_server();
  S->ctx = ctx;
  S->device = ctx->device;
  S->budget = budget;
  S->max_slots = max_slots;
  S->iters = iters;
  S->t0 = Clock::now();
  int rc = PAFEM_OK;
  // non-blocking streams: a synchronous copy of the setup thread on the null
  // stream neither waits for the rounds nor joins them
  if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&S->stream32, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&S->setup_stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&S->main_done, hipEventDisableTiming) != hipSuccess)
    rc = PAFEM_ERR_HIP;
  if (rc == PAFEM_OK) rc = S->d_states.ensure(sizeof(CgState) * max_slots);
  if (rc == PAFEM_OK &&
      hipHostMalloc((void**)&S->h_states, sizeof(CgState) * max_slots) != hipSuccess)
    rc = PAFEM_ERR_HIP;
  if (rc == PAFEM_OK) rc = batch_init(S->b64, max_slots);
  if (rc == PAFEM_OK) rc = batch_init(S->b32, max_slots);
  if (rc == PAFEM_OK) rc = batch_capture(*S, S->b64);
  if (rc == PAFEM_OK) rc = batch_capture(*S, S->b32);
  if (rc != PAFEM_OK) {
    batch_free(S->b64);
    batch_free(S->b32);
    if (S->h_states) (void)hipHostFree(S->h_states);
    if (S->stream) (void)hipStreamDestroy(S->stream);
    if (S->stream32) (void)hipStreamDestroy(S->stream32);
    if (S->setup_stream) (void)hipStreamDestroy(S->setup_stream);
    if (S->main_done) (void)hipEventDestroy(S->main_done);
    delete S;
    if (rc == PAFEM_ERR_HIP) set_error("HIP error creating the server");
    return rc;
  }
  for (int i = max_slots - 1; i >= 0; --i) S->free_slots.push_back(i);
  ++ctx->refs;
  S->setup_th = std::thread([S] { setup_worker(*S); });
  S->th = std::thread([S] { engine(*S); });
  *out = S;
  return PAFEM_OK;
}

int pafem_server_submit(pafem_server* S, const pafem_request* req, uint64_t* ticket) {
  clear_error();
  if (!S || !req || !ticket) {
    set_error("NULL argument");
    return PAFEM_ERR_INVALID_ARG;
  }
  if (!request_valid(*req)) {
    set_error("invalid request (sizes, order, mode, coefficient kind or tolerances)");
    return PAFEM_ERR_INVALID_ARG;
  }
  auto r = std::make_unique<Req>();
  r->spec = *req;
  const int64_t nv = (int64_t)(req->nx + 1) * (req->ny + 1) * (req->nz + 1) * 3;
  r->verts.assign(req->verts_host, req->verts_host + nv);
  r->spec.verts_host = nullptr;
  r->ir = req->mode == PAFEM_SOLVE_IR_FP32;
  r->mixed = req->mode == PAFEM_SOLVE_MIXED_FP32;
  r->ne = (int64_t)req->nx * req->ny * req->nz;
  r->ndofs = ((int64_t)req->nx * req->p + 1) * ((int64_t)req->ny * req->p + 1) *
             ((int64_t)req->nz * req->p + 1);
  r->footprint = footprint_of(*req);
  {
    std::lock_guard<std::mutex> g(S->mu);
    if (S->stopping) {
      set_error("server is shutting down");
      return PAFEM_ERR_INVALID_ARG;
    }
    r->ticket = S->next_ticket++;
    r->t_arrive = S->now();
    *ticket = r->ticket;
    S->queue.push_back(r.get());
    S->reqs[r->ticket] = std::move(r);
    ++S->n_submitted;
  }
  S->cv_work.notify_one();
  return PAFEM_OK;
}

int pafem_server_poll(pafem_server* S, uint64_t ticket, pafem_result* out) {
  clear_error();
  if (!S || !out) {
    set_error("NULL argument");
    return PAFEM_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) {
    set_error("unknown ticket");
    return PAFEM_ERR_INVALID_ARG;
  }
  const Req* r = it->second.get();
  out->status = r->status;
  out->error = r->error;
  out->ndofs = r->ndofs;
  out->footprint_bytes = r->footprint;
  out->iterations = r->iterations;
  out->outer_iterations = r->outer;
  out->rel_res = r->rel_res;
  out->t_arrive = r->t_arrive;
  out->t_admit = r->t_admit;
  out->t_done = r->t_done;
  return PAFEM_OK;
}

int pafem_server_get_solution(pafem_server* S, uint64_t ticket, double* x, int64_t n) {
  clear_error();
  if (!S || !x) {
    set_error("NULL argument");
    return PAFEM_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end() || !it->second->has_solution) {
    set_error("no solution for this ticket (unknown, not finished, failed or already taken)");
    return PAFEM_ERR_INVALID_ARG;
  }
  Req* r = it->second.get();
  if (n != r->ndofs) {
    set_error("n differs from the request's dof count");
    return PAFEM_ERR_INVALID_ARG;
  }
  std::memcpy(x, r->solution.data(), n * sizeof(double));
  std::vector<double>().swap(r->solution);
  r->has_solution = false;
  return PAFEM_OK;
}

int pafem_server_drain(pafem_server* S) {
  clear_error();
  if (!S) {
    set_error("NULL argument");
    return PAFEM_ERR_INVALID_ARG;
  }
  std::unique_lock<std::mutex> lk(S->mu);
  S->cv_done.wait(lk, [S] { return S->n_completed + S->n_failed >= S->n_submitted; });
  return PAFEM_OK;
}

int pafem_server_stats(pafem_server* S, pafem_server_counters* out) {
  clear_error();
  if (!S || !out) {
    set_error("NULL argument");
    return PAFEM_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> g(S->mu);
  out->submitted = S->n_submitted;
  out->completed = S->n_completed;
  out->failed = S->n_failed;
  out->rounds = S->n_rounds;
  out->peak_bytes = S->peak;
  out->max_active = S->max_active;
  out->dof_iterations = S->dof_iters;
  out->seconds = S->now();
  return PAFEM_OK;
}

int pafem_server_destroy(pafem_server* S) {
  if (!S) return PAFEM_OK;
  pafem_server_drain(S);
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stopping = true;
  }
  S->cv_work.notify_all();
  S->cv_setup.notify_all();
  if (S->th.joinable()) S->th.join();
  if (S->setup_th.joinable()) S->setup_th.join();
  (void)hipSetDevice(S->device);
  batch_free(S->b64);
  batch_free(S->b32);
  if (S->h_states) (void)hipHostFree(S->h_states);
  if (S->stream) (void)hipStreamDestroy(S->stream);
  if (S->stream32) (void)hipStreamDestroy(S->stream32);
  if (S->setup_stream) (void)hipStreamDestroy(S->setup_stream);
  if (S->main_done) (void)hipEventDestroy(S->main_done);
  pafem_ctx* ctx = S->ctx;
  delete S;
  pafem_ctx_destroy(ctx);  // drops the server's reference
  return PAFEM_OK;
}

}  // extern "C"
