// Whole Jacobi-PCG iterations in one persistent, cooperatively launched
// kernel (the fully fused form of the paper's section on kernel fusion, with
// grid-wide synchronization in place of separate launches).
//
// One launch runs up to `iters` iterations; each iteration is two phases
// separated by grid barriers.  The direction update is deferred: the vector p
// in memory holds the previous direction, and the current one,
// p_k = dinv r_k + beta p_(k-1), is formed wherever it is read (the same
// expression, so the same bits, in both phases):
//   1. the element pass of A p_k (the same device code as the separate
//      kernel, with the direction formed at its gather: x-interleaved E-vector
//      and per-element-group partials of p . A p), each workgroup walking its
//      share of the element groups in a fixed order (one contiguous range per
//      XCD); its partials are summed per workgroup in that order;
//   2. every workgroup sums the G workgroup partials in the same fixed order
//      (so every workgroup holds the same alpha), then the ordered E^T sum of
//      its node chunks with p = p_k stored, x += alpha p_k, r -= alpha A p_k
//      and the partials of (r . z, r . r); after the barrier every workgroup
//      forms the same (r . z, r . r), beta and the stopping test.
// The CG scalars stay in registers of every workgroup; workgroup 0 writes them
// (beta included, for the next launch) to the state at the end.  The grid is at most what the device can hold at
// once (cooperative launch refuses more), and every barrier wait is bounded:
// a wait that exceeds the spin limit sets the error flag and its workgroup
// leaves, so the others' waits end the same way and the launch always drains.
#include "apply_impl.h"
#include "vec_impl.h"

namespace pafem {

namespace {

using apply::Cfg;
using vec::kXRowsNodes;
using vec::XRowsGeom;
using vec::XRowsLoads;
using vec::xrows_geom;
using vec::xrows_load;
using vec::xrows_sum;

// Barrier words, each on its own 128-byte line: one arrival counter and one
// generation per group of workgroups (workgroup b in group b mod ngroups,
// ngroups = min(G, 8), so with the round-robin dealing a group is one XCD's
// workgroups), and a root counter and generation over the groups.
constexpr int kLine = 32;  // unsigned words per 128-byte line
struct PcgBarrier {
  unsigned count[8 * kLine];
  unsigned gen[8 * kLine];
  unsigned root_count[kLine];
  unsigned root_gen[kLine];
};
static_assert(sizeof(PcgBarrier) == kPersistentBarrierBytes, "barrier words");

template <typename T>
struct PcgArgs {
  ApplyArgs<T> a;      // x = direction p, yE = x-interleaved E-vector, dot_part = group partials
  XRowsGeom g;
  T* xs;               // solution
  T* r;
  const T* dinv;
  double* bpart;       // [G]: per-workgroup sums of the group partials of p . A p
  double* npart;       // [G][2]: per-workgroup (r . z, r . r)
  CgState* st;
  PcgBarrier* bar;
  int* err;
  long long spin_limit;
  int iters;
  int64_t groups;
};

// Bounded wait until *w differs from `seen`; false (and the error flag set)
// when the spin limit is reached.
__device__ __forceinline__ bool wait_change(const unsigned* w, unsigned seen, long long spin_limit,
                                            int* err) {
  long long k = 0;
  while (__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == seen) {
    if (++k > spin_limit) {
      atomicOr(err, 1);
      return false;
    }
    __builtin_amdgcn_s_sleep(8);
  }
  return true;
}

// Grid-wide barrier in two levels: the last workgroup to arrive in its group
// arrives at the root; the last group to arrive advances the root generation;
// each group's last arriver, once it sees that, advances its group's
// generation, which the rest of the group waits on.  So at most eight
// workgroups poll the root and the others spread over eight words.  Release
// fences before each arrival and acquire fences after each observed
// generation carry every workgroup's writes to every other.  Every wait is
// bounded; a workgroup whose wait runs out sets the error flag and reports
// false, and those waiting on it run out the same way.
__device__ __forceinline__ bool grid_barrier(PcgBarrier* bar, unsigned nblocks,
                                             long long spin_limit, int* err) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned ng = nblocks < 8u ? nblocks : 8u;
    const unsigned grp = blockIdx.x % ng;
    const unsigned members = (nblocks - grp + ng - 1) / ng;
    unsigned* cnt = &bar->count[grp * kLine];
    unsigned* gen = &bar->gen[grp * kLine];
    const unsigned g0 = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    bool good = true;
    if (atomicAdd(cnt, 1u) == members - 1) {
      // last of the group: the others' writes, then arrival at the root
      atomicExch(cnt, 0u);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
      const unsigned r0 =
          __hip_atomic_load(bar->root_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (atomicAdd(bar->root_count, 1u) == ng - 1) {
        atomicExch(bar->root_count, 0u);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        atomicAdd(bar->root_gen, 1u);
      } else {
        good = wait_change(bar->root_gen, r0, spin_limit, err);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
      }
      atomicAdd(gen, 1u);  // release the group (also when the wait ran out)
    } else {
      good = wait_change(gen, g0, spin_limit, err);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    ok = good ? 1 : 0;
  }
  __syncthreads();
  return ok != 0;
}

#ifndef PAFEM_PCG_PHASE2_NODES
#define PAFEM_PCG_PHASE2_NODES 2
#endif
constexpr int kPhase2Nodes = PAFEM_PCG_PHASE2_NODES;

// The items [0, total) a workgroup walks.  Workgroups are dealt to the XCDs
// round-robin; each XCD takes one contiguous range of items, walked by its
// workgroups in turn (neighbouring element groups share face dofs in that
// XCD's L2).  With fewer workgroups than XCDs, a plain strided walk.
struct Walk {
  int64_t first, end, stride;
};
__device__ __forceinline__ Walk xcd_walk(int64_t b, int64_t G, int64_t total) {
  using apply::kXcds;
  if (G < kXcds) return {b, total, G};
  const int64_t x = b % kXcds, l = b / kXcds;
  const int64_t gx = (G - x + kXcds - 1) / kXcds;  // workgroups on XCD x (>= 1)
  const int64_t q = total / kXcds, r = total % kXcds;
  const int64_t start = x * q + (x < r ? x : r);
  return {start + l, start + q + (x < r ? 1 : 0), gx};
}

// Sum over the workgroup of NV values per thread, returned to every thread.
template <int NV, int THREADS>
__device__ __forceinline__ void sum_all(double (&v)[NV]) {
  constexpr int NW = THREADS / 64;
  __shared__ double sh[NV][NW];
  const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double w = vec::wave_sum(v[k]);
    if (lane == 0) sh[k][wid] = w;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double t = 0.0;
    for (int i = 0; i < NW; ++i) t += sh[k][i];
    v[k] = t;
  }
  __syncthreads();
}

// (2 waves per SIMD: the whole iteration in one kernel would otherwise take
// more registers than leave room for a second wave)
template <int P, typename T, int KIND>
__global__ __launch_bounds__((Cfg<P, P + 2, T, KIND>::THREADS), 2) void k_pcg_persistent(
    PcgArgs<T> pa) {
  using C = Cfg<P, P + 2, T, KIND>;
  // phase 2 takes R nodes per thread at a time, all their loads issued before
  // the first use (few waves per SIMD fit next to the element pass, so each
  // keeps several loads in flight)
  constexpr int NT = C::THREADS, R = kPhase2Nodes;
  __shared__ T smem[C::NE * C::L];
  const unsigned G = gridDim.x;
  const int tid = threadIdx.x;
  const XRowsGeom& g = pa.g;
  double rz = pa.st->rz, rr = pa.st->rr, pAp = 0.0, alpha = 0.0, beta = pa.st->beta;
  const double rr_stop = pa.st->rr_stop;
  int iter = pa.st->iter, done = pa.st->done;
  const int maxit = pa.st->maxit;
  T* p = const_cast<T*>(pa.a.x);
  const Walk wg = xcd_walk(blockIdx.x, G, pa.groups);
  const Walk wn = xcd_walk(blockIdx.x, G, (g.n + NT * R - 1) / (NT * R));
  for (int it = 0; it < pa.iters && !done; ++it) {
    const T beta_t = (T)beta;
    // ---- 1: element pass of A p_k, p_k = dinv r + beta p formed at the gather ----
    double mine = 0.0;  // this workgroup's groups, in walking order (thread 0)
    for (int64_t grp = wg.first; grp < wg.end; grp += wg.stride) {
      if constexpr (KIND == PAFEM_DIFFUSION)
        apply::diff_elements<P, P + 2, T, kScatterXRowsDot, PAFEM_INDEX_LATTICE, C::NE, false,
                             false, true>(pa.a, grp * C::NE, smem, tid, beta_t);
      else
        apply::mass_elements<P, P + 2, T, kScatterXRowsDot, PAFEM_INDEX_LATTICE, C::NE, false,
                             false, true>(pa.a, grp * C::NE, smem, tid, beta_t);
      if (tid == 0) mine += pa.a.dot_part[grp];
      __syncthreads();  // the LDS regions are reused by the next group
    }
    if (tid == 0) pa.bpart[blockIdx.x] = mine;
    if (!grid_barrier(pa.bar, G, pa.spin_limit, pa.err)) break;
    // ---- 2: alpha, E^T sum, p, x and r updates ------------------------------------
    {
      double v[1] = {0.0};
      for (unsigned i = tid; i < G; i += NT) v[0] += pa.bpart[i];
      sum_all<1, NT>(v);
      pAp = v[0];
    }
    alpha = rz / pAp;
    double v2[2] = {0.0, 0.0};
    const T alpha_t = (T)alpha;
    for (int64_t c = wn.first; c < wn.end; c += wn.stride) {
      const int64_t base = c * (NT * R) + tid;
      XRowsLoads<T> L[R];
      T dv[R], rv[R], pv[R], xv[R];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int64_t iq = base + q * NT;
        xrows_load<T, P>(pa.a.yE, g, (int)(iq < g.n ? iq : g.n - 1), L[q]);
      }
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int64_t iq = base + q * NT;
        const int64_t ic = iq < g.n ? iq : g.n - 1;
        dv[q] = pa.dinv[ic];
        rv[q] = pa.r[ic];
        pv[q] = p[ic];
        xv[q] = pa.xs[ic];
      }
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int64_t i = base + q * NT;
        if (i >= g.n) break;
        const T pi = dv[q] * rv[q] + beta_t * pv[q];
        p[i] = pi;
        const T acc = L[q].ess ? pi : xrows_sum(L[q]);
        pa.xs[i] = xv[q] + alpha_t * pi;
        const T ri = rv[q] - alpha_t * acc;
        pa.r[i] = ri;
        const T zi = dv[q] * ri;
        v2[0] += (double)ri * (double)zi;
        v2[1] += (double)ri * (double)ri;
      }
    }
    sum_all<2, NT>(v2);
    if (tid == 0) {
      pa.npart[2 * blockIdx.x] = v2[0];
      pa.npart[2 * blockIdx.x + 1] = v2[1];
    }
    if (!grid_barrier(pa.bar, G, pa.spin_limit, pa.err)) break;
    {
      double v[2] = {0.0, 0.0};
      for (unsigned i = tid; i < G; i += NT) {
        v[0] += pa.npart[2 * i];
        v[1] += pa.npart[2 * i + 1];
      }
      sum_all<2, NT>(v);
      beta = v[0] / rz;
      rz = v[0];
      rr = v[1];
    }
    iter += 1;
    done = (rr <= rr_stop || iter >= maxit || !isfinite(rr)) ? 1 : 0;
  }
  if (blockIdx.x == 0 && tid == 0) {
    pa.st->rz = rz;
    pa.st->rr = rr;
    pa.st->pAp = pAp;
    pa.st->alpha = alpha;
    pa.st->beta = beta;
    pa.st->iter = iter;
    pa.st->done = done;
  }
}

template <int P, typename T, int KIND>
hipError_t launch_p(const PcgArgs<T>& pa0, int max_blocks, int* grid_out, hipStream_t s) {
  using C = Cfg<P, P + 2, T, KIND>;
  auto kern = k_pcg_persistent<P, T, KIND>;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, C::THREADS, 0);
  if (e != hipSuccess) return e;
  int dev = 0, cus = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  int64_t grid = (int64_t)per_cu * cus;
  if (grid > pa0.groups) grid = pa0.groups;
  if (grid > max_blocks) grid = max_blocks;
  if (grid < 1) return hipErrorInvalidConfiguration;
  *grid_out = (int)grid;
  PcgArgs<T> pa = pa0;
  void* args[] = {&pa};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3((unsigned)grid),
                                    dim3(C::THREADS), args, 0, s);
}

template <typename T, int KIND>
hipError_t launch_kind(int p, const PcgArgs<T>& pa, int max_blocks, int* grid, hipStream_t s) {
  switch (p) {
    case 1: return launch_p<1, T, KIND>(pa, max_blocks, grid, s);
    case 2: return launch_p<2, T, KIND>(pa, max_blocks, grid, s);
    case 3: return launch_p<3, T, KIND>(pa, max_blocks, grid, s);
    case 4: return launch_p<4, T, KIND>(pa, max_blocks, grid, s);
    case 5: return launch_p<5, T, KIND>(pa, max_blocks, grid, s);
    case 6: return launch_p<6, T, KIND>(pa, max_blocks, grid, s);
    case 7: return launch_p<7, T, KIND>(pa, max_blocks, grid, s);
    case 8: return launch_p<8, T, KIND>(pa, max_blocks, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// Up to `iters` FP64 Jacobi-PCG iterations in one cooperative launch.  a is
// the element-pass argument block (x = direction, yE = E-vector, dot_part =
// one partial per element group); bpart and npart hold at least max_blocks
// and 2 max_blocks doubles; bar holds kPersistentBarrierBytes whose arrival
// counters are zero on entry and on return.
hipError_t launch_pcg_persistent(int kind, int p, const ApplyArgs<double>& a, int64_t groups,
                                 double* xs, double* r, const double* dinv, double* bpart,
                                 double* npart, CgState* st, void* bar, int* err,
                                 long long spin_limit, int iters, int max_blocks, int* grid,
                                 hipStream_t s) {
  if (a.x == nullptr || a.yE == nullptr || a.dot_part == nullptr || a.qd == nullptr ||
      xs == nullptr || r == nullptr || dinv == nullptr || bpart == nullptr || npart == nullptr ||
      st == nullptr || bar == nullptr || err == nullptr || groups < 1 || iters < 1)
    return hipErrorInvalidValue;
  const int64_t n = ((int64_t)a.nx * p + 1) * ((int64_t)a.ny * p + 1) * ((int64_t)a.nz * p + 1);
  if (n > 0x7fffffff) return hipErrorInvalidValue;
  PcgArgs<double> pa;
  pa.a = a;
  pa.a.dir_r = r;
  pa.a.dir_dinv = dinv;
  pa.g = xrows_geom(a.nx, a.ny, a.nz, p);
  pa.xs = xs;
  pa.r = r;
  pa.dinv = dinv;
  pa.bpart = bpart;
  pa.npart = npart;
  pa.st = st;
  pa.bar = static_cast<PcgBarrier*>(bar);
  pa.err = err;
  pa.spin_limit = spin_limit;
  pa.iters = iters;
  pa.groups = groups;
  if (kind == PAFEM_DIFFUSION) return launch_kind<double, PAFEM_DIFFUSION>(p, pa, max_blocks, grid, s);
  return launch_kind<double, PAFEM_MASS>(p, pa, max_blocks, grid, s);
}

hipError_t upload_tables_persistent(const double* t64, const float* t32, size_t words) {
  if (words != (size_t)apply::kTabWords) return hipErrorInvalidValue;
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(apply::c_tab64), t64, words * sizeof(double));
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(apply::c_tab32), t32, words * sizeof(float));
  return e;
}

}  // namespace pafem
