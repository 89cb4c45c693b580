// Batched kernels of the serving engine: one launch per order p (the tuned
// element kernel of that order) and one launch per vector step cover every
// active request of a batch, so several Poisson solves share each persistent
// launch and the whole CG iteration can be captured once in a HIP graph and
// replayed while requests join and leave (the membership lives in a
// device-side table, not in kernel arguments).
//
// Results are bitwise independent of the batch composition: each element is
// computed by the same code with the same operands, E^T sums in a fixed
// per-node order, and every reduction is split into fixed per-request chunks
// summed in a fixed order.
#include "apply_impl.h"
#include "vec_impl.h"

namespace pafem {

namespace {

constexpr int kBatchGrid = 2048;  // persistent workgroups (256 CUs x 8)

// The device table stores every pointer of an entry as its byte offset from
// the table itself (nullptr stays nullptr).  Rebuilding the pointers from the
// kernel's table argument lets the compiler see global memory (scalar table
// loads, global instead of flat accesses), which a pointer read from memory
// would hide.
template <typename P>
__device__ __forceinline__ P* rebase(const void* base, P* off) {
  return off == nullptr ? nullptr : (P*)((const char*)base + (int64_t)off);
}

template <typename T>
__device__ __forceinline__ BatchEntry<T> live(const BatchEntry<T>* ents, int i) {
  BatchEntry<T> e = ents[i];
  e.a.x = rebase(ents, e.a.x);
  e.a.y = rebase(ents, e.a.y);
  e.a.yE = rebase(ents, e.a.yE);
  e.a.qd = rebase(ents, e.a.qd);
  e.a.qd16 = rebase(ents, e.a.qd16);
  e.a.E = rebase(ents, e.a.E);
  e.a.ess_mask = rebase(ents, e.a.ess_mask);
  e.a.B = rebase(ents, e.a.B);
  e.a.G = rebase(ents, e.a.G);
  e.a.skip = rebase(ents, e.a.skip);
  e.x = rebase(ents, e.x);
  e.r = rebase(ents, e.r);
  e.dir = rebase(ents, e.dir);
  e.Ad = rebase(ents, e.Ad);
  e.dinv = rebase(ents, e.dinv);
  e.st = rebase(ents, e.st);
  e.partials = rebase(ents, e.partials);
  e.x64 = rebase(ents, e.x64);
  return e;
}

// Entry owning index w of a prefix-partitioned space (entries sorted, n small).
template <typename T>
__device__ __forceinline__ int find_work(const BatchEntry<T>* e, int n, int64_t w) {
  int r = 0;
  while (r + 1 < n && w >= e[r].work_end) ++r;
  return r;
}
template <typename T>
__device__ __forceinline__ int find_chunk(const BatchEntry<T>* e, int n, int64_t c) {
  int r = 0;
  while (r + 1 < n && c >= e[r].chunk_end) ++r;
  return r;
}

// Element pass of every active entry of order P: a persistent grid over the
// work items [p_begin[P], p_end[P]) (entries are grouped by order), each item
// the tuned workgroup of the single-operator kernel of that order.
template <typename T, int P>
__global__ __launch_bounds__((apply::Cfg<P, P + 2, T, PAFEM_DIFFUSION>::THREADS),
                             (apply::Cfg<P, P + 2, T, PAFEM_DIFFUSION>::MIN_WAVES)) void k_b_apply(
    const BatchEntry<T>* __restrict__ ents, const BatchHeader* __restrict__ hdr) {
  using C = apply::Cfg<P, P + 2, T, PAFEM_DIFFUSION>;
  __shared__ T smem[C::NE * C::L];
  const int n = hdr->n;
  const int64_t end = hdr->p_end[P];
  for (int64_t w = hdr->p_begin[P] + blockIdx.x; w < end; w += gridDim.x) {
    const BatchEntry<T> E = live(ents, find_work(ents, n, w));
    if (E.st->done) continue;  // the same for the whole workgroup
    const int64_t item = w - E.work_begin;
    apply::diff_elements<P, P + 2, T, kScatterXRows, PAFEM_INDEX_LATTICE, C::NE>(
        E.a, item * C::NE, smem, threadIdx.x);
    __syncthreads();  // LDS is reused by the next work item
  }
}

template <typename T, int P>
__device__ __forceinline__ void gather_chunk(const BatchEntry<T>& E, int64_t i0) {
  for (int j = threadIdx.x; j < kBatchChunk; j += kBatchThreads) {
    const int64_t i = i0 + j;
    if (i < E.ndofs)
      vec::gather_lattice_node<T, true, P>(E.a.yE, E.a.nx, E.a.ny, E.a.nz, P, 1, 0, E.dir, E.Ad, i);
  }
}

// E^T of the chunk's nodes from the x-interleaved E-vector, then the chunk's
// partial of dir . A dir.
template <typename T>
__global__ __launch_bounds__(kBatchThreads) void k_b_gather_dot(
    const BatchEntry<T>* __restrict__ ents, const BatchHeader* __restrict__ hdr) {
  const int n = hdr->n;
  const int64_t total = hdr->total_chunks;
  for (int64_t c = blockIdx.x; c < total; c += gridDim.x) {
    const BatchEntry<T> E = live(ents, find_chunk(ents, n, c));
    if (E.st->done) continue;
    const int64_t k = c - E.chunk_begin;
    const int64_t i0 = k * kBatchChunk;
    switch (E.p) {  // the order at compile time: divisions by constants
      case 1: gather_chunk<T, 1>(E, i0); break;
      case 2: gather_chunk<T, 2>(E, i0); break;
      case 3: gather_chunk<T, 3>(E, i0); break;
      case 4: gather_chunk<T, 4>(E, i0); break;
      case 5: gather_chunk<T, 5>(E, i0); break;
      case 6: gather_chunk<T, 6>(E, i0); break;
      case 7: gather_chunk<T, 7>(E, i0); break;
      default: gather_chunk<T, 8>(E, i0); break;
    }
    __syncthreads();  // the chunk's A dir is complete (the block wrote it)
    double v[1] = {0.0}, out[1];
    for (int j = threadIdx.x; j < kBatchChunk; j += kBatchThreads) {
      const int64_t i = i0 + j;
      if (i < E.ndofs) v[0] += (double)E.dir[i] * (double)E.Ad[i];
    }
    vec::block_sum<1>(v, out);
    if (threadIdx.x == 0) E.partials[2 * k] = out[0];
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(kBatchThreads) void k_b_alpha(const BatchEntry<T>* __restrict__ ents,
                                                           const BatchHeader* __restrict__ hdr) {
  if ((int)blockIdx.x >= hdr->n) return;
  const BatchEntry<T> E = live(ents, blockIdx.x);
  CgState* st = E.st;
  if (st->done) return;
  double r[4];
  vec::final_sums(E.partials, E.nchunks, 2, r);  // column 0 = dir . A dir
  if (threadIdx.x == 0) {
    st->pAp = r[0];
    st->alpha = st->rz / r[0];
  }
}

template <typename T>
__global__ __launch_bounds__(kBatchThreads) void k_b_update(const BatchEntry<T>* __restrict__ ents,
                                                            const BatchHeader* __restrict__ hdr) {
  const int n = hdr->n;
  const int64_t total = hdr->total_chunks;
  for (int64_t c = blockIdx.x; c < total; c += gridDim.x) {
    const BatchEntry<T> E = live(ents, find_chunk(ents, n, c));
    if (E.st->done) continue;
    const T alpha = (T)E.st->alpha;
    const double alpha_x = E.st->alpha;
    const int64_t k = c - E.chunk_begin;
    double v[2] = {0.0, 0.0}, out[2];
    for (int j = threadIdx.x; j < kBatchChunk; j += kBatchThreads) {
      const int64_t i = k * kBatchChunk + j;
      if (i < E.ndofs) {
        if (E.x64 != nullptr)  // mixed CG: FP64 solution, FP64 alpha (uniform per entry)
          E.x64[i] += alpha_x * (double)E.dir[i];
        else
          E.x[i] += alpha * E.dir[i];
        const T ri = E.r[i] - alpha * E.Ad[i];
        E.r[i] = ri;
        const T zi = E.dinv[i] * ri;
        v[0] += (double)ri * (double)zi;
        v[1] += (double)ri * (double)ri;
      }
    }
    vec::block_sum<2>(v, out);
    if (threadIdx.x == 0) {
      E.partials[2 * k] = out[0];
      E.partials[2 * k + 1] = out[1];
    }
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(kBatchThreads) void k_b_beta(const BatchEntry<T>* __restrict__ ents,
                                                          const BatchHeader* __restrict__ hdr) {
  if ((int)blockIdx.x >= hdr->n) return;
  const BatchEntry<T> E = live(ents, blockIdx.x);
  CgState* st = E.st;
  if (st->done) return;
  double r[4];
  vec::final_sums(E.partials, E.nchunks, 2, r);
  if (threadIdx.x == 0) {
    st->rz_prev = st->rz;
    st->beta = r[0] / st->rz;
    st->rz = r[0];
    st->rr = r[1];
    st->iter += 1;
    if (r[1] <= st->rr_stop || st->iter >= st->maxit || !isfinite(r[1]))
      st->done = 1;
    else if (st->delta2 > 0.0 && r[1] <= st->delta2 * st->rr_ref)
      st->done = 2;  // mixed CG: pause for a residual replacement
  }
}

template <typename T>
__global__ __launch_bounds__(kBatchThreads) void k_b_dir(const BatchEntry<T>* __restrict__ ents,
                                                         const BatchHeader* __restrict__ hdr) {
  const int n = hdr->n;
  const int64_t total = hdr->total_chunks;
  for (int64_t c = blockIdx.x; c < total; c += gridDim.x) {
    const BatchEntry<T> E = live(ents, find_chunk(ents, n, c));
    if (E.st->done) continue;
    const T beta = (T)E.st->beta;
    const int64_t k = c - E.chunk_begin;
    for (int j = threadIdx.x; j < kBatchChunk; j += kBatchThreads) {
      const int64_t i = k * kBatchChunk + j;
      if (i < E.ndofs) E.dir[i] = E.dinv[i] * E.r[i] + beta * E.dir[i];
    }
  }
}

template <typename T, int P>
void launch_b_apply(const BatchEntry<T>* ents, const BatchHeader* hdr, hipStream_t s) {
  using C = apply::Cfg<P, P + 2, T, PAFEM_DIFFUSION>;
  hipLaunchKernelGGL((k_b_apply<T, P>), dim3(kBatchGrid), dim3(C::THREADS), 0, s, ents, hdr);
}

}  // namespace

template <typename T>
int batch_elems(int p) {
  switch (p) {
    case 1: return apply::Cfg<1, 3, T, PAFEM_DIFFUSION>::NE;
    case 2: return apply::Cfg<2, 4, T, PAFEM_DIFFUSION>::NE;
    case 3: return apply::Cfg<3, 5, T, PAFEM_DIFFUSION>::NE;
    case 4: return apply::Cfg<4, 6, T, PAFEM_DIFFUSION>::NE;
    case 5: return apply::Cfg<5, 7, T, PAFEM_DIFFUSION>::NE;
    case 6: return apply::Cfg<6, 8, T, PAFEM_DIFFUSION>::NE;
    case 7: return apply::Cfg<7, 9, T, PAFEM_DIFFUSION>::NE;
    case 8: return apply::Cfg<8, 10, T, PAFEM_DIFFUSION>::NE;
    default: return 1;
  }
}
template int batch_elems<double>(int);
template int batch_elems<float>(int);

template <typename T>
hipError_t launch_batch_iterations(const BatchEntry<T>* ents, const BatchHeader* hdr,
                                   int max_entries, int iters, hipStream_t s) {
  const dim3 blk(kBatchThreads);
  for (int it = 0; it < iters; ++it) {
    launch_b_apply<T, 1>(ents, hdr, s);
    launch_b_apply<T, 2>(ents, hdr, s);
    launch_b_apply<T, 3>(ents, hdr, s);
    launch_b_apply<T, 4>(ents, hdr, s);
    launch_b_apply<T, 5>(ents, hdr, s);
    launch_b_apply<T, 6>(ents, hdr, s);
    launch_b_apply<T, 7>(ents, hdr, s);
    launch_b_apply<T, 8>(ents, hdr, s);
    hipLaunchKernelGGL((k_b_gather_dot<T>), dim3(kBatchGrid), blk, 0, s, ents, hdr);
    hipLaunchKernelGGL((k_b_alpha<T>), dim3(max_entries), blk, 0, s, ents, hdr);
    hipLaunchKernelGGL((k_b_update<T>), dim3(kBatchGrid), blk, 0, s, ents, hdr);
    hipLaunchKernelGGL((k_b_beta<T>), dim3(max_entries), blk, 0, s, ents, hdr);
    hipLaunchKernelGGL((k_b_dir<T>), dim3(kBatchGrid), blk, 0, s, ents, hdr);
  }
  return hipGetLastError();
}
template hipError_t launch_batch_iterations<double>(const BatchEntry<double>*, const BatchHeader*,
                                                    int, int, hipStream_t);
template hipError_t launch_batch_iterations<float>(const BatchEntry<float>*, const BatchHeader*,
                                                   int, int, hipStream_t);

hipError_t upload_tables_batched(const double* t64, const float* t32, size_t words) {
  if (words != (size_t)apply::kTabWords) return hipErrorInvalidValue;
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(apply::c_tab64), t64, words * sizeof(double));
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(apply::c_tab32), t32, words * sizeof(float));
  return e;
}

}  // namespace pafem
