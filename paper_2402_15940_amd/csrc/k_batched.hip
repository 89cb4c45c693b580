// Batched kernels of the serving engine: one launch covers every active
// request of a batch, whatever its order p, so several Poisson solves share
// each persistent launch and the whole CG iteration can be captured once in a
// HIP graph and replayed while requests join and leave (the membership lives
// in a device-side table, not in kernel arguments).
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

template <typename T>
constexpr int serve_lds_words() {
  using apply::Cfg;
  constexpr int l[8] = {
      batch_elems(3) * Cfg<1, 3, T, PAFEM_DIFFUSION>::L, batch_elems(4) * Cfg<2, 4, T, PAFEM_DIFFUSION>::L,
      batch_elems(5) * Cfg<3, 5, T, PAFEM_DIFFUSION>::L, batch_elems(6) * Cfg<4, 6, T, PAFEM_DIFFUSION>::L,
      batch_elems(7) * Cfg<5, 7, T, PAFEM_DIFFUSION>::L, batch_elems(8) * Cfg<6, 8, T, PAFEM_DIFFUSION>::L,
      batch_elems(9) * Cfg<7, 9, T, PAFEM_DIFFUSION>::L, batch_elems(10) * Cfg<8, 10, T, PAFEM_DIFFUSION>::L};
  int m = 0;
  for (int i = 0; i < 8; ++i) m = l[i] > m ? l[i] : m;
  return m;
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

template <typename T>
__global__ __launch_bounds__(kBatchThreads, (sizeof(T) == 4 ? 2 : 1)) void k_b_apply(const BatchEntry<T>* __restrict__ ents,
                                                           const BatchHeader* __restrict__ hdr) {
  __shared__ T smem[serve_lds_words<T>()];
  const int n = hdr->n;
  const int64_t total = hdr->total_work;
  constexpr int DET = kScatterXRows, LAT = PAFEM_INDEX_LATTICE;
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const BatchEntry<T>& E = ents[find_work(ents, n, w)];
    if (E.st->done) continue;  // the same for the whole workgroup
    const int64_t item = w - E.work_begin;
    const int tid = threadIdx.x;
    switch (E.p) {
      case 1: apply::diff_elements<1, 3, T, DET, LAT, batch_elems(3)>(E.a, item * batch_elems(3), smem, tid); break;
      case 2: apply::diff_elements<2, 4, T, DET, LAT, batch_elems(4)>(E.a, item * batch_elems(4), smem, tid); break;
      case 3: apply::diff_elements<3, 5, T, DET, LAT, batch_elems(5)>(E.a, item * batch_elems(5), smem, tid); break;
      case 4: apply::diff_elements<4, 6, T, DET, LAT, batch_elems(6)>(E.a, item * batch_elems(6), smem, tid); break;
      case 5: apply::diff_elements<5, 7, T, DET, LAT, batch_elems(7)>(E.a, item * batch_elems(7), smem, tid); break;
      case 6: apply::diff_elements<6, 8, T, DET, LAT, batch_elems(8)>(E.a, item * batch_elems(8), smem, tid); break;
      case 7: apply::diff_elements<7, 9, T, DET, LAT, batch_elems(9)>(E.a, item * batch_elems(9), smem, tid); break;
      default: apply::diff_elements<8, 10, T, DET, LAT, batch_elems(10)>(E.a, item * batch_elems(10), smem, tid); break;
    }
    __syncthreads();  // LDS is reused by the next work item
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
    const BatchEntry<T>& E = ents[find_chunk(ents, n, c)];
    if (E.st->done) continue;
    const int64_t k = c - E.chunk_begin;
    const int64_t i0 = k * kBatchChunk;
    for (int j = threadIdx.x; j < kBatchChunk; j += kBatchThreads) {
      const int64_t i = i0 + j;
      if (i < E.ndofs)
        vec::gather_lattice_node<T, true>(E.a.yE, E.a.nx, E.a.ny, E.a.nz, E.p, 1, 0, E.dir, E.Ad, i);
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
  const BatchEntry<T>& E = ents[blockIdx.x];
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
    const BatchEntry<T>& E = ents[find_chunk(ents, n, c)];
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
  const BatchEntry<T>& E = ents[blockIdx.x];
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
    if (r[1] <= st->rr_stop || st->iter >= st->maxit)
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
    const BatchEntry<T>& E = ents[find_chunk(ents, n, c)];
    if (E.st->done) continue;
    const T beta = (T)E.st->beta;
    const int64_t k = c - E.chunk_begin;
    for (int j = threadIdx.x; j < kBatchChunk; j += kBatchThreads) {
      const int64_t i = k * kBatchChunk + j;
      if (i < E.ndofs) E.dir[i] = E.dinv[i] * E.r[i] + beta * E.dir[i];
    }
  }
}

}  // namespace

template <typename T>
hipError_t launch_batch_iterations(const BatchEntry<T>* ents, const BatchHeader* hdr,
                                   int max_entries, int iters, hipStream_t s) {
  const dim3 blk(kBatchThreads);
  for (int it = 0; it < iters; ++it) {
    hipLaunchKernelGGL((k_b_apply<T>), dim3(kBatchGrid), blk, 0, s, ents, hdr);
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

}  // namespace pafem
