// Per-operator launches of the fused partial-assembly element kernels
// (bodies in apply_impl.h) and their dispatch over p, precision, output
// (E-vector or atomic E^T) and restriction source.
#include <type_traits>

#include "apply_impl.h"

namespace pafem {

namespace {

using apply::Cfg;
using apply::xcd_block;

template <int P, int Q, typename T, int SCATTER, int IDX, bool QD16, bool MF = false>
__global__ __launch_bounds__((Cfg<P, Q, T, PAFEM_DIFFUSION>::THREADS),
                             (SCATTER == kScatterXRowsDot
                                  ? Cfg<P, Q, T, PAFEM_DIFFUSION>::MIN_WAVES_DOT
                                  : Cfg<P, Q, T, PAFEM_DIFFUSION>::MIN_WAVES)) void k_apply_diff(
    ApplyArgs<T> a) {
  using C = Cfg<P, Q, T, PAFEM_DIFFUSION>;
  __shared__ T smem[C::NE * C::L];
  if (a.skip != nullptr && *a.skip) return;
  const int64_t nb = (a.ne + C::NE - 1) / C::NE;
  const int64_t e0 = xcd_block(blockIdx.x, nb) * C::NE;
  apply::diff_elements<P, Q, T, SCATTER, IDX, C::NE, QD16, MF>(a, e0, smem, threadIdx.x);
}

template <int P, int Q, typename T, int SCATTER, int IDX, bool QD16, bool MF = false>
__global__ __launch_bounds__((Cfg<P, Q, T, PAFEM_MASS>::THREADS)) void k_apply_mass(
    ApplyArgs<T> a) {
  using C = Cfg<P, Q, T, PAFEM_MASS>;
  __shared__ T smem[C::NE * C::L];
  if (a.skip != nullptr && *a.skip) return;
  const int64_t nb = (a.ne + C::NE - 1) / C::NE;
  const int64_t e0 = xcd_block(blockIdx.x, nb) * C::NE;
  apply::mass_elements<P, Q, T, SCATTER, IDX, C::NE, QD16, MF>(a, e0, smem, threadIdx.x);
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
template <int P, typename T, int KIND, int SCATTER, int IDX>
hipError_t launch_one(const ApplyArgs<T>& a, hipStream_t s) {
  constexpr int Q = P + 2;
  using C = Cfg<P, Q, T, KIND>;
  const int64_t nb = (a.ne + C::NE - 1) / C::NE;
  // fully matrix-free form: lattice numbering, E-vector outputs only
  if constexpr (IDX == PAFEM_INDEX_LATTICE && SCATTER != PAFEM_SCATTER_ATOMIC) {
    if (a.mf) {
      if (KIND == PAFEM_DIFFUSION)
        hipLaunchKernelGGL((k_apply_diff<P, Q, T, SCATTER, IDX, false, true>), dim3(nb), dim3(C::THREADS), 0, s, a);
      else
        hipLaunchKernelGGL((k_apply_mass<P, Q, T, SCATTER, IDX, false, true>), dim3(nb), dim3(C::THREADS), 0, s, a);
      return hipGetLastError();
    }
  }
  // bfloat16 quadrature data is a compile-time variant (FP32 arithmetic only),
  // so the FP64 and FP32 kernels carry no branch between their load streams
  if constexpr (std::is_same<T, float>::value) {
    if (a.qd16 != nullptr) {
      if (KIND == PAFEM_DIFFUSION)
        hipLaunchKernelGGL((k_apply_diff<P, Q, T, SCATTER, IDX, true>), dim3(nb), dim3(C::THREADS), 0, s, a);
      else
        hipLaunchKernelGGL((k_apply_mass<P, Q, T, SCATTER, IDX, true>), dim3(nb), dim3(C::THREADS), 0, s, a);
      return hipGetLastError();
    }
  }
  if (KIND == PAFEM_DIFFUSION)
    hipLaunchKernelGGL((k_apply_diff<P, Q, T, SCATTER, IDX, false>), dim3(nb), dim3(C::THREADS), 0, s, a);
  else
    hipLaunchKernelGGL((k_apply_mass<P, Q, T, SCATTER, IDX, false>), dim3(nb), dim3(C::THREADS), 0, s, a);
  return hipGetLastError();
}

template <int P, typename T, int KIND>
hipError_t apply_kind(int scatter, int idx, const ApplyArgs<T>& a, hipStream_t s) {
  constexpr int ATO = PAFEM_SCATTER_ATOMIC, EVC = kScatterEvector, XR = kScatterXRows;
  constexpr int XRD = kScatterXRowsDot;
  constexpr int MAP = PAFEM_INDEX_MAP, LAT = PAFEM_INDEX_LATTICE;
  if (scatter == XR) return launch_one<P, T, KIND, XR, LAT>(a, s);
  if (scatter == XRD) return launch_one<P, T, KIND, XRD, LAT>(a, s);
  if (scatter == EVC)
    return idx == MAP ? launch_one<P, T, KIND, EVC, MAP>(a, s) : launch_one<P, T, KIND, EVC, LAT>(a, s);
  return idx == MAP ? launch_one<P, T, KIND, ATO, MAP>(a, s) : launch_one<P, T, KIND, ATO, LAT>(a, s);
}

template <int P, typename T>
hipError_t apply_p(int kind, int scatter, int idx, const ApplyArgs<T>& a, hipStream_t s) {
  if (a.ne == 0) return hipSuccess;
  if (kind == PAFEM_DIFFUSION) return apply_kind<P, T, PAFEM_DIFFUSION>(scatter, idx, a, s);
  return apply_kind<P, T, PAFEM_MASS>(scatter, idx, a, s);
}

}  // namespace

template <typename T>
hipError_t launch_apply(int kind, int p, int q, int scatter_mode, int index_mode,
                        const ApplyArgs<T>& a, hipStream_t s) {
  if (q != p + 2) {
    // a non-default quadrature size: the run-time-sized kernel (its lattice
    // numbering equals the stored maps, so either E^T follows it)
    if (index_mode == PAFEM_INDEX_MAP && scatter_mode != PAFEM_SCATTER_ATOMIC &&
        scatter_mode != kScatterEvector)
      return hipErrorInvalidValue;
    return launch_apply_generic<T>(kind, p, q, scatter_mode, a, s);
  }
  const bool xrows = scatter_mode == kScatterXRows || scatter_mode == kScatterXRowsDot;
  if (scatter_mode != PAFEM_SCATTER_ATOMIC && scatter_mode != kScatterEvector && !xrows)
    return hipErrorInvalidValue;
  if (xrows && index_mode != PAFEM_INDEX_LATTICE) return hipErrorInvalidValue;
  if (scatter_mode == kScatterXRowsDot && a.dot_part == nullptr) return hipErrorInvalidValue;
  // the stored maps must be on the device before a kernel may read them
  if (index_mode == PAFEM_INDEX_MAP && (a.E == nullptr || a.ess_mask == nullptr))
    return hipErrorInvalidValue;
  if (a.mf) {
    // recomputed geometry: lattice numbering and an E-vector output only
    if (index_mode != PAFEM_INDEX_LATTICE || scatter_mode == PAFEM_SCATTER_ATOMIC ||
        a.verts == nullptr || a.qpts == nullptr || a.qwts == nullptr || a.qd16 != nullptr)
      return hipErrorInvalidValue;
  } else if (a.qd == nullptr && a.qd16 == nullptr) {
    return hipErrorInvalidValue;
  }
  if (a.x == nullptr || a.B == nullptr || a.G == nullptr) return hipErrorInvalidValue;
  if (scatter_mode != PAFEM_SCATTER_ATOMIC && a.yE == nullptr) return hipErrorInvalidValue;
  if (scatter_mode == PAFEM_SCATTER_ATOMIC && a.y == nullptr) return hipErrorInvalidValue;
  switch (p) {
    case 1: return apply_p<1, T>(kind, scatter_mode, index_mode, a, s);
    case 2: return apply_p<2, T>(kind, scatter_mode, index_mode, a, s);
    case 3: return apply_p<3, T>(kind, scatter_mode, index_mode, a, s);
    case 4: return apply_p<4, T>(kind, scatter_mode, index_mode, a, s);
    case 5: return apply_p<5, T>(kind, scatter_mode, index_mode, a, s);
    case 6: return apply_p<6, T>(kind, scatter_mode, index_mode, a, s);
    case 7: return apply_p<7, T>(kind, scatter_mode, index_mode, a, s);
    case 8: return apply_p<8, T>(kind, scatter_mode, index_mode, a, s);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_apply<double>(int, int, int, int, int, const ApplyArgs<double>&,
                                         hipStream_t);
template hipError_t launch_apply<float>(int, int, int, int, int, const ApplyArgs<float>&,
                                        hipStream_t);

hipError_t upload_tables_apply(const double* t64, const float* t32, size_t words) {
  if (words != (size_t)apply::kTabWords) return hipErrorInvalidValue;
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(apply::c_tab64), t64, words * sizeof(double));
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(apply::c_tab32), t32, words * sizeof(float));
  return e;
}

namespace {
template <typename T, int KIND>
int64_t blocks_p(int p, int64_t ne) {
  switch (p) {
    case 1: return (ne + Cfg<1, 3, T, KIND>::NE - 1) / Cfg<1, 3, T, KIND>::NE;
    case 2: return (ne + Cfg<2, 4, T, KIND>::NE - 1) / Cfg<2, 4, T, KIND>::NE;
    case 3: return (ne + Cfg<3, 5, T, KIND>::NE - 1) / Cfg<3, 5, T, KIND>::NE;
    case 4: return (ne + Cfg<4, 6, T, KIND>::NE - 1) / Cfg<4, 6, T, KIND>::NE;
    case 5: return (ne + Cfg<5, 7, T, KIND>::NE - 1) / Cfg<5, 7, T, KIND>::NE;
    case 6: return (ne + Cfg<6, 8, T, KIND>::NE - 1) / Cfg<6, 8, T, KIND>::NE;
    case 7: return (ne + Cfg<7, 9, T, KIND>::NE - 1) / Cfg<7, 9, T, KIND>::NE;
    case 8: return (ne + Cfg<8, 10, T, KIND>::NE - 1) / Cfg<8, 10, T, KIND>::NE;
    default: return 0;
  }
}
}  // namespace

int64_t element_blocks(int kind, int p, int64_t ne, bool f32) {
  if (kind == PAFEM_DIFFUSION)
    return f32 ? blocks_p<float, PAFEM_DIFFUSION>(p, ne) : blocks_p<double, PAFEM_DIFFUSION>(p, ne);
  return f32 ? blocks_p<float, PAFEM_MASS>(p, ne) : blocks_p<double, PAFEM_MASS>(p, ne);
}

}  // namespace pafem
