// pafem_op_apply_noalloc: the operator apply with its E-vector workspace in a
// fixed device array of the library instead of memory allocated on first use,
// for callers that cannot allocate (code under HIP graph capture, serving
// loops or harnesses that forbid hipMalloc).
//
// The array is a file-scope __device__ object: every GPU the library runs on
// holds its own copy, at its own address, from code-object load until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host that name is only a stand-in for the symbol); the device address is
// looked up once per device, with that device current, when a context is
// created, and kept here.
#include <mutex>

#include "internal.h"

namespace pafem {

namespace {

constexpr int kMaxDevices = 64;
constexpr size_t kScratchBytes = PAFEM_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

}  // namespace

// Look up the device address of `scratch` on `device` (which must be current).
int noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("device index beyond the allocation-free workspace table");
    return PAFEM_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device] != nullptr) return PAFEM_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr) {
    set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    return PAFEM_ERR_HIP;
  }
  g_scratch[device] = ptr;
  return PAFEM_OK;
}

}  // namespace pafem

using namespace pafem;

extern "C" int pafem_op_apply_noalloc(pafem_op* op, int prec, const void* x, void* y, int flags,
                                      void* stream) {
  clear_error();
  if (!op || !x || !y) {
    set_error("NULL argument");
    return PAFEM_ERR_INVALID_ARG;
  }
  if (x == y) {
    set_error("x and y must not alias");
    return PAFEM_ERR_INVALID_ARG;
  }
  if ((flags & ~(PAFEM_APPLY_CONSTRAINED | PAFEM_APPLY_ACCUMULATE)) != 0) {
    set_error("unknown apply flags");
    return PAFEM_ERR_INVALID_ARG;
  }
  const Ctx* ctx = op->space->mesh->ctx;
  if (ctx->host_only) {
    set_error("operation needs a GPU context (created with device >= 0)");
    return PAFEM_ERR_UNSUPPORTED;
  }
  void* work = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (ctx->device >= 0 && ctx->device < kMaxDevices) work = g_scratch[ctx->device];
  }
  if (work == nullptr) {
    set_error("allocation-free workspace not set up on this device");
    return PAFEM_ERR_HIP;
  }
  PAFEM_TRY_HIP(hipSetDevice(ctx->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool f64 = prec == PAFEM_FP64;
  if (!f64 && prec != PAFEM_FP32 && prec != PAFEM_BF16) {
    set_error("prec must be PAFEM_FP64, PAFEM_FP32 or PAFEM_BF16");
    return PAFEM_ERR_INVALID_ARG;
  }
  if ((f64 && !op->have64) || (prec == PAFEM_FP32 && !op->have32) ||
      (prec == PAFEM_BF16 && !op->have16)) {
    set_error("quadrature data of that precision not assembled");
    return PAFEM_ERR_INVALID_ARG;
  }
  const int64_t need = f64 ? apply_work_bytes<double>(op) : apply_work_bytes<float>(op);
  if (need > (int64_t)kScratchBytes) {
    set_error("allocation-free apply needs " + std::to_string(need) +
              " bytes of workspace; the fixed workspace holds " + std::to_string(kScratchBytes));
    return PAFEM_ERR_INVALID_ARG;
  }
  if (f64)
    return apply_impl<double>(op, (const double*)x, (double*)y, flags, nullptr, s, 0, work);
  return apply_impl<float>(op, (const float*)x, (float*)y, flags, nullptr, s, prec, work);
}
