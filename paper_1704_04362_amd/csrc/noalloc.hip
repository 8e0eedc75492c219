// Slice picks for callers that cannot allocate device memory: the sampling
// call of tp_tsample with its scratch (quantised weights, prefix sums,
// selection keys, the float64 weight vectors and the slice-norm partials)
// taken from a fixed array in device memory instead of a caller workspace.
//
// The array `scratch` is a file-scope __device__ variable: every GPU the
// library runs on holds its own copy at its own address for the life of the
// process. On the host its name is only a stand-in for that symbol, so its
// device address is looked up once per device (hipGetSymbolAddress, with
// that device current) and kept; kernels receive that address. Calls on one
// GPU share the array: two calls that overlap on a GPU (different streams,
// or different host threads without ordering) race on it.
#include <mutex>

#include "common.hpp"

namespace tp {
namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of the array, looked up on first use.
int scratch_ptr(void** out) {
  int dev = 0;
  TP_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(TP_EUNSUPPORTED, "device ordinal above 63");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    TP_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(TP_EHIP, "hipGetSymbolAddress returned a null scratch address");
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return TP_OK;
}

}  // namespace
}  // namespace tp

using namespace tp;

extern "C" {

size_t tp_tsample_noalloc_max_bytes(void) { return kScratchBytes; }

int tp_tsample_noalloc(int kind, const tp_tensor* A, const tp_tensor* B, const double* w, int64_t n, int64_t c,
                       int mode, uint64_t seed, uint64_t stream_id, tp_sample* out, void* stream) {
  // every argument is validated exactly as tp_tsample does it: without a
  // workspace that call checks everything, enqueues nothing and reports
  // only the missing workspace when the arguments are good
  const int pre = tp_tsample(kind, A, B, w, n, c, mode, seed, stream_id, out, nullptr, 0, stream);
  if (pre != TP_EWORKSPACE) return pre;
  const size_t need = tsample_ws_full(kind, A, n);
  if (need > kScratchBytes)
    return fail(TP_EUNSUPPORTED, "tp_tsample_noalloc: these sizes need " + std::to_string(need) +
                                     " bytes of scratch, above its fixed " + std::to_string(kScratchBytes));
  void* ptr = nullptr;
  if (int rc = scratch_ptr(&ptr)) return rc;
  return tp_tsample(kind, A, B, w, n, c, mode, seed, stream_id, out, ptr, kScratchBytes, stream);
}

}  // extern "C"
