// The sketch S A (Section 2) for callers that cannot allocate device memory
// or pass a workspace: the bucket plan lives in a fixed array of this library
// on each device.
#include <mutex>

#include "kernels.hpp"

namespace skls {
namespace {

constexpr size_t kScratchBytes = SKLS_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// The plan of skls_sketch_noalloc.  Host code never uses this name as an
// address: it resolves the device address once per device (scratch_address).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Address of `scratch` on the current device, resolved on the first call
// there (with that device current) and kept.
int32_t scratch_address(void** out) {
  int dev = 0;
  SKLS_TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d beyond the %d devices the library tracks", dev, kMaxDevices);
    return SKLS_ERR_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[dev] == nullptr) {
    void* p = nullptr;
    SKLS_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr) {
      set_error("hipGetSymbolAddress returned no address for the scratch array");
      return SKLS_ERR_DEVICE;
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return SKLS_OK;
}

}  // namespace
}  // namespace skls

using namespace skls;

extern "C" {

int32_t skls_sketch_noalloc(const skls_matrix* A, const void* b, int32_t b_dtype, int64_t t, uint64_t seed,
                            const float* w, int32_t variant, void* SA, void* Sb, int32_t out_dtype, void* stream) {
  clear_error();
  SKLS_TRY(check_sketch_args(A, b, b_dtype, t, variant, SA, Sb, out_dtype));
  const size_t need = sketch_ws_bytes(*A, t, variant);
  if (need > kScratchBytes) {
    set_error("skls_sketch_noalloc: this input needs %zu bytes of plan, more than the %zu bytes of its fixed "
              "scratch; use skls_sketch with a workspace",
              need, kScratchBytes);
    return SKLS_ERR_WORKSPACE;
  }
  void* ws = nullptr;
  SKLS_TRY(scratch_address(&ws));
  return run_sketch_key(*A, b, b_dtype, t, plain_key(seed), w, variant, SA, Sb, out_dtype, ws, kScratchBytes,
                        as_stream(stream));
}

}  // extern "C"
