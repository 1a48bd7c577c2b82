// Scratch memory of select_kth_noalloc: one file-scope device array per GPU instead of the
// handle's allocated workspace, for callers that cannot allocate (code under stream capture,
// serving loops, harnesses that forbid hipMalloc).
//
// In host code `scratch` names a host-side stand-in, not device memory.  Its device address
// is taken once per device, with that device current, by noalloc_bind (called from
// cps_create) and kept in g_ptr; every host use of the array (kernel arguments, the clearing
// launch) goes through that address.  Each GPU holds its own copy until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "cps_kernels.h"

namespace cps {

namespace {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Zero `words` 8-byte words from p (a fill kernel rather than a memset node, so the call
// can be captured in a graph).
__global__ __launch_bounds__(256) void scratch_clear_kernel(uint64_t *p, int64_t words) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (int64_t)gridDim.x * 256)
    p[i] = 0;
}

}  // namespace

hipError_t noalloc_bind(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return hipSuccess;
  void *p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_ptr[device] = p;
  return hipSuccess;
}

void *noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ptr[device];
}

hipError_t launch_scratch_clear(void *p, size_t bytes, hipStream_t stream) {
  const int64_t words = (int64_t)(bytes / 8);
  if (words < 1) return hipSuccess;
  int64_t blocks = (words + 255) / 256;
  if (blocks > 64) blocks = 64;
  scratch_clear_kernel<<<dim3((unsigned)blocks), dim3(256), 0, stream>>>((uint64_t *)p, words);
  return hipGetLastError();
}

}  // namespace cps
