// la_noalloc.hip -- la_forward_noalloc: the forward pass with its workspace
// in a fixed device array of this library instead of caller memory, for
// callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid allocation).
//
// The array lives in this file's code object.  Its address on a device is
// taken once per device with hipGetSymbolAddress (the array's name in host
// code is only a host-side stand-in for it) and kept; every later call on
// that device passes the kept address to the forward pass as its
// workspace, exactly where la_forward takes the caller's.  Each device
// holds its own copy of the array until the process ends.  The forward
// pass writes every workspace byte it later reads (partial sums, FP64
// summary, operand images) before reading it, so nothing left by an
// earlier call needs clearing.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/la.h"
#include "la_kernels.h"

namespace {

constexpr size_t kScratchBytes = size_t(LA_NOALLOC_SCRATCH_BYTES);
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// The device address of this device's array (taken on first use).
la_status scratch_for_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (la_status)la::record_hip_error((int32_t)e);
  if (dev < 0 || dev >= kMaxDevices) return LA_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (la_status)la::record_hip_error((int32_t)e);
    if (!p) return LA_ERR_HIP;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return LA_OK;
}

}  // namespace

extern "C" la_status la_forward_noalloc(const la_attn_desc* desc, const void* q, const void* k,
                                        const void* v, void* o, double* s_out, double* z_out,
                                        la_stream stream) {
  size_t need = 0;
  la_status st = la_workspace_size(desc, 0, &need);
  if (st != LA_OK) return st;
  if (need > kScratchBytes) return LA_ERR_OOM;  // beyond the fixed array
  void* ws = nullptr;
  st = scratch_for_current_device(&ws);
  if (st != LA_OK) return st;
  return la_forward(desc, q, k, v, o, s_out, z_out, ws, kScratchBytes, stream);
}
