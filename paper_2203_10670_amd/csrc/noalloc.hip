// fcfs_backward_noalloc: the backward with its workspace in a fixed device
// array instead of a caller-supplied buffer, for callers that cannot
// allocate device memory (code under HIP graph capture, serving loops that
// must not allocate). The kernels are fcfs_backward's.
//
// The array is a file-scope __device__ variable: every GPU the library is
// loaded on holds its own copy, at its own address, until the process ends.
// Its name in host code is only a stand-in for the symbol, so the device
// address is looked up once per device (hipGetSymbolAddress, with that device
// current) and that address is what the kernels receive.

#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>

#include "fcfs_internal.h"

namespace fcfs {
namespace {

static __device__ __align__(256) unsigned char scratch[FCFS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::atomic<void*> g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// Device address of `scratch` on device `dev` (looked up on the first call
// for that device).
fcfs_status scratch_on(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return FCFS_E_UNSUPPORTED;
  void* p = g_scratch[dev].load(std::memory_order_acquire);
  if (!p) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    p = g_scratch[dev].load(std::memory_order_relaxed);
    if (!p) {
      int cur = 0;
      if (hipGetDevice(&cur) != hipSuccess) return FCFS_E_DEVICE;
      if (cur != dev && hipSetDevice(dev) != hipSuccess) return FCFS_E_DEVICE;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (cur != dev && hipSetDevice(cur) != hipSuccess) return FCFS_E_DEVICE;
      if (e != hipSuccess || !p) return FCFS_E_DEVICE;
      g_scratch[dev].store(p, std::memory_order_release);
    }
  }
  *out = p;
  return FCFS_OK;
}

}  // namespace
}  // namespace fcfs

extern "C" fcfs_status fcfs_backward_noalloc(fcfs_plan_t plan, fcfs_dtype dtype, int64_t n, int64_t c_in,
                                             int64_t h, int64_t w, const void* x, const void* weight,
                                             int64_t c_out, const void* dy, void* dx, float* dw,
                                             hipStream_t stream) {
  size_t need = 0;
  fcfs_status st = fcfs::backward_workspace_need(plan, dtype, n, c_in, h, w, c_out, dw != nullptr, &need);
  if (st != FCFS_OK) return st;
  if (need > (size_t)FCFS_NOALLOC_SCRATCH_BYTES) return FCFS_E_UNSUPPORTED;
  if (need == 0) return fcfs_backward(plan, dtype, n, c_in, h, w, x, weight, c_out, dy, dx, dw, nullptr, 0, stream);
  // the kernels run on the stream's device
  int dev = 0;
  const hipError_t e = stream ? hipStreamGetDevice(stream, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess) return FCFS_E_DEVICE;
  void* ws = nullptr;
  st = fcfs::scratch_on(dev, &ws);
  if (st != FCFS_OK) return st;
  // Every workspace word the kernels read is written first by an earlier
  // kernel of the same call (adjoint tables, then partial sums), so nothing
  // left by a previous call is read and no clearing is needed.
  return fcfs_backward(plan, dtype, n, c_in, h, w, x, weight, c_out, dy, dx, dw, ws,
                       (size_t)FCFS_NOALLOC_SCRATCH_BYTES, stream);
}
