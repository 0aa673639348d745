// The LDS arrays of the host emulation (one workgroup runs at a time). Each
// kernel namespace declares `extern __shared__ float smem[]` at block scope,
// which names an array in that namespace.
#include "hip/hip_runtime.h"
namespace fcfs {
namespace fwd {
alignas(16) float smem[hostemu::kLdsFloats];
}  // namespace fwd
namespace bwd {
alignas(16) float smem[hostemu::kLdsFloats];
}  // namespace bwd
namespace mix {
alignas(16) float smem[hostemu::kLdsFloats];
}  // namespace mix
namespace bwdmix {
alignas(16) float smem[hostemu::kLdsFloats];
}  // namespace bwdmix
namespace mixf32 {
alignas(16) float smem[hostemu::kLdsFloats];
}  // namespace mixf32
}  // namespace fcfs

namespace hostemu {
float* const lds_arrays[] = {fcfs::fwd::smem, fcfs::bwd::smem, fcfs::mix::smem, fcfs::bwdmix::smem,
                             fcfs::mixf32::smem};
const int n_lds_arrays = sizeof(lds_arrays) / sizeof(lds_arrays[0]);
}  // namespace hostemu
