// Instantiation of the fused forward kernels for F32 storage.
#include "fwd_kernel.h"

namespace fcfs {

fcfs_status launch_forward_f32(int method, const FwdArgs& a, const FwdGeom& g, hipStream_t stream) {
  return fwd::launch_forward_dt<FCFS_F32>(method, a, g, stream);
}

}  // namespace fcfs
