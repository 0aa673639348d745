// Instantiation of the fused forward kernels for F16 storage.
#include "fwd_kernel.h"

namespace fcfs {

fcfs_status launch_forward_f16(int method, const FwdArgs& a, const FwdGeom& g, hipStream_t stream) {
  return fwd::launch_forward_dt<FCFS_F16>(method, a, g, stream);
}

}  // namespace fcfs
