// Instantiation of the backward kernels for F32 storage.
#include "bwd_kernel.h"

namespace fcfs {

fcfs_status launch_backward_f32(const BwdArgs& a, bool learned, hipStream_t stream) {
  return bwd::launch_backward_dt<FCFS_F32>(a, learned, stream);
}

}  // namespace fcfs
