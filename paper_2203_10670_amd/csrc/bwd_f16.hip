// Instantiation of the backward kernels for F16 storage.
#include "bwd_kernel.h"

namespace fcfs {

fcfs_status launch_backward_f16(const BwdArgs& a, bool learned, hipStream_t stream) {
  return bwd::launch_backward_dt<FCFS_F16>(a, learned, stream);
}

}  // namespace fcfs
