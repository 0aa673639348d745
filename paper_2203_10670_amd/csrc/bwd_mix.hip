// Instantiation of the channel-mixing backward kernels (16-bit storage).
#include "bwd_mix.h"

namespace fcfs {

fcfs_status launch_backward_mix_bf16(const BwdArgs& a, hipStream_t stream) {
  return bwdmix::launch_backward_mix_dt<FCFS_BF16>(a, stream);
}

fcfs_status launch_backward_mix_f16(const BwdArgs& a, hipStream_t stream) {
  return bwdmix::launch_backward_mix_dt<FCFS_F16>(a, stream);
}

}  // namespace fcfs
