// Instantiation of the channel-mixing MFMA kernels (BF16 and FP16 storage).
#include "mix4_kernel.h"
#include "mix4_cl.h"

namespace fcfs {

fcfs_status launch_mix4(int dtype, const MixArgs& a, hipStream_t stream) {
  if (dtype == FCFS_BF16) return mix::launch_mix4_dt<FCFS_BF16>(a, stream);
  if (dtype == FCFS_F16) return mix::launch_mix4_dt<FCFS_F16>(a, stream);
  return FCFS_E_UNSUPPORTED;
}

}  // namespace fcfs
