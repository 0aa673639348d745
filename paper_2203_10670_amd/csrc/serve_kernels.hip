// Kernels of the serving loop: the batched forward (one launch covering many
// requests) and the seeded input generator.
#include "fwd_kernel.h"

namespace fcfs {
namespace serve {

using fwd::fwd_wave;

// Wave w of the batch finds its request r (wave_start[r] <= w < wave_start[r+1])
// and runs that request's forward instance on its own wave index (offset by
// the first wave of the request's chunk in this batch).
__global__ __launch_bounds__(256) void fwd_batch_kernel(const BatchArgs b) {
  extern __shared__ float smem[];
  const int lane = threadIdx.x & 63;
  const int wslot = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t wid = (int64_t)blockIdx.x * fwd::kWaves + wslot;
  if (wid >= b.total_waves) return;
  int lo = 0, hi = b.nreq - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.wave_start[mid] <= wid) lo = mid;
    else hi = mid - 1;
  }
  const BatchDesc& d = b.desc[lo];
  const int64_t lw = wid - b.wave_start[lo] + d.wave_begin;
  if (lw >= d.args.waves) return;
  switch (d.variant) {
    case 0: fwd_wave<FCFS_F32, 1, 4, 8, false>(d.args, lw, wslot, lane, smem); break;
    case 1: fwd_wave<FCFS_F32, 1, 1, 8, false>(d.args, lw, wslot, lane, smem); break;
    case 2: fwd_wave<FCFS_F32, 2, 4, 8, false>(d.args, lw, wslot, lane, smem); break;
    case 3: fwd_wave<FCFS_F32, 2, 1, 8, false>(d.args, lw, wslot, lane, smem); break;
    case 4: fwd_wave<FCFS_F32, 4, 4, 8, false>(d.args, lw, wslot, lane, smem); break;
    case 5: fwd_wave<FCFS_F32, 4, 1, 8, false>(d.args, lw, wslot, lane, smem); break;
    case 6: fwd_wave<FCFS_BF16, 1, 4, 8, false>(d.args, lw, wslot, lane, smem); break;
    case 7: fwd_wave<FCFS_BF16, 1, 1, 8, false>(d.args, lw, wslot, lane, smem); break;
    case 8: fwd_wave<FCFS_BF16, 2, 4, 8, false>(d.args, lw, wslot, lane, smem); break;
    case 9: fwd_wave<FCFS_BF16, 2, 1, 8, false>(d.args, lw, wslot, lane, smem); break;
    case 10: fwd_wave<FCFS_BF16, 4, 4, 8, false>(d.args, lw, wslot, lane, smem); break;
    default: fwd_wave<FCFS_BF16, 4, 1, 8, false>(d.args, lw, wslot, lane, smem); break;
  }
}

// splitmix64 of (seed, index): the published mixing function of Steele, Lea
// and Flood's SplittableRandom, applied to seed + (index + 1) * golden gamma.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void generate_kernel(const GenArgs g) {
  const int64_t blk = blockIdx.x;
  if (blk >= g.total_blocks) return;
  int lo = 0, hi = g.ngen - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g.block_start[mid] <= blk) lo = mid;
    else hi = mid - 1;
  }
  const GenDesc& d = g.desc[lo];
  const int64_t base = (blk - g.block_start[lo]) * kGenPerBlock;
  for (int k = 0; k < kGenPerBlock / 256; ++k) {
    const int64_t i = base + (int64_t)k * 256 + threadIdx.x;
    if (i >= d.count) break;
    const float v = (float)(splitmix64(d.seed, (uint64_t)i) >> 40) * (1.0f / 16777216.0f);
    if (d.dtype == FCFS_F32) reinterpret_cast<float*>(d.x)[i] = v;
    else fwd::Store<FCFS_BF16>::store(reinterpret_cast<uint16_t*>(d.x) + i, v);
  }
}

}  // namespace serve

fcfs_status launch_forward_batch(const BatchArgs& b, hipStream_t stream) {
  if (b.total_waves <= 0) return FCFS_OK;
  const size_t lds = sizeof(float) * fwd::kWaves * fwd::kRowMax;
  hipLaunchKernelGGL(serve::fwd_batch_kernel, dim3((unsigned)((b.total_waves + fwd::kWaves - 1) / fwd::kWaves)),
                     dim3(256), lds, stream, b);
  return hipGetLastError() == hipSuccess ? FCFS_OK : FCFS_E_DEVICE;
}

fcfs_status launch_generate(const GenArgs& g, hipStream_t stream) {
  if (g.total_blocks <= 0) return FCFS_OK;
  hipLaunchKernelGGL(serve::generate_kernel, dim3((unsigned)g.total_blocks), dim3(256), 0, stream, g);
  return hipGetLastError() == hipSuccess ? FCFS_OK : FCFS_E_DEVICE;
}

}  // namespace fcfs
