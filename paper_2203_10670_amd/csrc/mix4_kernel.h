// Learned channel-mixing FCFS layer on MFMA (gfx950).
//
// For every phase (jh, jw) the layer is a dense contraction (an implicit
// GEMM): y[n][o][p_h*mh + jh][p_w*mw + jw] = sum over c < C_in and the 4x4
// taps (a, b) of W[jh][jw][o][c][a][b] * ext(x)[n][c][q_h*mh + off_h[jh] + a]
// [q_w*mw + off_w[jw] + b], i.e. rows M = cells (n, mh, mw), columns N = o,
// reduction K = (c, a, b) with k = 16c + 4a + b.
//
// Workgroup: 4 waves, 128 cells (TH x TW), 64 output channels, one height
// phase jh and a group of up to kGroup width phases. The K loop takes two
// input channels at a time (one MFMA K-step of 32): the workgroup stages the
// padded input patch those cells read (for every phase of the group: they
// share it) and the weight chunk of the group in LDS; each wave then builds
// its A fragments from the patch and reads its B fragments from the chunk.
// Wave tile: 32 cells x 64 channels per phase, v_mfma_f32_16x16x32 (bf16 or
// f16), FP32 accumulation. The epilogue stages 16 output channels at a time
// in LDS and writes whole output row segments.
//
// Operand layouts of v_mfma_f32_16x16x32_{bf16,f16} (checked on the device):
// A lane l holds row l%16, k = 8*(l/16) + i (i < 8); B lane l holds column
// l%16, the same k; D lane l holds column l%16, rows 4*(l/16) + i (i < 4).
#pragma once

#include <hip/hip_runtime.h>

#include "fcfs_internal.h"
#include "fwd_kernel.h"

namespace fcfs {
namespace mix {

using fwd::pad_source;

constexpr int kThreads = 256;
constexpr int kGroup = 5;     // width phases per workgroup
constexpr int kOut = 64;      // output channels per workgroup

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

template <int DT> struct Mfma;
template <> struct Mfma<FCFS_BF16> {
  typedef __bf16 v8 __attribute__((ext_vector_type(8)));
  static __device__ __forceinline__ f32x4 mma(u16x8 a, u16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8, a), __builtin_bit_cast(v8, b), c, 0, 0, 0);
  }
  static __device__ __forceinline__ uint16_t to_store(float v) {
    const uint32_t u = __float_as_uint(v);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
  }
};
template <> struct Mfma<FCFS_F16> {
  typedef _Float16 v8 __attribute__((ext_vector_type(8)));
  static __device__ __forceinline__ f32x4 mma(u16x8 a, u16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(v8, a), __builtin_bit_cast(v8, b), c, 0, 0, 0);
  }
  static __device__ __forceinline__ uint16_t to_store(float v) {
    return __builtin_bit_cast(uint16_t, (_Float16)v);
  }
};

template <int DT>
__global__ __launch_bounds__(kThreads) void mix4_kernel(const MixArgs a) {
  using M = Mfma<DT>;
  extern __shared__ float smem[];
  const AxisTable& TH = a.th;
  const AxisTable& TW = a.tw_tab;

  // block -> (n, tile row, tile col, jh, group, output-channel tile)
  int64_t b = blockIdx.x;
  const int otile = (int)(b % a.otiles); b /= a.otiles;
  const int group = (int)(b % a.groups); b /= a.groups;
  const int jh = (int)(b % TH.p); b /= TH.p;
  const int tcol = (int)(b % a.tiles_w); b /= a.tiles_w;
  const int trow = (int)(b % a.tiles_h); b /= a.tiles_h;
  const int n = (int)b;

  const int mh0 = trow * a.th_cells, mw0 = tcol * a.tw_cells;
  const int jw0 = group * kGroup;
  const int P = min(kGroup, TW.p - jw0);
  const int o0 = otile * kOut;

  // input patch of the tile for this jh and the group's width phases
  const int r0 = TH.q * mh0 + TH.off[jh];
  const int R = TH.q * (a.th_cells - 1) + 4;
  const int cbase = TW.off[jw0];
  const int c0 = TW.q * mw0 + cbase;
  const int Cc = (TW.q * (a.tw_cells - 1) + TW.off[jw0 + P - 1] - cbase + 4 + 1) & ~1;   // even
  uint16_t* patch = reinterpret_cast<uint16_t*>(smem);                  // [2][R][Cc]
  uint16_t* wch = patch + 2 * R * Cc;                                    // [P][64][2][16]
  wch = reinterpret_cast<uint16_t*>((reinterpret_cast<uintptr_t>(wch) + 15) & ~(uintptr_t)15);

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int g4 = lane >> 4;        // k group of this lane: channel g4/2, taps 8*(g4%2)..
  const int li = lane & 15;

  // cells of this lane's A rows (two M tiles of 16)
  int arow[2], acol[2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    const int cell = wave * 32 + mt * 16 + li;
    const int lh = cell / a.tw_cells, lw = cell % a.tw_cells;
    arow[mt] = TH.q * lh + 2 * (g4 & 1);
    acol[mt] = TW.q * lw;
  }
  const int ach = g4 >> 1;

  f32x4 acc[kGroup][2][4];
#pragma unroll
  for (int ph = 0; ph < kGroup; ++ph)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[ph][mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};

  const uint16_t* xin = reinterpret_cast<const uint16_t*>(a.x);
  const uint16_t* win = reinterpret_cast<const uint16_t*>(a.w);

  for (int cc = 0; cc < a.Cin; cc += 2) {
    __syncthreads();
    // stage the padded input patch of channels cc, cc+1
    for (int idx = threadIdx.x; idx < 2 * R * Cc; idx += kThreads) {
      const int ch = idx / (R * Cc);
      const int rem = idx - ch * R * Cc;
      const int rr = rem / Cc, col = rem - rr * Cc;
      const int sr = pad_source(r0 + rr, a.H, a.pad), sc = pad_source(c0 + col, a.W, a.pad);
      uint16_t v = 0;
      if (cc + ch < a.Cin && sr >= 0 && sc >= 0)
        v = xin[(((int64_t)n * a.Cin + cc + ch) * a.H + sr) * a.W + sc];
      patch[idx] = v;
    }
    // stage the weights: [ph][o][ch][16 taps], 8 taps (16 bytes) per item
    for (int idx = threadIdx.x; idx < P * kOut * 2 * 2; idx += kThreads) {
      const int half = idx & 1;
      const int ch = (idx >> 1) & 1;
      const int o = (idx >> 2) % kOut;
      const int ph = (idx >> 2) / kOut;
      uint4 v = {0u, 0u, 0u, 0u};
      if (o0 + o < a.Cout && cc + ch < a.Cin) {
        const int64_t e = ((((int64_t)jh * TW.p + jw0 + ph) * a.Cout + o0 + o) * a.Cin + cc + ch) * 16 + half * 8;
        v = *reinterpret_cast<const uint4*>(win + e);
      }
      *reinterpret_cast<uint4*>(wch + ((ph * kOut + o) * 2 + ch) * 16 + half * 8) = v;
    }
    __syncthreads();
#pragma unroll
    for (int ph = 0; ph < kGroup; ++ph) {
      if (ph >= P) break;   // uniform; unrolled so acc[ph] stays in registers
      const int dcol = TW.off[jw0 + ph] - cbase;
      u16x8 af[2];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        const uint16_t* p0 = patch + (ach * R + arow[mt]) * Cc + acol[mt] + dcol;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          af[mt][i] = p0[i];
          af[mt][4 + i] = p0[Cc + i];
        }
      }
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const u16x8 bf =
            *reinterpret_cast<const u16x8*>(wch + ((ph * kOut + nt * 16 + li) * 2 + ach) * 16 + (g4 & 1) * 8);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) acc[ph][mt][nt] = M::mma(af[mt], bf, acc[ph][mt][nt]);
      }
    }
  }

  // epilogue: 16 output channels at a time through LDS, whole row segments out
  __syncthreads();
  uint16_t* ob = reinterpret_cast<uint16_t*>(smem);   // [16][th_cells][tw_cells * P]
  const int segw = a.tw_cells * P;
  uint16_t* yout = reinterpret_cast<uint16_t*>(a.y);
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
    for (int ph = 0; ph < kGroup; ++ph) {
      if (ph >= P) break;
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int cell = wave * 32 + mt * 16 + 4 * g4 + i;
          const int lh = cell / a.tw_cells, lw = cell % a.tw_cells;
          ob[(li * a.th_cells + lh) * segw + lw * P + ph] = M::to_store(acc[ph][mt][nt][i]);
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < 16 * a.th_cells * segw; idx += kThreads) {
      const int ol = idx / (a.th_cells * segw);
      const int rem = idx - ol * a.th_cells * segw;
      const int lh = rem / segw, e = rem - lh * segw;
      const int lw = e / P, ph = e - lw * P;
      const int o = o0 + nt * 16 + ol, mh = mh0 + lh, mw = mw0 + lw;
      if (o < a.Cout && mh < a.Mh && mw < a.Mw)
        __builtin_nontemporal_store(ob[idx], yout + (((int64_t)n * a.Cout + o) * a.Ho + TH.p * mh + jh) * a.Wo +
                                                 TW.p * mw + jw0 + ph);
    }
    __syncthreads();
  }
}

template <int DT>
fcfs_status launch_mix4_dt(const MixArgs& a, hipStream_t stream) {
  const int64_t blocks = (int64_t)a.N * a.tiles_h * a.tiles_w * a.th.p * a.groups * a.otiles;
  hipLaunchKernelGGL((mix4_kernel<DT>), dim3((unsigned)blocks), dim3(kThreads), a.lds_bytes, stream, a);
  return hipGetLastError() == hipSuccess ? FCFS_OK : FCFS_E_DEVICE;
}

}  // namespace mix
}  // namespace fcfs
