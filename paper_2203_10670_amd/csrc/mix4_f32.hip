// Channel-mixing FCFS layer with FP32 storage on the FP32 matrix cores
// (v_mfma_f32_16x16x4_f32), gfx950.
//
// Same contraction as the 16-bit kernels (Sec. 7's learnable weights, mixing
// channels): for every phase (jh, jw),
//   y[n][o][p_h mh + jh][p_w mw + jw] = sum over c, a, b of
//     W[jh][jw][o][c][a][b] * ext(x)[n][c][q_h mh + off_h(jh) + a][q_w mw + off_w(jw) + b],
// an implicit GEMM with rows M = cells, columns N = output channels and
// reduction K = (c, a, b). One MFMA K-step is the 4 tap columns b of one
// (channel, tap row). Operand layouts of v_mfma_f32_16x16x4_f32: A lane l
// holds row l % 16, k = l / 16; B lane l holds column l % 16, the same k; D
// lane l holds column l % 16, rows 4 (l / 16) + i.
//
// Workgroup: 4 waves; 64 cells (4 cell rows of 16 cells, one M tile per cell
// row); 64 output channels (wave w: outputs 16 w .. 16 w + 15, one N tile);
// one height phase jh and a group of G width phases, which share the staged
// patch. A stage is kCS input channels. Its patch holds, for each cell, the 4
// tap rows and the wspan tap columns the group's phases reach,
// [c][4 lh + a][lw][kWS] floats, so any q stages only what the taps read. Two
// LDS buffers: the next stage's samples are loaded into registers before the
// stage's MFMAs and stored after them, one barrier per stage. B fragments (the
// weights) are read straight from global memory, where every workgroup shares
// them, two K-steps ahead. At FP32 an MFMA takes 32 cycles, so the operands'
// 8 bytes per lane per MFMA are far below what LDS and the caches deliver.
#include <hip/hip_runtime.h>

#include "fcfs_internal.h"
#include "fwd_kernel.h"

namespace fcfs {
namespace mixf32 {

using fwd::pad_source;
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kCS = 4;     // input channels per stage
constexpr int kTH = 4;     // cell rows per workgroup (one M tile each)
constexpr int kTW = 16;    // cells per cell row
constexpr int kOut = 64;   // output channels per workgroup
constexpr int kWS = 8;     // patch columns per cell (the group's tap columns, wspan <= 8)
constexpr int kPatch = kCS * 4 * kTH * kTW * kWS;   // floats per stage buffer
constexpr int kItems = kPatch / kThreads;           // staged samples per thread

template <int G>
__global__ __launch_bounds__(kThreads) void mix4_f32_kernel(const MixArgs a) {
  extern __shared__ float smem[];
  const AxisTable& TH = a.th;
  const AxisTable& TW = a.tw_tab;
  // Block b runs on XCD b % 8; renumbering gives each XCD a contiguous range,
  // so the output tiles and phase groups that share a patch meet in one L2.
  int64_t blk = blockIdx.x;
  {
    const int64_t per = (int64_t)gridDim.x / 8;
    if (blk < 8 * per) blk = (blk % 8) * per + blk / 8;
  }
  const int otile = (int)(blk % a.otiles); blk /= a.otiles;
  const int group = (int)(blk % a.groups); blk /= a.groups;
  const int jh = (int)(blk % TH.p); blk /= TH.p;
  const int tcol = (int)(blk % a.tiles_w); blk /= a.tiles_w;
  const int trow = (int)(blk % a.tiles_h); blk /= a.tiles_h;
  const int n = (int)blk;

  const int mh0 = trow * kTH, mw0 = tcol * kTW;
  const int jw0 = group * G;
  const int P = min(G, TW.p - jw0);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, g4 = lane >> 4;
  const int wspan = a.wspan;
  const int cbase = TW.off[jw0];
  const int64_t plane = (int64_t)a.H * a.W;
  const float* const xin = reinterpret_cast<const float*>(a.x) + (int64_t)n * a.Cin * plane;
  const float* const win = reinterpret_cast<const float*>(a.w);
  float* const lds = smem;

  // ---- staging: item it = tid + 256 r is (c, 4 lh + a, lw, column u) of the
  // patch, in that order (u fastest); columns u >= wspan are never read and
  // are left unloaded
  float pre[kItems];
  auto load_stage = [&](int cs) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const int it = tid + kThreads * r;
      const int u = it % kWS, lw = (it / kWS) % kTW, rr = (it / (kWS * kTW)) % 16, c = it / (kWS * kTW * 16);
      const int sr = pad_source(TH.q * (mh0 + (rr >> 2)) + TH.off[jh] + (rr & 3), a.H, a.pad);
      const int sc = pad_source(TW.q * (mw0 + lw) + cbase + u, a.W, a.pad);
      const bool ok = u < wspan && sr >= 0 && sc >= 0 && cs + c < a.Cin;
      const float v = xin[ok ? (int64_t)(cs + c) * plane + (int64_t)sr * a.W + sc : 0];
      pre[r] = ok ? v : 0.f;
    }
  };
  auto store_stage = [&](float* buf) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < kItems; ++r) buf[tid + kThreads * r] = pre[r];
  };

  // ---- B fragments: lane (output li of this wave's tile, tap column g4) of
  // phase ph and K-step (c, a): W[jh][jw0 + ph][o][c][a][g4]
  const int oo = otile * kOut + 16 * wave + li;   // this lane's output channel
  int64_t wrow[G];   // index of W[jh][jw0 + ph][oo][0][0][g4], or -1 when absent
#pragma unroll
  for (int ph = 0; ph < G; ++ph) {
    const bool ok = ph < P && oo < a.Cout;
    wrow[ph] = ok ? ((((int64_t)jh * TW.p + jw0 + ph) * a.Cout + oo) * a.Cin) * 16 + g4 : -1;
  }
  auto load_b = [&](float (&dst)[G], int cin, int ta) __attribute__((always_inline)) {
#pragma unroll
    for (int ph = 0; ph < G; ++ph) {
      const bool ok = wrow[ph] >= 0 && cin < a.Cin;
      const float v = win[ok ? wrow[ph] + (int64_t)cin * 16 + 4 * ta : 0];
      dst[ph] = ok ? v : 0.f;
    }
  };

  int dcol[G];   // tap column offset of each phase in the group (0 past P)
#pragma unroll
  for (int ph = 0; ph < G; ++ph) dcol[ph] = ph < P ? TW.off[jw0 + ph] - cbase : 0;

  f32x4 acc[G][kTH];
#pragma unroll
  for (int ph = 0; ph < G; ++ph)
#pragma unroll
    for (int mt = 0; mt < kTH; ++mt) acc[ph][mt] = f32x4{0.f, 0.f, 0.f, 0.f};

  // one stage: 16 K-steps (c, a), each G phases x 4 M tiles
  auto compute = [&](const float* buf, int cs) __attribute__((always_inline)) {
    float bq[3][G];
    load_b(bq[0], cs, 0);
    load_b(bq[1], cs, 1);
#pragma unroll
    for (int k = 0; k < kCS * 4; ++k) {
      const int c = k >> 2, ta = k & 3;
      if (k + 2 < kCS * 4) load_b(bq[(k + 2) % 3], cs + ((k + 2) >> 2), (k + 2) & 3);
#pragma unroll
      for (int ph = 0; ph < G; ++ph) {
#pragma unroll
        for (int mt = 0; mt < kTH; ++mt) {
          const float av = buf[((c * 16 + 4 * mt + ta) * kTW + li) * kWS + dcol[ph] + g4];
          acc[ph][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bq[k % 3][ph], acc[ph][mt], 0, 0, 0);
        }
      }
    }
  };

  const int nst = (a.Cin + kCS - 1) / kCS;
  load_stage(0);
  store_stage(lds);
  __syncthreads();
  for (int s = 0; s < nst; ++s) {
    float* const cur = lds + (s & 1) * kPatch;
    float* const nxt = lds + ((s + 1) & 1) * kPatch;
    const bool more = s + 1 < nst;
    if (more) load_stage(kCS * (s + 1));
    __builtin_amdgcn_sched_barrier(0);
    compute(cur, kCS * s);
    __builtin_amdgcn_sched_barrier(0);
    if (more) store_stage(nxt);
    __syncthreads();
  }

  // ---- epilogue: cell row by cell row, each wave stages its 16 outputs x
  // (16 cells x P phases) in its own LDS block ([output][lw P + ph]) and
  // writes each output's row segment: runs of P adjacent samples per cell
  float* const ob = lds + wave * (16 * kTW * G);
  const int segw = kTW * P;
  const int64_t ostride = (int64_t)a.Ho * a.Wo;
  float* const ybase = reinterpret_cast<float*>(a.y) + ((int64_t)n * a.Cout + otile * kOut + 16 * wave) * ostride;
#pragma unroll
  for (int mt = 0; mt < kTH; ++mt) {
#pragma unroll
    for (int ph = 0; ph < G; ++ph) {
      if (ph >= P) break;
#pragma unroll
      for (int i = 0; i < 4; ++i) ob[li * segw + (4 * g4 + i) * P + ph] = acc[ph][mt][i];
    }
    fwd::wave_lds_sync();
    const int mh = mh0 + mt;
    if (mh < a.Mh) {
      const int64_t rowoff = (int64_t)(TH.p * mh + jh) * a.Wo;
      for (int ol = 0; ol < 16; ++ol) {
        if (otile * kOut + 16 * wave + ol >= a.Cout) break;
        float* const rp = ybase + ol * ostride + rowoff;
        for (int e = lane; e < segw; e += 64) {
          const int lw = e / P, ph = e - lw * P;
          if (mw0 + lw < a.Mw) __builtin_nontemporal_store(ob[ol * segw + e], rp + TW.p * (mw0 + lw) + jw0 + ph);
        }
      }
    }
    fwd::wave_lds_sync();
  }
}

}  // namespace mixf32

fcfs_status launch_mix4_f32(const MixArgs& a, hipStream_t stream) {
  const dim3 block(mixf32::kThreads);
  const int64_t blocks = (int64_t)a.N * a.tiles_h * a.tiles_w * a.th.p * a.groups * a.otiles;
  const dim3 grid((unsigned)blocks);
  const size_t lds = sizeof(float) * 2 * mixf32::kPatch;
  switch (a.gsize) {
    case 1: hipLaunchKernelGGL((mixf32::mix4_f32_kernel<1>), grid, block, lds, stream, a); break;
    case 2: hipLaunchKernelGGL((mixf32::mix4_f32_kernel<2>), grid, block, lds, stream, a); break;
    case 3: hipLaunchKernelGGL((mixf32::mix4_f32_kernel<3>), grid, block, lds, stream, a); break;
    case 4: hipLaunchKernelGGL((mixf32::mix4_f32_kernel<4>), grid, block, lds, stream, a); break;
    default: hipLaunchKernelGGL((mixf32::mix4_f32_kernel<5>), grid, block, lds, stream, a); break;
  }
  return hipGetLastError() == hipSuccess ? FCFS_OK : FCFS_E_DEVICE;
}

}  // namespace fcfs
