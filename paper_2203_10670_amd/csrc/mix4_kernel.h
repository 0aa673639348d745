// Learned channel-mixing FCFS layer on MFMA (gfx950).
//
// For every phase (jh, jw) the layer is a dense contraction (an implicit
// GEMM): y[n][o][p_h*mh + jh][p_w*mw + jw] = sum over c < C_in and the 4x4
// taps (a, b) of W[jh][jw][o][c][a][b] * ext(x)[n][c][q_h*mh + off_h[jh] + a]
// [q_w*mw + off_w[jw] + b], i.e. rows M = cells (n, mh, mw), columns N = o,
// reduction K = (c, a, b) with k = 16c + 4a + b.
//
// Workgroup: 4 waves, 128 cells (th_cells x tw_cells), kOut output channels,
// one height phase jh and a group of up to kGroup width phases, which share
// the staged input patch. The K loop takes two input channels per step (one
// MFMA K-step of 32). Each step's patch (2 channels) and weights (the group's
// phases x kOut outputs x 32 k) sit in one of two LDS buffers: while the waves
// run the step's MFMAs from one buffer, the next step's data is already on
// its way into registers, and is written to the other buffer afterwards, so
// one barrier per step orders everything and the global-memory latency hides
// behind the matrix work. (When two buffers do not fit, one buffer and a
// second barrier per step.)
//
// Wave tile: 32 cells x kOut channels per phase, v_mfma_f32_16x16x32 (bf16
// or f16), FP32 accumulation. The epilogue stages 16 output channels at a time
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
constexpr int kGroup = 5;      // width phases per workgroup, at most
constexpr int kOut = kMixOut;  // output channels per workgroup
constexpr int kWPitch = 32;    // 16-bit units per (phase, output) weight row in LDS (2 channels x 16 taps);
                               // its four 16-byte quads are stored rotated by ((o >> 1) & 3), so the
                               // 16-byte reads of 8 consecutive outputs hit distinct banks
constexpr int kRowsFast = 8;   // patch (channel, row) pairs per wave carried in registers across a step
constexpr int kSlotsFast = 3;  // ... times 64-column slots per row

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

template <int DT> struct Mfma;
template <> struct Mfma<FCFS_BF16> {
  typedef __bf16 v8 __attribute__((ext_vector_type(8)));
  static __device__ __forceinline__ f32x4 mma(u16x8 a, u16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8, a), __builtin_bit_cast(v8, b), c, 0, 0, 0);
  }
  static __device__ __forceinline__ uint16_t to_store(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
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

// FAST: the patch of a step is at most kRowsFast (channel, row) pairs per
// wave by kSlotsFast column slots, and two stage buffers fit: the next step's
// loads are issued before the step's MFMAs and land in the other buffer after
// them. Otherwise (large q or patches) one buffer, staged between steps.
// G: phases per group (min(5, p_w)); a group with fewer phases (the last of
// a p_w above 5) runs its missing phases on zero weights.
template <int DT, int G, bool FAST>
__global__ __launch_bounds__(kThreads) void mix4_kernel(const MixArgs a) {
  using M = Mfma<DT>;
  extern __shared__ float smem[];
  uint16_t* const lds = reinterpret_cast<uint16_t*>(smem);
  const AxisTable& TH = a.th;
  const AxisTable& TW = a.tw_tab;

  // block -> (n, tile row, tile col, jh, group, output-channel tile)
  int64_t blk = blockIdx.x;
  const int otile = (int)(blk % a.otiles); blk /= a.otiles;
  const int group = (int)(blk % a.groups); blk /= a.groups;
  const int jh = (int)(blk % TH.p); blk /= TH.p;
  const int tcol = (int)(blk % a.tiles_w); blk /= a.tiles_w;
  const int trow = (int)(blk % a.tiles_h); blk /= a.tiles_h;
  const int n = (int)blk;

  const int mh0 = trow * a.th_cells, mw0 = tcol * a.tw_cells;
  const int jw0 = group * G;
  const int P = min(G, TW.p - jw0);
  const int o0 = otile * kOut;
  const int r0 = TH.q * mh0 + TH.off[jh];          // first input row of the patch
  const int cbase = TW.off[jw0];
  const int c0 = TW.q * mw0 + cbase;                // first input column of the patch

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: row math stays scalar
  const int g4 = lane >> 4;        // k group of this lane: channel g4/2, tap rows 2*(g4%2), +1
  const int li = lane & 15;

  // ---- staging plan of this lane (fixed over the K loop)
  // Patch items: (channel, row) pair pr = wave + 4*i (channel pr / R, row
  // pr % R), column lane + 64*j. Columns past Cc are written to the spare
  // column Cc of the row (never read), so stores need no lane conditions.
  const uint16_t* xin = reinterpret_cast<const uint16_t*>(a.x) + (int64_t)n * a.Cin * a.H * a.W;
  auto src_col = [&](int pc) -> int {   // input column of patch column pc, or -1 (zero)
    const int c = a.cstep == TW.q ? c0 + pc : c0 + TW.q * (pc / a.wspan) + pc % a.wspan;
    return pad_source(c, a.W, a.pad);
  };
  auto src_row = [&](int rr) -> int {
    const int r = a.rstep == TH.q ? r0 + rr : r0 + TH.q * (rr >> 2) + (rr & 3);
    return pad_source(r, a.H, a.pad);
  };
  // weights: 16-byte quads (phase, output, quad) = it / (4 kOut),
  // (it / 4) % kOut, it % 4 (an output's 2 channels x 16 taps are 4 quads);
  // thread t moves items t, t + 256, ...; items past 4 G kOut go to a spare quad
  const uint16_t* win = reinterpret_cast<const uint16_t*>(a.w);
  constexpr int kWItems = (G * kOut * 4 + kThreads - 1) / kThreads;
  int64_t woff[kWItems];
  int wlds[kWItems];
  uint32_t wmask[kWItems];   // all ones when the quad exists (before the C_in check)
  int wch_hi[kWItems];       // channel (0 or 1) of the quad
#pragma unroll
  for (int k = 0; k < kWItems; ++k) {
    const int it = tid + kThreads * k;
    const int ph = it / (kOut * 4), o = (it / 4) % kOut, quad = it % 4;
    const bool ok = ph < P && o0 + o < a.Cout;
    wmask[k] = ok ? 0xffffffffu : 0u;
    wch_hi[k] = quad >> 1;
    woff[k] = ok ? ((((int64_t)jh * TW.p + jw0 + ph) * a.Cout + o0 + o) * a.Cin) * 16 + quad * 8 : 0;
    wlds[k] = ph < G ? (ph * kOut + o) * kWPitch + (quad ^ ((o >> 1) & 3)) * 8 : G * kOut * kWPitch;
  }
  // (the mask is applied where the quad is stored, so that the load itself
  // stays in flight until then)
  auto load_w = [&](int k, int cc) -> uint4 {
    const bool ok = wmask[k] && cc + wch_hi[k] < a.Cin;
    return *reinterpret_cast<const uint4*>(win + (ok ? woff[k] + cc * 16 : 0));
  };
  auto mask_w = [&](int k, int cc, uint4 v) -> uint4 {
    // quads 2 and 3 hold channel cc + 1, which may be past C_in
    const uint32_t m = cc + wch_hi[k] < a.Cin ? wmask[k] : 0u;
    return uint4{v.x & m, v.y & m, v.z & m, v.w & m};
  };

  // cells of this lane's A rows (two M tiles of 16)
  int abase[2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    const int cell = wave * 32 + mt * 16 + li;
    const int lh = cell / a.tw_cells, lw = cell - lh * a.tw_cells;
    abase[mt] = ((g4 >> 1) * a.R + a.rstep * lh + 2 * (g4 & 1)) * a.CP + a.cstep * lw;
  }

  constexpr int kNT = kOut / 16;
  f32x4 acc[G][2][kNT];
#pragma unroll
  for (int ph = 0; ph < G; ++ph)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < kNT; ++nt) acc[ph][mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};

  auto compute = [&](const uint16_t* patch) {
    const uint16_t* wch = patch + a.woff_u16;
#pragma unroll
    for (int ph = 0; ph < G; ++ph) {
      // (every phase of G, so the accumulators stay put in their registers)
      const int dcol = ph < P ? TW.off[jw0 + ph] - cbase : 0;
      u16x8 af[2];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        // 16-bit reads, kept apart (volatile): the window starts at any
        // element, and a merged 64-bit read of it would be misaligned
        const volatile __attribute__((address_space(3))) uint16_t* p0 =
            (const volatile __attribute__((address_space(3))) uint16_t*)(patch + abase[mt] + dcol);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          af[mt][i] = p0[i];
          af[mt][4 + i] = p0[a.CP + i];
        }
      }
#pragma unroll
      for (int nt = 0; nt < kNT; ++nt) {
        const u16x8 bf = *reinterpret_cast<const u16x8*>(wch + (ph * kOut + nt * 16 + li) * kWPitch +
                                                          (g4 ^ ((li >> 1) & 3)) * 8);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) acc[ph][mt][nt] = M::mma(af[mt], bf, acc[ph][mt][nt]);
      }
    }
  };

  const int nsteps = (a.Cin + 1) / 2;
  if constexpr (FAST) {
    // Per-lane plan of the patch items: byte offset of (row, column) in a
    // channel plane, and one bit per item, set unless zero padding supplies
    // it. Tiles clear of the image border under zero padding (and every tile
    // under replicate or reflect padding) load without masks.
    const int64_t plane = (int64_t)a.H * a.W;
    uint32_t ioff[kRowsFast][kSlotsFast];
    uint32_t vbits = 0;
#pragma unroll
    for (int j = 0; j < kSlotsFast; ++j) {
      const int pc = lane + 64 * j;
      const int sc = pc < a.Cc ? src_col(pc) : -1;
#pragma unroll
      for (int i = 0; i < kRowsFast; ++i) {
        const int pr = wave + 4 * i;
        const int ch = pr >= a.R ? 1 : 0;
        const int sr = pr < 2 * a.R ? src_row(pr - ch * a.R) : -1;
        const bool ok = sr >= 0 && sc >= 0;
        ioff[i][j] = 2u * (uint32_t)((ok ? sr : 0) * a.W + (ok ? sc : 0));   // bytes
        vbits |= (ok ? 1u : 0u) << (i * kSlotsFast + j);
      }
    }
    const int rlast = a.rstep == TH.q ? r0 + a.R - 1 : r0 + TH.q * (a.th_cells - 1) + 3;
    const int clast = a.cstep == TW.q ? c0 + a.Cc - 1 : c0 + TW.q * (a.tw_cells - 1) + a.wspan - 1;
    const bool masked = a.pad == FCFS_PAD_ZERO && (r0 < 0 || rlast >= a.H || c0 < 0 || clast >= a.W);

    uint32_t pre[kRowsFast][kSlotsFast];
    uint4 wpre[kWItems];
    // loads of a step: raw values; the masks apply when they are stored
    auto load_step = [&](int cc) {
      const uint16_t* b0 = xin + (int64_t)cc * plane;
      const uint16_t* b1 = cc + 1 < a.Cin ? b0 + plane : b0;
#pragma unroll
      for (int i = 0; i < kRowsFast; ++i) {
        const char* b = reinterpret_cast<const char*>(wave + 4 * i >= a.R ? b1 : b0);
#pragma unroll
        for (int j = 0; j < kSlotsFast; ++j) pre[i][j] = *reinterpret_cast<const uint16_t*>(b + ioff[i][j]);
      }
#pragma unroll
      for (int k = 0; k < kWItems; ++k) wpre[k] = load_w(k, cc);
    };
    auto store_step = [&](uint16_t* patch, int cc, bool mask) {
      const uint32_t m1 = cc + 1 < a.Cin ? 0xffffu : 0u;   // the step's second channel may be past C_in
#pragma unroll
      for (int i = 0; i < kRowsFast; ++i) {
        const int pr = wave + 4 * i;
        if (pr >= 2 * a.R) break;
#pragma unroll
        for (int j = 0; j < kSlotsFast; ++j) {
          uint32_t v = pre[i][j];
          if (pr >= a.R) v &= m1;
          if (mask) v &= ((vbits >> (i * kSlotsFast + j)) & 1u) ? 0xffffu : 0u;
          patch[pr * a.CP + min(lane + 64 * j, a.Cc)] = (uint16_t)v;
        }
      }
      uint16_t* wch = patch + a.woff_u16;
#pragma unroll
      for (int k = 0; k < kWItems; ++k) *reinterpret_cast<uint4*>(wch + wlds[k]) = mask_w(k, cc, wpre[k]);
    };
    auto run = [&](bool mask) {
      load_step(0);
      store_step(lds, 0, mask);
      __syncthreads();
      for (int s = 0; s < nsteps; ++s) {
        uint16_t* cur = lds + (s & 1) * a.buf_u16;
        if (s + 1 < nsteps) load_step(2 * (s + 1));
        __builtin_amdgcn_sched_barrier(0);   // the next step's loads go out before the MFMAs
        compute(cur);
        __builtin_amdgcn_sched_barrier(0);
        if (s + 1 < nsteps) store_step(lds + ((s + 1) & 1) * a.buf_u16, 2 * (s + 1), mask);
        __syncthreads();
      }
    };
    if (masked) run(true);
    else run(false);
  } else {
    for (int s = 0; s < nsteps; ++s) {
      const int cc = 2 * s;
      // every row of the patch, then the weights, straight into the buffer
      for (int pr = wave; pr < 2 * a.R; pr += 4) {
        const int ch = pr >= a.R ? 1 : 0;
        const int sr = src_row(pr - ch * a.R);
        const bool rok = cc + ch < a.Cin && sr >= 0;
        const uint16_t* rowp = xin + ((int64_t)(rok ? cc + ch : 0) * a.H + (rok ? sr : 0)) * a.W;
        for (int pc = lane; pc < a.Cc; pc += 64) {
          const int sc = src_col(pc);
          lds[pr * a.CP + pc] = (rok && sc >= 0) ? rowp[sc] : (uint16_t)0;
        }
      }
      uint16_t* wch = lds + a.woff_u16;
#pragma unroll
      for (int k = 0; k < kWItems; ++k) *reinterpret_cast<uint4*>(wch + wlds[k]) = mask_w(k, cc, load_w(k, cc));
      __syncthreads();
      compute(lds);
      __syncthreads();
    }
  }

  // epilogue: 16 output channels at a time through LDS, whole row segments out
  uint16_t* ob = lds;   // [16][th_cells][tw_cells * P]
  const int segw = a.tw_cells * P;
  uint16_t* yout = reinterpret_cast<uint16_t*>(a.y);
#pragma unroll
  for (int nt = 0; nt < kNT; ++nt) {
#pragma unroll
    for (int ph = 0; ph < G; ++ph) {
      if (ph >= P) break;
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int cell = wave * 32 + mt * 16 + 4 * g4 + i;
          const int lh = cell / a.tw_cells, lw = cell - lh * a.tw_cells;
          ob[(li * a.th_cells + lh) * segw + lw * P + ph] = M::to_store(acc[ph][mt][nt][i]);
        }
    }
    __syncthreads();
    for (int idx = tid; idx < 16 * a.th_cells * segw; idx += kThreads) {
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

template <int DT, int G>
void launch_g(const MixArgs& a, dim3 grid, hipStream_t stream) {
  if (a.nbuf == 2) hipLaunchKernelGGL((mix4_kernel<DT, G, true>), grid, dim3(kThreads), a.lds_bytes, stream, a);
  else hipLaunchKernelGGL((mix4_kernel<DT, G, false>), grid, dim3(kThreads), a.lds_bytes, stream, a);
}

template <int DT, int G>
void launch_cl(const MixArgs& a, dim3 grid, hipStream_t stream);

template <int DT>
fcfs_status launch_mix4_dt(const MixArgs& a, hipStream_t stream) {
  const int64_t blocks = (int64_t)a.N * a.tiles_h * a.tiles_w * a.th.p * a.groups * a.otiles;
  const dim3 grid((unsigned)blocks);
  if (a.cl) {
    switch (a.gsize) {
      case 1: launch_cl<DT, 1>(a, grid, stream); break;
      case 2: launch_cl<DT, 2>(a, grid, stream); break;
      case 3: launch_cl<DT, 3>(a, grid, stream); break;
      case 4: launch_cl<DT, 4>(a, grid, stream); break;
      default: launch_cl<DT, 5>(a, grid, stream); break;
    }
    return hipGetLastError() == hipSuccess ? FCFS_OK : FCFS_E_DEVICE;
  }
  switch (a.gsize) {
    case 1: launch_g<DT, 1>(a, grid, stream); break;
    case 2: launch_g<DT, 2>(a, grid, stream); break;
    case 3: launch_g<DT, 3>(a, grid, stream); break;
    case 4: launch_g<DT, 4>(a, grid, stream); break;
    default: launch_g<DT, 5>(a, grid, stream); break;
  }
  return hipGetLastError() == hipSuccess ? FCFS_OK : FCFS_E_DEVICE;
}

}  // namespace mix
}  // namespace fcfs
