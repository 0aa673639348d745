// Backward of the channel-mixing FCFS layer (Sec. 7's learnable weights with
// channel mixing) for gfx950, 16-bit storage with FP32 accumulation.
//
// Forward: y[n][o][p*mh + jh][p*mw + jw] = sum over c, a, b of
//   W[jh][jw][o][c][a][b] * ext(x)[n][c][q*mh + off_h(jh) + a][q*mw + off_w(jw) + b].
//
// Input gradient (dx_mix_kernel): the adjoint, gathered per input sample from
// the adjoint tables of bwd_kernel.h (entries (k, j, tap) per input index,
// with the padding folded in):
//   dx[n][c][i][j] = sum over height entries (kh, jh, a), width entries
//   (kw, jw, b) and outputs o of W[jh][jw][o][c][a][b] * dy[n][o][kh][kw].
// A workgroup takes 256 columns of one input row and 32 input channels, one
// column per thread and the 32 channels in registers. The row's height
// entries are the same for every thread, so for each (height entry, chunk of
// 16 outputs) the weights of every width phase and tap are staged in LDS as
// [jw][b][output pair][c] words of two 16-bit weights, and each thread adds,
// for each of its width entries and each output pair, the pair of dy samples
// times 32 weight pairs with v_dot2 (two products into an FP32 accumulator;
// 8 broadcast 16-byte reads). Every sum runs in a fixed order; there are no
// atomics.
//
// Weight gradient (dw_mix_partial_kernel, dw_mix_reduce_kernel): for each
// phase a GEMM over cells, dW[o][(c, a, b)] = sum over cells of
// dy[cell][o] * ext(x)[cell's tap (a, b)][c], on MFMA 16x16x32 with the cells
// as the reduction: a workgroup takes one phase, 32 outputs, 8 input channels
// (128 columns (c, a, b)) and a chunk of cell rows; each wave stages its own
// cell rows (no barriers), 32 cells at a time, as [o][cell] and
// [(c, a, b)][cell] in LDS so that both fragments are 16-byte reads, and
// accumulates 2 x 8 tiles. The waves' tiles are added in a fixed order, and
// the chunks in a second kernel, in order.
#pragma once

#include <hip/hip_runtime.h>

#include "bwd_kernel.h"
#include "fcfs_internal.h"
#include "fwd_kernel.h"
#include "mix4_kernel.h"

namespace fcfs {
namespace bwdmix {

using fwd::pad_source;
using fwd::Store;
using mix::f32x4;
using mix::Mfma;
using mix::u16x8;

constexpr int kThreads = 256;
constexpr int kDxChannels = 32;   // input channels per input-gradient workgroup
constexpr int kDxPairs = 8;       // output pairs (16 outputs) per staged weight slice
// One (jw, b) block of the slice is kDxPairs x kDxChannels words (two 16-bit
// weights of consecutive outputs each, 1 KB); blocks sit 1 KB + 16 B apart,
// so that the lanes of a half-wave, which read from up to p_w * 4 blocks, hit
// different LDS banks.
constexpr int kDxBlock = kDxPairs * kDxChannels + 4;

// v_dot2 (two 16-bit products added to an FP32 accumulator) for each storage type
template <int DT> struct Dot2;
template <> struct Dot2<FCFS_BF16> {
  typedef __bf16 v2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ float dot(uint32_t a, uint32_t b, float c) {
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(v2, a), __builtin_bit_cast(v2, b), c, false);
  }
};
template <> struct Dot2<FCFS_F16> {
  typedef _Float16 v2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ float dot(uint32_t a, uint32_t b, float c) {
    return __builtin_amdgcn_fdot2(__builtin_bit_cast(v2, a), __builtin_bit_cast(v2, b), c, false);
  }
};

template <int DT>
__global__ __launch_bounds__(kThreads) void dx_mix_kernel(const BwdArgs a) {
  using S = Store<DT>;
  using TS = typename S::T;
  using D2 = Dot2<DT>;
  extern __shared__ float smem[];   // p_w * 4 blocks of kDxBlock words: [pair][c]
  uint32_t* const wl = reinterpret_cast<uint32_t*>(smem);
  const AxisTable& TW = a.tw_tab;
  int64_t blk = bwd::xcd_block();
  const int cblk = (int)(blk % a.mix_cblocks); blk /= a.mix_cblocks;
  const int colb = (int)(blk % a.col_blocks); blk /= a.col_blocks;
  const int i = (int)(blk % a.H);
  const int n = (int)(blk / a.H);
  const int c0 = cblk * kDxChannels;
  const int j = colb * kThreads + threadIdx.x;
  const bool live = j < a.W;
  const int* rh = a.tab_h + (int64_t)i * (3 + a.cmax_h);
  const int* rw = a.tab_w + (live ? j : 0);   // field f at f * W
  const int nh = rh[0], nw = live ? rw[0] : 0;
  const uint16_t* wt = reinterpret_cast<const uint16_t*>(a.mix_weight);
  const uint16_t* dyn = reinterpret_cast<const uint16_t*>(a.dy) + (int64_t)n * a.Cout * a.Ho * a.Wo;
  const int64_t oplane = (int64_t)a.Ho * a.Wo;
  float acc[kDxChannels];
#pragma unroll
  for (int c = 0; c < kDxChannels; ++c) acc[c] = 0.f;

  for (int o0 = 0; o0 < a.Cout; o0 += 2 * kDxPairs) {
    for (int eh = 0; eh < nh; ++eh) {
      const int ent = rh[3 + eh];
      const int kh = ent >> 7, jh = (ent >> 2) & 31, ta = ent & 3;
      __syncthreads();   // the previous slice is consumed
      // stage W[jh][jw][o][c0 + c][ta][0..3] for o = o0 + 2 pr, + 1: words
      // (W[o], W[o + 1]) per (jw, b, pr, c); missing outputs and channels are 0
      for (int it = threadIdx.x; it < TW.p * kDxPairs * kDxChannels; it += kThreads) {
        const int c = it % kDxChannels, pr = (it / kDxChannels) % kDxPairs, jw = it / (kDxChannels * kDxPairs);
        uint2 r[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int o = o0 + 2 * pr + h;
          r[h] = make_uint2(0u, 0u);
          if (o < a.Cout && c0 + c < a.C)   // 4 taps, 8-byte aligned
            r[h] = *reinterpret_cast<const uint2*>(wt + ((((int64_t)jh * TW.p + jw) * a.Cout + o) * a.C + c0 + c) * 16 + ta * 4);
        }
        uint32_t* dst = wl + (jw * 4) * kDxBlock + pr * kDxChannels + c;
        dst[0 * kDxBlock] = __builtin_amdgcn_perm(r[1].x, r[0].x, 0x05040100u);
        dst[1 * kDxBlock] = __builtin_amdgcn_perm(r[1].x, r[0].x, 0x07060302u);
        dst[2 * kDxBlock] = __builtin_amdgcn_perm(r[1].y, r[0].y, 0x05040100u);
        dst[3 * kDxBlock] = __builtin_amdgcn_perm(r[1].y, r[0].y, 0x07060302u);
      }
      __syncthreads();
      const uint16_t* dyr = dyn + (int64_t)o0 * oplane + (int64_t)kh * a.Wo;
      for (int ew = 0; ew < nw; ++ew) {
        const int went = rw[(int64_t)(3 + ew) * a.W];
        const int kw = went >> 7, jw = (went >> 2) & 31, tb = went & 3;
        const uint32_t* ws = wl + (jw * 4 + tb) * kDxBlock;
        uint32_t dv[kDxPairs];   // (dy[o], dy[o + 1]) as one word; missing outputs read as 0
#pragma unroll
        for (int pr = 0; pr < kDxPairs; ++pr) {
          const int o = o0 + 2 * pr;
          const uint32_t lo = o < a.Cout ? dyr[(int64_t)(2 * pr) * oplane + kw] : 0u;
          const uint32_t hi = o + 1 < a.Cout ? dyr[(int64_t)(2 * pr + 1) * oplane + kw] : 0u;
          dv[pr] = lo | (hi << 16);
        }
#pragma unroll
        for (int pr = 0; pr < kDxPairs; ++pr) {
          const uint4* w4 = reinterpret_cast<const uint4*>(ws + pr * kDxChannels);
#pragma unroll
          for (int q4 = 0; q4 < kDxChannels / 4; ++q4) {
            const uint4 w = w4[q4];
            acc[4 * q4 + 0] = D2::dot(w.x, dv[pr], acc[4 * q4 + 0]);
            acc[4 * q4 + 1] = D2::dot(w.y, dv[pr], acc[4 * q4 + 1]);
            acc[4 * q4 + 2] = D2::dot(w.z, dv[pr], acc[4 * q4 + 2]);
            acc[4 * q4 + 3] = D2::dot(w.w, dv[pr], acc[4 * q4 + 3]);
          }
        }
      }
    }
  }
  if (!live) return;
  TS* dxp = reinterpret_cast<TS*>(a.dx) + ((int64_t)n * a.C * a.H + i) * a.W + j;
#pragma unroll
  for (int c = 0; c < kDxChannels; ++c)
    if (c0 + c < a.C) S::store(dxp + (int64_t)(c0 + c) * a.H * a.W, acc[c]);
}

constexpr int kDwOuts = 32;   // outputs per weight-gradient workgroup (2 M tiles)
constexpr int kDwChan = 8;    // input channels per workgroup: 8 x 16 taps = 128 columns (8 N tiles)
constexpr int kDwCells = 32;  // cells per MFMA reduction step

constexpr int kRawPitch = 136;   // 16-bit samples per staged x row (128 columns and a bank skew)

// Partial sums of one chunk of cell rows: partial[chunk][phase][o][c][16].
// RAW (q <= 4, so the 31 q + 4 columns of a step's 32 cells fit in 128): the
// step's x rows are loaded whole, two adjacent columns per lane (coalesced),
// into LDS rows, and each B fragment gathers its 8 cells from there;
// otherwise each lane loads the samples of its own (cell pair, b) column.
template <int DT, bool RAW>
__global__ __launch_bounds__(kThreads, 2) void dw_mix_partial_kernel(
    const BwdArgs a) {
  using M = Mfma<DT>;
  extern __shared__ float smem[];
  const AxisTable& TH = a.th;
  const AxisTable& TW = a.tw_tab;
  int64_t blk = blockIdx.x;
  const int chunk = (int)(blk % a.mix_kchunks); blk /= a.mix_kchunks;
  const int ctile = (int)(blk % a.mix_ctiles); blk /= a.mix_ctiles;
  const int otile = (int)(blk % a.mix_otiles); blk /= a.mix_otiles;
  const int ph = (int)blk;
  const int jh = ph / TW.p, jw = ph % TW.p;
  const int o0 = otile * kDwOuts, c0 = ctile * kDwChan;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, g4 = lane >> 4;
  // wave-private staging: A [32 o][32 cells], B [128 (c, a, b)][32 cells] (16-bit)
  constexpr int kWaveLds = RAW ? kDwOuts * kDwCells + 4 * kDwChan * kRawPitch : (kDwOuts + 16 * kDwChan) * kDwCells;
  uint16_t* const As = reinterpret_cast<uint16_t*>(smem) + wave * kWaveLds;
  uint16_t* const Bs = As + kDwOuts * kDwCells;   // RAW: the x rows [c][ta][kRawPitch]
  const int G = a.planes_n * a.Mh;   // cell rows (n, mh)
  const int g_lo = (int)((int64_t)G * chunk / a.mix_kchunks);
  const int g_hi = (int)((int64_t)G * (chunk + 1) / a.mix_kchunks);
  // both operands move as raw 16-bit samples
  const uint16_t* dyb = reinterpret_cast<const uint16_t*>(a.dy);
  const uint16_t* xb = reinterpret_cast<const uint16_t*>(a.x);
  const int64_t oplane = (int64_t)a.Ho * a.Wo, iplane = (int64_t)a.H * a.W;

  f32x4 acc[2][8];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};

  // A staging: lane -> cells 2 k2, 2 k2 + 1 and outputs (lane >> 4) + 4 t, t < 8.
  // B staging: lane -> the same cells and columns (c, ta, tb) = (t >> 2,
  // t & 3, lane >> 4), t < 32 (16-bit samples in 32-bit registers, packed in
  // pairs of cells when stored).
  const int k2 = lane & 15, hi = lane >> 4;
  const int tb = hi;
  uint32_t pa[8][2], pb[32][2];
  // the K steps of this wave: (cell row g, 32 cells from mw0)
  const int nks = (a.Mw + kDwCells - 1) / kDwCells;
  // Loads are unconditional, from clamped (valid) addresses; their masks are
  // kept and applied when the step is stored, so nothing waits on a load
  // before the step's MFMAs. Row bases of x are the same for the whole wave.
  bool okA[2], okB[2];
  uint32_t rowmask = 0;   // bit ta: tap row ta of this step is not zero padding
  auto load_step = [&](int g, int mw0) __attribute__((always_inline)) {
    const int n = g / a.Mh, mh = g % a.Mh;
    const int orow = TH.p * mh + jh;
    int colA[2], colB[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int mw = mw0 + 2 * k2 + e;
      const bool kok = mw < a.Mw;
      colA[e] = TW.p * (kok ? mw : 0) + jw;
      okA[e] = kok;
      const int sc = pad_source(TW.q * (kok ? mw : 0) + TW.off[jw] + tb, a.W, a.pad);
      colB[e] = sc >= 0 ? sc : 0;
      okB[e] = kok && sc >= 0;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int o = hi + 4 * t;
      const uint16_t* row = dyb + ((int64_t)n * a.Cout + min(o0 + o, a.Cout - 1)) * oplane + (int64_t)orow * a.Wo;
#pragma unroll
      for (int e = 0; e < 2; ++e) pa[t][e] = row[colA[e]];
    }
    rowmask = 0;
    if constexpr (RAW) {
      // columns cb + 2 lane + e of the step's segment (cb = q mw0 + off_w(jw));
      // past the step's last tap, or in zero padding, they are masked
      const int cb = TW.q * mw0 + TW.off[jw];
      const int used = TW.q * (min(kDwCells, a.Mw - mw0) - 1) + 4;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int sc = pad_source(cb + 2 * lane + e, a.W, a.pad);
        colB[e] = sc >= 0 ? sc : 0;
        okB[e] = sc >= 0 && 2 * lane + e < used;
      }
    }
#pragma unroll
    for (int ta = 0; ta < 4; ++ta) {
      const int sr = pad_source(TH.q * mh + TH.off[jh] + ta, a.H, a.pad);
      rowmask |= (sr >= 0 ? 1u : 0u) << ta;
#pragma unroll
      for (int c = 0; c < kDwChan; ++c) {
        const uint16_t* row = xb + ((int64_t)n * a.C + min(c0 + c, a.C - 1)) * iplane + (int64_t)(sr >= 0 ? sr : 0) * a.W;
#pragma unroll
        for (int e = 0; e < 2; ++e) pb[c * 4 + ta][e] = row[colB[e]];
      }
    }
  };
  auto store_step = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const bool ook = o0 + hi + 4 * t < a.Cout;
      const uint32_t lo = (ook && okA[0]) ? pa[t][0] : 0u, hi16 = (ook && okA[1]) ? pa[t][1] : 0u;
      *reinterpret_cast<uint32_t*>(As + (hi + 4 * t) * kDwCells + 2 * k2) = lo | (hi16 << 16);
    }
#pragma unroll
    for (int t = 0; t < 32; ++t) {
      const int c = t >> 2, ta = t & 3;
      const bool cok = ((rowmask >> ta) & 1u) && c0 + c < a.C;
      const uint32_t lo = (cok && okB[0]) ? pb[t][0] : 0u, hi16 = (cok && okB[1]) ? pb[t][1] : 0u;
      if constexpr (RAW) {
        *reinterpret_cast<uint32_t*>(Bs + t * kRawPitch + 2 * lane) = lo | (hi16 << 16);
      } else {
        const int col = c * 16 + ta * 4 + tb;
        *reinterpret_cast<uint32_t*>(Bs + col * kDwCells + 2 * k2) = lo | (hi16 << 16);
      }
    }
  };
  // this wave's steps: cell rows g_lo + wave, + 4, ...; 32-cell steps within each
  const int rows_w = g_hi - g_lo > wave ? (g_hi - g_lo - wave + 3) / 4 : 0;
  const int nsteps = rows_w * nks;
  if (nsteps > 0) load_step(g_lo + wave, 0);
  for (int s = 0; s < nsteps; ++s) {
    store_step();
    fwd::wave_lds_sync();
    if (s + 1 < nsteps) {
      const int s1 = s + 1;
      load_step(g_lo + wave + 4 * (s1 / nks), (s1 % nks) * kDwCells);
    }
    u16x8 af[2], bf[8];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) af[mt] = *reinterpret_cast<const u16x8*>(As + (mt * 16 + li) * kDwCells + 8 * g4);
    if constexpr (RAW) {
      // column (c, ta, tb) = (nt, li >> 2, li & 3): cells 8 g4 + i sit at
      // q (8 g4 + i) + tb of x row (c, ta); each fragment is gathered just
      // before its two MFMAs (the next one's reads are issued first)
      auto gather = [&](int nt) __attribute__((always_inline)) {
        const uint16_t* xr = Bs + (nt * 4 + (li >> 2)) * kRawPitch + TW.q * 8 * g4 + (li & 3);
        u16x8 f;
#pragma unroll
        for (int i = 0; i < 8; ++i) f[i] = xr[TW.q * i];
        return f;
      };
      bf[0] = gather(0);
#pragma unroll
      for (int nt = 0; nt < 8; ++nt) {
        if (nt + 1 < 8) bf[nt + 1] = gather(nt + 1);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) acc[mt][nt] = M::mma(af[mt], bf[nt], acc[mt][nt]);
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
#pragma unroll
      for (int nt = 0; nt < 8; ++nt) bf[nt] = *reinterpret_cast<const u16x8*>(Bs + (nt * 16 + li) * kDwCells + 8 * g4);
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 8; ++nt) acc[mt][nt] = M::mma(af[mt], bf[nt], acc[mt][nt]);
    }
    fwd::wave_lds_sync();
  }
  // add the 4 waves' tiles in order (wave 0 first) through LDS, then write
  // partial[chunk][ph][o][c][tap]
  __syncthreads();
  float* red = smem;   // [4 waves][32 o][128 cols]
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < 8; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = mt * 16 + 4 * g4 + r, col = nt * 16 + li;   // D: col l%16, rows 4(l/16)+r
        red[(wave * kDwOuts + o) * 128 + col] = acc[mt][nt][r];
      }
  __syncthreads();
  float* out = a.partial + (((int64_t)chunk * TH.p * TW.p + ph) * a.Cout) * a.C * 16;
  for (int e = threadIdx.x; e < kDwOuts * 128; e += kThreads) {
    const int o = e / 128, col = e % 128, c = col >> 4, tap = col & 15;
    if (o0 + o >= a.Cout || c0 + c >= a.C) continue;
    float s = red[o * 128 + col];
    for (int w = 1; w < 4; ++w) s += red[(w * kDwOuts + o) * 128 + col];
    out[((int64_t)(o0 + o) * a.C + c0 + c) * 16 + tap] = s;
  }
}

// dw[ph][o][c][tap] = sum of the chunks' partials, in chunk order.
__global__ __launch_bounds__(kThreads) void dw_mix_reduce_kernel(const BwdArgs a) {
  const int64_t per = (int64_t)a.th.p * a.tw_tab.p * a.Cout * a.C * 16;
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= per) return;
  float s = 0.f;
  for (int k = 0; k < a.mix_kchunks; ++k) s += a.partial[k * per + e];
  a.dw[e] = s;
}

template <int DT>
fcfs_status launch_backward_mix_dt(const BwdArgs& a, hipStream_t stream) {
  const dim3 block(kThreads);
  hipLaunchKernelGGL((bwd::adjoint_tables_kernel<DT>), dim3((unsigned)(((int64_t)a.H + a.W + kThreads - 1) / kThreads)),
                     block, 0, stream, a);
  if (hipGetLastError() != hipSuccess) return FCFS_E_DEVICE;
  if (a.dx) {
    const int64_t blocks = (int64_t)a.planes_n * a.H * a.col_blocks * a.mix_cblocks;
    const size_t lds = sizeof(uint32_t) * a.tw_tab.p * 4 * kDxBlock;
    hipLaunchKernelGGL((dx_mix_kernel<DT>), dim3((unsigned)blocks), block, lds, stream, a);
    if (hipGetLastError() != hipSuccess) return FCFS_E_DEVICE;
  }
  if (a.dw) {
    const int64_t blocks = (int64_t)a.th.p * a.tw_tab.p * a.mix_otiles * a.mix_ctiles * a.mix_kchunks;
    const size_t lds = sizeof(float) * 4 * kDwOuts * 128;   // >= the staging (4 x 11 KB)
    if (a.tw_tab.q <= 4) hipLaunchKernelGGL((dw_mix_partial_kernel<DT, true>), dim3((unsigned)blocks), block, lds, stream, a);
    else hipLaunchKernelGGL((dw_mix_partial_kernel<DT, false>), dim3((unsigned)blocks), block, lds, stream, a);
    if (hipGetLastError() != hipSuccess) return FCFS_E_DEVICE;
    const int64_t per = (int64_t)a.th.p * a.tw_tab.p * a.Cout * a.C * 16;
    hipLaunchKernelGGL((dw_mix_reduce_kernel), dim3((unsigned)((per + kThreads - 1) / kThreads)), block, 0, stream, a);
    if (hipGetLastError() != hipSuccess) return FCFS_E_DEVICE;
  }
  return FCFS_OK;
}

}  // namespace bwdmix
}  // namespace fcfs
