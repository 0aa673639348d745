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

// ---------------------------------------------------------------------------
// Input gradient on MFMA. The adjoint of pad -> strided convolution ->
// pixelshuffle is fold(C^T dy): z = C^T dy is the gradient with respect to the
// padded (extended) input, and the pad adjoint folds z's margins back onto the
// samples they copy (replicate: onto the edge sample; reflect: onto the mirror;
// zero: dropped). z needs no folding logic, so it is a plain implicit GEMM per
// residue class of the extended position e = (q_h u + rh, q_w v + rw):
//   z[n][c][e] = sum over (jh, a) with off_h(jh) + a = rh (mod q_h), over
//   (jw, b) likewise, and over o, of W[jh][jw][o][c][a][b] *
//   dy[n][o][p_h (u - dh) + jh][p_w (v - dw) + jw],  d = (off + tap - r) / q,
// with rows M = extended positions (16 consecutive v of one row and class),
// columns N = input channels and reduction K = (tap pair, o). Two cheap
// passes first lay dy out channel-last (dyc[n][ho][wo][o], o padded to a
// multiple of 32) and the weights as wpk[jh][jw][a][b][c][o] (c padded to a
// multiple of 64), so that every A and B fragment is one aligned 16-byte
// global load (no LDS: each wave streams its own operands, and the caches
// serve the re-reads). z is FP32, [n][c][extended row][rw][v]; the fold pass
// then writes each dx sample once, rounded once to the storage type.
constexpr int kDxgO = 32;    // outputs per MFMA K-step
constexpr int kDxgC = 64;    // channels per wave (4 N tiles)
constexpr int kDxgV = 64;    // positions per wave (4 M tiles of 16 consecutive v)

// dyc[n][ho][wo][o] (o < opad, zero past C_out) from dy[n][o][ho][wo]: a block
// takes 64 output columns of one output row, 64 outputs at a time through LDS.
constexpr int kDxcPitch = 66;   // LDS tile pitch (16-bit units)
__global__ __launch_bounds__(kThreads) void dx_mix_channel_last_kernel(const BwdArgs a) {
  extern __shared__ float smem[];
  uint16_t* const tile = reinterpret_cast<uint16_t*>(smem);   // [64 outputs][kDxcPitch]
  const int wblocks = (a.Wo + 63) / 64;
  int64_t blk = blockIdx.x;
  const int wb = (int)(blk % wblocks); blk /= wblocks;
  const int ho = (int)(blk % a.Ho);
  const int n = (int)(blk / a.Ho);
  const uint16_t* dyb = reinterpret_cast<const uint16_t*>(a.dy);
  uint16_t* out = a.mix_dyc;
  const int64_t oplane = (int64_t)a.Ho * a.Wo;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int o0 = 0; o0 < a.mix_opad; o0 += 64) {
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {   // read: consecutive columns
      const int o = o0 + r, wo = wb * 64 + tx;
      tile[r * kDxcPitch + tx] =
          (o < a.Cout && wo < a.Wo) ? dyb[((int64_t)n * a.Cout + o) * oplane + (int64_t)ho * a.Wo + wo] : 0;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {   // write: consecutive outputs
      const int wo = wb * 64 + r, o = o0 + tx;
      if (wo < a.Wo && o < a.mix_opad) out[(((int64_t)n * a.Ho + ho) * a.Wo + wo) * a.mix_opad + o] = tile[tx * kDxcPitch + r];
    }
  }
}

// wpk[jh][jw][a][b][c][o] (c < cpad, o < opad, zeros past C_in and C_out)
__global__ __launch_bounds__(kThreads) void dx_mix_pack_weights_kernel(const BwdArgs a) {
  const int64_t total = (int64_t)a.th.p * a.tw_tab.p * 16 * a.mix_cpad * a.mix_opad;
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= total) return;
  const int o = (int)(e % a.mix_opad);
  int64_t r = e / a.mix_opad;
  const int c = (int)(r % a.mix_cpad); r /= a.mix_cpad;
  const int tap = (int)(r % 16);
  const int ph = (int)(r / 16);   // jh * p_w + jw
  const uint16_t* wt = reinterpret_cast<const uint16_t*>(a.mix_weight);
  a.mix_wpk[e] = (o < a.Cout && c < a.C) ? wt[(((int64_t)ph * a.Cout + o) * a.C + c) * 16 + tap] : (uint16_t)0;
}

// z for 64 consecutive v of one extended row and width class, 64 channels.
template <int DT>
__global__ __launch_bounds__(kThreads) void dx_mix_gemm_kernel(const BwdArgs a) {
  using M = Mfma<DT>;
  const AxisTable& TH = a.th;
  const AxisTable& TW = a.tw_tab;
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, g4 = lane >> 4;
  int64_t wid = bwd::xcd_block() * 4 + (threadIdx.x >> 6);
  const int ctiles = a.mix_cpad / kDxgC;
  const int ct = (int)(wid % ctiles); wid /= ctiles;
  const int vc = (int)(wid % a.mix_vchunks); wid /= a.mix_vchunks;
  const int rw = (int)(wid % TW.q); wid /= TW.q;
  const int er = (int)(wid % a.mix_eh); wid /= a.mix_eh;
  const int n = (int)wid;
  if (n >= a.planes_n) return;
  const int eh = a.mix_eh0 + er;                       // extended row
  const int rh = fwd::mod_pos(eh, TH.q), uh = (eh - rh) / TH.q;
  const int c0 = ct * kDxgC;
  const int v0 = a.mix_v0 + vc * kDxgV;                // first v of the wave
  const uint16_t* const dyc = a.mix_dyc;
  const uint16_t* const wpk = a.mix_wpk;
  const int64_t rowstride = (int64_t)a.Wo * a.mix_opad;   // dyc row (16-bit units)

  f32x4 acc[4][4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};

  // positions of this lane's A rows (extended column q_w v + rw, v = v0 + 16 mt + li)
  int vv[4];
  bool vin[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    vv[mt] = v0 + 16 * mt + li;
    const int ew = TW.q * vv[mt] + rw;
    vin[mt] = ew >= a.mix_ew0 && ew <= a.mix_ew1;
  }
  const int nsteps = a.mix_opad / kDxgO;
  for (int jh = 0; jh < TH.p; ++jh)
    for (int ta = 0; ta < 4; ++ta) {
      const int dh4 = TH.off[jh] + ta - rh;
      if (fwd::mod_pos(dh4, TH.q) != 0) continue;
      const int mh = uh - dh4 / TH.q;                    // exact division
      if (mh < 0 || mh >= a.Mh) continue;
      const uint16_t* const dyrow = dyc + ((int64_t)n * a.Ho + TH.p * mh + jh) * rowstride;
      for (int jw = 0; jw < TW.p; ++jw)
        for (int tb = 0; tb < 4; ++tb) {
          const int dw4 = TW.off[jw] + tb - rw;
          if (fwd::mod_pos(dw4, TW.q) != 0) continue;
          const int dq = dw4 / TW.q;
          // A rows: dy column p_w (v - dq) + jw, valid for 0 <= v - dq < Mw
          int64_t aoff[4];
          bool aok[4];
#pragma unroll
          for (int mt = 0; mt < 4; ++mt) {
            const int mw = vv[mt] - dq;
            aok[mt] = vin[mt] && mw >= 0 && mw < a.Mw;
            aoff[mt] = aok[mt] ? (int64_t)(TW.p * mw + jw) * a.mix_opad + 8 * g4 : 0;
          }
          const uint16_t* const wrow =
              wpk + ((((int64_t)jh * TW.p + jw) * 16 + ta * 4 + tb) * a.mix_cpad + c0 + li) * a.mix_opad + 8 * g4;
          for (int os = 0; os < nsteps; ++os) {
            u16x8 af[4], bf[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
              const u16x8 v = *reinterpret_cast<const u16x8*>(dyrow + aoff[mt] + kDxgO * os);
              af[mt] = aok[mt] ? v : u16x8{0, 0, 0, 0, 0, 0, 0, 0};
            }
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
              bf[nt] = *reinterpret_cast<const u16x8*>(wrow + (int64_t)16 * nt * a.mix_opad + kDxgO * os);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
              for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = M::mma(af[mt], bf[nt], acc[mt][nt]);
          }
        }
    }
  // z[n][c][er][rw][v - v0_all] (rows of mix_vpitch, a multiple of 4, so the
  // 4 positions of a lane are one aligned 16-byte store): lane (c = c0 +
  // 16 nt + li) holds v = v0 + 16 mt + 4 g4 + i
  const int64_t zrow = (int64_t)TW.q * a.mix_vpitch;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int c = c0 + 16 * nt + li;
    if (c >= a.C) continue;
    float* const zp = a.mix_z + (((int64_t)n * a.C + c) * a.mix_eh + er) * zrow + (int64_t)rw * a.mix_vpitch;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const int vr = v0 + 16 * mt + 4 * g4 - a.mix_v0;
      if (vr < a.mix_vpitch) *reinterpret_cast<f32x4*>(zp + vr) = acc[mt][nt];
    }
  }
}

// dx[n][c][i][j] = sum of z over the extended positions the padding maps to
// (i, j) (itself, and for replicate / reflect the margin positions copying
// it), in a fixed order, rounded once to the storage type.
template <int DT>
__global__ __launch_bounds__(kThreads) void dx_mix_fold_kernel(const BwdArgs a) {
  using S = Store<DT>;
  const AxisTable& TH = a.th;
  const AxisTable& TW = a.tw_tab;
  int64_t blk = blockIdx.x;
  const int cb = (int)(blk % a.col_blocks); blk /= a.col_blocks;
  const int i = (int)(blk % a.H);
  const int64_t pc = blk / a.H;   // n * C + c
  const int j = cb * kThreads + threadIdx.x;
  if (j >= a.W) return;
  const int64_t zrow = (int64_t)TW.q * a.mix_vpitch;
  const float* const zp = a.mix_z + pc * a.mix_eh * zrow;
  auto zat = [&](int eh, int ew) -> float {
    const int rw = fwd::mod_pos(ew, TW.q), v = (ew - rw) / TW.q;
    return zp[(int64_t)(eh - a.mix_eh0) * zrow + (int64_t)rw * a.mix_vpitch + (v - a.mix_v0)];
  };
  // The extended positions that map to (i, j), in ascending order. Only
  // samples within the margins' reach of an edge (or every sample of a short
  // axis, which a reflection may wrap around) can receive folded terms.
  const int lm_w = -a.mix_ew0, rm_w = a.mix_ew1 - (a.W - 1);   // margins beyond the edges
  const int lm_h = -a.mix_eh0, rm_h = a.mix_eh0 + a.mix_eh - a.H;
  const bool zone_w = a.pad != FCFS_PAD_ZERO && (j <= lm_w || j >= a.W - 1 - rm_w || a.W <= lm_w + rm_w + 2);
  const bool zone_h = a.pad != FCFS_PAD_ZERO && (i <= lm_h || i >= a.H - 1 - rm_h || a.H <= lm_h + rm_h + 2);
  float s = 0.f;
  auto add_row = [&](int eh) {
    if (zone_w)
      for (int ew = a.mix_ew0; ew < 0; ++ew)
        if (pad_source(ew, a.W, a.pad) == j) s += zat(eh, ew);
    s += zat(eh, j);
    if (zone_w)
      for (int ew = a.W; ew <= a.mix_ew1; ++ew)
        if (pad_source(ew, a.W, a.pad) == j) s += zat(eh, ew);
  };
  if (zone_h)
    for (int eh = a.mix_eh0; eh < 0; ++eh)
      if (pad_source(eh, a.H, a.pad) == i) add_row(eh);
  add_row(i);
  if (zone_h)
    for (int eh = a.H; eh < a.mix_eh0 + a.mix_eh; ++eh)
      if (pad_source(eh, a.H, a.pad) == i) add_row(eh);
  (void)TH;
  S::store(reinterpret_cast<typename S::T*>(a.dx) + pc * a.H * a.W + (int64_t)i * a.W + j, s);
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
  if (a.dx && a.mix_z) {
    // channel-last dy, packed weights, z on MFMA, then the fold
    const int64_t cl_blocks = (int64_t)a.planes_n * a.Ho * ((a.Wo + 63) / 64);
    hipLaunchKernelGGL(dx_mix_channel_last_kernel, dim3((unsigned)cl_blocks), block,
                       sizeof(uint16_t) * 64 * kDxcPitch, stream, a);
    const int64_t wtotal = (int64_t)a.th.p * a.tw_tab.p * 16 * a.mix_cpad * a.mix_opad;
    hipLaunchKernelGGL(dx_mix_pack_weights_kernel, dim3((unsigned)((wtotal + kThreads - 1) / kThreads)), block, 0,
                       stream, a);
    const int64_t waves = (int64_t)a.planes_n * a.mix_eh * a.tw_tab.q * a.mix_vchunks * (a.mix_cpad / kDxgC);
    hipLaunchKernelGGL((dx_mix_gemm_kernel<DT>), dim3((unsigned)((waves + 3) / 4)), block, 0, stream, a);
    const int64_t fblocks = (int64_t)a.planes_n * a.C * a.H * a.col_blocks;
    hipLaunchKernelGGL((dx_mix_fold_kernel<DT>), dim3((unsigned)fblocks), block, 0, stream, a);
    if (hipGetLastError() != hipSuccess) return FCFS_E_DEVICE;
  } else if (a.dx) {
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
