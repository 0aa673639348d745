// Channel-mixing FCFS layer on MFMA with a channel-last staged patch (gfx950).
//
// Same contraction as mix4_kernel.h (per phase (jh, jw): rows = cells,
// columns = output channels, reduction = (input channel, tap row a, tap
// column b)), with the reduction ordered so that both MFMA operands are one
// aligned 16-byte LDS read per lane:
//   K step (a, 8 input channels): k = 8*b + i  <->  tap column b, channel i.
// The input patch of a stage (8 input channels) is stored channel-last,
// [row][pixel][8 channels], so the A fragment of a cell for tap (a, b) is the
// pixel at (4*lh + a, cstep*lw + b + phase offset): 16 bytes. The weights of
// the stage are stored [phase][a][output][b][8 channels], so a B fragment is
// 16 bytes too.
//
// Workgroup: 4 waves, 4 x 32 cells (wave w: cell row w, two M tiles of 16
// cells), kOut = 32 outputs (two N tiles), a group of G width phases, which
// share the patch. Stages of 8 input channels go through two LDS buffers: the
// next stage's loads (dword pairs of adjacent columns, or single samples near
// padded borders) are issued before the stage's MFMAs and stored after them.
//
// The patch rows are the 4 tap rows of each of the 4 cell rows (16 rows), the
// columns a contiguous range (q <= span of a cell's taps) or, for large q, only
// the tapped columns of each cell.
#pragma once

#include <hip/hip_runtime.h>

#include "fcfs_internal.h"
#include "fwd_kernel.h"
#include "mix4_kernel.h"

namespace fcfs {
namespace mix {

constexpr int kClCh = 8;       // input channels per stage
constexpr int kClRows = 4;     // patch rows per wave (16 = 4 cell rows x 4 tap rows)
constexpr int kClPairs = 2;    // 128-column slots of column pairs per lane (fast staging)
constexpr int kClSlots = 3;    // 64-column slots per lane (sample-by-sample staging)

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// Fourth word of a raw buffer resource on gfx9-family parts (32-bit data
// format; reads past the record count return zero).
constexpr int kBufferWord3 = 0x00020000;

// The fixed schedule for G phases with tap columns at offsets 0..G-1: blocks
// (d, phase) for d = 0..G+2 and phase = max(0, d-3)..min(G-1, d), in order.
template <int G>
constexpr int fixed_block_d(int i) {
  for (int d = 0; d < G + 3; ++d) {
    const int lo = d > 3 ? d - 3 : 0, hi = d < G - 1 ? d : G - 1;
    if (i <= hi - lo) return d;
    i -= hi - lo + 1;
  }
  return 0;
}
template <int G>
constexpr int fixed_block_ph(int i) {
  for (int d = 0; d < G + 3; ++d) {
    const int lo = d > 3 ? d - 3 : 0, hi = d < G - 1 ? d : G - 1;
    if (i <= hi - lo) return lo + i;
    i -= hi - lo + 1;
  }
  return 0;
}
template <int G>
constexpr bool fixed_block_first(int i) {
  return i == 0 || fixed_block_d<G>(i) != fixed_block_d<G>(i - 1);
}

// MODE bit 0: the fixed schedule (every phase group has consecutive tap
// column offsets); bit 1: pair staging (contiguous patch columns, rows of
// aligned pairs). Each mode is its own kernel, so each gets its own register
// allocation.
template <int DT, int G, int MODE>
__global__ __launch_bounds__(kThreads, 2) void mix4_cl_kernel(const MixArgs a) {
  constexpr bool FIXED = (MODE & 1) != 0;
  constexpr bool PAIRS = (MODE & 2) != 0;
  using M = Mfma<DT>;
  extern __shared__ float smem[];
  uint16_t* const lds = reinterpret_cast<uint16_t*>(smem);
  const AxisTable& TH = a.th;
  const AxisTable& TW = a.tw_tab;

  // Block b runs on XCD b % 8; renumbering gives each XCD a contiguous range
  // of blocks, so the output tiles and phases that share a patch (and the
  // weights they cycle through) meet in one L2.
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

  const int mh0 = trow * 4, mw0 = tcol * 32;
  const int jw0 = group * G;
  const int P = min(G, TW.p - jw0);
  const int o0 = otile * kOut;
  const int r0 = TH.q * mh0 + TH.off[jh];
  const int cbase = TW.off[jw0];
  const int c0 = TW.q * mw0 + cbase;
  const bool contiguous = a.cstep == TW.q;
  const int cs = contiguous ? (c0 & ~1) : c0;   // input column of patch pixel 0 (even when contiguous)
  const int sh = c0 - cs;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g4 = lane >> 4;
  const int li = lane & 15;
  const int CPX = a.CP;                          // 16-byte slots per patch row (16 mod 32)
  const int S = a.slots;                         // slots per residue class of a row
  const int cstep = a.cstep;
  const int patch_u16 = 16 * CPX * kClCh;        // weights follow
  const int64_t plane = (int64_t)a.H * a.W;
  const uint16_t* xin = reinterpret_cast<const uint16_t*>(a.x) + (int64_t)n * a.Cin * plane;
  const uint16_t* win = reinterpret_cast<const uint16_t*>(a.w);

  auto src_row = [&](int rr) -> int { return fwd::pad_source(r0 + TH.q * (rr >> 2) + (rr & 3), a.H, a.pad); };
  auto src_col = [&](int px) -> int {   // input column of patch pixel px (before padding)
    return contiguous ? cs + px : c0 + TW.q * (px / a.wspan) + px % a.wspan;
  };
  // Slot of patch pixel px in its row: pixels are grouped by px mod cstep, so
  // that the pixels one tap column of 16 consecutive cells reads are 16
  // consecutive slots.
  auto slot_of = [&](int px) -> int { return (px % cstep) * S + px / cstep; };

  // Pair staging applies when the patch columns are contiguous and rows hold
  // whole aligned pairs; pixels whose column lies outside the row are then
  // fixed up from the patch itself.
  const int npx = a.Cc + sh;   // pixels the MFMAs read
  const bool pairs = PAIRS;   // the host chooses it only for contiguous columns and aligned pairs
  const int pad_left = pairs ? max(0, -cs) : 0;
  const int pad_right = pairs ? max(0, cs + npx - a.W) : 0;

  constexpr int kNT = kOut / 16;
  // ---- weights: items it = tid + 256 k: (phase, output, channel pair) =
  // (it / 128, (it / 4) % 32, it % 4); each moves 2 channels x 16 taps
  constexpr int kWItems = (G * kOut * 4 + kThreads - 1) / kThreads;
  int64_t woff[kWItems];
  int wlds[kWItems];
  bool wok[kWItems];     // the quad's phase and output exist (zeros otherwise)
  bool wlive[kWItems];   // the item exists (it < G * 128)
  int wch[kWItems];
#pragma unroll
  for (int k = 0; k < kWItems; ++k) {
    const int it = tid + kThreads * k;
    const int ph = it / (kOut * 4), o = (it >> 2) % kOut, cq = it & 3;
    wlive[k] = it < G * kOut * 4;
    wok[k] = wlive[k] && ph < P && o0 + o < a.Cout;
    wch[k] = 2 * cq;
    woff[k] = wok[k] ? ((((int64_t)jh * TW.p + jw0 + ph) * a.Cout + o0 + o) * a.Cin + 2 * cq) * 16 : 0;
    // u16 offset of (ph, b = 0, o, a = 0, channels 2cq, 2cq+1) in the layout
    // [phase][b][N tile][a][output in the tile][8 channels]: a B fragment is
    // then 64 consecutive 16-byte chunks, one per lane
    wlds[k] = patch_u16 + (((ph * 4 * kNT + o / 16) * 4) * 16 + o % 16) * kClCh + 2 * cq;
  }
  // Two channels' 16 taps (words of two taps each) become 16 words of one tap
  // and the two channels; only the last stage can hold channels past C_in,
  // which it zeroes (a missing output or phase only feeds results that are
  // never stored).
  auto store_w = [&](uint16_t* buf, int cb) {
    const bool tail = cb + kClCh > a.Cin;
#pragma unroll
    for (int k = 0; k < kWItems; ++k) {
      if (!wlive[k]) continue;
      // loaded here, one item at a time (few registers); each of the two
      // channels from its own row only when it exists
      const bool ok0 = wok[k] && cb + wch[k] < a.Cin, ok1 = wok[k] && cb + wch[k] + 1 < a.Cin;
      const uint16_t* src0 = win + (ok0 ? woff[k] + (int64_t)cb * 16 : 0);
      const uint16_t* src1 = win + (ok1 ? woff[k] + (int64_t)cb * 16 + 16 : 0);
      uint4 wv[4];
      wv[0] = *reinterpret_cast<const uint4*>(src0);
      wv[1] = *reinterpret_cast<const uint4*>(src0 + 8);
      wv[2] = *reinterpret_cast<const uint4*>(src1);
      wv[3] = *reinterpret_cast<const uint4*>(src1 + 8);
      uint32_t w0[8], w1[8];   // channel 2cq and 2cq + 1: 16 taps each
      __builtin_memcpy(w0, &wv[0], 32);
      __builtin_memcpy(w1, &wv[2], 32);
      if (tail) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          w0[t] = ok0 ? w0[t] : 0u;
          w1[t] = ok1 ? w1[t] : 0u;
        }
      }
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const int ta = t >> 2, tb = t & 3;
        const uint32_t v = __builtin_amdgcn_perm(w1[t >> 1], w0[t >> 1], (t & 1) ? 0x07060302u : 0x05040100u);
        *reinterpret_cast<uint32_t*>(buf + wlds[k] + (tb * kNT * 64 + ta * 16) * kClCh) = v;
      }
    }
  };

  // ---- patch, pair staging: rows rr = wave + 4 i, column pairs
  // cs + 2 lane + 128 j (+1), 8 channels
  uint32_t poff[kClRows][kClPairs];   // byte offset of the pair in a channel plane
#pragma unroll
  for (int i = 0; i < kClRows; ++i) {
    const int sr = src_row(wave + 4 * i);
#pragma unroll
    for (int j = 0; j < kClPairs; ++j) {
      const int c = min(max(cs + 2 * lane + 128 * j, 0), a.W - 2);   // clamped into the row
      // a zero-padding row, or a pair past the patch, takes a lane offset
      // past the buffer's range, for which the load returns zero without a
      // memory access
      poff[i][j] = (sr >= 0 && 2 * lane + 128 * j < npx) ? 2u * (uint32_t)(sr * a.W + c) : 0x7ffffffcu;
    }
  }
  // LDS pixel of each of the lane's two pixels per slot: pixels past the
  // patch, and pixels of columns outside the row (whose loads were clamped),
  // go to the spare pixel
  int pdst[kClPairs][2];
#pragma unroll
  for (int j = 0; j < kClPairs; ++j)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int px = 2 * lane + 128 * j + e;
      pdst[j][e] = (px < npx && cs + px >= 0 && cs + px < a.W) ? slot_of(px) : CPX - 1;
    }
  uint32_t pre[kClRows][kClPairs][kClCh];
  // The image's input as a raw buffer (the host keeps it under 2^31 bytes):
  // each load is the lane's offset in a plane plus the channel's offset as a
  // scalar, with no per-load address arithmetic.
  const __amdgpu_buffer_rsrc_t xrs =
      __builtin_amdgcn_make_buffer_rsrc((void*)xin, 0, (int)(2 * plane * a.Cin), kBufferWord3);
  auto load_patch = [&](int cb) {
#pragma unroll
    for (int ch = 0; ch < kClCh; ++ch) {
      // the scalar offset stays inside the tensor: the range check of a raw
      // buffer covers the lane offset, not necessarily the scalar one
      const int soff = 2 * (int)plane * min(cb + ch, a.Cin - 1);
#pragma unroll
      for (int i = 0; i < kClRows; ++i)
#pragma unroll
        for (int j = 0; j < kClPairs; ++j)
          pre[i][j][ch] = __builtin_amdgcn_raw_buffer_load_b32(xrs, (int)poff[i][j], soff, 0);
    }
  };
  auto store_patch = [&](uint16_t* buf, int cb) {
    // zero-padding rows came back as zeros; channels past C_in (last stage
    // only) are zeroed here
    if (cb + kClCh > a.Cin) {
#pragma unroll
      for (int ch = 0; ch < kClCh; ++ch)
        if (cb + ch >= a.Cin)
#pragma unroll
          for (int i = 0; i < kClRows; ++i)
#pragma unroll
            for (int j = 0; j < kClPairs; ++j) pre[i][j][ch] = 0u;
    }
#pragma unroll
    for (int i = 0; i < kClRows; ++i) {
#pragma unroll
      for (int j = 0; j < kClPairs; ++j) {
        const uint32_t* v = pre[i][j];
        u32x4 p0, p1;   // pixel 2 lane + 128 j (low halves) and the next (high halves)
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          p0[h] = __builtin_amdgcn_perm(v[2 * h + 1], v[2 * h], 0x05040100u);
          p1[h] = __builtin_amdgcn_perm(v[2 * h + 1], v[2 * h], 0x07060302u);
        }
        const int rr = wave + 4 * i;
        *reinterpret_cast<u32x4*>(buf + (rr * CPX + pdst[j][0]) * kClCh) = p0;
        *reinterpret_cast<u32x4*>(buf + (rr * CPX + pdst[j][1]) * kClCh) = p1;
      }
    }
  };
  // pixels of columns outside the row (pair staging near a border): the
  // samples the padding maps them to, fetched one by one, or zero
  auto fix_pad = [&](uint16_t* buf, int cb) {
    const int npad = pad_left + pad_right;
    for (int it = tid; it < 16 * npad; it += kThreads) {
      const int rr = it / npad, s = it - rr * npad;
      const int px = s < pad_left ? s : a.W - cs + (s - pad_left);
      const int sr = src_row(rr);
      const int sc = fwd::pad_source(cs + px, a.W, a.pad);
      uint32_t v[kClCh];
#pragma unroll
      for (int ch = 0; ch < kClCh; ++ch)
        v[ch] = (sr >= 0 && sc >= 0 && cb + ch < a.Cin) ? xin[(cb + ch) * plane + (int64_t)sr * a.W + sc] : 0u;
      u32x4 p;
#pragma unroll
      for (int h = 0; h < 4; ++h) p[h] = v[2 * h] | (v[2 * h + 1] << 16);
      *reinterpret_cast<u32x4*>(buf + (rr * CPX + slot_of(px)) * kClCh) = p;
    }
  };
  // sample-by-sample staging (large q, or rows without aligned pairs)
  auto stage_samples = [&](uint16_t* buf, int cb) {
    for (int i = 0; i < kClRows; ++i) {
      const int rr = wave + 4 * i;
      const int sr = src_row(rr);
      for (int j = 0; j < kClSlots; ++j) {
        const int px = lane + 64 * j;
        if (px >= npx) continue;
        const int sc = fwd::pad_source(src_col(px), a.W, a.pad);
        uint32_t v[kClCh];
#pragma unroll
        for (int ch = 0; ch < kClCh; ++ch)
          v[ch] = (sr >= 0 && sc >= 0 && cb + ch < a.Cin) ? xin[(cb + ch) * plane + (int64_t)sr * a.W + sc] : 0u;
        u32x4 p;
#pragma unroll
        for (int h = 0; h < 4; ++h) p[h] = v[2 * h] | (v[2 * h + 1] << 16);
        *reinterpret_cast<u32x4*>(buf + (rr * CPX + slot_of(px)) * kClCh) = p;
      }
    }
  };

  // ---- fragments. K step (tap column b, 8 input channels): k = 8 a + i
  // <-> tap row a, channel i. Lane (li, g4) of an A fragment reads patch row
  // 4 wave + g4 at the cell's pixel for column offset d = dcol(phase) + b,
  // which depends on the phase only through d: one A fragment per d serves
  // every (phase, b) with that d. B fragments are 64 consecutive chunks.
  const int abase = ((4 * wave + g4) * CPX + li) * kClCh;
  int dcol[G];   // tap column offset of each phase in the group (0 past P)
#pragma unroll
  for (int ph = 0; ph < G; ++ph) dcol[ph] = ph < P ? TW.off[jw0 + ph] - cbase : 0;
  // Phases whose tap columns start at consecutive offsets (dcol = phase, as
  // for 5/4, 4/3, 3/2 and 2/1) share A fragments: column offset d serves the
  // blocks (phase, d - phase) for phase = max(0, d - 3) .. min(G - 1, d).
  // slot for cell 0 of column offset d (fixed schedule) or of block (phase, b)
  int aslot[FIXED ? G + 3 : 4 * G];
#pragma unroll
  for (int i = 0; i < (FIXED ? G + 3 : 4 * G); ++i) aslot[i] = slot_of(sh + (FIXED ? i : dcol[i / 4] + i % 4));
  f32x4 acc[G][2][kNT];
#pragma unroll
  for (int ph = 0; ph < G; ++ph)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < kNT; ++nt) acc[ph][mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};

  // A stage is 4 G MFMA blocks (phase, b), each 2 x kNT MFMAs, as
  // straight-line code: block i's fragments are requested two blocks ahead
  // into three-slot register rings (scheduling barriers keep that order).
  // Consecutive offsets run the blocks in order of d with one A fragment per
  // d; other groups run them phase by phase with an A fragment per block.
  auto compute = [&](const uint16_t* buf) __attribute__((always_inline)) {
    constexpr int NB = 4 * G;
    u16x8 ar[3][2], br[3][kNT];
    auto load = [&](int i) __attribute__((always_inline)) {
      const int ph = FIXED ? fixed_block_ph<G>(i) : i / 4;
      const int b = FIXED ? fixed_block_d<G>(i) - ph : i % 4;
      if (!FIXED || fixed_block_first<G>(i)) {
        const int ring = FIXED ? fixed_block_d<G>(i) % 3 : i % 3;
        const int slot = aslot[FIXED ? fixed_block_d<G>(i) : i];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
          ar[ring][mt] = *reinterpret_cast<const u16x8*>(buf + abase + (slot + 16 * mt) * kClCh);
      }
#pragma unroll
      for (int nt = 0; nt < kNT; ++nt)
        br[i % 3][nt] = *reinterpret_cast<const u16x8*>(buf + patch_u16 + (((ph * 4 + b) * kNT + nt) * 64 + lane) * kClCh);
    };
    load(0);
    load(1);
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      if (i + 2 < NB) load(i + 2);
      __builtin_amdgcn_sched_barrier(0);
      const int ph = FIXED ? fixed_block_ph<G>(i) : i / 4;
      const int ring = FIXED ? fixed_block_d<G>(i) % 3 : i % 3;
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) acc[ph][mt][nt] = M::mma(ar[ring][mt], br[i % 3][nt], acc[ph][mt][nt]);
      __builtin_amdgcn_sched_barrier(0);
    }
  };

  const int nst = (a.Cin + kClCh - 1) / kClCh;
  // One LDS buffer per stage. Pairs: the next stage's patch loads are issued
  // before this stage's MFMAs and land after every wave is done with the
  // stage (another workgroup on the compute unit keeps the matrix cores busy
  // meanwhile). Samples: each stage is staged, then used.
  uint16_t* const buf = lds;
  const bool fix = pairs && pad_left + pad_right > 0;
  if (pairs) {
    load_patch(0);
    store_patch(buf, 0);
    store_w(buf, 0);
    if (fix) fix_pad(buf, 0);   // disjoint pixels: no barrier between
    __syncthreads();
  }
  for (int s = 0; s < nst; ++s) {
    if (!pairs) {
      stage_samples(buf, kClCh * s);
      store_w(buf, kClCh * s);
      __syncthreads();
    } else if (s + 1 < nst) {
      load_patch(kClCh * (s + 1));
    }
    __builtin_amdgcn_sched_barrier(0);
    compute(buf);
    __builtin_amdgcn_sched_barrier(0);
    if (pairs && s + 1 < nst) {
      __syncthreads();
      store_patch(buf, kClCh * (s + 1));
      store_w(buf, kClCh * (s + 1));
      if (fix) fix_pad(buf, kClCh * (s + 1));
    }
    __syncthreads();
  }

  // epilogue: each wave holds cell row mh0 + wave of every output and phase;
  // 16 outputs at a time go through the wave's own LDS rows ([output][lw, ph])
  // and leave as whole row segments of 32 P samples
  const int segw = 32 * P;
  uint16_t* const ob = lds + wave * (16 * 32 * G);
  int colrel[3];   // output column of slot lane + 64 k, relative to the segment start
  bool colok[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int e = lane + 64 * k;
    const int lw = e / P, ph = e - lw * P;
    colrel[k] = TW.p * lw + ph;
    colok[k] = e < segw && mw0 + lw < a.Mw;
  }
  const int mh = mh0 + wave;
  uint16_t* const yrow = reinterpret_cast<uint16_t*>(a.y) +
                         ((((int64_t)n * a.Cout + o0) * a.Ho + TH.p * mh + jh) * a.Wo + TW.p * mw0 + jw0);
  const int64_t ostride = (int64_t)a.Ho * a.Wo;
#pragma unroll
  for (int nt = 0; nt < kNT; ++nt) {
#pragma unroll
    for (int ph = 0; ph < G; ++ph) {
      if (ph >= P) break;
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          ob[li * segw + (mt * 16 + 4 * g4 + i) * P + ph] = M::to_store(acc[ph][mt][nt][i]);
    }
    fwd::wave_lds_sync();
    if (mh < a.Mh) {
      for (int ol = 0; ol < 16; ++ol) {
        if (o0 + nt * 16 + ol >= a.Cout) break;
        uint16_t* const rp = yrow + (nt * 16 + ol) * ostride;
#pragma unroll
        for (int k = 0; k < 3; ++k)
          if (colok[k]) __builtin_nontemporal_store(ob[ol * segw + lane + 64 * k], rp + colrel[k]);
      }
    }
    fwd::wave_lds_sync();
  }
}

template <int DT, int G>
void launch_cl(const MixArgs& a, dim3 grid, hipStream_t stream) {
  switch ((a.fixed ? 1 : 0) | (a.xpair ? 2 : 0)) {
    case 0: hipLaunchKernelGGL((mix4_cl_kernel<DT, G, 0>), grid, dim3(kThreads), a.lds_bytes, stream, a); break;
    case 1: hipLaunchKernelGGL((mix4_cl_kernel<DT, G, 1>), grid, dim3(kThreads), a.lds_bytes, stream, a); break;
    case 2: hipLaunchKernelGGL((mix4_cl_kernel<DT, G, 2>), grid, dim3(kThreads), a.lds_bytes, stream, a); break;
    default: hipLaunchKernelGGL((mix4_cl_kernel<DT, G, 3>), grid, dim3(kThreads), a.lds_bytes, stream, a); break;
  }
}

}  // namespace mix
}  // namespace fcfs
