// Backward of the channel-mixing FCFS layer (Sec. 7's learnable weights with
// channel mixing) for gfx950, 16-bit storage with FP32 accumulation.
//
// Forward: y[n][o][p*mh + jh][p*mw + jw] = sum over c, a, b of
//   W[jh][jw][o][c][a][b] * ext(x)[n][c][q*mh + off_h(jh) + a][q*mw + off_w(jw) + b].
//
// Input gradient: an implicit GEMM on MFMA per residue class of the padded
// input's positions, the pad adjoint folded at the edges
// (dx_mix_gemm_kernel and its layout passes). Weight gradient: for each phase
// and tap a GEMM over cells on MFMA, partial sums per chunk of cell rows
// added in order (dw_mix_gemm_kernel and its layout passes). Every sum runs
// in a fixed order; there are no atomics.
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
// ---------------------------------------------------------------------------
// Input gradient on MFMA. The adjoint of pad -> strided convolution ->
// pixelshuffle is fold(C^T dy): z = C^T dy is the gradient with respect to the
// padded (extended) input, and the pad adjoint folds z's margins back onto the
// samples they copy (replicate: onto the edge sample; reflect: onto the mirror;
// zero: dropped). z itself is a plain implicit GEMM per residue class of the
// extended position e = (q_h u + rh, q_w v + rw):
//   z[n][c][e] = sum over (jh, a) with off_h(jh) + a = rh + q_h dh, over
//   (jw, b) with off_w(jw) + b = rw + q_w dw, and over o, of
//   W[jh][jw][o][c][a][b] * dy[n][o][p_h (u - dh) + jh][p_w (v - dw) + jw],
// with rows M = extended positions (consecutive v of one row and class),
// columns N = input channels and reduction K = (tap pair, o).
//
// Two cheap passes first lay out dy by width phase and 32 outputs, cells
// contiguous with zero margin cells on both sides (dyc[n][ho][jw][o / 32]
// [cell][o % 32]), and the weights as wpk[jh][jw][a][b][o / 32][o % 32 / 8]
// [c][o % 8]. An A fragment (16 cells x 32 outputs) and a B fragment (32
// outputs x 16 channels) are then each 1 KB of consecutive memory, one
// 16-byte load per lane, and a cell outside the row reads zeros. (A call
// with both gradients gets dyc from the weight gradient's pass over dy.)
//
// A workgroup takes one extended row, kw chunks of 16 mtn consecutive v and
// 64 channels, for every width class (waves take the (class, chunk) slots in
// turn; with q_w = 4 one class each, so the four waves read the same dy
// cells and share them in L1). A wave walks its class's (tap pair, 32
// outputs) steps with the next two steps' fragments in flight during the
// current step's MFMAs. The epilogue interleaves the classes in LDS and writes each dx
// row segment contiguously, rounded once; the samples the pad adjoint folds
// (and the margins) go to the edge buffer in FP32, and a last pass adds each
// sample's preimages there in ascending order and rounds once.
constexpr int kDxgO = 32;    // outputs per MFMA K-step
constexpr int kDxgC = 64;    // channels per workgroup (4 N tiles)

// dyc from dy[n][o][ho][wo]: a block takes mix_clcells cells (all p_w phases, at most
// 256 columns col = cell * p_w + jw, wo = col - dleft * p_w; zeros outside
// the row) of one output row, 64 outputs at a time through an LDS tile
// [column][output]. With W_out even a lane reads an aligned column pair of 8
// outputs (8 dword loads, coalesced over pairs) and writes two 16-byte
// column chunks; then each lane moves 16-byte chunks of 8 outputs, ordered
// so that consecutive lanes write consecutive bytes of dyc.
constexpr int kDxcPitch = 72;   // LDS tile pitch (16-bit units): [kDxcColumns columns][64 outputs + 8]
__global__ __launch_bounds__(kThreads) void dx_mix_channel_last_kernel(const BwdArgs a) {
  extern __shared__ float smem[];
  uint16_t* const tile = reinterpret_cast<uint16_t*>(smem);
  const int pw = a.tw_tab.p;
  const int kcl = a.mix_clcells;   // cells per block
  const int cblocks = (a.mix_dcells + kcl - 1) / kcl;
  int64_t blk = blockIdx.x;
  const int cb = (int)(blk % cblocks); blk /= cblocks;
  const int ho = (int)(blk % a.Ho);
  const int n = (int)(blk / a.Ho);
  const int k0 = cb * kcl;
  const int ncols = kcl * pw;
  const int wlo = k0 * pw - a.mix_dleft * pw;   // dy column of tile column 0
  const uint16_t* const dyb = reinterpret_cast<const uint16_t*>(a.dy) + (int64_t)n * a.Cout * a.Ho * a.Wo + (int64_t)ho * a.Wo;
  const int64_t oplane = (int64_t)a.Ho * a.Wo;
  const int nst = a.mix_opad / kDxgO;
  uint16_t* const orow = a.mix_dyc + ((int64_t)n * a.Ho + ho) * pw * nst * a.mix_dcells * kDxgO;
  const bool pairs = (a.Wo & 1) == 0 && (reinterpret_cast<uintptr_t>(a.dy) & 3) == 0;
  for (int o0 = 0; o0 < a.mix_opad; o0 += 64) {
    __syncthreads();
    if (pairs) {
      // items (pair m, 8 outputs g): pairs cover [wlo, wlo + ncols)
      const int m0 = wlo >> 1;   // floor
      const int npairs = ((wlo + ncols - 1) >> 1) - m0 + 1;
      for (int it = threadIdx.x; it < npairs * 8; it += kThreads) {
        const int m = it % npairs, g = it / npairs;
        const int w0 = 2 * (m0 + m);
        const bool in = w0 >= 0 && w0 < a.Wo;   // W_out even: both columns or neither
        uint32_t v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int o = o0 + 8 * g + i;
          v[i] = (in && o < a.Cout) ? *reinterpret_cast<const uint32_t*>(dyb + (int64_t)o * oplane + w0) : 0u;
        }
        u16x8 lo, hi;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          lo[i] = (uint16_t)(v[i] & 0xffffu);
          hi[i] = (uint16_t)(v[i] >> 16);
        }
        const int c = w0 - wlo;
        if (c >= 0 && c < ncols) *reinterpret_cast<u16x8*>(tile + c * kDxcPitch + 8 * g) = lo;
        if (c + 1 >= 0 && c + 1 < ncols) *reinterpret_cast<u16x8*>(tile + (c + 1) * kDxcPitch + 8 * g) = hi;
      }
    } else {
      for (int it = threadIdx.x; it < 64 * ncols; it += kThreads) {
        const int c = it % ncols, r = it / ncols;
        const int wo = wlo + c, o = o0 + r;
        tile[c * kDxcPitch + r] = (wo >= 0 && wo < a.Wo && o < a.Cout) ? dyb[(int64_t)o * oplane + wo] : 0;
      }
    }
    __syncthreads();
    // chunks (jw, 32 outputs s, cell, 8 outputs g), g fastest
    const int nchunks = pw * 2 * kcl * 4;
    for (int e = threadIdx.x; e < nchunks; e += kThreads) {
      const int g = e & 3, cell = (e >> 2) % kcl, sj = (e >> 2) / kcl;
      const int sl = sj & 1, jw = sj >> 1;
      const int os = o0 / kDxgO + sl;
      if (os >= nst || k0 + cell >= a.mix_dcells) continue;
      *reinterpret_cast<u16x8*>(orow + (((int64_t)jw * nst + os) * a.mix_dcells + k0 + cell) * kDxgO + 8 * g) =
          *reinterpret_cast<const u16x8*>(tile + (cell * pw + jw) * kDxcPitch + sl * kDxgO + 8 * g);
    }
  }
}

// wpk from W[jh][jw][o][c][a][b] (zeros past C_in and C_out)
__global__ __launch_bounds__(kThreads) void dx_mix_pack_weights_kernel(const BwdArgs a) {
  const int64_t total = (int64_t)a.th.p * a.tw_tab.p * 16 * a.mix_cpad * a.mix_opad;
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= total) return;
  const int i = (int)(e % 8);
  int64_t r = e / 8;
  const int c = (int)(r % a.mix_cpad); r /= a.mix_cpad;
  const int og = (int)(r % (a.mix_opad / 8)); r /= a.mix_opad / 8;   // (o / 32, o % 32 / 8)
  const int tap = (int)(r % 16);
  const int ph = (int)(r / 16);   // jh * p_w + jw
  const int o = 8 * og + i;
  const uint16_t* wt = reinterpret_cast<const uint16_t*>(a.mix_weight);
  a.mix_wpk[e] = (o < a.Cout && c < a.C) ? wt[(((int64_t)ph * a.Cout + o) * a.C + c) * 16 + tap] : (uint16_t)0;
}

// Edge buffer index of extended position (eh, ew), which lies in a fold zone
// row (part R: [zone row][ew - q_w v0]) or else a fold zone column (part C:
// [eh - r0][zone column]).
__device__ __forceinline__ int64_t edge_index(const BwdArgs& a, int64_t pc, int eh, int ew) {
  const int ec0 = a.tw_tab.q * a.mix_v0, ecols = a.tw_tab.q * a.mix_vw;
  if (eh < a.mix_top || eh >= a.H - a.mix_bot) {
    const int r = eh < a.mix_top ? eh - a.mix_r0 : (a.mix_top - a.mix_r0) + eh - (a.H - a.mix_bot);
    return (pc * a.mix_rr + r) * ecols + (ew - ec0);
  }
  const int cc = ew < a.mix_cl ? ew - ec0 : (a.mix_cl - ec0) + ew - (a.W - a.mix_cr);
  return (int64_t)a.planes_n * a.C * a.mix_edge_c + (pc * a.mix_rows + (eh - a.mix_r0)) * a.mix_cc + cc;
}

// One extended row, kw chunks of 16 MTN consecutive v, 64 channels, every
// width class. Each wave keeps two steps of fragments in flight (one for
// MTN = 4).
template <int DT, int MTN>
__global__ __launch_bounds__(kThreads, 3) void dx_mix_gemm_kernel(const BwdArgs a) {
  using M = Mfma<DT>;
  using S = Store<DT>;
  using TS = typename S::T;
  extern __shared__ float smem[];
  uint16_t* const otile = reinterpret_cast<uint16_t*>(smem);   // [64 channels][cols] (storage type)
  const AxisTable& TH = a.th;
  const AxisTable& TW = a.tw_tab;
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, g4 = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int64_t blk = bwd::xcd_block();
  const int ctiles = a.mix_cpad / kDxgC;
  const int ct = (int)(blk % ctiles); blk /= ctiles;
  const int vg = (int)(blk % a.mix_vgroups); blk /= a.mix_vgroups;
  const int er = (int)(blk % a.mix_rows); blk /= a.mix_rows;
  const int n = (int)blk;
  if (n >= a.planes_n) return;
  const int eh = a.mix_r0 + er;                        // extended row
  const int rh = fwd::mod_pos(eh, TH.q), uh = (eh - rh) / TH.q;
  const int c0 = ct * kDxgC;
  const int opad = a.mix_opad, nst = opad / kDxgO;
  const int qw = TW.q;
  const int vbase = a.mix_v0 + vg * a.mix_kw * 16 * MTN;   // first v of the workgroup
  const int ncols = qw * a.mix_kw * 16 * MTN;              // extended columns of the workgroup
  const int64_t drow = (int64_t)TW.p * nst * a.mix_dcells * kDxgO;   // dyc row (16-bit units)
  const uint16_t* const dycn = a.mix_dyc + (int64_t)n * a.Ho * drow;
  const bool zero_pad = a.pad == FCFS_PAD_ZERO;
  const bool row_in = eh >= 0 && eh < a.H;
  const bool row_zone = eh < a.mix_top || eh >= a.H - a.mix_bot;
  const int vlim = a.mix_v0 + a.mix_vw;
  const bool lds_epi = a.mix_lds_epi != 0;

  // height entries whose dy row exists
  const int hs = a.mix_hl_start[rh], he = a.mix_hl_start[rh + 1];
  auto h_ok = [&](int k) {
    const int mh = uh - ((a.mix_hl[k] >> 7) - 64);
    return mh >= 0 && mh < a.Mh;
  };
  int hfirst = hs, hcount = 0;
  while (hfirst < he && !h_ok(hfirst)) ++hfirst;
  for (int k = hfirst; k < he; ++k) hcount += h_ok(k) ? 1 : 0;

  for (int slot = wave; slot < qw * a.mix_kw; slot += 4) {
    const int rw = slot % qw, kc = slot / qw;
    const int vb = vbase + kc * 16 * MTN;                // first v of the wave
    if (vb >= vlim) continue;
    const int ws = a.mix_wl_start[rw], we = a.mix_wl_start[rw + 1];
    // lane parts of the fragment offsets: A cell dleft + v (+ step's - dw),
    // outputs 8 g4 ..; B channel c0 + li (+ 16 nt), outputs 8 g4 ..
    uint32_t aoff[MTN];
#pragma unroll
    for (int mt = 0; mt < MTN; ++mt) aoff[mt] = (uint32_t)((a.mix_dleft + vb + 16 * mt + li) * kDxgO + 8 * g4);
    const uint32_t boff = (uint32_t)((g4 * a.mix_cpad + c0 + li) * 8);

    f32x4 acc[MTN][4];
#pragma unroll
    for (int mt = 0; mt < MTN; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};

    // steps (height entry hi, width entry wi, 32 outputs os). The fragment
    // addresses are linear in the three: running pointers, with the height
    // entry's row bases set when hi changes and the width entry's offsets
    // when wi changes (few scalar instructions per step).
    const int steps = hcount * (we - ws) * nst;
    const int64_t osA = (int64_t)a.mix_dcells * kDxgO, osB = (int64_t)4 * a.mix_cpad * 8;
    int hi = hfirst, wi = ws, os = 0;
    const uint16_t *rA = nullptr, *rB = nullptr, *pA = nullptr, *pB = nullptr;
    auto set_h = [&]() {
      const int e = a.mix_hl[hi];
      const int jh = e & 31, ta = (e >> 5) & 3, mh = uh - ((e >> 7) - 64);
      rA = dycn + (int64_t)(TH.p * mh + jh) * drow;
      rB = a.mix_wpk + (int64_t)(jh * TW.p * 16 + ta * 4) * nst * osB;
    };
    auto set_w = [&]() {
      const int e = a.mix_wl[wi];
      const int jw = e & 31, tb = (e >> 5) & 3, dw = (e >> 7) - 64;
      pA = rA + ((int64_t)jw * nst * a.mix_dcells - dw) * kDxgO;
      pB = rB + (int64_t)(jw * 16 + tb) * nst * osB;
    };
    if (steps > 0) {
      set_h();
      set_w();
    }
    auto advance = [&]() {
      if (++os < nst) {
        pA += osA;
        pB += osB;
        return;
      }
      os = 0;
      if (++wi < we) {
        set_w();
        return;
      }
      wi = ws;
      do ++hi;
      while (hi < he && !h_ok(hi));
      if (hi < he) {
        set_h();
        set_w();
      }
    };
    u16x8 af0[MTN], bf0[4], af1[MTN], bf1[4], af2[MTN], bf2[4];
    auto load = [&](u16x8 (&A)[MTN], u16x8 (&B)[4]) __attribute__((always_inline)) {
#pragma unroll
      for (int mt = 0; mt < MTN; ++mt) A[mt] = *reinterpret_cast<const u16x8*>(pA + aoff[mt]);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) B[nt] = *reinterpret_cast<const u16x8*>(pB + boff + 16 * 8 * nt);
      advance();
    };
    auto mma = [&](const u16x8 (&A)[MTN], const u16x8 (&B)[4]) __attribute__((always_inline)) {
#pragma unroll
      for (int mt = 0; mt < MTN; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = M::mma(A[mt], B[nt], acc[mt][nt]);
    };
    if constexpr (MTN <= 3) {
      // three register buffers: steps s + 1 and s + 2 load during step s's MFMAs
      if (steps > 0) load(af0, bf0);
      if (steps > 1) load(af1, bf1);
      int s = 0;
      for (; s + 2 < steps; s += 3) {
        load(af2, bf2);                      // step s + 2
        mma(af0, bf0);                       // step s
        if (s + 3 < steps) load(af0, bf0);   // step s + 3
        mma(af1, bf1);                       // step s + 1
        if (s + 4 < steps) load(af1, bf1);   // step s + 4
        mma(af2, bf2);                       // step s + 2
      }
      if (s < steps) mma(af0, bf0);          // the last one or two steps
      if (s + 1 < steps) mma(af1, bf1);
    } else {
      // two buffers (the registers of a third would spill)
      if (steps > 0) load(af0, bf0);
      for (int s = 0; s + 1 < steps; s += 2) {
        load(af1, bf1);                      // step s + 1
        mma(af0, bf0);                       // step s
        if (s + 2 < steps) load(af0, bf0);   // step s + 2
        mma(af1, bf1);                       // step s + 1
      }
      if (steps & 1) mma(af0, bf0);          // the last step
    }

    // slot epilogue: lane (c = c0 + 16 nt + li) holds v = vb + 16 mt + 4 g4 + i.
    // Fold-zone and margin positions go to the edge buffer; the others are
    // rounded into the LDS row tile (or, without it, stored directly).
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int cl = 16 * nt + li, c = c0 + cl;
      const int64_t pc = (int64_t)n * a.C + c;
#pragma unroll
      for (int mt = 0; mt < MTN; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int v = vb + 16 * mt + 4 * g4 + i;
          const int ew = qw * v + rw;
          const float z = acc[mt][nt][i];
          const bool direct = zero_pad || (!row_zone && ew >= a.mix_cl && ew < a.W - a.mix_cr);
          if (lds_epi) otile[cl * ncols + (ew - qw * vbase)] = Mfma<DT>::to_store(z);
          if (c >= a.C || v >= vlim) continue;
          if (!direct) {
            a.mix_edge[edge_index(a, pc, eh, ew)] = z;
          } else if (!lds_epi && row_in && ew >= 0 && ew < a.W) {
            S::store(reinterpret_cast<TS*>(a.dx) + (pc * a.H + eh) * a.W + ew, z);
          }
        }
    }
  }
  if (!lds_epi || !row_in) return;
  __syncthreads();
  // the row segment [q_w vbase, q_w vbase + ncols) of each channel, 256
  // consecutive columns per pass
  const int e0 = qw * vbase;
  for (int cl = 0; cl < kDxgC; ++cl) {
    const int c = c0 + cl;
    if (c >= a.C) break;
    TS* const dxr = reinterpret_cast<TS*>(a.dx) + (((int64_t)n * a.C + c) * a.H + eh) * a.W;
    for (int k = threadIdx.x; k < ncols; k += kThreads) {
      const int ew = e0 + k;
      if (ew < 0 || ew >= a.W) continue;
      if (!zero_pad && (row_zone || ew < a.mix_cl || ew >= a.W - a.mix_cr)) continue;
      if (ew >= qw * vlim) continue;
      reinterpret_cast<uint16_t*>(dxr)[ew] = otile[cl * ncols + k];
    }
  }
}

// dx at the samples the pad adjoint folds: the sum of z over the extended
// positions the padding maps to (i, j), in ascending order, rounded once.
template <int DT>
__global__ __launch_bounds__(kThreads) void dx_mix_edge_kernel(const BwdArgs a) {
  using S = Store<DT>;
  // blocks (x: 256 zone samples of a plane, y: planes, striding past 65535)
  int t = (int)blockIdx.x * kThreads + threadIdx.x;
  if (t >= a.mix_edge_per) return;
  int i, j;
  const int zr = a.mix_top + a.mix_bot;
  if (t < zr * a.W) {
    const int k = t / a.W;
    j = t - k * a.W;
    i = k < a.mix_top ? k : a.H - a.mix_bot + (k - a.mix_top);
  } else {
    t -= zr * a.W;
    const int zc = a.mix_cl + a.mix_cr;
    const int k = t / zc, m = t - k * zc;
    i = a.mix_top + k;
    j = m < a.mix_cl ? m : a.W - a.mix_cr + (m - a.mix_cl);
  }
  for (int64_t pc = blockIdx.y; pc < (int64_t)a.planes_n * a.C; pc += gridDim.y) {
  float s = 0.f;
  auto add_row = [&](int eh) {
    for (int ew = a.mix_ew0; ew < 0; ++ew)
      if (pad_source(ew, a.W, a.pad) == j) s += a.mix_edge[edge_index(a, pc, eh, ew)];
    s += a.mix_edge[edge_index(a, pc, eh, j)];
    for (int ew = a.W; ew <= a.mix_ew1; ++ew)
      if (pad_source(ew, a.W, a.pad) == j) s += a.mix_edge[edge_index(a, pc, eh, ew)];
  };
  for (int eh = a.mix_eh0; eh < 0; ++eh)
    if (pad_source(eh, a.H, a.pad) == i) add_row(eh);
  add_row(i);
  for (int eh = a.H; eh <= a.mix_eh1; ++eh)
    if (pad_source(eh, a.H, a.pad) == i) add_row(eh);
  S::store(reinterpret_cast<typename S::T*>(a.dx) + (pc * a.H + i) * a.W + j, s);
  }
}

// ---------------------------------------------------------------------------
// Weight gradient on MFMA from two re-laid-out operands. For phase (jh, jw)
// and tap (a, b),
//   dW[jh][jw][o][c][a][b] = sum over cells (n, mh, mw) of
//     dy[n][o][p_h mh + jh][p_w mw + jw] * ext(x)[n][c][q_h mh + off_h(jh) + a][q_w mw + s],
// s = off_w(jw) + b: a GEMM with rows M = outputs, columns N = input
// channels and the cells as the reduction K. Its fragments need 8
// consecutive cells per lane, so two passes first lay out
//   dyw[n][ho][jw][mw / 32][mw % 32 / 8][o][mw % 8]  (dy's cells of one phase), and
//   xa[n][row][s][mw / 32][mw % 32 / 8][c][mw % 8]   (ext(x) at column q_w mw + s,
//                                                     padding resolved, every tap offset s),
// so that a fragment (16 outputs or channels x 32 cells) is four 256-byte
// runs, one 16-byte load per lane. A workgroup takes one phase, one tap row a,
// 64 outputs, 64 channels and a chunk of cell rows; wave b takes tap column b
// (the four waves read the same dy fragments and share them in L1), with the
// next step's fragments in flight during the current step's MFMAs. The
// chunks' partial sums are added in chunk order by a last pass.
constexpr int kDwgT = 64;    // outputs and channels per workgroup tile (4 x 4 MFMA tiles)
constexpr int kDwyPitch = 258;   // LDS pitch (16-bit units) of the dy pass tile: 256 columns + 2

// dyw from dy: a block takes 64 outputs of one output row and dwcells cells
// (all p_w phases: at most 256 columns) through an LDS tile [o][column]. Wave
// w reads rows w, w + 4, ... of the tile (aligned column pairs when W_out is
// even), then lane o gathers 8 cells of one phase from its row (the pitch
// puts the 64 rows on distinct banks) and writes them as 16 bytes.
// DYC: also the input gradient's layout of the same cells (dyc, margins
// aside), so that a call with both gradients reads dy once.
template <bool DYC>
__global__ __launch_bounds__(kThreads) void dw_mix_dy_kernel(const BwdArgs a) {
  extern __shared__ float smem[];
  uint16_t* const tile = reinterpret_cast<uint16_t*>(smem);
  const int pw = a.tw_tab.p;
  const int bc = a.mix_dwcells;                     // cells per block (multiple of 8)
  const int cblocks = (a.mix_ncb * 32 + bc - 1) / bc;
  const int oblocks = a.mix_dwopad / 64;
  int64_t blk = blockIdx.x;
  const int ob = (int)(blk % oblocks); blk /= oblocks;
  const int cbk = (int)(blk % cblocks); blk /= cblocks;
  const int ho = (int)(blk % a.Ho);
  const int n = (int)(blk / a.Ho);
  const int mw0 = cbk * bc, o0 = ob * 64;
  const int ncols = bc * pw;                        // even (bc is)
  const int wo0 = mw0 * pw;                         // even
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint16_t* const dyb = reinterpret_cast<const uint16_t*>(a.dy) + (int64_t)n * a.Cout * a.Ho * a.Wo + (int64_t)ho * a.Wo;
  const int64_t oplane = (int64_t)a.Ho * a.Wo;
  // rows wave + 4 i (16 per wave), all loads of a wave issued before its LDS stores
  if ((a.Wo & 1) == 0 && (reinterpret_cast<uintptr_t>(a.dy) & 3) == 0) {
    uint32_t v[16][2];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int r = wave + 4 * i;
      const bool ok = o0 + r < a.Cout;
      const uint16_t* const src = dyb + (int64_t)(ok ? o0 + r : 0) * oplane;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int wo = wo0 + 2 * (lane + 64 * j);   // W_out even: wo + 1 < W_out when wo < W_out
        v[i][j] = (ok && 2 * (lane + 64 * j) < ncols && wo < a.Wo) ? *reinterpret_cast<const uint32_t*>(src + wo) : 0u;
      }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        if (2 * (lane + 64 * j) < ncols)
          *reinterpret_cast<uint32_t*>(tile + (wave + 4 * i) * kDwyPitch + 2 * (lane + 64 * j)) = v[i][j];
  } else {
    uint16_t v[16][4];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int r = wave + 4 * i;
      const bool ok = o0 + r < a.Cout;
      const uint16_t* const src = dyb + (int64_t)(ok ? o0 + r : 0) * oplane;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int t = lane + 64 * j;
        v[i][j] = (ok && t < ncols && wo0 + t < a.Wo) ? src[wo0 + t] : (uint16_t)0;
      }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (lane + 64 * j < ncols) tile[(wave + 4 * i) * kDwyPitch + lane + 64 * j] = v[i][j];
  }
  __syncthreads();
  const int ng = bc / 8;
  uint16_t* const orow = a.mix_dyw + ((int64_t)n * a.Ho + ho) * pw * a.mix_ncb * 32 * a.mix_dwopad;
  for (int k = wave; k < pw * ng; k += 4) {
    const int jw = k / ng, gb = k - jw * ng;
    const int mw = mw0 + 8 * gb;
    if (mw >= a.mix_ncb * 32) continue;
    u16x8 v;
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = tile[lane * kDwyPitch + pw * (8 * gb + i) + jw];
    *reinterpret_cast<u16x8*>(orow + ((((int64_t)jw * a.mix_ncb + mw / 32) * 4 + (mw % 32) / 8) * a.mix_dwopad + o0 + lane) * 8) = v;
  }
  if constexpr (DYC) {
    // chunks (jw, 32 outputs sl, cell, 8 outputs g), g fastest: dyc[..][jw][os][dleft + mw][32]
    const int nst = a.mix_opad / kDxgO;
    const int cells = min(bc, a.Mw - mw0);
    uint16_t* const crow = a.mix_dyc + ((int64_t)n * a.Ho + ho) * pw * nst * a.mix_dcells * kDxgO;
    for (int e = threadIdx.x; e < pw * 2 * bc * 4; e += kThreads) {
      const int g = e & 3, cell = (e >> 2) % bc, sj = (e >> 2) / bc;
      const int sl = sj & 1, jw = sj >> 1;
      const int os = o0 / kDxgO + sl;
      if (cell >= cells || os >= nst) continue;
      u16x8 v;
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = tile[(sl * kDxgO + 8 * g + i) * kDwyPitch + pw * cell + jw];
      *reinterpret_cast<u16x8*>(crow + (((int64_t)jw * nst + os) * a.mix_dcells + a.mix_dleft + mw0 + cell) * kDxgO + 8 * g) = v;
    }
  }
}

// Zeros in dyc's margin cells (before cell 0 and from cell M_w on), which the
// fused layout pass leaves: chunks (n, ho, jw, os, margin cell, 8 outputs).
__global__ __launch_bounds__(kThreads) void dx_mix_dyc_margin_kernel(const BwdArgs a) {
  const int nst = a.mix_opad / kDxgO;
  const int margin = a.mix_dcells - a.Mw;   // dleft + right margin
  const int64_t per_row = (int64_t)a.tw_tab.p * nst * margin * 4;
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= (int64_t)a.planes_n * a.Ho * per_row) return;
  const int64_t row = e / per_row;   // n * Ho + ho
  int64_t r = e - row * per_row;
  const int g = (int)(r % 4); r /= 4;
  const int m = (int)(r % margin); r /= margin;
  const int os = (int)(r % nst);
  const int jw = (int)(r / nst);
  const int cell = m < a.mix_dleft ? m : a.Mw + m;   // dyc cell index
  *reinterpret_cast<u16x8*>(a.mix_dyc + ((row * a.tw_tab.p + jw) * nst + os) * (int64_t)a.mix_dcells * kDxgO +
                            (int64_t)cell * kDxgO + 8 * g) = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
}

// xa from x: a block takes 64 channels of one extended row and dwxcells
// cells, reading the input columns those cells' taps reach (padding resolved
// once per column into LDS) into an LDS tile [c][column]; then lane c
// gathers 8 cells of one tap offset from its row and writes them as 16 bytes.
constexpr int kDwxPitch = 306;   // LDS pitch (16-bit units) of the x pass tile
__global__ __launch_bounds__(kThreads) void dw_mix_x_kernel(const BwdArgs a) {
  extern __shared__ float smem[];
  uint16_t* const tile = reinterpret_cast<uint16_t*>(smem);
  int* const scol = reinterpret_cast<int*>(tile + 64 * kDwxPitch);   // source column of each tile column
  const int q = a.tw_tab.q;
  const int bc = a.mix_dwxcells;
  const int cblocks = (a.mix_ncb * 32 + bc - 1) / bc;
  const int chunks = a.mix_cpad / 64;
  const int erows = a.mix_eh1 - a.mix_eh0 + 1;
  int64_t blk = blockIdx.x;
  const int cc = (int)(blk % chunks); blk /= chunks;
  const int cbk = (int)(blk % cblocks); blk /= cblocks;
  const int er = (int)(blk % erows); blk /= erows;
  const int n = (int)blk;
  const int mw0 = cbk * bc, c0 = cc * 64;
  const int ns = a.mix_ns;
  const int col0 = q * mw0 + a.mix_s0;
  const int ncols = q * (bc - 1) + ns;   // <= kDwxPitch - 2
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int sr = pad_source(a.mix_eh0 + er, a.H, a.pad);
  for (int t = threadIdx.x; t < ncols; t += kThreads) scol[t] = pad_source(col0 + t, a.W, a.pad);
  __syncthreads();
  const uint16_t* const xb = reinterpret_cast<const uint16_t*>(a.x) + (int64_t)n * a.C * a.H * a.W;
  // rows wave + 4 i in two batches of 8 per wave, all loads of a batch issued
  // before its LDS stores
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    uint16_t v[8][5];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int r = wave + 4 * (8 * h + i);
      const bool ok = sr >= 0 && c0 + r < a.C;
      const uint16_t* const src = xb + ((int64_t)(ok ? c0 + r : 0) * a.H + (sr >= 0 ? sr : 0)) * a.W;
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        const int t = lane + 64 * j;
        const int sc = t < ncols ? scol[t] : -1;
        v[i][j] = (ok && sc >= 0) ? src[sc] : (uint16_t)0;
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int j = 0; j < 5; ++j)
        if (lane + 64 * j < ncols) tile[(wave + 4 * (8 * h + i)) * kDwxPitch + lane + 64 * j] = v[i][j];
  }
  __syncthreads();
  const int ng = bc / 8;
  uint16_t* const orow = a.mix_xa + ((int64_t)n * erows + er) * ns * a.mix_ncb * 32 * a.mix_cpad;
  for (int k = wave; k < ns * ng; k += 4) {
    const int sidx = k / ng, gb = k - sidx * ng;
    const int mw = mw0 + 8 * gb;
    if (mw >= a.mix_ncb * 32) continue;
    u16x8 v;
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = (mw + i < a.Mw) ? tile[lane * kDwxPitch + q * (8 * gb + i) + sidx] : (uint16_t)0;
    *reinterpret_cast<u16x8*>(orow + ((((int64_t)sidx * a.mix_ncb + mw / 32) * 4 + (mw % 32) / 8) * a.mix_cpad + c0 + lane) * 8) = v;
  }
}

// Partial sums of one chunk of cell rows: partial[chunk][ph][tap][o][c].
// The four waves share each step's dy tile (64 outputs x 32 cells, 4 KB):
// wave w loads its quarter (cells 8 w .. 8 w + 7) with one 16-byte load per
// lane, stores it to LDS, and all read their A fragments from there (two LDS
// buffers, one barrier per step); the B fragments (each wave's own tap) come
// straight from global memory. The next step's loads are in flight during
// the current step's MFMAs.
template <int DT>
__global__ __launch_bounds__(kThreads, 2) void dw_mix_gemm_kernel(const BwdArgs a) {
  using M = Mfma<DT>;
  extern __shared__ float smem[];
  uint16_t* const alds = reinterpret_cast<uint16_t*>(smem);   // [2][4 groups][64 outputs][8 cells]
  const AxisTable& TH = a.th;
  const AxisTable& TW = a.tw_tab;
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, g4 = lane >> 4;
  const int tb = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int64_t blk = bwd::xcd_block();
  const int ctiles = a.mix_cpad / kDwgT, otiles = a.mix_dwopad / kDwgT;
  const int ct = (int)(blk % ctiles); blk /= ctiles;
  const int ot = (int)(blk % otiles); blk /= otiles;
  const int ta = (int)(blk % 4); blk /= 4;
  const int ph = (int)(blk % (TH.p * TW.p)); blk /= TH.p * TW.p;
  const int chunk = (int)blk;
  if (chunk >= a.mix_wchunks) return;
  const int jh = ph / TW.p, jw = ph % TW.p;
  const int s = TW.off[jw] + tb - a.mix_s0;
  const int erows = a.mix_eh1 - a.mix_eh0 + 1;
  const int ncb = a.mix_ncb;
  const int G = a.planes_n * a.Mh;   // cell rows (n, mh)
  const int g_lo = (int)((int64_t)G * chunk / a.mix_wchunks);
  const int g_hi = (int)((int64_t)G * (chunk + 1) / a.mix_wchunks);
  const int64_t ystride = (int64_t)4 * a.mix_dwopad * 8;   // one 32-cell block of dyw
  const int64_t xstride = (int64_t)4 * a.mix_cpad * 8;     // one 32-cell block of xa
  const uint32_t aoff = (uint32_t)((tb * a.mix_dwopad + ot * kDwgT + lane) * 8);   // this wave's quarter
  const uint32_t boff = (uint32_t)((g4 * a.mix_cpad + ct * kDwgT + li) * 8);

  f32x4 acc[4][4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int steps = (g_hi - g_lo) * ncb;
  int g = g_lo, cb = 0;
  // running pointers to the step's 32-cell blocks, set at each cell row
  const uint16_t *pa = nullptr, *pb = nullptr;
  auto set_row = [&]() {
    const int n = g / a.Mh, mh = g - n * a.Mh;
    const int ho = TH.p * mh + jh, er = TH.q * mh + TH.off[jh] + ta - a.mix_eh0;
    pa = a.mix_dyw + (((int64_t)n * a.Ho + ho) * TW.p + jw) * ncb * ystride;
    pb = a.mix_xa + (((int64_t)n * erows + er) * a.mix_ns + s) * ncb * xstride;
  };
  if (steps > 0) set_row();
  u16x8 ast, bf0[4], bf1[4];
  auto gload = [&](u16x8 (&B)[4]) __attribute__((always_inline)) {
    ast = *reinterpret_cast<const u16x8*>(pa + aoff);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) B[nt] = *reinterpret_cast<const u16x8*>(pb + boff + 16 * 8 * nt);
    pa += ystride;
    pb += xstride;
    if (++cb == ncb) {
      cb = 0;
      if (++g < g_hi) set_row();
    }
  };
  auto store_a = [&](int buf) __attribute__((always_inline)) {
    *reinterpret_cast<u16x8*>(alds + buf * 2048 + (tb * 64 + lane) * 8) = ast;
  };
  auto mma = [&](int buf, const u16x8 (&B)[4]) __attribute__((always_inline)) {
    u16x8 af[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) af[mt] = *reinterpret_cast<const u16x8*>(alds + buf * 2048 + (g4 * 64 + 16 * mt + li) * 8);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = M::mma(af[mt], B[nt], acc[mt][nt]);
  };
  if (steps > 0) {
    gload(bf0);
    store_a(0);
  }
  __syncthreads();
  int st = 0;
  for (; st + 1 < steps; st += 2) {
    gload(bf1);                      // step st + 1
    mma(0, bf0);                     // step st
    store_a(1);
    __syncthreads();
    if (st + 2 < steps) gload(bf0);  // step st + 2
    mma(1, bf1);                     // step st + 1
    if (st + 2 < steps) store_a(0);
    __syncthreads();
  }
  if (st < steps) mma(0, bf0);       // the last step (steps odd)

  // D: lane holds column c = 16 nt + li, rows o = 16 mt + 4 g4 + r
  float* const out = a.partial + (((int64_t)chunk * TH.p * TW.p + ph) * 16 + ta * 4 + tb) * a.Cout * a.C;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = ot * kDwgT + 16 * mt + 4 * g4 + r, c = ct * kDwgT + 16 * nt + li;
        if (o < a.Cout && c < a.C) out[(int64_t)o * a.C + c] = acc[mt][nt][r];
      }
}

// dw[ph][o][c][tap] = sum of the chunks' partial[chunk][ph][tap][o][c], in
// chunk order (threads run over the partials' order, so the reads coalesce).
__global__ __launch_bounds__(kThreads) void dw_mix_gemm_reduce_kernel(const BwdArgs a) {
  const int64_t oc = (int64_t)a.Cout * a.C;
  const int64_t per = (int64_t)a.th.p * a.tw_tab.p * 16 * oc;
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= per) return;
  float s = 0.f;
  for (int k = 0; k < a.mix_wchunks; ++k) s += a.partial[k * per + e];
  const int64_t r = e % oc, pt = e / oc;
  const int tap = (int)(pt % 16);
  const int64_t ph = pt / 16;
  a.dw[(ph * oc + r) * 16 + tap] = s;
}

template <int DT>
fcfs_status launch_backward_mix_dt(const BwdArgs& a, hipStream_t stream) {
  const dim3 block(kThreads);
  const int64_t ncb32 = (int64_t)a.mix_ncb * 32;
  const int64_t yblocks = (int64_t)a.planes_n * a.Ho * ((ncb32 + a.mix_dwcells - 1) / a.mix_dwcells) * (a.mix_dwopad / 64);
  if (a.dx && a.dw) {
    // both gradients: one pass over dy writes both layouts, then dyc's margins
    hipLaunchKernelGGL(dw_mix_dy_kernel<true>, dim3((unsigned)yblocks), block, sizeof(uint16_t) * 64 * kDwyPitch, stream, a);
    const int64_t mchunks = (int64_t)a.planes_n * a.Ho * a.tw_tab.p * (a.mix_opad / kDxgO) * (a.mix_dcells - a.Mw) * 4;
    if (mchunks > 0)
      hipLaunchKernelGGL(dx_mix_dyc_margin_kernel, dim3((unsigned)((mchunks + kThreads - 1) / kThreads)), block, 0, stream, a);
  } else if (a.dx) {
    const int64_t cl_blocks = (int64_t)a.planes_n * a.Ho * ((a.mix_dcells + a.mix_clcells - 1) / a.mix_clcells);
    hipLaunchKernelGGL(dx_mix_channel_last_kernel, dim3((unsigned)cl_blocks), block,
                       sizeof(uint16_t) * kDxcColumns * kDxcPitch, stream, a);
  } else if (a.dw) {
    hipLaunchKernelGGL(dw_mix_dy_kernel<false>, dim3((unsigned)yblocks), block, sizeof(uint16_t) * 64 * kDwyPitch, stream, a);
  }
  if (a.dx) {
    // packed weights, z on MFMA (dx directly, the fold zones to the edge
    // buffer), then the fold zones
    const int64_t wtotal = (int64_t)a.th.p * a.tw_tab.p * 16 * a.mix_cpad * a.mix_opad;
    hipLaunchKernelGGL(dx_mix_pack_weights_kernel, dim3((unsigned)((wtotal + kThreads - 1) / kThreads)), block, 0,
                       stream, a);
    const int64_t gblocks = (int64_t)a.planes_n * a.mix_rows * a.mix_vgroups * (a.mix_cpad / kDxgC);
    const dim3 ggrid((unsigned)gblocks);
    const size_t glds = a.mix_lds_epi ? sizeof(uint16_t) * kDxgC * a.tw_tab.q * a.mix_kw * 16 * a.mix_mtn : 0;
    switch (a.mix_mtn) {
      case 1: hipLaunchKernelGGL((dx_mix_gemm_kernel<DT, 1>), ggrid, block, glds, stream, a); break;
      case 2: hipLaunchKernelGGL((dx_mix_gemm_kernel<DT, 2>), ggrid, block, glds, stream, a); break;
      case 3: hipLaunchKernelGGL((dx_mix_gemm_kernel<DT, 3>), ggrid, block, glds, stream, a); break;
      default: hipLaunchKernelGGL((dx_mix_gemm_kernel<DT, 4>), ggrid, block, glds, stream, a); break;
    }
    if (a.mix_edge) {
      const int64_t eblocks = (a.mix_edge_per + kThreads - 1) / kThreads;
      const int64_t planes = (int64_t)a.planes_n * a.C;
      if (eblocks > 0)
        hipLaunchKernelGGL((dx_mix_edge_kernel<DT>), dim3((unsigned)eblocks, (unsigned)std::min<int64_t>(planes, 65535)),
                           block, 0, stream, a);
    }
    if (hipGetLastError() != hipSuccess) return FCFS_E_DEVICE;
  }
  if (a.dw) {
    // x by tap offset, the GEMM per (phase, tap row) and chunk, then the
    // chunks added in order
    const int64_t erows = a.mix_eh1 - a.mix_eh0 + 1;
    const int64_t xblocks = (int64_t)a.planes_n * erows * ((ncb32 + a.mix_dwxcells - 1) / a.mix_dwxcells) * (a.mix_cpad / 64);
    hipLaunchKernelGGL(dw_mix_x_kernel, dim3((unsigned)xblocks), block,
                       sizeof(uint16_t) * 64 * kDwxPitch + sizeof(int) * kDwxPitch, stream, a);
    const int64_t gblocks = (int64_t)a.mix_wchunks * a.th.p * a.tw_tab.p * 4 * (a.mix_dwopad / kDwgT) * (a.mix_cpad / kDwgT);
    hipLaunchKernelGGL((dw_mix_gemm_kernel<DT>), dim3((unsigned)gblocks), block, sizeof(uint16_t) * 2 * 2048, stream, a);
    const int64_t per = (int64_t)a.th.p * a.tw_tab.p * 16 * a.Cout * a.C;
    hipLaunchKernelGGL(dw_mix_gemm_reduce_kernel, dim3((unsigned)((per + kThreads - 1) / kThreads)), block, 0, stream, a);
    if (hipGetLastError() != hipSuccess) return FCFS_E_DEVICE;
  }
  return FCFS_OK;
}

}  // namespace bwdmix
}  // namespace fcfs
