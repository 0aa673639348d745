// FCFS backward for gfx950: the adjoint of the forward (input gradient) and
// the gradient of the learned depthwise taps.
//
// Adjoint tables. For each input index i of an axis the setup kernel lists the
// (output index k, tap t) pairs whose tap reads i once the padding is applied:
// the extended positions e that the padding maps to i (e = i itself, and for
// replicate / reflect the positions beyond the edges that copy or mirror i),
// and for each e every phase j and tap t with q*m + off[j] + t = e. Entries
// are kept in ascending e, j, t order, so every sum below runs in a fixed
// order. Table row i: [count, first k, last k, entry 0, entry 1, ...], an
// entry packing (k << 7) | (j << 2) | t (output index k = p*m + j < 2^24).
// The height table keeps each row contiguous (a workgroup reads one row);
// the width table stores field f of column j at f * W + j, so that the
// consecutive columns of a wave read consecutive words.
//
// Input gradient. One thread per input sample: dx[i][c] = sum over the row
// entries (kh, th) and column entries (kw, tw) of w * dy[kh][kw], where w is
// the product of the two tap weights (fixed methods) or the learned weight
// W[channel][kh mod p][kw mod p][th][tw]. No atomics: each input sample
// gathers its own terms, so the pad adjoint (folding the gradient of padded
// positions back onto the samples they copy) costs nothing extra.
//
// Weight gradient (learned depthwise). dw[c][jh][jw][a][b] = sum over batch
// and cells of dy * ext(x). The partial kernel gives each workgroup a chunk of
// cells of one (n, c) plane, stages the chunk's dy and padded x in LDS, and
// has each thread accumulate the 16 taps of one phase over a fixed subset of
// cells; subsets are then added in a fixed order. The reduce kernel adds the
// chunks of each (channel, phase, tap) in a fixed order. Results do not
// depend on timing.
#pragma once

#include <hip/hip_runtime.h>

#include "fcfs_internal.h"
#include "fwd_kernel.h"

namespace fcfs {
namespace bwd {

using fwd::pad_source;
using fwd::Store;

constexpr int kThreads = 256;
#ifndef FCFS_BWD_DX_ROWS
#define FCFS_BWD_DX_ROWS 8
#endif
constexpr int kDxRows = FCFS_BWD_DX_ROWS;   // input rows per input-gradient workgroup
constexpr int kDxPlanes = 4;                 // planes per input-gradient workgroup

// Block b runs on XCD b % 8. The logical order the kernels below decode
// gives each XCD a contiguous range, so that neighbouring rows (which read
// the same output-gradient rows) share one L2.
__device__ __forceinline__ int64_t xcd_block() {
  int64_t blk = blockIdx.x;
  const int64_t per = (int64_t)gridDim.x / 8;
  if (blk < 8 * per) blk = (blk % 8) * per + blk / 8;
  return blk;
}

// Setup: the adjoint tables of both axes (rows 0..H-1 of the height axis,
// then 0..W-1 of the width axis).
template <int DT>
__global__ __launch_bounds__(kThreads) void adjoint_tables_kernel(const BwdArgs a) {
  const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (g >= (int64_t)a.H + a.W) return;
  const bool height = g < a.H;
  const int i = height ? (int)g : (int)(g - a.H);
  const AxisTable& t = height ? a.th : a.tw_tab;
  const int n = height ? a.H : a.W;
  const int cells = height ? a.Mh : a.Mw;
  const int cmax = height ? a.cmax_h : a.cmax_w;
  int* row = height ? a.tab_h + (int64_t)i * (3 + cmax) : a.tab_w + i;
  const int64_t fs = height ? 1 : a.W;   // field stride
  const int emin = t.omin, emax = t.q * (cells - 1) + t.omax;
  int cnt = 0, klo = 1 << 30, khi = -1;
  auto add_position = [&](int e) {
    for (int j = 0; j < t.p; ++j)
      for (int tap = 0; tap < t.T; ++tap) {
        const int d = e - t.off[j] - tap;
        if (d < 0 || d % t.q != 0) continue;
        const int m = d / t.q;
        if (m >= cells) continue;
        const int k = t.p * m + j;
        if (cnt < cmax) row[(3 + cnt) * fs] = (k << 7) | (j << 2) | tap;
        ++cnt;
        klo = min(klo, k);
        khi = max(khi, k);
      }
  };
  for (int e = emin; e < 0; ++e)
    if (pad_source(e, n, a.pad) == i) add_position(e);
  add_position(i);
  for (int e = n; e <= emax; ++e)
    if (pad_source(e, n, a.pad) == i) add_position(e);
  row[0] = min(cnt, cmax);
  row[fs] = klo;
  row[2 * fs] = khi;
}

// FE: width entries of a column held in registers (4 or 8, at least the
// most any interior column has); columns with more (the replicate / reflect
// edges) take the rest in a loop.
template <int DT, bool LEARNED, int FE>
__global__ __launch_bounds__(kThreads) void dx_kernel(const BwdArgs a) {
  constexpr int kFastEntries = FE;
  using S = Store<DT>;
  using TS = typename S::T;
  extern __shared__ float smem[];   // learned: the planes' taps [plane][p_h][p_w][4][4]
  const AxisTable& TH = a.th;
  const AxisTable& TW = a.tw_tab;
  // A workgroup: kDxRows consecutive rows of kDxPlanes consecutive planes,
  // 256 columns. The column's width entries and the planes' weights are set
  // up once; each row's height entries (decoded by the scalar unit) serve
  // all the planes.
  const int row_groups = (a.H + kDxRows - 1) / kDxRows;
  const int64_t per_group_blocks = (int64_t)row_groups * a.col_blocks;
  const int64_t lblk = xcd_block();
  const int64_t pgroup = lblk / per_group_blocks;
  const int rem = (int)(lblk - pgroup * per_group_blocks);
  const int i0 = (rem / a.col_blocks) * kDxRows;
  const int j = (rem % a.col_blocks) * kThreads + threadIdx.x;
  const int64_t plane0 = pgroup * kDxPlanes;
  const int np = (int)min((int64_t)kDxPlanes, a.planes - plane0);
  const int nwt = TH.p * TW.p * 16;
  if constexpr (LEARNED) {
    for (int k = threadIdx.x; k < kDxPlanes * nwt; k += kThreads) {
      const int pl = k / nwt;
      smem[k] = pl < np ? a.weight[(int64_t)((plane0 + pl) % a.C) * nwt + k % nwt] : 0.f;
    }
    __syncthreads();
  }
  if (j >= a.W) return;
  const int* rw = a.tab_w + j;   // field f at f * W
  const int64_t fw = a.W;
  const int nw = rw[0];
  // this column's width entries: output column, and the tap weight (fixed
  // methods) or the weight's offset within a height phase's block (learned)
  int kw[kFastEntries];
  int wo[kFastEntries];
  float ww[kFastEntries];
#pragma unroll
  for (int e = 0; e < kFastEntries; ++e) {
    const int ent = e < nw ? rw[(3 + e) * fw] : 0;
    const int jw = (ent >> 2) & 31, tw = ent & 3;
    kw[e] = ent >> 7;
    wo[e] = jw * 16 + tw;
    ww[e] = LEARNED ? 0.f : TW.w[jw][tw];
  }
  const int64_t oplane = (int64_t)a.Ho * a.Wo, iplane = (int64_t)a.H * a.W;
  const TS* dyp = reinterpret_cast<const TS*>(a.dy) + plane0 * oplane;
  TS* dxp = reinterpret_cast<TS*>(a.dx) + plane0 * iplane;
  const int i1 = min(i0 + kDxRows, a.H);
  for (int i = i0; i < i1; ++i) {
    const int* rh = a.tab_h + (int64_t)i * (3 + a.cmax_h);
    const int nh = rh[0];
    float acc[kDxPlanes];
#pragma unroll
    for (int k = 0; k < kDxPlanes; ++k) acc[k] = 0.f;
    for (int eh = 0; eh < nh; ++eh) {
      const int ent = rh[3 + eh];
      const int kh = ent >> 7, jh = (ent >> 2) & 31, th = ent & 3;
      // every plane's samples are requested before the first FMA (planes
      // past the last read the first one's, and are not stored)
      float vv[kDxPlanes][kFastEntries];
#pragma unroll
      for (int k = 0; k < kDxPlanes; ++k) {
        const TS* dyrow = dyp + (k < np ? k : 0) * oplane + (int64_t)kh * a.Wo;
#pragma unroll
        for (int e = 0; e < kFastEntries; ++e) vv[k][e] = S::load(dyrow + kw[e]);
      }
      // Entries e >= nw (offsets 0: in bounds) enter with weight and sample
      // both selected to 0, rather than behind a branch, so the weight reads
      // of all entries are in flight together. (Adding +0 changes a sum only
      // in the sign of a zero.) The entries past the registers (columns at
      // the padded edges) follow for every plane, after all planes' register
      // entries: each plane's sum keeps its order.
      float inner[kDxPlanes];
#pragma unroll
      for (int k = 0; k < kDxPlanes; ++k) {
        const float* v = vv[k];
        if constexpr (LEARNED) {
          const float* wr = smem + k * nwt + jh * TW.p * 16 + th * 4;
#pragma unroll
          for (int e = 0; e < kFastEntries; ++e) {
            const bool live = e < nw;
            acc[k] = __builtin_fmaf(live ? wr[wo[e]] : 0.f, live ? v[e] : 0.f, acc[k]);
          }
        } else {
          inner[k] = 0.f;
#pragma unroll
          for (int e = 0; e < kFastEntries; ++e) {
            const bool live = e < nw;
            inner[k] = __builtin_fmaf(live ? ww[e] : 0.f, live ? v[e] : 0.f, inner[k]);
          }
        }
      }
      if (nw > kFastEntries) {
#pragma unroll
        for (int k = 0; k < kDxPlanes; ++k) {
          const TS* dyrow = dyp + (k < np ? k : 0) * oplane + (int64_t)kh * a.Wo;
          for (int e = kFastEntries; e < nw; ++e) {
            const int we = rw[(3 + e) * fw];
            if constexpr (LEARNED) {
              const float* wr = smem + k * nwt + jh * TW.p * 16 + th * 4;
              acc[k] = __builtin_fmaf(wr[((we >> 2) & 31) * 16 + (we & 3)], S::load(dyrow + (we >> 7)), acc[k]);
            } else {
              inner[k] = __builtin_fmaf(TW.w[(we >> 2) & 31][we & 3], S::load(dyrow + (we >> 7)), inner[k]);
            }
          }
        }
      }
      if constexpr (!LEARNED) {
#pragma unroll
        for (int k = 0; k < kDxPlanes; ++k) acc[k] = __builtin_fmaf(TH.w[jh][th], inner[k], acc[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < kDxPlanes; ++k)
      if (k < np) S::store(dxp + k * iplane + (int64_t)i * a.W + j, acc[k]);
  }
}

// Weight gradient, stage 1: per-chunk partial sums. A chunk is ch x cw cells
// of one plane; block b covers channel c = b / chunks_per_channel.
template <int DT>
__global__ __launch_bounds__(kThreads) void dw_partial_kernel(const BwdArgs a) {
  using S = Store<DT>;
  using TS = typename S::T;
  extern __shared__ float smem[];
  const AxisTable& TH = a.th;
  const AxisTable& TW = a.tw_tab;
  const int64_t lblk = xcd_block();
  const int c = (int)(lblk / a.chunks_per_channel);
  const int r = (int)(lblk % a.chunks_per_channel);
  const int n = r / (a.nch * a.ncw);
  const int cb = r % (a.nch * a.ncw);
  const int mh0 = (cb / a.ncw) * a.ch, mw0 = (cb % a.ncw) * a.cw;
  const int mh1 = min(mh0 + a.ch, a.Mh), mw1 = min(mw0 + a.cw, a.Mw);
  const int64_t plane = (int64_t)n * a.C + c;
  // staged patches: dy rows p*mh0 .. p*mh1-1, cols p*mw0 .. ; x rows from
  // q*mh0 + omin, cols from q*mw0 + omin (padded)
  const int dyr = TH.p * (mh1 - mh0), dyc = TW.p * (mw1 - mw0);
  const int xr = TH.q * (mh1 - mh0 - 1) + TH.omax - TH.omin + 1;
  const int xc = TW.q * (mw1 - mw0 - 1) + TW.omax - TW.omin + 1;
  float* dys = smem;
  float* xs = smem + dyr * dyc;
  float* red = smem;           // [subsets][phases][16], over the staged patches once they are used
  const TS* dyp = reinterpret_cast<const TS*>(a.dy) + plane * (int64_t)a.Ho * a.Wo;
  const TS* xp = reinterpret_cast<const TS*>(a.x) + plane * (int64_t)a.H * a.W;
  // rows by wave, columns by lane (128-column blocks); loads of four rows
  // are issued before their stores
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int cb0 = 0; cb0 < dyc; cb0 += 128)
    for (int rr0 = wave; rr0 < dyr; rr0 += 16) {
      float v[4][2];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int rr = min(rr0 + 4 * u, dyr - 1), cc = min(cb0 + lane + 64 * h, dyc - 1);
          v[u][h] = S::load(dyp + (int64_t)(TH.p * mh0 + rr) * a.Wo + TW.p * mw0 + cc);
        }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          if (rr0 + 4 * u < dyr && cb0 + lane + 64 * h < dyc) dys[(rr0 + 4 * u) * dyc + cb0 + lane + 64 * h] = v[u][h];
    }
  const int xr0 = TH.q * mh0 + TH.omin, xc0 = TW.q * mw0 + TW.omin;
  for (int cb0 = 0; cb0 < xc; cb0 += 128) {
    int scol[2];
    bool cok[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int sc = pad_source(xc0 + min(cb0 + lane + 64 * h, xc - 1), a.W, a.pad);
      cok[h] = sc >= 0;
      scol[h] = sc >= 0 ? sc : 0;
    }
    for (int rr0 = wave; rr0 < xr; rr0 += 16) {
      float v[4][2];
      bool rok[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int sr = pad_source(xr0 + min(rr0 + 4 * u, xr - 1), a.H, a.pad);
        rok[u] = sr >= 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) v[u][h] = S::load(xp + (int64_t)(sr >= 0 ? sr : 0) * a.W + scol[h]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          if (rr0 + 4 * u < xr && cb0 + lane + 64 * h < xc)
            xs[(rr0 + 4 * u) * xc + cb0 + lane + 64 * h] = (rok[u] && cok[h]) ? v[u][h] : 0.f;
    }
  }
  __syncthreads();
  const int P2 = TH.p * TW.p;
  const int subsets = kThreads / P2;
  const int phase = threadIdx.x % P2, sub = threadIdx.x / P2;
  float acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = 0.f;
  if (sub < subsets) {
    const int jh = phase / TW.p, jw = phase % TW.p;
    const int oh = TH.off[jh] - TH.omin, ow = TW.off[jw] - TW.omin;
    const int cw = mw1 - mw0;
    int lh = sub / cw, lw = sub % cw;   // cell sub, then every subsets-th cell (no division per cell)
    for (; lh < mh1 - mh0;) {
      const float g = dys[(TH.p * lh + jh) * dyc + TW.p * lw + jw];
      const float* xb = xs + (TH.q * lh + oh) * xc + TW.q * lw + ow;
#pragma unroll
      for (int ta = 0; ta < 4; ++ta)
#pragma unroll
        for (int tb = 0; tb < 4; ++tb) acc[ta * 4 + tb] = __builtin_fmaf(g, xb[ta * xc + tb], acc[ta * 4 + tb]);
      lw += subsets;
      while (lw >= cw) {
        lw -= cw;
        ++lh;
      }
    }
  }
  __syncthreads();   // the staged patches are no longer read
  if (sub < subsets) {
    float* rp = red + (sub * P2 + phase) * 16;
#pragma unroll
    for (int k = 0; k < 16; ++k) rp[k] = acc[k];
  }
  __syncthreads();
  // add the subsets in a fixed order: thread t handles (phase, tap) pairs;
  // partials are laid out [C][phase, tap][chunk]
  float* out = a.partial + (int64_t)c * P2 * 16 * a.chunks_per_channel + r;
  for (int pt = threadIdx.x; pt < P2 * 16; pt += kThreads) {
    float s = 0.f;
    for (int sb = 0; sb < subsets; ++sb) s += red[sb * P2 * 16 + pt];
    out[(int64_t)pt * a.chunks_per_channel] = s;
  }
}

// Weight gradient, stage 2: the chunks of each (channel, phase, tap), one
// wave each: lane l adds chunks l, l + 64, ... in order, then lane 0 adds the
// 64 lane sums in order.
template <int DT>
__global__ __launch_bounds__(kThreads) void dw_reduce_kernel(const BwdArgs a) {
  extern __shared__ float smem[];
  float* lsum = smem;   // [kThreads]
  const int P2 = a.th.p * a.tw_tab.p;
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);   // (c, phase, tap)
  const bool live = g < (int64_t)a.C * P2 * 16;
  float s = 0.f;
  if (live) {
    const float* src = a.partial + g * a.chunks_per_channel;
    for (int r = lane; r < a.chunks_per_channel; r += 64) s += src[r];
  }
  lsum[threadIdx.x] = s;
  __syncthreads();
  if (live && lane == 0) {
    float t = 0.f;
    for (int l = 0; l < 64; ++l) t += lsum[threadIdx.x + l];
    a.dw[g] = t;   // layout [C][p_h][p_w][4][4] = [C][phase][16]
  }
}

template <int DT>
fcfs_status launch_backward_dt(const BwdArgs& a, bool learned, hipStream_t stream) {
  const dim3 block(kThreads);
  hipLaunchKernelGGL((adjoint_tables_kernel<DT>), dim3((unsigned)(((int64_t)a.H + a.W + kThreads - 1) / kThreads)),
                     block, 0, stream, a);
  if (hipGetLastError() != hipSuccess) return FCFS_E_DEVICE;
  if (a.dx) {
    const int64_t blocks =
        ((a.planes + kDxPlanes - 1) / kDxPlanes) * (int64_t)((a.H + kDxRows - 1) / kDxRows) * a.col_blocks;
    const size_t wl = sizeof(float) * kDxPlanes * a.th.p * a.tw_tab.p * 16;
    const dim3 grid((unsigned)blocks);
    if (a.fast_w <= 4) {
      if (learned) hipLaunchKernelGGL((dx_kernel<DT, true, 4>), grid, block, wl, stream, a);
      else hipLaunchKernelGGL((dx_kernel<DT, false, 4>), grid, block, 0, stream, a);
    } else {
      if (learned) hipLaunchKernelGGL((dx_kernel<DT, true, 8>), grid, block, wl, stream, a);
      else hipLaunchKernelGGL((dx_kernel<DT, false, 8>), grid, block, 0, stream, a);
    }
    if (hipGetLastError() != hipSuccess) return FCFS_E_DEVICE;
  }
  if (a.dw) {
    hipLaunchKernelGGL((dw_partial_kernel<DT>), dim3((unsigned)(a.C * (int64_t)a.chunks_per_channel)), block,
                       a.dw_lds_bytes, stream, a);
    if (hipGetLastError() != hipSuccess) return FCFS_E_DEVICE;
    const int64_t n = (int64_t)a.C * a.th.p * a.tw_tab.p * 16;   // one wave each
    hipLaunchKernelGGL((dw_reduce_kernel<DT>), dim3((unsigned)((n + 3) / 4)), block, sizeof(float) * kThreads,
                       stream, a);
    if (hipGetLastError() != hipSuccess) return FCFS_E_DEVICE;
  }
  return FCFS_OK;
}

}  // namespace bwd
}  // namespace fcfs
