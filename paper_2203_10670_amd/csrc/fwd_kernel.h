// Fused FCFS forward for gfx950: virtual padding + stride-q per-phase
// convolution + pixelshuffle in one pass (paper Sec. 3.1 / Sec. 4.2).
//
// Work decomposition. One wave (64 lanes) owns a strip of `tw` output columns
// of one (n, c) plane and a band of `band_cells` hidden-layer cells (groups
// of p output rows). Waves never synchronise with
// each other: each has a private LDS row buffer, so a workgroup is just four
// independent waves.
//
// Per wave the kernel streams the input rows its band needs, top to bottom:
//   1. the row segment the strip needs is prefetched kPrefetch rows ahead
//      into registers (coalesced dword loads; padding is applied by remapping
//      the source row and column, zero padding by a select afterwards, so the
//      loads themselves are unconditional and stay in flight),
//   2. the row is staged in the wave's LDS buffer and every lane evaluates the
//      horizontal taps of its output columns (the separable kernel's width
//      pass), giving one value per column,
//   3. that value is pushed into a per-lane FIFO holding the last T rows,
//   4. every output row whose last vertical tap is this input row is finished
//      from the FIFO with the phase's height taps and stored at its
//      pixelshuffled position (output row p*m + j).
// The hidden layer of the paper is never materialised and each output sample
// is written exactly once. Rows no tap reads (nearest, large q) are not
// fetched: their slot re-reads the nearest row below that is (a cache hit).
//
// The learned depthwise variant keeps the T x T raw taps per column in the
// FIFO instead (its 4x4 kernels are not separable) and reads the per-channel
// weights of the phase from LDS.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "fcfs_internal.h"

namespace fcfs {
namespace fwd {

#ifndef FCFS_FWD_PREFETCH
#define FCFS_FWD_PREFETCH 4
#endif
#ifndef FCFS_FWD_XCD_SWIZZLE
#define FCFS_FWD_XCD_SWIZZLE 0
#endif
#ifndef FCFS_FWD_NT_STORE
#define FCFS_FWD_NT_STORE 1
#endif

constexpr int kWaves = 4;       // waves per workgroup
constexpr int kRowMax = 512;    // staged row segment per wave (floats)
constexpr int kPrefetch = FCFS_FWD_PREFETCH;   // rows in flight per wave
constexpr int kXcds = 8;        // MI355X: workgroups are dealt round-robin to 8 XCDs

// ---------------------------------------------------------------- storage types
typedef float f32x2 __attribute__((ext_vector_type(2)));
template <int DT> struct Store;
template <> struct Store<FCFS_F32> {
  using T = float;
  static __device__ __forceinline__ float load(const T* p) { return *p; }
  static __device__ __forceinline__ void store(T* p, float v) {
    if (FCFS_FWD_NT_STORE) __builtin_nontemporal_store(v, p);
    else *p = v;
  }
};
template <> struct Store<FCFS_BF16> {
  using T = uint16_t;
  typedef __bf16 x2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ float from_bits(uint32_t b) { return __uint_as_float(b << 16); }
  static __device__ __forceinline__ float load(const T* p) {
    const uint32_t b = *p;
    return __uint_as_float(b << 16);
  }
  // round to nearest even (NaN stays a quiet NaN)
  static __device__ __forceinline__ void store(T* p, float v) {
    const T r = __builtin_bit_cast(T, (__bf16)v);
    if (FCFS_FWD_NT_STORE) __builtin_nontemporal_store(r, p);
    else *p = r;
  }
  // p[0] = lo, p[1] = hi (p 4-byte aligned)
  static __device__ __forceinline__ void store2(T* p, float lo, float hi) {
    const f32x2 v = {lo, hi};
    const uint32_t r = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, x2));
    if (FCFS_FWD_NT_STORE) __builtin_nontemporal_store(r, reinterpret_cast<uint32_t*>(p));
    else *reinterpret_cast<uint32_t*>(p) = r;
  }
};
template <> struct Store<FCFS_F16> {
  using T = _Float16;
  typedef _Float16 x2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ float from_bits(uint32_t b) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)b);
  }
  static __device__ __forceinline__ float load(const T* p) { return (float)*p; }
  static __device__ __forceinline__ void store(T* p, float v) {
    if (FCFS_FWD_NT_STORE) __builtin_nontemporal_store((_Float16)v, p);
    else *p = (_Float16)v;
  }
  static __device__ __forceinline__ void store2(T* p, float lo, float hi) {
    const f32x2 v = {lo, hi};
    const uint32_t r = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, x2));
    if (FCFS_FWD_NT_STORE) __builtin_nontemporal_store(r, reinterpret_cast<uint32_t*>(p));
    else *reinterpret_cast<uint32_t*>(p) = r;
  }
};

// Source index of position i of an axis of length n under the padding mode,
// or -1 for a zero-padded position.
__device__ __forceinline__ int pad_source(int i, int n, int mode) {
  if ((unsigned)i < (unsigned)n) return i;
  if (mode == FCFS_PAD_ZERO) return -1;
  if (mode == FCFS_PAD_REPLICATE) return i < 0 ? 0 : n - 1;
  if (n == 1) return 0;
  const int period = 2 * (n - 1);
  int m = i % period;
  if (m < 0) m += period;
  return m < n ? m : period - m;
}

__device__ __forceinline__ int mod_pos(int a, int q) {
  const int m = a % q;
  return m < 0 ? m + q : m;
}

// Orders this wave's LDS writes before its later LDS reads and vice versa
// (LDS operations of one wave execute in order; this keeps the compiler from
// moving them across each other).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Input column the strip of wave `wid` stages first, aligned down to an even
// column in paired mode.
template <bool PAIR>
__device__ __forceinline__ int strip_first_column(const FwdArgs& a, int64_t wid) {
  const AxisTable& TW = a.tw_tab;
  const int ow0 = (int)(wid % a.strips) * a.tw;
  const int c = TW.q * (ow0 / TW.p) + TW.omin;
  return PAIR ? (c & ~1) : c;
}

// The per-wave work of the forward: wave `wid` of the launch described by `a`
// (a may live in the kernel-argument segment or in device memory).
// PAIR (16-bit storage, even widths, 4-byte aligned tensors, and a staged
// segment wholly inside the row): every lane loads and stores two adjacent
// samples as one dword; its output columns are the adjacent pairs
// ow0 + 2*lane + 128*g + {0, 1}.
// T: width taps; TV: height taps (equal, except that an axis at 1/1 which
// samples its inputs exactly copies them with one tap while the other axis
// keeps the method's taps).
template <int DT, int T, int KC, int L, bool LEARNED, bool PAIR = false, int TV = T>
__device__ __forceinline__ void fwd_wave(const FwdArgs& a, int64_t wid, int wslot, int lane, float* smem) {
  using S = Store<DT>;
  using TS = typename S::T;
  static_assert(!PAIR || (DT != FCFS_F32 && KC % 2 == 0 && L <= 4), "paired I/O: 16-bit, column pairs");
  static_assert(!LEARNED || TV == T, "learned taps on both axes");
  const AxisTable& TH = a.th;
  const AxisTable& TW = a.tw_tab;

  const int strip = (int)(wid % a.strips);
  const int64_t t1 = wid / a.strips;
  const int band = (int)(t1 % a.bands);
  const int64_t plane = t1 / a.bands;

  const int ow0 = strip * a.tw;
  const int owEnd = min(ow0 + a.tw, a.Wo);
  const int m0 = band * a.band_cells;
  const int m1 = min(m0 + a.band_cells, a.Mh);
  const int cs = strip_first_column<PAIR>(a, wid);

  float* row = smem + wslot * kRowMax;
  float* wl = nullptr;
  if constexpr (LEARNED) {
    const int nph = TH.p * TW.p;
    wl = smem + kWaves * kRowMax + wslot * (nph * 16);
    const float* wsrc = a.weight + (int64_t)(plane % a.C) * nph * 16;
    for (int i = lane; i < nph * 16; i += 64) wl[i] = wsrc[i];
    wave_lds_sync();
  }

  // Output columns of this lane: ow0 + lane + 64*c (paired: ow0 + 2*lane +
  // 128*(c/2) + c%2).
  int pos[KC];
  int ocol[KC];
  int wbase[KC];
  bool cvalid[KC];
  float wc[KC][T];
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    const int ow = PAIR ? ow0 + 2 * lane + 128 * (c >> 1) + (c & 1) : ow0 + lane + 64 * c;
    cvalid[c] = ow < owEnd;
    const int owc = cvalid[c] ? ow : ow0;
    const int n = owc / TW.p;
    const int jw = owc - n * TW.p;
    ocol[c] = owc;
    pos[c] = TW.q * n + TW.off[jw] - cs;
    wbase[c] = jw * 16;
#pragma unroll
    for (int b = 0; b < T; ++b) wc[c][b] = LEARNED ? 0.f : TW.w[jw][b];
  }

  // Last staged column any tap of this strip reads (positions are
  // nondecreasing in the output column). Slots past it load that column
  // again instead of the next strip's samples, so a wave fetches only what
  // it uses (their staged values are never read).
  int need;
  {
    const int n = (owEnd - 1) / TW.p;
    need = TW.q * n + TW.off[owEnd - 1 - n * TW.p] - cs + T - 1;
  }

  // Source column of staged slot s of this lane (single samples: column
  // cs + min(lane + 64*s, need), clamped into the row, ckeep = false where
  // zero padding supplies the value; pairs: columns cs + 2*u + {0, 1} with
  // u = min(lane + 64*s, need / 2), inside the row by construction).
  int scol[L];
  bool ckeep[L];
#pragma unroll
  for (int s = 0; s < L; ++s) {
    if constexpr (PAIR) {
      scol[s] = cs + 2 * min(lane + 64 * s, need >> 1);
      ckeep[s] = true;
    } else {
      const int src = pad_source(cs + min(lane + 64 * s, need), a.W, a.pad);
      ckeep[s] = src >= 0;
      scol[s] = src >= 0 ? src : 0;
    }
  }

  const TS* xplane = reinterpret_cast<const TS*>(a.x) + plane * (int64_t)a.H * a.W;
  TS* yplane = reinterpret_cast<TS*>(a.y) + plane * (int64_t)a.Ho * a.Wo;

  // Band rows rs..re, streamed top to bottom. A row no tap reads (nearest,
  // large q) is replaced by the nearest row below that one does (already
  // fetched: a cache hit); fetches past re repeat the last row.
  const int rs = TH.q * m0 + TH.omin;
  const int re = TH.q * (m1 - 1) + TH.omax;
  auto source_row = [&](int r, int r_mod_q) -> int { return pad_source(r - TH.back[r_mod_q], a.H, a.pad); };
  const int src_last = source_row(re, mod_pos(re, TH.q));

  // prefetched rows: FP32 values, or raw sample pairs in paired mode
  using Raw = typename std::conditional<PAIR, uint32_t, float>::type;
  Raw buf[kPrefetch][L];
  int bsrc[kPrefetch];   // source row of each slot, -1 for a zero row
  int fr = rs, frho = mod_pos(rs, TH.q);   // next row to fetch, and it mod q
  auto fetch_next = [&](Raw (&dst)[L], int& src_out) __attribute__((always_inline)) {
    const int sr = fr <= re ? source_row(fr, frho) : src_last;
    src_out = sr;
    const TS* src = xplane + (int64_t)(sr < 0 ? 0 : sr) * a.W;
#pragma unroll
    for (int s = 0; s < L; ++s) {
      if constexpr (PAIR) dst[s] = *reinterpret_cast<const uint32_t*>(src + scol[s]);
      else dst[s] = S::load(src + scol[s]);
    }
    ++fr;
    frho = (frho + 1 == TH.q) ? 0 : frho + 1;
  };

  // FIFO of the last TV rows: fixed methods keep the width-filtered value per
  // column, the learned variant the T raw taps per column.
  constexpr int FT = LEARNED ? T : 1;
  float fifo[KC][TV][FT];
#pragma unroll
  for (int c = 0; c < KC; ++c)
#pragma unroll
    for (int t = 0; t < TV; ++t)
#pragma unroll
      for (int b = 0; b < FT; ++b) fifo[c][t][b] = 0.f;

#pragma unroll
  for (int d = 0; d < kPrefetch; ++d) fetch_next(buf[d], bsrc[d]);

  int rho = mod_pos(rs, TH.q);     // row being processed, mod q
  int rq = (rs - rho) / TH.q;      // ... and divided by q (floor)

  // One band row from prefetch slot d (a compile-time constant once unrolled).
  auto step = [&](const int d) __attribute__((always_inline)) {
    // stage the row (zero padding applied here), then refill the slot
    const bool zrow = bsrc[d] < 0;
    if constexpr (PAIR) {
#pragma unroll
      for (int s = 0; s < L; ++s) {
        const uint32_t raw = buf[d][s];
        row[2 * (lane + 64 * s)] = zrow ? 0.f : S::from_bits(raw & 0xffffu);
        row[2 * (lane + 64 * s) + 1] = zrow ? 0.f : S::from_bits(raw >> 16);
      }
    } else {
#pragma unroll
      for (int s = 0; s < L; ++s) row[lane + 64 * s] = (ckeep[s] && !zrow) ? buf[d][s] : 0.f;
    }
    fetch_next(buf[d], bsrc[d]);
    wave_lds_sync();
    float cur[KC][FT];
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      if constexpr (LEARNED) {
#pragma unroll
        for (int b = 0; b < T; ++b) cur[c][b] = row[pos[c] + b];
      } else if constexpr (T == 1) {
        cur[c][0] = row[pos[c]];
      } else {
        float h = wc[c][0] * row[pos[c]];
#pragma unroll
        for (int b = 1; b < T; ++b) h = __builtin_fmaf(wc[c][b], row[pos[c] + b], h);
        cur[c][0] = h;
      }
    }
    wave_lds_sync();
#pragma unroll
    for (int c = 0; c < KC; ++c) {
#pragma unroll
      for (int t = 0; t + 1 < TV; ++t)
#pragma unroll
        for (int b = 0; b < FT; ++b) fifo[c][t][b] = fifo[c][t + 1][b];
#pragma unroll
      for (int b = 0; b < FT; ++b) fifo[c][TV - 1][b] = cur[c][b];
    }

    // Finish every output row whose last height tap is this row.
    const int e1 = TH.emit_start[rho + 1];
    for (int e = TH.emit_start[rho]; e < e1; ++e) {
      const EmitRec er = a.emit[e];
      const int m = rq - er.lag;
      if (m < m0 || m >= m1) continue;
      TS* orow = yplane + (int64_t)(TH.p * m + er.j) * a.Wo;
      float outv[KC];
      if constexpr (LEARNED) {
        const float* wj = wl + er.j * TW.p * 16;
#pragma unroll
        for (int c = 0; c < KC; ++c) {
          const float* wk = wj + wbase[c];
          float acc = 0.f;
#pragma unroll
          for (int t = 0; t < T; ++t)
#pragma unroll
            for (int b = 0; b < T; ++b) acc = __builtin_fmaf(wk[t * 4 + b], fifo[c][t][b], acc);
          outv[c] = acc;
        }
      } else if constexpr (TV == 1) {
#pragma unroll
        for (int c = 0; c < KC; ++c) outv[c] = fifo[c][0][0];
      } else {
#pragma unroll
        for (int c = 0; c < KC; ++c) {
          float acc = er.w[0] * fifo[c][0][0];
#pragma unroll
          for (int t = 1; t < TV; ++t) acc = __builtin_fmaf(er.w[t], fifo[c][t][0], acc);
          outv[c] = acc;
        }
      }
      if constexpr (PAIR) {
        // both columns of a pair are valid or neither (even widths and starts)
#pragma unroll
        for (int g = 0; g < KC / 2; ++g)
          if (cvalid[2 * g]) S::store2(orow + ocol[2 * g], outv[2 * g], outv[2 * g + 1]);
      } else {
#pragma unroll
        for (int c = 0; c < KC; ++c)
          if (cvalid[c]) S::store(orow + ocol[c], outv[c]);
      }
    }
    if (++rho == TH.q) {
      rho = 0;
      ++rq;
    }
  };

  // Whole groups of kPrefetch rows, then the remainder. (Keeping the partial
  // group out of the loop lets every wait on a prefetched row count the three
  // younger rows' loads as still in flight.)
  const int nrows = re - rs + 1;
  for (int g = nrows / kPrefetch; g > 0; --g) {
#pragma unroll
    for (int d = 0; d < kPrefetch; ++d) step(d);
  }
  const int tail = nrows % kPrefetch;
#pragma unroll
  for (int d = 0; d + 1 < kPrefetch; ++d) {
    if (d >= tail) break;
    step(d);
  }
}

template <int DT, int T, int KC, int L, bool LEARNED, bool PAIR = false, int TV = T>
__global__ __launch_bounds__(256) void fcfs_fwd_kernel(const FwdArgs a) {
  extern __shared__ float smem[];
  const int lane = threadIdx.x & 63;
  const int wslot = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int64_t blk = blockIdx.x;
  if (FCFS_FWD_XCD_SWIZZLE) {
    // Workgroup b runs on XCD b % 8. Give each XCD a contiguous range of the
    // logical order, so that neighbouring strips and bands (which share
    // halo cache lines) meet in the same L2.
    const int64_t nb = gridDim.x;
    const int64_t per = nb / kXcds, rem = nb % kXcds;
    const int64_t x = blk % kXcds, i = blk / kXcds;
    blk = x * per + min(x, rem) + i;
  }
  const int64_t wid = blk * kWaves + wslot;
  if (wid >= a.waves) return;
  if constexpr (PAIR) {
    // strips whose staged segment reaches past either end of the row (and so
    // needs padding) move single samples
    const int cs = strip_first_column<true>(a, wid);
    if (cs < 0 || cs + 128 * L > a.W) fwd_wave<DT, T, KC, 2 * L, LEARNED, false, TV>(a, wid, wslot, lane, smem);
    else fwd_wave<DT, T, KC, L, LEARNED, true, TV>(a, wid, wslot, lane, smem);
  } else {
    fwd_wave<DT, T, KC, L, LEARNED, false, TV>(a, wid, wslot, lane, smem);
  }
}

template <int DT, int T, int KC, bool LEARNED, int TV = T>
fcfs_status launch_l(const FwdArgs& a, const FwdGeom& g, hipStream_t stream) {
  const dim3 block(64 * kWaves);
  const dim3 grid((unsigned)((g.waves + kWaves - 1) / kWaves));
  size_t lds = sizeof(float) * kWaves * kRowMax;
  if (LEARNED) lds += sizeof(float) * kWaves * a.th.p * a.tw_tab.p * 16;
  if constexpr (DT != FCFS_F32 && !LEARNED && KC % 2 == 0) {
    if (g.paired) {
      if (g.slots <= 2) hipLaunchKernelGGL((fcfs_fwd_kernel<DT, T, KC, 2, LEARNED, true, TV>), grid, block, lds, stream, a);
      else hipLaunchKernelGGL((fcfs_fwd_kernel<DT, T, KC, 4, LEARNED, true, TV>), grid, block, lds, stream, a);
      return hipGetLastError() == hipSuccess ? FCFS_OK : FCFS_E_DEVICE;
    }
  }
  switch (g.slots) {
    case 2: hipLaunchKernelGGL((fcfs_fwd_kernel<DT, T, KC, 2, LEARNED, false, TV>), grid, block, lds, stream, a); break;
    case 4: hipLaunchKernelGGL((fcfs_fwd_kernel<DT, T, KC, 4, LEARNED, false, TV>), grid, block, lds, stream, a); break;
    default: hipLaunchKernelGGL((fcfs_fwd_kernel<DT, T, KC, 8, LEARNED, false, TV>), grid, block, lds, stream, a); break;
  }
  return hipGetLastError() == hipSuccess ? FCFS_OK : FCFS_E_DEVICE;
}

template <int DT, int T, int TV = T>
fcfs_status launch_kc(const FwdArgs& a, const FwdGeom& g, hipStream_t stream) {
  switch (g.kc) {
    case 4: return launch_l<DT, T, 4, false, TV>(a, g, stream);
    case 2: return launch_l<DT, T, 2, false, TV>(a, g, stream);
    default: return launch_l<DT, T, 1, false, TV>(a, g, stream);
  }
}

template <int DT>
fcfs_status launch_forward_dt(int method, const FwdArgs& a, const FwdGeom& g, hipStream_t stream) {
  if (method == FCFS_LEARNED_DW4) return launch_l<DT, 4, 1, true>(a, g, stream);
  switch (a.tw_tab.T * 10 + a.th.T) {
    case 11: return launch_kc<DT, 1>(a, g, stream);
    case 22: return launch_kc<DT, 2>(a, g, stream);
    case 44: return launch_kc<DT, 4>(a, g, stream);
    case 21: return launch_kc<DT, 2, 1>(a, g, stream);   // height axis copies
    case 41: return launch_kc<DT, 4, 1>(a, g, stream);
    case 12: return launch_kc<DT, 1, 2>(a, g, stream);   // width axis copies
    case 14: return launch_kc<DT, 1, 4>(a, g, stream);
    default: return FCFS_E_UNSUPPORTED;
  }
}

}  // namespace fwd
}  // namespace fcfs
