// Fused FCFS forward for gfx950: virtual padding + stride-q per-phase
// convolution + pixelshuffle in one pass (paper Sec. 3.1 / Sec. 4.2).
//
// Work decomposition. One wave (64 lanes) owns a strip of `tw` output columns
// of one (n, c) plane and a band of hidden-layer cells (`band_cells` groups of
// p output rows). Waves never synchronise with each other: each has a private
// LDS row buffer, so a workgroup is just four independent waves.
//
// Per wave the kernel streams the input rows its band needs, top to bottom:
//   1. the row segment the strip needs is prefetched D rows ahead into
//      registers (coalesced loads, padding applied by remapping the source
//      column; zero padding loads nothing),
//   2. the row is staged in the wave's LDS buffer and every lane evaluates the
//      horizontal taps of its output columns (the separable kernel's width
//      pass), giving one value per column,
//   3. that value is pushed into a per-lane FIFO holding the last T rows,
//   4. every output row whose last vertical tap is this input row is finished
//      from the FIFO with the phase's height taps and stored at its
//      pixelshuffled position (output row p*m + j).
// The hidden layer of the paper is never materialised and each output sample
// is written exactly once. Rows no tap reads (nearest, large q) are skipped.
//
// The learned depthwise variant keeps the T x T raw taps per column in the
// FIFO instead (its 4x4 kernels are not separable) and reads the per-channel
// weights of the phase from LDS.

#include <hip/hip_runtime.h>

#include "fcfs_internal.h"

namespace fcfs {
namespace {

constexpr int kWaves = 4;       // waves per workgroup
constexpr int kRowDwords = 8;   // row-segment slots per lane (segment <= 512 samples)
constexpr int kPrefetch = 4;    // rows in flight per wave

// ---------------------------------------------------------------- storage types
template <int DT> struct Store;
template <> struct Store<FCFS_F32> {
  using T = float;
  static __device__ __forceinline__ float load(const T* p) { return *p; }
  static __device__ __forceinline__ void store(T* p, float v) { __builtin_nontemporal_store(v, p); }
};
template <> struct Store<FCFS_BF16> {
  using T = uint16_t;
  static __device__ __forceinline__ float load(const T* p) {
    uint32_t b = *p;
    return __uint_as_float(b << 16);
  }
  static __device__ __forceinline__ void store(T* p, float v) {
    uint32_t u = __float_as_uint(v);
    uint16_t r;
    if ((u & 0x7fffffffu) > 0x7f800000u) r = (uint16_t)((u >> 16) | 0x40u);   // quiet NaN
    else r = (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);               // round to nearest even
    __builtin_nontemporal_store(r, p);
  }
};
template <> struct Store<FCFS_F16> {
  using T = _Float16;
  static __device__ __forceinline__ float load(const T* p) { return (float)*p; }
  static __device__ __forceinline__ void store(T* p, float v) { __builtin_nontemporal_store((_Float16)v, p); }
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
  int m = a % q;
  return m < 0 ? m + q : m;
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int DT, int T, int KC, bool LEARNED>
__global__ __launch_bounds__(256) void fcfs_fwd_kernel(const FwdArgs a) {
  using S = Store<DT>;
  using TS = typename S::T;
  extern __shared__ float smem[];

  const int lane = threadIdx.x & 63;
  const int wslot = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t wid = (int64_t)blockIdx.x * kWaves + wslot;
  if (wid >= a.waves) return;

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

  const int n0 = ow0 / TW.p;
  const int cs = TW.q * n0 + TW.omin;                      // first input column staged
  const int nLast = (owEnd - 1) / TW.p;
  const int CW = TW.q * (nLast - n0) + TW.omax - TW.omin + 1;  // staged columns

  float* row = smem + wslot * (kRowDwords * 64);
  float* wl = nullptr;
  const int nph = TH.p * TW.p;
  if constexpr (LEARNED) {
    wl = smem + kWaves * (kRowDwords * 64) + wslot * (nph * 16);
    const float* wsrc = a.weight + (int64_t)(plane % a.C) * nph * 16;
    for (int i = lane; i < nph * 16; i += 64) wl[i] = wsrc[i];
    wave_lds_sync();
  }

  // Columns of this lane: ow0 + lane + 64*c.
  int pos[KC];
  int ocol[KC];
  int wbase[KC];
  bool cvalid[KC];
  float wc[KC][T];
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    const int ow = ow0 + lane + 64 * c;
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

  // Source column of each staged slot (lane + 64*s); -1 = zero.
  int scol[kRowDwords];
#pragma unroll
  for (int s = 0; s < kRowDwords; ++s) {
    const int i = lane + 64 * s;
    scol[s] = (i < CW) ? pad_source(cs + i, a.W, a.pad) : -1;
  }

  const TS* xplane = reinterpret_cast<const TS*>(a.x) + plane * (int64_t)a.H * a.W;
  TS* yplane = reinterpret_cast<TS*>(a.y) + plane * (int64_t)a.Ho * a.Wo;

  const int rs = TH.q * m0 + TH.omin;
  const int re = TH.q * (m1 - 1) + TH.omax;

  auto row_needed = [&](int r) -> bool { return (TH.need_mask >> mod_pos(r, TH.q)) & 1u; };

  float buf[kPrefetch][kRowDwords];
  auto load_row = [&](int r, float (&dst)[kRowDwords]) {
    if (r > re || !row_needed(r)) return;
    const int sr = pad_source(r, a.H, a.pad);
    if (sr < 0) {
#pragma unroll
      for (int s = 0; s < kRowDwords; ++s) dst[s] = 0.f;
      return;
    }
    const TS* src = xplane + (int64_t)sr * a.W;
#pragma unroll
    for (int s = 0; s < kRowDwords; ++s) {
      if (64 * s < CW) dst[s] = (scol[s] >= 0) ? S::load(src + scol[s]) : 0.f;
    }
  };

  // FIFO of the last T rows: fixed methods keep the width-filtered value per
  // column, the learned variant the T raw taps per column.
  constexpr int FT = LEARNED ? T : 1;
  float fifo[KC][T][FT];
#pragma unroll
  for (int c = 0; c < KC; ++c)
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int b = 0; b < FT; ++b) fifo[c][t][b] = 0.f;

#pragma unroll
  for (int d = 0; d < kPrefetch; ++d) load_row(rs + d, buf[d]);

  int rho = mod_pos(rs, TH.q);
  for (int rb = rs; rb <= re; rb += kPrefetch) {
#pragma unroll
    for (int d = 0; d < kPrefetch; ++d) {
      const int r = rb + d;
      if (r > re) break;
      const bool need = (TH.need_mask >> rho) & 1u;
      float cur[KC][FT];
      if (need) {
#pragma unroll
        for (int s = 0; s < kRowDwords; ++s)
          if (64 * s < CW) row[lane + 64 * s] = buf[d][s];
        load_row(r + kPrefetch, buf[d]);
        wave_lds_sync();
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
      } else {
        load_row(r + kPrefetch, buf[d]);
#pragma unroll
        for (int c = 0; c < KC; ++c)
#pragma unroll
          for (int b = 0; b < FT; ++b) cur[c][b] = 0.f;
      }
#pragma unroll
      for (int c = 0; c < KC; ++c) {
#pragma unroll
        for (int t = 0; t + 1 < T; ++t)
#pragma unroll
          for (int b = 0; b < FT; ++b) fifo[c][t][b] = fifo[c][t + 1][b];
#pragma unroll
        for (int b = 0; b < FT; ++b) fifo[c][T - 1][b] = cur[c][b];
      }

      // Finish every output row whose last height tap is input row r.
      const int e1 = TH.emit_start[rho + 1];
      for (int e = TH.emit_start[rho]; e < e1; ++e) {
        const int j = TH.emit_list[e];
        const int last = TH.off[j] + T - 1;
        const int m = (r - last) / TH.q;   // exact: r = last (mod q)
        if (m < m0 || m >= m1) continue;
        TS* orow = yplane + (int64_t)(TH.p * m + j) * a.Wo;
        if constexpr (LEARNED) {
          const float* wj = wl + j * TW.p * 16;
#pragma unroll
          for (int c = 0; c < KC; ++c) {
            const float* wk = wj + wbase[c];
            float acc = 0.f;
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
              for (int b = 0; b < T; ++b) acc = __builtin_fmaf(wk[t * 4 + b], fifo[c][t][b], acc);
            if (cvalid[c]) S::store(orow + ocol[c], acc);
          }
        } else if constexpr (T == 1) {
#pragma unroll
          for (int c = 0; c < KC; ++c)
            if (cvalid[c]) S::store(orow + ocol[c], fifo[c][0][0]);
        } else {
          float wv[T];
#pragma unroll
          for (int t = 0; t < T; ++t) wv[t] = TH.w[j][t];
#pragma unroll
          for (int c = 0; c < KC; ++c) {
            float acc = wv[0] * fifo[c][0][0];
#pragma unroll
            for (int t = 1; t < T; ++t) acc = __builtin_fmaf(wv[t], fifo[c][t][0], acc);
            if (cvalid[c]) S::store(orow + ocol[c], acc);
          }
        }
      }
      rho = (rho + 1 == TH.q) ? 0 : rho + 1;
    }
  }
}

template <int DT, int T, bool LEARNED>
fcfs_status launch_kc(const FwdArgs& a, const FwdGeom& g, hipStream_t stream) {
  const dim3 block(64 * kWaves);
  const dim3 grid((unsigned)((g.waves + kWaves - 1) / kWaves));
  size_t lds = sizeof(float) * kWaves * kRowDwords * 64;
  if (LEARNED) lds += sizeof(float) * kWaves * a.th.p * a.tw_tab.p * 16;
  switch (g.kc) {
    case 4: hipLaunchKernelGGL((fcfs_fwd_kernel<DT, T, 4, LEARNED>), grid, block, lds, stream, a); break;
    case 2: hipLaunchKernelGGL((fcfs_fwd_kernel<DT, T, 2, LEARNED>), grid, block, lds, stream, a); break;
    default: hipLaunchKernelGGL((fcfs_fwd_kernel<DT, T, 1, LEARNED>), grid, block, lds, stream, a); break;
  }
  return hipGetLastError() == hipSuccess ? FCFS_OK : FCFS_E_DEVICE;
}

template <int DT>
fcfs_status launch_dt(const fcfs_plan_* plan, const FwdArgs& a, const FwdGeom& g, hipStream_t stream) {
  if (plan->method == FCFS_LEARNED_DW4) return launch_kc<DT, 4, true>(a, g, stream);
  switch (plan->ah.T) {
    case 1: return launch_kc<DT, 1, false>(a, g, stream);
    case 2: return launch_kc<DT, 2, false>(a, g, stream);
    default: return launch_kc<DT, 4, false>(a, g, stream);
  }
}

}  // namespace

fcfs_status launch_forward_fixed(const fcfs_plan_* plan, int dtype, const FwdArgs& a,
                                 const FwdGeom& g, hipStream_t stream) {
  if (g.waves <= 0) return FCFS_OK;
  switch (dtype) {
    case FCFS_F32: return launch_dt<FCFS_F32>(plan, a, g, stream);
    case FCFS_BF16: return launch_dt<FCFS_BF16>(plan, a, g, stream);
    case FCFS_F16: return launch_dt<FCFS_F16>(plan, a, g, stream);
    default: return FCFS_E_INVAL;
  }
}

}  // namespace fcfs
