// C ABI of libfcfs: plans (per-axis tap tables), argument validation and
// dispatch to the HIP kernels.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "fcfs_internal.h"

namespace fcfs {
namespace {

int64_t floor_div(int64_t a, int64_t b) {
  int64_t d = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --d;
  return d;
}

int gcd_int(int a, int b) {
  while (b) {
    int t = a % b;
    a = b;
    b = t;
  }
  return a;
}

int mod_pos(int a, int q) {
  int m = a % q;
  return m < 0 ? m + q : m;
}

// Keys cubic convolution weights (a = -1/2, paper Sec. 5.2.3) of the four
// samples at offsets -1, 0, 1, 2 from floor(u), for fractional part t.
void keys_taps(double t, double w[4]) {
  const double t2 = t * t, t3 = t2 * t;
  w[0] = 0.5 * (-t3 + 2.0 * t2 - t);
  w[1] = 0.5 * (3.0 * t3 - 5.0 * t2 + 2.0);
  w[2] = 0.5 * (-3.0 * t3 + 4.0 * t2 + t);
  w[3] = 0.5 * (t3 - t2);
}

// Overflow-checked product.
bool mul_ok(int64_t a, int64_t b, int64_t* out) {
  if (a < 0 || b < 0) return false;
  if (a != 0 && b > INT64_MAX / a) return false;
  *out = a * b;
  return true;
}

}  // namespace

// Sampling position of phase j of a cell, as a numerator over 2p of the
// offset from q*m (paper Sec. 3.1.1: each of the p kernels interpolates at
// its own sub-cell offset), for each grid reading.
static int64_t grid_numerator(int p, int q, int j, int grid) {
  switch (grid) {
    case FCFS_GRID_PAPER: return (int64_t)(2 * j + 1) * q;
    case FCFS_GRID_ASYM: return (int64_t)2 * j * q;
    default: return (int64_t)(2 * j + 1) * q - p;
  }
}

fcfs_status build_axis(int p, int q, int method, int grid, bool allow_copy, AxisTable* t) {
  std::memset(t, 0, sizeof(*t));
  const int g = gcd_int(p, q);
  p /= g;
  q /= g;
  if (p > kMaxFactor || q > kMaxFactor) return FCFS_E_UNSUPPORTED;
  t->p = p;
  t->q = q;
  const bool learned = method == FCFS_LEARNED_DW4 || method == FCFS_LEARNED_MIX4;
  // At 1/1 the half and asym grids sample every input exactly: a copy.
  const bool identity = allow_copy && !learned && p == 1 && q == 1 && grid != FCFS_GRID_PAPER;
  int T = 4;
  if (!learned) {
    if (method == FCFS_NEAREST || identity) T = 1;
    else if (method == FCFS_BILINEAR) T = 2;
  }
  t->T = T;
  int omin = 1 << 30, omax = -(1 << 30);
  for (int j = 0; j < p; ++j) {
    const int64_t A = grid_numerator(p, q, j, grid);
    const int64_t two_p = 2 * (int64_t)p;
    const int64_t b = floor_div(A, two_p);
    const double frac = (double)(A - two_p * b) / (double)two_p;
    int off;
    double w[4] = {0, 0, 0, 0};
    if (T == 1) {
      off = (int)floor_div(A + p, two_p);   // floor(u + 1/2)
      w[0] = 1.0;
    } else if (T == 2) {
      off = (int)b;
      w[0] = 1.0 - frac;
      w[1] = frac;
    } else {
      off = (int)b - 1;
      if (!learned) keys_taps(frac, w);
    }
    t->off[j] = off;
    for (int k = 0; k < 4; ++k) t->w[j][k] = (float)w[k];
    omin = std::min(omin, off);
    omax = std::max(omax, off + T - 1);
  }
  t->omin = omin;
  t->omax = omax;
  bool read[kMaxFactor] = {false};
  for (int j = 0; j < p; ++j)
    for (int k = 0; k < T; ++k) read[mod_pos(t->off[j] + k, q)] = true;
  for (int r = 0; r < q; ++r) {
    int d = 0;
    while (!read[mod_pos(r - d, q)]) ++d;
    t->back[r] = d;
  }
  int n = 0;
  for (int r = 0; r < q; ++r) {
    t->emit_start[r] = n;
    for (int j = 0; j < p; ++j)
      if (mod_pos(t->off[j] + T - 1, q) == r) t->emit_list[n++] = j;
  }
  t->emit_start[q] = n;
  return FCFS_OK;
}

// Upper bound of the adjoint-table entries of any input index of an axis of
// length n with `cells` hidden cells: (most (phase, tap) pairs that read one
// extended position) x (most extended positions the padding maps onto one
// input index).
// Most (phase, tap) pairs that read one extended position.
static int adjoint_per_position(const AxisTable& t) {
  int per_pos = 0;
  for (int r = 0; r < t.q; ++r) {
    int c = 0;
    for (int j = 0; j < t.p; ++j)
      for (int k = 0; k < t.T; ++k)
        if (mod_pos(t.off[j] + k - r, t.q) == 0) ++c;
    per_pos = std::max(per_pos, c);
  }
  return per_pos;
}

static int adjoint_cmax(const AxisTable& t, int n, int cells, int pad) {
  int per_pos = 0;
  for (int r = 0; r < t.q; ++r) {
    int c = 0;
    for (int j = 0; j < t.p; ++j)
      for (int k = 0; k < t.T; ++k)
        if (mod_pos(t.off[j] + k - r, t.q) == 0) ++c;
    per_pos = std::max(per_pos, c);
  }
  const int64_t emax = (int64_t)t.q * (cells - 1) + t.omax;
  int64_t outside = std::max<int64_t>(0, -(int64_t)t.omin) + std::max<int64_t>(0, emax - n + 1);
  int64_t positions = pad == FCFS_PAD_ZERO ? 1 : 1 + outside;
  return (int)std::min<int64_t>((int64_t)per_pos * positions, 1 << 20);
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }


// The (phase, tap) pairs of each residue class of an axis's extended index,
// for the channel-mixing input gradient: e = q u + r is read by tap t of
// phase j in cell u - d when off[j] + t = r + q d. Also the range of d.
static void mix_residue_lists(const AxisTable& t, int* start, int* list, int* dmin, int* dmax) {
  int k = 0;
  *dmin = 1 << 20;
  *dmax = -(1 << 20);
  for (int r = 0; r < t.q; ++r) {
    start[r] = k;
    for (int j = 0; j < t.p; ++j)
      for (int tap = 0; tap < 4; ++tap) {
        const int s = t.off[j] + tap - r;
        if (mod_pos(s, t.q) != 0) continue;
        const int d = (int)floor_div(s, t.q);
        list[k++] = j | tap << 5 | (d + 64) << 7;
        *dmin = std::min(*dmin, d);
        *dmax = std::max(*dmax, d);
      }
  }
  start[t.q] = k;
}

// Fills the size-dependent fields of the backward arguments and returns the
// workspace layout: [height table][width table][weight-gradient partials].
static fcfs_status plan_backward(const fcfs_plan_* plan, int64_t n, int64_t c, int64_t c_out, int h, int w,
                                 int ho, int wo, bool need_dw, BwdArgs* a, size_t* ws_bytes, size_t* off_w,
                                 size_t* off_p) {
  a->planes = n * c;
  a->planes_n = (int)n;
  a->Cout = (int)c_out;
  a->C = (int)c;
  a->H = h;
  a->W = w;
  a->Ho = ho;
  a->Wo = wo;
  a->Mh = ho / plan->ah.p;
  a->Mw = wo / plan->aw.p;
  a->pad = plan->pad;
  a->th = plan->ah;
  a->tw_tab = plan->aw;
  a->col_blocks = (w + 255) / 256;
  a->cmax_h = adjoint_cmax(plan->ah, h, a->Mh, plan->pad);
  a->cmax_w = adjoint_cmax(plan->aw, w, a->Mw, plan->pad);
  a->fast_w = adjoint_per_position(plan->aw);
  size_t bytes = align256(sizeof(int) * (size_t)h * (3 + a->cmax_h));
  *off_w = bytes;
  bytes += align256(sizeof(int) * (size_t)w * (3 + a->cmax_w));
  *off_p = bytes;
  if (plan->method == FCFS_LEARNED_MIX4) {
    // no adjoint tables: the workspace is [weight-gradient partials][input
    // gradient's buffers][weight gradient's buffers]
    bytes = 0;
    *off_w = 0;
    *off_p = 0;
    const int64_t rows = n * (int64_t)a->Mh;
    const AxisTable &th = plan->ah, &tw = plan->aw;
    a->mix_opad = (int)((c_out + 31) / 32 * 32);
    a->mix_cpad = (int)((c + 63) / 64 * 64);
    // weight gradient on MFMA: dy by phase and x by tap offset, cells in
    // blocks of 32; chunks of cell rows for about 4096 workgroups (2048 and
    // 8192 ran 3-5% slower at 16x64x512^2, 5/4)
    a->mix_dwopad = (int)((c_out + 63) / 64 * 64);
    a->mix_ncb = (a->Mw + 31) / 32;
    a->mix_s0 = tw.omin;
    a->mix_ns = tw.omax - tw.omin + 1;
    a->mix_dwcells = std::max(8, std::min(64, (256 / tw.p) / 8 * 8));
    a->mix_dwxcells = tw.q <= 4 ? 64 : (tw.q <= 8 ? 32 : 8);
    const int64_t per_chunk = (int64_t)th.p * tw.p * 4 * (a->mix_dwopad / 64) * (a->mix_cpad / 64);
#ifndef FCFS_MIX_DW_WORKGROUPS
#define FCFS_MIX_DW_WORKGROUPS 4096
#endif
    a->mix_wchunks = (int)std::max<int64_t>(
        1, std::min<int64_t>(rows, (FCFS_MIX_DW_WORKGROUPS + per_chunk - 1) / per_chunk));
    const int64_t erows = (int64_t)th.q * (a->Mh - 1) + th.omax - th.omin + 1;
    const int64_t dyw_elems = n * (int64_t)ho * tw.p * a->mix_ncb * 32 * a->mix_dwopad;
    const int64_t xa_elems = n * erows * a->mix_ns * a->mix_ncb * 32 * a->mix_cpad;
    const int64_t ncb32 = (int64_t)a->mix_ncb * 32;
    // every grid within 2^31 workgroups
    const int64_t lim = 1LL << 31;
    if (need_dw && (per_chunk * a->mix_wchunks >= lim ||
                    n * ho * ((ncb32 + a->mix_dwcells - 1) / a->mix_dwcells) * (a->mix_dwopad / 64) >= lim ||
                    n * erows * ((ncb32 + a->mix_dwxcells - 1) / a->mix_dwxcells) * (a->mix_cpad / 64) >= lim ||
                    ((int64_t)th.p * tw.p * 16 * c_out * c + 255) / 256 >= lim))
      return FCFS_E_UNSUPPORTED;
    if (need_dw) bytes += align256(sizeof(float) * (size_t)a->mix_wchunks * th.p * tw.p * a->Cout * c * 16);
    // input gradient on MFMA: channel-last dy, packed weights and the edge
    // buffer (the offsets follow the partial sums)
    int dhmin, dhmax, dwmin, dwmax;
    mix_residue_lists(th, a->mix_hl_start, a->mix_hl, &dhmin, &dhmax);
    mix_residue_lists(tw, a->mix_wl_start, a->mix_wl, &dwmin, &dwmax);
    // the extended positions the taps read, and the GEMM's range: those and
    // every input sample (samples no tap reads get 0)
    a->mix_eh0 = th.omin;
    a->mix_eh1 = th.q * (a->Mh - 1) + th.omax;
    a->mix_ew0 = tw.omin;
    a->mix_ew1 = tw.q * (a->Mw - 1) + tw.omax;
    a->mix_r0 = std::min(a->mix_eh0, 0);
    a->mix_rows = std::max(a->mix_eh1 + 1, h) - a->mix_r0;
    a->mix_v0 = (int)std::min<int64_t>(floor_div(a->mix_ew0, tw.q), 0);
    const int64_t v1 = std::max<int64_t>(floor_div(a->mix_ew1, tw.q) + 1, (w + tw.q - 1) / tw.q);
    a->mix_vw = (int)(v1 - a->mix_v0);
    // a workgroup takes every width class of kw chunks of 16 mtn positions
    // (one chunk per wave when q_w <= 4)
    const int chunks = (a->mix_vw + 63) / 64;
    a->mix_mtn = (a->mix_vw + 16 * chunks - 1) / (16 * chunks);
    a->mix_kw = tw.q >= 4 ? 1 : 4 / tw.q;
    a->mix_vgroups = (chunks + a->mix_kw - 1) / a->mix_kw;
    a->mix_vchunks = a->mix_vgroups * a->mix_kw;
    a->mix_lds_epi = tw.q * a->mix_kw <= 8;
    // dy cells the A rows reach: v - d for v in the chunks and every d
    const int64_t vend = a->mix_v0 + (int64_t)a->mix_vchunks * 16 * a->mix_mtn;
    a->mix_dleft = std::max(0, dwmax - a->mix_v0);
    const int64_t dright = std::max<int64_t>(0, vend - 1 - dwmin - (a->Mw - 1));
    const int64_t dcells = a->mix_dleft + a->Mw + dright;
    a->mix_dcells = (int)std::min<int64_t>(dcells, 1 << 30);
    a->mix_clcells = std::max(1, kDxcColumns / tw.p);
    // fold zones of replicate / reflect: the samples the margins copy (every
    // sample of an axis short enough for a reflection to wrap)
    auto zone = [&](int len, int e0, int e1, int* lo, int* hi) {
      const int lm = std::max(0, -e0), rm = std::max(0, e1 - (len - 1));
      if (plan->pad == FCFS_PAD_ZERO) {
        *lo = *hi = 0;
      } else if (len <= lm + rm + 2) {
        *lo = len;
        *hi = 0;
      } else {
        *lo = lm + 1;
        *hi = rm + 1;
      }
    };
    zone(h, a->mix_eh0, a->mix_eh1, &a->mix_top, &a->mix_bot);
    zone(w, a->mix_ew0, a->mix_ew1, &a->mix_cl, &a->mix_cr);
    const int64_t ec0 = (int64_t)tw.q * a->mix_v0, ecols = (int64_t)tw.q * a->mix_vw;
    a->mix_rr = (int)((a->mix_top - a->mix_r0) + (a->mix_r0 + a->mix_rows - (h - a->mix_bot)));
    a->mix_cc = (int)((a->mix_cl - ec0) + (ec0 + ecols - (w - a->mix_cr)));
    a->mix_edge_c = (int64_t)a->mix_rr * ecols;
    a->mix_edge_per = (int64_t)(a->mix_top + a->mix_bot) * w + (int64_t)(h - a->mix_top - a->mix_bot) * (a->mix_cl + a->mix_cr);
    const int64_t gemm_blocks = n * (int64_t)a->mix_rows * a->mix_vgroups * (a->mix_cpad / 64);
    const int64_t edge_blocks = (n * c * a->mix_edge_per + 255) / 256;
    const int64_t dyc_row = dcells * tw.p * a->mix_opad;
    const int64_t cl_blocks = n * ho * ((dcells + a->mix_clcells - 1) / a->mix_clcells);
    const int64_t wpk_elems = (int64_t)th.p * tw.p * 16 * a->mix_cpad * a->mix_opad;
    if (gemm_blocks >= lim || edge_blocks >= lim || cl_blocks >= lim || (wpk_elems + 255) / 256 >= lim ||
        dcells * kMaxFactor * 32 >= lim)
      return FCFS_E_UNSUPPORTED;
    a->mix_ws_dyc = bytes;
    bytes += align256(sizeof(uint16_t) * (size_t)n * ho * dyc_row);
    a->mix_ws_wpk = bytes;
    bytes += align256(sizeof(uint16_t) * (size_t)wpk_elems);
    a->mix_ws_edge = bytes;
    if (plan->pad != FCFS_PAD_ZERO)
      bytes += align256(sizeof(float) * (size_t)n * c * (a->mix_edge_c + (int64_t)a->mix_rows * a->mix_cc));
    if (need_dw) {
      a->mix_ws_dyw = bytes;
      bytes += align256(sizeof(uint16_t) * (size_t)dyw_elems);
      a->mix_ws_xa = bytes;
      bytes += align256(sizeof(uint16_t) * (size_t)xa_elems);
    }
    *ws_bytes = bytes;
    return FCFS_OK;
  }
  if (need_dw) {
    // chunks of ch x cw cells: staged x patch within 8192 floats
    const AxisTable &th = plan->ah, &tw = plan->aw;
    const int P2 = th.p * tw.p;
    int side = 16;
    auto lds_floats = [&](int ch, int cw) {
      const int xr = th.q * (ch - 1) + th.omax - th.omin + 1, xc = tw.q * (cw - 1) + tw.omax - tw.omin + 1;
      return std::max(th.p * ch * tw.p * cw + xr * xc, (256 / P2) * P2 * 16);   // the sums reuse the patches' space
    };
    while (side > 1 && lds_floats(side, side) > 14336) --side;
    a->ch = std::min(side, a->Mh);
    a->cw = std::min(side, a->Mw);
    a->nch = (a->Mh + a->ch - 1) / a->ch;
    a->ncw = (a->Mw + a->cw - 1) / a->cw;
    int64_t cpc = n * (int64_t)a->nch * a->ncw;
    if (cpc > (1 << 30)) return FCFS_E_UNSUPPORTED;
    a->chunks_per_channel = (int)cpc;
    a->dw_lds_bytes = (int)(sizeof(float) * lds_floats(a->ch, a->cw));
    if (a->dw_lds_bytes > 65536) return FCFS_E_UNSUPPORTED;
    bytes += align256(sizeof(float) * (size_t)c * cpc * P2 * 16);
  }
  *ws_bytes = bytes;
  return FCFS_OK;
}

}  // namespace fcfs

using namespace fcfs;

extern "C" {

fcfs_status fcfs_plan_ex(int p_h, int q_h, int p_w, int q_w, fcfs_method method, fcfs_pad pad,
                         fcfs_grid grid, fcfs_plan_t* out) {
  if (!out) return FCFS_E_INVAL;
  *out = nullptr;
  if (p_h < 1 || q_h < 1 || p_w < 1 || q_w < 1) return FCFS_E_INVAL;
  if ((int)method < FCFS_NEAREST || (int)method > FCFS_LEARNED_MIX4) return FCFS_E_INVAL;
  if ((int)pad < FCFS_PAD_ZERO || (int)pad > FCFS_PAD_REFLECT) return FCFS_E_INVAL;
  if ((int)grid < FCFS_GRID_HALF || (int)grid > FCFS_GRID_ASYM) return FCFS_E_INVAL;
  fcfs_plan_* pl = new (std::nothrow) fcfs_plan_();
  if (!pl) return FCFS_E_NOMEM;
  pl->method = method;
  pl->pad = pad;
  pl->grid = grid;
  fcfs_status st = build_axis(p_h, q_h, method, grid, true, &pl->ah);
  if (st == FCFS_OK) st = build_axis(p_w, q_w, method, grid, true, &pl->aw);
  // (Only the 1/1 copy shortcut makes the axes' tap counts differ; the
  // forward kernel has instances for a copying height or width axis.)
  if (st != FCFS_OK) {
    delete pl;
    return st;
  }
  *out = pl;
  return FCFS_OK;
}

fcfs_status fcfs_plan(int p, int q, fcfs_method method, fcfs_pad pad, fcfs_plan_t* out) {
  return fcfs_plan_ex(p, q, p, q, method, pad, FCFS_GRID_HALF, out);
}

fcfs_status fcfs_plan_destroy(fcfs_plan_t plan) {
  delete plan;
  return FCFS_OK;
}

fcfs_status fcfs_plan_query(fcfs_plan_t plan, int* p_red, int* q_red, int* taps) {
  if (!plan) return FCFS_E_INVAL;
  if (p_red) *p_red = plan->ah.p;
  if (q_red) *q_red = plan->ah.q;
  if (taps) *taps = std::max(plan->ah.T, plan->aw.T);
  return FCFS_OK;
}

fcfs_status fcfs_plan_taps(fcfs_plan_t plan, int axis, int phase, int* first_offset, float* w) {
  if (!plan || !first_offset || !w || (axis != 0 && axis != 1)) return FCFS_E_INVAL;
  const AxisTable& t = axis == 0 ? plan->ah : plan->aw;
  if (phase < 0 || phase >= t.p) return FCFS_E_INVAL;
  *first_offset = t.off[phase];
  for (int k = 0; k < 4; ++k) w[k] = k < t.T ? t.w[phase][k] : 0.f;
  return FCFS_OK;
}

fcfs_status fcfs_output_size(fcfs_plan_t plan, int64_t h, int64_t w, int64_t* h_out, int64_t* w_out) {
  if (!plan || h < 1 || w < 1) return FCFS_E_INVAL;
  const int64_t cells_h = (h + plan->ah.q - 1) / plan->ah.q;
  const int64_t cells_w = (w + plan->aw.q - 1) / plan->aw.q;
  if (h_out) *h_out = plan->ah.p * cells_h;
  if (w_out) *w_out = plan->aw.p * cells_w;
  return FCFS_OK;
}

static fcfs_status check_common(fcfs_plan_t plan, fcfs_dtype dtype, int64_t n, int64_t c_in, int64_t h,
                                 int64_t w, int64_t c_out, int64_t* ho, int64_t* wo) {
  if (!plan) return FCFS_E_INVAL;
  if ((int)dtype < FCFS_F32 || (int)dtype > FCFS_F16) return FCFS_E_INVAL;
  if (n < 0 || c_in < 0 || h < 0 || w < 0 || c_out < 0) return FCFS_E_INVAL;
  if (plan->method != FCFS_LEARNED_MIX4 && c_out != c_in) return FCFS_E_INVAL;
  *ho = plan->ah.p * ((h + plan->ah.q - 1) / plan->ah.q);
  *wo = plan->aw.p * ((w + plan->aw.q - 1) / plan->aw.q);
  int64_t in_plane, out_plane, tmp;
  if (!mul_ok(h, w, &in_plane) || !mul_ok(*ho, *wo, &out_plane)) return FCFS_E_UNSUPPORTED;
  if (in_plane >= (1LL << 31) || out_plane >= (1LL << 31) || *ho >= (1LL << 31) || *wo >= (1LL << 31))
    return FCFS_E_UNSUPPORTED;
  if (!mul_ok(n, c_in, &tmp) || !mul_ok(tmp, in_plane, &tmp)) return FCFS_E_INVAL;
  if (!mul_ok(n, c_out, &tmp) || !mul_ok(tmp, out_plane, &tmp)) return FCFS_E_INVAL;
  if (c_in >= (1LL << 31) || c_out >= (1LL << 31)) return FCFS_E_UNSUPPORTED;
  return FCFS_OK;
}

// Channel-mixing layer, FP32 storage: the largest group of at most 5 width
// phases whose taps span at most 8 columns per cell.
static fcfs_status forward_mix4_f32(fcfs_plan_t plan, const MixArgs& base, hipStream_t stream) {
  MixArgs a = base;
  const AxisTable& tw = plan->aw;
  int G = std::min(5, tw.p), wspan = 0;
  for (; G >= 1; --G) {
    int spread = 0;
    for (int j0 = 0; j0 < tw.p; j0 += G) {
      const int j1 = std::min(tw.p, j0 + G) - 1;
      spread = std::max(spread, tw.off[j1] - tw.off[j0]);
    }
    wspan = spread + 4;
    if (wspan <= 8) break;
  }
  a.gsize = G;
  a.groups = (tw.p + G - 1) / G;
  a.wspan = wspan;
  a.tiles_h = (a.Mh + 3) / 4;
  a.tiles_w = (a.Mw + 15) / 16;
  a.otiles = (a.Cout + 63) / 64;
  const int64_t blocks = (int64_t)a.N * a.tiles_h * a.tiles_w * plan->ah.p * a.groups * a.otiles;
  if (blocks >= (1LL << 31)) return FCFS_E_UNSUPPORTED;
  return launch_mix4_f32(a, stream);
}

// Channel-mixing layer: weights in the storage type; 16-bit storage on the
// 16-bit matrix cores, FP32 storage on the FP32 ones.
static fcfs_status forward_mix4(fcfs_plan_t plan, fcfs_dtype dtype, int64_t n, int64_t c_in, int64_t h,
                                int64_t w, int64_t ho, int64_t wo, const void* x, const void* weight,
                                int64_t c_out, void* y, hipStream_t stream) {
  if ((reinterpret_cast<uintptr_t>(weight) & 15) != 0) return FCFS_E_INVAL;
  if (n > INT32_MAX || c_in > INT32_MAX || c_out > INT32_MAX) return FCFS_E_UNSUPPORTED;
  MixArgs a;
  std::memset(&a, 0, sizeof(a));
  a.x = x;
  a.w = weight;
  a.y = y;
  a.N = (int)n;
  a.Cin = (int)c_in;
  a.Cout = (int)c_out;
  a.H = (int)h;
  a.W = (int)w;
  a.Ho = (int)ho;
  a.Wo = (int)wo;
  a.Mh = (int)(ho / plan->ah.p);
  a.Mw = (int)(wo / plan->aw.p);
  a.pad = plan->pad;
  a.th = plan->ah;
  a.tw_tab = plan->aw;
  if (dtype == FCFS_F32) return forward_mix4_f32(plan, a, stream);
  const int P = std::min(5, plan->aw.p);   // width phases per group
  a.gsize = P;
  a.groups = (plan->aw.p + P - 1) / P;
  a.otiles = (int)((c_out + kMixOut - 1) / kMixOut);
  int spread = 0;
  for (int g = 0; g < a.groups; ++g) {
    const int j0 = g * P, j1 = std::min(plan->aw.p, j0 + P) - 1;
    spread = std::max(spread, plan->aw.off[j1] - plan->aw.off[j0]);
  }
  // The channel-last kernel: 4 x 32 cells, 16 patch rows (the 4 tap rows of
  // each cell row), Cc columns of 8-channel pixels (plus one of shift to an
  // even start) held in cstep residue classes of S slots, a spare slot, and
  // a row pitch of 16 mod 32 slots (the half-wave reading two rows then
  // covers all 128 LDS banks once), within the 160 KB of LDS a gfx950
  // workgroup may use.
  {
    const int wspan0 = spread + 4;
    const int cstep = plan->aw.q < wspan0 ? plan->aw.q : wspan0;
    const int Cc = cstep * 31 + wspan0;
    const int S = (Cc + 1 + cstep - 1) / cstep;
    int CPX = cstep * S + 1;
    CPX += ((16 - CPX) % 32 + 32) % 32;
    const int buf_u16 = 16 * CPX * 8 + P * 4 * kMixOut * 4 * 8;
    const size_t lds = sizeof(uint16_t) * (size_t)buf_u16;
    if (Cc + 1 <= 3 * 64 && lds <= 163840 && 2 * c_in * h * w < (int64_t)1 << 31) {
      a.cl = 1;
      a.xpair = cstep == plan->aw.q && (w % 2 == 0) && (reinterpret_cast<uintptr_t>(x) & 3) == 0;
      a.fixed = 1;
      for (int g = 0; g < a.groups; ++g)
        for (int j = g * P; j < std::min(plan->aw.p, g * P + P); ++j)
          if (plan->aw.off[j] - plan->aw.off[g * P] != j - g * P) a.fixed = 0;
      a.th_cells = 4;
      a.tw_cells = 32;
      a.rstep = 4;
      a.R = 16;
      a.wspan = wspan0;
      a.cstep = cstep;
      a.Cc = Cc;
      a.CP = CPX;
      a.slots = S;
      a.buf_u16 = buf_u16;
      a.nbuf = 1;
      a.lds_bytes = (int)lds;
      a.tiles_h = (a.Mh + 3) / 4;
      a.tiles_w = (a.Mw + 31) / 32;
      const int64_t blocks = n * (int64_t)a.tiles_h * a.tiles_w * plan->ah.p * a.groups * a.otiles;
      if (blocks >= (1LL << 31)) return FCFS_E_UNSUPPORTED;
      return launch_mix4(dtype, a, stream);
    }
  }
  // Cell tile: 128 cells. The first shape whose staged patch travels in
  // registers (at most 8 (channel, row) pairs per wave and 3 column slots of
  // 64) with two stage buffers in 64 KB of LDS (the pipelined kernel); else
  // the first whose one buffer fits (the kernel that stages between steps).
  const int qh = plan->ah.q, qw = plan->aw.q;
  const int wspan = spread + 4;
  static const int shapes[][2] = {{4, 32}, {8, 16}, {2, 64}, {16, 8}, {1, 128}, {32, 4}, {64, 2}, {128, 1}};
  bool found = false;
  for (int pass = 0; pass < 2 && !found; ++pass) {
    for (const auto& sh : shapes) {
      MixArgs t = a;
      t.th_cells = sh[0];
      t.tw_cells = sh[1];
      t.rstep = std::min(qh, 4);
      t.R = t.rstep * (t.th_cells - 1) + 4;
      t.wspan = wspan;
      t.cstep = qw < wspan ? qw : wspan;
      t.Cc = t.cstep * (t.tw_cells - 1) + wspan;
      t.CP = (t.Cc + 1) | 1;   // a spare column; odd pitch: neighbouring rows start in different banks
      t.npr = (2 * t.R + 3) / 4;
      t.ncs = (t.Cc + 63) / 64;
      t.items = t.npr * t.ncs;
      t.woff_u16 = (2 * t.R * t.CP + 7) & ~7;
      t.buf_u16 = t.woff_u16 + P * kMixOut * 32 + 8;   // + a spare quad
      t.nbuf = pass == 0 ? 2 : 1;
      const size_t epi = sizeof(uint16_t) * 16 * (size_t)t.th_cells * t.tw_cells * P;
      const size_t lds = std::max(sizeof(uint16_t) * t.nbuf * (size_t)t.buf_u16, epi);
      const bool regs = t.npr <= 8 && t.ncs <= 3;
      if (lds > 65536 || (pass == 0 && !regs)) continue;
      t.lds_bytes = (int)lds;
      a = t;
      found = true;
      break;
    }
  }
  if (!found) return FCFS_E_UNSUPPORTED;
  a.tiles_h = (a.Mh + a.th_cells - 1) / a.th_cells;
  a.tiles_w = (a.Mw + a.tw_cells - 1) / a.tw_cells;
  const int64_t blocks = n * (int64_t)a.tiles_h * a.tiles_w * plan->ah.p * a.groups * a.otiles;
  if (blocks >= (1LL << 31)) return FCFS_E_UNSUPPORTED;
  return launch_mix4(dtype, a, stream);
}

fcfs_status fcfs_forward(fcfs_plan_t plan, fcfs_dtype dtype, int64_t n, int64_t c_in, int64_t h,
                         int64_t w, const void* x, const void* weight, int64_t c_out, void* y,
                         hipStream_t stream) {
  int64_t ho = 0, wo = 0;
  fcfs_status st = check_common(plan, dtype, n, c_in, h, w, c_out, &ho, &wo);
  if (st != FCFS_OK) return st;
  const bool learned = plan->method == FCFS_LEARNED_DW4 || plan->method == FCFS_LEARNED_MIX4;
  if (n == 0 || c_in == 0 || c_out == 0 || h == 0 || w == 0) return FCFS_OK;   // nothing to do
  if (!x || !y) return FCFS_E_INVAL;
  if (learned != (weight != nullptr)) return FCFS_E_INVAL;
  if (plan->method == FCFS_LEARNED_MIX4) return forward_mix4(plan, dtype, n, c_in, h, w, ho, wo, x, weight, c_out, y, stream);
  if (plan->method == FCFS_LEARNED_DW4 && plan->ah.p * plan->aw.p > 64) return FCFS_E_UNSUPPORTED;

  FwdArgs a;
  std::memset(&a, 0, sizeof(a));
  a.x = x;
  a.y = y;
  a.weight = static_cast<const float*>(weight);
  a.planes = n * c_in;
  a.C = (int)c_in;
  a.H = (int)h;
  a.W = (int)w;
  a.Ho = (int)ho;
  a.Wo = (int)wo;
  a.Mh = (int)(ho / plan->ah.p);
  a.pad = plan->pad;
  a.th = plan->ah;
  a.tw_tab = plan->aw;
  fill_emit(plan->ah, a.emit);
  // 16-bit samples can move two per dword when every row starts 4-byte aligned
  const bool pair_ok = dtype != FCFS_F32 && w % 2 == 0 && wo % 2 == 0 &&
                       (reinterpret_cast<uintptr_t>(x) & 3) == 0 && (reinterpret_cast<uintptr_t>(y) & 3) == 0;
  FwdGeom g;
  st = plan_forward_geom(plan, dtype, a.planes, a.H, a.W, a.Ho, a.Wo, pair_ok, &g);
  if (st != FCFS_OK) return st;
  a.tw = g.tw;
  a.strips = g.strips;
  a.band_cells = g.band_cells;
  a.bands = g.bands;
  a.waves = g.waves;
  if (g.waves <= 0) return FCFS_OK;
  switch (dtype) {
    case FCFS_F32: return launch_forward_f32(plan->method, a, g, stream);
    case FCFS_BF16: return launch_forward_bf16(plan->method, a, g, stream);
    default: return launch_forward_f16(plan->method, a, g, stream);
  }
}

fcfs_status fcfs_forward_1d(fcfs_plan_t plan, fcfs_dtype dtype, int64_t n, int64_t c, int64_t l,
                            const void* x, void* y, hipStream_t stream) {
  if (!plan) return FCFS_E_INVAL;
  if (plan->ah.p != 1 || plan->ah.q != 1) return FCFS_E_INVAL;
  if (plan->method == FCFS_LEARNED_DW4 || plan->method == FCFS_LEARNED_MIX4) return FCFS_E_INVAL;
  // the 1/1 height axis must sample its row exactly, which the paper grid's
  // half-sample offset does not
  if (plan->grid == FCFS_GRID_PAPER) return FCFS_E_UNSUPPORTED;
  if (n < 0 || c < 0 || l < 0) return FCFS_E_INVAL;
  // The height axis copies its rows, so the n*c signals can be the rows of
  // one plane (streamed in bands like an image) while that plane fits the
  // kernel's 32-bit in-plane indexing; else one row per plane.
  const int64_t wo = plan->aw.p * ((l + plan->aw.q - 1) / plan->aw.q);
  if (n * c * std::max(l, wo) < ((int64_t)1 << 31))
    return fcfs_forward(plan, dtype, 1, 1, n * c, l, x, nullptr, 1, y, stream);
  return fcfs_forward(plan, dtype, n, c, 1, l, x, nullptr, c, y, stream);
}

namespace {

// The two passes of a 3D forward: which one runs first and the intermediate's
// elements. HW first leaves [n][c][d][h_out][w_out]; D first [n][c][d_out][h][w].
struct Plan3d {
  int64_t d_out, h_out, w_out;
  bool hw_first;
  int64_t inter;
};

fcfs_status plan_3d(fcfs_plan_t plan_d, fcfs_plan_t plan_hw, fcfs_dtype dtype, int64_t n, int64_t c, int64_t d,
                    int64_t h, int64_t w, Plan3d* o) {
  if (!plan_d || !plan_hw) return FCFS_E_INVAL;
  if ((int)dtype < FCFS_F32 || (int)dtype > FCFS_F16) return FCFS_E_INVAL;
  if (n < 0 || c < 0 || d < 0 || h < 0 || w < 0) return FCFS_E_INVAL;
  const auto learned = [](fcfs_plan_t p) {
    return p->method == FCFS_LEARNED_DW4 || p->method == FCFS_LEARNED_MIX4;
  };
  if (learned(plan_d) || learned(plan_hw)) return FCFS_E_INVAL;
  if (plan_d->method != plan_hw->method || plan_d->pad != plan_hw->pad || plan_d->grid != plan_hw->grid)
    return FCFS_E_INVAL;
  if (plan_d->aw.p != 1 || plan_d->aw.q != 1) return FCFS_E_INVAL;
  // the depth pass's 1/1 width axis must copy, which the paper grid's
  // half-sample offset does not
  if (plan_d->grid == FCFS_GRID_PAPER) return FCFS_E_UNSUPPORTED;
  const int64_t pd = plan_d->ah.p, qd = plan_d->ah.q;
  o->d_out = pd * ((d + qd - 1) / qd);
  o->h_out = plan_hw->ah.p * ((h + plan_hw->ah.q - 1) / plan_hw->ah.q);
  o->w_out = plan_hw->aw.p * ((w + plan_hw->aw.q - 1) / plan_hw->aw.q);
  const int64_t a = n * c * d * o->h_out * o->w_out, b = n * c * o->d_out * h * w;
  o->hw_first = a <= b;
  o->inter = o->hw_first ? a : b;
  return FCFS_OK;
}

}  // namespace

fcfs_status fcfs_forward_3d_workspace(fcfs_plan_t plan_d, fcfs_plan_t plan_hw, fcfs_dtype dtype, int64_t n,
                                      int64_t c, int64_t d, int64_t h, int64_t w, size_t* bytes) {
  if (!bytes) return FCFS_E_INVAL;
  *bytes = 0;
  Plan3d g;
  fcfs_status st = plan_3d(plan_d, plan_hw, dtype, n, c, d, h, w, &g);
  if (st != FCFS_OK) return st;
  *bytes = (size_t)g.inter * (dtype == FCFS_F32 ? 4 : 2);
  return FCFS_OK;
}

fcfs_status fcfs_forward_3d(fcfs_plan_t plan_d, fcfs_plan_t plan_hw, fcfs_dtype dtype, int64_t n, int64_t c,
                            int64_t d, int64_t h, int64_t w, const void* x, void* y, void* workspace,
                            size_t ws_bytes, hipStream_t stream) {
  Plan3d g;
  fcfs_status st = plan_3d(plan_d, plan_hw, dtype, n, c, d, h, w, &g);
  if (st != FCFS_OK) return st;
  if (n == 0 || c == 0 || d == 0 || h == 0 || w == 0) return FCFS_OK;
  if (!x || !y || !workspace) return FCFS_E_INVAL;
  if (ws_bytes < (size_t)g.inter * (dtype == FCFS_F32 ? 4 : 2)) return FCFS_E_INVAL;
  if (g.hw_first) {
    // planes [n*c*d][h][w] -> workspace [n*c][d][h_out*w_out] -> y [n*c][d_out][h_out*w_out]
    st = fcfs_forward(plan_hw, dtype, n * c * d, 1, h, w, x, nullptr, 1, workspace, stream);
    if (st != FCFS_OK) return st;
    return fcfs_forward(plan_d, dtype, n * c, 1, d, g.h_out * g.w_out, workspace, nullptr, 1, y, stream);
  }
  // [n*c][d][h*w] -> workspace [n*c][d_out][h*w] = planes [n*c*d_out][h][w] -> y
  st = fcfs_forward(plan_d, dtype, n * c, 1, d, h * w, x, nullptr, 1, workspace, stream);
  if (st != FCFS_OK) return st;
  return fcfs_forward(plan_hw, dtype, n * c * g.d_out, 1, h, w, workspace, nullptr, 1, y, stream);
}

fcfs_status fcfs_forward_config(fcfs_plan_t plan, fcfs_dtype dtype, int64_t n, int64_t c_in,
                                int64_t h, int64_t w, int* kernel_id, int* strip_width,
                                int* band_cells, int64_t* waves) {
  int64_t ho = 0, wo = 0;
  const int64_t c_out = (plan && plan->method == FCFS_LEARNED_MIX4) ? 1 : c_in;
  fcfs_status st = check_common(plan, dtype, n, c_in, h, w, c_out, &ho, &wo);
  if (st != FCFS_OK) return st;
  FwdGeom g;
  std::memset(&g, 0, sizeof(g));
  if (n > 0 && c_in > 0 && h > 0 && w > 0) {
    const bool pair_ok = dtype != FCFS_F32 && w % 2 == 0 && wo % 2 == 0;   // tensors taken 4-byte aligned
    st = plan_forward_geom(plan, dtype, n * c_in, (int)h, (int)w, (int)ho, (int)wo, pair_ok, &g);
    if (st != FCFS_OK) return st;
  }
  int id = (int)dtype * 1000 + std::max(plan->ah.T, plan->aw.T) * 100 + g.kc * 10 + g.slots;
  if (g.paired) id += 50000;
  if (plan->ah.T < plan->aw.T) id += 100000;   // the height axis copies
  if (plan->aw.T < plan->ah.T) id += 200000;   // the width axis copies
  if (plan->method == FCFS_LEARNED_DW4) id += 10000;
  if (plan->method == FCFS_LEARNED_MIX4) id += 20000;
  if (kernel_id) *kernel_id = id;
  if (strip_width) *strip_width = g.tw;
  if (band_cells) *band_cells = g.band_cells;
  if (waves) *waves = g.waves;
  return FCFS_OK;
}

static fcfs_status backward_checks(fcfs_plan_t plan, fcfs_dtype dtype, int64_t n, int64_t c_in,
                                   int64_t h, int64_t w, int64_t c_out, bool need_dw, int64_t* ho,
                                   int64_t* wo) {
  fcfs_status st = check_common(plan, dtype, n, c_in, h, w, c_out, ho, wo);
  if (st != FCFS_OK) return st;
  if (plan->method == FCFS_LEARNED_MIX4 && dtype == FCFS_F32) return FCFS_E_UNSUPPORTED;
  if (plan->method == FCFS_LEARNED_DW4 && plan->ah.p * plan->aw.p > 64) return FCFS_E_UNSUPPORTED;
  if (need_dw && plan->method != FCFS_LEARNED_DW4 && plan->method != FCFS_LEARNED_MIX4) return FCFS_E_INVAL;
  if (*ho >= (1 << 24) || *wo >= (1 << 24)) return FCFS_E_UNSUPPORTED;   // adjoint table entries pack k < 2^24
  return FCFS_OK;
}

}  // extern "C"

namespace fcfs {

fcfs_status backward_workspace_need(fcfs_plan_t plan, fcfs_dtype dtype, int64_t n, int64_t c_in, int64_t h,
                                    int64_t w, int64_t c_out, bool need_dw, size_t* bytes) {
  int64_t ho = 0, wo = 0;
  if (!bytes) return FCFS_E_INVAL;
  *bytes = 0;
  fcfs_status st = backward_checks(plan, dtype, n, c_in, h, w, c_out, need_dw, &ho, &wo);
  if (st != FCFS_OK) return st;
  if (n == 0 || c_in == 0 || h == 0 || w == 0) return FCFS_OK;
  BwdArgs a;
  std::memset(&a, 0, sizeof(a));
  size_t off_w, off_p;
  return plan_backward(plan, n, c_in, c_out, (int)h, (int)w, (int)ho, (int)wo, need_dw, &a, bytes, &off_w, &off_p);
}

}  // namespace fcfs

extern "C" {

fcfs_status fcfs_backward_workspace(fcfs_plan_t plan, fcfs_dtype dtype, int64_t n, int64_t c_in,
                                    int64_t h, int64_t w, int64_t c_out, size_t* bytes) {
  if (!bytes) return FCFS_E_INVAL;
  *bytes = 0;
  if (!plan) return FCFS_E_INVAL;
  // sized for the weight gradient too when the method has weights
  const bool learned = plan->method == FCFS_LEARNED_DW4 || plan->method == FCFS_LEARNED_MIX4;
  return backward_workspace_need(plan, dtype, n, c_in, h, w, c_out, learned, bytes);
}

fcfs_status fcfs_backward(fcfs_plan_t plan, fcfs_dtype dtype, int64_t n, int64_t c_in, int64_t h,
                          int64_t w, const void* x, const void* weight, int64_t c_out,
                          const void* dy, void* dx, float* dw, void* workspace, size_t ws_bytes,
                          hipStream_t stream) {
  int64_t ho = 0, wo = 0;
  fcfs_status st = backward_checks(plan, dtype, n, c_in, h, w, c_out, dw != nullptr, &ho, &wo);
  if (st != FCFS_OK) return st;
  const bool mix = plan->method == FCFS_LEARNED_MIX4;
  const bool learned = plan->method == FCFS_LEARNED_DW4 || mix;
  if (n == 0 || c_in == 0 || h == 0 || w == 0) {
    // no samples: the weight gradient is an empty sum
    if (dw) {
      const size_t count = (size_t)c_in * (mix ? c_out : 1) * plan->ah.p * plan->aw.p * 16;
      if (hipMemsetAsync(dw, 0, sizeof(float) * count, stream) != hipSuccess) return FCFS_E_DEVICE;
    }
    return FCFS_OK;
  }
  if (!dx && !dw) return FCFS_OK;
  if (!dy) return FCFS_E_INVAL;
  if (dx && learned && !weight) return FCFS_E_INVAL;
  if (dw && !x) return FCFS_E_INVAL;
  if (!learned && weight) return FCFS_E_INVAL;
  BwdArgs a;
  std::memset(&a, 0, sizeof(a));
  size_t need = 0, off_w = 0, off_p = 0;
  if (mix && dx && (reinterpret_cast<uintptr_t>(weight) & 15) != 0) return FCFS_E_INVAL;
  st = plan_backward(plan, n, c_in, c_out, (int)h, (int)w, (int)ho, (int)wo, dw != nullptr, &a, &need, &off_w,
                     &off_p);
  if (st != FCFS_OK) return st;
  if (!workspace || ws_bytes < need) return FCFS_E_INVAL;
  char* ws = static_cast<char*>(workspace);
  a.x = x;
  a.weight = static_cast<const float*>(weight);
  a.dy = dy;
  a.dx = dx;
  a.dw = dw;
  a.tab_h = reinterpret_cast<int*>(ws);
  a.tab_w = reinterpret_cast<int*>(ws + off_w);
  a.partial = dw ? reinterpret_cast<float*>(ws + off_p) : nullptr;
  if (mix) {
    a.weight = nullptr;
    a.mix_weight = weight;
    if (dx) {
      a.mix_dyc = reinterpret_cast<uint16_t*>(ws + a.mix_ws_dyc);
      a.mix_wpk = reinterpret_cast<uint16_t*>(ws + a.mix_ws_wpk);
      a.mix_edge = plan->pad != FCFS_PAD_ZERO ? reinterpret_cast<float*>(ws + a.mix_ws_edge) : nullptr;
    }
    if (dw) {
      a.mix_dyw = reinterpret_cast<uint16_t*>(ws + a.mix_ws_dyw);
      a.mix_xa = reinterpret_cast<uint16_t*>(ws + a.mix_ws_xa);
    }
    return dtype == FCFS_BF16 ? launch_backward_mix_bf16(a, stream) : launch_backward_mix_f16(a, stream);
  }
  switch (dtype) {
    case FCFS_F32: return launch_backward_f32(a, learned, stream);
    case FCFS_BF16: return launch_backward_bf16(a, learned, stream);
    default: return launch_backward_f16(a, learned, stream);
  }
}

const char* fcfs_status_string(fcfs_status s) {
  switch (s) {
    case FCFS_OK: return "ok";
    case FCFS_E_INVAL: return "invalid argument";
    case FCFS_E_UNSUPPORTED: return "unsupported";
    case FCFS_E_NOMEM: return "out of memory";
    case FCFS_E_DEVICE: return "device error";
    case FCFS_E_AGAIN: return "busy, try again";
    case FCFS_E_PENDING: return "pending";
    case FCFS_E_CANCELLED: return "cancelled";
  }
  return "unknown status";
}

int fcfs_version(void) { return 100; }

}  // extern "C"
