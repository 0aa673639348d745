// Forward launch planning: the height emission records and the launch
// geometry (strip width, column groups, staged slots, bands) of the fused
// forward kernel, for single launches and for the batched serving kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "fcfs_internal.h"

namespace fcfs {
namespace {

int mod_pos(int a, int q) {
  const int m = a % q;
  return m < 0 ? m + q : m;
}

}  // namespace

void fill_emit(const AxisTable& t, EmitRec* out) {
  std::memset(out, 0, sizeof(EmitRec) * kMaxFactor);
  for (int e = 0; e < t.emit_start[t.q]; ++e) {
    const int j = t.emit_list[e];
    const int last = t.off[j] + t.T - 1;   // last tap row of cell 0, = e's residue (mod q)
    out[e].j = j;
    out[e].lag = (last - mod_pos(last, t.q)) / t.q;
    for (int k = 0; k < 4; ++k) out[e].w[k] = t.w[j][k];
  }
}

static fcfs_status forward_geom(const fcfs_plan_* plan, int dtype, int64_t planes, int h, int w, int ho,
                                int wo, bool batch, bool pair_ok, FwdGeom* g);

fcfs_status plan_forward_geom(const fcfs_plan_* plan, int dtype, int64_t planes, int h, int w, int ho, int wo,
                              bool pair_ok, FwdGeom* g) {
  return forward_geom(plan, dtype, planes, h, w, ho, wo, false, pair_ok, g);
}

// The batched kernel carries the instances with 4 or 1 column groups per lane
// and 8 staged slots.
fcfs_status plan_forward_geom_batch(const fcfs_plan_* plan, int dtype, int64_t planes, int h, int w, int ho,
                                    int wo, FwdGeom* g) {
  return forward_geom(plan, dtype, planes, h, w, ho, wo, true, false, g);
}

static fcfs_status forward_geom(const fcfs_plan_* plan, int dtype, int64_t planes, int h, int w, int ho,
                                int wo, bool batch, bool pair_ok, FwdGeom* g) {
  (void)h;
  (void)w;
  const AxisTable& aw = plan->aw;
  const AxisTable& ah = plan->ah;
  const int span = aw.omax - aw.omin + 1;
  // staged columns of a strip of tw outputs, at most (see the kernel)
  auto seg = [&](int tw) { return aw.q * ((tw + aw.p - 2) / aw.p) + span; };
  const bool learned = plan->method == FCFS_LEARNED_DW4;
#ifndef FCFS_FWD_MAX_KC
#define FCFS_FWD_MAX_KC 4
#endif
  int kc = learned ? 1 : FCFS_FWD_MAX_KC;
  while (kc > 1 && (seg(64 * kc) > 512 || wo <= 64 * (kc / 2))) kc = batch ? 1 : kc / 2;
  int tw = 64 * kc;
  while (tw > 1 && seg(tw) > 512) tw /= 2;
  if (seg(tw) > 512) return FCFS_E_UNSUPPORTED;
  const int need = seg(tw);
  g->slots = batch ? 8 : (need <= 128 ? 2 : (need <= 256 ? 4 : 8));
  // Paired 16-bit I/O: whole strips of 64*kc columns (kc even), and the staged
  // segment, which may start one column early to stay pair-aligned, fits in
  // 128 or 256 pairs.
  g->paired = pair_ok && !batch && !learned && kc % 2 == 0 && tw == 64 * kc && need + 1 <= 512;
  if (g->paired) g->slots = need + 1 <= 256 ? 2 : 4;
  g->kc = kc;
  g->tw = tw;
  g->strips = (wo + tw - 1) / tw;
  const int Mh = ho / ah.p;
  // Bands of cells. Consecutive waves take the strips of one band, then the
  // next band of the same plane, so the waves in flight together work on
  // nearby rows of few planes. A band of c cells streams q*(c-1) + span input
  // rows; bands are sized to about a set number of rows per tap count: small
  // enough for many waves (a short tail at the end of the launch), large
  // enough that the span - q rows re-read above each band, and the per-wave
  // set-up, stay a modest share. 16-bit storage moves half the bytes per row
  // for the same instructions, so it takes longer bands.
#ifndef FCFS_FWD_BAND_ROWS_T1
#define FCFS_FWD_BAND_ROWS_T1 6
#endif
#ifndef FCFS_FWD_BAND_ROWS_T2
#define FCFS_FWD_BAND_ROWS_T2 10
#endif
#ifndef FCFS_FWD_BAND_ROWS_T4
#define FCFS_FWD_BAND_ROWS_T4 14
#endif
#ifndef FCFS_FWD_BAND_ROWS16_T1
#define FCFS_FWD_BAND_ROWS16_T1 16
#endif
#ifndef FCFS_FWD_BAND_ROWS16_T2
#define FCFS_FWD_BAND_ROWS16_T2 24
#endif
#ifndef FCFS_FWD_BAND_ROWS16_T4
#define FCFS_FWD_BAND_ROWS16_T4 32
#endif
#ifndef FCFS_FWD_BAND_ROWS_LEARNED
#define FCFS_FWD_BAND_ROWS_LEARNED 24
#endif
  const int span_h = ah.omax - ah.omin + 1;
  // (the learned depthwise variant loads its phases' weights per wave, so
  // in FP32 it takes longer bands than bicubic)
  const int rows = learned && dtype == FCFS_F32 ? FCFS_FWD_BAND_ROWS_LEARNED
                   : dtype == FCFS_F32
                       ? (ah.T == 1 ? FCFS_FWD_BAND_ROWS_T1 : (ah.T == 2 ? FCFS_FWD_BAND_ROWS_T2 : FCFS_FWD_BAND_ROWS_T4))
                       : (ah.T == 1 ? FCFS_FWD_BAND_ROWS16_T1
                                    : (ah.T == 2 ? FCFS_FWD_BAND_ROWS16_T2 : FCFS_FWD_BAND_ROWS16_T4));
  // ... and at least four output rows per wave
  const int cells = std::max({1, (rows - span_h) / ah.q + 1, (4 + ah.p - 1) / ah.p});
  g->band_cells = cells;
  g->bands = (Mh + cells - 1) / cells;
  g->waves = planes * g->strips * (int64_t)g->bands;
  return FCFS_OK;
}

}  // namespace fcfs
