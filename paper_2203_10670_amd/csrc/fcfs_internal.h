// Internal declarations shared by the host plan code and the HIP kernels.
#pragma once

#include <stdint.h>

#include "../../include/fcfs.h"

namespace fcfs {

constexpr int kMaxFactor = 32;   // largest reduced p or q a plan accepts

// Per-axis tap table of a plan (paper Sec. 3.1.1 and Sec. 5.2): output sample
// k = p*m + j reads input samples q*m + off[j] + t, t = 0..T-1, with weights
// w[j][t]. Passed to kernels by value (it lives in the kernel-argument
// segment); every field is 4-byte aligned so uniform lookups are scalar loads.
struct AxisTable {
  int p, q;                  // reduced factor
  int T;                     // taps: 1 nearest, 2 bilinear, 4 bicubic / learned
  int omin, omax;            // smallest first tap and largest last tap offset
  int off[kMaxFactor];       // first tap offset of each phase (in [-2, q])
  int emit_start[kMaxFactor + 1];  // phases whose last tap is = r (mod q) are
  int emit_list[kMaxFactor];       //   emit_list[emit_start[r] .. emit_start[r+1])
  int back[kMaxFactor];      // per residue r: distance down to the nearest row
                             // index some tap reads (0 when taps read r itself)
  float w[kMaxFactor][4];    // tap weights (fixed methods; unused when learned)
};

}  // namespace fcfs

struct fcfs_plan_ {
  int method;   // fcfs_method
  int pad;      // fcfs_pad
  int grid;     // fcfs_grid
  fcfs::AxisTable ah, aw;
};

namespace fcfs {

// Builds one axis table; returns FCFS_OK or an error.
// allow_copy: at 1/1 on a grid that samples inputs exactly, use one tap.
fcfs_status build_axis(int p, int q, int method, int grid, bool allow_copy, AxisTable* out);

// Launch geometry of the fused forward kernel.
struct FwdGeom {
  int kc;            // output-column groups per lane (1, 2 or 4)
  int slots;         // staged row-segment dwords per lane (2, 4 or 8)
  bool paired;       // 16-bit samples move in pairs (slots then count pairs)
  int tw;            // output columns per wave strip
  int strips;        // strips per plane
  int band_cells;    // hidden-layer cells (groups of p output rows) per band
  int bands;         // bands per plane
  int64_t waves;     // total waves
};

// Height emission record of the forward kernel: when input row r arrives
// (r = q*rq + rho), the entries emit_start[rho] .. emit_start[rho+1] - 1
// finish output row p*(rq - lag) + j, with the phase's height taps w.
struct alignas(32) EmitRec {
  int j;
  int lag;
  float w[4];
  int pad_[2];
};
void fill_emit(const AxisTable& t, EmitRec* out);

struct FwdArgs {
  const void* x;
  void* y;
  const float* weight;   // learned depthwise taps [C][p_h][p_w][4][4] or null
  int64_t planes;        // n * c
  int C;
  int H, W, Ho, Wo, Mh;
  int pad;
  int tw, strips, band_cells, bands;
  int64_t waves;
  AxisTable th, tw_tab;
  EmitRec emit[kMaxFactor];   // height emission records (from th)
};

struct BwdArgs {
  const void* x;         // input (needed for the weight gradient)
  const float* weight;   // learned depthwise taps [C][p_h][p_w][4][4] or null
  const void* dy;        // output gradient
  void* dx;              // input gradient or null
  float* dw;             // weight gradient or null
  int64_t planes;        // n * c
  int C;
  int H, W, Ho, Wo, Mh, Mw;
  int pad;
  int col_blocks;        // input-gradient blocks per input row
  int cmax_h, cmax_w;    // adjoint table entries per index
  int fast_w;            // most width entries of any index away from the padded edges
  int* tab_h;            // adjoint tables (workspace), see bwd_kernel.h
  int* tab_w;
  float* partial;        // weight-gradient partial sums (workspace)
  int ch, cw, nch, ncw;  // weight-gradient chunk: ch x cw cells, nch x ncw chunks per plane
  int chunks_per_channel;
  int dw_lds_bytes;
  // channel-mixing layer
  int planes_n;            // batch
  int Cout;                // output channels (C = input channels)
  const void* mix_weight;  // [p_h][p_w][Cout][C][4][4], 16-bit storage
  // input gradient on MFMA (workspace): channel-last dy with zero margin
  // cells, packed weights, and the edge buffer of the pad adjoint
  uint16_t* mix_dyc;       // [n][ho][p_w][opad / 32][dcells][32]: dy[o][ho][p_w mw + jw] at cell dleft + mw
  uint16_t* mix_wpk;       // [p_h][p_w][4][4][opad / 32][4][cpad][8]: W[o][c] at (o / 32, o % 32 / 8, c, o % 8)
  float* mix_edge;         // z at the positions the pad adjoint folds (null for zero padding)
  int mix_opad, mix_cpad;  // C_out rounded up to 32, C_in rounded up to 64
  int mix_dleft, mix_dcells;                // margin cells left of cell 0; cells per phase row
  int mix_clcells;                          // cells per block of the channel-last pass (<= kDxcColumns columns)
  int mix_eh0, mix_eh1, mix_ew0, mix_ew1;   // extended positions the taps read (inclusive)
  int mix_r0, mix_rows;                     // extended rows of the GEMM: [r0, r0 + rows)
  int mix_v0, mix_vw, mix_mtn, mix_vchunks; // width-class positions [v0, v0 + vw) in chunks of 16 mtn
  int mix_kw, mix_vgroups;                  // chunks per workgroup (all width classes of each), groups per row
  int mix_lds_epi;                          // the workgroup interleaves the classes in LDS (q_w * kw <= 8)
  int mix_top, mix_bot, mix_cl, mix_cr;     // fold zones: rows [0, top), [H - bot, H); columns [0, cl), [W - cr, W)
  int mix_rr, mix_cc;                       // edge buffer: zone rows (part R), zone columns (part C)
  int64_t mix_edge_c;                       // floats of part R (part C follows)
  int64_t mix_edge_per;                     // input samples per plane in a fold zone
  size_t mix_ws_dyc, mix_ws_wpk, mix_ws_edge;   // workspace offsets of the three buffers
  // weight gradient on MFMA (workspace): dy by phase and x by tap column
  // offset, 8 cells per 16-byte group; partial sums [chunk][ph][tap][o][c]
  uint16_t* mix_dyw;       // [n][ho][p_w][ncb][4][dwopad][8]: dy[o][ho][p_w mw + jw] at mw = 32 block + 8 group + i
  uint16_t* mix_xa;        // [n][row - eh0][s][ncb][4][cpad][8]: ext(x)[c][row][q_w mw + s0 + s]
  int mix_dwopad, mix_ncb;        // C_out rounded up to 64; 32-cell blocks per cell row
  int mix_s0, mix_ns;             // tap column offsets s0 .. s0 + ns - 1
  int mix_dwcells, mix_dwxcells;  // cells per block of the dy and x passes
  int mix_wchunks;                // chunks of cell rows
  size_t mix_ws_dyw, mix_ws_xa;
  // (tap, d) of each residue r of the height / width axis: entries
  // [start[r], start[r + 1]), each phase | tap << 5 | (d + 64) << 7, where
  // the extended index q u + r reads cell u - d of that phase at that tap
  int mix_hl_start[kMaxFactor + 1], mix_hl[4 * kMaxFactor];
  int mix_wl_start[kMaxFactor + 1], mix_wl[4 * kMaxFactor];
  AxisTable th, tw_tab;
};

constexpr int kMixOut = 32;   // output channels per channel-mixing workgroup
constexpr int kDxcColumns = 256;   // dy columns per block of the input gradient's layout pass

struct MixArgs {
  const void* x;         // [N][Cin][H][W], 16-bit storage
  const void* w;         // [p_h][p_w][Cout][Cin][4][4], same storage type, 16-byte aligned
  void* y;               // [N][Cout][Ho][Wo]
  int N, Cin, Cout;
  int H, W, Ho, Wo, Mh, Mw;
  int pad;
  int th_cells, tw_cells;    // cell tile of a workgroup (th_cells * tw_cells = 128)
  int tiles_h, tiles_w, groups, otiles;
  int gsize;                 // width phases per group: min(5, p_w)
  int lds_bytes;
  // staged input patch of a workgroup, per input channel: R rows x Cc columns
  // (row pitch CP); cell (lh, lw) tap (a, b) of width phase jw sits at row
  // rstep*lh + a, column cstep*lw + off_w[jw] - off_w[first phase] + b
  int R, Cc, CP;
  int rstep, cstep;          // = q (all rows/columns staged) or 4 / wspan (only the tapped ones)
  int wspan;                 // columns a cell's taps cover over the phase group
  int npr, ncs, items;       // (channel, row) pairs per wave, 64-column slots per row, items per lane
  int nbuf;                  // LDS stage buffers (2, or 1 when two do not fit)
  int cl;                    // 1: the channel-last kernel (CP counts 16-byte slots of 8 channels)
  int slots;                 // channel-last: slots per residue class of a patch row
  int xpair;                 // channel-last: pair staging (contiguous patch columns, even W, 4-byte aligned x)
  int fixed;                 // channel-last: every phase group has consecutive tap column offsets
  int buf_u16, woff_u16;     // LDS stage buffer size and weight offset in it (16-bit units):
                             // patch [2][R][CP], then weights [gsize][32][32] and a spare quad
  AxisTable th, tw_tab;
};

// ---------------------------------------------------------------- serving
// One request of a batched launch (in device memory): waves wave_begin ..
// wave_begin + (its share of the batch) - 1 of the request's forward, so a
// large request runs as chunks spread over several batches.
struct BatchDesc {
  FwdArgs args;
  int64_t wave_begin;
  int variant;      // forward instance: dtype (0 f32, 1 bf16) * 6 + tap index (0: 1, 1: 2, 2: 4) * 2 + (kc == 4 ? 0 : 1)
  int pad_;
};
struct BatchArgs {
  const BatchDesc* desc;
  const int64_t* wave_start;   // [nreq + 1] prefix of waves per request
  int nreq;
  int64_t total_waves;
};
// A request whose input the server generates.
struct GenDesc {
  void* x;
  int64_t count;     // elements
  uint64_t seed;
  int dtype;
  int pad_;
};
struct GenArgs {
  const GenDesc* desc;
  const int64_t* block_start;  // [ngen + 1] prefix of blocks per request
  int ngen;
  int64_t total_blocks;
};
constexpr int kGenPerBlock = 256 * 16;   // elements per generator block

fcfs_status launch_forward_batch(const BatchArgs& b, hipStream_t stream);
// Launch geometry for a batched request (restricted to the batched kernel's instances).
fcfs_status plan_forward_geom_batch(const fcfs_plan_* plan, int dtype, int64_t planes, int h, int w, int ho,
                                    int wo, FwdGeom* g);
fcfs_status launch_generate(const GenArgs& g, hipStream_t stream);


// Channel-mixing launchers (mix4.hip); dtype FCFS_BF16 or FCFS_F16.
fcfs_status launch_mix4(int dtype, const MixArgs& a, hipStream_t stream);
// FP32 storage on the FP32 matrix cores (mix4_f32.hip): 64 cells (4 cell rows
// of 16) x 64 outputs x a group of gsize width phases per workgroup, with
// wspan <= 8 tap columns per cell.
fcfs_status launch_mix4_f32(const MixArgs& a, hipStream_t stream);

// Backward kernel launchers, one per storage type (bwd_<dtype>.hip).
fcfs_status launch_backward_f32(const BwdArgs& a, bool learned, hipStream_t stream);
fcfs_status launch_backward_bf16(const BwdArgs& a, bool learned, hipStream_t stream);
fcfs_status launch_backward_f16(const BwdArgs& a, bool learned, hipStream_t stream);
fcfs_status launch_backward_mix_bf16(const BwdArgs& a, hipStream_t stream);
fcfs_status launch_backward_mix_f16(const BwdArgs& a, hipStream_t stream);

// Workspace bytes fcfs_backward needs for these sizes, with or without the
// weight gradient (argument errors as fcfs_backward's).
fcfs_status backward_workspace_need(fcfs_plan_t plan, fcfs_dtype dtype, int64_t n, int64_t c_in, int64_t h,
                                    int64_t w, int64_t c_out, bool need_dw, size_t* bytes);

// Forward kernel launchers, one per storage type (fwd_<dtype>.hip).
fcfs_status launch_forward_f32(int method, const FwdArgs& a, const FwdGeom& g, hipStream_t stream);
fcfs_status launch_forward_bf16(int method, const FwdArgs& a, const FwdGeom& g, hipStream_t stream);
fcfs_status launch_forward_f16(int method, const FwdArgs& a, const FwdGeom& g, hipStream_t stream);

// Host-side launch geometry for a plane of (h, w) -> (ho, wo).
fcfs_status plan_forward_geom(const fcfs_plan_* plan, int dtype, int64_t planes, int h, int w, int ho,
                              int wo, bool pair_ok, FwdGeom* g);

}  // namespace fcfs
