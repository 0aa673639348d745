/*
 * fcfs.h — C ABI of libfcfs, fully convolutional fractional scaling (FCFS)
 * on AMD Instinct MI355X (gfx950).
 *
 * FCFS rescales each channel of an NCHW tensor by a rational factor p/q in
 * three steps (paper, Sec. 3.1 and its 2D form in Sec. 4.2):
 *   1. pad the input (Sec. 3, "Padding"),
 *   2. a stride-q convolution with p*p output channels per input channel, one
 *      per interpolation phase (Sec. 3, "Stride"; Sec. 3.1.1),
 *   3. pixelshuffle by p (Sec. 3, "Pixel Shuffling"; Sec. 4.1).
 * libfcfs fuses the three steps into one kernel: the padding is applied while
 * loading, the hidden layer is never written, and each output sample is
 * stored once at its pixelshuffled position.
 *
 * Conventions shared by every entry point
 *  - Tensors are dense, row-major NCHW, element-aligned device pointers owned
 *    by the caller. Scalars and tables are owned by the library.
 *  - p/q is reduced by its gcd; the output of an axis of length n has
 *    p * ceil(n / q) samples (Sec. 3.1.1: the hidden layer has ceil(n/q) cells;
 *    Sec. 5.1: 5 samples at 3/2 give 9).
 *  - Output sample k = p*m + j (cell m, phase j) samples the input at
 *    u = (k + 1/2) q/p - 1/2 (half-pixel grid, the default) — see fcfs_grid.
 *  - Weights multiply input samples in ascending index order (the printed
 *    kernels of Sec. 5.2 read that way).
 *  - fcfs_forward / fcfs_backward enqueue work on the given HIP stream and
 *    return without waiting. Argument errors are detected before anything is
 *    enqueued and leave every buffer untouched. A launch failure returns
 *    FCFS_E_DEVICE; a fault inside a kernel surfaces as FCFS_E_DEVICE from a
 *    later call that synchronises or from the caller's own stream sync.
 *  - Plans are immutable after creation and may be shared between threads.
 *  - No entry point throws; all report through fcfs_status.
 */
#ifndef FCFS_H_
#define FCFS_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FCFS_OK = 0,
  FCFS_E_INVAL = 1,        /* bad argument (sizes, factors, null pointers, layout) */
  FCFS_E_UNSUPPORTED = 2,  /* valid request outside what this build implements */
  FCFS_E_NOMEM = 3,        /* host or device allocation failed */
  FCFS_E_DEVICE = 4,       /* HIP runtime error (launch failure, earlier fault) */
  FCFS_E_AGAIN = 5,        /* resource busy / queue full, retry later */
  FCFS_E_PENDING = 6,      /* work not finished yet */
  FCFS_E_CANCELLED = 7     /* work was cancelled */
} fcfs_status;

/* Interpolation kernel of each phase (Sec. 5.2). */
typedef enum {
  FCFS_NEAREST = 0,     /* Sec. 5.2.1: the sample at floor(u + 1/2); a bit-exact copy */
  FCFS_BILINEAR = 1,    /* Sec. 5.2.2: 2 taps per axis, weights 1 - t, t */
  FCFS_BICUBIC = 2,     /* Sec. 5.2.3: 4 taps per axis, Keys cubic, a = -1/2 */
  FCFS_LEARNED_DW4 = 3, /* learnable depthwise 4x4 taps per phase and channel (Sec. 7) */
  FCFS_LEARNED_MIX4 = 4 /* learnable 4x4 taps per phase mixing C_in -> C_out channels */
} fcfs_method;

/* Virtual extension beyond the input's edges (Sec. 3, "Padding"). */
typedef enum {
  FCFS_PAD_ZERO = 0,      /* zeros */
  FCFS_PAD_REPLICATE = 1, /* repetition of the edge sample */
  FCFS_PAD_REFLECT = 2    /* mirror about the edge sample (edge not repeated), periodic */
} fcfs_pad;

/* Storage type of x, y, dy and dx. Arithmetic is always FP32. */
typedef enum { FCFS_F32 = 0, FCFS_BF16 = 1, FCFS_F16 = 2 } fcfs_dtype;

/* Where output sample k = p*m + j samples the input (u in input samples).
 * HALF : u = (k + 1/2) q/p - 1/2 (pixel centres; identity at p = q).
 * PAPER: u = (k + 1/2) q/p       (reproduces the 3/2 kernels printed in
 *                                 Sec. 5.2.1 and Sec. 5.2.2).
 * ASYM : u = k q/p               (channel j at offset j/p of a cell, the
 *                                 wording of Sec. 3.1.1). */
typedef enum { FCFS_GRID_HALF = 0, FCFS_GRID_PAPER = 1, FCFS_GRID_ASYM = 2 } fcfs_grid;

typedef struct fcfs_plan_* fcfs_plan_t;

/* Create a plan for scaling both axes by p/q (Sec. 3.1; Sec. 4.2 with equal
 * factors), on the half-pixel grid. Host only: builds the per-phase tap
 * tables (Sec. 5.2) in integer arithmetic, weights rounded once from FP64
 * to FP32. p and q are reduced by their gcd; after reduction both must be
 * <= 32. *out receives a plan that the caller frees with fcfs_plan_destroy.
 * Errors: FCFS_E_INVAL (p < 1, q < 1, bad enum, out == NULL),
 * FCFS_E_UNSUPPORTED (reduced p or q > 32), FCFS_E_NOMEM. */
fcfs_status fcfs_plan(int p, int q, fcfs_method method, fcfs_pad pad, fcfs_plan_t* out);

/* As fcfs_plan with a separate factor per axis (Sec. 4.2: r_1/s_1, r_2/s_2)
 * and a choice of sampling grid. */
fcfs_status fcfs_plan_ex(int p_h, int q_h, int p_w, int q_w, fcfs_method method, fcfs_pad pad,
                         fcfs_grid grid, fcfs_plan_t* out);

/* Free a plan. NULL is accepted. */
fcfs_status fcfs_plan_destroy(fcfs_plan_t plan);

/* Reduced factors of the height axis and the method's taps per axis (1, 2
 * or 4; an axis at 1/1 that samples its inputs exactly copies them with one
 * tap, see fcfs_plan_taps). Any output pointer may be NULL. */
fcfs_status fcfs_plan_query(fcfs_plan_t plan, int* p_red, int* q_red, int* taps);

/* Tap table of one phase (Sec. 3.1.1: phase j of every cell m interpolates
 * at its own offset; Sec. 5.2: the weights of each method). axis 0 = height,
 * 1 = width; phase in [0, p_red). Output sample p*m + phase reads input
 * samples q*m + *first_offset + t for t < taps with weights w[t] (FP32, the
 * values the kernels use; zeros for learned methods). w must hold 4 floats.
 * Errors: FCFS_E_INVAL for a bad axis, phase or NULL pointer. */
fcfs_status fcfs_plan_taps(fcfs_plan_t plan, int axis, int phase, int* first_offset, float* w);

/* Output size for an h x w input: p_h * ceil(h / q_h) by p_w * ceil(w / q_w)
 * (Sec. 3.1.1 and the 5 -> 9 example of Sec. 5.1). */
fcfs_status fcfs_output_size(fcfs_plan_t plan, int64_t h, int64_t w, int64_t* h_out, int64_t* w_out);

/* Forward rescale: y = FCFS(x) (Sec. 3.1 / Sec. 4.2 pseudocode).
 *   x      : device, [n][c_in][h][w] of dtype.
 *   weight : device. NULL for fixed methods. LEARNED_DW4: FP32 [c_in][p_h][p_w][4][4],
 *            4x4 taps per channel and phase, tap (a, b) reading input row
 *            q*m_h + floor(u_h) - 1 + a and column q*m_w + floor(u_w) - 1 + b.
 *            LEARNED_MIX4: [p_h][p_w][c_out][c_in][4][4] in the storage type
 *            (BF16 or FP16 run on the 16-bit matrix cores with FP32
 *            accumulation, FP32 on the FP32 matrix cores), 16-byte aligned;
 *            same taps, summed over c_in.
 *   c_out  : output channels; must equal c_in except for LEARNED_MIX4.
 *   y      : device, [n][c_out][h_out][w_out] of dtype; must not overlap x.
 *   stream : HIP stream the kernels are enqueued on (0 = the null stream).
 * An empty problem (n, c_in, h or w equal to 0) is valid and enqueues nothing;
 * its pointers are not inspected.
 * Errors: FCFS_E_INVAL (negative sizes, null pointers, weight missing for a learned
 * method or given for a fixed one, c_out mismatch, a misaligned MIX4 weight),
 * FCFS_E_UNSUPPORTED (a per-plane size at or above 2^31 samples, LEARNED_DW4
 * with more than 64 phases), FCFS_E_DEVICE (launch failed). */
fcfs_status fcfs_forward(fcfs_plan_t plan, fcfs_dtype dtype, int64_t n, int64_t c_in, int64_t h,
                         int64_t w, const void* x, const void* weight, int64_t c_out, void* y,
                         hipStream_t stream);

/* One-dimensional FCFS (Sec. 3.1; signals such as audio): x [n][c][l] ->
 * y [n][c][p * ceil(l / q)], where p/q is the plan's width factor. The plan's
 * height factor must be 1/1 (fcfs_plan_ex(1, 1, p, q, ...)), whose axis then
 * copies rows with one tap: the n*c signals run as the rows of one plane
 * (or, past 2^31 samples, as planes of one row) of fcfs_forward.
 * Fixed methods only. Errors: FCFS_E_INVAL for a height factor other than
 * 1/1 or a learned method, FCFS_E_UNSUPPORTED for FCFS_GRID_PAPER (its 1/1
 * axis samples half-way between rows, not the row), else as fcfs_forward. */
fcfs_status fcfs_forward_1d(fcfs_plan_t plan, fcfs_dtype dtype, int64_t n, int64_t c, int64_t l,
                            const void* x, void* y, hipStream_t stream);

/* Three-dimensional FCFS (Sec. 4.2 with the ND pixelshuffle of Sec. 4.1;
 * volumes such as medical scans) of NCDHW tensors for the fixed methods:
 *   plan_d  : the depth factor as its height factor, width factor 1/1
 *             (fcfs_plan_ex(p_d, q_d, 1, 1, method, pad, grid));
 *   plan_hw : the height and width factors (fcfs_plan_ex(p_h, q_h, p_w, q_w,
 *             method, pad, grid)), with the same method, padding and grid.
 *   x : device [n][c][d][h][w] of dtype; y : device [n][c][d_out][h_out][w_out].
 * The interpolants are separable, so the result is two passes of the fused
 * forward kernel through a device workspace (the smaller of the two possible
 * intermediates: [n][c][d][h_out][w_out] after the height-width pass, or
 * [n][c][d_out][h][w] after the depth pass), each pass exact up to rounding;
 * with 16-bit storage the intermediate is rounded to the storage type too.
 * The workspace is caller-owned, at least fcfs_forward_3d_workspace bytes,
 * 4-byte aligned, and must not overlap x or y.
 * Errors: FCFS_E_INVAL (null pointers, mismatched plans, a learned method,
 * a depth plan whose width factor is not 1/1, a small workspace),
 * FCFS_E_UNSUPPORTED for FCFS_GRID_PAPER (the depth pass's 1/1 width axis
 * would not copy), else as fcfs_forward. */
fcfs_status fcfs_forward_3d_workspace(fcfs_plan_t plan_d, fcfs_plan_t plan_hw, fcfs_dtype dtype, int64_t n,
                                      int64_t c, int64_t d, int64_t h, int64_t w, size_t* bytes);
fcfs_status fcfs_forward_3d(fcfs_plan_t plan_d, fcfs_plan_t plan_hw, fcfs_dtype dtype, int64_t n, int64_t c,
                            int64_t d, int64_t h, int64_t w, const void* x, void* y, void* workspace,
                            size_t ws_bytes, hipStream_t stream);

/* Launch geometry fcfs_forward would use for these sizes (introspection for
 * tests and benchmarks; enqueues nothing). kernel_id identifies the compiled
 * kernel instance: dtype*1000 + taps*100 + column groups per lane*10 + staged
 * row dwords per lane (+ 10000 for the learned depthwise layer, 20000 for the
 * channel-mixing layer, 50000 for the paired 16-bit instance, where the last
 * digit counts staged sample pairs; fcfs_forward takes that instance when
 * both widths are even and x and y are 4-byte aligned, which this call
 * assumes; 100000 when the height axis is a 1/1 copy with one tap beside a
 * resampled width, 200000 for the reverse; taps is the larger count). Any output pointer may be NULL. Errors: as fcfs_forward's
 * argument checks. */
fcfs_status fcfs_forward_config(fcfs_plan_t plan, fcfs_dtype dtype, int64_t n, int64_t c_in,
                                int64_t h, int64_t w, int* kernel_id, int* strip_width,
                                int* band_cells, int64_t* waves);

/* Device workspace bytes fcfs_backward needs for these sizes (0 if none),
 * with the weight gradient for learned methods. For LEARNED_MIX4 the
 * workspace holds re-laid-out copies of dy (two layouts), of the padded x (one
 * per tap column offset) and the weights, and the weight gradient's partial
 * sums: about 3.1 GB for 16x64x512^2 at 5/4. */
fcfs_status fcfs_backward_workspace(fcfs_plan_t plan, fcfs_dtype dtype, int64_t n, int64_t c_in,
                                    int64_t h, int64_t w, int64_t c_out, size_t* bytes);

/* Backward (the adjoint of fcfs_forward, for training the layer of Sec. 7).
 *   dy : device [n][c_out][h_out][w_out] of dtype, the gradient of y.
 *   dx : device [n][c_in][h][w] of dtype or NULL: receives A^T dy, i.e. for
 *        each input sample the sum of w * dy over every (output, tap) that
 *        read it, padding folded back (replicate: onto the edge sample;
 *        reflect: onto the mirrored sample; zero: dropped). Overwritten.
 *   dw : device FP32, same layout as weight, or NULL: receives the weight
 *        gradient sum over n and cells of dy * (padded x). Learned methods
 *        only. Overwritten (not accumulated). Deterministic: the summation
 *        order is fixed by the sizes alone.
 *   x  : needed iff dw != NULL. weight: needed for learned methods iff dx != NULL.
 *   LEARNED_MIX4 (16-bit storage): weight [p_h][p_w][c_out][c_in][4][4] in
 *        the storage type, 16-byte aligned; dx[c] sums over every output
 *        channel o too; dw is FP32 [p_h][p_w][c_out][c_in][4][4]. FP32
 *        storage returns FCFS_E_UNSUPPORTED (the forward has it).
 *   workspace / ws_bytes: device scratch of at least fcfs_backward_workspace
 *        bytes (NULL allowed when that is 0).
 * Errors: as fcfs_forward, plus FCFS_E_INVAL for a workspace that is too small,
 * and FCFS_E_UNSUPPORTED for an output axis of 2^24 samples or more, or (for
 * LEARNED_MIX4) sizes whose launches would pass 2^31 workgroups. */
fcfs_status fcfs_backward(fcfs_plan_t plan, fcfs_dtype dtype, int64_t n, int64_t c_in, int64_t h,
                          int64_t w, const void* x, const void* weight, int64_t c_out,
                          const void* dy, void* dx, float* dw, void* workspace, size_t ws_bytes,
                          hipStream_t stream);

/* Largest workspace fcfs_backward_noalloc can serve: 64 MiB (the 8x64x256^2
 * learned depthwise backward at 3/4 needs about 4.7 MB; the 16x64x512^2
 * channel-mixing backward at 5/4 needs about 3.1 GB and is refused). */
#define FCFS_NOALLOC_SCRATCH_BYTES (64u << 20)

/* fcfs_backward for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops and harnesses that forbid allocation): the
 * same kernels and results, with the workspace taken from a fixed device
 * array of FCFS_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it
 * runs on until the process ends. It allocates nothing; the caller still
 * passes x, weight, dy, dx and dw as for fcfs_backward. The kernels run on
 * the stream's device (the current device for the null stream); the first
 * call on a device looks up that device's array.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (on different streams, or from several threads without ordering)
 * race and give wrong results. Calls ordered on one stream are safe; no call
 * reads what an earlier one left in the array.
 * Errors: as fcfs_backward, plus FCFS_E_UNSUPPORTED when these sizes need a
 * workspace larger than FCFS_NOALLOC_SCRATCH_BYTES (fcfs_backward_workspace
 * gives the need, with the weight gradient) and FCFS_E_DEVICE when the
 * array's device address cannot be looked up. */
fcfs_status fcfs_backward_noalloc(fcfs_plan_t plan, fcfs_dtype dtype, int64_t n, int64_t c_in, int64_t h,
                                  int64_t w, const void* x, const void* weight, int64_t c_out,
                                  const void* dy, void* dx, float* dw, hipStream_t stream);

/* ------------------------------------------------------------------ serving
 * A persistent request loop on one GPU (continuous batching). Clients submit
 * rescale requests from any thread; a scheduler thread admits pending
 * requests while request slots and the device memory budget allow, and
 * launches one batched forward kernel per scheduling tick covering every
 * newly admitted request (mixed sizes, factors, methods and storage types),
 * alternating two HIP streams so that requests arriving while a batch runs
 * are launched next to it. A request with more waves than the chunk size
 * (FCFS_SERVER_CHUNK_WAVES) runs as chunks over consecutive batches. Buffers
 * stay on the device. A completion thread timestamps finished batches.
 * Results equal fcfs_forward's bit for bit (the same per-wave code runs). */

typedef struct fcfs_server_* fcfs_server_t;

typedef struct {
  int p, q;              /* scale factor (both axes, half-pixel grid) */
  fcfs_method method;    /* FCFS_NEAREST, FCFS_BILINEAR or FCFS_BICUBIC */
  fcfs_pad pad;
  fcfs_dtype dtype;      /* FCFS_F32 or FCFS_BF16 */
  int64_t n, c, h, w;
  const void* x;         /* device input owned by the caller (valid until done), or NULL:
                            the server generates it in its arena from `seed` (element i of
                            the NCHW tensor = top 24 bits of splitmix64(seed, i) / 2^24,
                            rounded to the storage type) */
  uint64_t seed;
  void* y;               /* device output owned by the caller, or NULL: allocated in the
                            server arena, valid until fcfs_release */
} fcfs_request;
/* Ordering of caller-owned buffers: the server runs its kernels on streams of
 * its own (created non-blocking, so they wait for no other stream, the null
 * stream included). Whatever writes x, or still reads or writes y, on the
 * caller's streams must be complete before fcfs_submit (synchronise those
 * streams first); x must stay unchanged and y untouched until the request's
 * poll or wait reports it finished. */

typedef struct {
  fcfs_status status;    /* FCFS_OK, or the request's own failure (FCFS_E_NOMEM: larger
                            than the memory budget; FCFS_E_DEVICE: its batch failed) */
  void* y;               /* device output */
  int64_t h_out, w_out;
  double t_arrive_us, t_start_us, t_done_us;   /* since server creation */
} fcfs_result;

/* Create a server on HIP device `device` with a device memory budget (the
 * arena holding generated inputs and server-owned outputs; allocated once,
 * here) and at most `max_slots` admitted, unfinished requests.
 * Errors: FCFS_E_INVAL, FCFS_E_NOMEM (arena), FCFS_E_DEVICE (no such device). */
fcfs_status fcfs_server_create(int device, size_t mem_budget_bytes, int max_slots, fcfs_server_t* out);

/* Queue a request; *ticket identifies it. Argument errors are returned here
 * and queue nothing: FCFS_E_INVAL (method, storage type, sizes), and
 * FCFS_E_UNSUPPORTED for a plane of 2^31 samples or more, a reduced factor
 * above 32 or sizes whose byte counts overflow. FCFS_E_AGAIN when the
 * pending queue is full. */
fcfs_status fcfs_submit(fcfs_server_t server, const fcfs_request* req, uint64_t* ticket);

/* FCFS_OK with *out filled when the request is finished (out->status holds
 * its outcome), FCFS_E_PENDING before that, FCFS_E_INVAL for an unknown
 * ticket. */
fcfs_status fcfs_poll(fcfs_server_t server, uint64_t ticket, fcfs_result* out);

/* As fcfs_poll, blocking up to timeout_us microseconds (negative: no limit). */
fcfs_status fcfs_wait(fcfs_server_t server, uint64_t ticket, int64_t timeout_us, fcfs_result* out);

/* Forget a finished request and free its server-owned output.
 * FCFS_E_PENDING if it is not finished. */
fcfs_status fcfs_release(fcfs_server_t server, uint64_t ticket);

/* Latency percentiles (arrival to completion) over finished requests,
 * finished requests per second and algorithmic GB/s over the span from the
 * first arrival to the last completion. Any pointer may be NULL. */
fcfs_status fcfs_server_stats(fcfs_server_t server, double* p50_us, double* p99_us, double* req_per_s,
                              double* gbps);

/* Test hooks (they force failure paths without faulting anything): hook 1
 * makes the next `value` requests at the head of the queue fail with
 * FCFS_E_NOMEM as if the arena had refused them; hook 2 makes the next
 * `value` batches fail as if their launch had failed (nothing is launched). */
fcfs_status fcfs_server_debug(fcfs_server_t server, int hook, int64_t value);

/* Server options. FCFS_SERVER_MAX_BATCH: most newly admitted requests per
 * batched launch (0 = no limit; 1 = one launch per request, for comparisons).
 * FCFS_SERVER_DISCARD_OUTPUTS: 1 = free server-owned outputs as soon as a
 * request finishes (its result then has y = NULL; for load tests).
 * FCFS_SERVER_CHUNK_WAVES: most waves (64 output columns by a band of rows
 * each) of one request per batch, default 16384: a larger request runs as
 * chunks in consecutive batches, next to the requests admitted meanwhile
 * (0 = no chunking). */
typedef enum {
  FCFS_SERVER_MAX_BATCH = 1,
  FCFS_SERVER_DISCARD_OUTPUTS = 2,
  FCFS_SERVER_CHUNK_WAVES = 3
} fcfs_server_option;
fcfs_status fcfs_server_config(fcfs_server_t server, int option, int64_t value);

/* Submit `count` requests from the calling thread, request i when
 * arrival_us[i] microseconds (non-decreasing) have passed since the call,
 * waiting between submissions; tickets[i] receives each ticket. Returns the
 * first submission error (earlier requests stay queued). For replaying
 * arrival traces at rates a client thread in Python cannot keep. */
fcfs_status fcfs_server_replay(fcfs_server_t server, const fcfs_request* reqs, const double* arrival_us,
                               int64_t count, uint64_t* tickets);

/* Forget the statistics gathered so far (latencies, counts, span). */
fcfs_status fcfs_server_reset_stats(fcfs_server_t server);

/* Finish every admitted request, stop the threads and free everything. Tickets
 * still pending are completed with FCFS_E_CANCELLED. */
fcfs_status fcfs_server_destroy(fcfs_server_t server);

/* Static text for a status code. */
const char* fcfs_status_string(fcfs_status status);

/* Library version as major*10000 + minor*100 + patch. */
int fcfs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FCFS_H_ */
