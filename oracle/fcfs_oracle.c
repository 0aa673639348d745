/*
 * FCFS oracle: a plain, slow, FP64 CPU implementation of fully convolutional
 * fractional scaling.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. It shares no source,
 * header, table or helper with the GPU library, and the GPU library never
 * calls it.
 *
 * What it computes follows the paper's own pipeline, in its order:
 *   1. pad the input (Sec. 3, "Padding"; pseudocode of Sec. 3.1 and Sec. 4.2),
 *   2. a stride-s convolution with r (1D) or r_1*r_2 (2D) output channels per
 *      input channel, each a dense (2K+1)-wide kernel (Sec. 3, eq. for the
 *      strided convolution; Sec. 3.1 pseudocode; Sec. 4.2 pseudocode),
 *   3. pixelshuffle by r (Sec. 3 "Pixel Shuffling"; Sec. 4.1).
 * The hidden layer of step 2 is materialised, as the paper does (Sec. 3.1.1).
 * Everything is FP64; sums run over ascending kernel indices.
 *
 * Readings of points the paper leaves open (each listed in the design notes):
 *  - Scale factor r/s is reduced by its gcd first (sampling positions are
 *    unchanged; only the output size uses the reduced form).
 *  - Output length is r * ceil(N / s): the hidden layer has ceil(N/s) cells,
 *    which is what a valid stride-s convolution with kernel 2K+1 over an input
 *    padded by K on each side yields (Sec. 3.1.1, Sec. 5.1 example 5 -> 9).
 *  - Channel j of a cell m samples the input at a coordinate u given as a
 *    numerator over 2r: u = s*m + A_j / (2r). Three grids are offered:
 *       half  : A_j = (2j+1)s - r   (u = (k+1/2) s/r - 1/2, half-pixel centres)
 *       paper : A_j = (2j+1)s       (u = (k+1/2) s/r; reproduces the printed
 *                                    3/2 kernels of Sec. 5.2.1 and 5.2.2)
 *       asym  : A_j = 2 j s         (u = k s/r, the "offset i+(j-1)/r" text
 *                                    of Sec. 3.1.1)
 *    with k = r*m + j. "half" is the default.
 *  - Weights of a kernel multiply the input in the convolution orientation of
 *    Sec. 3 eq. (1): hidden[m] = sum_k xpad[s*m - k] * h[k], and h[k] is the
 *    interpolation weight of the input sample at offset o = -k from s*m.
 *  - Nearest picks floor(u + 1/2); bilinear uses the tent 1-|d|; bicubic uses
 *    the cubic of Sec. 5.2.3 with its constant term read as Keys' a = -1/2.
 *  - Padding is a virtual extension: zero, replicate (edge repeated) or
 *    reflect (mirror about the edge samples, edge not repeated, periodic with
 *    period 2(N-1); N = 1 gives a constant).
 *  - The learnable depthwise layer ("dw4") and the channel-mixing layer
 *    ("mix4") use 4x4 taps per phase anchored at floor(u) - 1, the same
 *    support as bicubic (the paper proposes learning the kernel weights in
 *    Sec. 7 without fixing a support).
 *
 * The backward pass is the exact adjoint of the same pipeline, built by
 * running the forward index maps and accumulating: un-shuffle, transposed
 * strided convolution, then the adjoint of the padding (contributions that
 * landed on padded positions are folded back onto the input samples they were
 * copied from; zero padding drops them).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OM_NEAREST = 0, OM_BILINEAR = 1, OM_BICUBIC = 2, OM_DW4 = 3, OM_MIX4 = 4 };
enum { OP_ZERO = 0, OP_REPLICATE = 1, OP_REFLECT = 2 };
enum { OG_HALF = 0, OG_PAPER = 1, OG_ASYM = 2 };

static long o_gcd(long a, long b) {
  while (b) { long t = a % b; a = b; b = t; }
  return a;
}

/* floor(a / b) for b > 0 */
static long o_floordiv(long a, long b) {
  long d = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) d -= 1;
  return d;
}

/* Numerator (over 2r) of the sampling offset of channel j inside a cell. */
static long o_grid_num(long r, long s, long j, int grid) {
  switch (grid) {
    case OG_PAPER: return (2 * j + 1) * s;
    case OG_ASYM:  return 2 * j * s;
    default:       return (2 * j + 1) * s - r;
  }
}

/* Bicubic kernel of Sec. 5.2.3 with a = -1/2 (so the -4a term is +2). */
static double o_cubic(double d) {
  double ad = fabs(d);
  if (ad <= 1.0) return 1.5 * ad * ad * ad - 2.5 * ad * ad + 1.0;
  if (ad < 2.0) return -0.5 * ad * ad * ad + 2.5 * ad * ad - 4.0 * ad + 2.0;
  return 0.0;
}

static double o_tent(double d) {
  double ad = fabs(d);
  return ad < 1.0 ? 1.0 - ad : 0.0;
}

/* Source index of padded position i of an axis of length n, or -1 when the
 * position reads the constant zero. */
static long o_padmap(long i, long n, int mode) {
  if (i >= 0 && i < n) return i;
  if (mode == OP_ZERO) return -1;
  if (mode == OP_REPLICATE) return i < 0 ? 0 : n - 1;
  if (n == 1) return 0;
  long period = 2 * (n - 1);
  long m = i % period;
  if (m < 0) m += period;
  return m < n ? m : period - m;
}

/* Half width of the dense kernel: wide enough for every tap of every method. */
static long o_half_width(long s) { return s + 2; }

long fcfs_oracle_out_len(long r, long s, long n) {
  if (r < 1 || s < 1 || n < 1) return -1;
  long g = o_gcd(r, s);
  r /= g; s /= g;
  return r * ((n + s - 1) / s);
}

/* Dense 1D kernel of channel j for a fixed method: h[K + k], k in [-K, K],
 * multiplies the input sample at offset -k from s*m. Returns K. */
long fcfs_oracle_phase_kernel(long r, long s, int method, int grid, long j, double* h) {
  long g = o_gcd(r, s);
  r /= g; s /= g;
  long K = o_half_width(s);
  long A = o_grid_num(r, s, j, grid);
  long two_r = 2 * r;
  long nearest = o_floordiv(A + r, two_r);      /* floor(u + 1/2) - s*m */
  for (long k = -K; k <= K; ++k) {
    long o = -k;
    double d = (double)(A - two_r * o) / (double)two_r; /* u - (s*m + o) */
    double w = 0.0;
    if (method == OM_NEAREST) w = (o == nearest) ? 1.0 : 0.0;
    else if (method == OM_BILINEAR) w = o_tent(d);
    else if (method == OM_BICUBIC) w = o_cubic(d);
    h[K + k] = w;
  }
  return K;
}

/* Anchor of the learnable 4-tap window of channel j: floor(u) - 1 - s*m. */
static long o_anchor(long r, long s, long j, int grid) {
  return o_floordiv(o_grid_num(r, s, j, grid), 2 * r) - 1;
}

typedef struct {
  long rh, sh, rw, sw;     /* reduced factors per axis */
  long Kh, Kw;             /* dense kernel half widths */
  long H, W, Hp, Wp;       /* input and padded sizes */
  long Mh, Mw;             /* hidden-layer cells per axis */
  long Ho, Wo;             /* output sizes */
  long P;                  /* phases per channel = rh * rw */
} o_geom;

static int o_geom_init(o_geom* g, long rh, long sh, long rw, long sw, long H, long W) {
  if (rh < 1 || sh < 1 || rw < 1 || sw < 1 || H < 1 || W < 1) return -1;
  long a = o_gcd(rh, sh), b = o_gcd(rw, sw);
  g->rh = rh / a; g->sh = sh / a; g->rw = rw / b; g->sw = sw / b;
  g->Kh = o_half_width(g->sh); g->Kw = o_half_width(g->sw);
  g->H = H; g->W = W;
  g->Hp = H + 2 * g->Kh; g->Wp = W + 2 * g->Kw;
  g->Mh = (H + g->sh - 1) / g->sh; g->Mw = (W + g->sw - 1) / g->sw;
  g->Ho = g->rh * g->Mh; g->Wo = g->rw * g->Mw;
  g->P = g->rh * g->rw;
  return 0;
}

/* Dense 2D kernels for every (in-channel group, phase): the paper's conv
 * weight tensor W with (2Kh+1) x (2Kw+1) taps. For fixed methods the kernel
 * of phase (jh, jw) is the outer product of the two 1D kernels (the methods
 * are separable); for dw4 it holds W[c][jh][jw] placed at its anchor; for mix4
 * W[jh][jw][o][c]. Layout: ker[((grp * P + ph) * KH + kh) * KW + kw]. */
static double* o_build_kernels(const o_geom* g, int method, int grid, const double* weight,
                               long cin, long cout, long* ngroups_out, int absw) {
  long KH = 2 * g->Kh + 1, KW = 2 * g->Kw + 1;
  long ngroups = 1;
  if (method == OM_DW4) ngroups = cin;
  if (method == OM_MIX4) ngroups = cout * cin;
  *ngroups_out = ngroups;
  double* ker = (double*)calloc((size_t)(ngroups * g->P * KH * KW), sizeof(double));
  if (!ker) return NULL;
  if (method <= OM_BICUBIC) {
    double* hh = (double*)malloc(sizeof(double) * (size_t)KH);
    double* hw = (double*)malloc(sizeof(double) * (size_t)KW);
    for (long jh = 0; jh < g->rh; ++jh) {
      fcfs_oracle_phase_kernel(g->rh, g->sh, method, grid, jh, hh);
      for (long jw = 0; jw < g->rw; ++jw) {
        fcfs_oracle_phase_kernel(g->rw, g->sw, method, grid, jw, hw);
        double* k = ker + (jh * g->rw + jw) * KH * KW;
        for (long a = 0; a < KH; ++a)
          for (long b = 0; b < KW; ++b) k[a * KW + b] = absw ? fabs(hh[a] * hw[b]) : hh[a] * hw[b];
      }
    }
    free(hh); free(hw);
    return ker;
  }
  for (long grp = 0; grp < ngroups; ++grp) {
    for (long jh = 0; jh < g->rh; ++jh) {
      long ah = o_anchor(g->rh, g->sh, jh, grid);
      for (long jw = 0; jw < g->rw; ++jw) {
        long aw = o_anchor(g->rw, g->sw, jw, grid);
        const double* w4;
        if (method == OM_DW4) {
          w4 = weight + ((grp * g->rh + jh) * g->rw + jw) * 16;         /* [C][rh][rw][4][4] */
        } else {
          long o = grp / cin, c = grp % cin;                            /* [rh][rw][Co][Ci][4][4] */
          w4 = weight + ((((jh * g->rw + jw) * cout + o) * cin + c) * 16);
        }
        double* k = ker + (grp * g->P + jh * g->rw + jw) * KH * KW;
        for (long a = 0; a < 4; ++a)
          for (long b = 0; b < 4; ++b) {
            long kh = -(ah + a), kw = -(aw + b);   /* offset o = -k */
            k[(g->Kh + kh) * KW + (g->Kw + kw)] = absw ? fabs(w4[a * 4 + b]) : w4[a * 4 + b];
          }
      }
    }
  }
  return ker;
}

/* pad(x): materialise one padded plane. */
static void o_pad_plane(const o_geom* g, int pad, const double* x, double* xp) {
  for (long i = 0; i < g->Hp; ++i) {
    long si = o_padmap(i - g->Kh, g->H, pad);
    for (long j = 0; j < g->Wp; ++j) {
      long sj = o_padmap(j - g->Kw, g->W, pad);
      xp[i * g->Wp + j] = (si < 0 || sj < 0) ? 0.0 : x[si * g->W + sj];
    }
  }
}

/* One hidden-layer value: the strided convolution of Sec. 3 at cell (mh, mw):
 * sum_k xpad[s*m - k] h[k], with xpad indices shifted by K. */
static double o_conv_at(const o_geom* g, const double* xp, const double* k, long mh, long mw) {
  long KH = 2 * g->Kh + 1, KW = 2 * g->Kw + 1;
  double acc = 0.0;
  for (long kh = -g->Kh; kh <= g->Kh; ++kh) {
    const double* row = xp + (g->sh * mh + g->Kh - kh) * g->Wp;
    const double* krow = k + (g->Kh + kh) * KW;
    for (long kw = -g->Kw; kw <= g->Kw; ++kw)
      acc += row[g->sw * mw + g->Kw - kw] * krow[g->Kw + kw];
  }
  (void)KH;
  return acc;
}

/*
 * Forward. x: [N][Cin][H][W], y: [N][Cout][Ho][Wo] (Cout = Cin unless mix4).
 * weight: dw4 [Cin][rh][rw][4][4]; mix4 [rh][rw][Cout][Cin][4][4]; else unused.
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
static int o_forward(long rh, long sh, long rw, long sw, int method, int pad, int grid,
                     long N, long Cin, long H, long W, const double* x,
                     const double* weight, long Cout, double* y, int absw) {
  o_geom g;
  if (o_geom_init(&g, rh, sh, rw, sw, H, W)) return -1;
  if (method < 0 || method > OM_MIX4 || pad < 0 || pad > OP_REFLECT || grid < 0 || grid > OG_ASYM) return -1;
  if (method != OM_MIX4) Cout = Cin;
  if ((method == OM_DW4 || method == OM_MIX4) && !weight) return -1;
  long ngroups;
  double* ker = o_build_kernels(&g, method, grid, weight, Cin, Cout, &ngroups, absw);
  if (!ker) return -1;
  long KHW = (2 * g.Kh + 1) * (2 * g.Kw + 1);
  long plane_in = H * W, plane_p = g.Hp * g.Wp, cells = g.Mh * g.Mw;
  double* xpad = (double*)malloc(sizeof(double) * (size_t)(N * Cin * plane_p));
  double* hidden = (double*)malloc(sizeof(double) * (size_t)(N * Cout * g.P * cells));
  if (!xpad || !hidden) { free(ker); free(xpad); free(hidden); return -1; }

  /* 1. pad */
#pragma omp parallel for schedule(static)
  for (long nc = 0; nc < N * Cin; ++nc) o_pad_plane(&g, pad, x + nc * plane_in, xpad + nc * plane_p);

  /* 2. strided convolution into the hidden layer, channel index
   *    cout * P + jh * rw + jw */
#pragma omp parallel for schedule(dynamic, 1)
  for (long no = 0; no < N * Cout; ++no) {
    long n = no / Cout, o = no % Cout;
    for (long ph = 0; ph < g.P; ++ph) {
      double* hid = hidden + (no * g.P + ph) * cells;
      for (long mh = 0; mh < g.Mh; ++mh)
        for (long mw = 0; mw < g.Mw; ++mw) {
          double acc = 0.0;
          if (method == OM_MIX4) {
            for (long c = 0; c < Cin; ++c)
              acc += o_conv_at(&g, xpad + (n * Cin + c) * plane_p,
                               ker + ((o * Cin + c) * g.P + ph) * KHW, mh, mw);
          } else {
            long grp = (method == OM_DW4) ? o : 0;
            acc = o_conv_at(&g, xpad + no * plane_p, ker + (grp * g.P + ph) * KHW, mh, mw);
          }
          hid[mh * g.Mw + mw] = acc;
        }
    }
  }

  /* 3. pixelshuffle */
#pragma omp parallel for schedule(static)
  for (long no = 0; no < N * Cout; ++no)
    for (long mh = 0; mh < g.Mh; ++mh)
      for (long jh = 0; jh < g.rh; ++jh)
        for (long mw = 0; mw < g.Mw; ++mw)
          for (long jw = 0; jw < g.rw; ++jw)
            y[(no * g.Ho + g.rh * mh + jh) * g.Wo + g.rw * mw + jw] =
                hidden[(no * g.P + jh * g.rw + jw) * cells + mh * g.Mw + mw];

  free(ker); free(xpad); free(hidden);
  return 0;
}

int fcfs_oracle_forward(long rh, long sh, long rw, long sw, int method, int pad, int grid,
                        long N, long Cin, long H, long W, const double* x,
                        const double* weight, long Cout, double* y) {
  return o_forward(rh, sh, rw, sw, method, pad, grid, N, Cin, H, W, x, weight, Cout, y, 0);
}

/* Conditioning of each output for error bounds: the same pipeline with every
 * kernel tap replaced by its absolute value. Called with |x| it gives
 * S = sum over taps of |w| |x|, the scale a rounding error of the output's
 * dot product is measured against. */
int fcfs_oracle_forward_absw(long rh, long sh, long rw, long sw, int method, int pad, int grid,
                             long N, long Cin, long H, long W, const double* x,
                             const double* weight, long Cout, double* y) {
  return o_forward(rh, sh, rw, sw, method, pad, grid, N, Cin, H, W, x, weight, Cout, y, 1);
}

/*
 * Backward: the adjoint of the forward pipeline.
 * dy: [N][Cout][Ho][Wo]. dx (nullable): [N][Cin][H][W]. dw (nullable, dw4/mix4
 * only): same layout as weight. x is needed only for dw.
 */
static int o_backward(long rh, long sh, long rw, long sw, int method, int pad, int grid,
                      long N, long Cin, long H, long W, const double* x,
                      const double* weight, long Cout, const double* dy,
                      double* dx, double* dw, int absw) {
  o_geom g;
  if (o_geom_init(&g, rh, sh, rw, sw, H, W)) return -1;
  if (method < 0 || method > OM_MIX4 || pad < 0 || pad > OP_REFLECT || grid < 0 || grid > OG_ASYM) return -1;
  if (method != OM_MIX4) Cout = Cin;
  int learned = (method == OM_DW4 || method == OM_MIX4);
  if (learned && !weight) return -1;
  if (dw && (!learned || !x)) return -1;
  long ngroups;
  double* ker = o_build_kernels(&g, method, grid, weight, Cin, Cout, &ngroups, absw);
  if (!ker) return -1;
  long KH = 2 * g.Kh + 1, KW = 2 * g.Kw + 1, KHW = KH * KW;
  long plane_in = H * W, plane_p = g.Hp * g.Wp, cells = g.Mh * g.Mw;
  double* dhid = (double*)malloc(sizeof(double) * (size_t)(N * Cout * g.P * cells));
  if (!dhid) { free(ker); return -1; }

  /* adjoint of pixelshuffle */
#pragma omp parallel for schedule(static)
  for (long no = 0; no < N * Cout; ++no)
    for (long mh = 0; mh < g.Mh; ++mh)
      for (long jh = 0; jh < g.rh; ++jh)
        for (long mw = 0; mw < g.Mw; ++mw)
          for (long jw = 0; jw < g.rw; ++jw)
            dhid[(no * g.P + jh * g.rw + jw) * cells + mh * g.Mw + mw] =
                dy[(no * g.Ho + g.rh * mh + jh) * g.Wo + g.rw * mw + jw];

  int rc = 0;
  if (dx) {
    double* dxpad = (double*)calloc((size_t)(N * Cin * plane_p), sizeof(double));
    if (!dxpad) { rc = -1; goto done; }
    /* adjoint of the strided convolution: scatter every hidden value back
     * through its kernel onto the padded input */
#pragma omp parallel for schedule(dynamic, 1)
    for (long nc = 0; nc < N * Cin; ++nc) {
      long n = nc / Cin, c = nc % Cin;
      double* dp = dxpad + nc * plane_p;
      long olo = (method == OM_MIX4) ? 0 : c, ohi = (method == OM_MIX4) ? Cout : c + 1;
      for (long o = olo; o < ohi; ++o) {
        long grp = (method == OM_MIX4) ? o * Cin + c : (method == OM_DW4 ? c : 0);
        for (long ph = 0; ph < g.P; ++ph) {
          const double* k = ker + (grp * g.P + ph) * KHW;
          const double* dh = dhid + ((n * Cout + o) * g.P + ph) * cells;
          for (long mh = 0; mh < g.Mh; ++mh)
            for (long mw = 0; mw < g.Mw; ++mw) {
              double v = dh[mh * g.Mw + mw];
              for (long kh = -g.Kh; kh <= g.Kh; ++kh) {
                double* row = dp + (g.sh * mh + g.Kh - kh) * g.Wp;
                const double* krow = k + (g.Kh + kh) * KW;
                for (long kw = -g.Kw; kw <= g.Kw; ++kw)
                  row[g.sw * mw + g.Kw - kw] += krow[g.Kw + kw] * v;
              }
            }
        }
      }
    }
    /* adjoint of the padding: fold padded positions back to their sources */
#pragma omp parallel for schedule(static)
    for (long nc = 0; nc < N * Cin; ++nc) {
      double* d = dx + nc * plane_in;
      const double* dp = dxpad + nc * plane_p;
      for (long i = 0; i < plane_in; ++i) d[i] = 0.0;
      for (long i = 0; i < g.Hp; ++i) {
        long si = o_padmap(i - g.Kh, H, pad);
        if (si < 0) continue;
        for (long j = 0; j < g.Wp; ++j) {
          long sj = o_padmap(j - g.Kw, W, pad);
          if (sj < 0) continue;
          d[si * W + sj] += dp[i * g.Wp + j];
        }
      }
    }
    free(dxpad);
  }

  if (dw) {
    double* xpad = (double*)malloc(sizeof(double) * (size_t)(N * Cin * plane_p));
    double* dker = (double*)calloc((size_t)(ngroups * g.P * KHW), sizeof(double));
    if (!xpad || !dker) { free(xpad); free(dker); rc = -1; goto done; }
#pragma omp parallel for schedule(static)
    for (long nc = 0; nc < N * Cin; ++nc) o_pad_plane(&g, pad, x + nc * plane_in, xpad + nc * plane_p);
    /* gradient of every dense kernel tap: sum over batch and cells of
     * dhidden * the input sample that tap multiplies */
#pragma omp parallel for schedule(dynamic, 1)
    for (long grp = 0; grp < ngroups; ++grp) {
      long o = (method == OM_MIX4) ? grp / Cin : grp;
      long c = (method == OM_MIX4) ? grp % Cin : grp;
      for (long ph = 0; ph < g.P; ++ph) {
        double* dk = dker + (grp * g.P + ph) * KHW;
        for (long n = 0; n < N; ++n) {
          const double* xp = xpad + (n * Cin + c) * plane_p;
          const double* dh = dhid + ((n * Cout + o) * g.P + ph) * cells;
          for (long mh = 0; mh < g.Mh; ++mh)
            for (long mw = 0; mw < g.Mw; ++mw) {
              double v = dh[mh * g.Mw + mw];
              for (long kh = -g.Kh; kh <= g.Kh; ++kh) {
                const double* row = xp + (g.sh * mh + g.Kh - kh) * g.Wp;
                double* dkrow = dk + (g.Kh + kh) * KW;
                for (long kw = -g.Kw; kw <= g.Kw; ++kw)
                  dkrow[g.Kw + kw] += row[g.sw * mw + g.Kw - kw] * v;
              }
            }
        }
      }
    }
    /* the learnable weights are the dense taps at their anchors */
    for (long grp = 0; grp < ngroups; ++grp)
      for (long jh = 0; jh < g.rh; ++jh) {
        long ah = o_anchor(g.rh, g.sh, jh, grid);
        for (long jw = 0; jw < g.rw; ++jw) {
          long aw = o_anchor(g.rw, g.sw, jw, grid);
          const double* dk = dker + (grp * g.P + jh * g.rw + jw) * KHW;
          double* d4;
          if (method == OM_DW4) d4 = dw + ((grp * g.rh + jh) * g.rw + jw) * 16;
          else {
            long o = grp / Cin, c = grp % Cin;
            d4 = dw + ((((jh * g.rw + jw) * Cout + o) * Cin + c) * 16);
          }
          for (long a = 0; a < 4; ++a)
            for (long b = 0; b < 4; ++b)
              d4[a * 4 + b] = dk[(g.Kh - (ah + a)) * KW + (g.Kw - (aw + b))];
        }
      }
    free(xpad); free(dker);
  }
done:
  free(ker); free(dhid);
  return rc;
}

int fcfs_oracle_backward(long rh, long sh, long rw, long sw, int method, int pad, int grid,
                         long N, long Cin, long H, long W, const double* x,
                         const double* weight, long Cout, const double* dy,
                         double* dx, double* dw) {
  return o_backward(rh, sh, rw, sw, method, pad, grid, N, Cin, H, W, x, weight, Cout, dy, dx, dw, 0);
}

/* Conditioning of the input gradient for error bounds: the adjoint with every
 * kernel tap replaced by its absolute value (apply it to |dy|). */
int fcfs_oracle_backward_absw(long rh, long sh, long rw, long sw, int method, int pad, int grid,
                              long N, long Cin, long H, long W, const double* x,
                              const double* weight, long Cout, const double* dy,
                              double* dx, double* dw) {
  return o_backward(rh, sh, rw, sw, method, pad, grid, N, Cin, H, W, x, weight, Cout, dy, dx, dw, 1);
}

/* Threads later parallel regions use (for timing the oracle on one core). */
void fcfs_oracle_set_threads(int n) {
#ifdef _OPENMP
  extern void omp_set_num_threads(int);
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* Number of OpenMP threads a parallel region uses (for reporting). */
int fcfs_oracle_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}
