"""CPU pins of the oracle's conditioning scales.

Every GPU parity bound is u|r| + 1e-5 S, with S the sum over an output's taps
of |weight| * |input sample| (``oracle.condition``), and for gradients the
same sum over the adjoint's terms (``oracle.condition_backward``). A wrong S
would loosen or tighten every parity test at once, so S is pinned here to a
computation that shares nothing with the oracle's pipeline: the tap lists of
the exact-rational direct sampler (``oracle.exact.axis_weights``: the
interpolant of Sec. 5.2 evaluated at the mapped coordinate, no phase tables,
no dense kernels, no padding buffer), or, for the learned layers, the 4x4
window anchored at floor(u) - 1 written out from the coordinate, summed per
tap in exact rationals.
"""
from fractions import Fraction
from math import floor, gcd

import numpy as np
import pytest

import oracle
from oracle import exact
import synth

METHODS = ["nearest", "bilinear", "bicubic"]
PADS = ["zero", "replicate", "reflect"]
FRACS = [(3, 2), (2, 3), (5, 4), (4, 5), (3, 4), (1, 1), (4, 1), (2, 11), (27, 11)]


def _reduce(p, q):
    g = gcd(p, q)
    return p // g, q // g


def _fixed_taps(k, p, q, method, grid):
    """[(input index, exact weight)] of output k on one axis."""
    return exact.axis_weights(k, p, q, method, grid)


def _window(k, p, q, grid="half"):
    """(phase j, first input index) of the 4-tap learned window of output k:
    4 taps from floor(u_k) - 1."""
    return k % p, floor(exact.coord(k, p, q, grid)) - 1


def _x_at(xf, i, j, pad):
    """Exact value of the padded plane at (i, j), or 0 for a zero pad."""
    H, W = len(xf), len(xf[0])
    si, sj = exact.ext_index(i, H, pad), exact.ext_index(j, W, pad)
    if si is None or sj is None:
        return Fraction(0)
    return xf[si][sj]


def _exact_plane(a):
    return [[Fraction(float(v)) for v in row] for row in a]


def _close(got, ref, what, scale=1.0):
    """Equal up to the FP64 evaluation of the weights: each weight of the
    oracle carries an absolute error of a few units of 2^-53, so the sum can
    differ from the exact one by about 16 such errors times the largest
    sample (``scale``). A dropped, duplicated or misplaced tap changes S by a
    weight times a sample, many orders of magnitude more."""
    ref = np.asarray(ref, dtype=np.float64)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-14 * scale, err_msg=what)


# ------------------------------------------------------------- forward scale

def _cases_fixed():
    out = []
    for (p, q) in FRACS:
        for m in METHODS:
            for pad in PADS:
                out.append((p, q, m, pad, "half"))
    for (p, q) in [(3, 2), (2, 3), (5, 4)]:
        for g in ("paper", "asym"):
            out.append((p, q, "bicubic", "reflect", g))
    return out


@pytest.mark.parametrize("case", _cases_fixed())
def test_condition_fixed_equals_per_tap_abs_sum(case):
    p, q, method, pad, grid = case
    pr, qr = _reduce(p, q)
    shape = (1, 2, 7, 6) if qr < 10 else (1, 1, 12, 13)
    # signed inputs, so |x| differs from x
    x = synth.normal(500 + 7 * p + q, shape).astype(np.float64)
    S = oracle.condition(x, p, q, method, pad, grid)
    Ho, Wo = exact.out_len(pr, qr, shape[2]), exact.out_len(pr, qr, shape[3])
    assert S.shape == (shape[0], shape[1], Ho, Wo)
    wh = [_fixed_taps(k, pr, qr, method, grid) for k in range(Ho)]
    ww = [_fixed_taps(k, pr, qr, method, grid) for k in range(Wo)]
    for c in range(shape[1]):
        xf = _exact_plane(x[0, c])
        ref = [[sum((abs(ah * aw) * abs(_x_at(xf, ih, iw, pad))
                     for ih, ah in wh[kh] for iw, aw in ww[kw]), Fraction(0))
                for kw in range(Wo)] for kh in range(Ho)]
        _close(S[0, c], [[float(v) for v in r] for r in ref], f"{case} c={c}", np.abs(x).max())


@pytest.mark.parametrize("p,q", FRACS)
@pytest.mark.parametrize("method", ["nearest", "bilinear"])
@pytest.mark.parametrize("pad", PADS)
def test_condition_nonnegative_taps_is_forward_of_abs(p, q, method, pad):
    # nearest and bilinear weights are >= 0, so sum |w||x| = forward(|x|)
    x = synth.normal(600 + p + q, (2, 2, 9, 8)).astype(np.float64)
    S = oracle.condition(x, p, q, method, pad)
    np.testing.assert_array_equal(S, oracle.forward(np.abs(x), p, q, method, pad))


def test_condition_bicubic_exceeds_forward_of_abs_where_taps_are_negative():
    # bicubic has negative side taps, so S is larger than forward(|x|)
    # wherever a negative tap product meets a nonzero sample. One unit
    # sample at (2, 2), 3/2 on the half grid, u_k = (2k + 1)/3 - 1/2:
    x = np.zeros((1, 1, 6, 6))
    x[0, 0, 2, 2] = 1.0
    S = oracle.condition(x, 3, 2, "bicubic", "zero")
    F = oracle.forward(np.abs(x), 3, 2, "bicubic", "zero")
    assert (S >= F - 1e-15).all()
    assert (S > F + 1e-6).any()
    # k = 1: u = 1/2, taps at -1..2, sample 2 is the last tap, W(3/2) = -1/16
    w_last = exact.keys_cubic(Fraction(1, 2) - 2)
    assert w_last == Fraction(-1, 16)
    # output (1, 1): the only nonzero tap has weight (-1/16)^2, so S = F = 1/256
    assert abs(S[0, 0, 1, 1] - 1 / 256) < 1e-16
    assert abs(F[0, 0, 1, 1] - 1 / 256) < 1e-16
    # output (1, 2): column u = 7/6, taps 0..3, sample 2 has weight W(5/6) > 0,
    # so the product is -W(5/6)/16: S = W(5/6)/16 while F = -W(5/6)/16
    w56 = float(exact.keys_cubic(Fraction(5, 6)))
    assert w56 > 0
    assert abs(S[0, 0, 1, 2] - w56 / 16) < 1e-16
    assert abs(F[0, 0, 1, 2] + w56 / 16) < 1e-16


def _learned_cases():
    return [(p, q, pad) for (p, q) in [(3, 4), (3, 2), (5, 4), (2, 3), (2, 11), (4, 1)] for pad in PADS]


@pytest.mark.parametrize("p,q,pad", _learned_cases())
def test_condition_dw4_equals_window_abs_sum(p, q, pad):
    pr, qr = _reduce(p, q)
    shape = (1, 2, 7, 6) if qr < 10 else (1, 1, 12, 13)
    x = synth.normal(700 + p + q, shape).astype(np.float64)
    w = synth.normal(701 + p, (shape[1], pr, pr, 4, 4)).astype(np.float64)
    S = oracle.condition(x, p, q, "dw4", pad, weight=w)
    Ho, Wo = exact.out_len(pr, qr, shape[2]), exact.out_len(pr, qr, shape[3])
    for c in range(shape[1]):
        xf = _exact_plane(x[0, c])
        ref = np.zeros((Ho, Wo))
        for kh in range(Ho):
            jh, ih0 = _window(kh, pr, qr)
            for kw in range(Wo):
                jw, iw0 = _window(kw, pr, qr)
                acc = Fraction(0)
                for a in range(4):
                    for b in range(4):
                        acc += abs(Fraction(float(w[c, jh, jw, a, b]))) * abs(_x_at(xf, ih0 + a, iw0 + b, pad))
                ref[kh, kw] = float(acc)
        _close(S[0, c], ref, f"dw4 {p}/{q} {pad} c={c}", np.abs(x).max() * np.abs(w).max())


@pytest.mark.parametrize("p,q,pad", _learned_cases())
def test_condition_mix4_equals_window_abs_sum(p, q, pad):
    pr, qr = _reduce(p, q)
    shape = (1, 3, 6, 7) if qr < 10 else (1, 2, 12, 12)
    co = 2
    x = synth.normal(800 + p + q, shape).astype(np.float64)
    w = synth.normal(801 + p, (pr, pr, co, shape[1], 4, 4)).astype(np.float64)
    S = oracle.condition(x, p, q, "mix4", pad, weight=w, cout=co)
    Ho, Wo = exact.out_len(pr, qr, shape[2]), exact.out_len(pr, qr, shape[3])
    assert S.shape == (1, co, Ho, Wo)
    xf = [_exact_plane(x[0, c]) for c in range(shape[1])]
    for o in range(co):
        ref = np.zeros((Ho, Wo))
        for kh in range(Ho):
            jh, ih0 = _window(kh, pr, qr)
            for kw in range(Wo):
                jw, iw0 = _window(kw, pr, qr)
                acc = Fraction(0)
                for c in range(shape[1]):
                    for a in range(4):
                        for b in range(4):
                            acc += (abs(Fraction(float(w[jh, jw, o, c, a, b])))
                                    * abs(_x_at(xf[c], ih0 + a, iw0 + b, pad)))
                ref[kh, kw] = float(acc)
        _close(S[0, o], ref, f"mix4 {p}/{q} {pad} o={o}", np.abs(x).max() * np.abs(w).max())


def test_condition_scales_with_inputs_and_weights():
    # S is absolutely homogeneous of degree 1 in x and in the weights, and
    # blind to their signs
    x = synth.normal(900, (1, 2, 8, 7)).astype(np.float64)
    w = synth.normal(901, (2, 3, 3, 4, 4)).astype(np.float64)
    S = oracle.condition(x, 3, 4, "dw4", "reflect", weight=w)
    np.testing.assert_array_equal(oracle.condition(-x, 3, 4, "dw4", "reflect", weight=-w), S)
    np.testing.assert_allclose(oracle.condition(2.0 * x, 3, 4, "dw4", "reflect", weight=-3.0 * w),
                               6.0 * S, rtol=1e-15)


# ------------------------------------------------------------ backward scales

def _fixed_adjoint_scale(dy_plane, H, W, p, q, method, pad, grid="half"):
    """sum over (output, tap) with ext(tap) = input sample of |w| |dy|, in
    exact rationals, walking the direct sampler's taps."""
    Ho, Wo = len(dy_plane), len(dy_plane[0])
    wh = [_fixed_taps(k, p, q, method, grid) for k in range(Ho)]
    ww = [_fixed_taps(k, p, q, method, grid) for k in range(Wo)]
    acc = [[Fraction(0)] * W for _ in range(H)]
    for kh in range(Ho):
        for kw in range(Wo):
            g = abs(dy_plane[kh][kw])
            for ih, ah in wh[kh]:
                si = exact.ext_index(ih, H, pad)
                if si is None:
                    continue
                for iw, aw in ww[kw]:
                    sj = exact.ext_index(iw, W, pad)
                    if sj is None:
                        continue
                    acc[si][sj] += abs(ah * aw) * g
    return np.array([[float(v) for v in r] for r in acc])


@pytest.mark.parametrize("p,q", [(3, 2), (2, 3), (5, 4), (3, 4), (4, 1), (2, 11)])
@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("pad", PADS)
def test_condition_backward_fixed_per_tap(p, q, method, pad):
    pr, qr = _reduce(p, q)
    H, W = (6, 5) if qr < 10 else (12, 13)
    Ho, Wo = exact.out_len(pr, qr, H), exact.out_len(pr, qr, W)
    dy = synth.normal(1000 + p + q, (1, 2, Ho, Wo)).astype(np.float64)
    S_dx, S_dw = oracle.condition_backward(dy, (1, 2, H, W), p, q, method, pad)
    assert S_dw is None
    for c in range(2):
        ref = _fixed_adjoint_scale(_exact_plane(dy[0, c]), H, W, pr, qr, method, pad)
        _close(S_dx[0, c], ref, f"{p}/{q} {method} {pad} c={c}", np.abs(dy).max())


@pytest.mark.parametrize("pad", PADS)
def test_condition_backward_bounds_abs_jacobian(pad):
    # |J|^T |dy| <= S_dx elementwise (taps of one output landing on the same
    # sample may cancel in J but not in S), with equality for zero padding,
    # where no two taps of one output share a sample; J from Jacobian columns
    # of the direct sampler
    p, q, method = 3, 2, "bicubic"
    H, W = 4, 5
    dy = synth.normal(1100, (1, 1, 6, 9)).astype(np.float64)
    S_dx, _ = oracle.condition_backward(dy, (1, 1, H, W), p, q, method, pad)
    lower = np.zeros((H, W))
    for i in range(H):
        for j in range(W):
            e = np.zeros((H, W))
            e[i, j] = 1.0
            col = np.array([[float(v) for v in r] for r in exact.resample2d(e, p, q, method, pad)])
            lower[i, j] = (np.abs(col) * np.abs(dy[0, 0])).sum()
    assert (lower <= S_dx[0, 0] * (1 + 1e-13)).all()
    if pad == "zero":
        np.testing.assert_allclose(S_dx[0, 0], lower, rtol=1e-13)
    else:
        assert (S_dx[0, 0] > lower * (1 + 1e-9)).any()


@pytest.mark.parametrize("p,q,pad", [(3, 4, "reflect"), (3, 2, "zero"), (5, 4, "replicate"),
                                     (2, 3, "reflect"), (4, 1, "zero")])
def test_condition_backward_dw4(p, q, pad):
    pr, qr = _reduce(p, q)
    N, C, H, W = 2, 2, 7, 6
    Ho, Wo = exact.out_len(pr, qr, H), exact.out_len(pr, qr, W)
    x = synth.normal(1200 + p, (N, C, H, W)).astype(np.float64)
    w = synth.normal(1201 + q, (C, pr, pr, 4, 4)).astype(np.float64)
    dy = synth.normal(1202, (N, C, Ho, Wo)).astype(np.float64)
    S_dx, S_dw = oracle.condition_backward(dy, x.shape, p, q, "dw4", pad, x=x, weight=w, need_dw=True)
    ref_dx = np.zeros((N, C, H, W))
    ref_dw = np.zeros((C, pr, pr, 4, 4))
    for n in range(N):
        for c in range(C):
            xf = _exact_plane(x[n, c])
            acc_dx = [[Fraction(0)] * W for _ in range(H)]
            acc_dw = {}
            for kh in range(Ho):
                jh, ih0 = _window(kh, pr, qr)
                for kw in range(Wo):
                    jw, iw0 = _window(kw, pr, qr)
                    g = abs(Fraction(float(dy[n, c, kh, kw])))
                    for a in range(4):
                        si = exact.ext_index(ih0 + a, H, pad)
                        for b in range(4):
                            sj = exact.ext_index(iw0 + b, W, pad)
                            key = (jh, jw, a, b)
                            acc_dw[key] = acc_dw.get(key, Fraction(0)) + g * abs(_x_at(xf, ih0 + a, iw0 + b, pad))
                            if si is None or sj is None:
                                continue
                            acc_dx[si][sj] += abs(Fraction(float(w[c, jh, jw, a, b]))) * g
            ref_dx[n, c] = [[float(v) for v in r] for r in acc_dx]
            for (jh, jw, a, b), v in acc_dw.items():
                ref_dw[c, jh, jw, a, b] += float(v)
    _close(S_dx, ref_dx, f"dw4 S_dx {p}/{q} {pad}", np.abs(dy).max() * np.abs(w).max())
    np.testing.assert_allclose(S_dw, ref_dw, rtol=1e-12, err_msg=f"dw4 S_dw {p}/{q} {pad}")


@pytest.mark.parametrize("p,q,pad", [(3, 4, "reflect"), (5, 4, "zero"), (2, 3, "replicate")])
def test_condition_backward_mix4(p, q, pad):
    pr, qr = _reduce(p, q)
    N, C, CO, H, W = 1, 3, 2, 6, 7
    Ho, Wo = exact.out_len(pr, qr, H), exact.out_len(pr, qr, W)
    x = synth.normal(1300 + p, (N, C, H, W)).astype(np.float64)
    w = synth.normal(1301 + q, (pr, pr, CO, C, 4, 4)).astype(np.float64)
    dy = synth.normal(1302, (N, CO, Ho, Wo)).astype(np.float64)
    S_dx, S_dw = oracle.condition_backward(dy, x.shape, p, q, "mix4", pad, x=x, weight=w, need_dw=True)
    ref_dx = np.zeros((N, C, H, W))
    ref_dw = np.zeros((pr, pr, CO, C, 4, 4))
    xf = [_exact_plane(x[0, c]) for c in range(C)]
    for c in range(C):
        acc_dx = [[Fraction(0)] * W for _ in range(H)]
        for o in range(CO):
            acc_dw = {}
            for kh in range(Ho):
                jh, ih0 = _window(kh, pr, qr)
                for kw in range(Wo):
                    jw, iw0 = _window(kw, pr, qr)
                    g = abs(Fraction(float(dy[0, o, kh, kw])))
                    for a in range(4):
                        si = exact.ext_index(ih0 + a, H, pad)
                        for b in range(4):
                            sj = exact.ext_index(iw0 + b, W, pad)
                            key = (jh, jw, a, b)
                            acc_dw[key] = acc_dw.get(key, Fraction(0)) + g * abs(_x_at(xf[c], ih0 + a, iw0 + b, pad))
                            if si is None or sj is None:
                                continue
                            acc_dx[si][sj] += abs(Fraction(float(w[jh, jw, o, c, a, b]))) * g
            for (jh, jw, a, b), v in acc_dw.items():
                ref_dw[jh, jw, o, c, a, b] = float(v)
        ref_dx[0, c] = [[float(v) for v in r] for r in acc_dx]
    _close(S_dx, ref_dx, f"mix4 S_dx {p}/{q} {pad}", np.abs(dy).max() * np.abs(w).max())
    _close(S_dw, ref_dw, f"mix4 S_dw {p}/{q} {pad}", np.abs(dy).max() * np.abs(x).max())
