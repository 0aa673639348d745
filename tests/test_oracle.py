"""CPU pins of the FP64 oracle against what the paper and the mathematics fix.

Each test pins the oracle to something other than itself: the exact-rational
direct sampler (a different construction: no phases, no dense kernels, no
padding buffer, no pixelshuffle), closed forms (ramps, quadratics, constants,
identity), the kernels printed in the paper, numpy/torch library routines and
the adjoint identities.
"""
import itertools
import json
import os
from fractions import Fraction
from math import floor

import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
from oracle import exact
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
METHODS = ["nearest", "bilinear", "bicubic"]
PADS = ["zero", "replicate", "reflect"]


def _frac_array(rows):
    return np.array([[float(v) for v in r] for r in rows], dtype=np.float64)


# ---------------------------------------------------------------- sizes

def test_output_sizes_printed():
    with open(os.path.join(GOLD, "output_sizes.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        assert oracle.out_len(c["p"], c["q"], c["n"]) == c["out"], c
    # the 5x5 example end to end
    y = oracle.forward(np.zeros((1, 1, 5, 5)), 3, 2, "bilinear", "zero")
    assert y.shape == (1, 1, 9, 9)


@pytest.mark.parametrize("p,q,n,out", [
    (3, 2, 64, 96), (2, 3, 64, 44), (3, 2, 1024, 1536), (2, 3, 1024, 684),
    (5, 4, 1024, 1280), (4, 5, 1024, 820), (3, 4, 256, 192), (5, 4, 512, 640),
    (4, 6, 67, 46), (6, 4, 5, 9), (7, 7, 13, 13), (2, 11, 1024, 188), (27, 11, 64, 162),
])
def test_output_size_closed_form(p, q, n, out):
    # p * ceil(n / q) after reducing p/q by its gcd
    assert oracle.out_len(p, q, n) == out


# ---------------------------------------------------------------- padding

@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_ext_index_matches_numpy_pad(n):
    x = np.arange(n, dtype=np.float64) + 10.0
    for pad, mode in [("zero", "constant"), ("replicate", "edge"), ("reflect", "reflect")]:
        width = 3 * n + 4
        if mode == "reflect" and n == 1:
            ref = np.full(n + 2 * width, x[0])
        else:
            ref = np.pad(x, width, mode=mode)
        got = []
        for i in range(-width, n + width):
            s = exact.ext_index(i, n, pad)
            got.append(0.0 if s is None else x[s])
        np.testing.assert_array_equal(np.array(got), ref, err_msg=f"{pad} n={n}")


# ---------------------------------------------------------------- direct sampler

def _cases_tiny():
    fracs = [(1, 1), (3, 2), (2, 3), (5, 4), (4, 5), (1, 2), (2, 1), (3, 4), (7, 3), (6, 4), (2, 11)]
    sizes = [(1, 1), (1, 4), (3, 2), (5, 5), (7, 4)]
    rng = np.random.default_rng(123)
    out = []
    for (p, q), (H, W), m, pad in itertools.product(fracs, sizes, METHODS, PADS):
        out.append((p, q, H, W, m, pad, "half"))
    # other grids and anisotropic factors on a sample
    for _ in range(40):
        p, q = fracs[rng.integers(len(fracs))]
        pw, qw = fracs[rng.integers(len(fracs))]
        H, W = sizes[rng.integers(len(sizes))]
        out.append((p, q, H, W, METHODS[rng.integers(3)], PADS[rng.integers(3)],
                    ["half", "paper", "asym"][rng.integers(3)], pw, qw))
    return out


@pytest.mark.parametrize("case", _cases_tiny())
def test_pipeline_equals_direct_sampler(case):
    p, q, H, W, method, pad, grid = case[:7]
    pw, qw = (case[7], case[8]) if len(case) > 7 else (p, q)
    x = synth.uniform(1000 + H * 31 + W, (1, 2, H, W)).astype(np.float64) - 0.25
    y = oracle.forward(x, p, q, method, pad, grid, pw=pw, qw=qw)
    for c in range(2):
        ref = _frac_array(exact.resample2d(x[0, c], p, q, method, pad, grid, pw=pw, qw=qw))
        assert y.shape[2:] == ref.shape
        np.testing.assert_allclose(y[0, c], ref, rtol=0, atol=1e-12)


def test_paper_extreme_fractions_direct():
    # the two factors the paper shows (2/11 down, 27/11 up)
    x = synth.uniform(7, (1, 1, 12, 13)).astype(np.float64)
    for p, q in [(2, 11), (27, 11)]:
        for m in METHODS:
            for pad in PADS:
                y = oracle.forward(x, p, q, m, pad)
                ref = _frac_array(exact.resample2d(x[0, 0], p, q, m, pad))
                np.testing.assert_allclose(y[0, 0], ref, rtol=0, atol=1e-12)


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("p", [1, 2, 3, 5])
@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("pad", PADS)
def test_identity_when_p_equals_q(p, method, pad):
    x = synth.normal(3, (2, 3, 7, 5)).astype(np.float64)
    y = oracle.forward(x, p, p, method, pad)
    np.testing.assert_array_equal(y, x)


def _interior(k_list, n, method):
    lo, hi = {"nearest": (0, 0), "bilinear": (0, 1), "bicubic": (-1, 2)}[method]
    return [k for k, u in k_list if floor(u) + lo >= 0 and floor(u) + hi <= n - 1
            and (method != "nearest" or floor(u + Fraction(1, 2)) <= n - 1)]


@pytest.mark.parametrize("p,q", [(3, 2), (2, 3), (5, 4), (4, 5), (3, 4), (7, 3), (2, 11), (27, 11)])
@pytest.mark.parametrize("method", ["bilinear", "bicubic"])
def test_linear_ramp_reproduced(p, q, method):
    # x_i = a*i + b along each axis: interior outputs equal a*u_k + b, with
    # u_k = (k + 1/2) q/p - 1/2 the half-pixel coordinate written out here.
    H, W = 23, 29
    a_h, a_w, b = 0.75, -1.25, 3.0
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    x = (a_h * ii + a_w * jj + b)[None, None].astype(np.float64)
    for pad in PADS:
        y = oracle.forward(x, p, q, method, pad)[0, 0]
        from math import gcd
        g = gcd(p, q)
        pr, qr = p // g, q // g
        uh = [(k, (Fraction(2 * k + 1) * qr / (2 * pr)) - Fraction(1, 2)) for k in range(y.shape[0])]
        uw = [(k, (Fraction(2 * k + 1) * qr / (2 * pr)) - Fraction(1, 2)) for k in range(y.shape[1])]
        kh = _interior(uh, H, method)
        kw = _interior(uw, W, method)
        assert len(kh) > 0 and len(kw) > 0
        for i in kh:
            for j in kw:
                ref = a_h * float(uh[i][1]) + a_w * float(uw[j][1]) + b
                assert abs(y[i, j] - ref) < 1e-12, (pad, i, j)


@pytest.mark.parametrize("p,q", [(3, 2), (2, 3), (5, 4), (3, 4), (27, 11)])
def test_bicubic_reproduces_quadratics(p, q):
    # Keys' cubic with a = -1/2 reproduces polynomials of degree 2
    H, W = 17, 19
    ii, jj = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    x = (0.5 * ii * ii - 0.25 * jj * jj + ii * jj - 2.0)[None, None]
    y = oracle.forward(x, p, q, "bicubic", "replicate")[0, 0]
    from math import gcd
    g = gcd(p, q)
    pr, qr = p // g, q // g
    uh = [(k, Fraction(2 * k + 1) * qr / (2 * pr) - Fraction(1, 2)) for k in range(y.shape[0])]
    uw = [(k, Fraction(2 * k + 1) * qr / (2 * pr) - Fraction(1, 2)) for k in range(y.shape[1])]
    for i in _interior(uh, H, "bicubic"):
        for j in _interior(uw, W, "bicubic"):
            a, c = uh[i][1], uw[j][1]
            ref = float(Fraction(1, 2) * a * a - Fraction(1, 4) * c * c + a * c - 2)
            assert abs(y[i, j] - ref) < 1e-11


def test_quadratic_worked_example():
    # x = [0, 1, 4, 9, 16] at 3/2: the sampling points are u_k = k*2/3 - 1/6,
    # so bicubic interior outputs are u_k^2 = 49/36, 121/36, 25/4 (k = 2, 3, 4).
    row = np.array([0, 1, 4, 9, 16], dtype=np.float64)
    x = np.tile(row, (5, 1))[None, None]
    for pad in PADS:
        y = oracle.forward(x, 3, 2, "bicubic", pad)[0, 0, 3]
        np.testing.assert_allclose(y[2:5], [49 / 36, 121 / 36, 25 / 4], rtol=0, atol=1e-13)
    # reflect is even about 0, so u^2 also holds at k = 0, 1
    y = oracle.forward(x, 3, 2, "bicubic", "reflect")[0, 0, 3]
    np.testing.assert_allclose(y[:2], [1 / 36, 1 / 4], rtol=0, atol=1e-13)
    # zero padding at k = 0: W(5/6)*0 + W(1/6)*1 + W(7/6)*4 = -25/432
    y = oracle.forward(x, 3, 2, "bicubic", "zero")[0, 0, 3]
    assert abs(y[0] - (-25 / 432)) < 1e-14


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("p,q", [(3, 2), (2, 3), (5, 4), (4, 5), (2, 11)])
def test_constant_image(method, p, q):
    x = np.full((1, 2, 9, 11), 2.5)
    for pad in ["replicate", "reflect"]:
        y = oracle.forward(x, p, q, method, pad)
        np.testing.assert_allclose(y, 2.5, rtol=0, atol=1e-13)


@pytest.mark.parametrize("p,q", [(3, 2), (5, 4), (2, 3)])
def test_shift_equivariance(p, q):
    # shifting the input by q samples shifts the output by p (interior)
    x = synth.normal(11, (1, 1, 8, 30)).astype(np.float64)
    xs = x[..., q:]
    for m in METHODS:
        y = oracle.forward(x, p, q, m, "replicate")
        ys = oracle.forward(xs, p, q, m, "replicate")
        n = ys.shape[-1] - 2 * p - 8
        np.testing.assert_allclose(ys[..., 4:4 + n], y[..., p + 4: p + 4 + n], atol=1e-13)


# ---------------------------------------------------------------- weights

def test_keys_closed_forms():
    # taps at -1, 0, 1, 2 for fractional offsets t = 0, 1/2, 1/3
    for t, ref in [(Fraction(0), [0, 1, 0, 0]),
                   (Fraction(1, 2), [Fraction(-1, 16), Fraction(9, 16), Fraction(9, 16), Fraction(-1, 16)]),
                   (Fraction(1, 3), [Fraction(-2, 27), Fraction(21, 27), Fraction(9, 27), Fraction(-1, 27)])]:
        got = [exact.keys_cubic(t - i) for i in (-1, 0, 1, 2)]
        assert got == ref
    # the oracle's dense kernels: 1/2 on the half grid has t = 1/2 at every cell
    h = oracle.phase_kernel(1, 2, "bicubic", "half", 0)
    K = (len(h) - 1) // 2
    taps = [h[K - o] for o in (-1, 0, 1, 2)]
    np.testing.assert_allclose(taps, [-1 / 16, 9 / 16, 9 / 16, -1 / 16], atol=1e-15)
    # 3/2 on the paper grid, phase 0 has t = 1/3
    h = oracle.phase_kernel(3, 2, "bicubic", "paper", 0)
    K = (len(h) - 1) // 2
    np.testing.assert_allclose([h[K - o] for o in (-1, 0, 1, 2)],
                               [-2 / 27, 21 / 27, 9 / 27, -1 / 27], atol=1e-15)


@pytest.mark.parametrize("p,q", [(3, 2), (2, 3), (5, 4), (4, 5), (27, 11)])
@pytest.mark.parametrize("grid", ["half", "paper", "asym"])
def test_kernel_moments(p, q, grid):
    from math import gcd
    g = gcd(p, q)
    pr, qr = p // g, q // g
    for j in range(pr):
        u = exact.coord(j, pr, qr, grid)     # offset of channel j from q*m
        for m in METHODS:
            h = oracle.phase_kernel(p, q, m, grid, j)
            K = (len(h) - 1) // 2
            offs = np.array([-k for k in range(-K, K + 1)], dtype=np.float64)
            assert abs(h.sum() - 1.0) < 1e-14                       # partition of unity
            if m != "nearest":
                assert abs((h * offs).sum() - float(u)) < 1e-13     # first moment = u
            if m == "bicubic":
                assert abs((h * offs ** 2).sum() - float(u) ** 2) < 1e-12


def test_printed_kernels():
    with open(os.path.join(GOLD, "printed_kernels_3_2.json")) as f:
        gold = json.load(f)
    p, q = gold["p"], gold["q"]
    for method in ("nearest", "bilinear"):
        for name, (jh, jw) in gold["phases"].items():
            hh = oracle.phase_kernel(p, q, method, gold["grid"], jh)
            hw = oracle.phase_kernel(p, q, method, gold["grid"], jw)
            K = (len(hh) - 1) // 2
            bh = floor(exact.coord(jh, p, q, gold["grid"]))
            bw = floor(exact.coord(jw, p, q, gold["grid"]))
            win = np.array([[hh[K - (bh + a)] * hw[K - (bw + b)] for b in range(2)] for a in range(2)])
            np.testing.assert_array_equal(np.round(win, gold["decimals"]), np.array(gold[method][name]),
                                          err_msg=f"{method} {name}")


def test_printed_kernels_not_matched_by_half_grid():
    # documents the grid reading: the default half-pixel grid does not give the
    # printed 3/2 bilinear kernel (the paper grid does, see test_printed_kernels)
    hh = oracle.phase_kernel(3, 2, "bilinear", "half", 0)
    K = (len(hh) - 1) // 2
    b = floor(exact.coord(0, 3, 2, "half"))
    win = np.array([[hh[K - (b + a)] * hh[K - (b + c)] for c in range(2)] for a in range(2)])
    assert not np.allclose(np.round(win, 2), [[0.44, 0.22], [0.22, 0.11]])


# ---------------------------------------------------------------- library pins

@pytest.mark.parametrize("p,q", [(3, 2), (2, 3), (5, 4), (4, 5), (7, 3), (2, 11), (27, 11)])
def test_bilinear_replicate_matches_torch_interpolate(p, q):
    x = synth.uniform(5, (2, 3, 22, 17)).astype(np.float64)
    y = oracle.forward(x, p, q, "bilinear", "replicate")
    t = F.interpolate(torch.from_numpy(x), scale_factor=p / q, mode="bilinear",
                      align_corners=False).numpy()
    h, w = t.shape[2:]
    np.testing.assert_allclose(y[:, :, :h, :w], t, rtol=0, atol=1e-9)


@pytest.mark.parametrize("p,q", [(3, 2), (2, 3), (5, 4), (4, 5), (7, 3), (3, 7), (2, 11), (27, 11)])
def test_nearest_matches_torch_nearest_exact(p, q):
    x = synth.uniform(6, (1, 2, 26, 19)).astype(np.float64)
    y = oracle.forward(x, p, q, "nearest", "replicate")
    t = F.interpolate(torch.from_numpy(x), scale_factor=p / q, mode="nearest-exact").numpy()
    h, w = t.shape[2:]
    # compare off exact ties, where float index math may round either way
    def off_tie(n):
        return [k for k in range(n) if (2 * k + 1) * q % (2 * p) != 0]
    kh, kw = off_tie(h), off_tie(w)
    np.testing.assert_array_equal(y[:, :, kh][:, :, :, kw], t[:, :, kh][:, :, :, kw])


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_integer_upscale_is_pixelshuffle(p):
    x = synth.uniform(8, (2, 3, 6, 5)).astype(np.float64)
    y = oracle.forward(x, p, 1, "nearest", "zero")
    xt = torch.from_numpy(x)
    ref = F.pixel_shuffle(xt.repeat_interleave(p * p, dim=1), p).numpy()
    np.testing.assert_array_equal(y, ref)
    np.testing.assert_array_equal(y[0, 0], np.kron(x[0, 0], np.ones((p, p))))


def _anchor(j, p, q):
    return floor(exact.coord(j, p, q, "half"))


def _union_weights(w4, p, q, mix):
    """Embed per-phase 4x4 windows into one conv2d (correlation) kernel of
    size q+4 whose window starts 2 samples before q*m."""
    KS = q + 4
    if mix:
        _, _, co, ci, _, _ = w4.shape
        U = np.zeros((co * p * p, ci, KS, KS))
        for jh in range(p):
            for jw in range(p):
                ah, aw = _anchor(jh, p, q) - 1 + 2, _anchor(jw, p, q) - 1 + 2
                for o in range(co):
                    U[o * p * p + jh * p + jw, :, ah:ah + 4, aw:aw + 4] = w4[jh, jw, o]
        return U
    C = w4.shape[0]
    U = np.zeros((C * p * p, 1, KS, KS))
    for c in range(C):
        for jh in range(p):
            for jw in range(p):
                ah, aw = _anchor(jh, p, q) - 1 + 2, _anchor(jw, p, q) - 1 + 2
                U[c * p * p + jh * p + jw, 0, ah:ah + 4, aw:aw + 4] = w4[c, jh, jw]
    return U


@pytest.mark.parametrize("p,q", [(3, 4), (3, 2), (5, 4), (2, 3)])
@pytest.mark.parametrize("pad,mode", [("zero", "constant"), ("replicate", "replicate"), ("reflect", "reflect")])
def test_learned_layers_match_torch_conv2d(p, q, pad, mode):
    x = synth.normal(9, (2, 3, 11, 13)).astype(np.float64)
    H, W = x.shape[2:]
    Mh, Mw = -(-H // q), -(-W // q)
    xt = F.pad(torch.from_numpy(x), (2, q * Mw + 2 - W, 2, q * Mh + 2 - H), mode=mode)
    w_dw = synth.normal(10, (3, p, p, 4, 4)).astype(np.float64)
    y = oracle.forward(x, p, q, "dw4", pad, weight=w_dw)
    ref = F.pixel_shuffle(F.conv2d(xt, torch.from_numpy(_union_weights(w_dw, p, q, False)),
                                   stride=q, groups=3), p).numpy()
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-12)
    w_mx = synth.normal(11, (p, p, 4, 3, 4, 4)).astype(np.float64)
    y = oracle.forward(x, p, q, "mix4", pad, weight=w_mx)
    ref = F.pixel_shuffle(F.conv2d(xt, torch.from_numpy(_union_weights(w_mx, p, q, True)),
                                   stride=q), p).numpy()
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-12)


def bicubic_taps(p, q):
    """4 Keys taps per phase, from the exact module (anchor floor(u) - 1)."""
    out = []
    for j in range(p):
        u = exact.coord(j, p, q, "half")
        b = floor(u)
        out.append([float(exact.keys_cubic(u - (b - 1 + a))) for a in range(4)])
    return np.array(out)


@pytest.mark.parametrize("p,q", [(3, 4), (5, 4), (2, 3), (3, 2)])
def test_learned_layers_reduce_to_bicubic(p, q):
    x = synth.normal(12, (2, 3, 10, 9)).astype(np.float64)
    t = bicubic_taps(p, q)
    w_dw = np.einsum("ia,jb->ijab", t, t)[None].repeat(3, axis=0)
    ref = oracle.forward(x, p, q, "bicubic", "reflect")
    np.testing.assert_allclose(oracle.forward(x, p, q, "dw4", "reflect", weight=w_dw), ref, atol=1e-13)
    w_mx = np.zeros((p, p, 3, 3, 4, 4))
    for o in range(3):
        w_mx[:, :, o, o] = np.einsum("ia,jb->ijab", t, t)
    np.testing.assert_allclose(oracle.forward(x, p, q, "mix4", "reflect", weight=w_mx), ref, atol=1e-13)


# ---------------------------------------------------------------- adjoint

ADJ_CASES = [(3, 2), (2, 3), (5, 4), (4, 5), (3, 4), (2, 11), (27, 11), (1, 1), (4, 1)]


@pytest.mark.parametrize("p,q", ADJ_CASES)
@pytest.mark.parametrize("method", METHODS + ["dw4", "mix4"])
@pytest.mark.parametrize("pad", PADS)
def test_adjoint_dot_product(p, q, method, pad):
    from math import gcd
    g = gcd(p, q)
    pr = p // g
    shape = (2, 3, 9, 7) if q < 10 else (1, 2, 13, 12)
    x = synth.normal(20, shape).astype(np.float64)
    w = None
    if method == "dw4":
        w = synth.normal(21, (shape[1], pr, pr, 4, 4)).astype(np.float64)
    if method == "mix4":
        w = synth.normal(22, (pr, pr, 2, shape[1], 4, 4)).astype(np.float64)
    y = oracle.forward(x, p, q, method, pad, weight=w)
    gy = synth.normal(23, y.shape).astype(np.float64)
    dx, dw = oracle.backward(gy, x.shape, p, q, method, pad, x=x, weight=w,
                             need_dw=method in ("dw4", "mix4"))
    lhs, rhs = float((y * gy).sum()), float((x * dx).sum())
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs), np.abs(y * gy).sum())
    if dw is not None:
        # y is linear in the weights: <y(W), g> = sum W * dW
        r2 = float((w * dw).sum())
        assert abs(lhs - r2) <= 1e-12 * max(1.0, abs(lhs), np.abs(y * gy).sum())


@pytest.mark.parametrize("method", ["bicubic", "dw4"])
def test_finite_differences(method):
    p, q = 3, 4
    x = synth.normal(30, (1, 2, 8, 9)).astype(np.float64)
    w = synth.normal(31, (2, 3, 3, 4, 4)).astype(np.float64) if method == "dw4" else None
    gy = synth.normal(32, oracle.forward(x, p, q, method, "replicate", weight=w).shape)
    f = lambda xx, ww: float((oracle.forward(xx, p, q, method, "replicate", weight=ww) * gy).sum())
    dx, dw = oracle.backward(gy, x.shape, p, q, method, "replicate", x=x, weight=w,
                             need_dw=w is not None)
    rng = np.random.default_rng(33)
    h = 1e-3
    for _ in range(3):
        v = rng.standard_normal(x.shape)
        fd = (f(x + h * v, w) - f(x - h * v, w)) / (2 * h)
        assert abs(fd - (dx * v).sum()) < 1e-8 * max(1, abs(fd))
        if w is not None:
            v = rng.standard_normal(w.shape)
            fd = (f(x, w + h * v) - f(x, w - h * v)) / (2 * h)
            assert abs(fd - (dw * v).sum()) < 1e-8 * max(1, abs(fd))


def test_backward_brute_force_tiny():
    # dX from the definition: dX[i] = sum_k dy[k] * d y[k] / d x[i], with the
    # Jacobian columns probed one input sample at a time through the direct sampler
    p, q = 3, 2
    for method in METHODS:
        for pad in PADS:
            x0 = np.zeros((3, 4))
            gy = synth.normal(40, (1, 1, 6, 6)).astype(np.float64)
            dx, _ = oracle.backward(gy, (1, 1, 3, 4), p, q, method, pad)
            for i in range(3):
                for j in range(4):
                    e = x0.copy()
                    e[i, j] = 1.0
                    col = _frac_array(exact.resample2d(e, p, q, method, pad))
                    assert abs((col * gy[0, 0]).sum() - dx[0, 0, i, j]) < 1e-12
