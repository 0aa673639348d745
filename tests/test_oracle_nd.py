"""Pins of the ND oracle (oracle.nd): two axes reproduce the 2D pipeline
oracle, one and three axes the exact-rational direct sampler, and r/1
nearest upscaling is np.repeat on every axis (the ND pixelshuffle order)."""
import numpy as np
import pytest

import oracle
from oracle import nd

METHODS = ["nearest", "bilinear", "bicubic"]
PADS = ["zero", "replicate", "reflect"]


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("pad", PADS)
def test_two_axes_match_2d_oracle(method, pad):
    rng = np.random.default_rng(11)
    x = rng.standard_normal((2, 2, 9, 11))
    for (ph, qh, pw, qw) in [(3, 2, 3, 2), (2, 3, 5, 4), (4, 5, 1, 1), (7, 3, 2, 5)]:
        y = nd.forward_nd(x, [(ph, qh), (pw, qw)], method, pad)
        r = oracle.forward(x, ph, qh, method, pad, pw=pw, qw=qw)
        np.testing.assert_allclose(y, r, rtol=0, atol=1e-12)


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("pad", PADS)
def test_one_axis_matches_exact_sampler(method, pad):
    rng = np.random.default_rng(12)
    x = rng.standard_normal((1, 2, 13))
    for (p, q) in [(3, 2), (2, 3), (5, 4), (4, 5), (27, 11), (2, 11)]:
        y = nd.forward_nd(x, [(p, q)], method, pad)
        r = nd.exact_nd(x, [(p, q)], method, pad)
        np.testing.assert_allclose(y, r, rtol=0, atol=1e-12)


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("pad", ["zero", "reflect"])
def test_three_axes_match_exact_sampler(method, pad):
    rng = np.random.default_rng(13)
    x = rng.standard_normal((1, 1, 4, 5, 3))
    for fac in ([(3, 2), (2, 3), (5, 4)], [(1, 1), (4, 3), (2, 5)]):
        y = nd.forward_nd(x, fac, method, pad)
        r = nd.exact_nd(x, fac, method, pad)
        np.testing.assert_allclose(y, r, rtol=0, atol=1e-12)


def test_integer_nearest_is_repeat():
    rng = np.random.default_rng(14)
    x = rng.standard_normal((2, 3, 3, 4, 5))
    y = nd.forward_nd(x, [(2, 1), (3, 1), (1, 1)], "nearest", "zero")
    r = np.repeat(np.repeat(x, 2, axis=2), 3, axis=3)
    np.testing.assert_array_equal(y, r)


def test_abs_weights_bound_the_error_scale():
    # |forward(x)| <= forward(|x|, |h|) elementwise (triangle inequality)
    rng = np.random.default_rng(15)
    x = rng.standard_normal((1, 2, 5, 6, 4))
    fac = [(3, 2), (5, 4), (2, 3)]
    y = nd.forward_nd(x, fac, "bicubic", "reflect")
    s = nd.forward_nd(np.abs(x), fac, "bicubic", "reflect", abs_weights=True)
    assert np.all(np.abs(y) <= s + 1e-12)
