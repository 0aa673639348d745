"""Direct exact-rational sampler for FCFS — TEST INFRASTRUCTURE ONLY.

This is the second, independent definition the FP64 pipeline oracle is pinned
against. It uses no phase decomposition, no dense kernels, no padding buffer
and no pixelshuffle: every output index k is mapped straight to its input
coordinate u_k, and the textbook interpolant is evaluated there with Python
``fractions`` (so results are exact rationals, given exact inputs).

 * coordinate of output k on one axis (reduced p/q): numerator over 2p,
       half  grid: u_k = ((2k+1) q - p) / (2p)
       paper grid: u_k = (2k+1) q / (2p)
       asym  grid: u_k = 2 k q / (2p)
 * nearest : the sample at floor(u + 1/2)
 * bilinear: (1 - t) x[i] + t x[i+1], i = floor(u), t = u - i
 * bicubic : sum over i = floor(u)-1 .. floor(u)+2 of W(u - i) x[i], with W
             the cubic of the paper's Sec. 5.2.3 (Keys, a = -1/2)
 * the input is extended beyond its ends by zero / replicate / reflect.
Two-dimensional results are the tensor product of the two axes.
Only for tiny inputs (pure Python loops).
"""
from __future__ import annotations

from fractions import Fraction
from math import ceil, floor, gcd


def ext_index(i: int, n: int, pad: str):
    """Source index of position i (any integer) of an axis of length n, or
    None for a zero-padded position."""
    if 0 <= i < n:
        return i
    if pad == "zero":
        return None
    if pad == "replicate":
        return 0 if i < 0 else n - 1
    if pad == "reflect":
        # bounce between the two end samples until inside (edge not repeated)
        if n == 1:
            return 0
        while i < 0 or i >= n:
            if i < 0:
                i = -i
            if i >= n:
                i = 2 * (n - 1) - i
        return i
    raise ValueError(pad)


def coord(k: int, p: int, q: int, grid: str) -> Fraction:
    if grid == "half":
        return Fraction((2 * k + 1) * q - p, 2 * p)
    if grid == "paper":
        return Fraction((2 * k + 1) * q, 2 * p)
    if grid == "asym":
        return Fraction(k * q, p)
    raise ValueError(grid)


def keys_cubic(d: Fraction) -> Fraction:
    """W(d) of Sec. 5.2.3 with a = -1/2."""
    a = abs(d)
    if a <= 1:
        return Fraction(3, 2) * a ** 3 - Fraction(5, 2) * a ** 2 + 1
    if a < 2:
        return Fraction(-1, 2) * a ** 3 + Fraction(5, 2) * a ** 2 - 4 * a + 2
    return Fraction(0)


def axis_weights(k: int, p: int, q: int, method: str, grid: str):
    """[(input index, weight)] of output k along one axis."""
    u = coord(k, p, q, grid)
    i0 = floor(u)
    if method == "nearest":
        return [(floor(u + Fraction(1, 2)), Fraction(1))]
    if method == "bilinear":
        t = u - i0
        return [(i0, 1 - t), (i0 + 1, t)]
    if method == "bicubic":
        return [(i, keys_cubic(u - i)) for i in range(i0 - 1, i0 + 3)]
    raise ValueError(method)


def out_len(p: int, q: int, n: int) -> int:
    g = gcd(p, q)
    p, q = p // g, q // g
    return p * ceil(n / q)


def resample2d(x, p: int, q: int, method: str, pad: str, grid: str = "half",
               pw: int | None = None, qw: int | None = None):
    """Exact resampling of one 2D plane ``x`` (list of rows, or 2D array of
    floats; converted exactly). Returns a list of rows of Fractions."""
    pw = p if pw is None else pw
    qw = q if qw is None else qw
    gh, gw = gcd(p, q), gcd(pw, qw)
    ph, qh, pw, qw = p // gh, q // gh, pw // gw, qw // gw
    rows = [[Fraction(float(v)) for v in r] for r in x]
    H, W = len(rows), len(rows[0])
    Ho, Wo = out_len(ph, qh, H), out_len(pw, qw, W)
    wh = [axis_weights(k, ph, qh, method, grid) for k in range(Ho)]
    ww = [axis_weights(k, pw, qw, method, grid) for k in range(Wo)]
    out = []
    for kh in range(Ho):
        orow = []
        for kw in range(Wo):
            acc = Fraction(0)
            for ih, ah in wh[kh]:
                sh = ext_index(ih, H, pad)
                if sh is None or ah == 0:
                    continue
                for iw, aw in ww[kw]:
                    sw = ext_index(iw, W, pad)
                    if sw is None or aw == 0:
                        continue
                    acc += ah * aw * rows[sh][sw]
            orow.append(acc)
        out.append(orow)
    return out
