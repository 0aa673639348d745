"""FP64 oracle for N-dimensional FCFS — TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
call this; the GPU library never imports it.

It follows the paper's ND construction (Sec. 4.2) for fixed interpolation
methods, axis by axis with its own factor r_i / s_i:
 1. the input is extended beyond every end of every spatial axis (the
    virtual padding of the 2D oracle: zero / replicate / reflect);
 2. a strided convolution with stride s_i on axis i and prod_i r_i output
    channels per input channel, one per phase tuple (j_1, ..., j_n), whose
    kernel is the outer product of the 1D phase kernels (each of length
    2K_i + 1, K_i = s_i + 2, convolution orientation: entry K + k multiplies
    the sample at offset -k from s_i * m);
 3. the ND pixelshuffle (Sec. 4.1): output index r_i * m_i + j_i on every
    axis takes hidden channel (j_1, ..., j_n) at cell (m_1, ..., m_n). The
    channel order (first axis's phase most significant) is internal.

The 1D phase kernels come from the 2D oracle (``oracle.phase_kernel``, pinned
against the paper's printed kernels and the exact sampler). Everything here
is numpy in FP64, for small inputs.

Pins (tests/test_oracle_nd.py): two axes reproduce the 2D pipeline oracle;
one and three axes reproduce the exact-rational sampler; r_i / 1 nearest is
np.repeat along every axis.
"""
from __future__ import annotations

import itertools
from math import gcd

import numpy as np

from . import exact, phase_kernel


def _reduce(p: int, q: int):
    g = gcd(p, q)
    return p // g, q // g


def forward_nd(x, factors, method: str = "bilinear", pad: str = "replicate", grid: str = "half",
               abs_weights: bool = False) -> np.ndarray:
    """FCFS of ``x`` [N, C, S_1, ..., S_n] with per-axis factors
    ``factors`` = [(r_1, s_1), ..., (r_n, s_n)], in FP64.

    ``abs_weights``: use |h| for every tap (with |x| as input this gives the
    per-output scale of a rounding error, as ``oracle.condition`` does)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.ndim - 2
    if n < 1 or len(factors) != n:
        raise ValueError("one (r, s) factor per spatial axis")
    if method not in ("nearest", "bilinear", "bicubic"):
        raise ValueError("fixed interpolation methods only")
    fac = [_reduce(int(r), int(s)) for r, s in factors]
    sizes = x.shape[2:]
    K = [s + 2 for _, s in fac]
    M = [-(-sizes[i] // fac[i][1]) for i in range(n)]
    # 1. the extended input over positions -K_i .. s_i (M_i - 1) + K_i
    idx = []
    for i in range(n):
        pos = np.arange(-K[i], fac[i][1] * (M[i] - 1) + K[i] + 1)
        src = np.array([exact.ext_index(int(e), sizes[i], pad) for e in pos], dtype=object)
        idx.append(src)
    xp = x
    for i in range(n):
        src = idx[i]
        keep = np.array([s is not None for s in src])
        take = np.array([s if s is not None else 0 for s in src], dtype=np.int64)
        xp = np.take(xp, take, axis=2 + i)
        shape = [1] * xp.ndim
        shape[2 + i] = len(take)
        xp = xp * keep.reshape(shape)
    # 2. per phase tuple: strided correlation with the separable kernel
    kern = [[phase_kernel(fac[i][0], fac[i][1], method, grid, j) for j in range(fac[i][0])] for i in range(n)]
    if abs_weights:
        kern = [[np.abs(k) for k in ax] for ax in kern]
    N, C = x.shape[:2]
    out_shape = (N, C) + tuple(fac[i][0] * M[i] for i in range(n))
    y = np.zeros(out_shape, dtype=np.float64)
    for phase in itertools.product(*[range(fac[i][0]) for i in range(n)]):
        hid = np.zeros((N, C) + tuple(M), dtype=np.float64)
        for off in itertools.product(*[range(-K[i], K[i] + 1) for i in range(n)]):
            w = 1.0
            for i in range(n):
                w *= kern[i][phase[i]][K[i] + off[i]]
            if w == 0.0:
                continue
            # sample at s_i m_i - off_i, i.e. padded index s_i m_i - off_i + K_i
            sl = [slice(None), slice(None)]
            for i in range(n):
                start = K[i] - off[i]
                sl.append(slice(start, start + fac[i][1] * (M[i] - 1) + 1, fac[i][1]))
            hid += w * xp[tuple(sl)]
        # 3. pixelshuffle: output r_i m_i + j_i
        osl = [slice(None), slice(None)] + [slice(phase[i], None, fac[i][0]) for i in range(n)]
        y[tuple(osl)] = hid
    return y


def exact_nd(x, factors, method: str, pad: str, grid: str = "half") -> np.ndarray:
    """The exact-rational direct sampler in n dimensions (tensor product of
    the per-axis interpolants of ``oracle.exact``), for tiny inputs."""
    from fractions import Fraction
    x = np.asarray(x, dtype=np.float64)
    n = x.ndim - 2
    fac = [_reduce(int(r), int(s)) for r, s in factors]
    sizes = x.shape[2:]
    outs = [exact.out_len(fac[i][0], fac[i][1], sizes[i]) for i in range(n)]
    wts = [[exact.axis_weights(k, fac[i][0], fac[i][1], method, grid) for k in range(outs[i])] for i in range(n)]
    N, C = x.shape[:2]
    y = np.zeros((N, C) + tuple(outs), dtype=np.float64)
    for b in range(N):
        for c in range(C):
            plane = x[b, c]
            for ko in itertools.product(*[range(o) for o in outs]):
                acc = Fraction(0)
                for taps in itertools.product(*[wts[i][ko[i]] for i in range(n)]):
                    w = Fraction(1)
                    src = []
                    for i, (ii, wi) in enumerate(taps):
                        s = exact.ext_index(ii, sizes[i], pad)
                        if s is None or wi == 0:
                            w = Fraction(0)
                            break
                        w *= wi
                        src.append(s)
                    if w != 0:
                        acc += w * Fraction(float(plane[tuple(src)]))
                y[(b, c) + ko] = float(acc)
    return y
