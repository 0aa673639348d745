"""FP64 CPU oracle for fully convolutional fractional scaling (FCFS).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers. The GPU library never imports, links or
calls anything here, and nothing here imports the GPU package.

The arithmetic lives in ``fcfs_oracle.c`` (the paper's pad -> strided
convolution -> pixelshuffle pipeline, Sec. 3.1 and Sec. 4.2, in FP64); this
module compiles it with gcc on first use and wraps it for numpy arrays. The
independent direct sampler that pins it lives in ``oracle.exact``.

Parity unpinned: none of the functions here is unpinned; every one has CPU
tests against closed forms, exact-rational sampling, library routines or the
paper's printed kernels. The conditioning scales ``condition`` and
``condition_backward`` are pinned to per-tap sums of |w| |x| (and |w| |dy|,
|dy| |x| for the gradients) taken in exact rationals over the direct
sampler's tap lists and the learned layers' 4x4 windows, and to forward(|x|)
where every weight is non-negative.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fcfs_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_SO = os.path.join(_BUILD, "libfcfs_oracle.so")

METHODS = {"nearest": 0, "bilinear": 1, "bicubic": 2, "dw4": 3, "mix4": 4}
PADS = {"zero": 0, "replicate": 1, "reflect": 2}
GRIDS = {"half": 0, "paper": 1, "asym": 2}

_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle library with gcc (FP64, OpenMP). Returns its path."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
               "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(build())
            L, I, P = ctypes.c_long, ctypes.c_int, ctypes.c_void_p
            lib.fcfs_oracle_out_len.argtypes = [L, L, L]
            lib.fcfs_oracle_out_len.restype = L
            lib.fcfs_oracle_phase_kernel.argtypes = [L, L, I, I, L, P]
            lib.fcfs_oracle_phase_kernel.restype = L
            lib.fcfs_oracle_forward.argtypes = [L, L, L, L, I, I, I, L, L, L, L, P, P, L, P]
            lib.fcfs_oracle_forward.restype = I
            lib.fcfs_oracle_forward_absw.argtypes = lib.fcfs_oracle_forward.argtypes
            lib.fcfs_oracle_forward_absw.restype = I
            lib.fcfs_oracle_backward.argtypes = [L, L, L, L, I, I, I, L, L, L, L, P, P, L, P, P, P]
            lib.fcfs_oracle_backward.restype = I
            lib.fcfs_oracle_backward_absw.argtypes = lib.fcfs_oracle_backward.argtypes
            lib.fcfs_oracle_backward_absw.restype = I
            lib.fcfs_oracle_set_threads.argtypes = [I]
            lib.fcfs_oracle_set_threads.restype = None
            lib.fcfs_oracle_threads.argtypes = []
            lib.fcfs_oracle_threads.restype = I
            _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _axes(p, q, pw, qw):
    return p, q, (p if pw is None else pw), (q if qw is None else qw)


def out_len(p: int, q: int, n: int) -> int:
    """Output length of one axis: p * ceil(n / q) after reducing p/q."""
    v = _load().fcfs_oracle_out_len(p, q, n)
    if v < 0:
        raise ValueError("bad arguments")
    return int(v)


def phase_kernel(p: int, q: int, method: str, grid: str, j: int) -> np.ndarray:
    """Dense 1D kernel of channel j (length 2K+1). Entry K + k multiplies the
    input sample at offset -k from q*m (convolution orientation)."""
    import math
    g = math.gcd(p, q)
    K = q // g + 2
    h = np.zeros(2 * K + 1, dtype=np.float64)
    _load().fcfs_oracle_phase_kernel(p, q, METHODS[method], GRIDS[grid], j, _ptr(h))
    return h


def forward(x, p, q, method="bilinear", pad="replicate", grid="half", weight=None,
            cout=None, pw=None, qw=None, abs_weights=False) -> np.ndarray:
    """FCFS forward of an NCHW array in FP64.

    ``p/q`` scales both axes unless ``pw/qw`` gives the width factor.
    ``weight``: dw4 [C, ph, pw, 4, 4]; mix4 [ph, pw, Cout, Cin, 4, 4].
    ``abs_weights``: use |w| for every tap (see ``condition``).
    """
    x = _f64(x)
    if x.ndim != 4:
        raise ValueError("x must be NCHW")
    N, C, H, W = x.shape
    ph, qh, pw_, qw_ = _axes(p, q, pw, qw)
    m = METHODS[method]
    co = C if m != METHODS["mix4"] else (cout if cout is not None else np.asarray(weight).shape[2])
    Ho, Wo = out_len(ph, qh, H), out_len(pw_, qw_, W)
    y = np.empty((N, co, Ho, Wo), dtype=np.float64)
    w = _f64(weight)
    fn = _load().fcfs_oracle_forward_absw if abs_weights else _load().fcfs_oracle_forward
    rc = fn(ph, qh, pw_, qw_, m, PADS[pad], GRIDS[grid], N, C, H, W, _ptr(x), _ptr(w), co, _ptr(y))
    if rc != 0:
        raise ValueError("oracle forward rejected its arguments")
    return y


def condition(x, p, q, method="bilinear", pad="replicate", grid="half", weight=None,
              cout=None, pw=None, qw=None) -> np.ndarray:
    """Per-output scale S = sum over taps of |w| * |x| (same shape as the
    output), the size a rounding error of each output's dot product is
    measured against."""
    return forward(np.abs(np.asarray(x, dtype=np.float64)), p, q, method, pad, grid, weight,
                   cout, pw, qw, abs_weights=True)


def backward(dy, x_shape, p, q, method="bilinear", pad="replicate", grid="half", x=None,
             weight=None, need_dx=True, need_dw=False, pw=None, qw=None, abs_weights=False):
    """Adjoint of ``forward``: returns (dx or None, dw or None) in FP64.
    ``abs_weights``: use |w| for every tap (see ``condition_backward``)."""
    dy = _f64(dy)
    N, C, H, W = x_shape
    ph, qh, pw_, qw_ = _axes(p, q, pw, qw)
    m = METHODS[method]
    co = dy.shape[1]
    dx = np.empty((N, C, H, W), dtype=np.float64) if need_dx else None
    w = _f64(weight)
    dw = np.empty_like(w) if need_dw else None
    xx = _f64(x)
    fn = _load().fcfs_oracle_backward_absw if abs_weights else _load().fcfs_oracle_backward
    rc = fn(ph, qh, pw_, qw_, m, PADS[pad], GRIDS[grid], N, C, H, W,
            _ptr(xx), _ptr(w), co, _ptr(dy), _ptr(dx), _ptr(dw))
    if rc != 0:
        raise ValueError("oracle backward rejected its arguments")
    return dx, dw


def condition_backward(dy, x_shape, p, q, method="bilinear", pad="replicate", grid="half", x=None,
                       weight=None, need_dw=False, pw=None, qw=None):
    """Per-element scales of the gradients' rounding errors: the input
    gradient's sum over taps of |w| |dy|, and the weight gradient's sum of
    |dy| |x| (returned as (S_dx, S_dw))."""
    ady = np.abs(np.asarray(dy, dtype=np.float64))
    ax = None if x is None else np.abs(np.asarray(x, dtype=np.float64))
    return backward(ady, x_shape, p, q, method, pad, grid, ax, weight, True, need_dw, pw, qw,
                    abs_weights=True)


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().fcfs_oracle_threads())


def set_threads(n: int) -> None:
    """Use n OpenMP threads in later calls (timing on one core and on all)."""
    _load().fcfs_oracle_set_threads(int(n))
