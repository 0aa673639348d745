"""Runs forward cases through the host-emulated libfcfs (CPU, sanitizers on)
and compares them with the FP64 oracle. Invoked by the test in a subprocess
with the address-sanitizer runtime preloaded. Prints one line per case and
exits non-zero on the first mismatch."""
import ctypes
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
import synth  # noqa: E402

METHODS = {"nearest": 0, "bilinear": 1, "bicubic": 2, "dw4": 3, "mix4": 4}
PADS = {"zero": 0, "replicate": 1, "reflect": 2}
GRIDS = {"half": 0, "paper": 1, "asym": 2}
DT = {"f32": 0, "bf16": 1, "f16": 2}
UNIT = {"f32": 2.0 ** -24, "bf16": 2.0 ** -8, "f16": 2.0 ** -11}
UNIT_ABS = {"f32": 2.0 ** -150, "bf16": 2.0 ** -134, "f16": 2.0 ** -25}


def to_storage(x, dt):
    if dt == "f32":
        return np.ascontiguousarray(x, np.float32), np.ascontiguousarray(x, np.float32)
    if dt == "f16":
        h = np.ascontiguousarray(x, np.float32).astype(np.float16)
        return h, h.astype(np.float32)
    r = synth.bf16_round(x)
    bits = (r.view(np.uint32) >> 16).astype(np.uint16)
    return bits, r


def from_storage(y, dt):
    if dt == "bf16":
        return (y.astype(np.uint32) << 16).view(np.float32)
    return y.astype(np.float32)


def run_backward(lib, plan, c, i, xs, xv, w, N, C, H, W, Ho, Wo, p, q, pw, qw, m, pad, grid, dt, wptr=None, Co=None):
    Co = C if Co is None else Co
    dyv = synth.normal(3000 + i, (N, Co, Ho, Wo))
    dys, dyv = to_storage(dyv, dt)
    need_dw = m in ("dw4", "mix4")
    parts = c.get("parts", "both")   # "dx" / "dw": one gradient only
    need_dx = parts != "dw"
    need_dw = need_dw and parts != "dx"
    ws = ctypes.c_size_t()
    assert lib.fcfs_backward_workspace(plan, DT[dt], N, C, H, W, Co, ctypes.byref(ws)) == 0
    wsb = np.zeros(max(1, ws.value) // 4 + 64, dtype=np.int32)
    dx = np.zeros((N, C, H, W), dtype=xs.dtype)
    dw = np.zeros(w.shape, dtype=np.float32) if need_dw else None
    if wptr is None and w is not None:
        wptr = w.ctypes.data
    st = lib.fcfs_backward(plan, DT[dt], N, C, H, W, xs.ctypes.data, wptr, Co,
                           dys.ctypes.data, dx.ctypes.data if need_dx else None, None if dw is None else dw.ctypes.data,
                           wsb.ctypes.data, ws.value, None)
    assert st == 0, st
    rdx, rdw = oracle.backward(dyv.astype(np.float64), (N, C, H, W), p, q, m, pad, grid, x=xv, weight=w,
                               need_dw=need_dw, pw=pw, qw=qw)
    sdx, sdw = oracle.condition_backward(dyv, (N, C, H, W), p, q, m, pad, grid, x=xv, weight=w,
                                         need_dw=need_dw, pw=pw, qw=qw)
    gdx = from_storage(dx, dt).astype(np.float64)
    if not need_dx:
        gdx = rdx   # (dx left unwritten: checked to stay zero below)
        assert not dx.any()
    ok = bool((np.abs(gdx - rdx) <= UNIT[dt] * np.abs(rdx) + UNIT_ABS[dt] + 1e-5 * sdx + 1e-30).all())
    if not ok:
        bad = np.argwhere(np.abs(gdx - rdx) > UNIT[dt] * np.abs(rdx) + UNIT_ABS[dt] + 1e-5 * sdx + 1e-30)
        print("dx first bad", bad[:5].tolist(), gdx[tuple(bad[0])], rdx[tuple(bad[0])], flush=True)
    if need_dw:
        okw = bool((np.abs(dw - rdw) <= 1e-5 * sdw + 1e-30).all())
        if not okw:
            bad = np.argwhere(np.abs(dw - rdw) > 1e-5 * sdw + 1e-30)
            print("dw first bad", bad[:5].tolist(), dw[tuple(bad[0])], rdw[tuple(bad[0])], flush=True)
        ok = ok and okw
    return ok


def main():
    lib = ctypes.CDLL(sys.argv[1])
    cases = json.loads(sys.argv[2])
    P = ctypes.c_void_p
    lib.fcfs_plan_ex.argtypes = [ctypes.c_int] * 7 + [ctypes.POINTER(P)]
    lib.fcfs_forward.argtypes = [P, ctypes.c_int] + [ctypes.c_int64] * 4 + [P, P, ctypes.c_int64, P, P]
    lib.fcfs_output_size.argtypes = [P, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int64)]
    lib.fcfs_forward_config.argtypes = [P, ctypes.c_int] + [ctypes.c_int64] * 4 + [P, P, P, P]
    lib.fcfs_backward_workspace.argtypes = [P, ctypes.c_int] + [ctypes.c_int64] * 5 + [ctypes.POINTER(ctypes.c_size_t)]
    lib.fcfs_backward.argtypes = [P, ctypes.c_int] + [ctypes.c_int64] * 4 + [P, P, ctypes.c_int64, P, P, P, P,
                                                                             ctypes.c_size_t, P]
    for i, c in enumerate(cases):
        p, q, pw, qw = c["p"], c["q"], c.get("pw", c["p"]), c.get("qw", c["q"])
        N, C, H, W = c["shape"]
        m, pad, grid, dt = c["method"], c["pad"], c.get("grid", "half"), c.get("dtype", "f32")
        plan = P()
        assert lib.fcfs_plan_ex(p, q, pw, qw, METHODS[m], PADS[pad], GRIDS[grid], ctypes.byref(plan)) == 0
        ho, wo = ctypes.c_int64(), ctypes.c_int64()
        lib.fcfs_output_size(plan, H, W, ctypes.byref(ho), ctypes.byref(wo))
        x = synth.normal(1000 + i, (N, C, H, W))
        xs, xv = to_storage(x, dt)
        w = None
        wptr = None
        Co = C
        from math import gcd
        if m == "dw4":
            w = synth.normal(2000 + i, (C, p // gcd(p, q), pw // gcd(pw, qw), 4, 4)).astype(np.float32)
            wptr = w.ctypes.data
        if m == "mix4":
            Co = c.get("cout", C)
            wraw = synth.normal(2000 + i, (p // gcd(p, q), pw // gcd(pw, qw), Co, C, 4, 4), std=1 / 32)
            wbits, w = to_storage(wraw, dt)
            wbits = np.ascontiguousarray(wbits)
            wptr = wbits.ctypes.data
        if c.get("mode") == "bwd":
            ok = run_backward(lib, plan, c, i, xs, xv, w, N, C, H, W, ho.value, wo.value, p, q, pw, qw, m, pad,
                              grid, dt, wptr=wptr, Co=Co)
            print("case", i, json.dumps(c), "ok" if ok else "MISMATCH", flush=True)
            if not ok:
                sys.exit(1)
            continue
        if c.get("expect_paired") is not None:
            kid = ctypes.c_int()
            assert lib.fcfs_forward_config(plan, DT[dt], N, C, H, W, ctypes.byref(kid), None, None, None) == 0
            # (the configuration query takes tensors to be aligned)
            assert (kid.value >= 50000) == c["expect_paired"], kid.value
        if c.get("misalign"):
            # output one element past a 4-byte boundary: the unpaired instance
            ybuf = np.zeros(N * Co * ho.value * wo.value + 1, dtype=xs.dtype)
            y = ybuf[1:].reshape(N, Co, ho.value, wo.value)
        else:
            y = np.zeros((N, Co, ho.value, wo.value), dtype=xs.dtype)
        st = lib.fcfs_forward(plan, DT[dt], N, C, H, W, xs.ctypes.data, wptr, Co, y.ctypes.data, None)
        if c.get("expect_status") is not None:
            ok = st == c["expect_status"]
            print("case", i, json.dumps(c), "ok" if ok else "MISMATCH status %d" % st, flush=True)
            if not ok:
                sys.exit(1)
            continue
        assert st == 0, st
        yv = from_storage(y, dt).astype(np.float64)
        r = oracle.forward(xv.astype(np.float64), p, q, m, pad, grid, weight=w, pw=pw, qw=qw, cout=Co)
        if m == "nearest":
            ok = np.array_equal(yv, r)
        else:
            S = oracle.condition(xv, p, q, m, pad, grid, weight=w, pw=pw, qw=qw, cout=Co)
            ok = bool((np.abs(yv - r) <= UNIT[dt] * np.abs(r) + UNIT_ABS[dt] + 1e-5 * S + 1e-30).all())
        print("case", i, json.dumps(c), "ok" if ok else "MISMATCH", flush=True)
        if not ok:
            bad = np.argwhere(np.abs(yv - r) > 1e-5 * np.abs(r) + 1e-6)
            print("first bad", bad[:5].tolist(), yv[tuple(bad[0])], r[tuple(bad[0])], flush=True)
            sys.exit(1)


if __name__ == "__main__":
    main()
