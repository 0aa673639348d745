"""GPU parity at the benchmarked sizes, on sampled planes and row bands
against the FP64 oracle:
- the 32x3x1024^2 batch at every benchmarked factor, method and padding, in
  FP32 and BF16 storage (the launch configuration the benchmark times);
- the end-to-end error of 16-bit storage against the oracle on the FP32
  input (input rounding, FP32 arithmetic and the rounded store together),
  asserted at 1e-2 of S = sum |w||x| per element, on that batch and on the
  16x64x512^2 N(0,1) feature maps at 5/4 bicubic;
- served requests at the serving workload's sizes (planes of 64..2048,
  p and q in 1..8), each equal bit for bit to its solo fcfs_forward and on
  sampled bands to the oracle."""
import sys
from math import gcd

import numpy as np
import pytest

import synth
from fcfs_testutil import (band_check, oracle_band_cond, splitmix64_uniform, storage_round,
                           torch_dtype)

pytestmark = pytest.mark.gpu

FRACS = [(3, 2), (2, 3), (5, 4), (4, 5)]
METHODS = ["nearest", "bilinear", "bicubic"]
PADS = ["zero", "reflect"]
SWEEP = [(p, q, m, pad) for (p, q) in FRACS for m in METHODS for pad in PADS]
# end-to-end tolerance of 16-bit storage against the FP32-input oracle,
# relative to S (input rounding u S, store rounding u |y| <= u S, FP32 sums)
E2E = 1e-2


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


_X = {}


def _batch():
    """The 32x3x1024^2 U[0,1) batch (seed 2) on the host and the device."""
    if "x" not in _X:
        import torch
        x = synth.uniform(2, (32, 3, 1024, 1024))
        _X["x"] = x
        _X["xt"] = torch.from_numpy(x).cuda()
    return _X["x"], _X["xt"]


def _bands(ho_cells):
    return [(0, 6), (ho_cells // 2 - 2, ho_cells // 2 + 2), (ho_cells - 5, ho_cells)]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("p,q,method,pad", SWEEP)
def test_sweep_1024_every_case(p, q, method, pad, dtype):
    """Every case of the benchmarked step, 3 planes x 3 bands each, at the
    kernel's bound (16-bit: against the oracle on the rounded input), and for
    BF16 also end to end against the oracle on the FP32 input."""
    import torch
    import paper_2203_10670_amd as fc
    x, xt = _batch()
    pl = fc.Plan(p, q, method, pad)
    xin = xt if dtype == "f32" else xt.to(torch_dtype(dtype))
    y = pl.forward(xin)
    torch.cuda.synchronize()
    pr = pl.p_red
    _say("1024 sweep", dtype, p, q, method, pad, tuple(y.shape))
    worst = 0.0
    for n, c in [(0, 0), (31, 2), (17, 1)]:
        plane32 = x[n, c]
        plane = plane32 if dtype == "f32" else storage_round(plane32, dtype)
        for m_lo, m_hi in _bands(y.shape[2] // pr):
            g = y[n, c, pr * m_lo: pr * m_hi].float().cpu().numpy()
            r, S = oracle_band_cond(plane, p, q, method, pad, m_lo, m_hi)
            band_check(g, r, S, dtype, method=method, what=f"{dtype} {p}/{q} {method} {pad} plane {n},{c}")
            if dtype != "f32":
                r32, S32 = oracle_band_cond(plane32, p, q, method, pad, m_lo, m_hi)
                err = np.abs(g.astype(np.float64) - r32)
                bad = err > E2E * S32 + 1e-30
                assert not bad.any(), "end to end %s %d/%d %s: %d bad" % (dtype, p, q, method, int(bad.sum()))
                worst = max(worst, float((err / np.maximum(S32, 1e-30)).max()))
    if dtype != "f32":
        _say("  end-to-end max |y - r| / S =", worst)
    del y


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_16bit_end_to_end_feature_maps(dtype):
    """16x64x512^2 N(0,1) (seed 4), 5/4 bicubic, reflect: 16-bit storage
    against the oracle on the FP32 input, per element within 1e-2 S, and
    against the oracle on the rounded input within the kernel's bound."""
    import torch
    import paper_2203_10670_amd as fc
    shape = (16, 64, 512, 512)
    x = synth.normal(4, shape)
    pl = fc.Plan(5, 4, "bicubic", "reflect")
    y = pl.forward(torch.from_numpy(x).cuda().to(torch_dtype(dtype)))
    torch.cuda.synchronize()
    worst, norm_err, norm_ref = 0.0, 0.0, 0.0
    for n, c in [(0, 0), (15, 63), (7, 31), (3, 5)]:
        plane32 = x[n, c]
        for m_lo, m_hi in _bands(y.shape[2] // 5):
            g = y[n, c, 5 * m_lo: 5 * m_hi].float().cpu().numpy()
            r32, S32 = oracle_band_cond(plane32, 5, 4, "bicubic", "reflect", m_lo, m_hi)
            err = np.abs(g.astype(np.float64) - r32)
            bad = err > E2E * S32 + 1e-30
            assert not bad.any(), "end to end %s: %d bad" % (dtype, int(bad.sum()))
            worst = max(worst, float((err / S32).max()))
            norm_err, norm_ref = max(norm_err, float(err.max())), max(norm_ref, float(np.abs(r32).max()))
            r, S = oracle_band_cond(storage_round(plane32, dtype), 5, 4, "bicubic", "reflect", m_lo, m_hi)
            band_check(g, r, S, dtype, what=f"{dtype} feature maps plane {n},{c}")
    _say("16x64x512^2 5/4 bicubic %s: end-to-end max |y - r|/S = %.3e, max|y - r| / max|r| = %.3e"
         % (dtype, worst, norm_err / norm_ref))


def _served_requests():
    """About 30 requests of the serving workload (seed 9: C = 3, H and W in
    64..2048, p and q in 1..8, method, padding and FP32/BF16 uniform), plus a
    2048-wide request at q = 8 and the largest upscale, p = 8 on 2048^2."""
    meta = synth.request_stream(9, 28, rate_per_s=0.0)
    reqs = [(r.p, r.q, METHODS[r.method], ["zero", "replicate", "reflect"][r.pad], ["f32", "bf16"][r.dtype],
             (1, r.c, r.h, r.w), r.seed) for r in meta]
    reqs.append((3, 8, "bicubic", "reflect", "f32", (1, 3, 700, 2048), 1234))
    reqs.append((7, 8, "bilinear", "zero", "bf16", (1, 3, 333, 2048), 1235))
    reqs.append((8, 1, "bicubic", "replicate", "bf16", (1, 3, 2048, 2048), 1236))
    reqs.append((8, 3, "nearest", "reflect", "f32", (1, 3, 1500, 1999), 1237))
    return reqs


def test_served_requests_at_serving_sizes():
    import torch
    import paper_2203_10670_amd as fc
    reqs = _served_requests()
    srv = fc.Server(0, 24 << 30, 64)
    tickets = [srv.submit(p, q, m, pad, dt, shape, seed=seed) for (p, q, m, pad, dt, shape, seed) in reqs]
    _say("submitted", len(tickets), "served requests")
    for k, (t, (p, q, m, pad, dt, shape, seed)) in enumerate(zip(tickets, reqs)):
        r = srv.wait(t)
        assert r.status == 0, (k, r.status)
        out_shape = (shape[0], shape[1], r.h_out, r.w_out)
        _say("served", k, p, q, m, pad, dt, shape, "->", out_shape)
        got = fc.device_view(r.y, out_shape, dt)
        srv.release(t)
        x = storage_round(splitmix64_uniform(seed, int(np.prod(shape))).reshape(shape), dt)
        solo = fc.Plan(p, q, m, pad).forward(torch.from_numpy(x).cuda().to(torch_dtype(dt)))
        assert torch.equal(got, solo), (k, p, q, m, pad, dt, shape)
        del solo
        g_ = gcd(p, q)
        pr = p // g_
        cells = r.h_out // pr
        for c in range(shape[1]):
            for m_lo, m_hi in _bands(cells) if cells >= 8 else [(0, cells)]:
                g = got[0, c, pr * m_lo: pr * m_hi].float().cpu().numpy()
                rr, S = oracle_band_cond(x[0, c], p, q, m, pad, m_lo, m_hi)
                band_check(g, rr, S, dt, method=m, what=f"served {k} {p}/{q} {m} {pad} {dt} {shape}")
        del got
    srv.close()
