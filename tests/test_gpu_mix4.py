"""GPU parity of the channel-mixing layer (implicit GEMM on MFMA: BF16/FP16
storage with FP32 accumulation, and FP32 storage on the FP32 matrix cores)
against the FP64 oracle, through the C ABI."""
import sys

import numpy as np
import pytest

import oracle
import synth
from fcfs_testutil import UNIT, UNIT_ABS, oracle_crop, storage_round, torch_dtype

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_mix4(x, w, p, q, pad, dtype, cout):
    import torch
    import paper_2203_10670_amd as fc
    td = torch_dtype(dtype)
    pl = fc.Plan(p, q, "mix4", pad)
    xt = torch.from_numpy(x).cuda().to(td)
    wt = torch.from_numpy(w).cuda().to(td)
    y = pl.forward(xt, wt)
    torch.cuda.synchronize()
    return y


def check(y, x, w, p, q, pad, dtype, cout, what):
    r = oracle.forward(x, p, q, "mix4", pad, weight=w, cout=cout)
    S = oracle.condition(x, p, q, "mix4", pad, weight=w, cout=cout)
    bad = np.abs(y - r) > UNIT[dtype] * np.abs(r) + UNIT_ABS[dtype] + 1e-5 * S + 1e-30
    assert not bad.any(), "%s: %d of %d bad; first %s gpu %r oracle %r" % (
        what, int(bad.sum()), bad.size, np.argwhere(bad)[0], y[tuple(np.argwhere(bad)[0])],
        r[tuple(np.argwhere(bad)[0])])


@pytest.mark.parametrize("dtype", ["bf16", "f16", "f32"])
@pytest.mark.parametrize("p,q,pad", [(5, 4, "reflect"), (3, 2, "zero"), (2, 3, "replicate"), (7, 5, "reflect"),
                                     (3, 4, "zero"), (1, 1, "zero"), (2, 7, "reflect"), (9, 8, "replicate"),
                                     (6, 5, "reflect")])
def test_mix4_small(dtype, p, q, pad):
    from math import gcd
    g = gcd(p, q)
    cin, cout = 6, 5
    x = storage_round(synth.normal(100 + p, (2, cin, 23, 70)), dtype)
    w = storage_round(synth.normal(101 + q, (p // g, p // g, cout, cin, 4, 4), std=1 / 32), dtype)
    y = run_mix4(x, w, p, q, pad, dtype, cout).float().cpu().numpy()
    check(y, x, w, p, q, pad, dtype, cout, f"{dtype} {p}/{q} {pad}")


def test_mix4_channel_tiles_and_ragged():
    # more than 64 output channels, odd input channel count, ragged cell tiles
    x = storage_round(synth.normal(110, (1, 7, 41, 141)), "bf16")
    w = storage_round(synth.normal(111, (5, 5, 70, 7, 4, 4), std=1 / 32), "bf16")
    y = run_mix4(x, w, 5, 4, "zero", "bf16", 70).float().cpu().numpy()
    check(y, x, w, 5, 4, "zero", "bf16", 70, "70 out")


def test_mix4_fp32_channel_tiles_and_ragged():
    # FP32 storage: more than 64 output channels, odd input channel count,
    # ragged cell tiles in both directions
    x = synth.normal(112, (1, 7, 41, 141))
    w = synth.normal(113, (5, 5, 70, 7, 4, 4), std=1 / 32)
    y = run_mix4(x, w, 5, 4, "zero", "f32", 70).cpu().numpy()
    check(y, x, w, 5, 4, "zero", "f32", 70, "fp32 70 out")


def test_mix4_misaligned_weight_refused():
    import torch
    import paper_2203_10670_amd as fc
    pl = fc.Plan(5, 4, "mix4", "zero")
    x = torch.zeros((1, 2, 8, 8), device="cuda")
    y = torch.zeros((1, 2, 10, 10), device="cuda")
    # a weight not aligned to 16 bytes is refused
    wb = torch.zeros(5 * 5 * 2 * 2 * 16 + 8, device="cuda", dtype=torch.bfloat16)
    xb = x.to(torch.bfloat16)
    yb = y.to(torch.bfloat16)
    assert fc.fcfs_forward(pl.handle, 1, 1, 2, 8, 8, xb.data_ptr(), wb.data_ptr() + 2, 2, yb.data_ptr(),
                           None) == fc.E_INVAL


def test_mix4_16x64x512_sampled():
    # the N=16, C=64, 512x512 BF16 layer at 5/4, 64 -> 64 channels, weights
    # N(0, 1/1024): checked on crops (corners and interior) of every plane
    N, C, H, W, p, q = 16, 64, 512, 512, 5, 4
    x = storage_round(synth.normal(4, (N, C, H, W)), "bf16")
    w = storage_round(synth.normal(5, (p, p, C, C, 4, 4), std=1 / 32), "bf16")
    y = run_mix4(x, w, p, q, "reflect", "bf16", C)
    _say("mix4 16x64x512 done", tuple(y.shape))
    for n in (0, 15):
        for mh, mw in [((0, 5), (0, 5)), ((60, 64), (31, 36)), ((123, 128), (123, 128))]:
            xs = x[n:n + 1]
            r = oracle_crop(xs, p, q, "mix4", "reflect", mh, mw, weight=w, cout=C)
            g = y[n:n + 1, :, p * mh[0]: p * mh[1], p * mw[0]: p * mw[1]].float().cpu().numpy()
            # |w| sums: bound by the rows' conditioning S from the crop
            from fcfs_testutil import oracle_crop as oc
            S = oc(np.abs(xs), p, q, "mix4", "reflect", mh, mw, weight=np.abs(w), cout=C)
            bad = np.abs(g - r) > UNIT["bf16"] * np.abs(r) + 1e-5 * S + 1e-30
            assert not bad.any(), (n, mh, mw, int(bad.sum()))


def test_mix4_fp32_16x64x512_sampled():
    # the N=16, C=64, 512x512 layer at 5/4 in FP32 storage, 64 -> 64 channels,
    # weights N(0, 1/1024): checked on crops of two planes
    N, C, H, W, p, q = 16, 64, 512, 512, 5, 4
    x = synth.normal(4, (N, C, H, W))
    w = synth.normal(5, (p, p, C, C, 4, 4), std=1 / 32)
    y = run_mix4(x, w, p, q, "reflect", "f32", C)
    _say("mix4 fp32 16x64x512 done", tuple(y.shape))
    for n in (0, 15):
        for mh, mw in [((0, 5), (0, 5)), ((60, 64), (31, 36)), ((123, 128), (123, 128))]:
            xs = x[n:n + 1]
            r = oracle_crop(xs, p, q, "mix4", "reflect", mh, mw, weight=w, cout=C)
            g = y[n:n + 1, :, p * mh[0]: p * mh[1], p * mw[0]: p * mw[1]].cpu().numpy()
            S = oracle_crop(np.abs(xs), p, q, "mix4", "reflect", mh, mw, weight=np.abs(w), cout=C)
            bad = np.abs(g - r) > UNIT["f32"] * np.abs(r) + 1e-5 * S + 1e-30
            assert not bad.any(), (n, mh, mw, int(bad.sum()))
