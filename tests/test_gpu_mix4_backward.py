"""GPU parity of the channel-mixing layer's backward (input gradient as an
implicit GEMM on MFMA per residue class with the pad adjoint folded at the
edges, weight gradient on MFMA over cells) against the FP64 oracle's adjoint,
through the C ABI, plus the autograd wrapper on it."""
import sys
from math import gcd

import numpy as np
import pytest

import oracle
import synth
from fcfs_testutil import UNIT, UNIT_ABS, storage_round, torch_dtype

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [
    # (p, q, pad, dtype, (N, Cin, H, W), Cout)
    (5, 4, "reflect", "bf16", (2, 16, 21, 150), 24),
    (3, 2, "zero", "f16", (1, 33, 17, 70), 40),
    (2, 3, "replicate", "bf16", (2, 8, 30, 400), 8),
    (7, 5, "reflect", "f16", (1, 5, 12, 33), 3),
    (1, 1, "zero", "bf16", (1, 64, 9, 64), 64),
    (4, 1, "reflect", "bf16", (1, 3, 5, 20), 70),
    # first taps past the edge (q >= 3p): samples no tap reads get 0
    (1, 8, "replicate", "bf16", (1, 4, 40, 75), 6),
    (2, 7, "reflect", "f16", (1, 5, 30, 61), 4),
    # axes short enough for every sample to take folded margins; 70 channels
    # (two channel tiles of the GEMM)
    (5, 4, "reflect", "bf16", (1, 3, 3, 5), 3),
    (3, 2, "replicate", "bf16", (1, 70, 2, 9), 70),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_mix4_backward_parity(case):
    import torch
    import paper_2203_10670_amd as fc
    p, q, pad, dt, shape, cout = CASES[case]
    _say("mix4 backward", CASES[case])
    N, C, H, W = shape
    g = gcd(p, q)
    pr, qr = p // g, q // g
    ho, wo = pr * -(-H // qr), pr * -(-W // qr)
    x = storage_round(synth.normal(60 + case, shape), dt)
    dy = storage_round(synth.normal(70 + case, (N, cout, ho, wo)), dt)
    w = storage_round(synth.normal(80 + case, (pr, pr, cout, C, 4, 4), std=1 / 32), dt)
    td = torch_dtype(dt)
    pl = fc.Plan(p, q, "mix4", pad)
    dx, dw = pl.backward(torch.from_numpy(dy).cuda().to(td), shape, x=torch.from_numpy(x).cuda().to(td),
                         weight=torch.from_numpy(w).cuda().to(td).contiguous(), need_dx=True, need_dw=True)
    torch.cuda.synchronize()
    gdx, gdw = dx.float().cpu().numpy(), dw.cpu().numpy()
    rdx, rdw = oracle.backward(dy.astype(np.float64), shape, p, q, "mix4", pad, x=x, weight=w, need_dw=True)
    sdx, sdw = oracle.condition_backward(dy, shape, p, q, "mix4", pad, x=x, weight=w, need_dw=True)
    bad = np.abs(gdx - rdx) > UNIT[dt] * np.abs(rdx) + UNIT_ABS[dt] + 1e-5 * sdx + 1e-30
    assert not bad.any(), "dx: %d bad, first %s gpu %r oracle %r" % (
        int(bad.sum()), np.argwhere(bad)[0], gdx[tuple(np.argwhere(bad)[0])], rdx[tuple(np.argwhere(bad)[0])])
    assert gdw.shape == rdw.shape
    bad = np.abs(gdw - rdw) > 1e-5 * sdw + 1e-30
    assert not bad.any(), "dw: %d bad of %d, first %s gpu %r oracle %r" % (
        int(bad.sum()), bad.size, np.argwhere(bad)[0], gdw[tuple(np.argwhere(bad)[0])], rdw[tuple(np.argwhere(bad)[0])])


def test_mix4_backward_deterministic_and_autograd():
    # fixed summation order: two runs agree bit for bit; the autograd wrapper
    # returns the same gradients as the C entry point
    import torch
    import paper_2203_10670_amd as fc
    shape, cout = (2, 12, 19, 90), 20
    x = torch.from_numpy(storage_round(synth.normal(90, shape), "bf16")).cuda().to(torch.bfloat16)
    w = torch.from_numpy(storage_round(synth.normal(91, (5, 5, cout, 12, 4, 4), std=1 / 32), "bf16")).cuda()
    w = w.to(torch.bfloat16).contiguous()
    pl = fc.Plan(5, 4, "mix4", "reflect")
    ho, wo = pl.output_size(19, 90)
    dy = torch.from_numpy(storage_round(synth.normal(92, (2, cout, ho, wo)), "bf16")).cuda().to(torch.bfloat16)
    a = pl.backward(dy, shape, x=x, weight=w, need_dx=True, need_dw=True)
    b = pl.backward(dy, shape, x=x, weight=w, need_dx=True, need_dw=True)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    xr = x.clone().requires_grad_(True)
    wr = w.clone().requires_grad_(True)
    y = fc.FCFSFunction.apply(xr, wr, pl)
    y.backward(dy)
    torch.cuda.synchronize()
    assert torch.equal(xr.grad, a[0])
    assert torch.equal(wr.grad, a[1].to(torch.bfloat16))


@pytest.mark.parametrize("p,q,pad,shape,cout", [(5, 4, "reflect", (2, 16, 21, 150), 24),
                                                (3, 2, "replicate", (1, 70, 9, 40), 33)])
def test_mix4_one_gradient_at_a_time_equals_both(p, q, pad, shape, cout):
    # one dy pass writes both re-laid-out copies of dy when both gradients are
    # asked for; each gradient asked for alone takes its own pass: the results
    # agree bit for bit
    import torch
    import paper_2203_10670_amd as fc
    N, C, H, W = shape
    g = gcd(p, q)
    pr, qr = p // g, q // g
    ho, wo = pr * -(-H // qr), pr * -(-W // qr)
    x = torch.from_numpy(storage_round(synth.normal(93, shape), "bf16")).cuda().to(torch.bfloat16)
    w = storage_round(synth.normal(94, (pr, pr, cout, C, 4, 4), std=1 / 32), "bf16")
    w = torch.from_numpy(w).cuda().to(torch.bfloat16).contiguous()
    dy = torch.from_numpy(storage_round(synth.normal(95, (N, cout, ho, wo)), "bf16")).cuda().to(torch.bfloat16)
    pl = fc.Plan(p, q, "mix4", pad)
    _say("mix4 one gradient at a time", p, q, pad, shape, cout)
    dx_only, _ = pl.backward(dy, shape, weight=w, need_dx=True)
    _, dw_only = pl.backward(dy, shape, x=x, weight=w, need_dx=False, need_dw=True)
    dx_both, dw_both = pl.backward(dy, shape, x=x, weight=w, need_dx=True, need_dw=True)
    torch.cuda.synchronize()
    assert torch.equal(dx_only, dx_both)
    assert torch.equal(dw_only, dw_both)


def test_mix4_input_gradient_16x64x512_sampled():
    """The 16x64x512^2 layer at 5/4 (BF16, 64 -> 64): the input gradient at the
    benchmarked size, checked on corner and interior windows against the
    oracle's adjoint of a crop that holds every output reading them."""
    import torch
    import paper_2203_10670_amd as fc
    N, C, H, W, p, q = 16, 64, 512, 512, 5, 4
    Ho = Wo = 640
    dy = storage_round(synth.normal(8, (N, C, Ho, Wo)), "bf16")
    w = storage_round(synth.normal(5, (p, p, C, C, 4, 4), std=1 / 32), "bf16")
    pl = fc.Plan(p, q, "mix4", "reflect")
    dx, _ = pl.backward(torch.from_numpy(dy).cuda().to(torch.bfloat16), (N, C, H, W),
                        weight=torch.from_numpy(w).cuda().to(torch.bfloat16).contiguous(), need_dx=True)
    torch.cuda.synchronize()
    _say("mix4 dx 16x64x512 done")
    # crop of input rows/cols [R0, R1) at multiples of q; outputs p*R0/q .. p*R1/q;
    # dx is compared 8 samples inside the crop's cut edges
    for n, (R0, R1), (C0, C1) in [(0, (0, 32), (0, 32)), (15, (480, 512), (480, 512)), (7, (240, 272), (100, 132))]:
        dyc = dy[n:n + 1, :, p * R0 // q: p * R1 // q, p * C0 // q: p * C1 // q]
        shape = (1, C, R1 - R0, C1 - C0)
        r, _ = oracle.backward(dyc.astype(np.float64), shape, p, q, "mix4", "reflect", weight=w)
        S, _ = oracle.condition_backward(dyc, shape, p, q, "mix4", "reflect", weight=w)
        ra, rb = (0 if R0 == 0 else 8), (R1 - R0 if R1 == H else R1 - R0 - 8)
        ca, cb = (0 if C0 == 0 else 8), (C1 - C0 if C1 == W else C1 - C0 - 8)
        g = dx[n:n + 1, :, R0 + ra: R0 + rb, C0 + ca: C0 + cb].float().cpu().numpy()
        rr, SS = r[:, :, ra:rb, ca:cb], S[:, :, ra:rb, ca:cb]
        bad = np.abs(g - rr) > UNIT["bf16"] * np.abs(rr) + UNIT_ABS["bf16"] + 1e-5 * SS + 1e-30
        assert not bad.any(), (n, R0, C0, int(bad.sum()))


def test_mix4_weight_gradient_16x64x512_windows():
    """The weight gradient of the 16x64x512^2 layer at 5/4 (BF16, 64 -> 64)
    through the full-size launch (every chunk of cell rows and the chunk
    reduction), with dy zero outside three windows of 8 x 8 cells: the top
    left corner of image 0 and the bottom right corner of image 15 (where the
    reflect padding supplies taps) and an interior window of image 7. By
    linearity the result is the sum of the windows' weight gradients, each
    from the oracle's adjoint on a crop that holds every tap of its cells."""
    import torch
    import paper_2203_10670_amd as fc
    N, C, H, W, p, q = 16, 64, 512, 512, 5, 4
    Mh = Mw = 128
    x = storage_round(synth.normal(4, (N, C, H, W)), "bf16")
    w = storage_round(synth.normal(5, (p, p, C, C, 4, 4), std=1 / 32), "bf16")
    win = [(0, (0, 8), (0, 8)), (15, (Mh - 8, Mh), (Mw - 8, Mw)), (7, (60, 68), (33, 41))]
    dy = np.zeros((N, C, p * Mh, p * Mw), dtype=np.float32)
    for k, (n, (a0, a1), (b0, b1)) in enumerate(win):
        vals = storage_round(synth.normal(20 + k, (C, p * (a1 - a0), p * (b1 - b0))), "bf16")
        dy[n, :, p * a0: p * a1, p * b0: p * b1] = vals
    pl = fc.Plan(p, q, "mix4", "reflect")
    _, gdw = pl.backward(torch.from_numpy(dy).cuda().to(torch.bfloat16), (N, C, H, W),
                         x=torch.from_numpy(x).cuda().to(torch.bfloat16),
                         weight=torch.from_numpy(w).cuda().to(torch.bfloat16).contiguous(), need_dw=True)
    torch.cuda.synchronize()
    gdw = gdw.cpu().numpy()
    _say("mix4 dw 16x64x512 windows done")
    rdw = np.zeros(w.shape, dtype=np.float64)
    sdw = np.zeros(w.shape, dtype=np.float64)
    for n, (a0, a1), (b0, b1) in win:
        # crop at multiples of q with two cells of margin (every tap of the
        # window's cells inside it; cut edges far from them)
        r0, r1 = max(0, q * (a0 - 2)), min(H, q * (a1 + 2))
        c0, c1 = max(0, q * (b0 - 2)), min(W, q * (b1 + 2))
        xc = x[n:n + 1, :, r0:r1, c0:c1]
        shape = xc.shape
        hc, wc = -(-(r1 - r0) // q), -(-(c1 - c0) // q)
        dyc = np.zeros((1, C, p * hc, p * wc), dtype=np.float64)
        ka, kb = a0 - r0 // q, b0 - c0 // q
        dyc[0, :, p * ka: p * (ka + a1 - a0), p * kb: p * (kb + b1 - b0)] = dy[n, :, p * a0: p * a1, p * b0: p * b1]
        _, r = oracle.backward(dyc, shape, p, q, "mix4", "reflect", x=xc, weight=w, need_dx=False, need_dw=True)
        _, sc = oracle.condition_backward(dyc, shape, p, q, "mix4", "reflect", x=xc, weight=w, need_dw=True)
        rdw += r
        sdw += sc
    bad = np.abs(gdw - rdw) > 1e-5 * sdw + 1e-30
    assert not bad.any(), "dw: %d bad of %d, first %s gpu %r oracle %r" % (
        int(bad.sum()), bad.size, np.argwhere(bad)[0], gdw[tuple(np.argwhere(bad)[0])], rdw[tuple(np.argwhere(bad)[0])])
