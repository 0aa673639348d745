"""GPU parity of the backward kernels (input gradient for every method, weight
gradient of the learned depthwise layer) against the FP64 oracle's adjoint,
through the C ABI, plus the autograd wrapper against finite differences."""
import sys

import numpy as np
import pytest

import oracle
import synth
from fcfs_testutil import UNIT, UNIT_ABS, storage_round, torch_dtype

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_backward(x32, dy32, p, q, method, pad, dtype="f32", weight=None, need_dx=True, need_dw=False,
                 pw=None, qw=None):
    import torch
    import paper_2203_10670_amd as fc
    td = torch_dtype(dtype)
    xt = torch.from_numpy(x32).cuda().to(td)
    dyt = torch.from_numpy(dy32).cuda().to(td)
    wt = None if weight is None else torch.from_numpy(np.ascontiguousarray(weight, np.float32)).cuda()
    pl = fc.Plan(p, q, method, pad, "half", pw, qw)
    dx, dw = pl.backward(dyt, tuple(x32.shape), x=xt if need_dw else None, weight=wt, need_dx=need_dx,
                         need_dw=need_dw)
    torch.cuda.synchronize()
    return (None if dx is None else dx.float().cpu().numpy(), None if dw is None else dw.cpu().numpy())


def check_grads(x, dy, p, q, method, pad, dtype="f32", weight=None, need_dw=False, pw=None, qw=None, what=""):
    gdx, gdw = gpu_backward(x, dy, p, q, method, pad, dtype, weight, True, need_dw, pw, qw)
    rdx, rdw = oracle.backward(dy.astype(np.float64), x.shape, p, q, method, pad, x=x, weight=weight,
                               need_dw=need_dw, pw=pw, qw=qw)
    sdx, sdw = oracle.condition_backward(dy, x.shape, p, q, method, pad, x=x, weight=weight, need_dw=need_dw,
                                         pw=pw, qw=qw)
    bad = np.abs(gdx - rdx) > UNIT[dtype] * np.abs(rdx) + UNIT_ABS[dtype] + 1e-5 * sdx + 1e-30
    assert not bad.any(), "%s dx: %d bad, first %s gpu %r oracle %r" % (
        what, int(bad.sum()), np.argwhere(bad)[0], gdx[tuple(np.argwhere(bad)[0])], rdx[tuple(np.argwhere(bad)[0])])
    if need_dw:
        bad = np.abs(gdw - rdw) > 1e-5 * sdw + 1e-30
        assert not bad.any(), "%s dw: %d bad of %d" % (what, int(bad.sum()), bad.size)


FRACS = [(3, 2), (2, 3), (5, 4), (4, 5), (3, 4), (1, 1), (4, 1), (2, 11), (27, 11)]


@pytest.mark.parametrize("p,q", FRACS)
@pytest.mark.parametrize("method", ["nearest", "bilinear", "bicubic"])
@pytest.mark.parametrize("pad", ["zero", "replicate", "reflect"])
def test_input_gradient_fixed(p, q, method, pad):
    x = synth.normal(50 + p + q, (2, 2, 37, 300))
    from math import gcd
    g = gcd(p, q)
    ho, wo = (p // g) * -(-37 // (q // g)), (p // g) * -(-300 // (q // g))
    dy = synth.normal(60 + p * q, (2, 2, ho, wo))
    _say("dx", p, q, method, pad)
    check_grads(x, dy, p, q, method, pad, what=f"{p}/{q} {method} {pad}")


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_input_gradient_16bit(dtype):
    for p, q, m in [(3, 2, "bicubic"), (3, 4, "bilinear"), (2, 11, "nearest")]:
        x = storage_round(synth.normal(70, (1, 3, 41, 150)), dtype)
        from math import gcd
        g = gcd(p, q)
        dy = storage_round(synth.normal(71, (1, 3, (p // g) * -(-41 // (q // g)), (p // g) * -(-150 // (q // g)))), dtype)
        check_grads(x, dy, p, q, m, "reflect", dtype, what=f"{dtype} {p}/{q} {m}")


@pytest.mark.parametrize("p,q", [(3, 4), (3, 2), (5, 4), (2, 3)])
@pytest.mark.parametrize("pad", ["zero", "replicate", "reflect"])
def test_learned_depthwise_gradients(p, q, pad):
    x = synth.normal(80, (3, 4, 45, 130))
    w = synth.normal(81, (4, p, p, 4, 4))
    from math import gcd
    g = gcd(p, q)
    dy = synth.normal(82, (3, 4, (p // g) * -(-45 // (q // g)), (p // g) * -(-130 // (q // g))))
    check_grads(x, dy, p, q, "dw4", pad, weight=w, need_dw=True, what=f"dw4 {p}/{q} {pad}")


@pytest.mark.parametrize("p,q,pad,dtype", [(2, 3, "reflect", "f32"), (3, 4, "replicate", "bf16")])
def test_learned_depthwise_wide_rows_one_gradient_at_a_time(p, q, pad, dtype):
    # rows of 600 samples (three column blocks of the input-gradient kernel);
    # each gradient requested alone equals the oracle's, and equals the one
    # computed beside the other bit for bit
    from math import gcd
    g = gcd(p, q)
    x = storage_round(synth.normal(83, (2, 3, 23, 600)), dtype)
    w = synth.normal(84, (3, p // g, p // g, 4, 4))
    dy = storage_round(synth.normal(85, (2, 3, (p // g) * -(-23 // (q // g)), (p // g) * -(-600 // (q // g)))), dtype)
    _say("dw4 wide", p, q, pad, dtype)
    dx_only, _ = gpu_backward(x, dy, p, q, "dw4", pad, dtype, w, need_dx=True, need_dw=False)
    _, dw_only = gpu_backward(x, dy, p, q, "dw4", pad, dtype, w, need_dx=False, need_dw=True)
    dx_both, dw_both = gpu_backward(x, dy, p, q, "dw4", pad, dtype, w, need_dx=True, need_dw=True)
    assert np.array_equal(dx_only, dx_both) and np.array_equal(dw_only, dw_both)
    rdx, rdw = oracle.backward(dy.astype(np.float64), x.shape, p, q, "dw4", pad, x=x, weight=w, need_dw=True)
    sdx, sdw = oracle.condition_backward(dy, x.shape, p, q, "dw4", pad, x=x, weight=w, need_dw=True)
    assert (np.abs(dx_only - rdx) <= UNIT[dtype] * np.abs(rdx) + UNIT_ABS[dtype] + 1e-5 * sdx + 1e-30).all()
    assert (np.abs(dw_only - rdw) <= 1e-5 * sdw + 1e-30).all()


def bicubic_init(p, q, C, noise_seed):
    """4x4 learned taps initialised to the bicubic outer product plus noise of
    variance 0.01, for every channel."""
    from fractions import Fraction
    from math import floor
    from oracle import exact
    taps = []
    for j in range(p):
        u = exact.coord(j, p, q, "half")
        b = floor(u)
        taps.append([float(exact.keys_cubic(u - (b - 1 + a))) for a in range(4)])
    t = np.array(taps)
    base = np.einsum("ia,jb->ijab", t, t)[None].repeat(C, axis=0)
    return (base + synth.normal(noise_seed, base.shape, std=0.1)).astype(np.float32)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_learned_layer_8x64x256(dtype):
    # the N=8, C=64, 256x256, 3/4 learned-layer workload, checked on 4 channels
    # (the weight gradient of a channel depends only on that channel's planes)
    import torch
    import paper_2203_10670_amd as fc
    N, C, H, W, p, q = 8, 64, 256, 256, 3, 4
    x = storage_round(synth.normal(6, (N, C, H, W)), dtype)
    w = bicubic_init(p, q, C, 7)
    dy = storage_round(synth.normal(8, (N, C, 192, 192)), dtype)
    td = torch_dtype(dtype)
    pl = fc.Plan(p, q, "dw4", "reflect")
    xt, dyt, wt = torch.from_numpy(x).cuda().to(td), torch.from_numpy(dy).cuda().to(td), torch.from_numpy(w).cuda()
    y = pl.forward(xt, wt)
    dx, dw = pl.backward(dyt, (N, C, H, W), x=xt, weight=wt, need_dx=True, need_dw=True)
    torch.cuda.synchronize()
    _say("learned 8x64x256", dtype)
    chans = [0, 17, 42, 63]
    xs, dys, ws = x[:, chans], dy[:, chans], w[chans]
    ry = oracle.forward(xs, p, q, "dw4", "reflect", weight=ws)
    sy = oracle.condition(xs, p, q, "dw4", "reflect", weight=ws)
    gy = y[:, chans].float().cpu().numpy()
    assert (np.abs(gy - ry) <= UNIT[dtype] * np.abs(ry) + UNIT_ABS[dtype] + 1e-5 * sy + 1e-30).all()
    rdx, rdw = oracle.backward(dys, xs.shape, p, q, "dw4", "reflect", x=xs, weight=ws, need_dw=True)
    sdx, sdw = oracle.condition_backward(dys, xs.shape, p, q, "dw4", "reflect", x=xs, weight=ws, need_dw=True)
    gdx = dx[:, chans].float().cpu().numpy()
    gdw = dw[chans].cpu().numpy()
    assert (np.abs(gdx - rdx) <= UNIT[dtype] * np.abs(rdx) + UNIT_ABS[dtype] + 1e-5 * sdx + 1e-30).all()
    assert (np.abs(gdw - rdw) <= 1e-5 * sdw + 1e-30).all()


def test_autograd_function_and_finite_differences():
    import torch
    import paper_2203_10670_amd as fc
    torch.manual_seed(0)
    p, q = 3, 4
    pl = fc.Plan(p, q, "dw4", "replicate")
    x = torch.from_numpy(synth.normal(90, (2, 3, 20, 28))).cuda().requires_grad_(True)
    w = torch.from_numpy(bicubic_init(p, q, 3, 91)).cuda().requires_grad_(True)
    y = fc.FCFSFunction.apply(x, w, pl)
    g = torch.from_numpy(synth.normal(92, tuple(y.shape))).cuda()
    (y * g).sum().backward()
    # oracle gradients
    rdx, rdw = oracle.backward(g.cpu().numpy(), tuple(x.shape), p, q, "dw4", "replicate",
                               x=x.detach().cpu().numpy(), weight=w.detach().cpu().numpy(), need_dw=True)
    np.testing.assert_allclose(x.grad.cpu().numpy(), rdx, rtol=1e-4, atol=1e-4)
    np.testing.assert_allclose(w.grad.cpu().numpy(), rdw, rtol=1e-4, atol=1e-3)
    # finite differences of the (linear) objective in FP32 on the GPU
    def f(xx, ww):
        with torch.no_grad():
            return float((pl.forward(xx.contiguous(), ww.contiguous()).double() * g.double()).sum())
    rng = np.random.default_rng(93)
    for _ in range(3):
        v = torch.from_numpy(rng.standard_normal(tuple(x.shape)).astype(np.float32)).cuda()
        h = 1e-2
        fd = (f(x.detach() + h * v, w.detach()) - f(x.detach() - h * v, w.detach())) / (2 * h)
        an = float((x.grad * v).sum())
        assert abs(fd - an) <= 1e-3 * max(1.0, abs(an))
        vw = torch.from_numpy(rng.standard_normal(tuple(w.shape)).astype(np.float32)).cuda()
        fd = (f(x.detach(), w.detach() + h * vw) - f(x.detach(), w.detach() - h * vw)) / (2 * h)
        an = float((w.grad * vw).sum())
        assert abs(fd - an) <= 1e-3 * max(1.0, abs(an))
    # fixed method: autograd dx equals the oracle adjoint
    pb = fc.Plan(5, 4, "bicubic", "reflect")
    xb = torch.from_numpy(synth.normal(94, (1, 2, 17, 33))).cuda().requires_grad_(True)
    yb = fc.FCFSFunction.apply(xb, None, pb)
    gb = torch.from_numpy(synth.normal(95, tuple(yb.shape))).cuda()
    (yb * gb).sum().backward()
    rdx, _ = oracle.backward(gb.cpu().numpy(), tuple(xb.shape), 5, 4, "bicubic", "reflect")
    np.testing.assert_allclose(xb.grad.cpu().numpy(), rdx, rtol=1e-5, atol=1e-5)


def test_backward_validation():
    import torch
    import paper_2203_10670_amd as fc
    pl = fc.Plan(3, 2, "bicubic", "zero")
    dy = torch.zeros((1, 1, 6, 6), device="cuda")
    # a weight gradient for a fixed method is refused before any launch
    st = fc.fcfs_backward(pl.handle, 0, 1, 1, 4, 4, dy.data_ptr(), None, 1, dy.data_ptr(), None,
                          dy.data_ptr(), dy.data_ptr(), 1 << 20, None)
    assert st == fc.E_INVAL
    # too small a workspace
    dx = torch.empty((1, 1, 4, 4), device="cuda")
    st = fc.fcfs_backward(pl.handle, 0, 1, 1, 4, 4, None, None, 1, dy.data_ptr(), dx.data_ptr(), None,
                          dy.data_ptr(), 8, None)
    assert st == fc.E_INVAL
