"""The allocation-free backward (fcfs_backward_noalloc, workspace in the
library's fixed device array) against fcfs_backward with a caller-supplied
workspace, through the C ABI: the same kernels, so the gradients must agree
bit for bit. Two calls in a row per method, the second on a smaller input,
so the second reads an array the first one left behind."""
import sys
from math import gcd

import numpy as np
import pytest

import synth
from fcfs_testutil import storage_round, torch_dtype

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _out_size(p, q, n):
    g = gcd(p, q)
    return (p // g) * -(-n // (q // g))


def _run_both(p, q, method, pad, dtype, shape, cout, seed):
    """(dx, dw) from fcfs_backward and from fcfs_backward_noalloc on the same
    seeded inputs, as numpy arrays (None where the method has no weights)."""
    import torch
    import paper_2203_10670_amd as fc
    n, c, h, w = shape
    ho, wo = _out_size(p, q, h), _out_size(p, q, w)
    td = torch_dtype(dtype)
    pr = p // gcd(p, q)
    x = torch.from_numpy(storage_round(synth.normal(seed, shape), dtype)).cuda().to(td)
    dy = torch.from_numpy(storage_round(synth.normal(seed + 1, (n, cout, ho, wo)), dtype)).cuda().to(td)
    if method == "dw4":
        wt = torch.from_numpy(synth.normal(seed + 2, (c, pr, pr, 4, 4))).cuda()
        wshape = tuple(wt.shape)
    elif method == "mix4":
        wt = torch.from_numpy(storage_round(synth.normal(seed + 2, (pr, pr, cout, c, 4, 4), std=1 / 32),
                                            dtype)).cuda().to(td).contiguous()
        wshape = tuple(wt.shape)
    else:
        wt, wshape = None, None
    pl = fc.Plan(p, q, method, pad)
    code = fc.DTYPES[dtype]
    sp = torch.cuda.current_stream().cuda_stream
    outs = []
    for noalloc in (False, True):
        dx = torch.full(shape, 7.0, dtype=td, device="cuda")
        dw = None if wshape is None else torch.full(wshape, 7.0, dtype=torch.float32, device="cuda")
        xp = x.data_ptr() if dw is not None else None
        wp = None if wt is None else wt.data_ptr()
        dwp = None if dw is None else dw.data_ptr()
        torch.cuda.synchronize()
        if noalloc:
            st = fc.fcfs_backward_noalloc(pl.handle, code, n, c, h, w, xp, wp, cout, dy.data_ptr(), dx.data_ptr(),
                                          dwp, sp)
        else:
            need = fc.fcfs_backward_workspace(pl.handle, code, n, c, h, w, cout)
            assert need <= fc.FCFS_NOALLOC_SCRATCH_BYTES, need
            ws = torch.empty(max(1, need), dtype=torch.uint8, device="cuda")
            st = fc.fcfs_backward(pl.handle, code, n, c, h, w, xp, wp, cout, dy.data_ptr(), dx.data_ptr(), dwp,
                                  ws.data_ptr(), need, sp)
        assert st == 0, (noalloc, fc.fcfs_status_string(st))
        torch.cuda.synchronize()
        outs.append((dx.float().cpu().numpy(), None if dw is None else dw.cpu().numpy()))
    return outs


CASES = [
    # method, p, q, pad, dtype, first shape, second (smaller) shape, c_out factor
    ("dw4", 3, 4, "reflect", "f32", (2, 8, 70, 300), (1, 3, 33, 41)),
    ("dw4", 5, 4, "zero", "bf16", (2, 4, 45, 130), (1, 2, 20, 17)),
    ("bicubic", 3, 2, "replicate", "f32", (2, 3, 37, 300), (1, 1, 9, 11)),
    ("mix4", 5, 4, "reflect", "bf16", (2, 16, 21, 150), (1, 8, 9, 40)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_noalloc_backward_matches_workspace_backward(case):
    method, p, q, pad, dtype, big, small = CASES[case]
    for k, shape in enumerate((big, small)):
        cout = shape[1] + 8 if method == "mix4" else shape[1]
        _say("noalloc backward", method, p, q, pad, dtype, shape, cout)
        (dx0, dw0), (dx1, dw1) = _run_both(p, q, method, pad, dtype, shape, cout, 300 + 10 * case + k)
        np.testing.assert_array_equal(dx1, dx0)
        assert np.isfinite(dx0).all()
        if dw0 is not None:
            np.testing.assert_array_equal(dw1, dw0)
            assert np.isfinite(dw0).all()


def test_noalloc_refuses_a_workspace_above_its_array():
    """A channel-mixing weight gradient whose partial sums exceed the fixed
    array is refused before anything is enqueued (the buffers are real, so
    even a launch would stay in bounds)."""
    import torch
    import paper_2203_10670_amd as fc
    n, c, h, w, cout = 1, 256, 64, 64, 256
    pl = fc.Plan(5, 4, "mix4", "zero")
    need = fc.fcfs_backward_workspace(pl.handle, 1, n, c, h, w, cout)
    assert need > fc.FCFS_NOALLOC_SCRATCH_BYTES
    x = torch.zeros((n, c, h, w), dtype=torch.bfloat16, device="cuda")
    dy = torch.zeros((n, cout, 80, 80), dtype=torch.bfloat16, device="cuda")
    wt = torch.zeros((5, 5, cout, c, 4, 4), dtype=torch.bfloat16, device="cuda")
    dx = torch.full((n, c, h, w), 3.0, dtype=torch.bfloat16, device="cuda")
    dw = torch.full(tuple(wt.shape), 3.0, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    st = fc.fcfs_backward_noalloc(pl.handle, 1, n, c, h, w, x.data_ptr(), wt.data_ptr(), cout, dy.data_ptr(),
                                  dx.data_ptr(), dw.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert st == fc.E_UNSUPPORTED
    assert bool((dx == 3.0).all()) and bool((dw == 3.0).all())
