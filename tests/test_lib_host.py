"""Host-side checks of libfcfs that need no GPU: the library loads, exports
every entry point its header declares, validates arguments, and its plan
tables (built by the library's own integer code) agree with the oracle's
dense per-phase kernels."""
import ctypes
import glob
import os
import re
import subprocess
import sys

import numpy as np
import pytest

import oracle
import paper_2203_10670_amd as fc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b(fcfs_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 10
    lib = ctypes.CDLL(fc.library_path)
    out = subprocess.run(["nm", "-D", "--defined-only", fc.library_path], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (fcfs_\w+)", out))
    for n in names:
        assert hasattr(lib, n), n
        assert n in exported, n


def test_status_strings_and_version():
    assert fc.fcfs_status_string(0) == "ok"
    assert "invalid" in fc.fcfs_status_string(1)
    assert fc.fcfs_version() >= 100


@pytest.mark.parametrize("args", [(0, 1, 0, 0), (1, 0, 0, 0), (3, 2, 9, 0), (3, 2, 0, 7), (-1, 2, 1, 1)])
def test_plan_rejects_bad_arguments(args):
    with pytest.raises(fc.FcfsError) as e:
        fc.fcfs_plan(*args)
    assert e.value.status == fc.E_INVAL


def test_plan_rejects_large_factors():
    with pytest.raises(fc.FcfsError) as e:
        fc.fcfs_plan(33, 1, 1, 0)
    assert e.value.status == fc.E_UNSUPPORTED
    # reduces before checking: 66/64 = 33/32 is too large, 64/32 = 2/1 is fine
    fc.fcfs_plan_destroy(fc.fcfs_plan(64, 32, 1, 0))


def test_forward_validation_needs_no_gpu():
    plan = fc.fcfs_plan(3, 2, 1, 1)
    # null pointers, bad sizes, weight given to a fixed method, dtype out of range
    assert fc.fcfs_forward(plan, 0, 1, 1, 8, 8, None, None, 1, None, None) == fc.E_INVAL
    assert fc.fcfs_forward(plan, 0, -1, 1, 8, 8, 16, None, 1, 16, None) == fc.E_INVAL
    # an empty problem is a valid no-op, whatever its pointers
    assert fc.fcfs_forward(plan, 0, 0, 1, 8, 8, None, None, 1, None, None) == fc.OK
    assert fc.fcfs_forward(plan, 0, 1, 1, 0, 8, None, None, 1, None, None) == fc.OK
    assert fc.fcfs_forward(plan, 0, 1, 1, 8, 8, 16, 16, 1, 16, None) == fc.E_INVAL
    assert fc.fcfs_forward(plan, 5, 1, 1, 8, 8, 16, None, 1, 16, None) == fc.E_INVAL
    assert fc.fcfs_forward(plan, 0, 1, 2, 8, 8, 16, None, 3, 16, None) == fc.E_INVAL
    # a plane of 2^31 output samples is refused before any launch
    assert fc.fcfs_forward(plan, 0, 1, 1, 40000, 40000, 16, None, 1, 16, None) == fc.E_UNSUPPORTED
    dw = fc.fcfs_plan(3, 2, 3, 1)
    assert fc.fcfs_forward(dw, 0, 1, 1, 8, 8, 16, None, 1, 16, None) == fc.E_INVAL
    fc.fcfs_plan_destroy(plan)
    fc.fcfs_plan_destroy(dw)


def test_noalloc_backward_validation_needs_no_gpu():
    """Argument errors and sizes beyond the fixed device array are refused
    before the array is looked up or anything is enqueued."""
    assert fc.fcfs_backward_noalloc(None, 0, 1, 1, 8, 8, None, None, 1, 16, 16, None, None) == fc.E_INVAL
    fixed = fc.fcfs_plan(3, 2, 2, 1)
    # a weight gradient for a fixed method, a c_out mismatch
    assert fc.fcfs_backward_noalloc(fixed, 0, 1, 1, 8, 8, 16, None, 1, 16, None, 16, None) == fc.E_INVAL
    assert fc.fcfs_backward_noalloc(fixed, 0, 1, 2, 8, 8, None, None, 3, 16, 16, None, None) == fc.E_INVAL
    # an empty problem needs no workspace and enqueues nothing
    assert fc.fcfs_backward_noalloc(fixed, 0, 0, 1, 8, 8, None, None, 1, None, 16, None, None) == fc.OK
    mix = fc.fcfs_plan(5, 4, 4, 0)
    need = fc.fcfs_backward_workspace(mix, 1, 1, 256, 64, 64, 256)
    assert need > fc.FCFS_NOALLOC_SCRATCH_BYTES
    assert fc.fcfs_backward_noalloc(mix, 1, 1, 256, 64, 64, 16, 16, 256, 16, 16, 16, None) == fc.E_UNSUPPORTED
    fc.fcfs_plan_destroy(fixed)
    fc.fcfs_plan_destroy(mix)


FRACS = [(1, 1), (3, 2), (2, 3), (5, 4), (4, 5), (3, 4), (1, 2), (2, 1), (7, 3), (6, 4), (2, 11),
         (27, 11), (8, 1), (1, 8), (32, 31), (31, 32)]


@pytest.mark.parametrize("p,q", FRACS)
@pytest.mark.parametrize("method", ["nearest", "bilinear", "bicubic"])
@pytest.mark.parametrize("grid", ["half", "paper", "asym"])
def test_plan_tables_match_oracle_kernels(p, q, method, grid):
    pl = fc.Plan(p, q, method, "zero", grid)
    for j in range(pl.p_red):
        off, w = fc.fcfs_plan_taps(pl.handle, 0, j)
        h = oracle.phase_kernel(p, q, method, grid, j)
        K = (len(h) - 1) // 2
        dense = np.zeros_like(h)
        for t in range(pl.taps):
            o = off + t
            assert -K <= o <= K
            dense[K - o] += w[t]
        # FP32 weights from FP64: one rounding
        np.testing.assert_allclose(dense, h, rtol=0, atol=2e-7, err_msg=f"phase {j}")


@pytest.mark.parametrize("p,q", FRACS)
def test_output_size_matches_oracle(p, q):
    pl = fc.Plan(p, q, "bilinear", "zero")
    for n in (1, 2, 5, 7, 64, 67, 1023, 1024, 2048):
        assert pl.output_size(n, n + 1) == (oracle.out_len(p, q, n), oracle.out_len(p, q, n + 1))


def test_anisotropic_plan():
    pl = fc.Plan(3, 2, "bicubic", "reflect", pw=5, qw=4)
    assert pl.output_size(10, 16) == (15, 20)
    # an axis at 1/1 next to a resampled one copies with one tap (the other
    # keeps the method's four), on the grids that sample inputs exactly
    pl = fc.Plan(1, 1, "bicubic", "reflect", pw=3, qw=2)
    assert pl.taps == 4
    assert fc.fcfs_plan_taps(pl.handle, 0, 0) == (0, [1.0, 0.0, 0.0, 0.0])
    assert fc.fcfs_forward_config(pl.handle, 0, 1, 1, 64, 4096)[0] // 100000 == 1
    pl = fc.Plan(3, 2, "bilinear", "zero", pw=1, qw=1)
    assert fc.fcfs_plan_taps(pl.handle, 1, 0) == (0, [1.0, 0.0, 0.0, 0.0])
    assert fc.fcfs_forward_config(pl.handle, 0, 1, 1, 64, 4096)[0] // 100000 == 2
    # the paper grid's 1/1 axis interpolates half-way between samples: no copy
    pl = fc.Plan(1, 1, "bicubic", "reflect", "paper", pw=3, qw=2)
    assert fc.fcfs_plan_taps(pl.handle, 0, 0)[1] != [1.0, 0.0, 0.0, 0.0]


def test_request_structs_match_header(tmp_path):
    # the ctypes mirrors of fcfs_request / fcfs_result have the C layout
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "fcfs.h"\n'
                   'int main(){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(fcfs_request), sizeof(fcfs_result),'
                   'offsetof(fcfs_request, n), offsetof(fcfs_request, seed), offsetof(fcfs_request, y),'
                   'offsetof(fcfs_result, t_done_us));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe)], check=True)
    got = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    want = [ctypes.sizeof(fc.fcfs_request), ctypes.sizeof(fc.fcfs_result), fc.fcfs_request.n.offset,
            fc.fcfs_request.seed.offset, fc.fcfs_request.y.offset, fc.fcfs_result.t_done_us.offset]
    assert [int(v) for v in got] == want


def test_server_needs_a_device():
    # no GPU here: creation reports a device error and nothing else happens
    with pytest.raises(fc.FcfsError) as e:
        fc.Server(0, 1 << 20, 4)
    assert e.value.status in (fc.E_DEVICE, fc.E_NOMEM)
    h = ctypes.c_void_p()
    assert fc.lib.fcfs_server_create(0, 1 << 20, 0, ctypes.byref(h)) == fc.E_INVAL


def test_one_hip_runtime_with_torch():
    # importing the package before torch must not bring a second HIP runtime
    # into the process (the library binds to the one torch uses)
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_2203_10670_amd, torch\n"
            "libs = set(l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l)\n"
            "print(len(libs), sorted(libs))\n" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.startswith("1 "), out.stdout


def test_nd_entry_points_validate_without_gpu():
    # 1D: the plan's height factor must be 1/1, fixed methods, not the paper grid
    one = fc.fcfs_plan_ex(1, 1, 3, 2, 2, 2, 0)
    assert fc.fcfs_forward_1d(one, 0, 0, 3, 100, None, None, None) == fc.OK        # empty: no-op
    assert fc.fcfs_forward_1d(one, 0, 1, 3, 100, None, None, None) == fc.E_INVAL   # null pointers
    two = fc.fcfs_plan_ex(3, 2, 3, 2, 2, 2, 0)
    assert fc.fcfs_forward_1d(two, 0, 1, 3, 100, 16, 16, None) == fc.E_INVAL
    paper = fc.fcfs_plan_ex(1, 1, 3, 2, 1, 2, 1)
    assert fc.fcfs_forward_1d(paper, 0, 1, 3, 100, 16, 16, None) == fc.E_UNSUPPORTED
    # 3D: depth plan with a 1/1 width axis, matching method / pad / grid
    pd = fc.fcfs_plan_ex(3, 2, 1, 1, 2, 2, 0)
    phw = fc.fcfs_plan_ex(5, 4, 2, 3, 2, 2, 0)
    n, c, d, h, w = 2, 3, 7, 9, 70
    ws = fc.fcfs_forward_3d_workspace(pd, phw, 0, n, c, d, h, w)
    do, ho, wo = 3 * 4, 5 * 3, 2 * 24
    assert ws == 4 * min(n * c * d * ho * wo, n * c * do * h * w)
    assert fc.fcfs_forward_3d_workspace(pd, phw, 1, n, c, d, h, w) == ws // 2
    assert fc.fcfs_forward_3d(pd, phw, 0, n, c, d, h, w, 16, 16, 16, ws - 1, None) == fc.E_INVAL
    assert fc.fcfs_forward_3d(pd, phw, 0, n, c, d, h, w, None, 16, 16, ws, None) == fc.E_INVAL
    assert fc.fcfs_forward_3d(pd, phw, 0, 0, c, d, h, w, None, None, None, 0, None) == fc.OK
    # the depth plan's width must be 1/1; methods must agree; paper grid refused
    assert fc.fcfs_forward_3d(phw, phw, 0, n, c, d, h, w, 16, 16, 16, 1 << 30, None) == fc.E_INVAL
    other = fc.fcfs_plan_ex(3, 2, 1, 1, 1, 2, 0)
    assert fc.fcfs_forward_3d(other, phw, 0, n, c, d, h, w, 16, 16, 16, 1 << 30, None) == fc.E_INVAL
    pd_paper = fc.fcfs_plan_ex(3, 2, 1, 1, 2, 2, 1)
    phw_paper = fc.fcfs_plan_ex(5, 4, 2, 3, 2, 2, 1)
    assert fc.fcfs_forward_3d(pd_paper, phw_paper, 0, n, c, d, h, w, 16, 16, 16, 1 << 30, None) == fc.E_UNSUPPORTED
    dw4 = fc.fcfs_plan_ex(3, 2, 1, 1, 3, 2, 0)
    assert fc.fcfs_forward_3d(dw4, phw, 0, n, c, d, h, w, 16, 16, 16, 1 << 30, None) == fc.E_INVAL
    for pl in (one, two, paper, pd, phw, other, pd_paper, phw_paper, dw4):
        fc.fcfs_plan_destroy(pl)


def test_binding_refuses_mismatched_weights():
    # the C ABI reads a learned layer's weight through a plain pointer whose
    # type and extent follow from the method; the binding checks them first
    # (these checks run before any device pointer is taken, so CPU tensors do)
    import torch
    x = torch.zeros((2, 3, 8, 8))
    dw = fc.Plan(3, 4, "dw4", "reflect")
    with pytest.raises(TypeError, match="float32"):
        dw.forward(x.to(torch.bfloat16), torch.zeros((3, 3, 3, 4, 4), dtype=torch.bfloat16))
    with pytest.raises(ValueError, match="shape"):
        dw.forward(x, torch.zeros((3, 3, 3, 4, 3)))
    with pytest.raises(ValueError, match="shape"):
        dw.forward(x, torch.zeros((2, 3, 3, 4, 4)))      # channel count
    with pytest.raises(ValueError, match="needs a weight"):
        dw.forward(x)
    # the reduced width factor sizes the phase axis: 6/8 -> 3 phases
    dw68 = fc.Plan(6, 8, "dw4", "reflect")
    with pytest.raises(ValueError, match="shape"):
        dw68.forward(x, torch.zeros((3, 6, 6, 4, 4)))
    mx = fc.Plan(5, 4, "mix4", "reflect", pw=3, qw=2)
    xb = x.to(torch.bfloat16)
    with pytest.raises(TypeError, match="activations' type"):
        mx.forward(xb, torch.zeros((5, 3, 4, 3, 4, 4)))
    with pytest.raises(ValueError, match="shape"):
        mx.forward(xb, torch.zeros((3, 5, 4, 3, 4, 4), dtype=torch.bfloat16))
    with pytest.raises(ValueError, match="shape"):
        mx.forward(xb, torch.zeros((5, 3, 4, 2, 4, 4), dtype=torch.bfloat16))
    with pytest.raises(ValueError, match="takes no weight"):
        fc.Plan(3, 2, "bicubic", "zero").forward(x, torch.zeros((3, 3, 3, 4, 4)))
    # a well-formed weight passes the checks and reaches the device-pointer check
    with pytest.raises(ValueError, match="device tensors"):
        dw.forward(x, torch.zeros((3, 3, 3, 4, 4)))
    with pytest.raises(ValueError, match="device tensors"):
        mx.forward(xb, torch.zeros((5, 3, 7, 3, 4, 4), dtype=torch.bfloat16))
    # backward: dy's channels must match the mixing weight's outputs
    with pytest.raises(ValueError, match="outputs"):
        mx.backward(torch.zeros((2, 6, 10, 12), dtype=torch.bfloat16), (2, 3, 8, 8),
                    weight=torch.zeros((5, 3, 7, 3, 4, 4), dtype=torch.bfloat16))
