"""The GPU kernels' source, compiled for the CPU under a host emulation of the
HIP dialect (tests/hostemu: one thread per lane, a barrier per wave) with the
address and undefined-behaviour sanitizers, checked against the FP64 oracle.

This validates the kernels' indexing, bounds and logic without a GPU. It does
not replace the GPU parity tests (tests/test_gpu_*.py), which run the real
gfx950 code objects; nothing in the library can reach this build.
"""
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "hostemu"))

import build as hostemu_build  # noqa: E402


def _run(cases):
    lib = hostemu_build.build()
    env = dict(os.environ, LD_PRELOAD=hostemu_build.asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([sys.executable, os.path.join(HERE, "hostemu", "run_cases.py"), lib, json.dumps(cases)],
                       env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert r.stdout.count(" ok") == len(cases), r.stdout[-4000:]


# Every factor with every method when FCFS_HOSTEMU_ALL=1; by default every
# factor with one method (rotating) and the benchmarked factors with all three.
ALL = os.environ.get("FCFS_HOSTEMU_ALL") == "1"
FIXED = []
for i, (p, q) in enumerate([(3, 2), (2, 3), (5, 4), (4, 5), (3, 4), (1, 1), (4, 1), (1, 4), (6, 4), (2, 11),
                            (27, 11), (1, 32), (32, 31)]):
    for k, m in enumerate(["nearest", "bilinear", "bicubic"]):
        if ALL or i < 4 or k == i % 3:
            FIXED.append({"p": p, "q": q, "method": m, "pad": ["zero", "replicate", "reflect"][(p + q) % 3],
                          "shape": [1, 2, 23, 70]})


def test_fixed_methods_all_factors():
    _run(FIXED)


def test_wide_rows_multiple_strips_and_bands():
    _run([{"p": 3, "q": 2, "method": "bicubic", "pad": "reflect", "shape": [1, 1, 40, 300]},
          {"p": 2, "q": 3, "method": "bilinear", "pad": "zero", "shape": [1, 1, 30, 700]},
          {"p": 1, "q": 8, "method": "bicubic", "pad": "replicate", "shape": [1, 1, 33, 1100]},
          # several strips, ragged last one
          {"p": 3, "q": 2, "method": "bicubic", "pad": "replicate", "shape": [1, 1, 20, 800]},
          {"p": 5, "q": 4, "method": "bilinear", "pad": "zero", "shape": [1, 2, 12, 900]}])


def test_storage_types():
    cases = []
    for dt in ["bf16", "f16"]:
        for (p, q) in [(3, 2), (4, 5), (27, 11)]:
            for m in ["nearest", "bicubic"]:
                cases.append({"p": p, "q": q, "method": m, "pad": "reflect", "dtype": dt, "shape": [1, 2, 17, 90]})
    _run(cases)


def test_paired_16bit_io():
    # even widths and aligned tensors take the paired instance: left and right
    # edge strips, several strips, staged segments of 128 and 256 pairs; the
    # misaligned output takes the unpaired one (the sanitizers flag a
    # misaligned dword store)
    cases = []
    for i, (p, q, m, W) in enumerate([(3, 2, "bicubic", 300), (2, 3, "bilinear", 700), (4, 5, "bicubic", 400),
                                      (5, 4, "bilinear", 208), (3, 4, "bicubic", 256), (27, 11, "nearest", 440),
                                      (1, 1, "bicubic", 258), (3, 2, "nearest", 132), (3, 2, "bicubic", 800),
                                      (5, 4, "nearest", 1000)]):
        for dt in ["bf16", "f16"]:
            cases.append({"p": p, "q": q, "method": m, "pad": ["zero", "replicate", "reflect"][i % 3],
                          "dtype": dt, "shape": [1, 2, 11, W], "expect_paired": True})
    cases.append({"p": 3, "q": 2, "method": "bicubic", "pad": "reflect", "dtype": "bf16", "shape": [1, 2, 9, 300],
                  "misalign": True, "expect_paired": True})
    _run(cases)


def test_copy_axis_beside_resampled_axis():
    # a 1/1 axis copies with one tap while the other keeps the method's taps
    # (the instances with separate height and width tap counts)
    cases = []
    for (p, q, pw, qw) in [(1, 1, 3, 2), (1, 1, 2, 7), (5, 4, 1, 1), (2, 3, 1, 1)]:
        for m in ["bilinear", "bicubic"]:
            cases.append({"p": p, "q": q, "pw": pw, "qw": qw, "method": m, "pad": "reflect", "shape": [1, 2, 21, 150]})
    cases.append({"p": 1, "q": 1, "pw": 3, "qw": 2, "method": "bicubic", "pad": "zero", "dtype": "bf16",
                  "shape": [1, 1, 12, 130]})
    _run(cases)


def test_channel_mixing_backward():
    # input gradient (implicit GEMM per residue class on MFMA, pad adjoint
    # folded at the edges) and weight gradient (MFMA over cells, chunks added
    # in order), 16-bit storage
    cases = []
    for i, (p, q, pad, dt, shape, cout) in enumerate([
            (5, 4, "reflect", "bf16", [2, 3, 9, 40], 5),
            (3, 2, "zero", "f16", [1, 9, 7, 35], 33),
            # first taps past the edge (q >= 3p): samples no tap reads get 0
            (1, 8, "replicate", "bf16", [1, 2, 20, 37], 3),
            # axes short enough for every sample to take folded margins
            (5, 4, "reflect", "bf16", [1, 2, 3, 5], 3),
            # several chunk groups per row
            (5, 4, "reflect", "bf16", [1, 3, 5, 700], 6),
            (2, 3, "replicate", "bf16", [1, 2, 11, 300], 3),
            (7, 5, "reflect", "bf16", [1, 33, 6, 21], 2),
            (2, 7, "reflect", "bf16", [1, 3, 15, 30], 4),
            (3, 2, "replicate", "f16", [1, 4, 2, 9], 70),
            # 8 width phases and several output steps
            (8, 3, "zero", "bf16", [1, 4, 10, 100], 70),
            (4, 7, "reflect", "f16", [1, 9, 17, 270], 20),
            # q_w > 8: the classes are stored without the LDS row tile
            (2, 11, "reflect", "bf16", [1, 2, 23, 50], 3)]):
        if ALL or i < 4:
            cases.append({"mode": "bwd", "p": p, "q": q, "method": "mix4", "pad": pad, "dtype": dt, "shape": shape,
                          "cout": cout})
    _run(cases)


def test_grids_anisotropic_degenerate():
    _run([{"p": 3, "q": 2, "pw": 4, "qw": 5, "method": "bicubic", "pad": "zero", "shape": [1, 1, 19, 80]},
          {"p": 3, "q": 2, "method": "bilinear", "pad": "reflect", "grid": "paper", "shape": [1, 1, 12, 40]},
          {"p": 5, "q": 4, "method": "nearest", "pad": "replicate", "grid": "asym", "shape": [1, 1, 12, 40]},
          {"p": 3, "q": 2, "method": "bicubic", "pad": "reflect", "shape": [2, 1, 1, 1]},
          {"p": 2, "q": 3, "method": "bicubic", "pad": "reflect", "shape": [1, 1, 2, 1]},
          {"p": 8, "q": 1, "method": "bilinear", "pad": "zero", "shape": [1, 1, 3, 5]}])


@pytest.mark.parametrize("pq", [(3, 4), (3, 2), (5, 4), (2, 11)])
def test_learned_depthwise(pq):
    p, q = pq
    # widths 75 and 300: one ragged strip, or several (two column groups per lane where the output is wider than 64)
    _run([{"p": p, "q": q, "method": "dw4", "pad": pad, "shape": shape}
          for pad in ["zero", "replicate", "reflect"] for shape in ([2, 3, 21, 75], [1, 2, 9, 300])])


def test_backward_fixed_methods():
    cases = []
    for (p, q) in [(3, 2), (2, 3), (3, 4), (27, 11), (2, 11), (1, 1), (4, 1)]:
        for m in ["nearest", "bilinear", "bicubic"]:
            for pad in ["zero", "replicate", "reflect"]:
                cases.append({"mode": "bwd", "p": p, "q": q, "method": m, "pad": pad, "shape": [1, 2, 13, 70]})
    _run(cases)


def test_backward_learned_and_edges():
    cases = []
    for (p, q) in [(3, 4), (3, 2), (5, 4), (2, 11)]:
        for pad in ["zero", "replicate", "reflect"]:
            cases.append({"mode": "bwd", "p": p, "q": q, "method": "dw4", "pad": pad, "shape": [2, 3, 21, 75]})
    cases += [{"mode": "bwd", "p": 3, "q": 2, "method": "bicubic", "pad": "reflect", "shape": [1, 1, 1, 1]},
              {"mode": "bwd", "p": 3, "q": 2, "method": "dw4", "pad": "reflect", "shape": [1, 1, 2, 3]},
              {"mode": "bwd", "p": 3, "q": 2, "method": "bicubic", "pad": "replicate", "dtype": "bf16",
               "shape": [1, 2, 9, 40]},
              {"mode": "bwd", "p": 3, "q": 4, "method": "dw4", "pad": "zero", "dtype": "bf16", "shape": [2, 2, 16, 40]},
              # one gradient at a time (dw alone: the one-pass kernel without
              # its input-gradient part; dx alone: the gather kernel); rows
              # wider than a workgroup
              {"mode": "bwd", "p": 3, "q": 4, "method": "dw4", "pad": "reflect", "parts": "dw", "shape": [1, 2, 37, 75]},
              {"mode": "bwd", "p": 5, "q": 4, "method": "dw4", "pad": "replicate", "parts": "dx",
               "shape": [1, 2, 19, 50]},
              {"mode": "bwd", "p": 2, "q": 3, "method": "dw4", "pad": "reflect", "shape": [1, 1, 26, 600]},
              {"mode": "bwd", "p": 3, "q": 2, "pw": 4, "qw": 5, "method": "bicubic", "pad": "zero",
               "shape": [1, 1, 11, 30]}]
    _run(cases)


def test_channel_mixing_mfma():
    cases = []
    for dt in ["bf16", "f16"]:
        for (p, q, pad) in [(5, 4, "reflect"), (3, 2, "zero"), (2, 3, "replicate"), (7, 5, "reflect")]:
            cases.append({"p": p, "q": q, "method": "mix4", "pad": pad, "dtype": dt, "shape": [1, 6, 13, 40],
                          "cout": 5})
    cases.append({"p": 5, "q": 4, "method": "mix4", "pad": "zero", "dtype": "bf16", "shape": [2, 4, 9, 150],
                  "cout": 70})
    # large q (only the tapped rows and columns are staged) and an odd channel count
    cases.append({"p": 2, "q": 7, "method": "mix4", "pad": "reflect", "dtype": "bf16", "shape": [1, 5, 30, 60],
                  "cout": 3})
    cases.append({"p": 9, "q": 8, "method": "mix4", "pad": "replicate", "dtype": "f16", "shape": [1, 3, 20, 75],
                  "cout": 4})
    # a second width-phase group that starts at an odd column (and has one phase)
    cases.append({"p": 6, "q": 5, "method": "mix4", "pad": "reflect", "dtype": "bf16", "shape": [1, 9, 12, 170],
                  "cout": 3})
    _run(cases)


def test_channel_mixing_fp32():
    # FP32 storage on the FP32 matrix cores: ragged cell tiles, two output
    # tiles, large q (only the tapped columns staged), several phase groups
    _run([{"p": 5, "q": 4, "method": "mix4", "pad": "zero", "dtype": "f32", "shape": [1, 2, 8, 8], "cout": 2},
          {"p": 5, "q": 4, "method": "mix4", "pad": "reflect", "dtype": "f32", "shape": [2, 6, 13, 70],
           "cout": 70},
          {"p": 9, "q": 8, "method": "mix4", "pad": "replicate", "dtype": "f32", "shape": [1, 3, 20, 75],
           "cout": 4}] +
         ([{"p": 2, "q": 7, "method": "mix4", "pad": "reflect", "dtype": "f32", "shape": [1, 5, 30, 60], "cout": 3},
           {"p": 3, "q": 2, "method": "mix4", "pad": "zero", "dtype": "f32", "shape": [1, 9, 7, 35], "cout": 17}]
          if ALL else []))
