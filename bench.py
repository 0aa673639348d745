#!/usr/bin/env python3
"""FCFS rescale benchmark on one MI355X.

One step is one pass of the fused forward over the batched workload
N=32, C=3, 1024x1024 FP32 (seeded U[0,1) values), at every scale factor
{3/2, 2/3, 5/4, 4/5}, every method {nearest, bilinear, bicubic} and both
paddings {zero, reflect}: 24 launches. The reported value is the achieved
algorithmic HBM throughput of the step (GB/s): for each launch, the input rows
any tap reads (full rows) plus the output, summed, over the step's time.

Inputs rotate over copies whose total exceeds the 256 MB last-level cache
(MALL), so consecutive launches do not find their input there.

Printed as one JSON line, with:
  roofline     : the kernel instance with the most time in the step, its
                 algorithmic bytes per launch over its average launch time
                 (HIP events around this run's launches), against the 8 TB/s
                 HBM peak; beside it the same figure from the committed
                 rocprofv3 kernel trace of the current kernel source
                 (rocprof_avg_us, rocprof_frac), and traffic: measured HBM
                 bytes per launch from rocprofv3 counters (null when no
                 counters for the current source are committed);
  cpu_baseline : the FP64 oracle on the host cores over a bounded sample of
                 the same launches (all threads, and one thread), with the
                 other workloads' samples beside it;
  breakdown    : per-case times, GB/s and output Mpixel/s, the BF16 sweep
                 beside the FP32 one with its normwise difference from the
                 FP32 results;
  rows         : the other workloads (16x64x512^2 bicubic, channel mixing and
                 its backward, the learned depthwise layer, 1D and 3D, the
                 quality report, serving).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_BF16_TFLOPS = 2500.0
MFMA_PEAK_F32_TFLOPS = 157.3
FRACS = [(3, 2), (2, 3), (5, 4), (4, 5)]
METHODS = ["nearest", "bilinear", "bicubic"]
PADS = ["zero", "reflect"]
SHAPE = (32, 3, 1024, 1024)


def rows_touched(fc, plan, n_in: int, axis: int) -> int:
    """Input rows in [0, n_in) that some tap of some output reads (height axis
    of the isotropic plans benchmarked here)."""
    p, q, T = plan.p_red, plan.q_red, plan.taps
    cells = (n_in + q - 1) // q
    hit = np.zeros(n_in + 64, dtype=bool)
    base = np.arange(cells) * q
    for j in range(p):
        off = fc.fcfs_plan_taps(plan.handle, axis, j)[0]
        for t in range(T):
            idx = base + off + t
            idx = idx[(idx >= 0) & (idx < n_in)]
            hit[idx] = True
    return int(hit[:n_in].sum())


def case_bytes(fc, plan, shape, esize: int) -> int:
    n, c, h, w = shape
    ho, wo = plan.output_size(h, w)
    return n * c * (rows_touched(fc, plan, h, 0) * w + ho * wo) * esize


def source_hash() -> str:
    """Hash of the FP32 forward kernel's sources: the kernel, its launch
    planning and the argument structures it reads (counters taken for other
    sources are not used)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2203_10670_amd", "csrc")
    for f in ("fwd_kernel.h", "fwd_f32.hip", "fwd_plan.cpp"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(csrc, "fcfs_internal.h"), "rb") as fh:
        text = fh.read()
    h.update(text[text.index(b"struct AxisTable"):text.index(b"struct BwdArgs")])
    return h.hexdigest()[:16]


MIX_SOURCES = ("mix4_cl.h", "mix4_kernel.h", "mix4.hip", "mix4_f32.hip", "bwd_mix.h", "bwd_mix.hip")


def mix_source_hash() -> str:
    """Hash of the channel-mixing kernels' sources (forward and backward)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2203_10670_amd", "csrc")
    for f in MIX_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def write_mfma(d):
    """MfmaUtil per channel-mixing kernel from a rocprofv3 --pmc MfmaUtil run
    of the mix4 row, into profiles/mix4_mfma.json keyed to their source."""
    out = {"source_hash": mix_source_hash(), "kernels": {}}
    per = {}
    for r in _counter_rows(d, "MfmaUtil"):
        name = r["Kernel_Name"]
        for key in ("mix4_cl_kernel", "mix4_f32_kernel", "mix4_kernel", "dx_mix_gemm", "dw_mix_gemm_kernel",
                    "dx_mix_kernel", "dw_mix_partial"):
            if key in name:
                per.setdefault(key, []).append(float(r["Counter_Value"]))
                break
    for k, v in per.items():
        out["kernels"][k] = {"mfma_util_pct": round(sum(v) / len(v), 2), "dispatches": len(v)}
    path = os.path.join(ROOT, "profiles", "mix4_mfma.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1, sort_keys=True))


def load_mfma():
    path = os.path.join(ROOT, "profiles", "mix4_mfma.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        d = json.load(f)
    return d.get("kernels", {}) if d.get("source_hash") == mix_source_hash() else {}


def load_traffic(kernel_id: int):
    path = os.path.join(ROOT, "profiles", "fwd_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash():
        return None
    e = d.get("kernels", {}).get(str(kernel_id))
    return None if e is None else e.get("bytes_per_launch")


def load_kernel_times(kernel_id: int):
    """Average launch time (us) of a forward kernel instance from the
    committed rocprofv3 kernel trace of the current source, or None."""
    path = os.path.join(ROOT, "profiles", "fwd_kernel_times.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash():
        return None
    e = d.get("kernels", {}).get(str(kernel_id))
    return None if e is None else e.get("avg_us")


def _timeit(fn, n):
    """Average microseconds of fn(i), i = 0..n-1, by HIP events on torch's
    current stream (the stream every launch here is enqueued on)."""
    import torch
    fn(0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(n):
        fn(i)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1000.0 / n


def _sets(nbytes_one: int) -> int:
    """Buffer sets to rotate so that their total exceeds twice the 256 MB
    last-level cache."""
    return max(1, min(8, -(-(512 << 20) // max(1, nbytes_one))))


def bicubic_dw4_init(p, q, C, seed):
    """Learned depthwise 4x4 taps initialised to the bicubic outer product
    (the plan's own taps) plus N(0, 0.01) noise, for every channel."""
    import paper_2203_10670_amd as fc
    import synth
    pl = fc.Plan(p, q, "bicubic", "zero")
    t = np.array([fc.fcfs_plan_taps(pl.handle, 0, j)[1] for j in range(pl.p_red)], dtype=np.float64)
    base = np.einsum("ia,jb->ijab", t, t)[None].repeat(C, axis=0)
    return (base + synth.normal(seed, base.shape, std=0.1)).astype(np.float32)


def row_c3_bicubic(reps: int):
    """16x64x512x512 N(0,1) (seed 4), bicubic 5/4, reflect: FP32 and BF16
    storage (one input set is 1.07 GB in FP32, 0.54 GB in BF16)."""
    import torch
    import paper_2203_10670_amd as fc
    import synth
    dev = torch.device("cuda:0")
    sp = torch.cuda.current_stream(dev).cuda_stream
    out = {}
    N, C, H, W = 16, 64, 512, 512
    x32 = torch.from_numpy(synth.normal(4, (N, C, H, W))).to(dev)
    pl = fc.Plan(5, 4, "bicubic", "reflect")
    ho, wo = pl.output_size(H, W)
    for name, xt, es in (("f32", x32, 4), ("bf16", x32.to(torch.bfloat16), 2)):
        y = torch.empty((N, C, ho, wo), dtype=xt.dtype, device=dev)
        code = fc.DTYPES[name]

        def run(i=0):
            st = fc.fcfs_forward(pl.handle, code, N, C, H, W, xt.data_ptr(), None, C, y.data_ptr(), sp)
            assert st == 0
        us = _timeit(run, reps)
        b = case_bytes(fc, pl, (N, C, H, W), es)
        out["bicubic_5_4_16x64x512_" + name] = {"us": round(us, 2), "bytes": b, "GBps": round(b / us / 1e3, 1),
                                                "Mpix_per_s": round(N * C * ho * wo / us, 1)}
        del y
    return out


def row_mix4(reps: int, backward: bool = True):
    """The channel-mixing layer on MFMA, 16x64x512^2 BF16 N(0,1) (seed 4),
    64 -> 64 channels, 5/4, weights N(0, 1/1024) (seed 5); its backward
    (input gradient, weight gradient), each the forward's flop count."""
    import torch
    import paper_2203_10670_amd as fc
    import synth
    dev = torch.device("cuda:0")
    sp = torch.cuda.current_stream(dev).cuda_stream
    out = {}
    N, C, H, W = 16, 64, 512, 512
    xb = torch.from_numpy(synth.normal(4, (N, C, H, W))).to(dev).to(torch.bfloat16)
    wm = torch.from_numpy(synth.normal(5, (5, 5, C, C, 4, 4), std=1 / 32)).to(dev).to(torch.bfloat16)
    plm = fc.Plan(5, 4, "mix4", "reflect")
    ho, wo = plm.output_size(H, W)
    ym = torch.empty((N, C, ho, wo), dtype=torch.bfloat16, device=dev)

    def runm(i=0):
        st = fc.fcfs_forward(plm.handle, 1, N, C, H, W, xb.data_ptr(), wm.data_ptr(), C, ym.data_ptr(), sp)
        assert st == 0
    us = _timeit(runm, max(3, reps // 2))
    flops = 2.0 * N * (ho // 5) * (wo // 5) * 25 * C * C * 16
    util = load_mfma()   # MfmaUtil of the committed counter run of these sources, if any

    def counter(key):
        e = util.get(key)
        return None if e is None else e["mfma_util_pct"]
    out["mix4_5_4_16x64x512_bf16"] = {"us": round(us, 2), "flop": flops,
                                      "TFLOPs": round(flops / us / 1e6, 1),
                                      "mfma_frac": round(flops / us / 1e6 / MFMA_PEAK_BF16_TFLOPS, 4),
                                      "mfma_util_counter_pct": counter("mix4_cl_kernel") or counter("mix4_kernel"),
                                      "Mpix_per_s": round(N * C * ho * wo / us, 1)}
    # FP32 storage on the FP32 matrix cores, same layer
    x32 = xb.float()
    w32 = wm.float()
    y32 = torch.empty((N, C, ho, wo), dtype=torch.float32, device=dev)

    def runf(i=0):
        st = fc.fcfs_forward(plm.handle, 0, N, C, H, W, x32.data_ptr(), w32.data_ptr(), C, y32.data_ptr(), sp)
        assert st == 0
    uf = _timeit(runf, max(2, reps // 4))
    out["mix4_5_4_16x64x512_f32"] = {"us": round(uf, 2), "flop": flops, "TFLOPs": round(flops / uf / 1e6, 1),
                                     "mfma_frac": round(flops / uf / 1e6 / MFMA_PEAK_F32_TFLOPS, 4),
                                     "mfma_util_counter_pct": counter("mix4_f32_kernel"),
                                     "Mpix_per_s": round(N * C * ho * wo / uf, 1)}
    del x32, w32, y32
    if backward:
        dym = ym
        dxm = torch.empty_like(xb)
        dwm = torch.empty(wm.shape, dtype=torch.float32, device=dev)
        wsb = fc.fcfs_backward_workspace(plm.handle, 1, N, C, H, W, C)
        wsm = torch.empty(max(1, wsb), dtype=torch.uint8, device=dev)

        def runbx(i=0):
            st = fc.fcfs_backward(plm.handle, 1, N, C, H, W, None, wm.data_ptr(), C, dym.data_ptr(), dxm.data_ptr(),
                                  None, wsm.data_ptr(), wsb, sp)
            assert st == 0

        def runbw(i=0):
            st = fc.fcfs_backward(plm.handle, 1, N, C, H, W, xb.data_ptr(), None, C, dym.data_ptr(), None,
                                  dwm.data_ptr(), wsm.data_ptr(), wsb, sp)
            assert st == 0
        def runbb(i=0):
            st = fc.fcfs_backward(plm.handle, 1, N, C, H, W, xb.data_ptr(), wm.data_ptr(), C, dym.data_ptr(),
                                  dxm.data_ptr(), dwm.data_ptr(), wsm.data_ptr(), wsb, sp)
            assert st == 0
        ux = _timeit(runbx, max(2, reps // 4))
        uw = _timeit(runbw, max(2, reps // 4))
        ub = _timeit(runbb, max(2, reps // 4))
        # whole passes (layout passes, GEMM, fold or reduction); the counter
        # figures are the GEMM kernels' own
        out["mix4_5_4_16x64x512_bf16_backward"] = {
            "dx_us": round(ux, 2), "dx_TFLOPs": round(flops / ux / 1e6, 1),
            "dx_mfma_frac": round(flops / ux / 1e6 / MFMA_PEAK_BF16_TFLOPS, 4),
            "dx_mfma_util_counter_pct": counter("dx_mix_gemm") or counter("dx_mix_kernel"),
            "dw_us": round(uw, 2), "dw_TFLOPs": round(flops / uw / 1e6, 1),
            "dw_mfma_frac": round(flops / uw / 1e6 / MFMA_PEAK_BF16_TFLOPS, 4),
            "dw_mfma_util_counter_pct": counter("dw_mix_gemm_kernel") or counter("dw_mix_partial"),
            "dx_dw_us": round(ub, 2), "dx_dw_TFLOPs": round(2 * flops / ub / 1e6, 1)}
        del dxm, dwm, wsm
    del xb, wm, ym
    torch.cuda.empty_cache()
    return out


def row_dw4(reps: int):
    """The learned depthwise layer 8x64x256^2 N(0,1) at 3/4 (taps: bicubic
    plus N(0, 0.01), seed 7; dY N(0,1)): forward and backward (input and
    weight gradients), FP32 and BF16, rotating buffer sets past the 256 MB
    last-level cache."""
    import torch
    import paper_2203_10670_amd as fc
    import synth
    dev = torch.device("cuda:0")
    sp = torch.cuda.current_stream(dev).cuda_stream
    out = {}
    N, C, H, W, p, q = 8, 64, 256, 256, 3, 4
    pld = fc.Plan(p, q, "dw4", "reflect")
    ho, wo = pld.output_size(H, W)
    wd = torch.from_numpy(bicubic_dw4_init(p, q, C, 7)).to(dev)
    for name, es in (("f32", 4), ("bf16", 2)):
        td = torch.float32 if name == "f32" else torch.bfloat16
        code = fc.DTYPES[name]
        k_sets = _sets((2 * N * C * H * W + 2 * N * C * ho * wo) * es)
        sets = []
        for k in range(k_sets):
            xt = torch.from_numpy(synth.normal(6 + 10 * k, (N, C, H, W))).to(dev).to(td)
            dyt = torch.from_numpy(synth.normal(8 + 10 * k, (N, C, ho, wo))).to(dev).to(td)
            sets.append((xt, dyt, torch.empty((N, C, ho, wo), dtype=td, device=dev),
                         torch.empty((N, C, H, W), dtype=td, device=dev)))
        dw = torch.empty_like(wd)
        wsb = fc.fcfs_backward_workspace(pld.handle, code, N, C, H, W, C)
        ws = torch.empty(max(1, wsb), dtype=torch.uint8, device=dev)

        def fwd(i=0):
            xt, _, yt, _ = sets[i % k_sets]
            assert fc.fcfs_forward(pld.handle, code, N, C, H, W, xt.data_ptr(), wd.data_ptr(), C, yt.data_ptr(), sp) == 0

        def bwd(i=0):
            xt, dyt, _, dxt = sets[i % k_sets]
            assert fc.fcfs_backward(pld.handle, code, N, C, H, W, xt.data_ptr(), wd.data_ptr(), C, dyt.data_ptr(),
                                    dxt.data_ptr(), dw.data_ptr(), ws.data_ptr(), wsb, sp) == 0
        uf = _timeit(fwd, reps)
        ub = _timeit(bwd, reps)
        bf = (N * C * H * W + N * C * ho * wo) * es
        bb = (N * C * ho * wo + 2 * N * C * H * W) * es
        out["dw4_3_4_8x64x256_" + name] = {"fwd_us": round(uf, 2), "fwd_GBps": round(bf / uf / 1e3, 1),
                                           "bwd_us": round(ub, 2), "bwd_GBps": round(bb / ub / 1e3, 1),
                                           "fwd_bytes": bf, "bwd_bytes": bb, "buffer_sets": k_sets}
        del sets, ws
        torch.cuda.empty_cache()
    return out


def row_nd(reps: int):
    """1D and 3D FCFS, FP32 bicubic reflect: 16 x 2 signals of 2^20 samples
    at 3/2 (one pass), and a 2 x 1 x 128 x 256 x 256 volume at 3/2 on every
    axis (two passes through a workspace), each over buffer sets whose total
    exceeds the 256 MB last-level cache. GB/s counts the input and output
    once; the 3D figure with the intermediate's write and read is given too."""
    import torch
    import paper_2203_10670_amd as fc
    import synth
    dev = torch.device("cuda:0")
    sp = torch.cuda.current_stream(dev).cuda_stream
    out = {}
    N, C, L = 16, 2, 1 << 20
    pl1 = fc.Plan(1, 1, "bicubic", "reflect", pw=3, qw=2)
    lo = pl1.output_size(1, L)[1]
    b = (N * C * L + N * C * lo) * 4
    k1 = _sets(b)
    s1 = [(torch.from_numpy(synth.normal(40 + k, (N, C, L))).to(dev), torch.empty((N, C, lo), device=dev))
          for k in range(k1)]

    def run1(i=0):
        x1, y1 = s1[i % k1]
        assert fc.fcfs_forward_1d(pl1.handle, 0, N, C, L, x1.data_ptr(), y1.data_ptr(), sp) == 0
    us = _timeit(run1, reps)
    out["nd_1d_3_2_16x2x1M_f32"] = {"us": round(us, 2), "bytes": b, "GBps": round(b / us / 1e3, 1),
                                    "buffer_sets": k1}
    del s1
    n, c, d, h, w = 2, 1, 128, 256, 256
    pld = fc.Plan(3, 2, "bicubic", "reflect", pw=1, qw=1)
    plhw = fc.Plan(3, 2, "bicubic", "reflect")
    do = pld.output_size(d, 1)[0]
    ho, wo = plhw.output_size(h, w)
    wsb = fc.fcfs_forward_3d_workspace(pld.handle, plhw.handle, 0, n, c, d, h, w)
    b = (n * c * d * h * w + n * c * do * ho * wo) * 4
    k3 = _sets(b + wsb)
    s3 = [(torch.from_numpy(synth.normal(41 + k, (n, c, d, h, w))).to(dev),
           torch.empty((n, c, do, ho, wo), device=dev), torch.empty(wsb, dtype=torch.uint8, device=dev))
          for k in range(k3)]

    def run3(i=0):
        x3, y3, ws = s3[i % k3]
        assert fc.fcfs_forward_3d(pld.handle, plhw.handle, 0, n, c, d, h, w, x3.data_ptr(), y3.data_ptr(),
                                  ws.data_ptr(), wsb, sp) == 0
    us = _timeit(run3, reps)
    out["nd_3d_3_2_2x1x128x256x256_f32"] = {"us": round(us, 2), "bytes": b, "GBps": round(b / us / 1e3, 1),
                                            "GBps_with_intermediate": round((b + 2 * wsb) / us / 1e3, 1),
                                            "buffer_sets": k3}
    del s3
    torch.cuda.empty_cache()
    return out


def measure_quality():
    """PSNR / SSIM of the FCFS output against torch's interpolate (same
    half-pixel grid, edge clamping) on the smooth synthetic set S
    (4 x 3 x 512^2), replicate padding, for up- and down-scaling factors
    including the paper's 27/11 and 2/11."""
    import torch
    import paper_2203_10670_amd as fc
    from paper_2203_10670_amd import quality
    import synth
    x = torch.from_numpy(synth.smooth(3, (4, 3, 512, 512))).cuda()
    rows = {}
    for p, q in ((3, 2), (5, 4), (2, 1), (27, 11), (2, 3), (4, 5), (1, 2), (2, 11)):
        for m in ("nearest", "bilinear", "bicubic"):
            y = fc.resize(x, p, q, m, "replicate")
            ps, ss = quality.compare_with_framework(y, x, p, q, m)
            rows["%d/%d %s" % (p, q, m)] = {"psnr_db": None if ps == float("inf") else round(ps, 2),
                                            "ssim": round(ss, 6)}
    return rows


def measure_serving(count: int, rhos=(0.25, 0.5, 0.8, 0.95), chunk_waves=None):
    """The serving loop on a seeded request stream: C=3, H and W uniform in
    64..2048, p and q uniform in 1..8, method uniform, FP32 or BF16 by seed,
    inputs generated on the device from each request's seed, outputs freed on
    completion, 64 GB arena, 256 slots. Capacity is the throughput when every
    request arrives at once; then Poisson arrivals at rho x capacity, served
    with continuous batching and with one launch per request."""
    import paper_2203_10670_amd as fc
    import synth
    meta = synth.request_stream(9, count, rate_per_s=0.0)
    reqs = [fc.fcfs_request(r.p, r.q, r.method, r.pad, r.dtype, 1, r.c, r.h, r.w, None, r.seed, None) for r in meta]
    srv = fc.Server(0, 64 << 30, 256)
    fc.fcfs_server_config(srv.handle, fc.FCFS_SERVER_DISCARD_OUTPUTS, 1)
    if chunk_waves is not None:
        fc.fcfs_server_config(srv.handle, fc.FCFS_SERVER_CHUNK_WAVES, chunk_waves)

    def run(arrivals, max_batch, subset=None):
        rq = reqs if subset is None else reqs[:subset]
        fc.fcfs_server_config(srv.handle, fc.FCFS_SERVER_MAX_BATCH, max_batch)
        fc.fcfs_server_reset_stats(srv.handle)
        st, tickets = fc.fcfs_server_replay(srv.handle, rq, arrivals[:len(rq)])
        if st != 0:
            raise fc.FcfsError(st, "fcfs_server_replay")
        bad = 0
        for t in tickets:
            r = srv.wait(t)
            bad += r.status != 0
            srv.release(t)
        p50, p99, rps, gbps = srv.stats()
        return {"p50_us": round(p50, 1), "p99_us": round(p99, 1), "req_per_s": round(rps, 1),
                "GBps": round(gbps, 1), "failed": int(bad)}

    run([0.0] * 200, 0, subset=200)   # warm up
    cap = run([0.0] * count, 0)
    cap1 = run([0.0] * count, 1)
    loads = []
    rng = np.random.default_rng(10)
    for rho in rhos:
        rate = rho * cap["req_per_s"]
        gaps = rng.exponential(1e6 / rate, size=count)
        arr = list(np.cumsum(gaps) - gaps[0])
        loads.append({"rho": rho, "offered_req_per_s": round(rate, 1),
                      "batched": run(arr, 0), "one_launch_per_request": run(arr, 1)})
    srv.close()
    return {"requests": count, "capacity_batched": cap, "capacity_one_launch_per_request": cap1,
            "loads": loads}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cases, x_np, target_planes: int, one_thread_planes: int):
    """The FP64 oracle timed on the host: the step's 24 launches on a sample of
    planes with every thread and with one thread, then bounded samples of the
    other workloads (all threads): the 1x1x64^2 cases, the 16x64x512^2 5/4
    bicubic layer, and the 8x64x256^2 learned depthwise layer's forward and
    backward. GB/s counts the same algorithmic bytes as the GPU figures."""
    import oracle
    import synth
    threads = oracle.threads()
    planes_all = x_np.reshape(-1, SHAPE[2], SHAPE[3])
    nplanes = SHAPE[0] * SHAPE[1]

    def sweep(k):
        planes = planes_all[:k][:, None].astype(np.float64)
        total_bytes, pix = 0, 0
        t0 = time.perf_counter()
        for cs in cases:
            y = oracle.forward(planes, cs["p"], cs["q"], cs["method"], cs["pad"])
            total_bytes += cs["bytes"] * k // nplanes
            pix += y.size
        return total_bytes, pix, time.perf_counter() - t0

    k = max(1, min(nplanes, target_planes or 6 * threads))
    b_all, pix_all, dt_all = sweep(k)
    k1 = max(1, min(nplanes, one_thread_planes))
    oracle.set_threads(1)
    try:
        b_one, pix_one, dt_one = sweep(k1)
    finally:
        oracle.set_threads(threads)
    other = {}
    # 1x1x64^2 U[0,1) (seed 1), replicate, 3/2 and 2/3, every method
    x1 = synth.uniform(1, (1, 1, 64, 64)).astype(np.float64)
    t0 = time.perf_counter()
    reps = 20
    for _ in range(reps):
        for (p, q) in ((3, 2), (2, 3)):
            for m in METHODS:
                oracle.forward(x1, p, q, m, "replicate")
    other["plain_1x1x64x64_6_cases_us"] = round((time.perf_counter() - t0) / reps * 1e6, 1)
    # 16x64x512^2 5/4 bicubic: 32 of the 1024 planes
    xs = synth.normal(4, (1, 32, 512, 512)).astype(np.float64)
    t0 = time.perf_counter()
    y = oracle.forward(xs, 5, 4, "bicubic", "reflect")
    dt = time.perf_counter() - t0
    b = 32 * (512 * 512 + 640 * 640) * 4
    other["bicubic_5_4_16x64x512"] = {"planes": 32, "s": round(dt, 3), "GBps": round(b / dt / 1e9, 4),
                                      "Mpix_per_s": round(y.size / dt / 1e6, 2)}
    # 8x64x256^2 3/4 learned depthwise: one batch entry (64 planes)
    xd = synth.normal(6, (1, 64, 256, 256)).astype(np.float64)
    wd = bicubic_dw4_init(3, 4, 64, 7).astype(np.float64)
    dyd = synth.normal(8, (1, 64, 192, 192)).astype(np.float64)
    t0 = time.perf_counter()
    y = oracle.forward(xd, 3, 4, "dw4", "reflect", weight=wd)
    dtf = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.backward(dyd, xd.shape, 3, 4, "dw4", "reflect", x=xd, weight=wd, need_dw=True)
    dtb = time.perf_counter() - t0
    bf = 64 * (256 * 256 + 192 * 192) * 4
    bb = 64 * (192 * 192 + 2 * 256 * 256) * 4
    other["dw4_3_4_8x64x256"] = {"planes": 64, "fwd_s": round(dtf, 3), "fwd_GBps": round(bf / dtf / 1e9, 4),
                                 "bwd_s": round(dtb, 3), "bwd_GBps": round(bb / dtb / 1e9, 4)}
    return {"value": round(b_all / dt_all / 1e9, 4), "unit": "GB/s", "cores": min(threads, k),
            "kind": "oracle",
            "sample": "FP64 oracle, %d of %d planes of each of the %d FP32 launches of a step "
                      "(%.1f s wall, %d threads)" % (k, nplanes, len(cases), dt_all, min(threads, k)),
            "Mpix_per_s": round(pix_all / dt_all / 1e6, 2),
            "one_thread": {"value": round(b_one / dt_one / 1e9, 4), "unit": "GB/s", "cores": 1,
                           "Mpix_per_s": round(pix_one / dt_one / 1e6, 3),
                           "sample": "%d planes of each launch (%.1f s wall)" % (k1, dt_one)},
            "cpu_model": _cpu_model(), "host_threads": os.cpu_count(),
            "other_workloads": other}


def summarize(d):
    """Per-kernel summary of rocprofv3 CSV output (kernel stats, and FETCH_SIZE /
    WRITE_SIZE counters per dispatch when present), printed as text."""
    import csv
    import glob
    stats = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    for f in stats:
        print("# kernel stats:", os.path.relpath(f, d))
        with open(f) as fh:
            rows = list(csv.DictReader(fh))
        rows.sort(key=lambda r: -float(r.get("TotalDurationNs", 0)))
        print("%-100s %6s %12s %12s %6s" % ("kernel", "calls", "avg_us", "total_us", "pct"))
        for r in rows:
            name = r["Name"]
            short = name if len(name) <= 100 else name[:97] + "..."
            print("%-100s %6s %12.2f %12.1f %6.2f" % (short, r["Calls"], float(r["AverageNs"]) / 1e3,
                                                       float(r["TotalDurationNs"]) / 1e3, float(r["Percentage"])))
    # overlap of consecutive batched serving launches (two streams): a launch
    # that starts before the previous one ends ran beside it
    for f in glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True):
        with open(f) as fh:
            ev = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in csv.DictReader(fh)
                        if "fwd_batch_kernel" in r["Kernel_Name"])
        if len(ev) < 2:
            continue
        over = [(a[1] - b[0]) for a, b in zip(ev, ev[1:]) if b[0] < a[1]]
        busy = sum(e - s_ for s_, e in ev)
        print("# serving overlap (%s): %d batched launches, %d start before the previous one ends; "
              "overlapped time %.1f us of %.1f us of kernel time (median overlap %.1f us)"
              % (os.path.relpath(f, d), len(ev), len(over), sum(over) / 1e3, busy / 1e3,
                 sorted(over)[len(over) // 2] / 1e3 if over else 0.0))
    ctr = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    for f in ctr:
        print("# counters:", os.path.relpath(f, d))
        agg = {}
        with open(f) as fh:
            for r in csv.DictReader(fh):
                key = (r["Kernel_Name"], r["Counter_Name"])
                a = agg.setdefault(key, [0.0, 0])
                a[0] += float(r["Counter_Value"])
                a[1] += 1
        print("%-100s %-30s %8s %18s" % ("kernel", "counter", "rows", "avg_per_dispatch"))
        for (k, c), (v, n) in sorted(agg.items()):
            short = k if len(k) <= 100 else k[:97] + "..."
            print("%-100s %-30s %8d %18.4g" % (short, c, n, v / n))


def _counter_rows(d, counter):
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            rows += [r for r in csv.DictReader(fh) if r["Counter_Name"] == counter]
    return rows


def _kernel_id(name):
    """Instance id of a forward kernel name fcfs_fwd_kernel<DT, T, KC, L, LEARNED,
    PAIR, TV> (as fcfs_forward_config reports it; T width taps, TV height taps)."""
    import re
    m = re.search(r"fcfs_fwd_kernel<(\d+), (\d+), (\d+), (\d+), (true|false)(?:, (true|false))?(?:, (\d+))?>",
                  name)
    if not m:
        return None
    dt, t, kc, sl = (int(m.group(i)) for i in range(1, 5))
    tv = int(m.group(7)) if m.group(7) else t
    return (dt * 1000 + max(t, tv) * 100 + kc * 10 + sl + (10000 if m.group(5) == "true" else 0) +
            (50000 if m.group(6) == "true" else 0) + (100000 if tv < t else 0) + (200000 if t < tv else 0))


def write_traffic(fetch_dir, write_dir):
    """HBM bytes per launch of each forward kernel instance from two counter
    runs: FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each scaled by what
    the same counter reads for a 1 GiB device copy (1 GiB read, 1 GiB
    written) in the same run."""
    out = {"source_hash": source_hash(), "kernels": {}}
    scale = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _counter_rows(d, counter)
        # the calibration dispatches: torch's neg kernel over 1 GiB (bench.py
        # --copy-calibration); runs taken with a device copy instead use the
        # largest copyBuffer dispatches (input uploads are copies too)
        copies = [float(r["Counter_Value"]) for r in rows if "neg_kernel" in r["Kernel_Name"]]
        if not copies:
            blits = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
            copies = [v for v in blits if v >= 0.9 * max(blits, default=0.0)]
        if not copies:
            raise SystemExit("no copy calibration dispatch in %s" % d)
        scale[counter] = (1 << 20) / (sum(copies) / len(copies))   # KiB of a 1 GiB copy / measured
        per = {}
        for r in rows:
            kid = _kernel_id(r["Kernel_Name"])
            if kid is None:
                continue
            per.setdefault(kid, []).append(float(r["Counter_Value"]))
        for kid, v in per.items():
            e = out["kernels"].setdefault(str(kid), {})
            e[counter + "_KiB_raw"] = sum(v) / len(v)
            e[counter + "_bytes"] = sum(v) / len(v) * 1024 * scale[counter]
            e["dispatches_" + counter] = len(v)
    for e in out["kernels"].values():
        if "FETCH_SIZE_bytes" in e and "WRITE_SIZE_bytes" in e:
            e["bytes_per_launch"] = int(e["FETCH_SIZE_bytes"] + e["WRITE_SIZE_bytes"])
    out["scale"] = scale
    path = os.path.join(ROOT, "profiles", "fwd_traffic.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1, sort_keys=True))


def write_kernel_times(d):
    """Average launch time of each forward kernel instance from a
    rocprofv3 --kernel-trace --stats run of this benchmark, into
    profiles/fwd_kernel_times.json keyed to the current kernel source."""
    import csv
    import glob
    out = {"source_hash": source_hash(), "kernels": {}}
    for f in glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                kid = _kernel_id(r["Name"])
                if kid is None:
                    continue
                out["kernels"][str(kid)] = {"avg_us": round(float(r["AverageNs"]) / 1e3, 3),
                                            "calls": int(r["Calls"])}
    path = os.path.join(ROOT, "profiles", "fwd_kernel_times.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1, sort_keys=True))


ROWS = ("c3", "mix4", "dw4", "nd", "quality", "serving")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--cpu-planes", type=int, default=0, help="planes per launch of the all-thread oracle sample")
    ap.add_argument("--cpu-planes-one-thread", type=int, default=6)
    ap.add_argument("--no-rows", action="store_true", help="skip the other workloads (mix4, learned layer, ...)")
    ap.add_argument("--rows", default=",".join(ROWS), help="which other workloads to run (comma list of %s)"
                    % ", ".join(ROWS))
    ap.add_argument("--no-sweep", action="store_true",
                    help="profiling only: skip the step sweep and print the rows' JSON (not a benchmark line)")
    ap.add_argument("--serve-requests", type=int, default=10000, help="requests of the serving run (0: skip)")
    ap.add_argument("--serve-chunk-waves", type=int, default=None,
                    help="most waves of one request per batch (0: no chunking; default: the server's)")
    ap.add_argument("--filter", default="", help="only cases whose name contains this text")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM counters)")
    ap.add_argument("--summarize", metavar="DIR", help="summarise rocprofv3 CSV output under DIR and exit")
    ap.add_argument("--traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn FETCH_SIZE / WRITE_SIZE counter runs (with --copy-calibration) into "
                         "profiles/fwd_traffic.json and exit")
    ap.add_argument("--mfma", metavar="DIR",
                    help="turn a rocprofv3 --pmc MfmaUtil run of the mix4 row into profiles/mix4_mfma.json and exit")
    ap.add_argument("--kernel-times", metavar="DIR",
                    help="turn a rocprofv3 kernel-trace run of the sweep into profiles/fwd_kernel_times.json "
                         "and exit")
    args = ap.parse_args()
    if args.summarize:
        summarize(args.summarize)
        return
    if args.traffic:
        write_traffic(*args.traffic)
        return
    if args.kernel_times:
        write_kernel_times(args.kernel_times)
        return
    if args.mfma:
        write_mfma(args.mfma)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the rescale path has no multi-GPU mode "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    rows_sel = [] if args.no_rows else [r for r in args.rows.split(",") if r]
    for r in rows_sel:
        if r not in ROWS:
            raise SystemExit("unknown row %r (choose from %s)" % (r, ", ".join(ROWS)))

    import torch
    import paper_2203_10670_amd as fc
    import synth

    dev = torch.device("cuda:0")
    stream_ptr = torch.cuda.current_stream(dev).cuda_stream

    def run_rows():
        reps = max(3, args.steps)
        rows = {}
        if "c3" in rows_sel:
            rows.update(row_c3_bicubic(reps))
        if "mix4" in rows_sel:
            rows.update(row_mix4(reps))
        if "dw4" in rows_sel:
            rows.update(row_dw4(reps))
        if "nd" in rows_sel:
            rows.update(row_nd(reps))
        if "quality" in rows_sel:
            rows["quality_vs_framework_resize"] = measure_quality()
        if "serving" in rows_sel and args.serve_requests > 0:
            rows["serving"] = measure_serving(args.serve_requests, chunk_waves=args.serve_chunk_waves)
        return rows

    if args.no_sweep:
        print(json.dumps({"rows": run_rows()}), flush=True)
        return

    x_np = synth.uniform(2, SHAPE)
    x32 = torch.from_numpy(x_np).to(dev)
    # input copies rotated launch by launch, past the 256 MB last-level cache
    xs32 = [x32] + [x32.clone() for _ in range(_sets(x32.numel() * 4) - 1)]

    def make_cases(dtype_name, xs, esize):
        cases = []
        for (p, q) in FRACS:
            for m in METHODS:
                for pad in PADS:
                    pl = fc.Plan(p, q, m, pad)
                    ho, wo = pl.output_size(SHAPE[2], SHAPE[3])
                    y = torch.empty((SHAPE[0], SHAPE[1], ho, wo), dtype=xs[0].dtype, device=dev)
                    code = fc.DTYPES[dtype_name]
                    kid = fc.fcfs_forward_config(pl.handle, code, SHAPE[0], SHAPE[1], SHAPE[2], SHAPE[3])[0]
                    cases.append({"p": p, "q": q, "method": m, "pad": pad, "plan": pl, "y": y, "xs": xs,
                                  "code": code, "kernel_id": kid, "dtype": dtype_name,
                                  "pixels": SHAPE[0] * SHAPE[1] * ho * wo,
                                  "bytes": case_bytes(fc, pl, SHAPE, esize)})
        return cases

    def launch(cs, i):
        x = cs["xs"][i % len(cs["xs"])]
        st = fc.fcfs_forward(cs["plan"].handle, cs["code"], SHAPE[0], SHAPE[1], SHAPE[2], SHAPE[3],
                             x.data_ptr(), None, SHAPE[1], cs["y"].data_ptr(), stream_ptr)
        if st != 0:
            raise fc.FcfsError(st, "fcfs_forward")

    def timed_sweep(cases, steps, warmup):
        i = 0
        for _ in range(warmup):
            for cs in cases:
                launch(cs, i)
                i += 1
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            for cs in cases:
                launch(cs, i)
                i += 1
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    def per_case(cases, reps):
        return [(cs, _timeit(lambda i, cs=cs: launch(cs, i), reps)) for cs in cases]

    if args.copy_calibration:
        # 1 GiB of FP32 read and 1 GiB written by one uniquely named kernel
        # (torch's elementwise negation), the reference the counter runs scale by
        n = 1 << 28
        a_ = torch.rand(n, device=dev)
        b_ = torch.empty_like(a_)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            torch.neg(a_, out=b_)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        print("copy 1 GiB: %.3f ms, %.1f GB/s (read + write)" % (ms, 2 * 4 * n / (ms * 1e-3) / 1e9),
              file=sys.stderr, flush=True)
        del a_, b_

    f32 = make_cases("f32", xs32, 4)
    f32_meta = [{k: c[k] for k in ("p", "q", "method", "pad", "bytes")} for c in f32]
    if args.filter:
        f32 = [c for c in f32 if args.filter in "%d/%d %s %s" % (c["p"], c["q"], c["method"], c["pad"])]
        f32_meta = [c for c in f32_meta if args.filter in "%d/%d %s %s" % (c["p"], c["q"], c["method"], c["pad"])]
    ms_step = timed_sweep(f32, args.steps, args.warmup)
    step_bytes = sum(c["bytes"] for c in f32)
    step_pixels = sum(c["pixels"] for c in f32)
    value = step_bytes / (ms_step * 1e-3) / 1e9
    print("step: %.3f ms, %.1f GB/s" % (ms_step, value), file=sys.stderr, flush=True)

    reps = max(3, args.steps)
    pc = per_case(f32, reps)
    groups = {}
    for cs, us in pc:
        g = groups.setdefault(cs["kernel_id"], {"us": 0.0, "bytes": 0, "n": 0})
        g["us"] += us
        g["bytes"] += cs["bytes"]
        g["n"] += 1
    dom = max(groups.items(), key=lambda kv: kv[1]["us"])
    kid, g = dom
    avg_us = g["us"] / g["n"]
    bytes_per_launch = g["bytes"] / g["n"]
    achieved = bytes_per_launch / (avg_us * 1e-6) / 1e9
    rp_us = load_kernel_times(kid)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": load_traffic(kid),
                "kernel_id": kid, "launches": g["n"], "avg_us": round(avg_us, 2),
                "avg_us_source": "HIP events around this run's launches",
                "rocprof_avg_us": rp_us,
                "rocprof_frac": None if rp_us is None else round(bytes_per_launch / (rp_us * 1e-6) / 1e9 /
                                                                 HBM_PEAK_GBS, 4),
                "bytes_per_launch": int(bytes_per_launch)}

    def case_row(c, us):
        return {"case": "%d/%d %s %s" % (c["p"], c["q"], c["method"], c["pad"]), "us": round(us, 2),
                "GBps": round(c["bytes"] / (us * 1e-6) / 1e9, 1), "Mpix_per_s": round(c["pixels"] / us, 1),
                "kernel_id": c["kernel_id"]}

    breakdown = {"f32": [case_row(c, us) for c, us in pc], "f32_input_sets": len(xs32)}
    bf16_value = None
    if not args.no_bf16 and not args.filter:
        xbf = x32.to(torch.bfloat16)
        xsbf = [xbf] + [xbf.clone() for _ in range(_sets(xbf.numel() * 2) - 1)]
        bf = make_cases("bf16", xsbf, 2)
        ms_bf = timed_sweep(bf, args.steps, args.warmup)
        bf16_value = sum(c["bytes"] for c in bf) / (ms_bf * 1e-3) / 1e9
        pcb = per_case(bf, reps)
        breakdown["bf16"] = [case_row(c, us) for c, us in pcb]
        breakdown["bf16_input_sets"] = len(xsbf)
        breakdown["bf16_step_ms"] = round(ms_bf, 4)
        breakdown["bf16_GBps"] = round(bf16_value, 1)
        # end-to-end difference of BF16 storage (input rounding, arithmetic,
        # rounded store) from the FP32 results on the same FP32 input
        worst = 0.0
        for cb, cf in zip(bf, f32):
            yf = cf["y"]
            d = (cb["y"].float() - yf).abs().max().item() / max(yf.abs().max().item(), 1e-30)
            worst = max(worst, d)
        breakdown["bf16_normwise_diff_from_f32"] = float("%.4g" % worst)
        del bf, pcb, xsbf, xbf
    torch.cuda.synchronize()

    rows = None
    if rows_sel and not args.filter:
        del f32, pc, x32, xs32
        torch.cuda.empty_cache()
        rows = run_rows()

    cpu = None
    if not args.no_cpu_baseline and not args.filter:
        cpu = cpu_baseline(f32_meta, x_np, args.cpu_planes, args.cpu_planes_one_thread)

    line = {
        "metric": "resample output GB/s vs HBM peak (FP32, BF16); served p50/p99 latency",
        "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "FCFS forward sweep: N=32 C=3 1024x1024 FP32 U[0,1); scales 3/2 2/3 5/4 4/5; "
                               "nearest bilinear bicubic; zero and reflect padding (24 launches per step)",
                   "batch": SHAPE[0], "channels": SHAPE[1], "height": SHAPE[2], "width": SHAPE[3],
                   "launches_per_step": len(f32_meta), "bytes_per_step": step_bytes},
        "output_Mpix_per_s": round(step_pixels / (ms_step * 1e3), 1),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "bf16_value": None if bf16_value is None else round(bf16_value, 1),
        "breakdown": breakdown,
        "rows": rows,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
