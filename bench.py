#!/usr/bin/env python3
"""FCFS rescale benchmark on one MI355X.

One step is one pass of the fused forward over the batched workload
N=32, C=3, 1024x1024 FP32 (seeded U[0,1) values), at every scale factor
{3/2, 2/3, 5/4, 4/5}, every method {nearest, bilinear, bicubic} and both
paddings {zero, reflect}: 24 launches. The reported value is the achieved
algorithmic HBM throughput of the step (GB/s): for each launch, the input rows
any tap reads (full rows) plus the output, summed, over the step's time.

Printed as one JSON line, with:
  roofline     : the kernel instance with the most time in the step, its
                 algorithmic bytes per launch over its average launch time,
                 against the 8 TB/s HBM peak (traffic: measured HBM bytes per
                 launch from rocprofv3 counters when a summary for the current
                 kernel source is committed under profiles/, else null);
  cpu_baseline : the FP64 oracle on the host cores over a bounded sample of
                 the same launches (a few planes of each);
  breakdown    : per-case times and GB/s, the BF16 sweep beside the FP32 one.
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


def bicubic_dw4_init(p, q, C, seed):
    """Learned depthwise 4x4 taps initialised to the bicubic outer product
    (the plan's own taps) plus N(0, 0.01) noise, for every channel."""
    import paper_2203_10670_amd as fc
    import synth
    pl = fc.Plan(p, q, "bicubic", "zero")
    t = np.array([fc.fcfs_plan_taps(pl.handle, 0, j)[1] for j in range(pl.p_red)], dtype=np.float64)
    base = np.einsum("ia,jb->ijab", t, t)[None].repeat(C, axis=0)
    return (base + synth.normal(seed, base.shape, std=0.1)).astype(np.float32)


def measure_rows(reps: int):
    """The other workloads of the hot path, each timed on its own:
    - 16x64x512x512 N(0,1) bicubic 5/4 forward, FP32 and BF16 storage;
    - the channel-mixing layer on MFMA on the same BF16 input (64 -> 64);
    - the learned depthwise layer 8x64x256x256 at 3/4: forward and backward
      (input and weight gradients), FP32 and BF16, over 3 rotating buffer sets
      (one set fits in the 256 MB last-level cache)."""
    import torch
    import paper_2203_10670_amd as fc
    import synth
    dev = torch.device("cuda:0")
    sp = torch.cuda.current_stream(dev).cuda_stream
    out = {}

    def timeit(fn, n):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(n):
            fn(i)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1000.0 / n

    # 16 x 64 x 512^2, 5/4 bicubic
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
        us = timeit(run, reps)
        b = case_bytes(fc, pl, (N, C, H, W), es)
        out["bicubic_5_4_16x64x512_" + name] = {"us": round(us, 2), "bytes": b, "GBps": round(b / us / 1e3, 1)}
        del y
    # channel mixing on MFMA, BF16
    xb = x32.to(torch.bfloat16)
    del x32
    wm = torch.from_numpy(synth.normal(5, (5, 5, C, C, 4, 4), std=1 / 32)).to(dev).to(torch.bfloat16)
    plm = fc.Plan(5, 4, "mix4", "reflect")
    ym = torch.empty((N, C, ho, wo), dtype=torch.bfloat16, device=dev)

    def runm(i=0):
        st = fc.fcfs_forward(plm.handle, 1, N, C, H, W, xb.data_ptr(), wm.data_ptr(), C, ym.data_ptr(), sp)
        assert st == 0
    us = timeit(runm, max(3, reps // 2))
    flops = 2.0 * N * (ho // 5) * (wo // 5) * 25 * C * C * 16
    out["mix4_5_4_16x64x512_bf16"] = {"us": round(us, 2), "flop": flops,
                                      "TFLOPs": round(flops / us / 1e6, 1),
                                      "mfma_frac": round(flops / us / 1e6 / MFMA_PEAK_BF16_TFLOPS, 4)}
    # its backward: input gradient (VALU gather) and weight gradient (MFMA), each
    # the same flop count as the forward
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
    ux = timeit(runbx, max(2, reps // 4))
    uw = timeit(runbw, max(2, reps // 4))
    out["mix4_5_4_16x64x512_bf16_backward"] = {
        "dx_us": round(ux, 2), "dx_TFLOPs": round(flops / ux / 1e6, 1),
        "dw_us": round(uw, 2), "dw_TFLOPs": round(flops / uw / 1e6, 1),
        "dw_mfma_frac": round(flops / uw / 1e6 / MFMA_PEAK_BF16_TFLOPS, 4)}
    del xb, wm, ym, dxm, dwm, wsm
    torch.cuda.empty_cache()
    # learned depthwise 8 x 64 x 256^2 at 3/4, forward and backward
    N, C, H, W, p, q = 8, 64, 256, 256, 3, 4
    pld = fc.Plan(p, q, "dw4", "reflect")
    ho, wo = pld.output_size(H, W)
    wd = torch.from_numpy(bicubic_dw4_init(p, q, C, 7)).to(dev)
    for name, es in (("f32", 4), ("bf16", 2)):
        td = torch.float32 if name == "f32" else torch.bfloat16
        code = fc.DTYPES[name]
        sets = []
        for k in range(3):
            xt = torch.from_numpy(synth.normal(6 + 10 * k, (N, C, H, W))).to(dev).to(td)
            dyt = torch.from_numpy(synth.normal(8 + 10 * k, (N, C, ho, wo))).to(dev).to(td)
            sets.append((xt, dyt, torch.empty((N, C, ho, wo), dtype=td, device=dev),
                         torch.empty((N, C, H, W), dtype=td, device=dev)))
        dw = torch.empty_like(wd)
        wsb = fc.fcfs_backward_workspace(pld.handle, code, N, C, H, W, C)
        ws = torch.empty(max(1, wsb), dtype=torch.uint8, device=dev)

        def fwd(i=0):
            xt, _, yt, _ = sets[i % 3]
            assert fc.fcfs_forward(pld.handle, code, N, C, H, W, xt.data_ptr(), wd.data_ptr(), C, yt.data_ptr(), sp) == 0

        def bwd(i=0):
            xt, dyt, _, dxt = sets[i % 3]
            assert fc.fcfs_backward(pld.handle, code, N, C, H, W, xt.data_ptr(), wd.data_ptr(), C, dyt.data_ptr(),
                                    dxt.data_ptr(), dw.data_ptr(), ws.data_ptr(), wsb, sp) == 0
        uf = timeit(fwd, reps)
        ub = timeit(bwd, reps)
        bf = (N * C * H * W + N * C * ho * wo) * es
        bb = (N * C * ho * wo + 2 * N * C * H * W) * es
        out["dw4_3_4_8x64x256_" + name] = {"fwd_us": round(uf, 2), "fwd_GBps": round(bf / uf / 1e3, 1),
                                           "bwd_us": round(ub, 2), "bwd_GBps": round(bb / ub / 1e3, 1),
                                           "fwd_bytes": bf, "bwd_bytes": bb}
        del sets, ws
        torch.cuda.empty_cache()
    out.update(measure_nd(reps))
    out["quality_vs_framework_resize"] = measure_quality()
    return out


def measure_nd(reps: int):
    """1D and 3D FCFS, FP32 bicubic reflect: 16 x 2 signals of 2^20 samples
    at 3/2 (one pass), and a 2 x 1 x 128 x 256 x 256 volume at 3/2 on every
    axis (two passes through a workspace). GB/s counts the input and output
    once; the 3D figure with the intermediate's write and read is given too."""
    import torch
    import paper_2203_10670_amd as fc
    import synth
    dev = torch.device("cuda:0")
    sp = torch.cuda.current_stream(dev).cuda_stream
    out = {}

    def timeit(fn, n):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1000.0 / n

    N, C, L = 16, 2, 1 << 20
    x1 = torch.from_numpy(synth.normal(40, (N, C, L))).to(dev)
    pl1 = fc.Plan(1, 1, "bicubic", "reflect", pw=3, qw=2)
    lo = pl1.output_size(1, L)[1]
    y1 = torch.empty((N, C, lo), device=dev)
    us = timeit(lambda: fc.fcfs_forward_1d(pl1.handle, 0, N, C, L, x1.data_ptr(), y1.data_ptr(), sp), reps)
    b = (N * C * L + N * C * lo) * 4
    out["nd_1d_3_2_16x2x1M_f32"] = {"us": round(us, 2), "bytes": b, "GBps": round(b / us / 1e3, 1)}
    del x1, y1
    n, c, d, h, w = 2, 1, 128, 256, 256
    x3 = torch.from_numpy(synth.normal(41, (n, c, d, h, w))).to(dev)
    pld = fc.Plan(3, 2, "bicubic", "reflect", pw=1, qw=1)
    plhw = fc.Plan(3, 2, "bicubic", "reflect")
    do = pld.output_size(d, 1)[0]
    ho, wo = plhw.output_size(h, w)
    y3 = torch.empty((n, c, do, ho, wo), device=dev)
    wsb = fc.fcfs_forward_3d_workspace(pld.handle, plhw.handle, 0, n, c, d, h, w)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    us = timeit(lambda: fc.fcfs_forward_3d(pld.handle, plhw.handle, 0, n, c, d, h, w, x3.data_ptr(), y3.data_ptr(),
                                           ws.data_ptr(), wsb, sp), reps)
    b = (n * c * d * h * w + n * c * do * ho * wo) * 4
    out["nd_3d_3_2_2x1x128x256x256_f32"] = {"us": round(us, 2), "bytes": b, "GBps": round(b / us / 1e3, 1),
                                            "GBps_with_intermediate": round((b + 2 * wsb) / us / 1e3, 1)}
    del x3, y3, ws
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


def measure_serving(count: int, rhos=(0.25, 0.5, 0.8, 0.95)):
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


def cpu_baseline(cases, x_np, target_planes: int):
    import oracle
    threads = oracle.threads()
    k = max(1, min(SHAPE[0] * SHAPE[1], target_planes or 6 * threads))
    planes = x_np.reshape(-1, SHAPE[2], SHAPE[3])[:k][:, None].astype(np.float64)
    total_bytes = 0
    t0 = time.perf_counter()
    for cs in cases:
        oracle.forward(planes, cs["p"], cs["q"], cs["method"], cs["pad"])
        total_bytes += cs["bytes"] * k // (SHAPE[0] * SHAPE[1])
    dt = time.perf_counter() - t0
    return {"value": round(total_bytes / dt / 1e9, 4), "unit": "GB/s", "cores": min(threads, k),
            "kind": "oracle",
            "sample": "FP64 oracle, %d of %d planes of each of the %d FP32 launches of a step "
                      "(%.1f s wall)" % (k, SHAPE[0] * SHAPE[1], len(cases), dt)}


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
        print("%-60s %6s %12s %12s %6s" % ("kernel", "calls", "avg_us", "total_us", "pct"))
        for r in rows:
            name = r["Name"]
            short = name if len(name) <= 60 else name[:57] + "..."
            print("%-60s %6s %12.2f %12.1f %6.2f" % (short, r["Calls"], float(r["AverageNs"]) / 1e3,
                                                      float(r["TotalDurationNs"]) / 1e3, float(r["Percentage"])))
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
        print("%-60s %-12s %8s %16s" % ("kernel", "counter", "rows", "avg_KiB_per_row"))
        for (k, c), (v, n) in sorted(agg.items()):
            short = k if len(k) <= 60 else k[:57] + "..."
            print("%-60s %-12s %8d %16.1f" % (short, c, n, v / n))


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
        copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--cpu-planes", type=int, default=0)
    ap.add_argument("--no-rows", action="store_true", help="skip the other workloads (mix4, learned layer, ...)")
    ap.add_argument("--serve-requests", type=int, default=10000, help="requests of the serving run (0: skip)")
    ap.add_argument("--filter", default="", help="only cases whose name contains this text")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM counters)")
    ap.add_argument("--summarize", metavar="DIR", help="summarise rocprofv3 CSV output under DIR and exit")
    ap.add_argument("--traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn FETCH_SIZE / WRITE_SIZE counter runs (with --copy-calibration) into "
                         "profiles/fwd_traffic.json and exit")
    args = ap.parse_args()
    if args.summarize:
        summarize(args.summarize)
        return
    if args.traffic:
        write_traffic(*args.traffic)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the rescale path has no multi-GPU mode "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2203_10670_amd as fc
    import synth

    dev = torch.device("cuda:0")
    stream_ptr = torch.cuda.current_stream(dev).cuda_stream
    x_np = synth.uniform(2, SHAPE)
    x32 = torch.from_numpy(x_np).to(dev)
    xbf = x32.to(torch.bfloat16)

    def make_cases(dtype_name, xt, esize):
        cases = []
        for (p, q) in FRACS:
            for m in METHODS:
                for pad in PADS:
                    pl = fc.Plan(p, q, m, pad)
                    ho, wo = pl.output_size(SHAPE[2], SHAPE[3])
                    y = torch.empty((SHAPE[0], SHAPE[1], ho, wo), dtype=xt.dtype, device=dev)
                    code = fc.DTYPES[dtype_name]
                    kid = fc.fcfs_forward_config(pl.handle, code, SHAPE[0], SHAPE[1], SHAPE[2], SHAPE[3])[0]
                    cases.append({"p": p, "q": q, "method": m, "pad": pad, "plan": pl, "y": y, "x": xt,
                                  "code": code, "kernel_id": kid, "dtype": dtype_name,
                                  "bytes": case_bytes(fc, pl, SHAPE, esize)})
        return cases

    def launch(cs):
        st = fc.fcfs_forward(cs["plan"].handle, cs["code"], SHAPE[0], SHAPE[1], SHAPE[2], SHAPE[3],
                             cs["x"].data_ptr(), None, SHAPE[1], cs["y"].data_ptr(), stream_ptr)
        if st != 0:
            raise fc.FcfsError(st, "fcfs_forward")

    def timed_sweep(cases, steps, warmup):
        for _ in range(warmup):
            for cs in cases:
                launch(cs)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            for cs in cases:
                launch(cs)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    def per_case(cases, reps):
        out = []
        for cs in cases:
            launch(cs)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                launch(cs)
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1000.0 / reps
            out.append((cs, us))
        return out

    if args.copy_calibration:
        n = 1 << 28   # 1 GiB of FP32 read and written
        a_ = torch.rand(n, device=dev)
        b_ = torch.empty_like(a_)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            b_.copy_(a_)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        print("copy 1 GiB: %.3f ms, %.1f GB/s (read + write)" % (ms, 2 * 4 * n / (ms * 1e-3) / 1e9),
              file=sys.stderr, flush=True)
        del a_, b_

    f32 = make_cases("f32", x32, 4)
    f32_meta = [{k: c[k] for k in ("p", "q", "method", "pad", "bytes")} for c in f32]
    if args.filter:
        f32 = [c for c in f32 if args.filter in "%d/%d %s %s" % (c["p"], c["q"], c["method"], c["pad"])]
        f32_meta = [c for c in f32_meta if args.filter in "%d/%d %s %s" % (c["p"], c["q"], c["method"], c["pad"])]
    ms_step = timed_sweep(f32, args.steps, args.warmup)
    step_bytes = sum(c["bytes"] for c in f32)
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
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": load_traffic(kid),
                "kernel_id": kid, "launches": g["n"], "avg_us": round(avg_us, 2),
                "bytes_per_launch": int(bytes_per_launch)}

    breakdown = {"f32": [{"case": "%d/%d %s %s" % (c["p"], c["q"], c["method"], c["pad"]),
                          "us": round(us, 2), "GBps": round(c["bytes"] / (us * 1e-6) / 1e9, 1),
                          "kernel_id": c["kernel_id"]} for c, us in pc]}
    bf16_value = None
    if not args.no_bf16 and not args.filter:
        bf = make_cases("bf16", xbf, 2)
        ms_bf = timed_sweep(bf, args.steps, args.warmup)
        bf16_value = sum(c["bytes"] for c in bf) / (ms_bf * 1e-3) / 1e9
        pcb = per_case(bf, reps)
        breakdown["bf16"] = [{"case": "%d/%d %s %s" % (c["p"], c["q"], c["method"], c["pad"]),
                              "us": round(us, 2), "GBps": round(c["bytes"] / (us * 1e-6) / 1e9, 1)}
                             for c, us in pcb]
        breakdown["bf16_step_ms"] = round(ms_bf, 4)
        breakdown["bf16_GBps"] = round(bf16_value, 1)
        del bf, pcb
    torch.cuda.synchronize()

    rows = None
    if not args.no_rows and not args.filter:
        del f32, pc, x32, xbf
        torch.cuda.empty_cache()
        rows = measure_rows(max(3, args.steps))
        if args.serve_requests > 0:
            rows["serving"] = measure_serving(args.serve_requests)

    cpu = None
    if not args.no_cpu_baseline and not args.filter:
        cpu = cpu_baseline(f32_meta, x_np, args.cpu_planes)

    line = {
        "metric": "resample output GB/s vs HBM peak (FP32, BF16); served p50/p99 latency",
        "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "FCFS forward sweep: N=32 C=3 1024x1024 FP32 U[0,1); scales 3/2 2/3 5/4 4/5; "
                               "nearest bilinear bicubic; zero and reflect padding (24 launches per step)",
                   "batch": SHAPE[0], "channels": SHAPE[1], "height": SHAPE[2], "width": SHAPE[3],
                   "launches_per_step": len(f32_meta), "bytes_per_step": step_bytes},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "bf16_value": None if bf16_value is None else round(bf16_value, 1),
        "breakdown": breakdown,
        "rows": rows,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
