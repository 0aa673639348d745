"""GPU tests of the serving loop: every result of a mixed, continuously
batched stream equals the same request run alone through fcfs_forward (bit
for bit) and the FP64 oracle (within tolerance); admission under a small
memory budget; failures stay with their own requests."""
import sys

import numpy as np
import pytest

import synth
from fcfs_testutil import assert_parity, splitmix64_uniform, storage_round, torch_dtype

pytestmark = pytest.mark.gpu

METHODS = ["nearest", "bilinear", "bicubic"]
PADS = ["zero", "replicate", "reflect"]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _read(fc, res, shape, dtype):
    return fc.device_view(res.y, shape, dtype)


def _solo(fc, x_t, p, q, method, pad):
    return fc.Plan(p, q, method, pad).forward(x_t)


def test_mixed_stream_equals_solo_and_oracle():
    import torch
    import paper_2203_10670_amd as fc
    rng = np.random.default_rng(9)
    srv = fc.Server(0, 4 << 30, 48)
    reqs = []
    for i in range(150):
        p, q = int(rng.integers(1, 9)), int(rng.integers(1, 9))
        m, pad = METHODS[int(rng.integers(3))], PADS[int(rng.integers(3))]
        dt = ["f32", "bf16"][int(rng.integers(2))]
        shape = (int(rng.integers(1, 3)), 3, int(rng.integers(5, 260)), int(rng.integers(5, 260)))
        seed = int(rng.integers(0, 2 ** 62))
        t = srv.submit(p, q, m, pad, dt, shape, seed=seed)
        reqs.append((t, p, q, m, pad, dt, shape, seed))
    _say("submitted", len(reqs))
    for k, (t, p, q, m, pad, dt, shape, seed) in enumerate(reqs):
        r = srv.wait(t)
        assert r.status == 0, (k, r.status)
        out_shape = (shape[0], shape[1], r.h_out, r.w_out)
        got = _read(fc, r, out_shape, dt)
        x = storage_round(splitmix64_uniform(seed, int(np.prod(shape))).reshape(shape), dt)
        xt = torch.from_numpy(x).cuda().to(torch_dtype(dt))
        solo = _solo(fc, xt, p, q, m, pad)
        assert torch.equal(got, solo), (k, p, q, m, pad, dt, shape)
        if k % 10 == 0:
            assert_parity(got.float().cpu().numpy(), x, p, q, m, pad, dt, what=f"served {k}")
        srv.release(t)
    p50, p99, rps, gbps = srv.stats()
    assert 0 < p50 <= p99 and rps > 0 and gbps > 0
    srv.close()


def test_caller_owned_buffers():
    import torch
    import paper_2203_10670_amd as fc
    srv = fc.Server(0, 1 << 30, 8)
    x = torch.from_numpy(synth.normal(3, (2, 3, 77, 131))).cuda()
    pl = fc.Plan(5, 4, "bicubic", "reflect")
    ho, wo = pl.output_size(77, 131)
    y = torch.full((2, 3, ho, wo), 7.0, device="cuda")
    # the fill runs on torch's stream; the server's streams do not wait for it
    torch.cuda.synchronize()
    t = srv.submit(5, 4, "bicubic", "reflect", "f32", tuple(x.shape), x=x, y=y)
    r = srv.wait(t)
    assert r.status == 0 and r.y == y.data_ptr()
    assert torch.equal(y, pl.forward(x))
    srv.release(t)
    srv.close()


def test_small_budget_admission_and_oversized_request():
    import paper_2203_10670_amd as fc
    # budget for about two requests of 3x128x128 fp32 at 3/2 (0.2 MB in + 0.44 MB out)
    srv = fc.Server(0, 1500 * 1024, 16)
    tickets = [srv.submit(3, 2, "bilinear", "zero", "f32", (1, 3, 128, 128), seed=s) for s in range(12)]
    big = srv.submit(4, 1, "nearest", "zero", "f32", (1, 3, 512, 512), seed=99)   # needs 12.6 MB
    more = srv.submit(3, 2, "bilinear", "zero", "f32", (1, 3, 128, 128), seed=100)
    for t in tickets:
        r = srv.wait(t)
        assert r.status == 0
        srv.release(t)
    rb = srv.wait(big)
    assert rb.status == fc.E_NOMEM
    srv.release(big)
    assert srv.wait(more).status == 0
    srv.release(more)
    srv.close()


def test_forced_failures_stay_isolated():
    import paper_2203_10670_amd as fc
    srv = fc.Server(0, 1 << 28, 4)
    assert fc.fcfs_server_debug(srv.handle, 1, 1) == 0
    a = srv.submit(3, 2, "bicubic", "reflect", "bf16", (1, 3, 40, 50), seed=1)
    ra = srv.wait(a)
    assert ra.status == fc.E_NOMEM
    assert fc.fcfs_server_debug(srv.handle, 2, 1) == 0
    b = srv.submit(3, 2, "bicubic", "reflect", "bf16", (1, 3, 40, 50), seed=2)
    rb = srv.wait(b)
    assert rb.status == fc.E_DEVICE
    c = srv.submit(3, 2, "bicubic", "reflect", "bf16", (1, 3, 40, 50), seed=3)
    rc = srv.wait(c)
    assert rc.status == 0
    for t in (a, b, c):
        srv.release(t)
    # unknown ticket, pending release
    assert fc.fcfs_poll(srv.handle, 10 ** 9)[0] == fc.E_INVAL
    srv.close()


def test_destroy_with_pending_requests():
    import paper_2203_10670_amd as fc
    srv = fc.Server(0, 1 << 30, 2)
    for s in range(40):
        srv.submit(2, 1, "nearest", "zero", "f32", (1, 3, 300, 300), seed=s)
    srv.close()   # finishes admitted work, cancels the rest, frees everything


def test_replay_one_launch_per_request_and_discard():
    import paper_2203_10670_amd as fc
    srv = fc.Server(0, 2 << 30, 32)
    meta = synth.request_stream(21, 60, rate_per_s=0.0, hw_lo=16, hw_hi=300)
    reqs = [fc.fcfs_request(r.p, r.q, r.method, r.pad, r.dtype, 1, r.c, r.h, r.w, None, r.seed, None)
            for r in meta]
    arr = [20.0 * i for i in range(len(reqs))]
    for max_batch in (1, 0):
        assert fc.fcfs_server_config(srv.handle, fc.FCFS_SERVER_MAX_BATCH, max_batch) == 0
        assert fc.fcfs_server_config(srv.handle, fc.FCFS_SERVER_DISCARD_OUTPUTS, 1) == 0
        assert fc.fcfs_server_reset_stats(srv.handle) == 0
        st, tickets = fc.fcfs_server_replay(srv.handle, reqs, arr)
        assert st == 0
        for t in tickets:
            r = srv.wait(t)
            assert r.status == 0 and r.y is None
            srv.release(t)
        p50, p99, rps, gbps = srv.stats()
        assert 0 < p50 <= p99 and rps > 0
    assert fc.fcfs_server_config(srv.handle, 99, 1) == fc.E_INVAL
    srv.close()


@pytest.mark.parametrize("chunk", [37, 1000, 0])
def test_chunked_requests_equal_solo(chunk):
    """Requests larger than the chunk size run as chunks over several batches
    (on both streams, after their input was generated on either); every
    result equals its solo run bit for bit, and one is checked against the
    oracle."""
    import torch
    import paper_2203_10670_amd as fc
    srv = fc.Server(0, 2 << 30, 16)
    assert fc.fcfs_server_config(srv.handle, fc.FCFS_SERVER_CHUNK_WAVES, chunk) == 0
    reqs = [(3, 2, "bicubic", "reflect", "f32", (1, 3, 300, 400), 11),
            (2, 3, "bilinear", "zero", "bf16", (2, 3, 77, 131), 12),
            (5, 4, "nearest", "replicate", "f32", (1, 3, 500, 520), 13),
            (7, 8, "bicubic", "zero", "bf16", (1, 3, 260, 700), 14),
            (3, 2, "bilinear", "replicate", "f32", (1, 1, 9, 11), 15)]
    tickets = [srv.submit(p, q, m, pad, dt, shape, seed=seed) for (p, q, m, pad, dt, shape, seed) in reqs]
    _say("chunk", chunk, "submitted", len(tickets))
    for k, (t, (p, q, m, pad, dt, shape, seed)) in enumerate(zip(tickets, reqs)):
        r = srv.wait(t)
        assert r.status == 0, (k, r.status)
        got = fc.device_view(r.y, (shape[0], shape[1], r.h_out, r.w_out), dt)
        x = storage_round(splitmix64_uniform(seed, int(np.prod(shape))).reshape(shape), dt)
        solo = _solo(fc, torch.from_numpy(x).cuda().to(torch_dtype(dt)), p, q, m, pad)
        assert torch.equal(got, solo), (chunk, k)
        if k == 0:
            assert_parity(got.float().cpu().numpy(), x, p, q, m, pad, dt, what="chunked %d" % chunk)
        srv.release(t)
    srv.close()


def test_chunked_failure_stays_with_its_request():
    """A failed batch fails the chunked request it held a chunk of (when its
    last launched chunk completes) and nothing else."""
    import paper_2203_10670_amd as fc
    srv = fc.Server(0, 1 << 30, 8)
    assert fc.fcfs_server_config(srv.handle, fc.FCFS_SERVER_CHUNK_WAVES, 50) == 0
    assert fc.fcfs_server_debug(srv.handle, 2, 1) == 0
    a = srv.submit(3, 2, "bicubic", "reflect", "f32", (1, 3, 300, 400), seed=1)
    ra = srv.wait(a)
    assert ra.status == fc.E_DEVICE
    b = srv.submit(3, 2, "bicubic", "reflect", "f32", (1, 3, 300, 400), seed=2)
    rb = srv.wait(b)
    assert rb.status == 0
    for t in (a, b):
        srv.release(t)
    srv.close()
