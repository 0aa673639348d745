"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and compare with the FP64 oracle element by element."""
import numpy as np

import oracle
import synth

# unit roundoff of each storage type (RNE store of an FP32 result), and the
# absolute rounding error bound in its subnormal range (half the smallest
# subnormal spacing)
UNIT = {"f32": 2.0 ** -24, "bf16": 2.0 ** -8, "f16": 2.0 ** -11}
UNIT_ABS = {"f32": 2.0 ** -150, "bf16": 2.0 ** -134, "f16": 2.0 ** -25}
# accumulation tolerance of the FP32 arithmetic, relative to S = sum |w||x|
# (at most 16 products and one rounded weight per tap: well below 1e-5)
ACC = 1e-5


def torch_dtype(name):
    import torch
    return {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[name]


def storage_round(x, dtype):
    """The values a tensor of this storage type holds (as float32)."""
    if dtype == "bf16":
        return synth.bf16_round(x)
    if dtype == "f16":
        return synth.f16_round(x)
    return np.ascontiguousarray(x, dtype=np.float32)


def gpu_forward(x32, p, q, method, pad, dtype="f32", grid="half", weight=None, pw=None, qw=None,
                stream=None):
    """x32: float32 NCHW numpy values already representable in ``dtype``."""
    import torch
    import paper_2203_10670_amd as fc
    xt = torch.from_numpy(x32).to("cuda").to(torch_dtype(dtype)).contiguous()
    wt = None if weight is None else torch.from_numpy(np.ascontiguousarray(weight, np.float32)).cuda()
    pl = fc.Plan(p, q, method, pad, grid, pw, qw)
    if stream is None:
        y = pl.forward(xt, wt)
    else:
        with torch.cuda.stream(stream):
            y = pl.forward(xt, wt)
        stream.synchronize()
    return y.float().cpu().numpy()


def assert_parity(y, x, p, q, method, pad, dtype="f32", grid="half", weight=None, pw=None, qw=None,
                  what=""):
    """|y - r| <= u |r| + ACC * S elementwise, r the FP64 oracle on the same
    (storage-rounded) inputs, S = sum |w||x| its conditioning."""
    x64 = np.asarray(x, dtype=np.float64)
    r = oracle.forward(x64, p, q, method, pad, grid, weight=weight, pw=pw, qw=qw)
    assert y.shape == r.shape, (y.shape, r.shape, what)
    if method == "nearest":
        np.testing.assert_array_equal(y, r.astype(np.float32), err_msg="nearest must be a bit-exact copy " + what)
        return
    S = oracle.condition(x64, p, q, method, pad, grid, weight=weight, pw=pw, qw=qw)
    err = np.abs(y.astype(np.float64) - r)
    bound = UNIT[dtype] * np.abs(r) + UNIT_ABS[dtype] + ACC * S + 1e-30
    bad = err > bound
    if bad.any():
        i = np.argwhere(bad)[0]
        raise AssertionError("%s: %d of %d outside tolerance; first at %s: gpu %r oracle %r S %r"
                             % (what, int(bad.sum()), bad.size, tuple(i), float(y[tuple(i)]),
                                float(r[tuple(i)]), float(S[tuple(i)])))
    return float((err / np.maximum(S, 1e-30)).max())


def oracle_band(xplane, p, q, method, pad, m_lo, m_hi, grid="half", weight=None, pw=None, qw=None):
    """Oracle output rows [p*m_lo, p*m_hi) of one plane (reduced p/q), from a
    crop of the input rows that holds every row those outputs read. The crop
    starts on a multiple of q, so cell m of the crop is cell m + start/q."""
    from math import gcd
    g = gcd(p, q)
    pr, qr = p // g, q // g
    H = xplane.shape[0]
    start = max(0, qr * (m_lo - 2))
    end = min(H, qr * (m_hi + 2))
    crop = np.asarray(xplane[start:end], dtype=np.float64)[None, None]
    if start > 0 and pad != "zero":
        pass  # rows read near the crop's top are inside the crop (margin >= q + 2)
    full = oracle.forward(crop, p, q, method, pad, grid, weight=weight, pw=pw, qw=qw)[0, 0]
    c0 = start // qr
    return full[pr * (m_lo - c0): pr * (m_hi - c0)]


def oracle_band_cond(xplane, p, q, method, pad, m_lo, m_hi):
    """As oracle_band, with the band's conditioning S = sum |w||x| beside it."""
    from math import gcd
    g = gcd(p, q)
    pr, qr = p // g, q // g
    H = xplane.shape[0]
    start = max(0, qr * (m_lo - 2))
    end = min(H, qr * (m_hi + 2))
    crop = np.asarray(xplane[start:end], dtype=np.float64)[None, None]
    r = oracle.forward(crop, p, q, method, pad)[0, 0]
    S = oracle.condition(crop, p, q, method, pad)[0, 0]
    c0 = start // qr
    sl = slice(pr * (m_lo - c0), pr * (m_hi - c0))
    return r[sl], S[sl]


def band_check(g, r, S, dtype, tol=ACC, method="", what=""):
    """|g - r| <= u |r| + u_sub + tol * S on a band (nearest: bit-exact);
    returns the largest |g - r| / S."""
    if method == "nearest":
        np.testing.assert_array_equal(g, r.astype(np.float32), err_msg="nearest must be a bit-exact copy " + what)
        return 0.0
    err = np.abs(np.asarray(g, np.float64) - r)
    bound = UNIT[dtype] * np.abs(r) + UNIT_ABS[dtype] + tol * S + 1e-30
    bad = err > bound
    if bad.any():
        i = tuple(np.argwhere(bad)[0])
        raise AssertionError("%s: %d of %d outside tolerance; first at %s: gpu %r oracle %r S %r"
                             % (what, int(bad.sum()), bad.size, i, float(g[i]), float(r[i]), float(S[i])))
    return float((err / np.maximum(S, 1e-30)).max())


def oracle_crop(x, p, q, method, pad, mh, mw, weight=None, cout=None):
    """Oracle outputs of cells mh = (lo, hi) x mw = (lo, hi) of every plane,
    computed from a crop of the input that holds every sample those cells
    read (crop starts on multiples of q, with q+2 samples of margin)."""
    from math import gcd
    g = gcd(p, q)
    pr, qr = p // g, q // g
    N, C, H, W = x.shape
    r0, r1 = max(0, qr * (mh[0] - 2)), min(H, qr * (mh[1] + 2))
    c0, c1 = max(0, qr * (mw[0] - 2)), min(W, qr * (mw[1] + 2))
    crop = np.asarray(x[:, :, r0:r1, c0:c1], dtype=np.float64)
    full = oracle.forward(crop, p, q, method, pad, weight=weight, cout=cout)
    # a crop that stops inside the image has a different edge; only cells whose
    # taps stay inside the crop are returned, and those do not see that edge
    a, b = r0 // qr, c0 // qr
    return full[:, :, pr * (mh[0] - a): pr * (mh[1] - a), pr * (mw[0] - b): pr * (mw[1] - b)]


def splitmix64_uniform(seed, count):
    """The serving loop's generated input, element i: the top 24 bits of
    splitmix64(seed + (i + 1) * 0x9E3779B97F4A7C15) over 2^24 (the published
    SplitMix64 finaliser), as float32."""
    with np.errstate(over="ignore"):
        i = np.arange(count, dtype=np.uint64)
        z = np.uint64(seed) + (i + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return ((z >> np.uint64(40)).astype(np.float64) / 16777216.0).astype(np.float32)
