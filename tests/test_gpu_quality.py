"""Quality of the HIP path against the framework resize on the smooth
synthetic set: the paper's visual-sameness reading (PSNR above 20 dB, SSIM
close to 1.00) for up- and down-scaling, and near-identity where both
resamplers sample the same grid with the same weights."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

UP = [(3, 2), (5, 4), (2, 1), (27, 11)]
DOWN = [(2, 3), (4, 5), (1, 2), (2, 11)]


@pytest.fixture(scope="module")
def smooth_set():
    import torch
    return torch.from_numpy(synth.smooth(3, (2, 3, 256, 256))).cuda()


@pytest.mark.parametrize("pq", UP + DOWN, ids=lambda t: "%d_%d" % t)
@pytest.mark.parametrize("method", ["nearest", "bilinear", "bicubic"])
def test_quality_against_framework_resize(smooth_set, pq, method):
    import torch
    import paper_2203_10670_amd as fc
    from paper_2203_10670_amd import quality
    p, q = pq
    print("quality", p, q, method, flush=True)
    sys.stdout.flush()
    y = fc.resize(smooth_set, p, q, method, "replicate")
    torch.cuda.synchronize()
    ps, ss = quality.compare_with_framework(y, smooth_set, p, q, method)
    assert ps > 20.0 and ss > 0.99, (ps, ss)
    if method == "bilinear":
        # same grid, same weights, edge clamping = replicate: FP32 rounding apart
        assert ps > 100.0, ps
    if method == "nearest":
        # the same samples, except where a float half-way test rounds the other way
        assert ps > 60.0, ps
