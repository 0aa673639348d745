"""The image-quality measures (PSNR, SSIM) against closed forms and an
independent computation from library primitives (CPU only)."""
import math

import numpy as np
import pytest
import torch
from scipy.ndimage import correlate1d
from scipy.signal.windows import gaussian

from paper_2203_10670_amd import quality


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a))


def test_psnr_closed_form():
    rng = np.random.default_rng(1)
    a = rng.random((2, 3, 16, 16))
    for d in (0.5, 0.1, 1e-3):
        assert quality.psnr(_t(a), _t(a + d)) == pytest.approx(-20.0 * math.log10(d), abs=1e-9)
    assert quality.psnr(_t(a), _t(a)) == math.inf
    # data range enters as R^2
    assert quality.psnr(_t(a), _t(a + 0.1), data_range=255.0) == pytest.approx(20 * math.log10(2550.0), abs=1e-9)


def test_ssim_identity_and_symmetry():
    rng = np.random.default_rng(2)
    a = rng.random((1, 2, 24, 30))
    b = np.clip(a + 0.1 * rng.standard_normal(a.shape), 0, 1)
    assert quality.ssim(_t(a), _t(a)) == pytest.approx(1.0, abs=1e-12)
    assert quality.ssim(_t(a), _t(b)) == pytest.approx(quality.ssim(_t(b), _t(a)), abs=1e-12)
    assert quality.ssim(_t(a), _t(b)) < 1.0


def test_ssim_constant_images_closed_form():
    # constant planes m and m + c: zero variances, so only the luminance term
    # (2 m (m + c) + C1) / (m^2 + (m + c)^2 + C1) is left
    c1 = (0.01) ** 2
    for m, c in ((0.3, 0.2), (0.7, -0.5), (0.0, 0.4)):
        a = np.full((1, 1, 12, 12), m)
        b = np.full((1, 1, 12, 12), m + c)
        want = (2 * m * (m + c) + c1) / (m * m + (m + c) ** 2 + c1)
        assert quality.ssim(_t(a), _t(b)) == pytest.approx(want, abs=1e-12)


def test_ssim_matches_library_filtering():
    # the same definition evaluated with scipy's Gaussian window and 1D
    # correlations ('valid' part), per plane
    rng = np.random.default_rng(3)
    a = rng.random((2, 2, 20, 27))
    b = np.clip(a + 0.2 * rng.standard_normal(a.shape), 0, 1)
    g = gaussian(11, 1.5)
    g = g / g.sum()

    def blur(x):
        y = correlate1d(x, g, axis=-1, mode="constant")
        y = correlate1d(y, g, axis=-2, mode="constant")
        return y[..., 5:-5, 5:-5]

    c1, c2 = 0.01 ** 2, 0.03 ** 2
    ma, mb = blur(a), blur(b)
    va, vb, cab = blur(a * a) - ma * ma, blur(b * b) - mb * mb, blur(a * b) - ma * mb
    want = np.mean((2 * ma * mb + c1) * (2 * cab + c2) / ((ma * ma + mb * mb + c1) * (va + vb + c2)))
    assert quality.ssim(_t(a), _t(b)) == pytest.approx(want, abs=1e-12)


def test_framework_grid_matches_fcfs_sample_points():
    # on a linear ramp, bilinear resampling reproduces the source coordinate
    # exactly away from the clamped edges: the framework resize is then
    # (k + 1/2) q / p - 1/2, the FCFS grid
    for p, q in ((3, 2), (2, 3), (5, 4), (27, 11)):
        n = 66
        x = torch.arange(n, dtype=torch.float32).view(1, 1, 1, n).repeat(1, 1, 4, 1)
        z = quality.framework_resize(x, p, q, "bilinear")[0, 0, 0].double().numpy()
        k = np.arange(z.size)
        u = (k + 0.5) * q / p - 0.5
        inside = (u >= 0) & (u <= n - 1)
        np.testing.assert_allclose(z[inside], u[inside], atol=2e-4)
