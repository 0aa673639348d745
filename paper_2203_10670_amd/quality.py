"""Image-quality measures for comparing FCFS output with another resampler.

The paper reports PSNR and SSIM of FCFS against a framework resize and reads
values above 20 dB and close to 1.00 as the two being visually the same
(Sec. 6.2). These functions compute both measures on NCHW tensors (CPU or
device), in float64:

- ``psnr``: 10 log10(R^2 / MSE) over the whole tensor, R the data range.
- ``ssim``: the structural similarity index of Wang, Bovik, Sheikh and
  Simoncelli (2004), with its usual constants: an 11-tap Gaussian window of
  standard deviation 1.5 applied separably with no padding, K1 = 0.01,
  K2 = 0.03, averaged over every channel and window position.
"""
from __future__ import annotations

import math


def _torch():
    import torch
    return torch


def psnr(a, b, data_range: float = 1.0) -> float:
    """Peak signal-to-noise ratio in dB (inf for identical inputs)."""
    torch = _torch()
    a = a.to(torch.float64)
    b = b.to(torch.float64)
    mse = float(torch.mean((a - b) ** 2))
    if mse == 0.0:
        return math.inf
    return 10.0 * math.log10(data_range * data_range / mse)


def _gaussian_window(size: int, sigma: float, device):
    torch = _torch()
    r = torch.arange(size, dtype=torch.float64, device=device) - (size - 1) / 2.0
    g = torch.exp(-(r * r) / (2.0 * sigma * sigma))
    return g / g.sum()


def _blur(x, g):
    """Separable 'valid' filtering of every (n, c) plane with the 1D window g."""
    torch = _torch()
    n, c, h, w = x.shape
    k = g.numel()
    planes = x.reshape(n * c, 1, h, w)
    planes = torch.nn.functional.conv2d(planes, g.view(1, 1, 1, k))
    planes = torch.nn.functional.conv2d(planes, g.view(1, 1, k, 1))
    return planes.reshape(n, c, h - k + 1, w - k + 1)


def ssim(a, b, data_range: float = 1.0, win: int = 11, sigma: float = 1.5,
         k1: float = 0.01, k2: float = 0.03) -> float:
    """Mean structural similarity of two NCHW tensors of the same shape."""
    torch = _torch()
    if a.shape != b.shape or a.dim() != 4:
        raise ValueError("ssim needs two NCHW tensors of one shape")
    if a.shape[2] < win or a.shape[3] < win:
        raise ValueError("ssim needs planes of at least %d x %d" % (win, win))
    a = a.to(torch.float64)
    b = b.to(torch.float64)
    g = _gaussian_window(win, sigma, a.device)
    c1 = (k1 * data_range) ** 2
    c2 = (k2 * data_range) ** 2
    mu_a = _blur(a, g)
    mu_b = _blur(b, g)
    var_a = _blur(a * a, g) - mu_a * mu_a
    var_b = _blur(b * b, g) - mu_b * mu_b
    cov = _blur(a * b, g) - mu_a * mu_b
    num = (2.0 * mu_a * mu_b + c1) * (2.0 * cov + c2)
    den = (mu_a * mu_a + mu_b * mu_b + c1) * (var_a + var_b + c2)
    return float(torch.mean(num / den))


# The framework resize each FCFS method is compared with: the same
# half-pixel grid (the scale factor is passed, so source coordinates are
# (k + 1/2) q / p - 1/2 exactly as in FCFS) and edge clamping (FCFS's
# replicate padding). Nearest rounds half up in both; bicubic differs in the
# cubic's free parameter (-0.75 in the framework, -1/2 in FCFS).
FRAMEWORK_MODE = {"nearest": "nearest-exact", "bilinear": "bilinear", "bicubic": "bicubic"}


def framework_resize(x, p: int, q: int, method: str):
    """torch's interpolate at scale p/q (float32 in, float32 out)."""
    torch = _torch()
    mode = FRAMEWORK_MODE[method]
    kw = {} if mode == "nearest-exact" else {"align_corners": False}
    return torch.nn.functional.interpolate(x.to(torch.float32), scale_factor=p / q, mode=mode,
                                           recompute_scale_factor=False, **kw)


def compare_with_framework(y, x, p: int, q: int, method: str):
    """(PSNR, SSIM) of an FCFS output y against the framework resize of x,
    over the output region both produce (FCFS has p*ceil(N/q) samples per
    axis, the framework floor(N*p/q))."""
    z = framework_resize(x, p, q, method)
    h = min(y.shape[2], z.shape[2])
    w = min(y.shape[3], z.shape[3])
    y = y[:, :, :h, :w].to(z.dtype)
    z = z[:, :, :h, :w]
    return psnr(y, z), ssim(y, z)
