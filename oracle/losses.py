"""FP64 oracle of the Stage 2/3 losses around the motion path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module; the product path never loads it.

Plain numpy in float64, written from the paper's loss definitions (Sec. 2.3.2):

* the projection loss of Eq. 10 / Eq. 12: an L1 term plus lambda_ssim = 0.25
  times a D-SSIM term, averaged over the views of the batch;
* the total-variation regulariser of Eq. 11 on a D x D x D sub-volume (D = 32)
  of the voxelized reference volume, weight lambda_tv = 0.05;
* the MBC normality loss of Eq. 13, weight lambda_MBC = 1 (Eq. 14).

The paper leaves the discretisations open; the readings taken here are:

* L1(p_r, p) is the mean over the view's pixels of |p_r - p|; its derivative
  at p_r = p is taken as 0.
* D-SSIM = 1 - SSIM with SSIM the pixel mean of the SSIM map of Zhou et al.
  (2004): local means, variances and covariance under an 11 x 11 Gaussian
  window (sigma 1.5, normalised, separable), computed with zero padding
  outside the detector (same-size windows), constants C1 = 0.01^2 and
  C2 = 0.03^2 (unit dynamic range; projections are not rescaled).
* TV is the anisotropic total variation of the sub-volume: the sum over
  forward differences with both voxels inside it of |V(p + e_a) - V(p)|,
  divided by D^3; the derivative of |.| at 0 is taken as 0.  The sub-volume is
  the block of the voxelized reference volume at a given corner (voxelizing
  the Gaussians on that sub-grid gives the same values).
* |e|^2 in Eq. 13 is the sum of squares of a basis volume over its level's
  own voxel grid; with B bases per level the sum runs over every (level,
  basis, component) channel and 1/9 becomes 1/(3 L B).

Gradients are the analytic derivatives of these definitions; the tests pin
them with central finite differences of the losses.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

SSIM_RADIUS = 5
SSIM_SIGMA = 1.5
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def ssim_window() -> np.ndarray:
    """The 11-tap Gaussian (sigma 1.5), normalised to sum 1; the 2-D window is
    its outer product."""
    d = np.arange(-SSIM_RADIUS, SSIM_RADIUS + 1, dtype=np.float64)
    w = np.exp(-0.5 * d * d / (SSIM_SIGMA * SSIM_SIGMA))
    return w / w.sum()


def _correlate_axis(a: np.ndarray, w: np.ndarray, axis: int) -> np.ndarray:
    """Same-size correlation along one axis with zeros outside the array."""
    r = len(w) // 2
    a = np.moveaxis(a, axis, -1)
    n = a.shape[-1]
    pad = np.zeros(a.shape[:-1] + (n + 2 * r,), dtype=np.float64)
    pad[..., r:r + n] = a
    out = np.zeros_like(a, dtype=np.float64)
    for k in range(len(w)):
        out += w[k] * pad[..., k:k + n]
    return np.moveaxis(out, -1, axis)


def blur(img: np.ndarray) -> np.ndarray:
    """Local Gaussian-weighted mean over the last two axes (v, u), zero padded."""
    w = ssim_window()
    return _correlate_axis(_correlate_axis(np.asarray(img, np.float64), w, -1), w, -2)


def ssim_map(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Per-pixel SSIM of images x and y (last two axes are v, u)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my = blur(x), blur(y)
    sxx = blur(x * x) - mx * mx
    syy = blur(y * y) - my * my
    sxy = blur(x * y) - mx * my
    return ((2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)) / \
        ((mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2))


def l1_dssim_loss(proj, target, lam: float = 0.25) -> Tuple[float, np.ndarray]:
    """Eq. 12 with the L1 and D-SSIM terms of Eq. 10: for views v of the batch,
    loss = (1/V) sum_v [ mean|x_v - y_v| + lam (1 - mean SSIM(x_v, y_v)) ],
    x = rendered projections [V][nv][nu], y = measured ones.  Returns the loss
    and d loss / d x."""
    x = np.asarray(proj, np.float64)
    y = np.asarray(target, np.float64)
    V = x.shape[0]
    npix = x.shape[1] * x.shape[2]
    mx, my = blur(x), blur(y)
    sxx = blur(x * x) - mx * mx
    syy = blur(y * y) - my * my
    sxy = blur(x * y) - mx * my
    a1 = 2 * mx * my + SSIM_C1
    a2 = 2 * sxy + SSIM_C2
    b1 = mx * mx + my * my + SSIM_C1
    b2 = sxx + syy + SSIM_C2
    s = (a1 * a2) / (b1 * b2)
    l1 = np.abs(x - y).sum(axis=(1, 2)) / npix
    ssim = s.sum(axis=(1, 2)) / npix
    loss = float(np.sum(l1 + lam * (1.0 - ssim)) / V)
    # S depends on x through m1 = blur(x), m2 = blur(x^2) and m12 = blur(x y)
    # (mx = m1, sxx = m2 - m1^2, sxy = m12 - m1 my); chain rule per pixel,
    # then the transpose of the blur, which for the symmetric window with
    # zero padding is the same blur.
    d_m1 = s * (2 * my / a1 - 2 * my / a2 - 2 * mx / b1 + 2 * mx / b2)
    d_m2 = -s / b2
    d_m12 = 2 * s / a2
    d_s = blur(d_m1) + 2 * x * blur(d_m2) + y * blur(d_m12)
    grad = (np.sign(x - y) - lam * d_s) / (npix * V)
    return loss, grad


def tv_loss(vol, corner: Sequence[int], D: int, weight: float = 1.0) -> Tuple[float, np.ndarray]:
    """weight * L_tv of the D^3 block of vol [n0][n1][n2] at `corner` (Eq. 11
    with the reading above).  Returns the weighted loss and its gradient with
    respect to the whole volume (zero outside the block)."""
    v = np.asarray(vol, np.float64)
    c0, c1, c2 = (int(c) for c in corner)
    sub = v[c0:c0 + D, c1:c1 + D, c2:c2 + D]
    assert sub.shape == (D, D, D), "block outside the volume"
    g_sub = np.zeros_like(sub)
    total = 0.0
    for axis in range(3):
        diff = np.diff(sub, axis=axis)          # V(p + e_a) - V(p), both inside
        total += np.abs(diff).sum()
        sg = np.sign(diff)
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, D - 1)
        hi[axis] = slice(1, D)
        g_sub[tuple(lo)] -= sg
        g_sub[tuple(hi)] += sg
    scale = weight / float(D ** 3)
    grad = np.zeros_like(v)
    grad[c0:c0 + D, c1:c1 + D, c2:c2 + D] = scale * g_sub
    return scale * total, grad


def mbc_normality_loss(bases: Sequence[np.ndarray], weight: float = 1.0
                       ) -> Tuple[float, List[np.ndarray]]:
    """weight * L_MBC of Eq. 13 for basis volumes bases[l] of shape [C][...]
    (C = 3 B channels per level): (1 / (L C)) sum_{l,c} (|E_l[c]|^2 - 1)^2.
    Returns the weighted loss and its gradient per level."""
    chans = [np.asarray(b, np.float64).reshape(np.shape(b)[0], -1) for b in bases]
    n = sum(c.shape[0] for c in chans)
    total = 0.0
    grads = []
    for c, b in zip(chans, bases):
        sq = (c * c).sum(axis=1)                 # |e|^2 per channel
        total += float(((sq - 1.0) ** 2).sum())
        g = (weight / n) * 2.0 * (sq - 1.0)[:, None] * 2.0 * c
        grads.append(g.reshape(np.shape(b)))
    return weight * total / n, grads
