"""Pins of the oracle's Stage 2/3 losses (Eq. 10-14) against facts that do
not come from the oracle: scipy's Gaussian filter for the SSIM window and
padding, a brute-force 2-D window sum, closed forms for constant and ramp
images, invariants, and central finite differences of each loss for its
gradient."""
import numpy as np
from scipy.ndimage import gaussian_filter

import oracle


def rng(seed):
    return np.random.default_rng(seed)


# ------------------------------------------------------------ D-SSIM, Eq. 10

def test_blur_is_scipy_gaussian_filter_with_zero_padding():
    """The local mean is scipy's Gaussian filter (sigma 1.5, radius 5, zeros
    outside), per view."""
    img = rng(1).uniform(-1.0, 3.0, (3, 23, 31))
    want = np.stack([gaussian_filter(v, 1.5, mode="constant", cval=0.0, truncate=5.0 / 1.5)
                     for v in img])
    assert np.allclose(oracle.blur(img), want, rtol=0, atol=1e-13)


def test_ssim_brute_force_2d_window():
    """Per-pixel SSIM from an explicit 11 x 11 window sum (2-D Gaussian,
    normalised, zero outside) and the constants 1e-4 and 9e-4."""
    r = rng(2)
    x = r.uniform(0.0, 2.0, (9, 12))
    y = x + r.normal(0.0, 0.3, x.shape)
    d = np.arange(-5, 6)
    w2 = np.exp(-(d[:, None] ** 2 + d[None, :] ** 2) / (2 * 1.5 ** 2))
    w2 /= w2.sum()
    want = np.zeros_like(x)
    for i in range(x.shape[0]):
        for j in range(x.shape[1]):
            m = {"x": 0.0, "y": 0.0, "xx": 0.0, "yy": 0.0, "xy": 0.0}
            for a in range(-5, 6):
                for b in range(-5, 6):
                    ii, jj = i + a, j + b
                    if 0 <= ii < x.shape[0] and 0 <= jj < x.shape[1]:
                        ww = w2[a + 5, b + 5]
                        m["x"] += ww * x[ii, jj]
                        m["y"] += ww * y[ii, jj]
                        m["xx"] += ww * x[ii, jj] ** 2
                        m["yy"] += ww * y[ii, jj] ** 2
                        m["xy"] += ww * x[ii, jj] * y[ii, jj]
            vx = m["xx"] - m["x"] ** 2
            vy = m["yy"] - m["y"] ** 2
            cxy = m["xy"] - m["x"] * m["y"]
            want[i, j] = ((2 * m["x"] * m["y"] + 1e-4) * (2 * cxy + 9e-4)) / \
                ((m["x"] ** 2 + m["y"] ** 2 + 1e-4) * (vx + vy + 9e-4))
    assert np.allclose(oracle.ssim_map(x[None], y[None])[0], want, rtol=0, atol=1e-12)


def test_ssim_invariants_and_constant_images():
    r = rng(3)
    x = r.uniform(0.0, 5.0, (2, 20, 24))
    y = r.uniform(0.0, 5.0, (2, 20, 24))
    assert np.allclose(oracle.ssim_map(x, x), 1.0, atol=1e-12)
    assert np.allclose(oracle.ssim_map(x, y), oracle.ssim_map(y, x), atol=1e-14)
    # constant images: away from the border the window sees no padding, the
    # variances vanish and SSIM = (2ab + C1) / (a^2 + b^2 + C1)
    a, b = 0.7, 1.9
    s = oracle.ssim_map(np.full((1, 30, 30), a), np.full((1, 30, 30), b))[0]
    want = (2 * a * b + 1e-4) / (a * a + b * b + 1e-4)
    assert np.allclose(s[5:-5, 5:-5], want, rtol=1e-12)
    assert not np.allclose(s[0, 0], want)      # the padding shows at the border


def test_l1_dssim_values():
    r = rng(4)
    y = r.uniform(0.0, 2.0, (3, 16, 18))
    loss, _ = oracle.l1_dssim_loss(y, y)
    assert abs(loss) < 1e-12                      # identical: both terms vanish
    c = 0.25
    sgn = np.where(r.uniform(size=y.shape) < 0.5, -1.0, 1.0)
    loss, _ = oracle.l1_dssim_loss(y + c * sgn, y, lam=0.0)
    assert abs(loss - c) < 1e-12                  # pure L1: mean |x - y|
    x = r.uniform(0.0, 2.0, y.shape)
    l_full, _ = oracle.l1_dssim_loss(x, y, lam=0.25)
    l_l1, _ = oracle.l1_dssim_loss(x, y, lam=0.0)
    ssim = oracle.ssim_map(x, y).mean(axis=(1, 2))
    assert abs(l_full - (l_l1 + 0.25 * np.mean(1.0 - ssim))) < 1e-12


def test_l1_dssim_gradient_finite_differences():
    r = rng(5)
    y = r.uniform(0.5, 2.0, (2, 13, 15))
    x = y + np.where(r.uniform(size=y.shape) < 0.5, -1.0, 1.0) * r.uniform(0.05, 0.3, y.shape)
    _, g = oracle.l1_dssim_loss(x, y)
    h = 1e-6
    for idx in [(0, 0, 0), (0, 6, 7), (1, 12, 14), (1, 3, 9), (0, 12, 1)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (oracle.l1_dssim_loss(xp, y)[0] - oracle.l1_dssim_loss(xm, y)[0]) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (idx, fd, g[idx])


# ------------------------------------------------------------------ TV, Eq. 11

def test_tv_ramp_closed_form_and_constant():
    n = (10, 9, 8)
    i, j, k = np.meshgrid(*[np.arange(m, dtype=np.float64) for m in n], indexing="ij")
    a, b, c = 0.5, -1.25, 2.0
    vol = a * i + b * j + c * k
    D = 4
    loss, g = oracle.tv_loss(vol, (3, 2, 1), D, weight=1.0)
    # each axis has D - 1 differences along it times D^2 lines, each |slope|
    assert abs(loss - (D - 1) * D * D * (abs(a) + abs(b) + abs(c)) / D ** 3) < 1e-12
    assert oracle.tv_loss(np.full(n, 3.0), (0, 0, 0), D)[0] == 0.0
    assert np.all(g[:3] == 0) and np.all(g[7:] == 0)       # zero outside the block


def test_tv_brute_force_and_gradient():
    r = rng(6)
    vol = r.normal(size=(7, 6, 8))
    corner, D, wgt = (2, 1, 3), 4, 0.05
    loss, g = oracle.tv_loss(vol, corner, D, weight=wgt)
    s = 0.0
    for p in np.ndindex(D, D, D):
        q = tuple(c + x for c, x in zip(corner, p))
        for a in range(3):
            if p[a] + 1 < D:
                q2 = list(q)
                q2[a] += 1
                s += abs(vol[tuple(q2)] - vol[q])
    assert abs(loss - wgt * s / D ** 3) < 1e-12
    h = 1e-7
    for idx in [(2, 1, 3), (3, 2, 4), (5, 4, 6), (4, 1, 5), (0, 0, 0)]:
        vp, vm = vol.copy(), vol.copy()
        vp[idx] += h
        vm[idx] -= h
        fd = (oracle.tv_loss(vp, corner, D, wgt)[0] - oracle.tv_loss(vm, corner, D, wgt)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-7, (idx, fd, g[idx])


# ------------------------------------------------------------ normality, Eq. 13

def test_mbc_normality_values_and_gradient():
    r = rng(7)
    # unit-norm channels give zero; channels s*u with |u| = 1 give (s^2 - 1)^2
    u = [r.normal(size=(3, 4, 5, 6)), r.normal(size=(3, 2, 3, 2))]
    u = [b / np.sqrt((b.reshape(3, -1) ** 2).sum(axis=1))[:, None, None, None] for b in u]
    assert abs(oracle.mbc_normality_loss(u)[0]) < 1e-24
    s = np.array([0.5, 1.5, 2.0])
    scaled = [b * s[:, None, None, None] for b in u]
    want = 2 * np.sum((s ** 2 - 1) ** 2) / 6
    assert abs(oracle.mbc_normality_loss(scaled)[0] - want) < 1e-12
    # gradient by central differences
    bases = [r.normal(0.0, 0.3, (3, 4, 5, 6)), r.normal(0.0, 0.5, (3, 2, 3, 2))]
    loss, g = oracle.mbc_normality_loss(bases, weight=1.0)
    h = 1e-6
    for l, idx in [(0, (0, 1, 2, 3)), (0, (2, 3, 4, 5)), (1, (1, 0, 2, 1)), (1, (2, 1, 1, 0))]:
        bp = [b.copy() for b in bases]
        bm = [b.copy() for b in bases]
        bp[l][idx] += h
        bm[l][idx] -= h
        fd = (oracle.mbc_normality_loss(bp)[0] - oracle.mbc_normality_loss(bm)[0]) / (2 * h)
        assert abs(fd - g[l][idx]) < 1e-7 * max(1.0, abs(fd)), (l, idx, fd, g[l][idx])
