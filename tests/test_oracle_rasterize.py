"""Pins of the oracle's X-ray Gaussian rasterizer (Eq. 7-9) against facts that
do not come from it: the exact line integral of a 3-D Gaussian (closed form,
itself checked by quadrature), the exactness of the local affine
approximation on the central ray, its first-order convergence as the source
recedes, the truncation ellipse, and finite differences of the autograd
gradients."""
import math

import numpy as np
import torch

from oracle import rasterize as R
from paper_2503_22139_amd.synth import Cone, GaussSet


def one(mu, s, q=(1.0, 0.0, 0.0, 0.0), rho=1.0):
    return GaussSet(np.array([mu], float), np.array([s], float), np.array([q], float),
                    np.array([[rho]], float))


CASES = [([10.0, -8.0, 6.0], [3.0, 1.5, 2.0], [0.9, 0.2, -0.3, 0.1], 1.1),
         ([5.0, 8.0, -4.0], [1.0, 4.0, 2.0], [0.5, 0.5, 0.5, 0.5], 2.5),
         ([-12.0, 3.0, 9.0], [0.8, 0.6, 1.2], [0.3, -0.4, 0.8, 0.2], 4.0)]


def test_line_integral_closed_form_by_quadrature():
    cone = Cone(1000.0, 1500.0, 9, 7, 2.0, 2.0)
    mu, s, q, th = CASES[0]
    ex = R.line_integral(mu, s, q, 0.7, cone, th)
    ct, st = math.cos(th), math.sin(th)
    o = np.array([1000 * ct, 1000 * st, 0.0])
    Rm = R._rotation(torch.tensor([q], dtype=torch.float64))[0].numpy()
    A = Rm @ np.diag(1.0 / np.array(s) ** 2) @ Rm.T
    for iv, iu in [(3, 4), (0, 0), (6, 8), (2, 5)]:
        a, b = (iu - 4) * 2.0, (iv - 3) * 2.0
        p = -500.0 * np.array([ct, st, 0.0]) + a * np.array([-st, ct, 0.0]) + b * np.array([0, 0, 1.0])
        d = (p - o) / np.linalg.norm(p - o)
        t = np.linspace(900.0, 1100.0, 400001)
        x = o + t[:, None] * d - np.array(mu)
        quad = np.trapezoid(0.7 * np.exp(-0.5 * np.einsum("pi,ij,pj->p", x, A, x)), t)
        assert abs(quad - ex[iv, iu]) <= 1e-9 * max(1.0, ex.max()), (iv, iu, quad, ex[iv, iu])


def test_central_ray_is_exact():
    """On the central ray the affine map is exact: an isotropic Gaussian gives
    rho sqrt(2 pi) sigma at the central pixel, at any depth."""
    cone = Cone(1000.0, 1500.0, 21, 15, 0.8, 0.8)
    for depth, sig, th in [(0.0, 2.0, 0.0), (60.0, 1.3, 0.7), (-80.0, 3.5, 2.2)]:
        ct, st = math.cos(th), math.sin(th)
        mu = [-depth * ct, -depth * st, 0.0]      # on the line source -> detector centre
        img = R.rasterize(one(mu, [sig] * 3, rho=0.4), cone, [th], k=float("inf"))[0]
        assert abs(img[7, 10] - 0.4 * math.sqrt(2 * math.pi) * sig) < 1e-12


def test_matches_exact_line_integrals_in_the_field_of_view():
    """Anisotropic, rotated Gaussians within 15 mm of the isocentre on a
    detector with pixel offsets: the splat matches the exact line integrals
    to the size of the local affine approximation (~1e-3 of the peak)."""
    cone = Cone(1000.0, 1500.0, 121, 101, 0.6, 0.6, off_u=0.3, off_v=-0.2)
    for mu, s, q, th in CASES:
        img = R.rasterize(one(mu, s, q, 0.7), cone, [th], k=float("inf"))[0]
        ex = R.line_integral(mu, s, q, 0.7, cone, th)
        assert np.abs(img - ex).max() <= 2e-3 * ex.max(), (mu, np.abs(img - ex).max() / ex.max())
        a = np.array(np.unravel_index(np.argmax(img), img.shape))
        b = np.array(np.unravel_index(np.argmax(ex), ex.shape))
        assert np.abs(a - b).max() <= 1, (a, b)       # same peak (up to a near-tie)


def test_first_order_convergence_as_the_source_recedes():
    """Scaling SAD and SDD by f (same magnification and pixel pitch) shrinks
    the affine approximation's error about f-fold."""
    mu, s, q, th = CASES[0]
    errs = []
    for f in (1.0, 10.0):
        cone = Cone(1000.0 * f, 1500.0 * f, 121, 101, 0.6, 0.6)
        img = R.rasterize(one(mu, s, q, 0.7), cone, [th], k=float("inf"))[0]
        ex = R.line_integral(mu, s, q, 0.7, cone, th)
        errs.append(np.abs(img - ex).max() / ex.max())
    assert errs[1] < errs[0] / 5.0, errs


def test_truncation_ellipse():
    cone = Cone(1000.0, 1500.0, 61, 51, 0.6, 0.6)
    mu, s, q, th = CASES[2]
    g = one(mu, s, q, 0.7)
    full = R.rasterize(g, cone, [th], k=float("inf"))[0]
    cut = R.rasterize(g, cone, [th], k=3.0)[0]
    inside = cut > 0
    assert inside.sum() > 20 and (~inside).sum() > 20
    assert np.allclose(cut[inside], full[inside], rtol=0, atol=1e-14)
    assert full[~inside].max() <= 0.7 * math.sqrt(2 * math.pi) * 1.3 * math.exp(-4.5) * 1.01


def test_gradients_finite_differences():
    rng = np.random.default_rng(3)
    cone = Cone(1000.0, 1500.0, 23, 17, 1.2, 1.2)
    gs = GaussSet(rng.uniform(-6, 6, (4, 3)), rng.uniform(1.0, 2.5, (4, 3)),
                  rng.normal(size=(4, 4)), rng.uniform(0.2, 1.0, (4, 1)))
    ang = [0.4, 2.0]
    gp = rng.normal(size=(2, 17, 23))
    g = R.rasterize_bwd(gs, cone, ang, float("inf"), gp)

    def f(mean=gs.mean, scale=gs.scale, quat=gs.quat, value=gs.value):
        return float((R.rasterize(GaussSet(mean, scale, quat, value), cone, ang,
                                  float("inf")) * gp).sum())
    h = 1e-6
    for name, arr in (("mean", gs.mean), ("scale", gs.scale), ("quat", gs.quat), ("value", gs.value)):
        for idx in [(0, 0), (2, arr.shape[1] - 1), (3, 1 % arr.shape[1])]:
            ap, am = arr.copy(), arr.copy()
            ap[idx] += h
            am[idx] -= h
            fd = (f(**{name: ap}) - f(**{name: am})) / (2 * h)
            assert abs(fd - g[name][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, g[name][idx])
