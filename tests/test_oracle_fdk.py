"""Pins of the oracle's FDK reconstruction (the initialisation of Sec. 2.3.2,
Feldkamp et al. 1984) against facts that do not come from it: the Ram-Lak
kernel's closed form and its response to a constant row, and reconstructions
of analytic ball phantoms (exact chord-length projections): the density
inside, zero outside, and the position of an off-centre ball."""
import math

import numpy as np

from oracle import fdk
from paper_2503_22139_amd.synth import Cone, Grid


def test_ramlak_kernel():
    tau = 0.8
    h = fdk.ramlak(6, tau)
    k = np.arange(-5, 6)
    kk = np.where(k == 0, 1, k)
    want = np.where(k == 0, 1 / (4 * tau * tau), np.where(k % 2 != 0, -1 / (math.pi * kk * tau) ** 2, 0.0))
    assert np.allclose(h, want, rtol=0, atol=1e-15)
    # the full (infinite) kernel sums to zero: it removes the mean of a long row
    big = fdk.ramlak(20001, tau)
    assert abs(big.sum() * tau) < 1e-4 / tau


def test_ball_density_inside_and_zero_outside():
    cone = Cone(1000.0, 1500.0, 128, 96, 1.6, 1.6)
    V = 180
    ang = 2 * np.pi * np.arange(V) / V
    rho, r = 0.02, 40.0
    p = fdk.ball_projections([0, 0, 0], r, rho, cone, ang)
    grid = Grid((48, 48, 24), (2.0, 2.0, 2.0))
    f = fdk.fdk(p, cone, ang, grid)
    ax = [(np.arange(grid.n[i]) - (grid.n[i] - 1) / 2.0) * grid.h[i] for i in range(3)]
    X, Y, Z = np.meshgrid(*ax, indexing="ij")
    R = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    inside = f[R < 30.0]
    assert abs(inside.mean() - rho) < 0.02 * rho, inside.mean()
    assert inside.std() < 0.03 * rho
    assert np.abs(f[R > 50.0]).mean() < 0.05 * rho


def test_off_centre_ball_position():
    cone = Cone(1000.0, 1500.0, 96, 72, 1.6, 1.6, off_u=0.5)
    V = 120
    ang = 2 * np.pi * np.arange(V) / V
    c = np.array([14.0, -10.0, 6.0])
    p = fdk.ball_projections(c, 8.0, 0.05, cone, ang)
    grid = Grid((40, 40, 24), (1.5, 1.5, 1.5))
    f = fdk.fdk(p, cone, ang, grid)
    ax = [(np.arange(grid.n[i]) - (grid.n[i] - 1) / 2.0) * grid.h[i] for i in range(3)]
    X, Y, Z = np.meshgrid(*ax, indexing="ij")
    wgt = np.clip(f, 0.0, None) * (f > 0.5 * f.max())
    centroid = np.array([(wgt * X).sum(), (wgt * Y).sum(), (wgt * Z).sum()]) / wgt.sum()
    assert np.linalg.norm(centroid - c) < 0.5, centroid
    assert abs(f[np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) < 4.0].mean() - 0.05) < 0.003
