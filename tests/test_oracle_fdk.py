"""Pins of the oracle's FDK reconstruction (the initialisation of Sec. 2.3.2,
Feldkamp et al. 1984) against facts that do not come from it: the Ram-Lak
kernel's closed form and its response to a constant row, and reconstructions
of analytic ball phantoms (exact chord-length projections): the density
inside, zero outside, and the position of an off-centre ball.  The
grid-based sampling of the FDK image into Gaussians: a full lattice returns
the voxel centres and values themselves, a linear image is sampled exactly
at the lattice points, and Gaussians of scale delta / sqrt(2 pi) on a
constant image voxelize back to that constant on average."""
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


def _grid_axes(grid):
    return [np.asarray(grid.center[i]) + (np.arange(grid.n[i]) - (grid.n[i] - 1) / 2.0) * grid.h[i]
            for i in range(3)]


def test_grid_init_full_lattice_is_the_voxels():
    grid = Grid((6, 5, 4), (1.5, 2.0, 2.5), (3.0, -1.0, 0.5))
    vol = np.random.default_rng(0).uniform(0.0, 1.0, grid.n)
    mean, sc, quat, val = fdk.grid_init(vol, grid, grid.n, 0.7)
    X, Y, Z = np.meshgrid(*_grid_axes(grid), indexing="ij")
    assert np.allclose(mean, np.stack([X, Y, Z], -1).reshape(-1, 3), rtol=0, atol=1e-12)
    assert np.allclose(val[:, 0], vol.reshape(-1), rtol=0, atol=1e-12)
    assert np.all(sc == 0.7) and np.all(quat == [1.0, 0.0, 0.0, 0.0])


def test_grid_init_linear_image_and_spacing():
    grid = Grid((12, 14, 9), (1.0, 1.5, 2.0), (-2.0, 1.0, 4.0))
    X, Y, Z = np.meshgrid(*_grid_axes(grid), indexing="ij")
    lin = lambda x, y, z: 0.3 * x - 0.2 * y + 0.05 * z + 1.0
    vol = lin(X, Y, Z)
    m = (5, 7, 3)
    mean, _, _, val = fdk.grid_init(vol, grid, m, 1.0)
    assert mean.shape == (105, 3)
    assert np.allclose(val[:, 0], lin(mean[:, 0], mean[:, 1], mean[:, 2]), rtol=0, atol=1e-10)
    P = mean.reshape(m + (3,))
    for a in range(3):
        L = grid.n[a] * grid.h[a]
        d = np.diff(np.moveaxis(P[..., a], a, 0), axis=0)
        assert np.allclose(d, L / m[a], rtol=0, atol=1e-12)
        first = np.moveaxis(P[..., a], a, 0)[0]
        assert np.allclose(first, grid.center[a] - 0.5 * L + 0.5 * L / m[a], rtol=0, atol=1e-12)


def test_grid_init_scale_preserves_the_mean_density():
    """With spacing delta and scale delta / sqrt(2 pi) each Gaussian's
    integral rho (2 pi)^(3/2) s^3 equals rho delta^3, so a constant image
    voxelizes back to the same constant on average (the lattice ripple
    averages out; untruncated Gaussians)."""
    import oracle
    from paper_2503_22139_amd.synth import GaussSet
    oracle.build()
    grid = Grid((40, 40, 40), (1.0, 1.0, 1.0))
    rho = 2.0
    vol = np.full(grid.n, rho)
    m = (10, 10, 10)
    delta = 4.0
    mean, sc, quat, val = fdk.grid_init(vol, grid, m, delta / math.sqrt(2 * math.pi))
    f = oracle.voxelize(GaussSet(mean, sc, quat, val), grid, float("inf")).reshape(grid.n)
    inner = f[12:28, 12:28, 12:28]
    assert abs(inner.mean() - rho) < 0.01 * rho, inner.mean()
