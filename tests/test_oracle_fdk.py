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


# ------------------------------------------------ the two FDK weights, wide fan

WIDE = dict(sad=80.0, sdd=120.0)


def test_backprojection_weight_closed_form():
    """With q = 1 on every pixel (a detector large enough that every point
    projects inside) the back-projection is (1/2) sum_views dtheta (SAD/U)^2
    = pi * mean over views of (SAD/U)^2, U the point's distance from the
    source along the central ray: computed here from the source position
    alone.  Short SAD, so the weight ranges over a factor of ~5."""
    cone = Cone(WIDE["sad"], WIDE["sdd"], 801, 61, 1.0, 1.0)
    V = 37
    ang = 2 * np.pi * np.arange(V) / V + 0.1
    pts = np.array([[0.0, 0.0, 0.0], [30.0, -12.0, 4.0], [-25.0, 20.0, -6.0], [5.0, 38.0, 0.0]])
    f = fdk.backproject(np.ones((V, cone.nv, cone.nu)), cone, ang, None, points=pts)
    want = np.zeros(len(pts))
    for th in ang:
        src = cone.sad * np.array([math.cos(th), math.sin(th), 0.0])
        axis = -src / np.linalg.norm(src)               # central ray direction
        U = (pts - src) @ axis
        want += (cone.sad / U) ** 2
    want *= math.pi / V
    assert np.allclose(f, want, rtol=1e-12, atol=0)
    assert want.max() / want.min() > 1.3


def test_filter_cosine_weight_impulse():
    """An impulse at a far off-axis pixel is filtered into the Ram-Lak
    kernel along its row, times tau and the cosine of the pixel's ray with
    the central ray (SDD over the source-pixel distance, from the pixel's
    position in space); here that cosine is ~0.74."""
    cone = Cone(WIDE["sad"], WIDE["sdd"], 41, 9, 6.0, 6.0)
    iu, iv = 38, 8
    p = np.zeros((1, cone.nv, cone.nu))
    p[0, iv, iu] = 1.0
    q = fdk.filter_rows(p, cone)
    src = np.array([cone.sad, 0.0, 0.0])
    pix = np.array([-(cone.sdd - cone.sad), (iu - 0.5 * (cone.nu - 1)) * cone.du,
                    (iv - 0.5 * (cone.nv - 1)) * cone.dv])
    cos_ray = cone.sdd / np.linalg.norm(pix - src)
    tau = cone.du * cone.sad / cone.sdd
    h = fdk.ramlak(cone.nu, tau)
    want = tau * cos_ray * h[np.arange(cone.nu) - iu + cone.nu - 1]
    assert np.allclose(q[0, iv], want, rtol=1e-13, atol=0)
    assert np.all(q[0, :iv] == 0) and cos_ray < 0.75


def test_wide_fan_ball_density_in_mid_plane():
    """FDK is exact in the mid-plane of a full circular scan (there it is
    fan-beam filtered back-projection) as long as no view truncates the
    object.  A ball 40 mm off the axis with a source only 80 mm from it: the
    ball's rays make fan angles up to ~32 degrees (cosine weights down to
    ~0.85) and (SAD/U)^2 averages ~1.5 at its centre, so dropping or
    misplacing either weight moves the density by far more than 5%.  The
    detector (+-135 mm at SDD, a 59 mm field of view) holds the ball (50 mm
    from the axis at most) in every view.  The mid-plane density inside the
    ball is pinned to 0.5%."""
    cone = Cone(WIDE["sad"], WIDE["sdd"], 675, 3, 0.4, 0.4)
    V = 360
    ang = 2 * np.pi * np.arange(V) / V
    c, r, rho = np.array([40.0, 0.0, 0.0]), 10.0, 0.02
    p = fdk.ball_projections(c, r, rho, cone, ang)
    rng = np.random.default_rng(5)
    phi = rng.uniform(0, 2 * np.pi, 40)
    rad = 8.0 * np.sqrt(rng.uniform(0, 1, 40))
    pts = np.stack([c[0] + rad * np.cos(phi), c[1] + rad * np.sin(phi), np.zeros(40)], 1)
    f = fdk.fdk(p, cone, ang, None, points=pts)
    assert np.all(np.abs(f - rho) < 0.005 * rho), (f.min() / rho, f.max() / rho)
    # the weights at the ball's centre are far from one
    U = cone.sad - (c[0] * np.cos(ang) + c[1] * np.sin(ang))
    assert np.mean((cone.sad / U) ** 2) > 1.3
    lat = -c[0] * np.sin(ang) + c[1] * np.cos(ang)
    assert np.min(np.cos(np.arctan(np.abs(lat) / U))) < 0.9
