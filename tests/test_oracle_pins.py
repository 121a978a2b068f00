"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test checks one function of ``oracle/`` against a closed form, a library
routine (scipy's rotation and interpolation), brute force on a tiny input or
an invariant that the mathematics fixes.  The paper prints no worked numeric
example, so every pin is analytic or structural.
"""
import math

import numpy as np
import pytest
from scipy.ndimage import map_coordinates
from scipy.spatial.transform import Rotation
from scipy.stats import chi2

import oracle
from paper_2503_22139_amd import synth
from paper_2503_22139_amd.synth import Cone, GaussSet, Grid


def one_gaussian(mu, s, q=(1.0, 0.0, 0.0, 0.0), rho=1.0):
    return GaussSet(np.array([mu], np.float64), np.array([s], np.float64),
                    np.array([q], np.float64), np.array([[rho]], np.float64))


def centres(grid):
    g = [np.asarray(grid.center[a]) + (np.arange(grid.n[a]) - (grid.n[a] - 1) / 2.0) * grid.h[a]
         for a in range(3)]
    return np.meshgrid(*g, indexing="ij")


# ------------------------------------------------------------------ Eq. 4/5

def test_voxelize_point_values():
    """Isotropic Gaussian on a voxel centre: rho there, rho exp(-h^2/2s^2) one voxel away."""
    grid = Grid((9, 9, 9), (1.0, 1.5, 2.0))
    X = centres(grid)
    mu = [X[0][4, 4, 4], X[1][4, 4, 4], X[2][4, 4, 4]]
    sig = 1.3
    v = oracle.voxelize(one_gaussian(mu, [sig] * 3, rho=0.7), grid, 3.0)[0]
    assert abs(v[4, 4, 4] - 0.7) < 1e-15
    for a, h in enumerate(grid.h):
        idx = [4, 4, 4]
        idx[a] = 5
        assert abs(v[tuple(idx)] - 0.7 * math.exp(-h * h / (2 * sig * sig))) < 1e-15


def test_voxelize_matches_scipy_rotation_bruteforce():
    """Brute force over every (voxel, Gaussian) pair, with the rotation matrix
    from scipy (scalar-last quaternions) and Sigma^-1 from a matrix inverse."""
    rng = np.random.default_rng(11)
    grid = Grid((10, 9, 8), (1.0, 1.25, 1.5), (0.3, -0.2, 0.1))
    gs = synth.gaussians(rng, 40, grid, s_vox=(0.6, 2.5), rho=(-0.5, 1.0))
    gs.quat = (gs.quat * rng.uniform(0.5, 2.0, (40, 1))).astype(np.float32)   # unnormalised
    X = np.stack(centres(grid), -1).reshape(-1, 3)
    for k in (3.0, math.inf):
        ref = np.zeros(X.shape[0])
        for i in range(gs.m):
            q = gs.quat[i].astype(np.float64)
            R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
            S = np.diag(gs.scale[i].astype(np.float64) ** 2)
            A = np.linalg.inv(R @ S @ R.T)
            d = X - gs.mean[i].astype(np.float64)
            m = np.einsum("pa,ab,pb->p", d, A, d)
            ref += np.where(m <= k * k, gs.value[i, 0] * np.exp(-0.5 * m), 0.0)
        got = oracle.voxelize(gs, grid, k)[0].reshape(-1)
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_voxelize_multichannel_signed():
    """Signed multi-channel values: channel c equals a one-channel run with value[:, c]."""
    rng = np.random.default_rng(12)
    grid = Grid((12, 11, 10), (2.0, 2.0, 2.5))
    gs = synth.gaussians(rng, 30, grid, c=5, value_sigma=2.0)
    full = oracle.voxelize(gs, grid, 3.0)
    for c in range(5):
        one = GaussSet(gs.mean, gs.scale, gs.quat, gs.value[:, c:c + 1])
        assert np.array_equal(full[c], oracle.voxelize(one, grid, 3.0)[0])


def test_voxelize_mass_closed_form():
    """Untruncated lattice sum times voxel volume = rho (2 pi)^(3/2) s1 s2 s3;
    truncated at 3 sigma the fraction is P(chi2_3 <= 9)."""
    grid = Grid((48, 48, 48), (1.0, 1.0, 1.0))
    q = np.array([0.8, 0.3, -0.4, 0.33])
    s = np.array([2.2, 3.1, 2.6])
    g = one_gaussian([0.21, -0.37, 0.11], s, q / np.linalg.norm(q) * 1.7, rho=0.9)
    exact = 0.9 * (2 * math.pi) ** 1.5 * np.prod(s)
    un = oracle.voxelize(g, grid, math.inf).sum()
    assert abs(un - exact) / exact < 1e-8
    tr = oracle.voxelize(g, grid, 3.0).sum()
    assert abs(tr / exact - chi2.cdf(9.0, 3)) < 5e-3
    assert abs(chi2.cdf(9.0, 3) - 0.970709) < 1e-6


def test_voxelize_quaternion_invariances():
    rng = np.random.default_rng(13)
    grid = Grid((14, 13, 12), (1.0, 1.0, 1.5))
    gs = synth.gaussians(rng, 20, grid)
    base = oracle.voxelize(gs, grid, 3.0)
    for f in (-1.0, 2.5, 0.3):
        g2 = gs.copy()
        g2.quat = gs.quat.astype(np.float64) * f
        assert np.max(np.abs(oracle.voxelize(g2, grid, 3.0) - base)) < 1e-14
    # a 90-degree turn about z swaps the first two scales
    s = np.array([1.1, 2.7, 1.9])
    mu = [0.4, -0.2, 0.3]
    c = math.cos(math.pi / 4)
    a = oracle.voxelize(one_gaussian(mu, s, (c, 0.0, 0.0, c)), grid, 3.0)
    b = oracle.voxelize(one_gaussian(mu, s[[1, 0, 2]]), grid, 3.0)
    assert np.max(np.abs(a - b)) < 1e-14


def test_voxelize_superposition():
    rng = np.random.default_rng(14)
    grid = Grid((16, 12, 10), (1.5, 1.5, 2.0))
    a = synth.gaussians(rng, 25, grid, c=2, value_sigma=1.0)
    b = synth.gaussians(rng, 17, grid, c=2, value_sigma=1.0)
    ab = GaussSet(*[np.concatenate([x, y]) for x, y in
                    zip((a.mean, a.scale, a.quat, a.value), (b.mean, b.scale, b.quat, b.value))])
    d = oracle.voxelize(ab, grid, 3.0) - oracle.voxelize(a, grid, 3.0) - oracle.voxelize(b, grid, 3.0)
    assert np.max(np.abs(d)) < 1e-13


def test_voxelize_truncation_bound():
    """Untruncated minus truncated is at most sum |rho| e^-4.5 per voxel."""
    rng = np.random.default_rng(15)
    grid = Grid((12, 12, 12), (1.0, 1.0, 1.0))
    gs = synth.gaussians(rng, 50, grid, rho=(0.0, 1.0))
    d = oracle.voxelize(gs, grid, math.inf) - oracle.voxelize(gs, grid, 3.0)
    assert d.min() >= 0.0
    assert d.max() <= np.abs(gs.value).sum() * math.exp(-4.5)


# ---------------------------------------------------------------- sample3d

def test_sample3d_matches_scipy_trilinear():
    """Inside the voxel-centre hull and on the half-voxel rim, trilinear
    interpolation equals scipy's order-1 map_coordinates (edge clamped);
    beyond the box the value is zero."""
    rng = np.random.default_rng(16)
    grid = Grid((7, 6, 5), (1.0, 2.0, 1.5), (0.5, -1.0, 0.25))
    vol = rng.normal(size=grid.n)
    lo, hi = grid.box()
    pts = lo - 0.2 * (hi - lo) + 1.4 * (hi - lo) * rng.random((4000, 3))
    got = oracle.sample_points(vol, grid, pts)
    c0 = np.asarray(grid.center) - (np.asarray(grid.n) - 1) / 2.0 * np.asarray(grid.h)
    u = (pts - c0) / np.asarray(grid.h)
    inside = np.all((u >= -0.5) & (u <= np.asarray(grid.n) - 0.5), axis=1)
    ref = map_coordinates(vol, u.T, order=1, mode="nearest")
    assert inside.sum() > 500 and (~inside).sum() > 500
    assert np.max(np.abs(got[inside] - ref[inside])) < 1e-13
    assert np.all(got[~inside] == 0.0)


def test_sample3d_gradient_fd():
    rng = np.random.default_rng(17)
    grid = Grid((7, 6, 5), (1.0, 2.0, 1.5))
    vol = rng.normal(size=grid.n)
    c0 = -(np.asarray(grid.n) - 1) / 2.0 * np.asarray(grid.h)
    u = 0.05 + rng.random((300, 3)) * (np.asarray(grid.n) - 1.1)
    pts = c0 + u * np.asarray(grid.h)
    _, g = oracle.sample_points(vol, grid, pts, grad=True)
    eps = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = eps
        fd = (oracle.sample_points(vol, grid, pts + e) - oracle.sample_points(vol, grid, pts - e)) / (2 * eps)
        frac = np.abs(u[:, a] - np.round(u[:, a]))
        ok = frac > 1e-4                                          # away from cell planes
        assert np.max(np.abs(fd[ok] - g[ok, a])) < 1e-7


# ------------------------------------------------------------------- Eq. 2

def test_warp_identity_and_shifts():
    rng = np.random.default_rng(18)
    grid = Grid((10, 9, 8), (1.0, 1.5, 2.0))
    ref = rng.normal(size=grid.n)
    zero = np.zeros((1, 3) + grid.n)
    assert np.max(np.abs(oracle.warp(ref, grid, zero)[0] - ref)) < 1e-13
    # integer shift by +2 voxels along y: out[:, j] = ref[:, j + 2], zero beyond
    d = np.zeros((1, 3) + grid.n)
    d[0, 1] = 2 * grid.h[1]
    out = oracle.warp(ref, grid, d)[0]
    assert np.max(np.abs(out[:, :-2] - ref[:, 2:])) < 1e-13
    assert np.all(out[:, -2:] == 0.0)
    # fractional shift of a volume linear along z: exact inside
    X = centres(grid)
    lin = 0.3 * X[2] + 1.0
    d = np.zeros((1, 3) + grid.n)
    d[0, 2] = 0.37 * grid.h[2]
    out = oracle.warp(lin, grid, d)[0]
    assert np.max(np.abs(out[:, :, :-1] - (lin[:, :, :-1] + 0.3 * 0.37 * grid.h[2]))) < 1e-12


def test_warp_matches_scipy_interior():
    rng = np.random.default_rng(19)
    grid = Grid((9, 8, 7), (1.5, 1.5, 2.0))
    ref = rng.normal(size=grid.n)
    dvf = rng.normal(0.0, 1.5, (2, 3) + grid.n)
    out = oracle.warp(ref, grid, dvf)
    X = np.stack(centres(grid), 0)
    c0 = -(np.asarray(grid.n) - 1) / 2.0 * np.asarray(grid.h)
    for v in range(2):
        u = (X + dvf[v] - c0[:, None, None, None]) / np.asarray(grid.h)[:, None, None, None]
        inside = np.all((u >= -0.5) & (u <= (np.asarray(grid.n) - 0.5)[:, None, None, None]), axis=0)
        ref_v = map_coordinates(ref, u.reshape(3, -1), order=1, mode="nearest").reshape(grid.n)
        assert np.max(np.abs(np.where(inside, ref_v, 0.0) - out[v])) < 1e-13


# ------------------------------------------------------------------- Eq. 3

def test_combine_upsample_reproduces_affine_field():
    """A coarse basis that is affine in x is reproduced exactly at fine voxel
    centres inside the coarse voxel-centre hull."""
    fine = Grid((24, 20, 16), (1.0, 1.2, 1.5))
    levels = synth.level_grids(fine, [(6, 5, 8), (12, 10, 16)])
    B = 2
    a = np.array([[0.3, -0.2, 0.1], [0.05, 0.4, -0.3]])
    bases = []
    for g in levels:
        Xl = centres(g)
        E = np.zeros((3 * B,) + g.n)
        for b in range(B):
            for k in range(3):
                E[b * 3 + k] = a[b, k] * Xl[k] + 0.5 * b - 0.25 * k
        bases.append(E)
    coeff = np.random.default_rng(20).normal(size=(3, 2, B, 3))
    dvf = oracle.combine(bases, levels, coeff, fine)
    X = centres(fine)
    c0 = np.asarray(levels[0].center) - (np.asarray(levels[0].n) - 1) / 2.0 * np.asarray(levels[0].h)
    c1 = c0 + (np.asarray(levels[0].n) - 1) * np.asarray(levels[0].h)
    hull = np.ones(fine.n, bool)
    for k in range(3):
        hull &= (X[k] >= c0[k]) & (X[k] <= c1[k])
    assert hull.sum() > 1000
    for v in range(3):
        for k in range(3):
            exp = sum(coeff[v, l, b, k] * (a[b, k] * X[k] + 0.5 * b - 0.25 * k)
                      for l in range(2) for b in range(B))
            assert np.max(np.abs(dvf[v, k][hull] - exp[hull])) < 1e-12


def test_combine_same_grid_is_weighted_sum():
    """When a level's grid equals the output grid, sampling is the identity."""
    g = Grid((8, 7, 6), (1.0, 1.0, 2.0))
    rng = np.random.default_rng(21)
    E = rng.normal(size=(3,) + g.n)
    coeff = rng.normal(size=(2, 1, 1, 3))
    dvf = oracle.combine([E], [g], coeff, g)
    for v in range(2):
        for k in range(3):
            assert np.max(np.abs(dvf[v, k] - coeff[v, 0, 0, k] * E[k])) < 1e-13


# ------------------------------------------------------------------- Eq. 6

def test_ray_geometry_magnification_isotropic_line_integral():
    """A ray through an isotropic Gaussian's centre integrates to
    rho sigma sqrt(2 pi) whatever its direction.  The centre is placed on the
    ray of a chosen pixel by similar triangles (detector coordinate = SDD/(SAD
    - depth) times the lateral offset), which pins the cone-beam geometry."""
    grid = Grid((128, 128, 112), (0.5, 0.5, 0.5))
    cone = Cone(1000.0, 1500.0, 33, 29, 0.6, 0.6)
    sig, rho = 4.0, 0.8
    for theta, (iu, iv) in ((0.0, (20, 9)), (1.1, (7, 21)), (3.9, (28, 14))):
        ct, st = math.cos(theta), math.sin(theta)
        depth = 3.0                                     # along the source direction
        u_mm = (iu - (cone.nu - 1) / 2) * cone.du
        v_mm = (iv - (cone.nv - 1) / 2) * cone.dv
        mag = cone.sdd / (cone.sad - depth)
        lat, ax = u_mm / mag, v_mm / mag
        mu = [depth * ct - lat * st, depth * st + lat * ct, ax]
        g = one_gaussian(mu, [sig] * 3, rho=rho)
        vol = oracle.voxelize(g, grid, math.inf)[0]
        p = oracle.project(vol, grid, cone, [theta])[0]
        want = rho * sig * math.sqrt(2 * math.pi)
        # trilinear interpolation across the two transverse axes is off by at
        # most h^2 / (8 sigma^2) each at the peak
        assert abs(p[iv, iu] - want) / want < 2 * grid.h[0] ** 2 / (8 * sig ** 2)
        assert p[iv, iu] == p.max()


def _box_chord_by_sampling(o, d, lo, hi, tmax, n=4_000_001):
    t = np.linspace(0.0, tmax, n)
    pts = o[None, :] + t[:, None] * d[None, :]
    inside = np.all((pts >= lo) & (pts <= hi), axis=1)
    return inside.sum() * (t[1] - t[0])


def test_chord_length_of_uniform_box():
    """All-ones volume: every pixel's value is its ray's chord through the box."""
    grid = Grid((20, 16, 12), (2.0, 2.5, 3.0), (1.0, -2.0, 0.5))
    cone = Cone(1000.0, 1500.0, 21, 17, 4.0, 4.0, step=0.0)
    ones = np.ones(grid.n)
    theta = 0.7
    p = oracle.project(ones, grid, cone, [theta])[0]
    info = oracle.ray_info(grid, cone, theta)
    assert np.max(np.abs(p - (info[..., 1] - info[..., 0]))) < 1e-12
    lo, hi = grid.box()
    ct, st = math.cos(theta), math.sin(theta)
    o = np.array([1000.0 * ct, 1000.0 * st, 0.0])
    for iu, iv in ((10, 8), (3, 14), (18, 2), (0, 0)):
        pix = (np.array([-500.0 * ct, -500.0 * st, 0.0]) + (iu - 10) * 4.0 * np.array([-st, ct, 0.0])
               + (iv - 8) * 4.0 * np.array([0.0, 0.0, 1.0]))
        d = (pix - o) / np.linalg.norm(pix - o)
        L = _box_chord_by_sampling(o, d, lo, hi, 1200.0)
        assert abs(p[iv, iu] - L) < 2e-3


def test_axis_aligned_central_ray_exact_sum():
    """theta = 0 (and 90 degrees): the central ray runs along x (y) through
    voxel centres, so the midpoint rule with step h/2 gives h * sum of the row."""
    rng = np.random.default_rng(22)
    grid = Grid((11, 9, 7), (1.0, 1.5, 2.0))
    vol = rng.random(grid.n)
    cone = Cone(1000.0, 1500.0, 5, 5, 1.0, 1.0, step=0.5)
    p = oracle.project(vol, grid, cone, [0.0])[0]
    assert abs(p[2, 2] - grid.h[0] * vol[:, 4, 3].sum()) < 1e-12
    p = oracle.project(vol, grid, cone, [math.pi / 2])[0]
    cone2 = Cone(1000.0, 1500.0, 5, 5, 1.0, 1.0, step=0.75)
    p2 = oracle.project(vol, grid, cone2, [math.pi / 2])[0]
    assert abs(p2[2, 2] - grid.h[1] * vol[5, :, 3].sum()) < 1e-12
    assert p.shape == (5, 5)


def test_anisotropic_gaussian_line_integral():
    """Voxelize (untruncated) then project converges to the closed form
    rho sqrt(2 pi / a) exp(-(c - b^2/a)/2), a = d'Ad, b = d'A(o-mu),
    c = (o-mu)'A(o-mu), at second order in h: halving h quarters the error,
    and the Richardson combination (4 P_h/2 - P_h)/3 is far closer still."""
    q = np.array([0.9, 0.2, -0.3, 0.25])
    s = np.array([5.0, 3.5, 4.0])
    mu = np.array([1.3, -2.1, 0.7])
    theta = 0.4
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]] / np.linalg.norm(q)).as_matrix()
    A = np.linalg.inv(R @ np.diag(s ** 2) @ R.T)
    ct, st = math.cos(theta), math.sin(theta)
    o = np.array([1000.0 * ct, 1000.0 * st, 0.0])
    want = np.zeros((7, 9))
    for iv in range(7):
        for iu in range(9):
            pix = (np.array([-500.0 * ct, -500.0 * st, 0.0]) + (iu - 4) * 3.0 * np.array([-st, ct, 0.0])
                   + (iv - 3) * 3.0 * np.array([0.0, 0.0, 1.0]))
            d = (pix - o) / np.linalg.norm(pix - o)
            a = d @ A @ d
            b = d @ A @ (o - mu)
            c = (o - mu) @ A @ (o - mu)
            want[iv, iu] = math.sqrt(2 * math.pi / a) * math.exp(-0.5 * (c - b * b / a))
    got = {}
    for h in (1.0, 0.5):
        grid = Grid((int(64 / h), int(64 / h), int(48 / h)), (h, h, h))
        cone = Cone(1000.0, 1500.0, 9, 7, 3.0, 3.0, step=h / 2)
        vol = oracle.voxelize(one_gaussian(mu, s, q), grid, math.inf)[0]
        got[h] = oracle.project(vol, grid, cone, [theta])[0]
    e1 = (got[1.0] - want) / want
    e2 = (got[0.5] - want) / want
    assert np.max(np.abs(e2)) < 1.5e-2
    big = np.abs(e1) > 5e-3
    ratio = e1[big] / e2[big]
    assert big.sum() > 20 and np.all((ratio > 3.5) & (ratio < 4.5)), ratio
    rich = (4.0 * got[0.5] - got[1.0]) / 3.0
    assert np.max(np.abs(rich - want) / want) < 1.5e-3


def test_line_integral_second_order():
    errs = {}
    for h in (1.0, 0.5):
        grid = Grid((int(40 / h), int(40 / h), int(40 / h)), (h, h, h))
        cone = Cone(1000.0, 1500.0, 3, 3, 2.0, 2.0, step=h / 2)
        g = one_gaussian([0.3, 0.1, -0.2], [3.0, 2.5, 2.0], (0.9, 0.3, 0.1, 0.2))
        vol = oracle.voxelize(g, grid, math.inf)[0]
        fine = oracle.voxelize(g, Grid((160, 160, 160), (0.25, 0.25, 0.25)), math.inf)[0]
        p = oracle.project(vol, grid, cone, [0.3])[0]
        pf = oracle.project(fine, Grid((160, 160, 160), (0.25, 0.25, 0.25)),
                            Cone(1000.0, 1500.0, 3, 3, 2.0, 2.0, step=0.125), [0.3])[0]
        errs[h] = np.max(np.abs(p - pf))
    ratio = errs[1.0] / errs[0.5]
    assert 3.0 < ratio < 5.5, errs


# ------------------------------------------------------------- adjoints (P10)

def _rel(a, b):
    return abs(a - b) / max(abs(a), abs(b), 1e-300)


def test_project_adjoint_identity():
    rng = np.random.default_rng(23)
    grid = Grid((14, 12, 10), (1.5, 1.5, 2.0))
    cone = Cone(1000.0, 1500.0, 19, 13, 1.6, 1.6)
    ang = np.array([0.1, 1.7, 4.0])
    x = rng.normal(size=(3,) + grid.n)
    y = rng.normal(size=(3, 13, 19))
    lhs = np.sum(oracle.project(x, grid, cone, ang, shared=False) * y)
    rhs = np.sum(x * oracle.project_bwd(y, grid, cone, ang, shared=False))
    assert _rel(lhs, rhs) < 1e-12
    xs = rng.normal(size=grid.n)
    lhs = np.sum(oracle.project(xs, grid, cone, ang, shared=True) * y)
    rhs = np.sum(xs * oracle.project_bwd(y, grid, cone, ang, shared=True))
    assert _rel(lhs, rhs) < 1e-12


def test_warp_adjoint_identity_in_ref():
    rng = np.random.default_rng(24)
    grid = Grid((10, 9, 8), (1.5, 1.5, 2.0))
    dvf = rng.normal(0, 2.0, (2, 3) + grid.n)
    x = rng.normal(size=grid.n)
    y = rng.normal(size=(2,) + grid.n)
    lhs = np.sum(oracle.warp(x, grid, dvf) * y)
    g_ref, _ = oracle.warp_bwd(x, grid, dvf, y)
    assert _rel(lhs, np.sum(x * g_ref)) < 1e-12


def test_combine_adjoint_identities():
    w = synth.small_motion()
    rng = np.random.default_rng(25)
    bases = [rng.normal(size=(3 * w.nbases,) + g.n) for g in w.levels]
    coeff = w.coeff.astype(np.float64)
    y = rng.normal(size=(len(w.angles), 3) + w.grid.n)
    D = oracle.combine(bases, w.levels, coeff, w.grid)
    gb, gc = oracle.combine_bwd(bases, w.levels, coeff, w.grid, y)
    lhs = np.sum(D * y)
    assert _rel(lhs, sum(np.sum(b * g) for b, g in zip(bases, gb))) < 1e-12
    assert _rel(lhs, np.sum(coeff * gc)) < 1e-12


def test_voxelize_adjoint_in_values():
    rng = np.random.default_rng(26)
    grid = Grid((12, 10, 9), (1.5, 1.5, 2.0))
    gs = synth.gaussians(rng, 40, grid, c=3, value_sigma=1.0)
    y = rng.normal(size=(3,) + grid.n)
    lhs = np.sum(oracle.voxelize(gs, grid, 3.0) * y)
    g = oracle.voxelize_bwd(gs, grid, 3.0, y)
    assert _rel(lhs, np.sum(gs.value.astype(np.float64) * g["value"])) < 1e-12


def test_project_linear_and_shared_stride():
    rng = np.random.default_rng(27)
    grid = Grid((10, 10, 8), (2.0, 2.0, 2.0))
    cone = Cone(1000.0, 1500.0, 12, 9, 3.0, 3.0)
    a, b = rng.normal(size=grid.n), rng.normal(size=grid.n)
    ang = [0.2, 2.0]
    pa = oracle.project(a, grid, cone, ang)
    pb = oracle.project(b, grid, cone, ang)
    pab = oracle.project(2.0 * a - 3.0 * b, grid, cone, ang)
    assert np.max(np.abs(pab - (2 * pa - 3 * pb))) < 1e-12
    stacked = oracle.project(np.stack([a, a]), grid, cone, ang, shared=False)
    assert np.array_equal(stacked, pa)


def test_project_rays_equals_project_at_every_pixel():
    """The selected-ray projector (used for sampled checks of large cases)
    gives every pixel of the full projector, bit for bit: a ragged,
    off-centre anisotropic grid with pixel offsets, a shared volume and one
    volume per view, the rays listed in a shuffled order."""
    rng = np.random.default_rng(28)
    grid = Grid((11, 9, 7), (2.0, 1.5, 2.5), (3.0, -2.0, 1.0))
    cone = Cone(1000.0, 1500.0, 13, 8, 3.0, 2.5, off_u=0.3, off_v=-0.6)
    ang = [0.3, 1.9, 4.4]
    vols = rng.normal(size=(3,) + grid.n)
    for vol, shared in ((vols[0], True), (vols, False)):
        full = oracle.project(vol, grid, cone, ang, shared=shared)
        v, iv, iu = np.meshgrid(np.arange(3), np.arange(cone.nv), np.arange(cone.nu), indexing="ij")
        rays = np.stack([v.ravel(), iu.ravel(), iv.ravel()], 1)
        order = rng.permutation(rays.shape[0])
        got = oracle.project_rays(vol, grid, cone, ang, rays[order], shared=shared)
        want = full[rays[order, 0], rays[order, 2], rays[order, 1]]
        assert np.array_equal(got, want)
        assert np.abs(want).max() > 0


def test_voxelize_points_equals_voxelize():
    """The brute-force voxelizer at selected voxels (every Gaussian tested)
    equals the box-walking voxelizer at those voxels: truncated and
    untruncated, three signed channels, a ragged off-centre grid."""
    rng = np.random.default_rng(29)
    grid = Grid((13, 10, 9), (1.5, 2.0, 1.0), (-1.0, 2.0, 0.5))
    gs = synth.gaussians(rng, 40, grid, c=3, value_sigma=1.0)
    idx = rng.choice(grid.size, size=300, replace=False)
    for k in (3.0, math.inf):
        want = oracle.voxelize(gs, grid, k).reshape(3, -1)[:, idx].T
        got = oracle.voxelize_points(gs, grid, k, idx)
        assert np.max(np.abs(got - want)) <= 1e-14 * max(1.0, np.abs(want).max())
        assert np.abs(want).max() > 0


def test_voxelize_band_matches_bruteforce():
    """The mask-margin split of Eq. 5 (used to check the GPU binning where
    pairs on the mask's edge may go either way) against brute force over
    every pair with scipy's rotation, for a band wide enough that every class
    holds pairs; inner + edge is the voxelizer itself."""
    rng = np.random.default_rng(31)
    grid = Grid((11, 9, 10), (1.0, 1.25, 1.5), (0.4, -0.3, 0.2))
    gs = synth.gaussians(rng, 30, grid, s_vox=(0.6, 2.0), c=2, value_sigma=1.0)
    X = np.stack(centres(grid), -1).reshape(-1, 3)
    k, band = 3.0, 2.5
    want = [np.zeros((2, X.shape[0])) for _ in range(4)]
    for i in range(gs.m):
        q = gs.quat[i].astype(np.float64)
        R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        A = np.linalg.inv(R @ np.diag(gs.scale[i].astype(np.float64) ** 2) @ R.T)
        d = X - gs.mean[i].astype(np.float64)
        m = np.einsum("pa,ab,pb->p", d, A, d)
        e = np.exp(-0.5 * m)
        for c in range(2):
            v = float(gs.value[i, c])
            want[0][c] += np.where(m <= k * k - band, v * e, 0.0)
            want[1][c] += np.where((m > k * k - band) & (m <= k * k), v * e, 0.0)
            want[2][c] += np.where(np.abs(m - k * k) <= band, abs(v) * e, 0.0)
            want[3][c] += np.where(m <= k * k + band, abs(v) * e, 0.0)
    got = [g.reshape(2, -1) for g in oracle.voxelize_band(gs, grid, k, band)]
    for a, b in zip(got, want):
        assert np.abs(b).max() > 0
        assert np.max(np.abs(a - b)) <= 1e-12 * np.abs(b).max()
    full = oracle.voxelize(gs, grid, k).reshape(2, -1)
    assert np.max(np.abs(got[0] + got[1] - full)) <= 1e-13 * np.abs(full).max()


def test_l2_loss_and_gradient():
    rng = np.random.default_rng(28)
    p = rng.normal(size=(3, 4, 5))
    t = rng.normal(size=(3, 4, 5))
    L, g = oracle.l2_loss(p, t)
    assert abs(L - np.sum((p - t) ** 2) / 3) < 1e-12
    e = 1e-6
    for idx in [(0, 1, 2), (2, 3, 4)]:
        pp = p.copy(); pp[idx] += e
        pm = p.copy(); pm[idx] -= e
        fd = (oracle.l2_loss(pp, t)[0] - oracle.l2_loss(pm, t)[0]) / (2 * e)
        assert abs(fd - g[idx]) < 1e-8


# ----------------------------------------------------- gradients by FD (P11)

def _fd_case():
    w = synth.small_motion(seed=31, trunc_k=math.inf)
    truth = synth.perturbed_truth(w, seed=32)
    target = oracle.forward(truth)
    return w, target


def _loss(w, target):
    p = oracle.forward(w)
    return float(np.sum((p - target) ** 2)) / len(w.angles)


@pytest.fixture(scope="module")
def fd_setup():
    w, target = _fd_case()
    # float64 parameters so perturbations are not rounded away
    w.ref = GaussSet(*[x.astype(np.float64) for x in (w.ref.mean, w.ref.scale, w.ref.quat, w.ref.value)])
    w.mbc = [GaussSet(*[x.astype(np.float64) for x in (s.mean, s.scale, s.quat, s.value)]) for s in w.mbc]
    w.coeff = w.coeff.astype(np.float64)
    loss, grads = oracle.step(w, target)
    return w, target, loss, grads


def _perturb(w, kind, which, idx, eps):
    import copy
    w2 = copy.copy(w)
    if kind == "coeff":
        c = w.coeff.copy(); c[idx] += eps; w2.coeff = c
        return w2
    sets = [w.ref] if which == "ref" else list(w.mbc)
    li = 0 if which == "ref" else which
    s = sets[li].copy()
    getattr(s, kind)[idx] += eps
    if which == "ref":
        w2.ref = s
    else:
        mb = list(w.mbc); mb[li] = s; w2.mbc = mb
    return w2


def test_loss_matches_forward(fd_setup):
    w, target, loss, _ = fd_setup
    assert _rel(loss, _loss(w, target)) < 1e-12


@pytest.mark.parametrize("which", ["ref", 0, 1, 2])
def test_gradients_central_fd(fd_setup, which):
    """Central differences (step 1e-6) of the untruncated full-chain loss.  The
    warp is piecewise trilinear, so a larger step can carry a sample across a
    cell plane and pick up the kink; 1e-6 mm keeps clear of that here."""
    w, target, loss, grads = fd_setup
    g = grads["ref"] if which == "ref" else grads["mbc"][which]
    s = w.ref if which == "ref" else w.mbc[which]
    rng = np.random.default_rng(33 + (0 if which == "ref" else which + 1))
    # Gaussians with the largest value-gradient, so the checks are not vacuous
    order = np.argsort(-np.abs(g["value"]).sum(axis=1))
    picks = list(order[:3]) + [int(rng.integers(s.m))]
    for i in picks:
        for kind, ncomp, eps in (("mean", 3, 1e-6), ("scale", 3, 1e-6), ("quat", 4, 1e-6),
                                 ("value", s.value.shape[1], 1e-6)):
            for c in range(ncomp):
                idx = (i, c)
                fp = _loss(_perturb(w, kind, which, idx, eps), target)
                fm = _loss(_perturb(w, kind, which, idx, -eps), target)
                fd = (fp - fm) / (2 * eps)
                an = g[kind][idx]
                scale = max(abs(an), abs(fd), 1e-6 * max(1.0, abs(loss)))
                assert abs(fd - an) / scale < 1e-5, (which, kind, idx, fd, an)


def test_coeff_gradient_central_fd(fd_setup):
    w, target, loss, grads = fd_setup
    rng = np.random.default_rng(40)
    for _ in range(8):
        idx = tuple(int(rng.integers(d)) for d in w.coeff.shape)
        eps = 1e-6
        fd = (_loss(_perturb(w, "coeff", None, idx, eps), target)
              - _loss(_perturb(w, "coeff", None, idx, -eps), target)) / (2 * eps)
        an = grads["coeff"][idx]
        assert abs(fd - an) / max(abs(an), abs(fd), 1e-8) < 1e-5, (idx, fd, an)


def test_zero_gradient_outside_every_ray():
    """A Gaussian that no ray's samples reach gets exactly zero gradient."""
    grid = Grid((30, 30, 30), (1.0, 1.0, 1.0))
    cone = Cone(1000.0, 1500.0, 6, 6, 1.0, 1.0)        # ~4 mm field at the isocentre
    gs = GaussSet(np.array([[0.0, 0.0, 0.0], [11.0, 11.0, 11.0]]), np.array([[1.0] * 3, [0.8] * 3]),
                  np.array([[1.0, 0, 0, 0], [0.9, 0.1, 0.2, 0.3]]), np.array([[1.0], [1.0]]))
    vol = oracle.voxelize(gs, grid, 3.0)[0]
    p = oracle.project(vol, grid, cone, [0.0])
    gvol = oracle.project_bwd(p, grid, cone, [0.0], shared=True)
    g = oracle.voxelize_bwd(gs, grid, 3.0, gvol.reshape(1, -1))
    assert np.abs(g["value"][0]).sum() > 0
    for k in ("mean", "scale", "quat", "value"):
        assert np.all(g[k][1] == 0.0)
