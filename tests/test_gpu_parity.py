"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars (relative L2 error per output tensor): 1e-4 for volumes and
projections, 1e-3 for gradients; integer-free paths only.  Inputs are the
seeded generators' float32 arrays, fed to both sides; expected values come
from the oracle only.
"""
import dataclasses
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2503_22139_amd import ops, synth
from paper_2503_22139_amd.model import MotionModel
from paper_2503_22139_amd.synth import Cone, GaussSet, Grid

pytestmark = pytest.mark.gpu

VOL_TOL = 1e-4
GRAD_TOL = 1e-3


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ops.lib()           # raises if libpmf.so is missing
    oracle.build()
    yield


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def N(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def gauss_t(s):
    return T(s.mean), T(s.scale), T(s.quat), T(s.value)


def f32(a):
    return np.asarray(a, np.float32)


# ---------------------------------------------------------------- voxelize

@pytest.mark.parametrize("case", ["c1", "small_ref", "small_mbc", "fd32_untruncated", "large_list",
                                  "edge"])
def test_voxelize_forward(case):
    say("voxelize", case)
    if case == "c1":
        w = synth.c1(); gs, grid, k = w.ref, w.grid, 3.0
    elif case == "small_ref":
        w = synth.small_motion(); gs, grid, k = w.ref, w.grid, 3.0
    elif case == "small_mbc":
        w = synth.small_motion(); gs, grid, k = w.mbc[2], w.levels[2], 3.0
    elif case == "fd32_untruncated":
        w = synth.fd32(); gs, grid, k = w.mbc[1], w.levels[1], math.inf
    elif case == "large_list":   # untruncated on a grid of 45 tiles: every Gaussian overflows the bins
        grid = Grid((70, 40, 40), (1.0, 1.2, 1.1))
        gs = synth.gaussians(np.random.default_rng(4), 200, grid)
        k = math.inf
    else:   # Gaussians beyond the grid, huge and tiny scales, ragged grid
        rng = np.random.default_rng(5)
        grid = Grid((19, 7, 33), (1.3, 2.1, 0.7), (3.0, -2.0, 1.0))
        gs = synth.gaussians(rng, 300, Grid((40, 20, 60), (1.3, 2.1, 0.7), (3.0, -2.0, 1.0)),
                             s_vox=(0.05, 12.0), c=3, value_sigma=1.0)
        k = 3.0
    want = oracle.voxelize(gs, grid, k)
    got = N(ops.pmf_voxelize(*gauss_t(gs), grid, k))
    assert got.shape == want.shape
    assert rel(got, want) < VOL_TOL, rel(got, want)


def test_voxelize_empty_set():
    grid = Grid((9, 8, 7), (1.0, 1.0, 1.0))
    z = np.zeros((0, 3), np.float32)
    gs = GaussSet(z, z, np.zeros((0, 4), np.float32), np.zeros((0, 2), np.float32))
    out = ops.pmf_voxelize(*gauss_t(gs), grid, 3.0, out=torch.full((2, 9, 8, 7), 7.0, device="cuda"))
    assert np.all(N(out) == 0.0)


def test_voxelize_c2_full_size():
    """200k-Gaussian reference at 256x256x128 (the benchmark's reference volume)."""
    say("voxelize c2 full")
    w = synth.c2()
    want = oracle.voxelize(w.ref, w.grid, 3.0)
    got = N(ops.pmf_voxelize(*gauss_t(w.ref), w.grid, 3.0))
    assert rel(got, want) < VOL_TOL, rel(got, want)


@pytest.mark.parametrize("case", ["c1", "small_mbc", "signed_c3", "signed_c9", "fd32_untruncated"])
def test_voxelize_backward(case):
    """One channel (c1, untruncated fd32), six (the small MBC level: the
    kernel's generic channel count) and three and nine signed channels (the
    MBC bases with B = 1 and B = 3)."""
    say("voxelize_bwd", case)
    if case == "c1":
        w = synth.c1(); gs, grid, k = w.ref, w.grid, 3.0
    elif case == "small_mbc":
        w = synth.small_motion(); gs, grid, k = w.mbc[1], w.levels[1], 3.0
    elif case in ("signed_c3", "signed_c9"):
        grid = Grid((30, 26, 22), (2.0, 2.5, 3.0), (1.0, -2.0, 0.5))
        gs = synth.gaussians(np.random.default_rng(17), 400, grid, c=3 if case == "signed_c3" else 9,
                             value_sigma=1.0)
        k = 3.0
    else:
        w = synth.fd32(); gs, grid, k = w.ref, w.grid, math.inf
    gv = synth.random_normal(3, (gs.c,) + tuple(grid.n))
    want = oracle.voxelize_bwd(gs, grid, k, gv)
    got = ops.pmf_voxelize_bwd(*gauss_t(gs), grid, k, T(gv))
    for name, g in zip(("mean", "scale", "quat", "value"), got):
        r = rel(N(g), want[name])
        assert r < GRAD_TOL, (name, r)


# ------------------------------------------------------------------ project

def _proj_case(case):
    if case == "c1":
        w = synth.c1()
        vol = f32(oracle.voxelize(w.ref, w.grid, 3.0)[0])
        return vol, w.grid, w.cone, w.angles
    if case == "aniso":   # odd detector, offsets, anisotropic off-centre grid
        grid = Grid((23, 17, 12), (1.7, 1.1, 2.3), (4.0, -3.0, 2.0))
        vol = synth.random_volume(8, grid.n)
        cone = Cone(800.0, 1300.0, 37, 29, 1.3, 1.1, off_u=0.3, off_v=-1.7, step=0.0)
        return vol, grid, cone, synth.evenly_spaced_angles(7) + np.float32(0.1)
    raise ValueError(case)


@pytest.mark.parametrize("case", ["c1", "aniso"])
def test_project_forward(case):
    say("project", case)
    vol, grid, cone, ang = _proj_case(case)
    want = oracle.project(vol, grid, cone, ang)
    got = N(ops.pmf_project(T(vol), grid, cone, T(ang)))
    assert rel(got, want) < VOL_TOL, rel(got, want)
    # per-view volumes
    vols = np.stack([vol, 2.0 * vol])
    want2 = oracle.project(vols, grid, cone, ang[:2], shared=False)
    got2 = N(ops.pmf_project(T(vols), grid, cone, T(ang[:2]), shared=False))
    assert rel(got2, want2) < VOL_TOL


def test_project_c2_full_size_sampled():
    """Full 256x256x128 volume, 8 views of 512x384: 4,000 sampled rays."""
    say("project c2 sampled")
    w = synth.c2()
    vol = f32(oracle.voxelize(w.ref, w.grid, 3.0)[0])
    got = N(ops.pmf_project(T(vol), w.grid, w.cone, T(w.angles)))
    rng = np.random.default_rng(9)
    rays = np.stack([rng.integers(0, 8, 4000), rng.integers(0, w.cone.nu, 4000),
                     rng.integers(0, w.cone.nv, 4000)], 1)
    want = oracle.project_rays(vol, w.grid, w.cone, w.angles, rays)
    g = got[rays[:, 0], rays[:, 2], rays[:, 1]]
    assert rel(g, want) < VOL_TOL, rel(g, want)


@pytest.mark.parametrize("case", ["c1", "aniso"])
def test_project_backward(case):
    say("project_bwd", case)
    vol, grid, cone, ang = _proj_case(case)
    V = len(ang)
    gp = synth.random_normal(4, (V, cone.nv, cone.nu))
    want = oracle.project_bwd(gp, grid, cone, ang, shared=False)
    got = N(ops.pmf_project_bwd(T(gp), grid, cone, T(ang), shared=False))
    assert rel(got, want) < VOL_TOL, rel(got, want)
    want_s = oracle.project_bwd(gp, grid, cone, ang, shared=True)
    got_s = N(ops.pmf_project_bwd(T(gp), grid, cone, T(ang), shared=True))
    assert rel(got_s, want_s) < VOL_TOL, rel(got_s, want_s)


def test_project_degenerate_cases():
    """Edge cases of Eq. 6 and its adjoint against the oracle: the smallest
    grid (2 voxels per axis) seen by a 5x3 detector whose outer rays miss
    it; a view whose detector is shifted off the volume (every ray misses:
    zero projections, zero adjoint); a residual on a single pixel; an all-zero
    residual (the back-projection's fixed-point scale is then 0)."""
    grid = Grid((2, 2, 2), (3.0, 2.5, 2.0), (0.4, -0.3, 0.2))
    cone = Cone(400.0, 700.0, 5, 3, 2.6, 2.2, off_u=0.3, off_v=-0.2, step=0.0)
    ang = np.asarray([0.1, 1.3, 2.9], np.float32)
    V = len(ang)
    vol = synth.random_volume(41, (V,) + grid.n, 0.5, 1.5)
    want = oracle.project(vol, grid, cone, ang, shared=False)
    got = N(ops.pmf_project(T(vol), grid, cone, T(ang), shared=False))
    assert np.any(want == 0.0) and np.any(want > 0.0)
    assert rel(got, want) < VOL_TOL, rel(got, want)
    gp = synth.random_normal(42, (V, cone.nv, cone.nu))
    want_b = oracle.project_bwd(gp, grid, cone, ang, shared=False)
    got_b = N(ops.pmf_project_bwd(T(gp), grid, cone, T(ang), shared=False))
    assert rel(got_b, want_b) < VOL_TOL, rel(got_b, want_b)
    # detector shifted far off the volume: every ray misses
    far = Cone(1000.0, 1500.0, 16, 12, 0.8, 0.8, off_u=400.0, step=0.0)
    g2 = Grid((12, 10, 8), (1.5, 1.5, 2.0))
    v2 = synth.random_volume(43, (1,) + g2.n)
    a2 = np.asarray([0.4], np.float32)
    assert np.all(oracle.project(v2, g2, far, a2, shared=False) == 0.0)
    assert np.all(N(ops.pmf_project(T(v2), g2, far, T(a2), shared=False)) == 0.0)
    gp2 = synth.random_normal(44, (1, far.nv, far.nu))
    assert np.all(N(ops.pmf_project_bwd(T(gp2), g2, far, T(a2), shared=False)) == 0.0)
    # one pixel's residual, and none at all
    c3 = Cone(1000.0, 1500.0, 24, 20, 1.6, 1.6, step=0.0)
    a3 = np.asarray([0.7, 2.2], np.float32)
    one = np.zeros((2, c3.nv, c3.nu), np.float32)
    one[1, 9, 13] = 2.5
    want_1 = oracle.project_bwd(one, g2, c3, a3, shared=False)
    got_1 = N(ops.pmf_project_bwd(T(one), g2, c3, T(a3), shared=False))
    assert np.abs(want_1).max() > 0.0
    assert rel(got_1, want_1) < VOL_TOL, rel(got_1, want_1)
    zero = np.zeros_like(one)
    assert np.all(N(ops.pmf_project_bwd(T(zero), g2, c3, T(a3), shared=False)) == 0.0)
    assert np.all(N(ops.pmf_project_bwd(T(zero), g2, c3, T(a3), shared=True)) == 0.0)


def test_project_adjoint_identity_fp32():
    vol, grid, cone, ang = _proj_case("aniso")
    V = len(ang)
    x = synth.random_normal(10, (V,) + grid.n)
    y = synth.random_normal(11, (V, cone.nv, cone.nu))
    px = N(ops.pmf_project(T(x), grid, cone, T(ang), shared=False))
    pty = N(ops.pmf_project_bwd(T(y), grid, cone, T(ang), shared=False))
    lhs, rhs = np.sum(px * y), np.sum(x * pty)
    assert abs(lhs - rhs) / max(abs(lhs), 1e-30) < 1e-5


# ------------------------------------------------------------ combine, warp

@pytest.fixture(scope="module")
def small():
    w = synth.small_motion()
    bases = [f32(oracle.voxelize(s, g, 3.0)) for s, g in zip(w.mbc, w.levels)]
    ref = f32(oracle.voxelize(w.ref, w.grid, 3.0)[0])
    return w, ref, bases


def test_combine_forward(small):
    w, ref, bases = small
    want = oracle.combine(bases, w.levels, w.coeff, w.grid)
    got = N(ops.pmf_combine_dvf([T(b) for b in bases], w.levels, T(w.coeff), w.grid))
    assert rel(got, want) < VOL_TOL, rel(got, want)


def test_combine_backward(small):
    w, ref, bases = small
    gd = synth.random_normal(12, (len(w.angles), 3) + w.grid.n)
    wb, wc = oracle.combine_bwd(bases, w.levels, w.coeff, w.grid, gd)
    gb, gc = ops.pmf_combine_dvf_bwd([T(b) for b in bases], w.levels, T(w.coeff), w.grid, T(gd))
    for a, b in zip(gb, wb):
        assert rel(N(a), b) < GRAD_TOL
    assert rel(N(gc), wc) < GRAD_TOL


def test_warp_forward_backward(small):
    w, ref, bases = small
    dvf = synth.random_normal(13, (3, 3) + w.grid.n, sigma=3.0)
    want = oracle.warp(ref, w.grid, dvf)
    got = N(ops.pmf_warp(T(ref), w.grid, T(dvf)))
    assert rel(got, want) < VOL_TOL
    go = synth.random_normal(14, (3,) + w.grid.n)
    wr, wd = oracle.warp_bwd(ref, w.grid, dvf, go)
    gr, gd = ops.pmf_warp_bwd(T(ref), w.grid, T(dvf), T(go))
    assert rel(N(gr), wr) < GRAD_TOL
    assert rel(N(gd), wd) < GRAD_TOL


@pytest.mark.parametrize("shape,offset", [((3, 7, 9), 0),     # float4 bulk + a 1-value tail
                                          ((3, 7, 9), 1),     # misaligned: the scalar kernel
                                          ((2, 384, 513), 0)])  # several hundred blocks
def test_l2_loss(shape, offset):
    p = synth.random_normal(15, shape)
    t = synth.random_normal(16, shape)
    want_l, want_g = oracle.l2_loss(p, t)
    n = p.size

    def placed(x):   # the values at a given float offset into a fresh buffer
        buf = torch.zeros(n + 1, device="cuda")
        buf[offset:offset + n] = T(x).reshape(-1)
        return buf[offset:offset + n].view(shape)

    l, g = ops.pmf_l2_loss(placed(p), placed(t))
    assert abs(float(N(l)) - want_l) / want_l < 1e-5
    assert rel(N(g), want_g) < 1e-6


# ------------------------------------------------------------ fused path

def test_warp_project_forward(small):
    w, ref, bases = small
    want = np.stack([oracle.project(oracle.warp(ref, w.grid, oracle.combine(bases, w.levels,
                                                                             w.coeff[v:v + 1], w.grid)),
                                    w.grid, w.cone, w.angles[v:v + 1])[0] for v in range(len(w.angles))])
    got = N(ops.pmf_warp_project(T(ref), w.grid, [T(b) for b in bases], w.levels, T(w.coeff), w.cone,
                                 T(w.angles)))
    assert rel(got, want) < VOL_TOL, rel(got, want)


def _oracle_target(w):
    truth = synth.perturbed_truth(w)
    return synth.add_target_noise(oracle.forward(truth))


def _compare_grads(got, want, tag):
    for name in ("mean", "scale", "quat", "value"):
        r = rel(N(got["ref"][name]), want["ref"][name])
        assert r < GRAD_TOL, (tag, "ref", name, r)
    for l, (a, b) in enumerate(zip(got["mbc"], want["mbc"])):
        for name in ("mean", "scale", "quat", "value"):
            r = rel(N(a[name]), b[name])
            assert r < GRAD_TOL, (tag, "mbc", l, name, r)
    r = rel(N(got["coeff"]), want["coeff"])
    assert r < GRAD_TOL, (tag, "coeff", r)


@pytest.mark.parametrize("case", ["small", "fd32"])
def test_full_step_plain_and_batched(case):
    say("step", case)
    w = synth.small_motion() if case == "small" else synth.fd32()
    target = _oracle_target(w)
    want_loss, want = oracle.step(w, target)
    m = MotionModel(w)
    for name, fn in (("plain", m.step_plain), ("batched", m.step_batched)):
        loss, grads = fn(T(target))
        assert abs(float(N(loss)) - want_loss) / want_loss < VOL_TOL, (name, float(N(loss)), want_loss)
        _compare_grads(grads, want, name)


def test_batched_equals_plain_ragged():
    """Ragged sizes, more views than one chunk of the fused adjoint."""
    w = synth.small_motion(seed=21, n=(13, 21, 10), level_dims=((5, 6, 4), (13, 21, 10), (7, 11, 5)),
                           nviews=70, det=(17, 13))
    target = synth.random_volume(22, (70, 13, 17), 0.0, 1.0)
    m = MotionModel(w)
    lp, gp = m.step_plain(T(target))
    lb, gb = m.step_batched(T(target))
    assert abs(float(N(lp)) - float(N(lb))) <= 1e-5 * abs(float(N(lp)))
    for name in ("mean", "scale", "quat", "value"):
        assert rel(N(gb["ref"][name]), N(gp["ref"][name])) < 1e-4
        for a, b in zip(gb["mbc"], gp["mbc"]):
            assert rel(N(a[name]), N(b[name])) < 1e-4
    assert rel(N(gb["coeff"]), N(gp["coeff"])) < 1e-4


# -------------------------------------------------- full size (benchmark)

def test_headline_full_size_sampled():
    """The benchmark iteration (32 views, 256x256x128, 200k + 21k Gaussians)
    in the batched launch configuration: sampled projection rays of two views
    and the view-0 coefficient gradient against the oracle; the adjoint
    identity in the reference volume; batched equals plain."""
    say("headline: build")
    w = synth.headline()
    m = MotionModel(w)
    V = len(w.angles)
    target = synth.random_volume(23, (V, w.cone.nv, w.cone.nu), 0.0, 20.0)
    say("headline: gpu step")
    proj = N(m.forward_batched())
    loss_b, grads_b = m.step_batched(T(target))
    say("headline: oracle volumes")
    ref, bases = oracle.forward_volumes(w)
    rng = np.random.default_rng(24)
    for v in (0, 17):
        dvf = oracle.combine(bases, w.levels, w.coeff[v:v + 1], w.grid)
        wv = oracle.warp(ref, w.grid, dvf)
        rays = np.stack([np.zeros(1500, np.int64), rng.integers(0, w.cone.nu, 1500),
                         rng.integers(0, w.cone.nv, 1500)], 1)
        want = oracle.project_rays(wv, w.grid, w.cone, w.angles[v:v + 1], rays)
        got = proj[v][rays[:, 2], rays[:, 1]]
        say("headline: view", v, "rel", rel(got, want))
        assert rel(got, want) < VOL_TOL, (v, rel(got, want))
    say("headline: oracle view-0 gradient")
    _, og = oracle.step(w, target, views=[0])
    r = rel(N(grads_b["coeff"][0]), og["coeff"][0])
    say("headline: g_coeff[0] rel", r)
    assert r < GRAD_TOL, r
    dvf0 = oracle.combine(bases, w.levels, w.coeff[0:1], w.grid)[0].reshape(3, -1)
    near = _near_faces(w, dvf0, _dvf_abs(w, 0))
    _coeff_within_face_jumps(w, ref, bases, target, N(grads_b["coeff"][0]), og["coeff"][0], near)
    flags = _mbc_flagged(w, near)
    say("headline: one-view gradients of every Gaussian parameter")
    # the oracle's view-0 share of the 32-view loss carries 1/32; a one-view
    # GPU iteration carries 1/1, so its gradients are scaled by 1/32 (exact)
    w1 = dataclasses.replace(w, angles=w.angles[:1], coeff=w.coeff[:1],
                             view_index=w.view_index[:1])
    m1 = MotionModel(w1)
    _, g1 = m1.step_batched(T(target[:1]))
    # reference Gaussians see dL/dI_ref, whose trilinear weights are
    # continuous across faces: every one is compared; MBC Gaussians that a
    # near-face voxel reaches are flagged and left out (they are few)
    for name in ("mean", "scale", "quat", "value"):
        r = rel(N(g1["ref"][name]) / V, og["ref"][name])
        say("headline: view 0 ref", name, r)
        assert r < GRAD_TOL, ("ref", name, r)
        for l in range(len(w.mbc)):
            keep = ~flags[l]
            r = rel(N(g1["mbc"][l][name])[keep] / V, og["mbc"][l][name][keep])
            r_all = rel(N(g1["mbc"][l][name]) / V, og["mbc"][l][name])
            say("headline: view 0 mbc", l, name, r, "flagged", int(flags[l].sum()), "of",
                flags[l].size, "all", r_all)
            assert r < GRAD_TOL, ("mbc", l, name, r)
    for l in range(len(w.mbc)):
        assert flags[l].mean() < 0.5, (l, flags[l].mean())
    del m1, g1
    say("headline: plain")
    loss_p, grads_p = m.step_plain(T(target))
    assert abs(float(N(loss_p)) - float(N(loss_b))) <= 1e-5 * float(N(loss_p))
    assert rel(N(grads_b["coeff"]), N(grads_p["coeff"])) < 1e-4
    for name in ("mean", "scale", "quat", "value"):
        assert rel(N(grads_b["ref"][name]), N(grads_p["ref"][name])) < 1e-4, name
    say("headline: adjoint identity in ref")
    ref_g, bases_g = m.volumes()

    def identity(x, y):
        px = ops.pmf_warp_project(x, w.grid, bases_g, w.levels, m.coeff, w.cone, m.angles)
        gx, _, _ = ops.pmf_warp_project_bwd(ref_g, w.grid, bases_g, w.levels, m.coeff, w.cone,
                                            m.angles, y)
        lhs = float(torch.sum(px.double() * y.double()))
        rhs = float(torch.sum(x.double() * gx.double()))
        norm = float(torch.linalg.vector_norm(px.double()) * torch.linalg.vector_norm(y.double()))
        return lhs, rhs, norm
    # nonnegative x and y: the inner product is a sum of nonnegative terms
    # (no cancellation), so its relative error is that of the terms: float
    # rounding and the back-projection's fixed point (each term rounded to
    # within 2^-31 * kbound * max|y * delta|, ~1e-7 of the largest)
    lhs, rhs, _ = identity(T(synth.random_volume(25, w.grid.n)),
                           T(synth.random_volume(26, (V, w.cone.nv, w.cone.nu))))
    say("headline: adjoint identity rel (nonnegative inputs)", abs(lhs - rhs) / abs(lhs))
    assert abs(lhs - rhs) / abs(lhs) < 1e-5, (lhs, rhs)
    # signed inputs: the inner product cancels, so the error is measured
    # against the Cauchy-Schwarz bound |<Px, y>| <= |Px| |y|
    lhs, rhs, norm = identity(T(synth.random_normal(27, w.grid.n)),
                              T(synth.random_normal(28, (V, w.cone.nv, w.cone.nu))))
    say("headline: adjoint identity (signed inputs), |lhs-rhs| / (|Px||y|)", abs(lhs - rhs) / norm)
    assert abs(lhs - rhs) / norm < 1e-6, (lhs, rhs, norm)


def _near_faces(w, dvf, dabs):
    """Voxel-axes whose warped point x_j + d_j lies within float rounding of
    a cell face, with the face coordinate.  The kernel decides the cell from
    t = d / h (float32); d is a sum of coefficient x basis-sample products,
    so its float error is bounded by a few dozen float epsilons of the sum
    of their magnitudes, dabs (the oracle's combine of |w| and the
    voxelization with |values|): the band is 5e-6 dabs / h, plus 2e-7 |t|
    for the scaling by 1/h."""
    n = np.asarray(w.grid.n)
    h = np.asarray(w.grid.h, np.float64)
    idx = np.indices(tuple(n)).reshape(3, -1)
    out = []
    for a in range(3):
        t = dvf[a] / h[a]
        band = 5e-6 * dabs[a] / h[a] + 2e-7 * np.abs(t)
        f = np.rint(t)
        face = idx[a] + f
        # dabs = 0: no basis reaches the voxel, d = 0 exactly on both sides
        near = np.nonzero((dabs[a] > 0.0) & (np.abs(t - f) <= band) & (face >= 0) &
                          (face <= n[a] - 1))[0]
        out.append((near, face[near]))
    return out


def _dvf_abs(w, view):
    """Sum over (level, basis) of |w| x the upsampled voxelization with
    |values|: a bound on the magnitudes the DVF of `view` is summed from."""
    babs = []
    for s, lg in zip(w.mbc, w.levels):
        a = s.copy()
        a.value = np.abs(a.value)
        babs.append(oracle.voxelize(a, lg, w.trunc_k))
    return oracle.combine(babs, w.levels, np.abs(w.coeff[view:view + 1]), w.grid)[0].reshape(3, -1)


def _coeff_within_face_jumps(w, ref, bases, target, got, want, near):
    """The validity check for dL/dw of view 0 where several results are
    correct.  The trilinear derivative along axis a jumps where a warped
    point crosses a cell face; a point within float rounding of a face may
    take either one-sided derivative.  Each coefficient (l, b, k) may then
    differ from the oracle by at most the sum, over the voxels whose warped
    point lies within FACE of a face normal to k, of
    |dL/dI(j)| |slope jump| |S(E_lbk, x_j)|, plus a float bar of 1e-4 of the
    gradient's norm."""
    V = len(w.angles)
    dvf = oracle.combine(bases, w.levels, w.coeff[0:1], w.grid)[0].reshape(3, -1)
    wv = oracle.warp(ref, w.grid, dvf.reshape((1, 3) + tuple(w.grid.n)))
    p0 = oracle.project(wv, w.grid, w.cone, w.angles[0:1])
    gp0 = 2.0 * (p0 - np.asarray(target[0:1], np.float64)) / V
    gw = oracle.project_bwd(gp0, w.grid, w.cone, w.angles[0:1]).reshape(-1)
    n = np.asarray(w.grid.n)
    h = np.asarray(w.grid.h, np.float64)
    c0 = np.asarray(w.grid.center, np.float64) - 0.5 * (n - 1) * h
    L, B = w.coeff.shape[1], w.coeff.shape[2]
    bound = np.zeros((L, B, 3))
    for a in range(3):
        vox, face_u = near[a]
        if vox.size == 0:
            continue
        X = c0 + np.stack(np.unravel_index(vox, tuple(n)), 1) * h
        P = X + dvf[:, vox].T
        P[:, a] = c0[a] + face_u * h[a]
        eps = np.zeros(3)
        eps[a] = 1e-6 * h[a]
        _, gm = oracle.sample_points(ref, w.grid, P - eps, grad=True)
        _, gpl = oracle.sample_points(ref, w.grid, P + eps, grad=True)
        jump = np.abs((gpl[:, a] - gm[:, a]) * gw[vox])
        for l in range(L):
            for b in range(B):
                s_e = oracle.sample_points(bases[l][b * 3 + a], w.levels[l], X)
                bound[l, b, a] += np.sum(jump * np.abs(s_e))
    diff = np.abs(np.asarray(got, np.float64) - want)
    fbar = 1e-4 * np.linalg.norm(want)
    say("headline: near-face voxel-axes", sum(v.size for v, _ in near), "max |diff|", diff.max(),
        "max bound", bound.max(), "float bar", fbar,
        "worst excess", float(np.max(diff - bound - fbar)))
    assert np.all(diff <= bound + fbar), (diff - bound - fbar).max()


def _mbc_flagged(w, near):
    """Per MBC level, the Gaussians whose gradient can see a near-face voxel
    (a gradient is not pinned where a cell-face crossing reaches it, so such
    parameters are flagged and excluded).  A fine voxel j feeds dL/dE_l at the corners of
    its upsampling cell on level l; a Gaussian is flagged when its mask
    holds such a corner (the voxelization adjoint of the corner indicator
    with unit values is then positive)."""
    n = np.asarray(w.grid.n)
    h = np.asarray(w.grid.h, np.float64)
    c0 = np.asarray(w.grid.center, np.float64) - 0.5 * (n - 1) * h
    vox = np.unique(np.concatenate([v for v, _ in near]))
    X = c0 + np.stack(np.unravel_index(vox, tuple(n)), 1) * h
    flags = []
    for lg, s in zip(w.levels, w.mbc):
        ln = np.asarray(lg.n)
        lh = np.asarray(lg.h, np.float64)
        lc0 = np.asarray(lg.center, np.float64) - 0.5 * (ln - 1) * lh
        u = np.clip((X - lc0) / lh, 0.0, ln - 1)
        i = np.minimum(np.floor(u).astype(np.int64), ln - 2)
        mark = np.zeros(tuple(ln))
        for c in range(8):
            o = np.array([(c >> 2) & 1, (c >> 1) & 1, c & 1])
            k = i + o
            mark[k[:, 0], k[:, 1], k[:, 2]] = 1.0
        ones = synth.GaussSet(s.mean, s.scale, s.quat, np.ones((s.m, 1), np.float32))
        g = oracle.voxelize_bwd(ones, lg, w.trunc_k, mark.reshape(1, -1))
        flags.append(g["value"][:, 0] > 0.0)
    return flags


def test_graph_replay_matches_eager():
    """The captured batched iteration, replayed several times with eager work
    and synchronisations between replays, equals the eager iteration."""
    from paper_2503_22139_amd.model import GraphStep
    w = synth.small_motion(seed=41, nviews=5)
    target = T(synth.random_volume(42, (5, w.cone.nv, w.cone.nu), 0.0, 2.0))
    m = MotionModel(w)
    loss_e, g_e = m.step_batched(target)
    want = (float(N(loss_e)), N(g_e["coeff"]), N(g_e["ref"]["mean"]), N(g_e["mbc"][2]["value"]))
    gs = GraphStep(m, target)
    for it in range(4):
        loss, g = gs.step(target)
        got = (float(N(loss)), N(g["coeff"]), N(g["ref"]["mean"]), N(g["mbc"][2]["value"]))
        assert abs(got[0] - want[0]) <= 1e-6 * abs(want[0]), (it, got[0], want[0])
        for a, b in zip(got[1:], want[1:]):
            assert rel(a, b) < 1e-5, it
        m.step_plain(target)            # eager work between replays
        torch.cuda.synchronize()


def test_launch_shapes_agree_and_autotune():
    """Every forward ray tile gives the same bits (per-ray sums); every
    back-projection brick gives the same values to within the fixed-point
    rounding (integer sums with a per-view scale, but a lane merges its
    consecutive samples in one cell before rounding, and which samples a lane
    takes depends on the brick); the autotuner picks valid shapes."""
    _, grid, cone, angles = _proj_case("aniso")
    V = len(angles)
    ang = T(angles)
    vol = T(synth.random_volume(80, (V,) + tuple(grid.n), 0.0, 1.0))
    gp = T(synth.random_normal(81, (V, cone.nv, cone.nu)))
    tile0 = ops.pmf_tune_get(ops.PMF_TUNE_PROJECT_TILE)
    brick0 = ops.pmf_tune_get(ops.PMF_TUNE_BACKPROJECT_BRICK)
    try:
        ref_p = ref_b = None
        for k in range(ops.pmf_tune_candidates(ops.PMF_TUNE_PROJECT_TILE)):
            ops.pmf_tune_set(ops.PMF_TUNE_PROJECT_TILE, k)
            p = ops.pmf_project(vol, grid, cone, ang, shared=False)
            ref_p = p.clone() if ref_p is None else ref_p
            assert torch.equal(p, ref_p), k
        want = np.asarray(oracle.project_bwd(N(gp), grid, cone, angles))
        want_s = want.sum(0)
        first = {}
        for k in range(ops.pmf_tune_candidates(ops.PMF_TUNE_BACKPROJECT_BRICK)):
            ops.pmf_tune_set(ops.PMF_TUNE_BACKPROJECT_BRICK, k)
            b = N(ops.pmf_project_bwd(gp, grid, cone, ang, shared=False))
            bs = N(ops.pmf_project_bwd(gp, grid, cone, ang, shared=True))
            assert rel(b.reshape(want.shape), want) < VOL_TOL, k
            assert rel(bs.reshape(want_s.shape), want_s) < VOL_TOL, k
            # shapes that first sum a ray's consecutive samples in one cell
            # (all but 1) round per merged group; within each kind the
            # fixed-point sums repeat up to the float additions at brick faces
            grp = k == 1
            if grp not in first:
                first[grp] = (b, bs)
            assert rel(b, first[grp][0]) < 1e-6, k
            assert rel(bs, first[grp][1]) < 1e-6, k
        res = ops.pmf_autotune_project(vol, grid, cone, ang, gp, reps=2)
        say("autotune", res)
        assert 0 <= res["project_tile"] < ops.pmf_tune_candidates(ops.PMF_TUNE_PROJECT_TILE)
        assert 0 <= res["backproject_brick"] < ops.pmf_tune_candidates(ops.PMF_TUNE_BACKPROJECT_BRICK)
        assert all(t > 0 for t in res["project_tile_ms"] + res["backproject_brick_ms"])
    finally:
        ops.pmf_tune_set(ops.PMF_TUNE_PROJECT_TILE, tile0)
        ops.pmf_tune_set(ops.PMF_TUNE_BACKPROJECT_BRICK, brick0)
