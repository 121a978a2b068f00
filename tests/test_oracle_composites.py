"""Pins of the oracle's composite iterations against finite differences of
their own total loss, assembled from the (separately pinned) forward pieces.

``oracle.step_paper_losses`` (Eq. 14: the L1 + D-SSIM projection loss of
Eq. 10/12, lambda_tv times the TV of Eq. 11 and lambda_MBC times the
normality loss of Eq. 13) and ``oracle.stage1_step`` (Eq. 10-11: the
rasterized view of Eq. 9 against a measured one, plus the TV of a sub-volume
voxelized from the same Gaussians) both assemble gradients from several
adjoints: the lambda weights, where the TV and normality gradients join the
path's, and the sub-grid placed at the block corner.  Here the total loss is
recomputed from forward calls only -- the motion path's projections, the
voxelized reference volume cut at the block, the basis volumes, the
rasterized view -- and its central differences must match every gradient
kind.  Each case also checks that switching one term off moves the gradient
by far more than the tolerance, so a dropped or misplaced join would fail.
Untruncated Gaussians (the truncation mask is a jump in the parameters)."""
import copy
import math

import numpy as np
import pytest

import oracle
from oracle import rasterize as R
from paper_2503_22139_amd import synth
from paper_2503_22139_amd.synth import GaussSet

EPS = 1e-6
TOL = 1e-5
# central differences of a loss f at step EPS carry a rounding error of about
# 1e-16 |f| / EPS: gradients below FLOOR |f| are compared on that scale
FLOOR = 1e-5


def _f64(s: GaussSet) -> GaussSet:
    return GaussSet(*[np.asarray(x, np.float64).copy() for x in (s.mean, s.scale, s.quat, s.value)])


def _perturb(w, kind, which, idx, eps):
    w2 = copy.copy(w)
    if kind == "coeff":
        c = w.coeff.copy()
        c[idx] += eps
        w2.coeff = c
        return w2
    if which == "ref":
        s = w.ref.copy()
        getattr(s, kind)[idx] += eps
        w2.ref = s
    else:
        mb = list(w.mbc)
        s = mb[which].copy()
        getattr(s, kind)[idx] += eps
        mb[which] = s
        w2.mbc = mb
    return w2


# ------------------------------------------------------------- Eq. 14

CORNER, D = (2, 3, 1), 8


@pytest.fixture(scope="module")
def motion_case():
    w = synth.small_motion(seed=51, n=(14, 12, 10), h=(2.0, 2.5, 3.0), m=80,
                           level_dims=((4, 3, 5), (7, 6, 5), (14, 12, 10)), counts=(4, 8, 16),
                           nviews=2, det=(22, 18), trunc_k=math.inf)
    w.ref = _f64(w.ref)
    # basis values scaled so |E|^2 is of order one: the normality term then
    # weighs about as much as the projection term in the MBC gradients
    w.mbc = [_f64(s) for s in w.mbc]
    for s in w.mbc:
        s.value *= 0.02
    w.coeff = np.asarray(w.coeff, np.float64) * 20.0
    truth = synth.perturbed_truth(w, seed=52)
    target = synth.add_target_noise(oracle.forward(truth), seed=53).astype(np.float64)
    return w, target


def _paper_total(w, target, lam):
    """Eq. 14's objective from forward calls only."""
    proj = oracle.forward(w)
    l_proj, _ = oracle.l1_dssim_loss(proj, target, lam[0])
    ref, bases = oracle.forward_volumes(w)
    block = ref.reshape(w.grid.n)[CORNER[0]:CORNER[0] + D, CORNER[1]:CORNER[1] + D,
                                  CORNER[2]:CORNER[2] + D]
    tv = sum(np.abs(np.diff(block, axis=a)).sum() for a in range(3)) / D ** 3
    norm = [((b.reshape(b.shape[0], -1) ** 2).sum(axis=1) - 1.0) ** 2 for b in bases]
    l_mbc = sum(x.sum() for x in norm) / sum(x.size for x in norm)
    return l_proj + lam[1] * tv + lam[2] * l_mbc


def _grads(w, target, lam):
    losses, g = oracle.step_paper_losses(w, target, CORNER, D, lam[0], lam[1], lam[2])
    return losses, g


def _sel(g, which, kind, idx):
    if kind == "coeff":
        return g["coeff"][idx]
    return (g["ref"] if which == "ref" else g["mbc"][which])[kind][idx]


def test_paper_objective_value(motion_case):
    w, target = motion_case
    lam = (0.25, 0.05, 1.0)
    losses, _ = _grads(w, target, lam)
    assert abs(losses["total"] - _paper_total(w, target, lam)) <= 1e-12 * abs(losses["total"])


@pytest.mark.parametrize("which", ["ref", 0, 2, "coeff"])
def test_paper_objective_gradients_fd(motion_case, which):
    """Central differences of Eq. 14 against step_paper_losses for mean,
    scale, quaternion and value of the reference Gaussians and of two MBC
    levels, and for the coefficients."""
    w, target = motion_case
    lam = (0.25, 0.05, 1.0)
    loss, g = _grads(w, target, lam)
    # the same gradients without the regulariser that joins this parameter
    off = (0.25, 0.0, 1.0) if which == "ref" else (0.25, 0.05, 0.0)
    _, g_off = _grads(w, target, off)
    rng = np.random.default_rng(54 + (0 if which in ("ref", "coeff") else which + 1))
    if which == "coeff":
        checks = [("coeff", tuple(int(rng.integers(d)) for d in w.coeff.shape)) for _ in range(6)]
    else:
        s = w.ref if which == "ref" else w.mbc[which]
        gv = (g["ref"] if which == "ref" else g["mbc"][which])["value"]
        picks = list(np.argsort(-np.abs(gv).sum(axis=1))[:2]) + [int(rng.integers(s.m))]
        checks = []
        for i in picks:
            for kind, nc in (("mean", 3), ("scale", 3), ("quat", 4), ("value", s.value.shape[1])):
                checks += [(kind, (int(i), c)) for c in range(nc)]
    moved = 0.0
    for kind, idx in checks:
        fp = _paper_total(_perturb(w, kind, which, idx, EPS), target, lam)
        fm = _paper_total(_perturb(w, kind, which, idx, -EPS), target, lam)
        fd = (fp - fm) / (2 * EPS)
        an = _sel(g, which, kind, idx)
        scale = max(abs(an), abs(fd), FLOOR * max(1.0, abs(loss["total"])))
        assert abs(fd - an) / scale < TOL, (which, kind, idx, fd, an)
        if kind != "coeff":
            moved = max(moved, abs(an - _sel(g_off, which, kind, idx)) / scale)
    if which != "coeff":
        # the regulariser's share is far above the tolerance
        assert moved > 100 * TOL, moved


# ---------------------------------------------------------- Eq. 10-11

S1_CORNER, S1_D = (3, 2, 4), 6


@pytest.fixture(scope="module")
def stage1_case():
    w = synth.small_motion(seed=61, n=(16, 14, 12), m=40, det=(26, 22), trunc_k=math.inf)
    w.ref = _f64(w.ref)
    ang = 0.7
    target = synth.add_target_noise(
        R.rasterize(synth.perturbed_truth(w, seed=62).ref, w.cone, [ang], math.inf), seed=63)
    return w, np.asarray(target, np.float64), ang


def _stage1_total(w, target, ang, lam_tv):
    p = R.rasterize(w.ref, w.cone, [ang], math.inf)
    l_proj, _ = oracle.l1_dssim_loss(p, target, 0.25)
    ref = oracle.voxelize(w.ref, w.grid, math.inf)[0].reshape(w.grid.n)
    c = S1_CORNER
    block = ref[c[0]:c[0] + S1_D, c[1]:c[1] + S1_D, c[2]:c[2] + S1_D]
    tv = sum(np.abs(np.diff(block, axis=a)).sum() for a in range(3)) / S1_D ** 3
    return l_proj + lam_tv * tv


def test_stage1_gradients_fd(stage1_case):
    """Central differences of Eq. 10-11 (the TV block cut from the full-grid
    voxelization) against stage1_step, whose TV gradient comes from a
    voxelization onto a sub-grid placed at the block."""
    w, target, ang = stage1_case
    lam_tv = 0.05
    losses, g = oracle.stage1_step(w, target, ang, S1_CORNER, S1_D, 0.25, lam_tv)
    total = _stage1_total(w, target, ang, lam_tv)
    assert abs(losses["proj"] + losses["tv"] - total) <= 1e-12 * abs(total)
    _, g_off = oracle.stage1_step(w, target, ang, S1_CORNER, S1_D, 0.25, 0.0)
    # Gaussians whose TV share is largest relative to their gradient, and one more
    share = np.abs(g["value"][:, 0] - g_off["value"][:, 0]) / (np.abs(g["value"][:, 0]) + 1e-30)
    picks = list(np.argsort(-share)[:3]) + [int(np.random.default_rng(64).integers(w.ref.m))]
    moved = 0.0
    for i in picks:
        for kind, nc in (("mean", 3), ("scale", 3), ("quat", 4), ("value", 1)):
            for c in range(nc):
                idx = (int(i), c)
                fp = _stage1_total(_perturb(w, kind, "ref", idx, EPS), target, ang, lam_tv)
                fm = _stage1_total(_perturb(w, kind, "ref", idx, -EPS), target, ang, lam_tv)
                fd = (fp - fm) / (2 * EPS)
                an = g[kind][idx]
                scale = max(abs(an), abs(fd), FLOOR * max(1.0, abs(total)))
                assert abs(fd - an) / scale < TOL, (kind, idx, fd, an)
                moved = max(moved, abs(an - g_off[kind][idx]) / scale)
    assert moved > 100 * TOL, moved
