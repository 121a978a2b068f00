"""The Stage 2/3 loss terms (Eq. 10-14) through the C ABI against the FP64
oracle: the L1 + D-SSIM projection loss (ragged tiles and the 32-view
512x384 batch), the TV of a sub-volume and the MBC normality loss (values
and gradients, which both regularisers add onto existing gradients), and a
whole iteration of the motion path with this objective.  Inputs are seeded
and synthetic; expected values come from the oracle only."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2503_22139_amd import ops, synth
from paper_2503_22139_amd.model import MotionModel

pytestmark = pytest.mark.gpu

LOSS_TOL = 1e-4     # scalar losses, as projections
GRAD_TOL = 1e-3


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ops.lib()
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


def pair(seed, V, nv, nu):
    x = synth.projection_like(seed, V, nv, nu)
    y = synth.add_target_noise(synth.projection_like(seed + 1, V, nv, nu) * 0.9 + 0.1 * x, seed)
    return x, y


@pytest.mark.parametrize("shape", [(3, 37, 45), (2, 16, 32), (1, 5, 7)])
def test_l1_dssim_ragged_tiles(shape):
    """Detectors that do not fill the 32 x 16 tiles, and one smaller than the window."""
    V, nv, nu = shape
    x, y = pair(11, V, nv, nu)
    say("l1_dssim", shape)
    loss, g = ops.pmf_l1_dssim_loss(T(x), T(y), 0.25)
    want, gw = oracle.l1_dssim_loss(x, y, 0.25)
    assert abs(float(N(loss)) - want) <= LOSS_TOL * abs(want), (float(N(loss)), want)
    assert rel(N(g), gw) < GRAD_TOL, rel(N(g), gw)


def test_l1_dssim_special_cases():
    x, y = pair(12, 2, 40, 50)
    l0, _ = ops.pmf_l1_dssim_loss(T(y), T(y), 0.25)
    assert abs(float(N(l0))) < 1e-6                       # identical images
    l1, g1 = ops.pmf_l1_dssim_loss(T(x), T(y), 0.0)       # L1 alone
    want, gw = oracle.l1_dssim_loss(x, y, 0.0)
    assert abs(float(N(l1)) - want) <= LOSS_TOL * want
    assert rel(N(g1), gw) < 1e-6
    lw, gn = ops.pmf_l1_dssim_loss(T(x), T(y), 0.25, want_grad=False)
    assert gn is None and abs(float(N(lw)) - oracle.l1_dssim_loss(x, y)[0]) <= LOSS_TOL * want


def test_l1_dssim_full_batch():
    """The 32-view batch on the 512 x 384 detector of the benchmark workload."""
    x, y = pair(13, 32, 384, 512)
    loss, g = ops.pmf_l1_dssim_loss(T(x), T(y), 0.25)
    want, gw = oracle.l1_dssim_loss(x, y, 0.25)
    say("full l1_dssim", float(N(loss)), want, rel(N(g), gw))
    assert abs(float(N(loss)) - want) <= LOSS_TOL * abs(want)
    assert rel(N(g), gw) < GRAD_TOL


@pytest.mark.parametrize("corner", [(10, 20, 5), (32, 32, 32), (0, 0, 0)])
def test_tv_block_adds_its_gradient(corner):
    grid = synth.Grid((64, 64, 64), (1.0, 1.0, 1.0))
    vol = synth.random_volume(21, grid.n, 0.0, 1.0)
    want, gw = oracle.tv_loss(vol, corner, 32, 0.05)
    g = torch.zeros(grid.n, device="cuda")
    loss = ops.pmf_tv_loss(T(vol), grid, corner, 32, 0.05, g_vol=g)
    assert abs(float(N(loss)) - want) <= 1e-5 * want
    assert rel(N(g), gw) < 1e-6         # signs of float differences are exact
    # added onto an existing gradient of the same magnitude
    g0 = synth.random_normal(22, grid.n, 1e-5)
    g = T(g0)
    ops.pmf_tv_loss(T(vol), grid, corner, 32, 0.05, g_vol=g)
    assert rel(N(g), g0 + gw) < 1e-6
    assert float(N(ops.pmf_tv_loss(T(vol), grid, corner, 32, 0.05))) == float(N(loss))


def test_mbc_normality_adds_its_gradient():
    # level 0 has 315 voxels (not a multiple of 4: the scalar kernels), the
    # others take the float4 kernels
    levels = [synth.Grid((9, 7, 5), (8.0, 8.0, 8.0)), synth.Grid((16, 12, 10), (4.0, 4.0, 4.0)),
              synth.Grid((24, 20, 18), (2.0, 2.0, 2.0))]
    bases = [synth.random_normal(31 + l, (9,) + g.n, 0.05) for l, g in enumerate(levels)]
    g0 = [synth.random_normal(41 + l, b.shape, 0.01) for l, b in enumerate(bases)]
    gt = [T(x) for x in g0]
    loss = ops.pmf_mbc_normality_loss([T(b) for b in bases], levels, 1.0, g_bases=gt)
    want, gw = oracle.mbc_normality_loss(bases, 1.0)
    assert abs(float(N(loss)) - want) <= LOSS_TOL * want
    for a, a0, b in zip(gt, g0, gw):
        assert rel(N(a) - a0, b) < 1e-5


def test_mbc_normality_benchmark_levels():
    """The three MBC levels of the benchmark workload (9 channels on 64^3,
    128^3 and 256 x 256 x 128)."""
    w = synth.headline()
    bases = [synth.random_normal(51 + l, (9,) + g.n, 2e-3) for l, g in enumerate(w.levels)]
    gt = [torch.zeros(b.shape, device="cuda") for b in bases]
    loss = ops.pmf_mbc_normality_loss([T(b) for b in bases], w.levels, 1.0, g_bases=gt)
    want, gw = oracle.mbc_normality_loss(bases, 1.0)
    say("normality", float(N(loss)), want)
    assert abs(float(N(loss)) - want) <= LOSS_TOL * want
    for a, b in zip(gt, gw):
        assert rel(N(a), b) < 1e-4


def test_paper_objective_step_matches_oracle():
    """A whole iteration with the Stage 2/3 objective of Eq. 14 on the small
    anisotropic motion case: every loss term and every gradient."""
    w = synth.small_motion()
    target = synth.add_target_noise(oracle.forward(synth.perturbed_truth(w)))
    corner, D = (3, 2, 4), 12
    m = MotionModel(w)
    losses, g = m.step_batched_paper(T(target), corner, D)
    want, gw = oracle.step_paper_losses(w, target, corner, D)
    for k in ("proj", "tv", "mbc"):
        say(k, float(N(losses[k])), want[k])
        assert abs(float(N(losses[k])) - want[k]) <= LOSS_TOL * abs(want[k]), k
    for name in ("mean", "scale", "quat", "value"):
        r = rel(N(g["ref"][name]), gw["ref"][name])
        assert r < GRAD_TOL, ("ref", name, r)
        for l, (a, b) in enumerate(zip(g["mbc"], gw["mbc"])):
            r = rel(N(a[name]), b[name])
            assert r < GRAD_TOL, ("mbc", l, name, r)
    r = rel(N(g["coeff"]), gw["coeff"])
    assert r < GRAD_TOL, ("coeff", r)
