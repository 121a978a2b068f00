"""Configurations and entry forms beyond the base parity cases, through the
C ABI against the FP64 oracle: the paper's own motion model (3 levels, one
basis per level and direction: 9 coefficients per view), two levels of four
bases, displacements far beyond the warp adjoint's LDS halo, the autograd
wrappers, and an exact check of the voxelizer's binning at full size.
Inputs are seeded and synthetic; expected values come from the oracle only."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2503_22139_amd import ops, synth
from paper_2503_22139_amd.model import MotionModel

pytestmark = pytest.mark.gpu

VOL_TOL = 1e-4
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


NAMES = ("mean", "scale", "quat", "value")


def compare_grads(got, want, tag, tol=GRAD_TOL):
    for name in NAMES:
        r = rel(N(got["ref"][name]), want["ref"][name])
        say(tag, "ref", name, r)
        assert r < tol, (tag, "ref", name, r)
    for l, (a, b) in enumerate(zip(got["mbc"], want["mbc"])):
        for name in NAMES:
            r = rel(N(a[name]), b[name])
            say(tag, "mbc", l, name, r)
            assert r < tol, (tag, "mbc", l, name, r)
    r = rel(N(got["coeff"]), want["coeff"])
    say(tag, "coeff", r)
    assert r < tol, (tag, "coeff", r)


def target_of(w):
    return synth.add_target_noise(oracle.forward(synth.perturbed_truth(w)))


def run_both_schedules(w, tag):
    target = target_of(w)
    want_loss, want = oracle.step(w, target)
    m = MotionModel(w)
    for name, fn in (("plain", m.step_plain), ("batched", m.step_batched)):
        say(tag, name)
        loss, grads = fn(T(target))
        got = float(N(loss))
        assert abs(got - want_loss) <= VOL_TOL * want_loss, (tag, name, got, want_loss)
        compare_grads(grads, want, f"{tag}/{name}")
    proj = N(m.forward_batched())
    want_p = oracle.forward(w)
    assert rel(proj, want_p) < VOL_TOL, rel(proj, want_p)


# ------------------------------------------------- motion-model shapes (L, B)

def test_paper_motion_model_three_levels_one_basis():
    """The paper's low-rank model: 3 levels x 3 directions, one basis each,
    i.e. 9 basis volumes and 9 coefficients per view (Sec. 2.3.1, Eq. 3)."""
    w = synth.small_motion(seed=61, nbases=1, nviews=4)
    assert w.coeff.shape[1:] == (3, 1, 3)
    run_both_schedules(w, "L3B1")


def test_two_levels_four_bases():
    w = synth.small_motion(seed=62, level_dims=((7, 6, 5), (24, 20, 18)), counts=(12, 60),
                           nbases=4, nviews=3)
    assert w.coeff.shape[1:] == (2, 4, 3)
    run_both_schedules(w, "L2B4")


def test_one_level_one_basis_and_four_levels():
    w = synth.small_motion(seed=63, level_dims=((24, 20, 18),), counts=(40,), nbases=1, nviews=2)
    run_both_schedules(w, "L1B1")
    w = synth.small_motion(seed=64, level_dims=((4, 4, 4), (6, 5, 9), (12, 10, 9), (24, 20, 18)),
                           counts=(4, 8, 24, 96), nbases=1, nviews=2)
    run_both_schedules(w, "L4B1")


# ------------------------------------------------------ large displacements

def large_motion_case():
    w = synth.small_motion(seed=51, n=(40, 36, 30), h=(1.5, 1.5, 2.0), m=500,
                           level_dims=((10, 9, 15), (20, 18, 15), (40, 36, 30)),
                           counts=(8, 24, 96), nbases=2, nviews=3, det=(64, 48), du=1.2)
    for s in w.mbc:
        s.value = (s.value.astype(np.float64) * 3.0).astype(np.float32)   # N(0, 6 mm)
    return w


def test_large_displacements_beyond_the_adjoint_halo():
    """Displacements up to ~18 voxels (5% of voxel-views beyond 3 voxels):
    the warp adjoint's contributions that leave its LDS box take the global
    path.  Projections, loss and every gradient against the oracle, both
    schedules."""
    w = large_motion_case()
    ref, bases = oracle.forward_volumes(w)
    d = oracle.combine(bases, w.levels, w.coeff, w.grid)
    mag = np.sqrt((d ** 2).sum(1)) / min(w.grid.h)
    say("large motion: max |d| voxels", mag.max(), "beyond 3:", (mag > 3).mean())
    assert mag.max() >= 10.0 and (mag > 3).mean() > 0.01
    run_both_schedules(w, "large")


# ------------------------------------------------------------- autograd

def leaf(a):
    return T(a).requires_grad_(True)


def test_autograd_step_by_step_and_fused():
    """loss.backward() through Voxelize -> CombineDVF -> Warp -> Project ->
    L2Loss, and through Voxelize -> WarpProject -> L2Loss, against the
    oracle's gradients of the same iteration."""
    w = synth.small_motion(seed=65, nviews=3)
    target = target_of(w)
    want_loss, want = oracle.step(w, target)
    for route in ("steps", "fused"):
        say("autograd", route)
        ref_p = [leaf(a) for a in (w.ref.mean, w.ref.scale, w.ref.quat, w.ref.value)]
        mbc_p = [[leaf(a) for a in (s.mean, s.scale, s.quat, s.value)] for s in w.mbc]
        coeff = leaf(w.coeff)
        angles = T(w.angles)
        vol = ops.Voxelize.apply(*ref_p, w.grid, w.trunc_k)
        ref = vol.reshape(tuple(w.grid.n))
        bases = [ops.Voxelize.apply(*p, lg, w.trunc_k) for p, lg in zip(mbc_p, w.levels)]
        if route == "steps":
            dvf = ops.CombineDVF.apply(coeff, w.grid, w.levels, *bases)
            wv = ops.Warp.apply(ref, dvf, w.grid)
            proj = ops.Project.apply(wv, angles, w.grid, w.cone)
        else:
            proj = ops.WarpProject.apply(ref, coeff, angles, w.grid, w.levels, w.cone, *bases)
        loss = ops.L2Loss.apply(proj, T(target))
        loss.backward()
        assert abs(float(N(loss)) - want_loss) <= VOL_TOL * want_loss
        got = {"ref": dict(zip(NAMES, [p.grad for p in ref_p])),
               "mbc": [dict(zip(NAMES, [p.grad for p in ps])) for ps in mbc_p],
               "coeff": coeff.grad}
        compare_grads(got, want, f"autograd/{route}")


# ------------------------------------------------------ binning, exactly

BAND = 1e-3     # pairs with |m - k^2| <= BAND may fall either side of the mask


@pytest.mark.parametrize("which", ["reference_200k", "mbc_16k_9ch"])
def test_voxelize_binning_keeps_every_pair(which):
    """Every (voxel, Gaussian) pair inside the mask reaches the voxel, at the
    benchmark's full size.  With unit values a pair the binning dropped
    would take e^(-m/2) >= e^(-4.5) ~ 0.011 from its voxel, far above the
    float bar of 1e-4 of the voxel's sum of |terms|; pairs within BAND of
    the mask's edge may go either way (several results are correct)."""
    w = synth.headline(nviews=1)
    if which == "reference_200k":
        gs, grid = w.ref.copy(), w.grid
    else:
        gs, grid = w.mbc[2].copy(), w.levels[2]
    gs.value = np.ones_like(gs.value)
    say("binning", which, gs.m, gs.c, grid.n)
    got = N(ops.pmf_voxelize(T(gs.mean), T(gs.scale), T(gs.quat), T(gs.value), grid, 3.0))
    inner, edge, amb, absum = oracle.voxelize_band(gs, grid, 3.0, BAND)
    tol = 1e-4 * absum + 1e-7
    assert tol.max() < 0.25 * math.exp(-4.5)      # a dropped pair would show
    bad = np.abs(got - inner) > amb + tol
    say("binning", which, "voxels off", int(bad.sum()), "max excess",
        float(np.max(np.abs(got - inner) - amb - tol)))
    assert not bad.any(), int(bad.sum())
    # and the whole volume at the volume bar
    assert rel(got, inner + edge) < VOL_TOL


# ------------------------------------------- stale workspace contents

def _poison_workspaces():
    """Fill every cached workspace with 0xFF bytes (NaN as float32)."""
    torch.cuda.synchronize()
    for buf in ops._ws_cache.values():
        buf.fill_(255)
    torch.cuda.synchronize()


def test_workspace_contents_never_leak_into_results():
    """Each entry point writes whatever it reads of its workspace: a second
    call after the cached workspaces were filled with NaN bytes gives the
    same result as the first (bit for bit where the sums are in a fixed
    order)."""
    w = synth.small_motion(seed=66, nviews=3)
    m = MotionModel(w)
    target = T(target_of(w))
    fdk_cone = synth.Cone(1000.0, 1500.0, 101, 77, 1.7, 1.9, off_u=0.4, off_v=-0.3)
    fdk_grid = synth.Grid((37, 41, 19), (2.1, 1.9, 2.5), (1.5, -2.0, 3.0))
    fdk_ang = T(synth.evenly_spaced_angles(48))
    fdk_proj = T(synth.projection_like(67, 48, 77, 101, peak=2.0))
    ref_cpu = w.ref
    rast_cone = synth.Cone(1000.0, 1500.0, 96, 80, 1.0, 1.0)

    def run():
        out = {}
        loss, g = m.step_batched(target)
        out["loss"] = N(loss)
        out["coeff"] = N(g["coeff"])
        out["ref_mean"] = N(g["ref"]["mean"])
        out["mbc2_value"] = N(g["mbc"][2]["value"])
        out["fdk"] = N(ops.pmf_fdk(fdk_proj, fdk_cone, fdk_ang, fdk_grid))
        ssim_l, ssim_g = ops.pmf_l1_dssim_loss(m.forward_batched(), target, 0.25)
        out["ssim"] = N(ssim_l)
        out["ssim_g"] = N(ssim_g)
        p = ops.pmf_rasterize(T(ref_cpu.mean), T(ref_cpu.scale), T(ref_cpu.quat), T(ref_cpu.value),
                              rast_cone, fdk_ang[:2], 3.0)
        out["rast"] = N(p)
        return out

    first = run()
    _poison_workspaces()
    second = run()
    for k in first:
        assert np.all(np.isfinite(second[k])), k
        if k == "rast":     # float sums in an arrival order
            assert rel(second[k], first[k]) < 1e-6, k
        else:
            assert np.array_equal(first[k], second[k]), k


# ------------------------------------------------------------ determinism

def _flat(loss, g):
    out = [N(loss).reshape(-1), N(g["coeff"]).reshape(-1)]
    for name in NAMES:
        out.append(N(g["ref"][name]).reshape(-1))
        for gm in g["mbc"]:
            out.append(N(gm[name]).reshape(-1))
    return out


def test_benchmark_iteration_repeats_bit_for_bit():
    """Two batched iterations of the benchmark workload (32 views,
    256x256x128, 221k Gaussians) give identical bits: every sum on the path
    is in a fixed order or in integers (fixed point), none is a float atomic."""
    w = synth.headline()
    m = MotionModel(w)
    target = T(synth.random_volume(23, (len(w.angles), w.cone.nv, w.cone.nu), 0.0, 20.0))
    a = _flat(*m.step_batched(target))
    b = _flat(*m.step_batched(target))
    for k, (x, y) in enumerate(zip(a, b)):
        assert np.array_equal(x, y), k


def test_plain_schedule_and_large_motion_repeat_bit_for_bit():
    """The plain schedule (warp adjoint in 64-bit fixed point) and the
    batched one with displacements beyond the adjoint's LDS halo (its
    overflow in 64-bit fixed point), twice each."""
    w = large_motion_case()
    m = MotionModel(w)
    target = T(target_of(w))
    for fn in (m.step_plain, m.step_batched):
        a = _flat(*fn(target))
        b = _flat(*fn(target))
        for k, (x, y) in enumerate(zip(a, b)):
            assert np.array_equal(x, y), (fn.__name__, k)


def test_rasterizer_and_untruncated_voxelization_repeat_bit_for_bit():
    """Stage 1's rasterizer (fixed-point pixel sums, large splats walked by
    the tiles) and an untruncated voxelization (every Gaussian on the large
    list) give identical bits twice."""
    w = synth.c2(m=20000, nviews=2)
    g = [T(a) for a in (w.ref.mean, w.ref.scale, w.ref.quat, w.ref.value)]
    ang = T(w.angles)
    small = synth.Cone(1000.0, 1500.0, 96, 80, 2.5, 2.5)
    for cone, k in ((w.cone, 3.0), (small, math.inf)):
        gg = g if k == 3.0 else [t[:300].contiguous() for t in g]
        a = N(ops.pmf_rasterize(*gg, cone, ang, k))
        b = N(ops.pmf_rasterize(*gg, cone, ang, k))
        assert np.array_equal(a, b), k
    f = synth.fd32()
    vg = [T(a) for a in (f.mbc[1].mean, f.mbc[1].scale, f.mbc[1].quat, f.mbc[1].value)]
    a = N(ops.pmf_voxelize(*vg, f.levels[1], math.inf))
    b = N(ops.pmf_voxelize(*vg, f.levels[1], math.inf))
    assert np.array_equal(a, b)


def test_voxelize_adjoint_batch_choices_agree_bit_for_bit():
    """Every PMF_TUNE_VOXELIZE_BWD choice (1 to 64 Gaussians per wavefront)
    gives the same bits: a Gaussian's sums are laid over the lanes and
    reduced the same way whatever batch it sits in.  One-channel column
    walk, nine-channel z-along-lanes walk (a set size that leaves the last
    batch ragged), each against the oracle too."""
    w = synth.small_motion()
    rng = np.random.default_rng(21)
    cases = [(w.ref, w.grid), (synth.gaussians(rng, 203, w.levels[2], c=9, value_sigma=1.0), w.levels[2])]
    knob = ops.PMF_TUNE_VOXELIZE_BWD
    prev = ops.pmf_tune_get(knob)
    try:
        for gs, grid in cases:
            gv = synth.random_normal(31, (gs.c,) + tuple(grid.n))
            want = oracle.voxelize_bwd(gs, grid, 3.0, gv)
            outs = []
            for choice in range(ops.pmf_tune_candidates(knob)):
                ops.pmf_tune_set(knob, choice)
                outs.append([N(t) for t in ops.pmf_voxelize_bwd(
                    T(gs.mean), T(gs.scale), T(gs.quat), T(gs.value), grid, 3.0, T(gv))])
            for o in outs[1:]:
                for x, y in zip(outs[0], o):
                    assert np.array_equal(x, y), gs.c
            for name, g in zip(("mean", "scale", "quat", "value"), outs[0]):
                assert rel(g, want[name]) < GRAD_TOL, (gs.c, name)
    finally:
        ops.pmf_tune_set(knob, prev)


# ---------------------------------------------- graphs and the tuner cache

def test_graph_capture_through_the_abi():
    """pmf_graph_capture records a batched iteration whose outputs come from
    an arena; replays with new coefficients and angles equal eager steps with
    the same inputs; a recording that allocates is refused."""
    from paper_2503_22139_amd.model import GraphStep
    w = synth.small_motion(seed=68, nviews=4)
    m = MotionModel(w)
    target = T(target_of(w))
    gs = GraphStep(m, target)
    assert gs.graph.kernel_count() > 10
    coeff0, ang0 = m.coeff.clone(), m.angles.clone()
    for it in range(3):
        c = coeff0 * (1.0 + 0.1 * it)
        a = ang0 + 0.05 * it
        loss, g = gs.step(target, coeff=c, angles=a)
        got = (float(N(loss)), N(g["coeff"]), N(g["ref"]["mean"]), N(g["mbc"][1]["scale"]))
        m.coeff.copy_(c)
        m.angles.copy_(a)
        le, ge = m.step_batched(target)
        want = (float(N(le)), N(ge["coeff"]), N(ge["ref"]["mean"]), N(ge["mbc"][1]["scale"]))
        assert got[0] == want[0], it
        for x, y in zip(got[1:], want[1:]):
            assert np.array_equal(x, y), it
        torch.cuda.synchronize()
    # a recording that allocates device memory is refused
    x = torch.empty(4096, device="cuda")
    del x
    with pytest.raises((RuntimeError, ops.PmfError)):
        ops.Graph(lambda: torch.empty(4096, device="cuda"), torch.cuda.Stream())


def test_autotune_cache_persists_the_choice(tmp_path):
    _, grid, cone, angles = None, synth.Grid((23, 17, 12), (1.7, 1.1, 2.3), (4.0, -3.0, 2.0)), \
        synth.Cone(800.0, 1300.0, 37, 29, 1.3, 1.1, off_u=0.3, off_v=-1.7), \
        synth.evenly_spaced_angles(7)
    V = len(angles)
    vol = T(synth.random_volume(80, (V,) + tuple(grid.n), 0.0, 1.0))
    gp = T(synth.random_normal(81, (V, cone.nv, cone.nu)))
    tile0 = ops.pmf_tune_get(ops.PMF_TUNE_PROJECT_TILE)
    brick0 = ops.pmf_tune_get(ops.PMF_TUNE_BACKPROJECT_BRICK)
    path = str(tmp_path / "tune.txt")
    try:
        first = ops.pmf_autotune(path, vol, grid, cone, T(angles), gp, reps=1)
        assert not first["cached"] and all(t > 0 for t in first["project_tile_ms"])
        ops.pmf_tune_set(ops.PMF_TUNE_PROJECT_TILE, 0)
        ops.pmf_tune_set(ops.PMF_TUNE_BACKPROJECT_BRICK, 0)
        second = ops.pmf_autotune(path, vol, grid, cone, T(angles), gp, reps=1)
        assert second["cached"]
        assert (second["project_tile"], second["backproject_brick"]) == \
            (first["project_tile"], first["backproject_brick"])
        assert all(t == -1.0 for t in second["project_tile_ms"])      # nothing timed
        lines = open(path).read().splitlines()
        assert len(lines) == 1 and lines[0].count("\t") == 2
        # another geometry misses the cache and adds its own line
        third = ops.pmf_autotune(path, vol[:3].contiguous(), grid, cone, T(angles[:3]),
                                 gp[:3].contiguous(), reps=1)
        assert not third["cached"]
        assert len(open(path).read().splitlines()) == 2
    finally:
        ops.pmf_tune_set(ops.PMF_TUNE_PROJECT_TILE, tile0)
        ops.pmf_tune_set(ops.PMF_TUNE_BACKPROJECT_BRICK, brick0)
