"""Ragged batches of independent scans (the batched form extended to several
instances): every stage of the motion path is one launch over all scans.

Checked through the C ABI against the FP64 oracle per scan (projections at
1e-4, loss and gradients at 1e-3), against one batched call per scan, and
under graph replay with the views' coefficients and angles replaced between
replays.  Inputs are seeded and synthetic; expected values come from the
oracle only."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2503_22139_amd import ops, synth
from paper_2503_22139_amd.model import GraphStep, MotionModel, MultiScanModel

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


def ragged_scans():
    """Three small scans with different grids, level grids, detectors and
    view counts (one motion-model shape: 3 levels, 2 bases)."""
    return [
        synth.small_motion(seed=51),
        synth.small_motion(seed=52, n=(16, 18, 20), h=(2.5, 2.0, 2.0), m=200,
                           level_dims=((4, 5, 5), (8, 9, 10), (16, 18, 20)), counts=(6, 20, 60),
                           nviews=5, det=(32, 24), du=2.0),
        synth.small_motion(seed=53, n=(20, 16, 12), h=(2.0, 2.0, 3.0), m=150,
                           level_dims=((5, 4, 6), (10, 8, 12), (20, 16, 12)), counts=(5, 16, 40),
                           nviews=2, det=(28, 36), du=2.2),
    ]


def grads_rel(got, want):
    out = {}
    for name in ("mean", "scale", "quat", "value"):
        out[("ref", name)] = rel(N(got["ref"][name]), want["ref"][name])
        for l, (a, b) in enumerate(zip(got["mbc"], want["mbc"])):
            out[("mbc", l, name)] = rel(N(a[name]), b[name])
    out["coeff"] = rel(N(got["coeff"]), want["coeff"])
    return out


def grads_np(g):
    return {"ref": {k: N(v) for k, v in g["ref"].items()},
            "mbc": [{k: N(v) for k, v in d.items()} for d in g["mbc"]],
            "coeff": N(g["coeff"])}


def test_scans_forward_matches_oracle_and_single_calls():
    ws = ragged_scans()
    mm = MultiScanModel(ws)
    projs = mm.forward_batched()
    for k, (w, m, p) in enumerate(zip(ws, mm.models, projs)):
        say("scan", k, w.grid.n, len(w.angles))
        single = m.forward_batched()
        assert rel(N(p), N(single)) <= 1e-6, k
        r = rel(N(p), oracle.forward(w))
        assert r < VOL_TOL, (k, r)


def test_scans_step_matches_oracle():
    ws = ragged_scans()
    targets = [synth.add_target_noise(oracle.forward(synth.perturbed_truth(w))) for w in ws]
    mm = MultiScanModel(ws)
    res = mm.step_batched([T(t) for t in targets])
    sep = mm.step_separate([T(t) for t in targets])
    for k, (w, t, (loss, g), (loss_s, g_s)) in enumerate(zip(ws, targets, res, sep)):
        want_loss, want = oracle.step(w, t)
        say("scan", k, "loss", float(N(loss)), want_loss)
        assert abs(float(N(loss)) - want_loss) <= VOL_TOL * want_loss, k
        for key, r in grads_rel(g, want).items():
            assert r < GRAD_TOL, (k, key, r)
        assert abs(float(N(loss)) - float(N(loss_s))) <= 1e-6 * abs(float(N(loss_s))), k
        for key, r in grads_rel(g, grads_np(g_s)).items():
            assert r < 1e-5, (k, key, r)


def test_scans_graph_replay_with_new_views():
    """The captured ragged iteration, replayed with each scan's coefficients
    and angles replaced in place (a new draw of views), equals the eager
    iteration on those views; eager work runs between replays."""
    ws = ragged_scans()
    targets = [T(synth.random_volume(60 + k, (len(w.angles), w.cone.nv, w.cone.nu), 0.0, 2.0))
               for k, w in enumerate(ws)]
    mm = MultiScanModel(ws)
    gs = GraphStep(mm, targets)
    rng = np.random.default_rng(61)
    for it in range(3):
        coeff = [m.coeff + T(0.1 * rng.standard_normal(tuple(m.coeff.shape))) for m in mm.models]
        angles = [m.angles + float(rng.uniform(0.0, 1.0)) for m in mm.models]
        got = gs.step(targets, coeff=coeff, angles=angles)
        got = [(float(N(l)), grads_np(g)) for l, g in got]
        # eager reference on the same buffers (now holding the new views)
        want = mm.step_batched(targets)
        for k, ((lg, gg), (lw, gw)) in enumerate(zip(got, want)):
            assert abs(lg - float(N(lw))) <= 1e-6 * abs(float(N(lw))), (it, k)
            for key, r in grads_rel(gw, gg).items():
                assert r < 1e-5, (it, k, key, r)
        mm.models[0].step_plain(targets[0])          # eager work between replays
        torch.cuda.synchronize()


def test_c5_scans_batched_equals_separate():
    """The three-scan workload at full size (256x256x128, 192x192x96 and
    128x128x64 grids; 100k / 60k / 25k Gaussians; 32 views each): the ragged
    batch equals one batched call per scan."""
    ws = synth.c5_scans()
    mm = MultiScanModel(ws)
    targets = [T(synth.random_volume(70 + k, (len(w.angles), w.cone.nv, w.cone.nu), 0.0, 20.0))
               for k, w in enumerate(ws)]
    say("c5: ragged forward")
    pr = mm.forward_batched()
    for k, (mdl, p) in enumerate(zip(mm.models, pr)):
        assert rel(N(p), N(mdl.forward_batched())) <= 1e-6, k
    say("c5: ragged step")
    res = mm.step_batched(targets)
    say("c5: separate steps")
    sep = mm.step_separate(targets)
    # Every sum of the path runs in a fixed order or in integers, and each
    # item of the ragged launch does the arithmetic of the separate call, so
    # the two agree to float rounding (in fact bit for bit).
    for k, ((l, g), (ls, gsp)) in enumerate(zip(res, sep)):
        assert abs(float(N(l)) - float(N(ls))) <= 1e-6 * abs(float(N(ls))), k
        r = rel(N(g["coeff"]), N(gsp["coeff"]))
        say("c5: scan", k, "coeff rel", r, "equal", np.array_equal(N(g["coeff"]), N(gsp["coeff"])))
        assert r <= 1e-6, (k, r)
        for name in ("mean", "scale", "quat", "value"):
            r = rel(N(g["ref"][name]), N(gsp["ref"][name]))
            say("c5: scan", k, "ref", name, "rel", r)
            assert r <= 1e-6, (k, name, r)
            for l_ in range(len(g["mbc"])):
                r = rel(N(g["mbc"][l_][name]), N(gsp["mbc"][l_][name]))
                assert r <= 1e-6, (k, "mbc", l_, name, r)
