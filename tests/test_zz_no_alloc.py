"""The allocation-free TV call (pmf_tv_loss_noalloc, static scratch) through
the C ABI against the workspace call pmf_tv_loss on the same inputs: equal
bits for the loss and the accumulated gradient, on consecutive calls whose
block size shrinks (the scratch keeps the previous call's partials), at the
largest supported block, and against the FP64 oracle at the loss bars."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2503_22139_amd import ops, synth

pytestmark = pytest.mark.gpu


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


def both(vol, grid, corner, D, weight, g0):
    """(loss, g) of the workspace call and of the allocation-free call, each
    accumulating onto its own copy of g0."""
    ga = g0.clone()
    la = ops.pmf_tv_loss(vol, grid, corner, D, weight, g_vol=ga)
    gb = g0.clone()
    lb = ops.pmf_tv_loss_noalloc(vol, grid, corner, D, weight, g_vol=gb)
    torch.cuda.synchronize()
    return float(la.cpu()), ga.cpu().numpy(), float(lb.cpu()), gb.cpu().numpy()


def test_noalloc_tv_matches_workspace_call_on_shrinking_blocks():
    grid = synth.Grid((136, 132, 130), (1.5, 1.5, 2.0))
    vol_np = synth.random_volume(31, grid.n, 0.0, 0.05)
    vol = torch.from_numpy(vol_np).cuda()
    g0 = torch.from_numpy(synth.random_normal(32, grid.n, 1e-9)).cuda()
    cases = [((3, 1, 2), ops.TV_NOALLOC_MAX_D),   # the largest block: the whole scratch
             ((40, 17, 9), 32),                    # smaller, after it
             ((100, 90, 97), 7)]                   # smaller again, ragged last block
    for corner, D in cases:
        say("noalloc tv", corner, D)
        la, ga, lb, gb = both(vol, grid, corner, D, 0.05, g0)
        assert la == lb, (la, lb)
        assert np.array_equal(ga, gb)
        want, gw = oracle.tv_loss(vol_np, corner, D, 0.05)
        assert abs(lb - want) <= 1e-4 * abs(want), (lb, want)
        g0n = g0.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(gb - g0n - gw) <= 1e-6 * np.linalg.norm(gw)


def test_noalloc_tv_without_gradient_and_repeat():
    grid = synth.Grid((40, 40, 40), (1.0, 1.0, 1.0))
    vol = torch.from_numpy(synth.random_volume(33, grid.n, 0.0, 1.0)).cuda()
    loss = torch.empty((), device="cuda")
    first = float(ops.pmf_tv_loss_noalloc(vol, grid, (4, 5, 6), 32, 0.05, loss=loss).cpu())
    second = float(ops.pmf_tv_loss_noalloc(vol, grid, (1, 2, 3), 9, 0.05, loss=loss).cpu())
    ref = float(ops.pmf_tv_loss(vol, grid, (1, 2, 3), 9, 0.05).cpu())
    assert second == ref
    again = float(ops.pmf_tv_loss_noalloc(vol, grid, (4, 5, 6), 32, 0.05, loss=loss).cpu())
    assert again == first


def test_noalloc_tv_rejects_blocks_beyond_the_scratch():
    grid = synth.Grid((140, 140, 140), (1.0, 1.0, 1.0))
    vol = torch.zeros(grid.n, device="cuda")
    with pytest.raises(ops.PmfError) as e:
        ops.pmf_tv_loss_noalloc(vol, grid, (0, 0, 0), ops.TV_NOALLOC_MAX_D + 1, 0.05)
    assert e.value.code == ops.PMF_EUNSUPPORTED
    assert "maximum" in str(e.value)
