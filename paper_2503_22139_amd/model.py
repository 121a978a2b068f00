"""One fwd+bwd iteration of the motion path, in two schedules.

``MotionModel`` holds the device copies of a workload's parameters (reference
Gaussians, MBC Gaussians per level, per-view temporal coefficients, view
angles) and runs the Stage 2/3 forward model of Sec. 2.3.2 with an L2
projection loss:

  plain   -- one view at a time, as a per-view projector would be driven:
             combine (Eq. 3), warp (Eq. 2) and project (Eq. 6) for view v,
             then the adjoints of view v in reverse, per-view DVFs kept.
  batched -- all views at once: the fused motion path (DVFs never stored,
             bases read once) and its fused adjoint.

Both return the same loss and gradients (up to float32 summation order).
Every step is a libpmf.so call; Python only orders the calls.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np
import torch

from . import ops
from .synth import GaussSet, Workload


@dataclasses.dataclass
class GaussT:
    mean: torch.Tensor
    scale: torch.Tensor
    quat: torch.Tensor
    value: torch.Tensor

    @staticmethod
    def from_set(s: GaussSet, device) -> "GaussT":
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        return GaussT(f(s.mean), f(s.scale), f(s.quat), f(s.value))


class MotionModel:
    def __init__(self, w: Workload, device="cuda"):
        self.w = w
        self.device = torch.device(device)
        self.grid = w.grid
        self.cone = w.cone
        self.levels = list(w.levels)
        self.k = float(w.trunc_k)
        self.ref = GaussT.from_set(w.ref, self.device)
        self.mbc = [GaussT.from_set(s, self.device) for s in w.mbc]
        self.coeff = torch.from_numpy(np.ascontiguousarray(w.coeff, np.float32)).to(self.device)
        self.angles = torch.from_numpy(np.ascontiguousarray(w.angles, np.float32)).to(self.device)
        self.V = int(self.angles.numel())

    # ------------------------------------------------------------ volumes
    def _side_streams(self):
        """One stream per MBC level (default priority), created on first use:
        the levels' voxelizations and adjoints run beside the reference's."""
        if getattr(self, "_streams", None) is None:
            self._streams = [torch.cuda.Stream(device=self.device) for _ in self.mbc]
        return self._streams

    def volumes(self):
        cur = torch.cuda.current_stream(self.device)
        side = self._side_streams()
        bases = [None] * len(self.mbc)
        for s_, g, lg, l in zip(side, self.mbc, self.levels, range(len(self.mbc))):
            s_.wait_stream(cur)
            with torch.cuda.stream(s_):
                bases[l] = ops.pmf_voxelize(g.mean, g.scale, g.quat, g.value, lg, self.k)
        ref = ops.pmf_voxelize(self.ref.mean, self.ref.scale, self.ref.quat, self.ref.value,
                               self.grid, self.k)[0]
        for s_, b in zip(side, bases):
            cur.wait_stream(s_)
            b.record_stream(cur)
        return ref, bases

    def volumes_bwd(self, g_ref, g_bases) -> Dict[str, object]:
        cur = torch.cuda.current_stream(self.device)
        side = self._side_streams()
        mbc = [None] * len(self.mbc)
        for s_, g, lg, gb, l in zip(side, self.mbc, self.levels, g_bases, range(len(self.mbc))):
            s_.wait_stream(cur)
            with torch.cuda.stream(s_):
                mbc[l] = ops.pmf_voxelize_bwd(g.mean, g.scale, g.quat, g.value, lg, self.k, gb)
            gb.record_stream(s_)
        r = ops.pmf_voxelize_bwd(self.ref.mean, self.ref.scale, self.ref.quat, self.ref.value,
                                 self.grid, self.k, g_ref.reshape(1, -1))
        out = {"ref": dict(zip(("mean", "scale", "quat", "value"), r)), "mbc": []}
        for s_, grads in zip(side, mbc):
            cur.wait_stream(s_)
            for t in grads:
                t.record_stream(cur)
            out["mbc"].append(dict(zip(("mean", "scale", "quat", "value"), grads)))
        return out

    # ------------------------------------------------------------ forward
    def forward_plain(self, ref=None, bases=None):
        if ref is None:
            ref, bases = self.volumes()
        proj = ops._empty((self.V, self.cone.nv, self.cone.nu), self.device)
        for v in range(self.V):
            dvf = ops.pmf_combine_dvf(bases, self.levels, self.coeff[v:v + 1], self.grid)
            wv = ops.pmf_warp(ref, self.grid, dvf)
            ops.pmf_project(wv, self.grid, self.cone, self.angles[v:v + 1], shared=False,
                            out=proj[v:v + 1])
        return proj

    def forward_batched(self, ref=None, bases=None):
        if ref is None:
            ref, bases = self.volumes()
        return ops.pmf_warp_project(ref, self.grid, bases, self.levels, self.coeff, self.cone,
                                    self.angles)

    # ------------------------------------------------------- fwd + bwd
    def step_plain(self, target):
        """One iteration, one view at a time (per-view DVFs kept for the backward)."""
        ref, bases = self.volumes()
        proj = ops._empty((self.V, self.cone.nv, self.cone.nu), self.device)
        dvfs = []
        for v in range(self.V):
            dvf = ops.pmf_combine_dvf(bases, self.levels, self.coeff[v:v + 1], self.grid)
            wv = ops.pmf_warp(ref, self.grid, dvf)
            ops.pmf_project(wv, self.grid, self.cone, self.angles[v:v + 1], shared=False,
                            out=proj[v:v + 1])
            dvfs.append(dvf)
        loss, g_proj = ops.pmf_l2_loss(proj, target)
        g_ref, g_bases = None, None
        g_coeff = ops._empty_like(self.coeff)
        for v in reversed(range(self.V)):
            g_wv = ops.pmf_project_bwd(g_proj[v:v + 1], self.grid, self.cone, self.angles[v:v + 1])
            gr, gd = ops.pmf_warp_bwd(ref, self.grid, dvfs[v], g_wv)
            gb, _ = ops.pmf_combine_dvf_bwd(bases, self.levels, self.coeff[v:v + 1], self.grid, gd,
                                            g_coeff_out=g_coeff[v:v + 1])
            if g_ref is None:
                g_ref, g_bases = gr, gb
            else:
                ops.pmf_accumulate(g_ref, gr)
                for a, b in zip(g_bases, gb):
                    ops.pmf_accumulate(a, b)
        grads = self.volumes_bwd(g_ref, g_bases)
        grads["coeff"] = g_coeff
        return loss, grads

    def step_batched(self, target):
        """One iteration with the fused motion path (no stored DVFs or warped volumes)."""
        ref, bases = self.volumes()
        proj = ops.pmf_warp_project(ref, self.grid, bases, self.levels, self.coeff, self.cone,
                                    self.angles)
        loss, g_proj = ops.pmf_l2_loss(proj, target)
        g_ref, g_bases, g_coeff = ops.pmf_warp_project_bwd(ref, self.grid, bases, self.levels,
                                                           self.coeff, self.cone, self.angles, g_proj)
        grads = self.volumes_bwd(g_ref, g_bases)
        grads["coeff"] = g_coeff
        return loss, grads


    def step_batched_paper(self, target, corner, D: int = 32, lam_ssim: float = 0.25,
                           lam_tv: float = 0.05, lam_mbc: float = 1.0):
        """One iteration with the Stage 2/3 objective (Eq. 14): L1 + D-SSIM
        projection loss (Eq. 12), lam_mbc x MBC normality (Eq. 13) and lam_tv x
        TV of the D^3 block of the reference volume at `corner` (Eq. 11); the
        regularisers add their gradients onto those of the motion path before
        the voxelization adjoints.  Returns ({"proj", "tv", "mbc"} device
        scalars, grads)."""
        ref, bases = self.volumes()
        proj = ops.pmf_warp_project(ref, self.grid, bases, self.levels, self.coeff, self.cone,
                                    self.angles)
        l_proj, g_proj = ops.pmf_l1_dssim_loss(proj, target, lam_ssim)
        g_ref, g_bases, g_coeff = ops.pmf_warp_project_bwd(ref, self.grid, bases, self.levels,
                                                           self.coeff, self.cone, self.angles, g_proj)
        l_tv = ops.pmf_tv_loss(ref, self.grid, corner, D, lam_tv, g_vol=g_ref)
        l_mbc = ops.pmf_mbc_normality_loss(bases, self.levels, lam_mbc, g_bases=g_bases)
        grads = self.volumes_bwd(g_ref, g_bases)
        grads["coeff"] = g_coeff
        return {"proj": l_proj, "tv": l_tv, "mbc": l_mbc}, grads


def sub_grid(grid, corner, D: int):
    """The D^3 block of `grid` whose first voxel is `corner`, as a grid of its own."""
    from .synth import Grid
    c = [grid.center[a] + (corner[a] + (D - 1) / 2.0 - (grid.n[a] - 1) / 2.0) * grid.h[a]
         for a in range(3)]
    return Grid((D, D, D), tuple(grid.h), tuple(c))


class Stage1Model:
    """Stage 1 of the training (Sec. 2.3.2, Eq. 10-11): the reference
    Gaussians drawn by the X-ray rasterizer (Eq. 9) at one view per
    iteration, the L1 + D-SSIM loss against the measured projection, and the
    TV of a D^3 sub-volume voxelized from the same Gaussians (Eq. 11)."""

    def __init__(self, w: Workload, device="cuda"):
        self.device = torch.device(device)
        self.grid = w.grid
        self.cone = w.cone
        self.k = float(w.trunc_k)
        self.ref = GaussT.from_set(w.ref, self.device)

    def step(self, target, angle, corner, D: int = 32, lam_ssim: float = 0.25,
             lam_tv: float = 0.05):
        """target [1][nv][nu], angle [1] (device); returns ({"proj", "tv"}
        device scalars, {"mean", "scale", "quat", "value"} gradients)."""
        g = self.ref
        V = angle.numel()
        if getattr(self, "_rws_key", None) != (g.mean.shape[0], V):
            self._rws = ops.rasterize_workspace(g.mean.shape[0], self.cone, V, self.device)
            self._rws_key = (g.mean.shape[0], V)
        # the adjoint reuses the forward's binning in the step's own workspace
        proj = ops.pmf_rasterize(g.mean, g.scale, g.quat, g.value, self.cone, angle, self.k,
                                 ws=self._rws)
        l_proj, g_proj = ops.pmf_l1_dssim_loss(proj, target, lam_ssim)
        grads = ops.pmf_rasterize_bwd(g.mean, g.scale, g.quat, g.value, self.cone, angle, self.k,
                                      g_proj, ws=self._rws, binned=True)
        sg = sub_grid(self.grid, corner, D)
        sub = ops.pmf_voxelize(g.mean, g.scale, g.quat, g.value, sg, self.k)
        g_sub = ops.pmf_fill(ops._empty_like(sub), 0.0)
        l_tv = ops.pmf_tv_loss(sub, sg, (0, 0, 0), D, lam_tv, g_vol=g_sub)
        tv = ops.pmf_voxelize_bwd(g.mean, g.scale, g.quat, g.value, sg, self.k, g_sub)
        for a, b in zip(grads, tv):
            ops.pmf_accumulate(a, b)
        return {"proj": l_proj, "tv": l_tv}, dict(zip(("mean", "scale", "quat", "value"), grads))


class MultiScanModel:
    """Several independent scans (different grids, geometries and view counts,
    one motion-model shape L, B) stepped together: per scan the voxelization
    and its adjoint, and for all scans at once the ragged batched motion path
    (each stage one kernel launch over every scan's voxels, tiles and bricks)."""

    def __init__(self, workloads, device="cuda"):
        self.models = [MotionModel(w, device) for w in workloads]
        shapes = {tuple(m.coeff.shape[1:]) for m in self.models}
        if len(shapes) != 1:
            raise ValueError(f"scans must share the motion-model shape (L, B, 3): {shapes}")

    def _scans(self, vols):
        return [dict(ref=r, grid=m.grid, bases=b, levels=m.levels, coeff=m.coeff, cone=m.cone,
                     angles=m.angles) for m, (r, b) in zip(self.models, vols)]

    def forward_batched(self):
        return ops.pmf_warp_project_scans(self._scans([m.volumes() for m in self.models]))

    def step_batched(self, targets):
        """One iteration of every scan; returns [(loss, grads)] per scan."""
        scans = self._scans([m.volumes() for m in self.models])
        projs = ops.pmf_warp_project_scans(scans)
        losses = []
        for sc, p, t in zip(scans, projs, targets):
            loss, g_proj = ops.pmf_l2_loss(p, t)
            sc["g_proj"] = g_proj
            losses.append(loss)
        outs = ops.pmf_warp_project_bwd_scans(scans)
        res = []
        for m, (g_ref, g_bases, g_coeff), loss in zip(self.models, outs, losses):
            grads = m.volumes_bwd(g_ref, g_bases)
            grads["coeff"] = g_coeff
            res.append((loss, grads))
        return res

    def step_separate(self, targets):
        """The same iteration scan by scan (one batched motion path per scan)."""
        return [m.step_batched(t) for m, t in zip(self.models, targets)]


def _clone(x):
    return [t.clone() for t in x] if isinstance(x, (list, tuple)) else x.clone()


def _copy(dst, src):
    if isinstance(dst, (list, tuple)):
        for d, s_ in zip(dst, src):
            d.copy_(s_)
    else:
        dst.copy_(src)


class GraphStep:
    """A batched iteration recorded once into a HIP graph by the library
    (pmf_graph_capture) and replayed (pmf_graph_replay).

    ``model`` is a MotionModel (target: one tensor) or a MultiScanModel
    (targets: one tensor per scan).  One eager warm-up step on the graph's
    own stream sizes every workspace and allocates the step's outputs in an
    Arena; the recording then reuses exactly those buffers, so it allocates
    nothing and every replay writes the same tensors (``self.out``; read them
    before the next replay).  Before each replay the new targets, and
    optionally new per-view coefficients and angles (the views drawn for this
    iteration), are copied into the device buffers the graph reads.  The
    library's kernels clear memory with fill kernels, never memset nodes
    (pmf_graph_capture refuses a recording with one).
    """

    def __init__(self, model, target, step=None):
        """step(target) is the iteration to record (model.step_batched by
        default, e.g. a closure over model.step_batched_paper)."""
        self.model = model
        self.target = _clone(target)
        fn = model.step_batched if step is None else step
        was = ops.pmf_profile(False)
        try:
            self.stream = torch.cuda.Stream()
            self.stream.wait_stream(torch.cuda.current_stream())
            self.arena = ops.Arena()
            with torch.cuda.stream(self.stream), ops.use_arena(self.arena):
                fn(self.target)                      # warm-up: outputs and workspaces
            self.arena.freeze()
            self.stream.synchronize()
            res = {}

            def record():
                with ops.use_arena(self.arena):
                    res["out"] = fn(self.target)

            self.graph = ops.Graph(record, self.stream)
            self.out = res["out"]
            # the graph holds raw pointers into the scratch buffers: keep them alive
            self._scratch = dict(ops._ws_cache)
        finally:
            ops.pmf_profile(was)

    def _models(self):
        return self.model.models if isinstance(self.model, MultiScanModel) else [self.model]

    def step(self, target=None, coeff=None, angles=None):
        """Replay; coeff / angles (per scan for a MultiScanModel) replace the
        views' temporal coefficients and angles in place (same shapes)."""
        if target is not None:
            _copy(self.target, target)
        ms = self._models()
        if coeff is not None:
            for m, c in zip(ms, coeff if len(ms) > 1 else [coeff]):
                m.coeff.copy_(c)
        if angles is not None:
            for m, a in zip(ms, angles if len(ms) > 1 else [angles]):
                m.angles.copy_(a)
        cur = torch.cuda.current_stream()
        self.stream.wait_stream(cur)
        self.graph.replay()
        cur.wait_stream(self.stream)
        return self.out
