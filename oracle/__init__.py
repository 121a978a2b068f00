"""FP64 CPU oracle of the PMF-STGR forward model -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (``libpmf.so`` and
its binding) never loads it.

The arithmetic lives in ``pmf_oracle.c`` (plain C, double precision, OpenMP);
this module compiles it with gcc on demand (``build()``) and wraps it with
ctypes.  Every wrapper accepts numpy arrays of any float dtype, promotes them
to float64, and returns float64 arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pmf_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile pmf_oracle.c into liboracle.so (gcc, -O2, OpenMP, IEEE math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fno-fast-math", "-ffp-contract=off",
                               "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = C.CDLL(LIB)
        _lib.oracle_l2_loss.restype = C.c_double
        _lib.oracle_get_threads.restype = C.c_int
    return _lib


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(lib().oracle_get_threads())


# ----------------------------------------------------------------- marshalling

def _d(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _grid(grid):
    n = np.ascontiguousarray(np.asarray(grid.n, dtype=np.int32))
    h = _d(grid.h)
    c = _d(grid.center)
    return n, h, c


def _cone(cone) -> np.ndarray:
    return _d([cone.sad, cone.sdd, cone.du, cone.dv, cone.off_u, cone.off_v, cone.step])


def _size(grid) -> int:
    return int(grid.n[0]) * int(grid.n[1]) * int(grid.n[2])


# ------------------------------------------------------------------ wrappers

def voxelize(gs, grid, k: float = 3.0) -> np.ndarray:
    """Eq. 5 on the grid's voxel centres -> [c][n0][n1][n2]."""
    mean, scale, quat, value = _d(gs.mean), _d(gs.scale), _d(gs.quat), _d(gs.value)
    m, c = value.shape
    n, h, ct = _grid(grid)
    out = np.zeros((c,) + tuple(int(v) for v in grid.n))
    rc = lib().oracle_voxelize(_p(mean), _p(scale), _p(quat), _p(value), C.c_long(m), C.c_int(c),
                               _p(n), _p(h), _p(ct), C.c_double(k), _p(out))
    assert rc == 0
    return out


def voxelize_bwd(gs, grid, k: float, g_vol) -> Dict[str, np.ndarray]:
    mean, scale, quat, value = _d(gs.mean), _d(gs.scale), _d(gs.quat), _d(gs.value)
    m, c = value.shape
    n, h, ct = _grid(grid)
    gv = _d(g_vol)
    assert gv.size == c * _size(grid)
    g = {"mean": np.zeros((m, 3)), "scale": np.zeros((m, 3)), "quat": np.zeros((m, 4)),
         "value": np.zeros((m, c))}
    rc = lib().oracle_voxelize_bwd(_p(mean), _p(scale), _p(quat), _p(value), C.c_long(m), C.c_int(c),
                                   _p(n), _p(h), _p(ct), C.c_double(k), _p(gv), _p(g["mean"]),
                                   _p(g["scale"]), _p(g["quat"]), _p(g["value"]))
    assert rc == 0
    return g


def voxelize_band(gs, grid, k: float, band: float):
    """Eq. 5 split by the mask margin (see oracle_voxelize_band): returns
    (inner, edge, amb, absum), each [c][n0][n1][n2]; inner + edge is
    voxelize(gs, grid, k)."""
    mean, scale, quat, value = _d(gs.mean), _d(gs.scale), _d(gs.quat), _d(gs.value)
    m, c = value.shape
    n, h, ct = _grid(grid)
    shape = (c,) + tuple(int(v) for v in grid.n)
    out = [np.zeros(shape) for _ in range(4)]
    rc = lib().oracle_voxelize_band(_p(mean), _p(scale), _p(quat), _p(value), C.c_long(m),
                                    C.c_int(c), _p(n), _p(h), _p(ct), C.c_double(k),
                                    C.c_double(band), *[_p(o) for o in out])
    assert rc == 0
    return tuple(out)


def voxelize_points(gs, grid, k: float, flat_idx) -> np.ndarray:
    mean, scale, quat, value = _d(gs.mean), _d(gs.scale), _d(gs.quat), _d(gs.value)
    m, c = value.shape
    n, h, ct = _grid(grid)
    idx = np.ascontiguousarray(np.asarray(flat_idx, dtype=np.int64))
    out = np.zeros((idx.size, c))
    rc = lib().oracle_voxelize_points(_p(mean), _p(scale), _p(quat), _p(value), C.c_long(m),
                                      C.c_int(c), _p(n), _p(h), _p(ct), C.c_double(k), _p(idx),
                                      C.c_long(idx.size), _p(out))
    assert rc == 0
    return out


def sample_points(vol, grid, pts, grad: bool = False):
    v = _d(vol)
    p = _d(pts).reshape(-1, 3)
    n, h, ct = _grid(grid)
    out = np.zeros(p.shape[0])
    g = np.zeros((p.shape[0], 3)) if grad else None
    lib().oracle_sample_points(_p(v), _p(n), _p(h), _p(ct), _p(p), C.c_long(p.shape[0]), _p(out),
                               _p(g) if grad else None)
    return (out, g) if grad else out


def _levels(levels):
    L = len(levels)
    ln = np.ascontiguousarray(np.asarray([g.n for g in levels], dtype=np.int32).reshape(L, 3))
    lh = _d([g.h for g in levels]).reshape(L, 3)
    lc = _d([g.center for g in levels]).reshape(L, 3)
    return ln, lh, lc


def combine(bases: Sequence[np.ndarray], levels, coeff, grid) -> np.ndarray:
    """Eq. 3 -> dvf [V][3][n0][n1][n2]; bases[l] is [3B][n_l], coeff [V][L][B][3]."""
    L = len(levels)
    cf = _d(coeff)
    V, _, B, _ = cf.shape
    bs = [_d(b) for b in bases]
    arr = (C.c_void_p * L)(*[b.ctypes.data for b in bs])
    ln, lh, lc = _levels(levels)
    n, h, ct = _grid(grid)
    out = np.zeros((V, 3) + tuple(int(v) for v in grid.n))
    rc = lib().oracle_combine(C.c_int(L), C.c_int(B), arr, _p(ln), _p(lh), _p(lc), _p(cf), C.c_int(V),
                              _p(n), _p(h), _p(ct), _p(out))
    assert rc == 0
    return out


def combine_bwd(bases, levels, coeff, grid, g_dvf):
    L = len(levels)
    cf = _d(coeff)
    V, _, B, _ = cf.shape
    bs = [_d(b) for b in bases]
    arr = (C.c_void_p * L)(*[b.ctypes.data for b in bs])
    gbs = [np.zeros_like(b) for b in bs]
    garr = (C.c_void_p * L)(*[b.ctypes.data for b in gbs])
    ln, lh, lc = _levels(levels)
    n, h, ct = _grid(grid)
    gd = _d(g_dvf)
    gc = np.zeros_like(cf)
    rc = lib().oracle_combine_bwd(C.c_int(L), C.c_int(B), arr, _p(ln), _p(lh), _p(lc), _p(cf),
                                  C.c_int(V), _p(n), _p(h), _p(ct), _p(gd), garr, _p(gc))
    assert rc == 0
    return gbs, gc


def warp(ref, grid, dvf) -> np.ndarray:
    """Eq. 2 -> [V][n0][n1][n2]; dvf [V][3][...]."""
    r = _d(ref)
    d = _d(dvf)
    V = d.shape[0]
    n, h, ct = _grid(grid)
    out = np.zeros((V,) + tuple(int(v) for v in grid.n))
    rc = lib().oracle_warp(_p(r), _p(n), _p(h), _p(ct), _p(d), C.c_int(V), _p(out))
    assert rc == 0
    return out


def warp_bwd(ref, grid, dvf, g_out):
    r = _d(ref)
    d = _d(dvf)
    V = d.shape[0]
    n, h, ct = _grid(grid)
    go = _d(g_out)
    g_ref = np.zeros(tuple(int(v) for v in grid.n))
    g_dvf = np.zeros_like(d)
    rc = lib().oracle_warp_bwd(_p(r), _p(n), _p(h), _p(ct), _p(d), C.c_int(V), _p(go), _p(g_ref),
                               _p(g_dvf))
    assert rc == 0
    return g_ref, g_dvf


def project(vol, grid, cone, angles, shared: Optional[bool] = None) -> np.ndarray:
    """Eq. 6 -> proj [V][nv][nu].  vol is [N] (shared by all views) or [V][N]."""
    v = _d(vol)
    ang = _d(angles).reshape(-1)
    V = ang.size
    N = _size(grid)
    if shared is None:
        shared = v.size == N
    stride = 0 if shared else N
    assert v.size == (N if shared else V * N)
    n, h, ct = _grid(grid)
    out = np.zeros((V, cone.nv, cone.nu))
    rc = lib().oracle_project(_p(v), C.c_long(stride), _p(n), _p(h), _p(ct), _p(_cone(cone)),
                              C.c_int(cone.nu), C.c_int(cone.nv), _p(ang), C.c_int(V), _p(out))
    assert rc == 0
    return out


def project_rays(vol, grid, cone, angles, rays, shared: Optional[bool] = None) -> np.ndarray:
    """Selected rays; rays is an int array [R][3] of (view, iu, iv)."""
    v = _d(vol)
    ang = _d(angles).reshape(-1)
    N = _size(grid)
    if shared is None:
        shared = v.size == N
    stride = 0 if shared else N
    r = np.ascontiguousarray(np.asarray(rays, dtype=np.int64).reshape(-1, 3))
    n, h, ct = _grid(grid)
    out = np.zeros(r.shape[0])
    rc = lib().oracle_project_rays(_p(v), C.c_long(stride), _p(n), _p(h), _p(ct), _p(_cone(cone)),
                                   C.c_int(cone.nu), C.c_int(cone.nv), _p(ang), _p(r),
                                   C.c_long(r.shape[0]), _p(out))
    assert rc == 0
    return out


def project_bwd(g_proj, grid, cone, angles, shared: bool = False) -> np.ndarray:
    ang = _d(angles).reshape(-1)
    V = ang.size
    N = _size(grid)
    gp = _d(g_proj)
    n, h, ct = _grid(grid)
    if shared:
        out = np.zeros(tuple(int(v) for v in grid.n))
        stride = 0
    else:
        out = np.zeros((V,) + tuple(int(v) for v in grid.n))
        stride = N
    rc = lib().oracle_project_bwd(_p(gp), _p(n), _p(h), _p(ct), _p(_cone(cone)), C.c_int(cone.nu),
                                  C.c_int(cone.nv), _p(ang), C.c_int(V), _p(out), C.c_long(stride))
    assert rc == 0
    return out


def ray_info(grid, cone, theta: float) -> np.ndarray:
    """[nv][nu][4]: (t_n, t_f, number of steps, step) of every pixel's ray."""
    n, h, ct = _grid(grid)
    out = np.zeros((cone.nv, cone.nu, 4))
    lib().oracle_ray_info(_p(n), _p(h), _p(ct), _p(_cone(cone)), C.c_int(cone.nu), C.c_int(cone.nv),
                          C.c_double(theta), _p(out))
    return out


def l2_loss(proj, target):
    p = _d(proj)
    t = _d(target)
    V = p.shape[0]
    g = np.zeros_like(p)
    L = lib().oracle_l2_loss(_p(p), _p(t), C.c_long(p.size // V), C.c_int(V), _p(g))
    return float(L), g


# ------------------------------------------------------------- whole iteration

def forward_volumes(w):
    """Reference volume and MBC basis volumes of a workload."""
    ref = voxelize(w.ref, w.grid, w.trunc_k)[0]
    bases = [voxelize(s, g, w.trunc_k) for s, g in zip(w.mbc, w.levels)]
    return ref, bases


def forward(w, views: Optional[Sequence[int]] = None):
    """Projections of the full motion path (voxelize, Eq. 3, Eq. 2, Eq. 6)."""
    ref, bases = forward_volumes(w)
    vs = list(range(len(w.angles))) if views is None else list(views)
    out = []
    for v in vs:
        dvf = combine(bases, w.levels, w.coeff[v:v + 1], w.grid)
        wv = warp(ref, w.grid, dvf)
        out.append(project(wv, w.grid, w.cone, w.angles[v:v + 1])[0])
    return np.stack(out)


def step(w, target, views: Optional[Sequence[int]] = None):
    """One fwd+bwd iteration of the L2 projection loss, one view at a time.

    Returns (loss, grads) with grads = {"ref": {...}, "mbc": [{...}] * L,
    "coeff": [V][L][B][3]}.  With ``views`` only those views are processed
    (the loss is still normalised by the full batch size V)."""
    V = len(w.angles)
    ref, bases = forward_volumes(w)
    N = _size(w.grid)
    g_ref_vol = np.zeros(N)
    g_bases = [np.zeros_like(b) for b in bases]
    g_coeff = np.zeros(w.coeff.shape)
    loss = 0.0
    vs = list(range(V)) if views is None else list(views)
    for v in vs:
        cv = w.coeff[v:v + 1]
        dvf = combine(bases, w.levels, cv, w.grid)
        wv = warp(ref, w.grid, dvf)
        p = project(wv, w.grid, w.cone, w.angles[v:v + 1])
        r = p - _d(target[v:v + 1])
        loss += float(np.sum(r * r)) / V
        gp = 2.0 * r / V
        gw = project_bwd(gp, w.grid, w.cone, w.angles[v:v + 1])
        gr, gd = warp_bwd(ref, w.grid, dvf, gw)
        g_ref_vol += gr.reshape(-1)
        gb, gc = combine_bwd(bases, w.levels, cv, w.grid, gd)
        for l in range(len(bases)):
            g_bases[l] += gb[l]
        g_coeff[v] = gc[0]
    grads = {"ref": voxelize_bwd(w.ref, w.grid, w.trunc_k, g_ref_vol),
             "mbc": [voxelize_bwd(s, g, w.trunc_k, gb) for s, g, gb in zip(w.mbc, w.levels, g_bases)],
             "coeff": g_coeff}
    return loss, grads


# Stage 2/3 losses around the path (plain numpy, float64)
from .losses import (blur, l1_dssim_loss, mbc_normality_loss, ssim_map,  # noqa: E402,F401
                     ssim_window, tv_loss)


def step_paper_losses(w, target, corner, D: int = 32, lam_ssim: float = 0.25,
                      lam_tv: float = 0.05, lam_mbc: float = 1.0):
    """One fwd+bwd iteration with the Stage 2/3 objective of Eq. 14: the
    L1 + D-SSIM projection loss of Eq. 12 over the batch, lam_mbc times the
    normality loss of Eq. 13 on the basis volumes and lam_tv times the TV of
    Eq. 11 on the D^3 block of the reference volume at `corner`.  Returns
    ({"proj", "tv", "mbc", "total"}, grads) with grads as in step()."""
    V = len(w.angles)
    ref, bases = forward_volumes(w)
    proj = forward(w)
    l_proj, g_proj = l1_dssim_loss(proj, target, lam_ssim)
    N = _size(w.grid)
    g_ref_vol = np.zeros(N)
    g_bases = [np.zeros_like(b) for b in bases]
    g_coeff = np.zeros(w.coeff.shape)
    for v in range(V):
        cv = w.coeff[v:v + 1]
        dvf = combine(bases, w.levels, cv, w.grid)
        gw = project_bwd(g_proj[v:v + 1], w.grid, w.cone, w.angles[v:v + 1])
        gr, gd = warp_bwd(ref, w.grid, dvf, gw)
        g_ref_vol += gr.reshape(-1)
        gb, gc = combine_bwd(bases, w.levels, cv, w.grid, gd)
        for l in range(len(bases)):
            g_bases[l] += gb[l]
        g_coeff[v] = gc[0]
    l_tv, g_tv = tv_loss(ref.reshape(w.grid.n), corner, D, lam_tv)
    g_ref_vol += g_tv.reshape(-1)
    l_mbc, g_mbc = mbc_normality_loss(bases, lam_mbc)
    for l in range(len(bases)):
        g_bases[l] += g_mbc[l]
    grads = {"ref": voxelize_bwd(w.ref, w.grid, w.trunc_k, g_ref_vol),
             "mbc": [voxelize_bwd(s, g, w.trunc_k, gb) for s, g, gb in zip(w.mbc, w.levels, g_bases)],
             "coeff": g_coeff}
    losses = {"proj": l_proj, "tv": l_tv, "mbc": l_mbc, "total": l_proj + l_tv + l_mbc}
    return losses, grads


def stage1_step(w, target, angle: float, corner, D: int = 32, lam_ssim: float = 0.25,
                lam_tv: float = 0.05):
    """One Stage 1 iteration (Eq. 10-11): the rasterized view (Eq. 9) of the
    reference Gaussians against the measured projection with L1 + lam_ssim
    D-SSIM, plus lam_tv times the TV of the D^3 block of the reference grid
    at `corner`, voxelized from the same Gaussians.  Returns
    ({"proj", "tv"}, {"mean", "scale", "quat", "value"})."""
    from types import SimpleNamespace
    from . import rasterize as _r
    p = _r.rasterize(w.ref, w.cone, [angle], w.trunc_k)
    l_proj, g_proj = l1_dssim_loss(p, target, lam_ssim)
    grads = _r.rasterize_bwd(w.ref, w.cone, [angle], w.trunc_k, g_proj)
    c = [w.grid.center[a] + (corner[a] + (D - 1) / 2.0 - (w.grid.n[a] - 1) / 2.0) * w.grid.h[a]
         for a in range(3)]
    sg = SimpleNamespace(n=(D, D, D), h=tuple(w.grid.h), center=tuple(c))
    sub = voxelize(w.ref, sg, w.trunc_k)[0].reshape(D, D, D)
    l_tv, g_sub = tv_loss(sub, (0, 0, 0), D, lam_tv)
    gt = voxelize_bwd(w.ref, sg, w.trunc_k, g_sub.reshape(1, -1))
    for name in grads:
        grads[name] = grads[name] + gt[name]
    return {"proj": l_proj, "tv": l_tv}, grads
