"""Python binding of libpmf.so: argument marshalling only.

Each ``pmf_*`` function here has the name and meaning of the C entry point in
``include/pmf.h``; tensors are CUDA (HIP) float32 tensors whose device
pointers are handed to the library together with torch's current stream.
Nothing is computed in Python: if the library is missing this module raises.

Autograd wrappers (``Voxelize``, ``CombineDVF``, ``Warp``, ``Project``,
``WarpProject``, ``L2Loss``) call the forward entry point in ``forward`` and the adjoint
entry point in ``backward``; they save inputs only, never intermediate
volumes (``WarpProject`` recomputes every view's DVF in its backward).
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import List, Optional, Sequence, Tuple

import torch

from .synth import Cone, Grid

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmf.so")

PMF_OK, PMF_EINVAL, PMF_EHIP, PMF_EWORKSPACE, PMF_EUNSUPPORTED = 0, -1, -2, -3, -4


class PmfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pmf status {code}: {msg}")
        self.code = code


class PmfGrid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("h", C.c_float * 3), ("center", C.c_float * 3)]


class PmfCone(C.Structure):
    _fields_ = [("sad", C.c_float), ("sdd", C.c_float), ("nu", C.c_int32), ("nv", C.c_int32),
                ("du", C.c_float), ("dv", C.c_float), ("off_u", C.c_float), ("off_v", C.c_float),
                ("step", C.c_float)]


class PmfGauss(C.Structure):
    _fields_ = [("mean", C.c_void_p), ("scale", C.c_void_p), ("quat", C.c_void_p),
                ("value", C.c_void_p), ("m", C.c_int64), ("c", C.c_int32)]


class PmfGaussGrad(C.Structure):
    _fields_ = [("mean", C.c_void_p), ("scale", C.c_void_p), ("quat", C.c_void_p),
                ("value", C.c_void_p)]


MAX_SCANS = 4
MAX_LEVELS = 4


class PmfScan(C.Structure):
    _fields_ = [("ref", C.c_void_p), ("grid", PmfGrid), ("bases", C.c_void_p * MAX_LEVELS),
                ("lvl", PmfGrid * MAX_LEVELS), ("coeff", C.c_void_p), ("V", C.c_int32),
                ("cone", PmfCone), ("angles", C.c_void_p), ("proj", C.c_void_p),
                ("g_proj", C.c_void_p), ("g_ref", C.c_void_p),
                ("g_bases", C.c_void_p * MAX_LEVELS), ("g_coeff", C.c_void_p)]


_P = C.c_void_p
_SZ = C.c_size_t
_SIGS = {
    "pmf_version": ([], C.c_int),
    "pmf_last_error": ([], C.c_char_p),
    "pmf_voxelize_workspace": ([C.c_int64, C.c_int32, C.POINTER(PmfGrid)], _SZ),
    "pmf_voxelize": ([C.POINTER(PmfGauss), C.POINTER(PmfGrid), C.c_float, _P, _P, _SZ, _P], C.c_int),
    "pmf_voxelize_bwd": ([C.POINTER(PmfGauss), C.POINTER(PmfGrid), C.c_float, _P,
                          C.POINTER(PmfGaussGrad), _P], C.c_int),
    "pmf_combine_dvf": ([C.c_int, C.c_int, _P, C.POINTER(PmfGrid), _P, C.c_int, C.POINTER(PmfGrid),
                         _P, _P], C.c_int),
    "pmf_combine_dvf_bwd_workspace": ([C.c_int, C.c_int, C.POINTER(PmfGrid), C.c_int,
                                       C.POINTER(PmfGrid)], _SZ),
    "pmf_combine_dvf_bwd": ([C.c_int, C.c_int, _P, C.POINTER(PmfGrid), _P, C.c_int,
                             C.POINTER(PmfGrid), _P, _P, _P, _P, _SZ, _P], C.c_int),
    "pmf_warp": ([_P, C.POINTER(PmfGrid), _P, C.c_int, _P, _P], C.c_int),
    "pmf_warp_bwd_workspace": ([C.POINTER(PmfGrid)], _SZ),
    "pmf_warp_bwd": ([_P, C.POINTER(PmfGrid), _P, C.c_int, _P, _P, _P, _P, _SZ, _P], C.c_int),
    "pmf_project": ([_P, C.c_int64, C.POINTER(PmfGrid), C.POINTER(PmfCone), _P, C.c_int, _P, _P],
                    C.c_int),
    "pmf_project_bwd_workspace": ([C.POINTER(PmfGrid), C.POINTER(PmfCone), C.c_int], _SZ),
    "pmf_project_bwd": ([_P, C.POINTER(PmfGrid), C.POINTER(PmfCone), _P, C.c_int, _P, C.c_int64,
                         _P, _SZ, _P], C.c_int),
    "pmf_l2_loss_workspace": ([C.c_int64, C.c_int], _SZ),
    "pmf_l2_loss": ([_P, _P, C.c_int64, C.c_int, _P, _P, _P, _SZ, _P], C.c_int),
    "pmf_accumulate": ([_P, _P, C.c_int64, _P], C.c_int),
    "pmf_fdk_workspace": ([C.POINTER(PmfCone), C.c_int], _SZ),
    "pmf_fdk": ([_P, C.POINTER(PmfCone), _P, C.c_int, C.POINTER(PmfGrid), _P, _P, _SZ, _P], C.c_int),
    "pmf_grid_init": ([_P, C.POINTER(PmfGrid), C.POINTER(C.c_int), C.c_float, _P, _P, _P, _P, _P],
                      C.c_int),
    "pmf_rasterize_workspace": ([C.c_int64, C.POINTER(PmfCone), C.c_int], _SZ),
    "pmf_rasterize": ([C.POINTER(PmfGauss), C.POINTER(PmfCone), _P, C.c_int, C.c_float, _P, _P,
                       _SZ, _P], C.c_int),
    "pmf_rasterize_bwd": ([C.POINTER(PmfGauss), C.POINTER(PmfCone), _P, C.c_int, C.c_float, _P,
                           C.POINTER(PmfGaussGrad), _P, _SZ, _P], C.c_int),
    "pmf_rasterize_bwd_binned": ([C.POINTER(PmfGauss), C.POINTER(PmfCone), _P, C.c_int, C.c_float, _P,
                           C.POINTER(PmfGaussGrad), _P, _SZ, _P], C.c_int),
    "pmf_l1_dssim_loss_workspace": ([C.c_int, C.c_int, C.c_int], _SZ),
    "pmf_l1_dssim_loss": ([_P, _P, C.c_int, C.c_int, C.c_int, C.c_float, _P, _P, _P, _SZ, _P],
                          C.c_int),
    "pmf_tv_loss_workspace": ([C.c_int], _SZ),
    "pmf_tv_loss": ([_P, C.POINTER(PmfGrid), C.POINTER(C.c_int32), C.c_int, C.c_float, _P, _P, _P,
                     _SZ, _P], C.c_int),
    "pmf_tv_loss_noalloc": ([_P, C.POINTER(PmfGrid), C.POINTER(C.c_int32), C.c_int, C.c_float, _P,
                             _P, _P], C.c_int),
    "pmf_mbc_normality_loss_workspace": ([C.c_int, C.c_int], _SZ),
    "pmf_mbc_normality_loss": ([C.c_int, C.c_int, _P, C.POINTER(PmfGrid), C.c_float, _P, _P, _P,
                                _SZ, _P], C.c_int),
    "pmf_profile": ([C.c_int], C.c_int),
    "pmf_profile_read": ([C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)], C.c_int),
    "pmf_profile_names": ([C.c_char_p, _SZ], _SZ),
    "pmf_warp_project_scans_workspace": ([C.c_int, C.c_int, C.POINTER(PmfScan), C.c_int], _SZ),
    "pmf_warp_project_scans": ([C.c_int, C.c_int, C.POINTER(PmfScan), C.c_int, _P, _SZ, _P], C.c_int),
    "pmf_warp_project_bwd_scans_workspace": ([C.c_int, C.c_int, C.POINTER(PmfScan), C.c_int], _SZ),
    "pmf_warp_project_bwd_scans": ([C.c_int, C.c_int, C.POINTER(PmfScan), C.c_int, _P, _SZ, _P],
                                   C.c_int),
    "pmf_autotune_project": ([_P, C.POINTER(PmfGrid), C.POINTER(PmfCone), _P, C.c_int, _P, _P, _P,
                              _P, _SZ, C.c_int, C.POINTER(C.c_float), _P], C.c_int),
    "pmf_autotune": ([C.c_char_p, _P, C.POINTER(PmfGrid), C.POINTER(PmfCone), _P, C.c_int, _P, _P, _P,
                      _P, _SZ, C.c_int, C.POINTER(C.c_float), C.POINTER(C.c_int), _P], C.c_int),
    "pmf_graph_capture": ([_P, _P, _P, C.POINTER(C.c_void_p)], C.c_int),
    "pmf_graph_replay": ([_P, _P], C.c_int),
    "pmf_graph_kernel_count": ([_P], C.c_int64),
    "pmf_graph_destroy": ([_P], C.c_int),
    "pmf_fill": ([_P, C.c_int64, C.c_float, _P], C.c_int),
    "pmf_tune_candidates": ([C.c_int], C.c_int),
    "pmf_tune_get": ([C.c_int], C.c_int),
    "pmf_tune_set": ([C.c_int, C.c_int], C.c_int),
    "pmf_warp_project_workspace": ([C.c_int, C.c_int, C.POINTER(PmfGrid), C.c_int,
                                    C.POINTER(PmfGrid), C.POINTER(PmfCone)], _SZ),
    "pmf_warp_project": ([_P, C.POINTER(PmfGrid), C.c_int, C.c_int, _P, C.POINTER(PmfGrid), _P,
                          C.c_int, C.POINTER(PmfCone), _P, _P, _P, _SZ, _P], C.c_int),
    "pmf_warp_project_bwd_workspace": ([C.c_int, C.c_int, C.POINTER(PmfGrid), C.c_int,
                                        C.POINTER(PmfGrid), C.POINTER(PmfCone)], _SZ),
    "pmf_warp_project_bwd": ([_P, C.POINTER(PmfGrid), C.c_int, C.c_int, _P, C.POINTER(PmfGrid),
                              _P, C.c_int, C.POINTER(PmfCone), _P, _P, _P, _P, _P, _P, _SZ, _P],
                             C.c_int),
}

_lib = None


def lib():
    """Load libpmf.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run paper_2503_22139_amd.build.build()")
        l = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(l, name)
            f.argtypes = args
            f.restype = res
        _lib = l
    return _lib


def exported_symbols() -> List[str]:
    return list(_SIGS)


def _check(rc: int):
    if rc != PMF_OK:
        raise PmfError(rc, lib().pmf_last_error().decode())


# ------------------------------------------------------------ marshalling

def make_grid(g: Grid) -> PmfGrid:
    s = PmfGrid()
    for a in range(3):
        s.n[a] = int(g.n[a])
        s.h[a] = float(g.h[a])
        s.center[a] = float(g.center[a])
    return s


def make_cone(c: Cone) -> PmfCone:
    return PmfCone(float(c.sad), float(c.sdd), int(c.nu), int(c.nv), float(c.du), float(c.dv),
                   float(c.off_u), float(c.off_v), float(c.step))


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous() and t.dtype == torch.float32, (t.device, t.dtype)
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


_ws_cache = {}


class Arena:
    """The output buffers of a fixed sequence of library calls.

    While an arena is active (``use_arena``), every tensor the binding would
    allocate for a call's outputs comes from it: the first pass over the
    sequence allocates them in call order, and after ``freeze()`` each later
    pass gets the same tensors back in the same order (shapes are checked).
    A step replayed from a graph thus reads and writes fixed buffers, and
    recording it allocates nothing."""

    def __init__(self):
        self.bufs: List[torch.Tensor] = []
        self.frozen = False
        self.pos = 0

    def freeze(self):
        self.frozen = True

    def take(self, shape, device, dtype):
        shape = tuple(int(x) for x in shape)
        if not self.frozen:
            t = torch.empty(shape, device=device, dtype=dtype)
            self.bufs.append(t)
            return t
        if self.pos >= len(self.bufs):
            raise RuntimeError("arena: more outputs than in the first pass")
        t = self.bufs[self.pos]
        if tuple(t.shape) != shape or t.dtype != dtype or t.device != torch.device(device):
            raise RuntimeError(f"arena: output {self.pos} is {tuple(t.shape)}, asked for {shape}")
        self.pos += 1
        return t


_arena: Optional[Arena] = None


class use_arena:
    """Context manager: the binding's outputs come from `arena` (from its
    first buffer on)."""

    def __init__(self, arena: Arena):
        self.arena = arena

    def __enter__(self):
        global _arena
        self.prev = _arena
        self.arena.pos = 0
        _arena = self.arena
        return self.arena

    def __exit__(self, *exc):
        global _arena
        _arena = self.prev
        return False


def _empty(shape, device, dtype=torch.float32) -> torch.Tensor:
    if _arena is not None:
        return _arena.take(shape, device, dtype)
    return torch.empty(tuple(shape), device=device, dtype=dtype)


def _empty_like(t: torch.Tensor) -> torch.Tensor:
    return _empty(t.shape, t.device, t.dtype)


def workspace(nbytes: int, device) -> torch.Tensor:
    """A reusable device scratch buffer of at least nbytes (grown on demand),
    one per device and stream, so calls on different streams never share it."""
    key = (str(device), torch.cuda.current_stream(device).cuda_stream)
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf


def _gauss(mean, scale, quat, value) -> PmfGauss:
    m = mean.shape[0]
    return PmfGauss(_ptr(mean), _ptr(scale), _ptr(quat), _ptr(value), m, value.shape[1])


def _levels(grids: Sequence[Grid]):
    arr = (PmfGrid * len(grids))(*[make_grid(g) for g in grids])
    return arr


def _ptr_array(ts: Sequence[torch.Tensor]):
    return (C.c_void_p * len(ts))(*[t.data_ptr() for t in ts])


# ------------------------------------------------------------ entry points

def pmf_version() -> int:
    return int(lib().pmf_version())


def pmf_voxelize(mean, scale, quat, value, grid: Grid, trunc_k: float = 3.0, out=None):
    c = value.shape[1]
    if out is None:
        out = _empty((c,) + tuple(grid.n), mean.device)
    g = make_grid(grid)
    nbytes = lib().pmf_voxelize_workspace(mean.shape[0], c, C.byref(g))
    ws = workspace(nbytes, mean.device)
    gs = _gauss(mean, scale, quat, value)
    _check(lib().pmf_voxelize(C.byref(gs), C.byref(g), float(trunc_k), _ptr(out),
                              C.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return out


def pmf_voxelize_bwd(mean, scale, quat, value, grid: Grid, trunc_k: float, g_vol):
    gm, gsc, gq, gv = (_empty_like(mean), _empty_like(scale), _empty_like(quat),
                       _empty_like(value))
    g = make_grid(grid)
    gs = _gauss(mean, scale, quat, value)
    gr = PmfGaussGrad(_ptr(gm), _ptr(gsc), _ptr(gq), _ptr(gv))
    _check(lib().pmf_voxelize_bwd(C.byref(gs), C.byref(g), float(trunc_k), _ptr(g_vol.contiguous()),
                                  C.byref(gr), _stream()))
    return gm, gsc, gq, gv


def pmf_combine_dvf(bases: Sequence[torch.Tensor], levels: Sequence[Grid], coeff, grid: Grid, out=None):
    V, L, B, _ = coeff.shape
    if out is None:
        out = _empty((V, 3) + tuple(grid.n), coeff.device)
    lv = _levels(levels)
    og = make_grid(grid)
    _check(lib().pmf_combine_dvf(L, B, _ptr_array(bases), lv, _ptr(coeff), V, C.byref(og), _ptr(out),
                                 _stream()))
    return out


def pmf_combine_dvf_bwd(bases, levels, coeff, grid: Grid, g_dvf, g_coeff_out=None):
    V, L, B, _ = coeff.shape
    lv = _levels(levels)
    og = make_grid(grid)
    g_bases = [_empty_like(b) for b in bases]
    g_coeff = _empty_like(coeff) if g_coeff_out is None else g_coeff_out
    nbytes = lib().pmf_combine_dvf_bwd_workspace(L, B, lv, V, C.byref(og))
    ws = workspace(nbytes, coeff.device)
    _check(lib().pmf_combine_dvf_bwd(L, B, _ptr_array(bases), lv, _ptr(coeff), V, C.byref(og),
                                     _ptr(g_dvf.contiguous()), _ptr_array(g_bases), _ptr(g_coeff),
                                     C.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return g_bases, g_coeff


def pmf_warp(ref, grid: Grid, dvf, out=None):
    V = dvf.shape[0]
    if out is None:
        out = _empty((V,) + tuple(grid.n), ref.device)
    g = make_grid(grid)
    _check(lib().pmf_warp(_ptr(ref), C.byref(g), _ptr(dvf), V, _ptr(out), _stream()))
    return out


def pmf_warp_bwd(ref, grid: Grid, dvf, g_out):
    V = dvf.shape[0]
    g_ref = _empty_like(ref)
    g_dvf = _empty_like(dvf)
    g = make_grid(grid)
    ws = workspace(lib().pmf_warp_bwd_workspace(C.byref(g)), ref.device)
    _check(lib().pmf_warp_bwd(_ptr(ref), C.byref(g), _ptr(dvf), V, _ptr(g_out.contiguous()),
                              _ptr(g_ref), _ptr(g_dvf), C.c_void_p(ws.data_ptr()), ws.numel(),
                              _stream()))
    return g_ref, g_dvf


def pmf_project(vol, grid: Grid, cone: Cone, angles, shared: Optional[bool] = None, out=None):
    V = angles.numel()
    N = grid.size
    if shared is None:
        shared = vol.numel() == N
    stride = 0 if shared else N
    if out is None:
        out = _empty((V, cone.nv, cone.nu), vol.device)
    g = make_grid(grid)
    cn = make_cone(cone)
    _check(lib().pmf_project(_ptr(vol), stride, C.byref(g), C.byref(cn), _ptr(angles), V, _ptr(out),
                             _stream()))
    return out


def pmf_project_bwd(g_proj, grid: Grid, cone: Cone, angles, shared: bool = False, out=None):
    V = angles.numel()
    N = grid.size
    if out is None:
        shape = tuple(grid.n) if shared else (V,) + tuple(grid.n)
        out = _empty(shape, g_proj.device)
    g = make_grid(grid)
    cn = make_cone(cone)
    nbytes = lib().pmf_project_bwd_workspace(C.byref(g), C.byref(cn), V)
    ws = workspace(nbytes, g_proj.device)
    _check(lib().pmf_project_bwd(_ptr(g_proj.contiguous()), C.byref(g), C.byref(cn), _ptr(angles), V,
                                 _ptr(out), 0 if shared else N, C.c_void_p(ws.data_ptr()),
                                 ws.numel(), _stream()))
    return out


def pmf_l2_loss(proj, target, want_grad: bool = True):
    V = proj.shape[0]
    npix = proj[0].numel()
    loss = _empty((), proj.device)
    g = _empty_like(proj) if want_grad else None
    nbytes = lib().pmf_l2_loss_workspace(npix, V)
    ws = workspace(nbytes, proj.device)
    _check(lib().pmf_l2_loss(_ptr(proj), _ptr(target), npix, V, _ptr(loss), _ptr(g),
                             C.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return loss, g


def pmf_fdk(proj, cone: Cone, angles, grid: Grid, out=None):
    """FDK reconstruction of a full-circle scan proj [V][nv][nu] onto grid."""
    V = proj.shape[0]
    if out is None:
        out = _empty(tuple(grid.n), proj.device)
    c = make_cone(cone)
    g = make_grid(grid)
    ws = workspace(lib().pmf_fdk_workspace(C.byref(c), V), proj.device)
    _check(lib().pmf_fdk(_ptr(proj), C.byref(c), _ptr(angles), V, C.byref(g), _ptr(out),
                         C.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return out


def grid_init_lattice(grid: Grid, M: int):
    """Lattice counts (m0, m1, m2) with about M points at equal spacing delta
    in mm over the volume box, and delta: delta = (box volume / M)^(1/3),
    m_a = round(box_len_a / delta) clamped to [1, n_a]."""
    L = [grid.n[a] * grid.h[a] for a in range(3)]
    delta = (L[0] * L[1] * L[2] / float(M)) ** (1.0 / 3.0)
    m = tuple(int(min(max(1, round(L[a] / delta)), grid.n[a])) for a in range(3))
    return m, delta


def pmf_grid_init(vol, grid: Grid, m, scale: float):
    """Initial Gaussians sampled from vol on an m0 x m1 x m2 lattice (Sec.
    2.3.2): (mean [M][3], scale [M][3], quat [M][4], value [M][1])."""
    M = int(m[0]) * int(m[1]) * int(m[2])
    dev = vol.device
    mean = _empty((M, 3), dev)
    sc = _empty((M, 3), dev)
    quat = _empty((M, 4), dev)
    val = _empty((M, 1), dev)
    g = make_grid(grid)
    mm = (C.c_int * 3)(*[int(x) for x in m])
    _check(lib().pmf_grid_init(_ptr(vol), C.byref(g), mm, float(scale), _ptr(mean), _ptr(sc),
                               _ptr(quat), _ptr(val), _stream()))
    return mean, sc, quat, val


def rasterize_workspace(m: int, cone: Cone, V: int, device) -> torch.Tensor:
    """A workspace of its own for a pmf_rasterize / pmf_rasterize_bwd(binned=True) pair."""
    c = make_cone(cone)
    return torch.empty(max(int(lib().pmf_rasterize_workspace(m, C.byref(c), V)), 256),
                       dtype=torch.uint8, device=device)


def pmf_rasterize(mean, scale, quat, value, cone: Cone, angles, trunc_k: float = 3.0, out=None,
                  ws=None):
    """X-ray Gaussian splatting (Eq. 9) of V views: [V][nv][nu].  ws: an own
    workspace (rasterize_workspace) that a following
    pmf_rasterize_bwd(..., ws=ws, binned=True) reuses."""
    V = angles.numel()
    if out is None:
        out = _empty((V, cone.nv, cone.nu), mean.device)
    c = make_cone(cone)
    gs = _gauss(mean, scale, quat, value)
    if ws is None:
        ws = workspace(lib().pmf_rasterize_workspace(mean.shape[0], C.byref(c), V), mean.device)
    _check(lib().pmf_rasterize(C.byref(gs), C.byref(c), _ptr(angles), V, float(trunc_k), _ptr(out),
                               C.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return out


def pmf_rasterize_bwd(mean, scale, quat, value, cone: Cone, angles, trunc_k: float, g_proj,
                      ws=None, binned: bool = False):
    """Gradients of sum(g_proj * rasterize) w.r.t. (mean, scale, quat, value).
    binned=True reuses the binning that pmf_rasterize left in ws (same
    inputs, nothing written to ws since)."""
    V = angles.numel()
    gm, gsc, gq, gv = (_empty_like(mean), _empty_like(scale), _empty_like(quat),
                       _empty_like(value))
    c = make_cone(cone)
    gs = _gauss(mean, scale, quat, value)
    gr = PmfGaussGrad(_ptr(gm), _ptr(gsc), _ptr(gq), _ptr(gv))
    if binned and ws is None:
        raise ValueError("binned=True needs the workspace of the forward call")
    if ws is None:
        ws = workspace(lib().pmf_rasterize_workspace(mean.shape[0], C.byref(c), V), mean.device)
    fn = lib().pmf_rasterize_bwd_binned if binned else lib().pmf_rasterize_bwd
    _check(fn(C.byref(gs), C.byref(c), _ptr(angles), V, float(trunc_k), _ptr(g_proj.contiguous()),
              C.byref(gr), C.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return gm, gsc, gq, gv


def pmf_l1_dssim_loss(proj, target, lambda_ssim: float = 0.25, want_grad: bool = True):
    """L1 + lambda_ssim * D-SSIM of a batch of views (Eq. 10 / 12): (loss, g_proj)."""
    V, nv, nu = proj.shape
    loss = _empty((), proj.device)
    g = _empty_like(proj) if want_grad else None
    nbytes = lib().pmf_l1_dssim_loss_workspace(nu, nv, V)
    ws = workspace(nbytes, proj.device)
    _check(lib().pmf_l1_dssim_loss(_ptr(proj), _ptr(target), nu, nv, V, float(lambda_ssim),
                                   _ptr(loss), _ptr(g), C.c_void_p(ws.data_ptr()), ws.numel(),
                                   _stream()))
    return loss, g


def pmf_tv_loss_noalloc(vol, grid: Grid, corner, D: int, weight: float, g_vol=None, loss=None):
    """pmf_tv_loss without a workspace (the library's static scratch; D <=
    TV_NOALLOC_MAX_D).  loss: an optional preallocated device scalar."""
    if loss is None:
        loss = _empty((), vol.device)
    g = make_grid(grid)
    c = (C.c_int32 * 3)(*[int(x) for x in corner])
    _check(lib().pmf_tv_loss_noalloc(_ptr(vol), C.byref(g), c, int(D), float(weight), _ptr(loss),
                                     _ptr(g_vol), _stream()))
    return loss


TV_NOALLOC_MAX_D = 128


def pmf_tv_loss(vol, grid: Grid, corner, D: int, weight: float, g_vol=None):
    """weight * TV of the D^3 block of vol at corner (Eq. 11); adds
    weight * d TV / d vol into g_vol when given.  Returns the loss."""
    loss = _empty((), vol.device)
    g = make_grid(grid)
    c = (C.c_int32 * 3)(*[int(x) for x in corner])
    nbytes = lib().pmf_tv_loss_workspace(int(D))
    ws = workspace(nbytes, vol.device)
    _check(lib().pmf_tv_loss(_ptr(vol), C.byref(g), c, int(D), float(weight), _ptr(loss),
                             _ptr(g_vol), C.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return loss


def pmf_mbc_normality_loss(bases, levels, weight: float, g_bases=None):
    """weight * MBC normality loss (Eq. 13) of the basis volumes [C][n_l];
    adds weight * d loss / d E into g_bases when given.  Returns the loss."""
    L = len(bases)
    Cc = bases[0].shape[0]
    loss = _empty((), bases[0].device)
    lv = _levels(levels)
    nbytes = lib().pmf_mbc_normality_loss_workspace(L, Cc)
    ws = workspace(nbytes, bases[0].device)
    for b in list(bases) + list(g_bases or []):
        _ptr(b)
    _check(lib().pmf_mbc_normality_loss(L, Cc, _ptr_array(bases), lv, float(weight), _ptr(loss),
                                        _ptr_array(g_bases) if g_bases is not None else None,
                                        C.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return loss


def pmf_accumulate(dst, src):
    """dst += src (same numel), in the library."""
    assert dst.numel() == src.numel()
    _check(lib().pmf_accumulate(_ptr(dst), _ptr(src.contiguous()), dst.numel(), _stream()))
    return dst


def pmf_profile(enable: bool) -> bool:
    return bool(lib().pmf_profile(1 if enable else 0))


def pmf_profile_names() -> List[str]:
    n = lib().pmf_profile_names(None, 0)
    buf = C.create_string_buffer(n + 1)
    lib().pmf_profile_names(buf, n + 1)
    s = buf.value.decode()
    return [x for x in s.split(",") if x]


def pmf_profile_read(kernel: str) -> Tuple[float, int]:
    """(total milliseconds, launches) recorded for one kernel name; clears them."""
    t = C.c_double()
    n = C.c_int64()
    _check(lib().pmf_profile_read(kernel.encode(), C.byref(t), C.byref(n)))
    return float(t.value), int(n.value)


PMF_TUNE_PROJECT_TILE = 0
PMF_TUNE_BACKPROJECT_BRICK = 1
PMF_TUNE_VOXELIZE_BWD = 2


def pmf_tune_candidates(knob: int) -> int:
    return int(lib().pmf_tune_candidates(knob))


def pmf_tune_get(knob: int) -> int:
    rc = lib().pmf_tune_get(knob)
    if rc < 0:
        _check(rc)
    return int(rc)


def pmf_tune_set(knob: int, choice: int) -> int:
    """Select a launch shape; returns the previous choice."""
    rc = lib().pmf_tune_set(knob, choice)
    if rc < 0:
        _check(rc)
    return int(rc)


def pmf_autotune_project(vol, grid: Grid, cone: Cone, angles, g_proj, reps: int = 3):
    """Run the library's autotuner on per-view volumes vol [V][...] and
    residuals g_proj [V][nv][nu]; returns the chosen shapes and the timings
    (ms per launch) of every candidate."""
    V = int(angles.numel())
    g = make_grid(grid)
    cn = make_cone(cone)
    proj = _empty((V, cone.nv, cone.nu), vol.device)
    g_vol = _empty_like(vol)
    nbytes = lib().pmf_project_bwd_workspace(C.byref(g), C.byref(cn), V)
    ws = workspace(nbytes, vol.device)
    nt = pmf_tune_candidates(PMF_TUNE_PROJECT_TILE)
    nb = pmf_tune_candidates(PMF_TUNE_BACKPROJECT_BRICK)
    ms = (C.c_float * (nt + nb))()
    _check(lib().pmf_autotune_project(_ptr(vol), C.byref(g), C.byref(cn), _ptr(angles), V, _ptr(proj),
                                      _ptr(g_proj.contiguous()), _ptr(g_vol),
                                      C.c_void_p(ws.data_ptr()), ws.numel(), reps, ms, _stream()))
    return {"project_tile": pmf_tune_get(PMF_TUNE_PROJECT_TILE),
            "backproject_brick": pmf_tune_get(PMF_TUNE_BACKPROJECT_BRICK),
            "project_tile_ms": [float(x) for x in ms[:nt]],
            "backproject_brick_ms": [float(x) for x in ms[nt:]]}


def pmf_autotune(cache_path: Optional[str], vol, grid: Grid, cone: Cone, angles, g_proj,
                 reps: int = 3):
    """pmf_autotune_project behind the library's shape cache at cache_path
    (None: no cache).  Returns the chosen shapes, whether they came from the
    cache, and the candidates' timings when they were measured."""
    V = int(angles.numel())
    g = make_grid(grid)
    cn = make_cone(cone)
    proj = _empty((V, cone.nv, cone.nu), vol.device)
    g_vol = _empty_like(vol)
    nbytes = lib().pmf_project_bwd_workspace(C.byref(g), C.byref(cn), V)
    ws = workspace(nbytes, vol.device)
    nt = pmf_tune_candidates(PMF_TUNE_PROJECT_TILE)
    nb = pmf_tune_candidates(PMF_TUNE_BACKPROJECT_BRICK)
    ms = (C.c_float * (nt + nb))(*([-1.0] * (nt + nb)))
    hit = C.c_int(0)
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(lib().pmf_autotune(path, _ptr(vol), C.byref(g), C.byref(cn), _ptr(angles), V, _ptr(proj),
                              _ptr(g_proj.contiguous()), _ptr(g_vol), C.c_void_p(ws.data_ptr()),
                              ws.numel(), reps, ms, C.byref(hit), _stream()))
    return {"project_tile": pmf_tune_get(PMF_TUNE_PROJECT_TILE),
            "backproject_brick": pmf_tune_get(PMF_TUNE_BACKPROJECT_BRICK),
            "cached": bool(hit.value),
            "project_tile_ms": [float(x) for x in ms[:nt]],
            "backproject_brick_ms": [float(x) for x in ms[nt:]]}


def pmf_fill(dst, value: float):
    """dst[:] = value, in the library (a fill kernel, never a memset)."""
    _check(lib().pmf_fill(_ptr(dst), dst.numel(), float(value), _stream()))
    return dst


RECORD_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_void_p)


class Graph:
    """The library calls that ``record()`` makes, captured once by
    pmf_graph_capture on ``stream`` (a torch stream; the current one by
    default) and replayed with pmf_graph_replay.  ``record`` runs with that
    stream current and must not allocate device memory (outputs from an
    Arena, workspaces sized beforehand): the capture checks torch's
    allocation counter and refuses a recording that allocated."""

    def __init__(self, record, stream=None):
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        err = []

        def cb(user, sptr):
            try:
                with torch.cuda.stream(self.stream):
                    record()
                return PMF_OK
            except Exception as e:          # re-raised once the capture has ended
                err.append(e)
                return PMF_EINVAL

        dev = self.stream.device
        before = torch.cuda.memory_stats(dev).get("allocation.all.allocated", 0)
        self._fn = RECORD_FN(cb)
        h = C.c_void_p()
        rc = lib().pmf_graph_capture(C.c_void_p(self.stream.cuda_stream), self._fn, None,
                                     C.byref(h))
        self._h = h if rc == PMF_OK else None
        if err:
            raise err[0]
        _check(rc)
        after = torch.cuda.memory_stats(dev).get("allocation.all.allocated", 0)
        if after != before:
            self.close()
            raise RuntimeError("the recorded calls allocated device memory")

    def replay(self, stream=None):
        s = self.stream if stream is None else stream
        _check(lib().pmf_graph_replay(self._h, C.c_void_p(s.cuda_stream)))

    def kernel_count(self) -> int:
        return int(lib().pmf_graph_kernel_count(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _check(lib().pmf_graph_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pmf_warp_project(ref, grid: Grid, bases, levels, coeff, cone: Cone, angles, out=None):
    V, L, B, _ = coeff.shape
    if out is None:
        out = _empty((V, cone.nv, cone.nu), ref.device)
    g = make_grid(grid)
    lv = _levels(levels)
    cn = make_cone(cone)
    nbytes = lib().pmf_warp_project_workspace(L, B, lv, V, C.byref(g), C.byref(cn))
    ws = workspace(nbytes, ref.device)
    _check(lib().pmf_warp_project(_ptr(ref), C.byref(g), L, B, _ptr_array(bases), lv, _ptr(coeff), V,
                                  C.byref(cn), _ptr(angles), _ptr(out), C.c_void_p(ws.data_ptr()),
                                  ws.numel(), _stream()))
    return out


def pmf_warp_project_bwd(ref, grid: Grid, bases, levels, coeff, cone: Cone, angles, g_proj):
    V, L, B, _ = coeff.shape
    g = make_grid(grid)
    lv = _levels(levels)
    cn = make_cone(cone)
    g_ref = _empty_like(ref)
    g_bases = [_empty_like(b) for b in bases]
    g_coeff = _empty_like(coeff)
    nbytes = lib().pmf_warp_project_bwd_workspace(L, B, lv, V, C.byref(g), C.byref(cn))
    ws = workspace(nbytes, ref.device)
    _check(lib().pmf_warp_project_bwd(_ptr(ref), C.byref(g), L, B, _ptr_array(bases), lv,
                                      _ptr(coeff), V, C.byref(cn), _ptr(angles),
                                      _ptr(g_proj.contiguous()), _ptr(g_ref), _ptr_array(g_bases),
                                      _ptr(g_coeff), C.c_void_p(ws.data_ptr()), ws.numel(),
                                      _stream()))
    return g_ref, g_bases, g_coeff


def _scan_array(scans):
    """Host array of PmfScan from dicts with keys ref, grid, bases, levels, coeff,
    cone, angles and optionally proj, g_proj, g_ref, g_bases, g_coeff (tensors)."""
    arr = (PmfScan * len(scans))()
    for k, sc in enumerate(scans):
        a = arr[k]
        a.ref = _ptr(sc["ref"]).value
        a.grid = make_grid(sc["grid"])
        for l, (b, lg) in enumerate(zip(sc["bases"], sc["levels"])):
            a.bases[l] = _ptr(b).value
            a.lvl[l] = make_grid(lg)
        a.coeff = _ptr(sc["coeff"]).value
        a.V = int(sc["coeff"].shape[0])
        a.cone = make_cone(sc["cone"])
        a.angles = _ptr(sc["angles"]).value
        for f in ("proj", "g_proj", "g_ref", "g_coeff"):
            if sc.get(f) is not None:
                setattr(a, f, _ptr(sc[f]).value)
        for l, gb in enumerate(sc.get("g_bases") or []):
            a.g_bases[l] = _ptr(gb).value
    return arr


def pmf_warp_project_scans(scans):
    """Ragged batch of motion-path forwards: one launch per stage over every
    scan.  Each scan dict holds ref, grid, bases, levels, coeff [V][L][B][3],
    cone, angles; returns the list of projections [V][nv][nu]."""
    L, B = int(scans[0]["coeff"].shape[1]), int(scans[0]["coeff"].shape[2])
    dev = scans[0]["ref"].device
    for sc in scans:
        sc["proj"] = _empty((sc["coeff"].shape[0], sc["cone"].nv, sc["cone"].nu), dev)
    arr = _scan_array(scans)
    nbytes = lib().pmf_warp_project_scans_workspace(L, B, arr, len(scans))
    ws = workspace(nbytes, dev)
    _check(lib().pmf_warp_project_scans(L, B, arr, len(scans), C.c_void_p(ws.data_ptr()),
                                        ws.numel(), _stream()))
    return [sc["proj"] for sc in scans]


def pmf_warp_project_bwd_scans(scans):
    """Adjoint of pmf_warp_project_scans given each scan's g_proj: returns a
    list of (g_ref, g_bases, g_coeff)."""
    L, B = int(scans[0]["coeff"].shape[1]), int(scans[0]["coeff"].shape[2])
    dev = scans[0]["ref"].device
    for sc in scans:
        sc["g_proj"] = sc["g_proj"].contiguous()
        sc["g_ref"] = _empty_like(sc["ref"])
        sc["g_bases"] = [_empty_like(b) for b in sc["bases"]]
        sc["g_coeff"] = _empty_like(sc["coeff"])
    arr = _scan_array(scans)
    nbytes = lib().pmf_warp_project_bwd_scans_workspace(L, B, arr, len(scans))
    ws = workspace(nbytes, dev)
    _check(lib().pmf_warp_project_bwd_scans(L, B, arr, len(scans), C.c_void_p(ws.data_ptr()),
                                            ws.numel(), _stream()))
    return [(sc["g_ref"], sc["g_bases"], sc["g_coeff"]) for sc in scans]


# ------------------------------------------------------------ autograd

class Voxelize(torch.autograd.Function):
    """Eq. 5: (mean, scale, quat, value) -> volume [c][n0][n1][n2]."""

    @staticmethod
    def forward(ctx, mean, scale, quat, value, grid: Grid, trunc_k: float = 3.0):
        ctx.save_for_backward(mean, scale, quat, value)
        ctx.grid, ctx.k = grid, trunc_k
        return pmf_voxelize(mean.contiguous(), scale.contiguous(), quat.contiguous(),
                            value.contiguous(), grid, trunc_k)

    @staticmethod
    def backward(ctx, g):
        mean, scale, quat, value = ctx.saved_tensors
        gm, gs, gq, gv = pmf_voxelize_bwd(mean, scale, quat, value, ctx.grid, ctx.k, g.contiguous())
        return gm, gs, gq, gv, None, None


class CombineDVF(torch.autograd.Function):
    """Eq. 3: (coeff [V][L][B][3], bases_l [3B][...]) -> dvf [V][3][...]."""

    @staticmethod
    def forward(ctx, coeff, grid: Grid, levels, *bases):
        ctx.save_for_backward(coeff, *bases)
        ctx.grid, ctx.levels = grid, levels
        return pmf_combine_dvf([b.contiguous() for b in bases], levels, coeff.contiguous(), grid)

    @staticmethod
    def backward(ctx, g):
        coeff, *bases = ctx.saved_tensors
        gb, gc = pmf_combine_dvf_bwd(bases, ctx.levels, coeff, ctx.grid, g.contiguous())
        return (gc, None, None, *gb)


class Warp(torch.autograd.Function):
    """Eq. 2: (ref [...], dvf [V][3][...]) -> [V][...]."""

    @staticmethod
    def forward(ctx, ref, dvf, grid: Grid):
        ctx.save_for_backward(ref, dvf)
        ctx.grid = grid
        return pmf_warp(ref.contiguous(), grid, dvf.contiguous())

    @staticmethod
    def backward(ctx, g):
        ref, dvf = ctx.saved_tensors
        g_ref, g_dvf = pmf_warp_bwd(ref, ctx.grid, dvf, g.contiguous())
        return g_ref, g_dvf, None


class Project(torch.autograd.Function):
    """Eq. 6: volume [V][...] (or one shared [...]) -> projections [V][nv][nu]."""

    @staticmethod
    def forward(ctx, vol, angles, grid: Grid, cone: Cone):
        ctx.save_for_backward(angles)
        ctx.grid, ctx.cone = grid, cone
        ctx.shared = vol.numel() == grid.size
        ctx.shape = vol.shape
        return pmf_project(vol.contiguous(), grid, cone, angles, shared=ctx.shared)

    @staticmethod
    def backward(ctx, g):
        (angles,) = ctx.saved_tensors
        gv = pmf_project_bwd(g.contiguous(), ctx.grid, ctx.cone, angles, shared=ctx.shared)
        return gv.reshape(ctx.shape), None, None, None


class L2Loss(torch.autograd.Function):
    """The L2 projection loss (1/V) sum (proj - target)^2 (pmf_l2_loss); the
    target gets no gradient.  The gradient pmf_l2_loss writes is scaled by the
    incoming scalar gradient (autograd glue)."""

    @staticmethod
    def forward(ctx, proj, target):
        loss, g = pmf_l2_loss(proj.contiguous(), target.contiguous())
        ctx.save_for_backward(g)
        return loss

    @staticmethod
    def backward(ctx, gl):
        (g,) = ctx.saved_tensors
        return g * gl, None


class WarpProject(torch.autograd.Function):
    """Batched Eq. 3 + Eq. 2 + Eq. 6 for all views; the backward recomputes
    each view's DVF instead of storing DVFs or warped volumes."""

    @staticmethod
    def forward(ctx, ref, coeff, angles, grid: Grid, levels, cone: Cone, *bases):
        ctx.save_for_backward(ref, coeff, angles, *bases)
        ctx.grid, ctx.levels, ctx.cone = grid, levels, cone
        return pmf_warp_project(ref.contiguous(), grid, [b.contiguous() for b in bases], levels,
                                coeff.contiguous(), cone, angles)

    @staticmethod
    def backward(ctx, g):
        ref, coeff, angles, *bases = ctx.saved_tensors
        g_ref, g_bases, g_coeff = pmf_warp_project_bwd(ref, ctx.grid, bases, ctx.levels, coeff,
                                                       ctx.cone, angles, g.contiguous())
        return (g_ref, g_coeff, None, None, None, None, *g_bases)
