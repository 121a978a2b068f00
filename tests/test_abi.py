"""The C ABI: libpmf.so loads, exports every function include/pmf.h declares,
and rejects invalid arguments on the host (no GPU needed: argument checks run
before any HIP call, so these calls never reach the runtime)."""
import ctypes as C
import math
import os
import re

import pytest

from paper_2503_22139_amd import ops
from paper_2503_22139_amd.synth import Cone, Grid

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "pmf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pmf_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ops.LIB_PATH):
        from paper_2503_22139_amd import build
        build.build(verbose=False)
    return ops.lib()


def test_exports_every_declared_function(lib):
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(ops.exported_symbols())


def test_noalloc_limit_matches_header():
    src = open(os.path.join(ROOT, "include", "pmf.h")).read()
    m = re.search(r"#define PMF_TV_NOALLOC_MAX_D (\d+)", src)
    assert m and int(m.group(1)) == ops.TV_NOALLOC_MAX_D


def test_version(lib):
    assert lib.pmf_version() == 100


def grid(n=(8, 8, 8), h=(1.0, 1.0, 1.0)):
    return ops.make_grid(Grid(n, h))


def err(lib):
    return lib.pmf_last_error().decode()


def test_voxelize_rejects_bad_arguments(lib):
    g = grid()
    gs = ops.PmfGauss(C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), 10, 1)
    ws = C.c_void_p(256)
    big = 1 << 40
    # null gaussians, bad grid, bad k, too many channels, null output, small workspace
    assert lib.pmf_voxelize(None, C.byref(g), 3.0, C.c_void_p(16), ws, big, None) == ops.PMF_EINVAL
    bad = grid(n=(1, 8, 8))
    assert lib.pmf_voxelize(C.byref(gs), C.byref(bad), 3.0, C.c_void_p(16), ws, big, None) == ops.PMF_EINVAL
    assert "n[0]" in err(lib)
    badh = grid(h=(1.0, 0.0, 1.0))
    assert lib.pmf_voxelize(C.byref(gs), C.byref(badh), 3.0, C.c_void_p(16), ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_voxelize(C.byref(gs), C.byref(g), 0.0, C.c_void_p(16), ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_voxelize(C.byref(gs), C.byref(g), float("nan"), C.c_void_p(16), ws, big, None) == ops.PMF_EINVAL
    gs17 = ops.PmfGauss(C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), 10, 17)
    assert lib.pmf_voxelize(C.byref(gs17), C.byref(g), 3.0, C.c_void_p(16), ws, big, None) == ops.PMF_EUNSUPPORTED
    gs0 = ops.PmfGauss(C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), 10, 0)
    assert lib.pmf_voxelize(C.byref(gs0), C.byref(g), 3.0, C.c_void_p(16), ws, big, None) == ops.PMF_EINVAL
    nullarr = ops.PmfGauss(None, C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), 10, 1)
    assert lib.pmf_voxelize(C.byref(nullarr), C.byref(g), 3.0, C.c_void_p(16), ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_voxelize(C.byref(gs), C.byref(g), 3.0, None, ws, big, None) == ops.PMF_EINVAL
    need = lib.pmf_voxelize_workspace(10, 1, C.byref(g))
    assert need > 0
    assert lib.pmf_voxelize(C.byref(gs), C.byref(g), 3.0, C.c_void_p(16), ws, need - 1, None) == ops.PMF_EWORKSPACE
    assert lib.pmf_voxelize(C.byref(gs), C.byref(g), 3.0, C.c_void_p(16), None, need, None) == ops.PMF_EWORKSPACE
    assert "workspace" in err(lib)


def test_project_rejects_bad_geometry(lib):
    g = grid()
    p = C.c_void_p(16)
    for cone in (Cone(1500.0, 1000.0, 8, 8, 1.0, 1.0),      # SDD < SAD
                 Cone(0.0, 1500.0, 8, 8, 1.0, 1.0),
                 Cone(1000.0, 1500.0, 0, 8, 1.0, 1.0),
                 Cone(1000.0, 1500.0, 8, 8, -1.0, 1.0),
                 Cone(1000.0, 1500.0, 8, 8, 1.0, 1.0, step=float("inf")),
                 Cone(3.0, 1500.0, 8, 8, 1.0, 1.0)):         # source inside the volume box
        c = ops.make_cone(cone)
        assert lib.pmf_project(p, 0, C.byref(g), C.byref(c), p, 1, p, None) == ops.PMF_EINVAL, cone
    c = ops.make_cone(Cone(1000.0, 1500.0, 8, 8, 1.0, 1.0))
    assert lib.pmf_project(p, 0, C.byref(g), C.byref(c), p, 0, p, None) == ops.PMF_EINVAL
    assert lib.pmf_project(p, 5, C.byref(g), C.byref(c), p, 1, p, None) == ops.PMF_EINVAL  # stride < N
    assert lib.pmf_project(None, 0, C.byref(g), C.byref(c), p, 1, p, None) == ops.PMF_EINVAL
    need = lib.pmf_project_bwd_workspace(C.byref(g), C.byref(c), 3)
    assert need >= 3 * 64 * 32
    assert lib.pmf_project_bwd(p, C.byref(g), C.byref(c), p, 3, p, 0, p, need - 1, None) == ops.PMF_EWORKSPACE


def test_combine_and_warp_reject_bad_arguments(lib):
    g = grid()
    lv = (ops.PmfGrid * 2)(grid(), grid(n=(4, 4, 4)))
    bases = (C.c_void_p * 2)(16, 16)
    p = C.c_void_p(16)
    assert lib.pmf_combine_dvf(0, 1, bases, lv, p, 1, C.byref(g), p, None) == ops.PMF_EINVAL
    assert lib.pmf_combine_dvf(5, 1, bases, lv, p, 1, C.byref(g), p, None) == ops.PMF_EUNSUPPORTED
    assert lib.pmf_combine_dvf(2, 5, bases, lv, p, 1, C.byref(g), p, None) == ops.PMF_EUNSUPPORTED
    nb = (C.c_void_p * 2)(16, None)
    assert lib.pmf_combine_dvf(2, 1, nb, lv, p, 1, C.byref(g), p, None) == ops.PMF_EINVAL
    assert lib.pmf_combine_dvf(2, 1, bases, lv, p, 0, C.byref(g), p, None) == ops.PMF_EINVAL
    assert lib.pmf_warp(p, C.byref(g), p, 0, p, None) == ops.PMF_EINVAL
    assert lib.pmf_warp(None, C.byref(g), p, 1, p, None) == ops.PMF_EINVAL
    big = 1 << 40
    assert lib.pmf_warp_bwd(p, C.byref(g), p, 1, p, None, p, p, big, None) == ops.PMF_EINVAL
    assert lib.pmf_warp_bwd(p, C.byref(g), p, 0, p, p, p, p, big, None) == ops.PMF_EINVAL
    need = lib.pmf_warp_bwd_workspace(C.byref(g))
    assert need >= 8 * 8 * 8 * 8
    assert lib.pmf_warp_bwd(p, C.byref(g), p, 1, p, p, p, p, need - 1, None) == ops.PMF_EWORKSPACE
    assert lib.pmf_l2_loss(p, p, 0, 1, p, p, p, 1 << 20, None) == ops.PMF_EINVAL
    assert lib.pmf_accumulate(None, p, 5, None) == ops.PMF_EINVAL
    assert lib.pmf_combine_dvf_bwd_workspace(2, 3, lv, 4, C.byref(g)) > 0


def test_workspace_queries_reject_invalid(lib):
    g = grid()
    assert lib.pmf_voxelize_workspace(-1, 1, C.byref(g)) == 0
    assert lib.pmf_voxelize_workspace(10, 1, None) == 0
    assert lib.pmf_project_bwd_workspace(None, None, 1) == 0
    assert lib.pmf_project_bwd_workspace(C.byref(g), None, 1) == 0
    c = ops.make_cone(Cone(1000.0, 1500.0, 8, 8, 1.0, 1.0))
    lv = (ops.PmfGrid * 1)(grid())
    assert lib.pmf_warp_project_workspace(1, 1, lv, 2, C.byref(g), C.byref(c)) >= 2 * 512 * 4
    assert lib.pmf_warp_project_bwd_workspace(1, 1, lv, 2, C.byref(g), C.byref(c)) > 0


def test_tune_knobs(lib):
    knob = ops.PMF_TUNE_PROJECT_TILE
    n = lib.pmf_tune_candidates(knob)
    assert n >= 2
    assert lib.pmf_tune_candidates(99) == 0
    assert lib.pmf_tune_candidates(ops.PMF_TUNE_VOXELIZE_BWD) == 8
    prev = lib.pmf_tune_get(knob)
    assert 0 <= prev < n
    assert lib.pmf_tune_set(knob, n - 1) == prev
    assert lib.pmf_tune_get(knob) == n - 1
    assert lib.pmf_tune_set(knob, n) == ops.PMF_EINVAL
    assert lib.pmf_tune_set(knob, -1) == ops.PMF_EINVAL
    assert lib.pmf_tune_set(99, 0) == ops.PMF_EINVAL
    assert lib.pmf_tune_get(99) == ops.PMF_EINVAL
    assert lib.pmf_tune_set(knob, prev) == n - 1


def test_scans_reject_bad_arguments(lib):
    s = ops.PmfScan()
    arr = (ops.PmfScan * 2)(s, s)
    assert lib.pmf_warp_project_scans(3, 3, None, 1, None, 0, None) == ops.PMF_EINVAL
    assert lib.pmf_warp_project_scans(3, 3, arr, 0, None, 0, None) == ops.PMF_EINVAL
    assert lib.pmf_warp_project_scans(3, 3, arr, 5, None, 0, None) == ops.PMF_EINVAL
    # scan 1 has a bad grid: the error names it
    good = ops.PmfScan()
    good.grid = grid()
    for l in range(3):
        good.lvl[l] = grid()
        good.bases[l] = 16
        good.g_bases[l] = 16
    good.ref = good.coeff = good.angles = good.proj = good.g_proj = good.g_ref = good.g_coeff = 16
    good.V = 2
    good.cone = ops.make_cone(Cone(1000.0, 1500.0, 16, 16, 1.0, 1.0))
    bad = ops.PmfScan.from_buffer_copy(good)
    bad.grid = grid(n=(8, 1, 8))
    arr = (ops.PmfScan * 2)(good, bad)
    assert lib.pmf_warp_project_scans(3, 3, arr, 2, C.c_void_p(256), 1 << 40, None) == ops.PMF_EINVAL
    assert "scan 1" in err(lib)
    assert lib.pmf_warp_project_bwd_scans(3, 3, arr, 2, C.c_void_p(256), 1 << 40, None) == ops.PMF_EINVAL
    assert "scan 1" in err(lib)
    arr = (ops.PmfScan * 2)(good, good)
    need = lib.pmf_warp_project_scans_workspace(3, 3, arr, 2)
    assert need > 0
    assert lib.pmf_warp_project_scans(3, 3, arr, 2, C.c_void_p(256), need - 1, None) == ops.PMF_EWORKSPACE
    needb = lib.pmf_warp_project_bwd_scans_workspace(3, 3, arr, 2)
    assert needb > need
    nullg = ops.PmfScan.from_buffer_copy(good)
    nullg.g_bases[2] = None
    arr = (ops.PmfScan * 2)(good, nullg)
    assert lib.pmf_warp_project_bwd_scans(3, 3, arr, 2, C.c_void_p(256), 1 << 40, None) == ops.PMF_EINVAL
    assert "g_bases[2]" in err(lib)


def test_autotune_rejects_bad_arguments(lib):
    g = grid()
    cn = ops.make_cone(Cone(1000.0, 1500.0, 16, 16, 1.0, 1.0))
    p = C.c_void_p(256)
    big = 1 << 40
    assert lib.pmf_autotune_project(None, C.byref(g), C.byref(cn), p, 2, p, p, p, p, big, 1, None, None) == ops.PMF_EINVAL
    assert lib.pmf_autotune_project(p, C.byref(g), C.byref(cn), p, 0, p, p, p, p, big, 1, None, None) == ops.PMF_EINVAL
    assert lib.pmf_autotune_project(p, C.byref(g), C.byref(cn), p, 2, p, p, p, p, big, 0, None, None) == ops.PMF_EINVAL
    assert "reps" in err(lib)
    assert lib.pmf_autotune_project(p, C.byref(g), C.byref(cn), p, 2, p, p, p, p, 1, 1, None, None) == ops.PMF_EWORKSPACE


def test_loss_terms_reject_bad_arguments(lib):
    p = C.c_void_p(256)
    ws = C.c_void_p(256)
    big = 1 << 40
    # L1 + D-SSIM: sizes, lambda, null pointers, workspace
    assert lib.pmf_l1_dssim_loss(p, p, 0, 4, 1, 0.25, p, p, ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_l1_dssim_loss(p, p, 4, 4, 1, -1.0, p, p, ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_l1_dssim_loss(p, p, 4, 4, 1, float("nan"), p, p, ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_l1_dssim_loss(None, p, 4, 4, 1, 0.25, p, p, ws, big, None) == ops.PMF_EINVAL
    need = lib.pmf_l1_dssim_loss_workspace(4, 4, 1)
    assert need > 0 and lib.pmf_l1_dssim_loss_workspace(0, 4, 1) == 0
    assert lib.pmf_l1_dssim_loss(p, p, 4, 4, 1, 0.25, p, p, ws, need - 1, None) == ops.PMF_EWORKSPACE
    # TV: block outside the grid, D < 1, null corner / volume, workspace
    g = grid(n=(8, 8, 8))
    c = (C.c_int32 * 3)(0, 0, 0)
    assert lib.pmf_tv_loss(p, C.byref(g), c, 9, 0.05, p, p, ws, big, None) == ops.PMF_EINVAL
    assert "outside" in err(lib)
    c2 = (C.c_int32 * 3)(0, 5, 0)
    assert lib.pmf_tv_loss(p, C.byref(g), c2, 4, 0.05, p, p, ws, big, None) == ops.PMF_EINVAL
    c3 = (C.c_int32 * 3)(-1, 0, 0)
    assert lib.pmf_tv_loss(p, C.byref(g), c3, 4, 0.05, p, p, ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_tv_loss(p, C.byref(g), c, 0, 0.05, p, p, ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_tv_loss(p, C.byref(g), None, 4, 0.05, p, p, ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_tv_loss(None, C.byref(g), c, 4, 0.05, p, p, ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_tv_loss(p, C.byref(g), c, 4, float("inf"), p, p, ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_tv_loss(p, C.byref(g), c, 4, 0.05, p, p, ws, 0, None) == ops.PMF_EWORKSPACE
    # the allocation-free TV call: same checks, and blocks beyond its static scratch
    assert lib.pmf_tv_loss_noalloc(p, C.byref(g), c, 9, 0.05, p, p, None) == ops.PMF_EINVAL
    assert lib.pmf_tv_loss_noalloc(p, C.byref(g), c, 0, 0.05, p, p, None) == ops.PMF_EINVAL
    assert lib.pmf_tv_loss_noalloc(p, C.byref(g), None, 4, 0.05, p, p, None) == ops.PMF_EINVAL
    assert lib.pmf_tv_loss_noalloc(None, C.byref(g), c, 4, 0.05, p, p, None) == ops.PMF_EINVAL
    assert lib.pmf_tv_loss_noalloc(p, C.byref(g), c, 4, float("nan"), p, p, None) == ops.PMF_EINVAL
    gbig = grid(n=(200, 200, 200))
    D = ops.TV_NOALLOC_MAX_D + 1
    assert lib.pmf_tv_loss_noalloc(p, C.byref(gbig), c, D, 0.05, p, p, None) == ops.PMF_EUNSUPPORTED
    assert "maximum" in err(lib)
    # normality: L, C, null pointers, L > 4
    lv = (ops.PmfGrid * 2)(grid(n=(4, 4, 4)), grid(n=(8, 8, 8)))
    bp = (C.c_void_p * 2)(256, 256)
    gp = (C.c_void_p * 2)(256, None)
    assert lib.pmf_mbc_normality_loss(0, 3, bp, lv, 1.0, p, None, ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_mbc_normality_loss(2, 0, bp, lv, 1.0, p, None, ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_mbc_normality_loss(5, 3, bp, lv, 1.0, p, None, ws, big, None) == ops.PMF_EUNSUPPORTED
    assert lib.pmf_mbc_normality_loss(2, 3, None, lv, 1.0, p, None, ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_mbc_normality_loss(2, 3, bp, lv, 1.0, p, gp, ws, big, None) == ops.PMF_EINVAL
    assert "g_bases[1]" in err(lib)
    need = lib.pmf_mbc_normality_loss_workspace(2, 3)
    assert lib.pmf_mbc_normality_loss(2, 3, bp, lv, 1.0, p, None, ws, need - 1, None) == ops.PMF_EWORKSPACE


def test_rasterize_rejects_bad_arguments(lib):
    p = C.c_void_p(256)
    ws = C.c_void_p(256)
    big = 1 << 40
    gs1 = ops.PmfGauss(p, p, p, p, 10, 1)
    gs3 = ops.PmfGauss(p, p, p, p, 10, 3)
    cone = ops.make_cone(Cone(1000.0, 1500.0, 32, 24, 1.0, 1.0))
    bad = ops.make_cone(Cone(1000.0, 900.0, 32, 24, 1.0, 1.0))
    gg = ops.PmfGaussGrad(p, p, p, p)
    assert lib.pmf_rasterize(C.byref(gs3), C.byref(cone), p, 2, 3.0, p, ws, big, None) == ops.PMF_EINVAL
    assert "c = 1" in err(lib)
    assert lib.pmf_rasterize(C.byref(gs1), C.byref(bad), p, 2, 3.0, p, ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_rasterize(C.byref(gs1), C.byref(cone), p, 0, 3.0, p, ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_rasterize(C.byref(gs1), C.byref(cone), p, 2, 0.0, p, ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_rasterize(C.byref(gs1), C.byref(cone), None, 2, 3.0, p, ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_rasterize(C.byref(gs1), C.byref(cone), p, 2, 3.0, None, ws, big, None) == ops.PMF_EINVAL
    need = lib.pmf_rasterize_workspace(10, C.byref(cone), 2)
    assert need > 0
    assert lib.pmf_rasterize(C.byref(gs1), C.byref(cone), p, 2, 3.0, p, ws, need - 1, None) == ops.PMF_EWORKSPACE
    assert lib.pmf_rasterize_bwd(C.byref(gs1), C.byref(cone), p, 2, 3.0, p, None, ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_rasterize_bwd(C.byref(gs1), C.byref(cone), p, 2, 3.0, None, C.byref(gg), ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_rasterize_bwd(C.byref(gs1), C.byref(cone), p, 2, 3.0, p, C.byref(gg), ws, need - 1, None) == ops.PMF_EWORKSPACE
    assert lib.pmf_rasterize_bwd_binned(C.byref(gs3), C.byref(cone), p, 2, 3.0, p, C.byref(gg), ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_rasterize_bwd_binned(C.byref(gs1), C.byref(cone), p, 2, 3.0, None, C.byref(gg), ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_rasterize_bwd_binned(C.byref(gs1), C.byref(cone), p, 2, 3.0, p, C.byref(gg), ws, need - 1, None) == ops.PMF_EWORKSPACE
    huge = ops.PmfGauss(p, p, p, p, 1 << 26, 1)
    assert lib.pmf_rasterize(C.byref(huge), C.byref(cone), p, 4, 3.0, p, ws, big, None) == ops.PMF_EUNSUPPORTED


def test_fdk_rejects_bad_arguments(lib):
    p = C.c_void_p(256)
    ws = C.c_void_p(256)
    big = 1 << 40
    g = grid(n=(16, 16, 8), h=(2.0, 2.0, 2.0))
    cone = ops.make_cone(Cone(1000.0, 1500.0, 32, 24, 1.0, 1.0))
    assert lib.pmf_fdk(p, C.byref(cone), p, 0, C.byref(g), p, ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_fdk(None, C.byref(cone), p, 4, C.byref(g), p, ws, big, None) == ops.PMF_EINVAL
    assert lib.pmf_fdk(p, C.byref(cone), p, 4, C.byref(g), None, ws, big, None) == ops.PMF_EINVAL
    wide = ops.make_cone(Cone(1000.0, 1500.0, 4097, 4, 0.1, 1.0))
    assert lib.pmf_fdk(p, C.byref(wide), p, 4, C.byref(g), p, ws, big, None) == ops.PMF_EUNSUPPORTED
    tall = ops.make_cone(Cone(1000.0, 1500.0, 4096, 40000, 0.01, 0.01))   # 16-byte taps past 2^31
    assert lib.pmf_fdk(p, C.byref(tall), p, 4, C.byref(g), p, ws, big, None) == ops.PMF_EUNSUPPORTED
    huge = grid(n=(2000, 16, 8), h=(2.0, 2.0, 2.0))            # outside the source circle
    assert lib.pmf_fdk(p, C.byref(cone), p, 4, C.byref(huge), p, ws, big, None) == ops.PMF_EINVAL
    need = lib.pmf_fdk_workspace(C.byref(cone), 4)
    assert need > 0
    assert lib.pmf_fdk(p, C.byref(cone), p, 4, C.byref(g), p, ws, need - 1, None) == ops.PMF_EWORKSPACE


def test_grid_init_rejects_bad_arguments(lib):
    p = C.c_void_p(256)
    g = grid(n=(16, 16, 8), h=(2.0, 2.0, 2.0))
    m = lambda *a: (C.c_int * 3)(*a)
    assert lib.pmf_grid_init(p, C.byref(g), m(4, 4, 9), 1.0, p, p, p, p, None) == ops.PMF_EINVAL
    assert lib.pmf_grid_init(p, C.byref(g), m(0, 4, 4), 1.0, p, p, p, p, None) == ops.PMF_EINVAL
    assert lib.pmf_grid_init(p, C.byref(g), m(4, 4, 4), 0.0, p, p, p, p, None) == ops.PMF_EINVAL
    assert lib.pmf_grid_init(p, C.byref(g), m(4, 4, 4), 1.0, p, None, p, p, None) == ops.PMF_EINVAL
    assert lib.pmf_grid_init(None, C.byref(g), m(4, 4, 4), 1.0, p, p, p, p, None) == ops.PMF_EINVAL
    assert ops.grid_init_lattice(Grid((256, 256, 128), (1.5, 1.5, 2.0)), 50_000)[0] == (42, 42, 28)


def test_graph_fill_and_autotune_reject_bad_arguments(lib):
    p = C.c_void_p(16)
    out = C.c_void_p()
    rec = ops.RECORD_FN(lambda u, s: 0)
    # no graph output, legacy default stream, no record function
    assert lib.pmf_graph_capture(p, rec, None, None) == ops.PMF_EINVAL
    assert lib.pmf_graph_capture(None, rec, None, C.byref(out)) == ops.PMF_EINVAL
    assert "default stream" in err(lib)
    assert lib.pmf_graph_capture(p, None, None, C.byref(out)) == ops.PMF_EINVAL
    assert out.value is None
    assert lib.pmf_graph_replay(None, p) == ops.PMF_EINVAL
    assert lib.pmf_graph_kernel_count(None) == -1
    assert lib.pmf_graph_destroy(None) == ops.PMF_OK
    assert lib.pmf_fill(None, 4, 0.0, None) == ops.PMF_EINVAL
    assert lib.pmf_fill(p, -1, 0.0, None) == ops.PMF_EINVAL
    g = grid()
    cn = ops.make_cone(Cone(1000.0, 1500.0, 8, 8, 1.0, 1.0))
    big = 1 << 40
    hit = C.c_int(7)
    ms = (C.c_float * 18)()
    assert lib.pmf_autotune(b"/nonexistent/x", p, C.byref(g), C.byref(cn), p, 0, p, p, p, p, big,
                            1, ms, C.byref(hit), None) == ops.PMF_EINVAL
    assert lib.pmf_autotune(None, p, C.byref(g), C.byref(cn), p, 2, p, p, p, p, big, 0, ms,
                            C.byref(hit), None) == ops.PMF_EINVAL
    assert lib.pmf_autotune(None, None, C.byref(g), C.byref(cn), p, 2, p, p, p, p, big, 1, ms,
                            C.byref(hit), None) == ops.PMF_EINVAL
    assert lib.pmf_autotune(None, p, C.byref(g), C.byref(cn), p, 2, p, p, p, p, 0, 1, ms,
                            C.byref(hit), None) == ops.PMF_EWORKSPACE
    assert hit.value == 7          # rejected before anything was looked up
