"""Benchmark: fwd+bwd iterations/s of the PMF-STGR motion path on one MI355X.

Workload (synthetic, seeded): 32 random views of the 660-view scan, a
200,000-Gaussian reference volume at 256x256x128 (1.5x1.5x2 mm), MBC levels of
1k/4k/16k Gaussians on 64^3/128^3/256x256x128 grids with 3 bases x 3
components, a 512x384 detector at 0.776 mm, SAD/SDD 1000/1500 mm, 0.75 mm
ray step, float32.  One step = voxelize (reference + 3 MBC levels), combine +
warp + project all 32 views, L2 loss against synthetic target projections,
and the full adjoint down to every Gaussian parameter and coefficient.

``value`` is the batched schedule (fused motion path, all views per launch)
captured once into a HIP graph and replayed; the plain schedule (one view at
a time, issued from Python) is timed beside it.  Per-kernel GPU times come
from HIP events the library records on its launch stream during a profiled
pass of the same batched iteration; the FP64 oracle is timed on a bounded
sample on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import re
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector (published)
CU_COUNT = 256                 # MI355X compute units
CLOCK_GHZ = 2.4                # MI355X peak engine clock
# One trilinear ray-march sample costs about 33 VALU lane operations (ray
# point, cell index and fractions, eight taps, seven lerps, the accumulate);
# 22 of them are floating-point arithmetic (7 lerps x 3 + 1 accumulate).  Its
# transpose in the back-projection does the same work per sample.
OPS_PER_SAMPLE = 33
FLOP_PER_SAMPLE = 22
GATHER_BYTES_PER_SAMPLE = 32   # 8 taps x 4 B


def ray_samples(grid, cone, angles) -> np.ndarray:
    """Samples per ray of the midpoint rule (float64 geometry), [V][nv][nu]."""
    n = np.asarray(grid.n, np.float64)
    h = np.asarray(grid.h, np.float64)
    c0 = np.asarray(grid.center, np.float64) - 0.5 * (n - 1) * h
    lo, hi = c0 - 0.5 * h, c0 + (n - 0.5) * h
    step = cone.step if cone.step > 0 else 0.5 * h.min()
    a = (np.arange(cone.nu) - 0.5 * (cone.nu - 1) + cone.off_u) * cone.du
    b = (np.arange(cone.nv) - 0.5 * (cone.nv - 1) + cone.off_v) * cone.dv
    A, Bv = np.meshgrid(a, b)
    out = []
    for th in np.asarray(angles, np.float64):
        ct, st = math.cos(th), math.sin(th)
        o = np.array([cone.sad * ct, cone.sad * st, 0.0])
        p = np.stack([-(cone.sdd - cone.sad) * ct - A * st, -(cone.sdd - cone.sad) * st + A * ct, Bv], -1)
        d = p - o
        d /= np.linalg.norm(d, axis=-1, keepdims=True)
        with np.errstate(divide="ignore", invalid="ignore"):
            ta = (lo - o) / d
            tb = (hi - o) / d
        t0 = np.nanmax(np.minimum(ta, tb), axis=-1)
        t1 = np.nanmin(np.maximum(ta, tb), axis=-1)
        L = np.maximum(t1 - np.maximum(t0, 0.0), 0.0)
        out.append(np.where(L > 0, np.maximum(1, np.ceil(L / step)), 0))
    return np.stack(out)


PROFILE_COUNTERS = "profiles/motion_fwdbwd_32views_256x256x128_counters.md"


def profiled_counters(kernel: str):
    """Per-launch counters of `kernel` (a library kernel name) from the
    committed rocprofv3 counter summary: HBM bytes (FETCH_SIZE + WRITE_SIZE,
    calibrated by a plain copy), SQ_INSTS_VALU, SQ_WAVES, ... as a dict, or
    None if there is no such line or the kernel's source file changed since
    the counters were taken (sha256 prefix of the file)."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, PROFILE_COUNTERS)
    if not os.path.exists(path):
        return None
    best = None
    for line in open(path):
        line = line.strip()
        if not line.startswith("counters: "):
            continue
        kv = dict(f.split("=", 1) for f in line[len("counters: "):].split() if "=" in f)
        if kv.get("kernel") != kernel:
            continue
        if best is None or int(kv["grid"]) > int(best["grid"]):
            best = kv
    if best is None:
        return None
    src = os.path.join(root, best["source"])
    if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != best["sha256"]:
        return None
    out = {}
    for k, v in best.items():
        try:
            out[k] = float(v)
        except ValueError:
            out[k] = v
    return out


def alu_roofline(name, avg_ms, samples):
    """Roofline entry of a ray-march kernel (project or project_bwd): the
    33-op sample count against the FP32 vector peak, the 22-FLOP figure beside
    it, the VALU-issue fraction and lane slots per sample from the committed
    SQ_INSTS_VALU, the gather rate and the measured HBM traffic."""
    S = float(samples)
    t = avg_ms * 1e-3
    ops_ = OPS_PER_SAMPLE * S
    c = profiled_counters(name)
    out = {"kernel": name, "bound": "alu", "achieved": ops_ / t / 1e12, "peak": FP32_VECTOR_PEAK_TFLOPS,
           "unit": "TFLOP/s", "frac": ops_ / t / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
           "traffic": c["hbm_bytes"] if c else None, "avg_launch_ms": avg_ms,
           "samples_per_launch": S, "ops_per_sample": OPS_PER_SAMPLE,
           "flop22": {"flop_per_sample": FLOP_PER_SAMPLE, "achieved": FLOP_PER_SAMPLE * S / t / 1e12,
                      "frac": FLOP_PER_SAMPLE * S / t / 1e12 / FP32_VECTOR_PEAK_TFLOPS},
           "gather": {"bytes_per_launch": GATHER_BYTES_PER_SAMPLE * S,
                      "achieved": GATHER_BYTES_PER_SAMPLE * S / t / 1e9, "unit": "GB/s"},
           "valu_issue": None}
    if c and "valu_insts" in c:
        # a CU issues at most one wave64 VALU instruction per cycle (four
        # SIMDs, four cycles each)
        out["valu_issue"] = {"valu_insts_per_launch": c["valu_insts"],
                             "frac": c["valu_insts"] / (CU_COUNT * CLOCK_GHZ * 1e9 * t),
                             "lane_slots_per_sample": 64.0 * c["valu_insts"] / S}
        if c.get("dur_ns"):
            out["valu_issue"]["frac_profiled_duration"] = \
                c["valu_insts"] / (CU_COUNT * CLOCK_GHZ * c["dur_ns"])
    return out


def hbm_phase(byts, ms):
    return {"algorithmic_bytes": byts, "ms": ms, "achieved": byts / (ms * 1e-3) / 1e9, "unit": "GB/s",
            "peak": HBM_PEAK_GBS, "frac": byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


def hbm_phases(m, steps: int):
    """HBM fractions of the phases that are HBM-bound: the MBC
    voxelizations, the voxelization adjoints (reference + MBC) and the plain
    schedule's per-view combine + warp, each timed on its own, serially on
    one stream."""
    import torch
    from paper_2503_22139_amd import ops
    N = m.grid.size
    C_l = [int(g.value.shape[1]) for g in m.mbc]
    n_l = [lg.size for lg in m.levels]
    basis_bytes = 4.0 * sum(n * c for n, c in zip(n_l, C_l))
    par = lambda g: 4.0 * g.mean.numel() + 4.0 * g.scale.numel() + 4.0 * g.quat.numel() + 4.0 * g.value.numel()

    def vox_mbc():
        return [ops.pmf_voxelize(g.mean, g.scale, g.quat, g.value, lg, m.k) for g, lg in zip(m.mbc, m.levels)]
    ms4 = _timed(vox_mbc, steps)
    a4 = hbm_phase(basis_bytes + sum(par(g) for g in m.mbc), ms4)
    ref, bases = m.volumes()
    g_ref = torch.ones(N, device="cuda") * 1e-3
    g_b = [torch.full_like(b, 1e-3) for b in bases]

    def vox_bwd():
        ops.pmf_voxelize_bwd(m.ref.mean, m.ref.scale, m.ref.quat, m.ref.value, m.grid, m.k, g_ref.reshape(1, -1))
        for g, lg, gb in zip(m.mbc, m.levels, g_b):
            ops.pmf_voxelize_bwd(g.mean, g.scale, g.quat, g.value, lg, m.k, gb)
    ms12 = _timed(vox_bwd, steps)
    a12 = hbm_phase(4.0 * N + basis_bytes + 2 * (par(m.ref) + sum(par(g) for g in m.mbc)), ms12)

    def plain_cw():
        for v in range(m.V):
            dvf = ops.pmf_combine_dvf(bases, m.levels, m.coeff[v:v + 1], m.grid)
            ops.pmf_warp(ref, m.grid, dvf)
    msp = _timed(plain_cw, max(2, steps // 2))
    # per view: every basis read, I_ref read, the DVF written and read back,
    # the warped volume written
    pcw = hbm_phase(m.V * (basis_bytes + 4.0 * N + 2 * 12.0 * N + 4.0 * N), msp)
    return {"a4_voxelize_mbc": a4, "a12_voxelize_bwd": a12, "plain_combine_warp": pcw}


def _timed(fn, steps: int, warmup: int = 1) -> float:
    """Mean wall milliseconds of fn() over `steps` calls after `warmup` calls,
    with the device synchronised around the timed region."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def _drain_profile():
    """Clear every kernel's recorded launch times before a profiled pass."""
    from paper_2503_22139_amd import ops
    for k in ops.pmf_profile_names():
        ops.pmf_profile_read(k)


def extras(steps: int):
    """The other configurations (forward-only C1-C3, the 16-view
    differentiable C4, the ragged three-scan C5 and B = 1 of the benchmark
    workload), each timed on its own after the headline run."""
    import torch
    from paper_2503_22139_amd import ops, synth
    from paper_2503_22139_amd.model import GraphStep, MotionModel, MultiScanModel
    out = {}

    def fwd_only(w):
        ref = T(w)
        ang = torch.from_numpy(np.ascontiguousarray(w.angles, np.float32)).cuda()

        def run():
            vol = ops.pmf_voxelize(ref[0], ref[1], ref[2], ref[3], w.grid, float(w.trunc_k))
            return ops.pmf_project(vol, w.grid, w.cone, ang)
        return run

    def T(w):
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
        return f(w.ref.mean), f(w.ref.scale), f(w.ref.quat), f(w.ref.value)

    for name, w in (("c1_forward", synth.c1()), ("c2_forward", synth.c2())):
        ms = _timed(fwd_only(w), steps)
        out[name] = {"ms": ms, "views": len(w.angles), "grid": list(w.grid.n), "gaussians": w.ref.m,
                     "what": "voxelize + project"}
        print(f"[bench] {name} {ms:.2f} ms", file=sys.stderr, flush=True)
    w3 = synth.c3()
    m3 = MotionModel(w3)
    ms = _timed(m3.forward_batched, steps)
    out["c3_forward"] = {"ms": ms, "views": len(w3.angles), "what": "voxelize + batched motion path"}
    print(f"[bench] c3_forward {ms:.2f} ms", file=sys.stderr, flush=True)
    tgt = torch.from_numpy(synth.add_target_noise(
        MotionModel(synth.perturbed_truth(w3)).forward_batched().cpu().numpy())).cuda()
    gs = GraphStep(m3, tgt)
    ms = _timed(gs.step, steps)
    out["c4_step"] = {"ms": ms, "iterations_per_s": 1e3 / ms, "views": len(w3.angles),
                      "what": "fwd+bwd, batched, graph replay"}
    print(f"[bench] c4_step {ms:.2f} ms", file=sys.stderr, flush=True)
    del gs, m3, tgt
    torch.cuda.empty_cache()
    ws5 = synth.c5_scans()
    mm = MultiScanModel(ws5)
    tg5 = [torch.from_numpy(synth.random_volume(90 + k, (len(w.angles), w.cone.nv, w.cone.nu),
                                                0.0, 20.0)).cuda() for k, w in enumerate(ws5)]
    gs = GraphStep(mm, tg5)
    ms = _timed(gs.step, steps)
    ms_sep = _timed(lambda: mm.step_separate(tg5), steps)
    out["c5_step"] = {"ms": ms, "iterations_per_s": 1e3 / ms, "separate_eager_ms": ms_sep,
                      "scans": [{"grid": list(w.grid.n), "gaussians": w.ref.m, "views": len(w.angles)}
                                for w in ws5],
                      "what": "3 ragged scans x 32 views, fwd+bwd, one launch per stage, graph replay"}
    print(f"[bench] c5_step {ms:.2f} ms (separate eager {ms_sep:.2f})", file=sys.stderr, flush=True)
    del gs, mm, tg5
    torch.cuda.empty_cache()
    # the benchmark workload with the Stage 2/3 objective of Eq. 14 (L1 +
    # 0.25 D-SSIM, 0.05 TV of a 32^3 block, MBC normality): eager with a new
    # random block each step, and graph-captured with one block
    wp = synth.headline()
    mp = MotionModel(wp)
    tp = torch.from_numpy(synth.add_target_noise(
        MotionModel(synth.perturbed_truth(wp)).forward_batched().cpu().numpy())).cuda()
    rng = np.random.default_rng(97)
    corners = [tuple(int(rng.integers(0, n - 32 + 1)) for n in wp.grid.n) for _ in range(steps + 8)]
    it = iter(corners)
    ms_e = _timed(lambda: mp.step_batched_paper(tp, next(it)), steps)
    gs = GraphStep(mp, tp, step=lambda t: mp.step_batched_paper(t, corners[0]))
    ms_g = _timed(gs.step, steps)
    _drain_profile()
    ops.pmf_profile(True)
    mp.step_batched_paper(tp, corners[1])
    torch.cuda.synchronize()
    ops.pmf_profile(False)
    kern = {}
    for k in ("ssim_fwd", "ssim_final", "ssim_bwd", "tv", "normality"):
        tot, cnt = ops.pmf_profile_read(k)
        kern[k] = tot
    out["paper_objective_step"] = {
        "ms": ms_g, "iterations_per_s": 1e3 / ms_g, "eager_ms": ms_e, "loss_kernels_ms": kern,
        "what": "benchmark workload with the Eq. 14 objective: L1 + 0.25 D-SSIM over the 32 views, "
                "0.05 TV of a random 32^3 block of I_ref, MBC normality; graph replay (eager: a new "
                "block each step)"}
    print(f"[bench] paper_objective_step {ms_g:.2f} ms (eager {ms_e:.2f}; loss kernels {kern})",
          file=sys.stderr, flush=True)
    del gs, mp, tp
    torch.cuda.empty_cache()
    # Stage 1 (Eq. 10-11): the 200k reference Gaussians rasterized at one
    # random view of the 660-view scan per iteration, L1 + 0.25 D-SSIM, and
    # 0.05 TV of a random 32^3 sub-volume voxelized from the same Gaussians
    from paper_2503_22139_amd.model import Stage1Model
    w2 = synth.c2()
    s1 = Stage1Model(w2)
    rng1 = np.random.default_rng(98)
    views = synth.scan_angle(rng1.integers(0, 660, steps + 8))
    tgt1 = ops.pmf_rasterize(s1.ref.mean, s1.ref.scale, s1.ref.quat, s1.ref.value * 1.05,
                             w2.cone, torch.from_numpy(np.asarray(views[:1], np.float32)).cuda())
    cs = [tuple(int(rng1.integers(0, n - 32 + 1)) for n in w2.grid.n) for _ in range(steps + 8)]
    angs = [torch.from_numpy(np.asarray([a], np.float32)).cuda() for a in views]
    it1 = iter(range(steps + 8))

    def stage1():
        i = next(it1)
        return s1.step(tgt1, angs[i], cs[i])
    ms1 = _timed(stage1, steps)
    gs1 = GraphStep(s1, tgt1, step=lambda t: s1.step(t, angs[0], cs[0]))
    ms1_g = _timed(gs1.step, steps)
    del gs1
    _drain_profile()
    ops.pmf_profile(True)
    s1.step(tgt1, angs[0], cs[0])
    torch.cuda.synchronize()
    ops.pmf_profile(False)
    k1 = {}
    for k in ("rasterize_bin", "rasterize", "rasterize_bwd", "ssim_fwd", "ssim_bwd", "tv",
              "voxelize_tile", "voxelize_bwd"):
        tot, cnt = ops.pmf_profile_read(k)
        k1[k] = tot
    out["stage1_step"] = {
        "ms": ms1, "iterations_per_s": 1e3 / ms1, "graph_ms": ms1_g, "gaussians": w2.ref.m,
        "kernels_ms": k1,
        "what": "Stage 1 iteration: rasterizer (Eq. 9) fwd+bwd at one random view, L1 + 0.25 "
                "D-SSIM, 0.05 TV of a random 32^3 sub-volume voxelized from the Gaussians; eager "
                "(graph_ms: replayed from a HIP graph with one view and block)"}
    print(f"[bench] stage1_step {ms1:.2f} ms (graph, one view and block: {ms1_g:.2f}; kernels {k1})",
          file=sys.stderr, flush=True)
    del s1, tgt1
    torch.cuda.empty_cache()
    # FDK initialisation (Sec. 2.3.2): the full 660-view scan of the 512 x 384
    # detector (ray-marched from the voxelized reference) reconstructed onto
    # the 256 x 256 x 128 grid
    rf = T(w2)
    vol2 = ops.pmf_voxelize(rf[0], rf[1], rf[2], rf[3], w2.grid, float(w2.trunc_k))
    ang_all = torch.from_numpy(synth.scan_angle(np.arange(660))).cuda()
    proj_all = ops.pmf_project(vol2, w2.grid, w2.cone, ang_all)
    del vol2, rf
    fvol = torch.empty(tuple(w2.grid.n), device="cuda")
    ms_f = _timed(lambda: ops.pmf_fdk(proj_all, w2.cone, ang_all, w2.grid, out=fvol), steps)
    _drain_profile()
    ops.pmf_profile(True)
    ops.pmf_fdk(proj_all, w2.cone, ang_all, w2.grid, out=fvol)
    torch.cuda.synchronize()
    ops.pmf_profile(False)
    kf = {k: ops.pmf_profile_read(k)[0] for k in ("fdk_filter", "fdk_backproject")}
    updates = float(np.prod(w2.grid.n)) * 660
    m_i, delta = ops.grid_init_lattice(w2.grid, 50_000)
    ms_i = _timed(lambda: ops.pmf_grid_init(fvol, w2.grid, m_i, delta / math.sqrt(2 * math.pi)),
                  steps)
    out["fdk_init"] = {
        "ms": ms_f, "kernels_ms": kf, "views": 660, "detector": [w2.cone.nv, w2.cone.nu],
        "grid": list(w2.grid.n),
        "voxel_view_updates_per_s": updates / (kf["fdk_backproject"] * 1e-3),
        "grid_init_ms": ms_i, "grid_init_points": int(np.prod(m_i)),
        "what": "FDK of the 660-view scan (cosine weight, Ram-Lak row filter, voxel-driven "
                "back-projection), then the grid-sampled initial Gaussians (M = 50,000); eager"}
    print(f"[bench] fdk_init {ms_f:.2f} ms (kernels {kf}); grid_init {ms_i:.3f} ms",
          file=sys.stderr, flush=True)
    del proj_all, fvol, ang_all
    torch.cuda.empty_cache()
    wb = synth.headline(nbases=1)
    mb = MotionModel(wb)
    tb = torch.from_numpy(synth.random_volume(95, (len(wb.angles), wb.cone.nv, wb.cone.nu),
                                              0.0, 20.0)).cuda()
    gs = GraphStep(mb, tb)
    ms = _timed(gs.step, steps)
    out["b1_step"] = {"ms": ms, "iterations_per_s": 1e3 / ms,
                      "what": "benchmark workload with B = 1 (9 coefficients per view)"}
    print(f"[bench] b1_step {ms:.2f} ms", file=sys.stderr, flush=True)
    del gs, mb, tb
    torch.cuda.empty_cache()
    # large motion: the benchmark workload with the MBC values scaled up, so
    # that many displacements leave the warp adjoint's 3-voxel LDS halo (its
    # overflow goes to a 64-bit fixed-point volume)
    lm = {}
    for scale in (1.0, 4.0):
        wl = synth.headline()
        for st in wl.mbc:
            st.value = (st.value * np.float32(scale)).astype(np.float32)
        ml = MotionModel(wl)
        ref, bases = ml.volumes()
        dvf = ops.pmf_combine_dvf(bases, ml.levels, ml.coeff[:1], ml.grid).reshape(3, -1)
        h = torch.tensor(wl.grid.h, device="cuda", dtype=torch.float32).reshape(3, 1)
        vox = (dvf.abs() / h).amax(0)
        tl = torch.from_numpy(synth.random_volume(96, (len(wl.angles), wl.cone.nv, wl.cone.nu),
                                                  0.0, 20.0)).cuda()
        gl = GraphStep(ml, tl)
        ms = _timed(gl.step, steps)
        lm[f"x{scale:g}"] = {"ms": ms, "max_disp_mm": float(dvf.abs().max()),
                             "frac_voxels_beyond_halo_view0": float((vox > 3.0).float().mean())}
        del gl, ml, tl, ref, bases, dvf
        torch.cuda.empty_cache()
    out["large_motion_step"] = dict(lm, what="benchmark workload with MBC values x1 and x4; "
                                    "displacement statistics of view 0")
    print(f"[bench] large_motion_step {lm}", file=sys.stderr, flush=True)
    return out


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, target, views: int = 2):
    """FP64 oracle on a bounded sample, on every core the process may use:
    the benchmark iteration (volumes, `views` views' fwd+bwd and the
    voxelization adjoints, extrapolated linearly to all views), the C1 and C2
    forward passes in full, the C3 forward on a few of its views
    (extrapolated), and C1 forward again on one core."""
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import oracle
    from paper_2503_22139_amd import synth
    oracle.build()
    cores = len(os.sched_getaffinity(0))
    oracle.set_threads(cores)
    cores = oracle.get_threads()
    t0 = time.perf_counter()
    ref, bases = oracle.forward_volumes(w)
    t_vol = time.perf_counter() - t0
    N = w.grid.size
    g_ref = np.zeros(N)
    g_bases = [np.zeros_like(b) for b in bases]
    t1 = time.perf_counter()
    for v in range(views):
        cv = w.coeff[v:v + 1]
        dvf = oracle.combine(bases, w.levels, cv, w.grid)
        wv = oracle.warp(ref, w.grid, dvf)
        p = oracle.project(wv, w.grid, w.cone, w.angles[v:v + 1])
        _, gp = oracle.l2_loss(p, target[v:v + 1])
        gp *= 1.0 / len(w.angles)
        gw = oracle.project_bwd(gp, w.grid, w.cone, w.angles[v:v + 1])
        gr, gd = oracle.warp_bwd(ref, w.grid, dvf, gw)
        g_ref += gr.reshape(-1)
        gb, _ = oracle.combine_bwd(bases, w.levels, cv, w.grid, gd)
        for a, b in zip(g_bases, gb):
            a += b
    t_view = (time.perf_counter() - t1) / views
    t2 = time.perf_counter()
    oracle.voxelize_bwd(w.ref, w.grid, w.trunc_k, g_ref.reshape(1, -1))
    for s, g, gb in zip(w.mbc, w.levels, g_bases):
        oracle.voxelize_bwd(s, g, w.trunc_k, gb)
    t_vb = time.perf_counter() - t2
    t_iter = t_vol + len(w.angles) * t_view + t_vb
    print(f"[bench] cpu baseline: iteration {t_iter:.1f} s (extrapolated)", file=sys.stderr, flush=True)

    def fwd_proj(wk):
        vol = oracle.voxelize(wk.ref, wk.grid, wk.trunc_k)[0]
        return oracle.project(vol, wk.grid, wk.cone, wk.angles)

    c1 = synth.c1()
    t = time.perf_counter()
    fwd_proj(c1)
    t_c1 = time.perf_counter() - t
    c2 = synth.c2()
    t = time.perf_counter()
    fwd_proj(c2)
    t_c2 = time.perf_counter() - t
    c3 = synth.c3()
    n3 = 2
    t = time.perf_counter()
    oracle.forward(c3, views=list(range(n3)))
    t_c3s = time.perf_counter() - t
    t = time.perf_counter()
    oracle.forward_volumes(c3)
    t_c3v = time.perf_counter() - t
    t_c3 = t_c3v + (t_c3s - t_c3v) * len(c3.angles) / n3
    oracle.set_threads(1)
    t = time.perf_counter()
    fwd_proj(c1)
    t_c1_1 = time.perf_counter() - t
    oracle.set_threads(cores)
    print(f"[bench] cpu baseline: c1 {t_c1:.2f} s, c2 {t_c2:.2f} s, c3 {t_c3:.2f} s, c1 on one core "
          f"{t_c1_1:.2f} s", file=sys.stderr, flush=True)
    return {"value": 1.0 / t_iter, "unit": "iterations/s", "cores": cores, "kind": "oracle",
            "cpu_model": _cpu_model(),
            "sample": (f"FP64 oracle: volumes ({t_vol:.2f} s) + {views} of {len(w.angles)} views "
                       f"fwd+bwd ({t_view:.2f} s/view) + voxelization adjoints ({t_vb:.2f} s), "
                       f"extrapolated linearly to {len(w.angles)} views = {t_iter:.1f} s/iteration"),
            "c1_forward_s": t_c1, "c2_forward_s": t_c2,
            "c3_forward_s": t_c3,
            "c3_sample": (f"volumes {t_c3v:.2f} s + {n3} of {len(c3.angles)} views, extrapolated "
                          f"linearly"),
            "c1_forward_1core_s": t_c1_1}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--views", type=int, default=32)
    ap.add_argument("--bases", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the other configurations")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--tune-cache", default=os.path.join("/tmp", f"pmf_tune_{os.getuid()}.txt"),
                    help="the autotuner's shape cache ('' for none)")
    ap.add_argument("--no-graph", action="store_true",
                    help="time the eager batched steps instead of graph replays (for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(views would shard across GPUs with one all-reduce of the parameter "
              "gradients; not implemented). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2503_22139_amd import ops, synth
    from paper_2503_22139_amd.model import GraphStep, MotionModel

    torch.cuda.init()
    # A plain device copy of known size (256 MiB read, 256 MiB written): under
    # rocprofv3 --pmc its FETCH_SIZE / WRITE_SIZE calibrate the HBM counters.
    src = torch.ones(64 << 20, device="cuda")
    torch.empty_like(src).copy_(src)
    torch.cuda.synchronize()
    del src
    w = synth.headline(nviews=args.views, nbases=args.bases)
    m = MotionModel(w)
    truth = MotionModel(synth.perturbed_truth(w))
    target_np = synth.add_target_noise(truth.forward_batched().cpu().numpy())
    del truth
    target = torch.from_numpy(target_np).cuda()
    V = len(w.angles)

    tuned = None
    if not args.no_autotune:
        # launch shapes for this geometry, timed on per-view volumes of its size
        vol = torch.from_numpy(synth.random_volume(7, (V,) + tuple(w.grid.n))).cuda()
        gp = torch.from_numpy(synth.random_normal(8, (V, w.cone.nv, w.cone.nu))).cuda()
        tuned = ops.pmf_autotune(args.tune_cache or None, vol, w.grid, w.cone, m.angles, gp, reps=2)
        del vol, gp
        torch.cuda.empty_cache()
        print(f"[bench] autotune {tuned}", file=sys.stderr, flush=True)

    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        m.step_batched(target)
    torch.cuda.synchronize()
    for name in ops.pmf_profile_names():
        ops.pmf_profile_read(name)

    # eager batched steps with per-kernel HIP events on the launch stream
    _drain_profile()
    ops.pmf_profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        m.step_batched(target)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ops.pmf_profile(False)
    ms_eager = (t1 - t0) / args.steps * 1e3
    kern = {}
    for name in ops.pmf_profile_names():
        tot, cnt = ops.pmf_profile_read(name)
        kern[name] = {"ms_per_step": tot / args.steps, "launches_per_step": cnt / args.steps,
                      "avg_ms": tot / max(cnt, 1)}
    print(f"[bench] batched eager {ms_eager:.2f} ms/step", file=sys.stderr, flush=True)

    # the timed region: the batched iteration replayed from a HIP graph
    if args.no_graph:
        ms = ms_eager
        loss, grads = m.step_batched(target)
    else:
        gs = GraphStep(m, target)
        for _ in range(2):
            gs.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            loss, grads = gs.step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms = (t1 - t0) / args.steps * 1e3
        print(f"[bench] batched graph {ms:.2f} ms/step", file=sys.stderr, flush=True)

    # plain schedule (one view at a time)
    ms_plain = float("nan")
    if args.plain_steps > 0:
        m.step_plain(target)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            m.step_plain(target)
        torch.cuda.synchronize()
        ms_plain = (time.perf_counter() - t0) / args.plain_steps * 1e3
        print(f"[bench] plain {ms_plain:.2f} ms/step", file=sys.stderr, flush=True)

    samples = float(ray_samples(w.grid, w.cone, w.angles).sum())
    # the dominant kernel of the step and the forward projection beside it
    march = [k for k in ("project_bwd", "project") if k in kern]
    dom = max(march, key=lambda k: kern[k]["ms_per_step"])
    roof = alu_roofline(dom, kern[dom]["avg_ms"], samples)
    N = w.grid.size
    byts = 4.0 * (V * N + V * w.cone.nu * w.cone.nv)
    roof["hbm"] = {"algorithmic_bytes": byts, "achieved": byts / (kern[dom]["avg_ms"] * 1e-3) / 1e9,
                   "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": byts / (kern[dom]["avg_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
    others = {k: alu_roofline(k, kern[k]["avg_ms"], samples) for k in march if k != dom}
    print(f"[bench] hbm phases", file=sys.stderr, flush=True)
    phases = hbm_phases(m, max(3, min(args.steps, 10)))

    out = {
        "metric": "fwd+bwd iterations/s (32 views, 256²×128) batched vs plain; % HBM roofline",
        "value": 1e3 / ms,
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"motion path fwd+bwd, {V} random views of 660, reference 200k Gaussians "
                                f"@256x256x128 (1.5x1.5x2 mm), MBC 1k/4k/16k @64^3/128^3/256x256x128, "
                                f"B={args.bases}, detector 512x384 @0.776 mm, SAD/SDD 1000/1500, step 0.75 mm"),
                   "views": V, "grid": list(w.grid.n), "detector": [w.cone.nu, w.cone.nv],
                   "schedule": "batched, " + ("eager" if args.no_graph else "replayed from a HIP graph")},
        "batched_eager_ms_per_step": ms_eager,
        "plain": ({"value": 1e3 / ms_plain, "ms_per_step": ms_plain, "steps": args.plain_steps}
                  if args.plain_steps > 0 else None),
        "speedup_vs_plain": ms_plain / ms if args.plain_steps > 0 else None,
        "loss": float(loss),
        "kernels": kern,
        "roofline": roof,
        "roofline_other": others,
        "hbm_phases": phases,
    }
    out["tuned"] = tuned
    if not args.no_extras:
        out["extras"] = extras(max(2, min(args.steps, 5)))
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, target_np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
