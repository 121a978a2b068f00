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
FLOP_PER_SAMPLE = 22           # trilinear sample: 7 lerps x 3 flops + 1 accumulate


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


def profiled_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated by a plain copy), or None if
    there is none or the kernel's source file changed since it was taken."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, PROFILE_COUNTERS)
    if not os.path.exists(path):
        return None
    best = None
    for line in open(path):
        m = re.match(r"traffic: kernel=(\S+) grid=(\d+) source=(\S+) sha256=(\S+) hbm_bytes=(\S+)", line.strip())
        if not m or m.group(1) != kernel:
            continue
        if best is None or int(m.group(2)) > best[0]:
            best = (int(m.group(2)), m.group(3), m.group(4), float(m.group(5)))
    if best is None:
        return None
    src = os.path.join(root, best[1])
    if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != best[2]:
        return None
    return best[3]


def kernel_model(name, w, V, samples):
    """Algorithmic work of one launch of a kernel in the batched step:
    (bound, achieved-unit quantity, hbm bytes)."""
    N = w.grid.size
    npix = w.cone.nu * w.cone.nv
    if name in ("project", "project_bwd"):
        flops = FLOP_PER_SAMPLE * float(samples.sum())
        byts = 4.0 * (V * N + V * npix)
        return "alu", flops, byts
    return None


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
    del gs, mb
    torch.cuda.empty_cache()
    return out


def cpu_baseline(w, target, views: int = 2):
    """FP64 oracle on a bounded sample: the volumes, `views` views' fwd+bwd and
    the voxelization adjoints; extrapolated linearly to all views."""
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import oracle
    oracle.build()
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
    return {"value": 1.0 / t_iter, "unit": "iterations/s", "cores": cores, "kind": "oracle",
            "sample": (f"FP64 oracle: volumes ({t_vol:.2f} s) + {views} of {len(w.angles)} views "
                       f"fwd+bwd ({t_view:.2f} s/view) + voxelization adjoints ({t_vb:.2f} s), "
                       f"extrapolated linearly to {len(w.angles)} views = {t_iter:.1f} s/iteration")}


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
        tuned = ops.pmf_autotune_project(vol, w.grid, w.cone, m.angles, gp, reps=2)
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

    samples = ray_samples(w.grid, w.cone, w.angles)
    dom = max((k for k in kern if kernel_model(k, w, V, samples)), key=lambda k: kern[k]["ms_per_step"])
    bound, flops, byts = kernel_model(dom, w, V, samples)
    avg_s = kern[dom]["avg_ms"] * 1e-3
    achieved = flops / avg_s / 1e12
    traffic = profiled_traffic(dom)
    roof = {"kernel": dom, "bound": bound, "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic,
            "avg_launch_ms": kern[dom]["avg_ms"], "algorithmic_flop": flops,
            "hbm": {"achieved": byts / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": byts / avg_s / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes": byts,
                    "measured_traffic_GBps": (traffic / avg_s / 1e9) if traffic else None}}

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
