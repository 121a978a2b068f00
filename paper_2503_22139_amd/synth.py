"""Seeded synthetic inputs for the forward model (no forward-model arithmetic).

This module only draws inputs: Gaussian parameter sets, grids, cone-beam
geometries, view angles and temporal coefficients.  It is shared by the HIP
path, the FP64 oracle and the benchmark, and holds none of the arithmetic of
the method itself (no voxelization, interpolation, warping or projection).

Every array is produced in float64 by numpy's PCG64 ``default_rng`` and then
rounded to float32, so the GPU (float32) and the oracle (float32 promoted to
float64) see bit-identical inputs.

Workload shapes follow the paper's XCAT simulation and patient geometry:
a 360-degree scan of 660 projections at 11 frames/s (Sec. 2.3.3), the Varian
full-fan detector of 512x384 pixels at 0.776 mm with SAD/SDD 1000/1500 mm
(Table I), breathing periods of 3-5 s (Sec. 1), three MBC levels (Sec. 2.3.1)
and reference sets of 10^4-10^5 Gaussians (Sec. 2.3.3).  The phantom, motion
curves and patient data themselves are not available; these generators stand
in for them with seeded random inputs of the same shapes.

Draw order inside ``gaussians`` (fixed): means, scales, quaternions, values.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

F32 = np.float32


@dataclasses.dataclass
class Grid:
    """Voxel grid: ``n`` voxels per axis, spacing ``h`` (mm), centre (mm).

    Voxel (i, j, k) sits at ``center + ((i, j, k) - (n - 1) / 2) * h``;
    memory order is ``[n0][n1][n2]`` with axis 2 fastest.
    """

    n: Tuple[int, int, int]
    h: Tuple[float, float, float]
    center: Tuple[float, float, float] = (0.0, 0.0, 0.0)

    @property
    def size(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    def box(self) -> Tuple[np.ndarray, np.ndarray]:
        """Physical extent [lo, hi] of the grid (voxel faces, mm)."""
        n = np.asarray(self.n, np.float64)
        h = np.asarray(self.h, np.float64)
        c = np.asarray(self.center, np.float64)
        return c - 0.5 * n * h, c + 0.5 * n * h

    def fov(self) -> np.ndarray:
        return np.asarray(self.n, np.float64) * np.asarray(self.h, np.float64)


@dataclasses.dataclass
class Cone:
    """Flat-panel cone-beam geometry (mm); ``step`` 0 means half the smallest voxel."""

    sad: float
    sdd: float
    nu: int
    nv: int
    du: float
    dv: float
    off_u: float = 0.0
    off_v: float = 0.0
    step: float = 0.0


@dataclasses.dataclass
class GaussSet:
    """Structure-of-arrays Gaussian set, float32.

    mean [m,3] mm, scale [m,3] mm (standard deviations, post-activation),
    quat [m,4] (w, x, y, z), value [m,c] (density, or signed MBC values).
    """

    mean: np.ndarray
    scale: np.ndarray
    quat: np.ndarray
    value: np.ndarray

    @property
    def m(self) -> int:
        return int(self.mean.shape[0])

    @property
    def c(self) -> int:
        return int(self.value.shape[1])

    def copy(self) -> "GaussSet":
        return GaussSet(self.mean.copy(), self.scale.copy(), self.quat.copy(), self.value.copy())


@dataclasses.dataclass
class Workload:
    """One complete input of the forward model."""

    name: str
    grid: Grid
    cone: Cone
    ref: GaussSet
    angles: np.ndarray                      # [V] rad, float32
    trunc_k: float = 3.0
    levels: List[Grid] = dataclasses.field(default_factory=list)
    mbc: List[GaussSet] = dataclasses.field(default_factory=list)
    coeff: Optional[np.ndarray] = None      # [V][L][B][3] float32
    nbases: int = 0
    view_index: Optional[np.ndarray] = None  # index into the 660-view scan


# ---------------------------------------------------------------- primitives

def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, np.float64).astype(F32))


def evenly_spaced_angles(nviews: int) -> np.ndarray:
    """theta_k = 2 pi k / n, k = 0..n-1."""
    return _f32(2.0 * math.pi * np.arange(nviews) / nviews)


SCAN_VIEWS = 660       # projections in the simulated 360-degree scan
SCAN_FPS = 11.0        # frames per second of that scan


def scan_angle(k) -> np.ndarray:
    return _f32(2.0 * math.pi * np.asarray(k, np.float64) / SCAN_VIEWS)


def scan_time(k) -> np.ndarray:
    return np.asarray(k, np.float64) / SCAN_FPS


def _uniform_in_box(rng, lo, hi, m) -> np.ndarray:
    return lo + (hi - lo) * rng.random((m, 3))


def _uniform_in_ellipsoid(rng, semi, m) -> np.ndarray:
    out = np.empty((0, 3))
    while out.shape[0] < m:
        p = (2.0 * rng.random((2 * m + 16, 3)) - 1.0) * semi
        r = np.sum((p / semi) ** 2, axis=1)
        out = np.concatenate([out, p[r <= 1.0]], axis=0)
    return out[:m]


def random_quaternions(rng, m) -> np.ndarray:
    q = rng.standard_normal((m, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def gaussians(rng, m: int, grid: Grid, *, s_vox=(0.5, 2.0), rho=(0.0, 0.05),
              c: int = 1, value_sigma: Optional[float] = None,
              body_frac: float = 0.0, body_semi=None) -> GaussSet:
    """Draw ``m`` anisotropic Gaussians inside ``grid``'s box.

    Means: ``body_frac`` of them uniform in a centred ellipsoid with semi-axes
    ``body_semi`` (mm), the rest uniform in the box.  Scales: per-axis
    log-uniform in ``s_vox`` voxels of the grid's smallest spacing.  Rotations:
    uniform random unit quaternions.  Values: U[rho] (c = 1 densities) or
    N(0, value_sigma) (signed, c channels).
    """
    lo, hi = grid.box()
    nb = int(round(body_frac * m))
    parts = []
    if nb:
        parts.append(_uniform_in_ellipsoid(rng, np.asarray(body_semi, np.float64), nb)
                     + np.asarray(grid.center, np.float64))
    parts.append(_uniform_in_box(rng, lo, hi, m - nb))
    mean = np.concatenate(parts, axis=0) if m else np.zeros((0, 3))
    hmin = float(min(grid.h))
    ls = rng.uniform(math.log(s_vox[0]), math.log(s_vox[1]), (m, 3))
    scale = np.exp(ls) * hmin
    quat = random_quaternions(rng, m) if m else np.zeros((0, 4))
    if value_sigma is None:
        value = rng.uniform(rho[0], rho[1], (m, c))
    else:
        value = rng.normal(0.0, value_sigma, (m, c))
    return GaussSet(_f32(mean), _f32(scale), _f32(quat), _f32(value))


def sinusoid_coefficients(rng, times: np.ndarray, nlevels: int, nbases: int,
                          period=(3.0, 5.0), jitter=0.1) -> np.ndarray:
    """w[v,l,b,k] = sin(2 pi t_v / T_lbk + phi_lbk) + jitter * xi.

    Breathing-like temporal coefficients: T ~ U[3,5] s, phi ~ U[0, 2 pi),
    xi ~ N(0,1) per entry.  Returns float32 [V][L][B][3].
    """
    shape = (nlevels, nbases, 3)
    T = rng.uniform(period[0], period[1], shape)
    phi = rng.uniform(0.0, 2.0 * math.pi, shape)
    t = np.asarray(times, np.float64).reshape(-1, 1, 1, 1)
    w = np.sin(2.0 * math.pi * t / T + phi) + jitter * rng.standard_normal((t.shape[0],) + shape)
    return _f32(w)


# ------------------------------------------------------------------ workloads

VARIAN = dict(sad=1000.0, sdd=1500.0, nu=512, nv=384, du=0.776, dv=0.776)
REF_GRID = Grid((256, 256, 128), (1.5, 1.5, 2.0))


def level_grids(grid: Grid, dims: Sequence[Sequence[int]]) -> List[Grid]:
    """MBC level grids covering the reference field of view (spacing = FOV / n)."""
    fov = grid.fov()
    return [Grid(tuple(int(v) for v in d), tuple(float(f) for f in fov / np.asarray(d, np.float64)),
                 grid.center) for d in dims]


def c1(seed: int = 0) -> Workload:
    """Projection-only case: 4,096 Gaussians in a 64^3 grid of 1 mm voxels,
    10 views evenly over 360 degrees, 128x96 detector at 2 mm, step 0.5 voxel."""
    rng = np.random.default_rng(seed)
    grid = Grid((64, 64, 64), (1.0, 1.0, 1.0))
    ref = gaussians(rng, 4096, grid, rho=(0.0, 0.05))
    cone = Cone(1000.0, 1500.0, 128, 96, 2.0, 2.0, step=0.5)
    return Workload("c1", grid, cone, ref, evenly_spaced_angles(10))


def body_semi_axes(grid: Grid) -> np.ndarray:
    """Ellipsoidal torso mask: semi-axes (0.42, 0.30, 0.45) of the FOV."""
    return grid.fov() * np.array([0.42, 0.30, 0.45])


def reference_set(rng, m: int, grid: Grid, rho=(0.0, 0.03)) -> GaussSet:
    return gaussians(rng, m, grid, rho=rho, body_frac=0.7, body_semi=body_semi_axes(grid))


def c2(seed: int = 1, m: int = 200_000, nviews: int = 8) -> Workload:
    """Reference-volume scale: 200k Gaussians (70% in a body ellipsoid) in
    256x256x128 at 1.5x1.5x2 mm, 8 views on the 512x384 detector."""
    rng = np.random.default_rng(seed)
    grid = REF_GRID
    ref = reference_set(rng, m, grid)
    cone = Cone(**VARIAN, step=0.75)
    return Workload("c2", grid, cone, ref, evenly_spaced_angles(nviews))


MBC_COUNTS = (1000, 4000, 16000)
NBASES = 3


def mbc_sets(rng, levels: Sequence[Grid], counts: Sequence[int], nbases: int,
             value_sigma: float = 2.0) -> List[GaussSet]:
    return [gaussians(rng, int(m), g, c=3 * nbases, value_sigma=value_sigma)
            for g, m in zip(levels, counts)]


def c3(seed: int = 2, nviews: int = 16, nbases: int = NBASES, ref_seed: int = 1,
       view_index: Optional[np.ndarray] = None) -> Workload:
    """Motion path: the 200k-Gaussian reference plus three MBC levels
    (1k/4k/16k Gaussians on 64^3, 128^3 and 256x256x128 grids), each carrying
    ``nbases`` bases x 3 displacement components with values N(0, 2 mm);
    views k_v = floor(v * 660 / nviews) of the 660-view scan."""
    base = c2(ref_seed)
    rng = np.random.default_rng(seed)
    levels = level_grids(base.grid, [(64, 64, 64), (128, 128, 128), (256, 256, 128)])
    mbc = mbc_sets(rng, levels, MBC_COUNTS, nbases)
    if view_index is None:
        view_index = (np.arange(nviews) * SCAN_VIEWS) // nviews
    coeff = sinusoid_coefficients(rng, scan_time(view_index), len(levels), nbases)
    return Workload("c3", base.grid, base.cone, base.ref, scan_angle(view_index), 3.0,
                    levels, mbc, coeff, nbases, np.asarray(view_index))


def random_views(seed: int, nviews: int, total: int = SCAN_VIEWS) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(total, size=nviews, replace=False))


def headline(nviews: int = 32, nbases: int = NBASES) -> Workload:
    """The measured fwd+bwd iteration: motion path with 32 random views of 660."""
    w = c3(nviews=nviews, nbases=nbases, view_index=random_views(5, nviews))
    w.name = "h"
    return w


def perturbed_truth(w: Workload, seed: int = 3) -> Workload:
    """Perturbed copy used to synthesise target projections: means + N(0, 0.25
    voxel), densities x (1 + U[-0.1, 0.1]), MBC values + N(0, 0.2 mm),
    coefficients + N(0, 0.05)."""
    rng = np.random.default_rng(seed)
    hmin = float(min(w.grid.h))
    ref = w.ref.copy()
    ref.mean = _f32(ref.mean.astype(np.float64) + rng.normal(0.0, 0.25 * hmin, ref.mean.shape))
    ref.value = _f32(ref.value.astype(np.float64) * (1.0 + rng.uniform(-0.1, 0.1, ref.value.shape)))
    mbc = []
    for s in w.mbc:
        s2 = s.copy()
        s2.value = _f32(s2.value.astype(np.float64) + rng.normal(0.0, 0.2, s2.value.shape))
        mbc.append(s2)
    coeff = None if w.coeff is None else _f32(w.coeff.astype(np.float64) + rng.normal(0.0, 0.05, w.coeff.shape))
    return dataclasses.replace(w, name=w.name + "_truth", ref=ref, mbc=mbc, coeff=coeff)


def add_target_noise(proj: np.ndarray, seed: int = 3) -> np.ndarray:
    """T = P + 0.01 sqrt(max(P,0) mean(P)) xi: 1% Poisson-like noise on given projections."""
    rng = np.random.default_rng(seed + 1000)
    p = np.asarray(proj, np.float64)
    sd = 0.01 * np.sqrt(np.maximum(p, 0.0) * max(float(p.mean()), 0.0))
    return _f32(p + sd * rng.standard_normal(p.shape))


def c5_scans(seed: int = 4, nviews: int = 32) -> List[Workload]:
    """Three concurrent scans of different sizes (ragged batch), spacing
    1.5x1.5x2 mm, 100k/60k/25k reference Gaussians, MBC grids at
    (n/4, n/4, nz/2), (n/2, n/2, nz), n."""
    out = []
    for s, (dims, m) in enumerate((((256, 256, 128), 100_000), ((192, 192, 96), 60_000),
                                    ((128, 128, 64), 25_000))):
        rng = np.random.default_rng(seed + s)
        grid = Grid(dims, (1.5, 1.5, 2.0))
        ref = reference_set(rng, m, grid)
        ld = [(dims[0] // 4, dims[1] // 4, dims[2] // 2), (dims[0] // 2, dims[1] // 2, dims[2]), dims]
        levels = level_grids(grid, ld)
        mbc = mbc_sets(rng, levels, MBC_COUNTS, NBASES)
        vi = np.sort(rng.choice(SCAN_VIEWS, size=nviews, replace=False))
        coeff = sinusoid_coefficients(rng, scan_time(vi), 3, NBASES)
        out.append(Workload(f"c5_{s}", grid, Cone(**VARIAN, step=0.75), ref, scan_angle(vi), 3.0,
                            levels, mbc, coeff, NBASES, vi))
    return out


def fd32(seed: int = 6, nbases: int = NBASES) -> Workload:
    """Finite-difference subcase: 32^3 grid at 2 mm, 1,000 reference Gaussians,
    MBC levels 8^3/16^3/32^3 with 16/64/256 Gaussians, 4 views of a 48x48
    detector at 2 mm, step 1 mm, untruncated."""
    rng = np.random.default_rng(seed)
    grid = Grid((32, 32, 32), (2.0, 2.0, 2.0))
    ref = gaussians(rng, 1000, grid, rho=(0.0, 0.05))
    levels = level_grids(grid, [(8, 8, 8), (16, 16, 16), (32, 32, 32)])
    mbc = mbc_sets(rng, levels, (16, 64, 256), nbases)
    vi = (np.arange(4) * SCAN_VIEWS) // 4
    coeff = sinusoid_coefficients(rng, scan_time(vi), 3, nbases)
    cone = Cone(1000.0, 1500.0, 48, 48, 2.0, 2.0, step=1.0)
    return Workload("fd32", grid, cone, ref, scan_angle(vi), math.inf, levels, mbc, coeff, nbases, vi)


def small_motion(seed: int = 7, n=(24, 20, 18), h=(2.0, 2.5, 3.0), m: int = 300,
                 level_dims=((6, 5, 9), (12, 10, 9), (24, 20, 18)), counts=(8, 24, 96),
                 nbases: int = 2, nviews: int = 3, det=(40, 30), du=2.5, step=0.0,
                 trunc_k: float = 3.0) -> Workload:
    """A small anisotropic motion-path case (ragged, non-power-of-two sizes)
    whose oracle runs in well under a second."""
    rng = np.random.default_rng(seed)
    grid = Grid(tuple(n), tuple(h))
    ref = gaussians(rng, m, grid, rho=(0.0, 0.05))
    levels = level_grids(grid, level_dims)
    mbc = mbc_sets(rng, levels, counts, nbases, value_sigma=2.0)
    vi = np.sort(rng.choice(SCAN_VIEWS, size=nviews, replace=False))
    coeff = sinusoid_coefficients(rng, scan_time(vi), len(levels), nbases)
    cone = Cone(1000.0, 1500.0, det[0], det[1], du, du, step=step)
    return Workload("small", grid, cone, ref, scan_angle(vi), trunc_k, levels, mbc, coeff, nbases, vi)


def random_volume(seed: int, shape, lo=0.0, hi=1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return _f32(rng.uniform(lo, hi, shape))


def random_normal(seed: int, shape, sigma=1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return _f32(rng.normal(0.0, sigma, shape))


def projection_like(seed: int, V: int, nv: int, nu: int, peak: float = 10.0) -> np.ndarray:
    """Seeded smooth non-negative images with the look of cone-beam line
    integrals (a body-shaped ellipse of level ~0.6 peak plus a few bright
    blobs, zero outside), [V][nv][nu] float32."""
    rng = np.random.default_rng(seed)
    vv, uu = np.meshgrid(np.linspace(-1, 1, nv), np.linspace(-1, 1, nu), indexing="ij")
    out = np.zeros((V, nv, nu))
    for v in range(V):
        a, b = rng.uniform(0.55, 0.8), rng.uniform(0.7, 0.95)
        r2 = (uu / a) ** 2 + (vv / b) ** 2
        img = 0.6 * peak * np.sqrt(np.clip(1.0 - r2, 0.0, None))
        for _ in range(6):
            cu, cv = rng.uniform(-0.5, 0.5, 2)
            s = rng.uniform(0.03, 0.15)
            img += rng.uniform(0.1, 0.4) * peak * np.exp(-((uu - cu) ** 2 + (vv - cv) ** 2) / (2 * s * s))
        out[v] = img
    return _f32(out)
