"""FP64 oracle of the FDK reconstruction used to initialise the Gaussians
(Sec. 2.3.2, Feldkamp et al. 1984) -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module; the product path never loads it.

Plain numpy in float64, the textbook circular-orbit FDK for a flat detector
in the projector's geometry (source at SAD (cos th, sin th, 0), detector at
SDD, u along (-sin th, cos th, 0), v = z, pixel centres as in the ray march),
written on the virtual detector through the isocentre (pitches scaled by
SAD / SDD):

1. cosine weighting p~(a, b) = p(a, b) SDD / sqrt(SDD^2 + a^2 + b^2), with
   (a, b) the pixel's detector coordinates;
2. ramp filtering of each detector row with the discrete Ram-Lak kernel of
   the virtual pitch tau (h[0] = 1 / (4 tau^2), h[n odd] = -1 / (pi n tau)^2,
   h[n even] = 0), rows zero-padded: q[n] = tau sum_k h[n - k] p~[k];
3. voxel-driven back-projection
   f(x) = 1/2 sum_views dtheta (SAD / U)^2 q(a', b'),
   U = the depth of x along the central ray from the source, (a', b') = SAD
   (t_u, t_v) / U its virtual-detector coordinates, q interpolated bilinearly
   between pixel centres (0 outside the detector), dtheta = 2 pi / V (views
   evenly covering 360 degrees).

Readings of what the paper leaves open ("a quick FDK reconstruction"): the
plain Ram-Lak kernel without apodisation, linear interpolation, full-scan
weighting 1/2, no short-scan (Parker) weights.

``grid_init`` is the grid-based sampling that seeds the reference Gaussians
from the FDK image (Sec. 2.3.2): lattice points keep their positions and the
image's intensities as densities.  Readings: the lattice evenly fills the
volume box (m_a points per axis at box_lo + (k + 1/2) box_len / m_a), the
intensity is the trilinear value of the image at the point, the initial
rotation is the identity and the scale is the caller's.
"""
from __future__ import annotations

import math

import numpy as np


def ramlak(n: int, tau: float) -> np.ndarray:
    """Kernel taps h[-(n-1)..(n-1)] of the discrete Ram-Lak filter."""
    k = np.arange(-(n - 1), n)
    h = np.zeros(2 * n - 1)
    h[k == 0] = 1.0 / (4.0 * tau * tau)
    odd = (k % 2) != 0
    h[odd] = -1.0 / (math.pi * k[odd] * tau) ** 2
    return h


def filter_rows(proj, cone) -> np.ndarray:
    """Steps 1-2: cosine-weighted, ramp-filtered projections [V][nv][nu]."""
    p = np.asarray(proj, np.float64)
    V, nv, nu = p.shape
    a = (np.arange(nu) - 0.5 * (nu - 1) + cone.off_u) * cone.du
    b = (np.arange(nv) - 0.5 * (nv - 1) + cone.off_v) * cone.dv
    w = cone.sdd / np.sqrt(cone.sdd ** 2 + a[None, :] ** 2 + b[:, None] ** 2)
    pw = p * w[None]
    tau = cone.du * cone.sad / cone.sdd
    h = ramlak(nu, tau)
    q = np.zeros_like(pw)
    for n in range(nu):
        # q[n] = tau sum_k h[n - k] pw[k]; h index of (n - k) is (n - k) + nu - 1
        q[:, :, n] = tau * (pw * h[n - np.arange(nu) + nu - 1][None, None, :]).sum(axis=2)
    return q


def backproject(q, cone, angles, grid, points=None) -> np.ndarray:
    """Step 3: the FDK volume [n0][n1][n2] from filtered projections q (or
    its values at world points [P][3])."""
    q = np.asarray(q, np.float64)
    V, nv, nu = q.shape
    if points is None:
        n = grid.n
        ax = [np.asarray(grid.center[i]) + (np.arange(n[i]) - (n[i] - 1) / 2.0) * grid.h[i]
              for i in range(3)]
        X, Y, Z = np.meshgrid(*ax, indexing="ij")
    else:
        pts = np.asarray(points, np.float64)
        X, Y, Z = pts[:, 0], pts[:, 1], pts[:, 2]
    f = np.zeros(X.shape)
    tau_u, tau_v = cone.du * cone.sad / cone.sdd, cone.dv * cone.sad / cone.sdd
    dth = 2.0 * math.pi / V
    for v in range(V):
        th = float(angles[v])
        ct, st = math.cos(th), math.sin(th)
        dx, dy = X - cone.sad * ct, Y - cone.sad * st
        tu = -st * dx + ct * dy
        td = -ct * dx - st * dy
        U = td
        ap = cone.sad * tu / U
        bp = cone.sad * Z / U
        # continuous pixel coordinates on the virtual detector
        fu = ap / tau_u + 0.5 * (nu - 1) - cone.off_u
        fv = bp / tau_v + 0.5 * (nv - 1) - cone.off_v
        i0 = np.floor(fu).astype(np.int64)
        j0 = np.floor(fv).astype(np.int64)
        wu = fu - i0
        wv = fv - j0
        val = np.zeros_like(f)
        for di, wi in ((0, 1.0 - wu), (1, wu)):
            for dj, wj in ((0, 1.0 - wv), (1, wv)):
                ii, jj = i0 + di, j0 + dj
                ok = (ii >= 0) & (ii < nu) & (jj >= 0) & (jj < nv)
                s = np.zeros_like(f)
                s[ok] = q[v, jj[ok], ii[ok]]
                val += wi * wj * s
        f += 0.5 * dth * (cone.sad / U) ** 2 * val
    return f


def fdk(proj, cone, angles, grid, points=None) -> np.ndarray:
    return backproject(filter_rows(proj, cone), cone, angles, grid, points)


def ball_projections(center, radius: float, rho: float, cone, angles) -> np.ndarray:
    """Exact line integrals of a uniform ball (2 rho sqrt(r^2 - d^2), d the
    distance of the ray from the centre): the analytic phantom of the pins."""
    c = np.asarray(center, np.float64)
    out = np.zeros((len(angles), cone.nv, cone.nu))
    a = (np.arange(cone.nu) - 0.5 * (cone.nu - 1) + cone.off_u) * cone.du
    b = (np.arange(cone.nv) - 0.5 * (cone.nv - 1) + cone.off_v) * cone.dv
    A, B = np.meshgrid(a, b)
    for v, th in enumerate(angles):
        ct, st = math.cos(th), math.sin(th)
        o = np.array([cone.sad * ct, cone.sad * st, 0.0])
        det = -(cone.sdd - cone.sad) * np.array([ct, st, 0.0])
        P = det[None, None, :] + A[..., None] * np.array([-st, ct, 0.0]) + B[..., None] * np.array([0, 0, 1.0])
        d = P - o
        d /= np.linalg.norm(d, axis=-1, keepdims=True)
        w = c - o
        proj_len = (d * w).sum(-1)
        dist2 = (w * w).sum() - proj_len ** 2
        out[v] = 2.0 * rho * np.sqrt(np.clip(radius * radius - dist2, 0.0, None))
    return out


def grid_init(vol, grid, m, scale: float):
    """Initial Gaussians from the lattice m = (m0, m1, m2) over the volume box
    (axis 2 fastest): mean [M][3], scale [M][3], quat [M][4], value [M][1]."""
    from oracle import sample_points
    axes = []
    for a in range(3):
        L = grid.n[a] * grid.h[a]
        lo = grid.center[a] - 0.5 * L
        axes.append(lo + (np.arange(m[a]) + 0.5) * L / m[a])
    P = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, 3)
    M = P.shape[0]
    val = sample_points(vol, grid, P)
    quat = np.zeros((M, 4))
    quat[:, 0] = 1.0
    return P, np.full((M, 3), float(scale)), quat, val.reshape(M, 1)
