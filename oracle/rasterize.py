"""FP64 oracle of the X-ray Gaussian rasterizer (Eq. 7-9) -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module; the product path never loads it.

Plain PyTorch CPU operations in float64; gradients by autograd.  The steps
follow Sec. 2.2 in the paper's order:

1. the view transform W (world to the source-centred frame whose axes are
   the detector's u and v directions and the central ray) and the projective
   map phi of Eq. 8: a point with view coordinates t goes to the continuous
   pixel coordinates (SDD t_u / (t_d du) + (nu-1)/2 - off_u,
   SDD t_v / (t_d dv) + (nv-1)/2 - off_v) and to the distance |t| from the
   source along its ray;
2. the local affine approximation: J = d phi / d t at the Gaussian's centre,
   Sigma~ = J W Sigma W^T J^T (Eq. 8);
3. integration along the ray coordinate (Eq. 9): the 2-D Gaussian with
   centre phi(p) (first two coordinates), covariance Sigma^ = the top-left
   2 x 2 block of Sigma~ and amplitude rho sqrt(2 pi |Sigma~| / |Sigma^|);
4. the pixel value is the sum over Gaussians of their 2-D Gaussians at the
   pixel centre (Eq. 9; X-ray values add, no compositing).

Readings of what the paper leaves open: the geometry is that of the
projector (source at SAD (cos th, sin th, 0), flat detector at distance SDD,
u axis (-sin th, cos th, 0), v = z, pixel centres as in the ray march);
Sigma = R(q) diag(s^2) R(q)^T with the normalised quaternion (as for the
voxelizer); each 2-D Gaussian is truncated to its ellipse
(x - mu)^T Sigma^-1 (x - mu) <= k^2 (k = 3, k = inf for none; the mask is
not differentiated); Gaussians whose centre is not in front of the source
(t_d <= 0) are skipped; no dilation of Sigma^ is added.
"""
from __future__ import annotations

import math
from typing import Dict, Optional, Sequence, Tuple

import numpy as np
import torch


def _rotation(q: torch.Tensor) -> torch.Tensor:
    q = q / torch.linalg.norm(q, dim=1, keepdim=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], 1)


def splat_params(mean, scale, quat, value, cone, theta: float):
    """Per Gaussian for one view: 2-D centre [M][2] (pixel units), 2-D
    covariance [M][2][2], amplitude rho^ [M] and the in-front mask [M]."""
    ct, st = math.cos(theta), math.sin(theta)
    o = torch.tensor([cone.sad * ct, cone.sad * st, 0.0], dtype=torch.float64)
    W = torch.tensor([[-st, ct, 0.0], [0.0, 0.0, 1.0], [-ct, -st, 0.0]], dtype=torch.float64)
    t = (mean - o) @ W.T                                        # view coordinates [M][3]
    front = t[:, 2] > 0
    td = torch.where(front, t[:, 2], torch.ones_like(t[:, 2]))
    su, sv = cone.sdd / cone.du, cone.sdd / cone.dv
    mu = torch.stack([su * t[:, 0] / td + 0.5 * (cone.nu - 1) - cone.off_u,
                      sv * t[:, 1] / td + 0.5 * (cone.nv - 1) - cone.off_v], -1)
    z = torch.zeros_like(td)
    nt = torch.linalg.norm(t, dim=1)
    J = torch.stack([
        torch.stack([su / td, z, -su * t[:, 0] / (td * td)], -1),
        torch.stack([z, sv / td, -sv * t[:, 1] / (td * td)], -1),
        t / nt[:, None],
    ], 1)                                                       # [M][3][3]
    R = _rotation(quat)
    Sig = R @ torch.diag_embed(scale * scale) @ R.transpose(1, 2)
    M = J @ W
    St = M @ Sig @ M.transpose(1, 2)                            # Sigma~ (Eq. 8)
    Sh = St[:, :2, :2]                                          # Sigma^ (Eq. 9)
    rho = value[:, 0] * torch.sqrt(2.0 * math.pi * torch.linalg.det(St) / torch.linalg.det(Sh))
    return mu, Sh, rho, front


def rasterize_t(mean, scale, quat, value, cone, angles: Sequence[float], k: float = 3.0,
                chunk: int = 256, pixels=None) -> torch.Tensor:
    """Projections [V][nv][nu] (torch, differentiable in the parameters), or
    with pixels = [P][2] integer (iu, iv) pairs the values at those pixels
    only, [V][P]."""
    if pixels is None:
        iv, iu = torch.meshgrid(torch.arange(cone.nv, dtype=torch.float64),
                                torch.arange(cone.nu, dtype=torch.float64), indexing="ij")
        pix = torch.stack([iu.reshape(-1), iv.reshape(-1)], -1)     # [P][2] (u, v)
    else:
        pix = torch.tensor(np.asarray(pixels, np.float64))
    out = []
    for th in angles:
        mu, Sh, rho, front = splat_params(mean, scale, quat, value, cone, float(th))
        A = torch.linalg.inv(Sh)
        img = torch.zeros(pix.shape[0], dtype=torch.float64)
        for c0 in range(0, mean.shape[0], chunk):
            sl = slice(c0, c0 + chunk)
            d = pix[None, :, :] - mu[sl, None, :]               # [c][P][2]
            m = torch.einsum("cpi,cij,cpj->cp", d, A[sl], d)
            keep = front[sl, None].expand_as(m)
            if math.isfinite(k):
                keep = keep & (m.detach() <= k * k)
            e = torch.where(keep, torch.exp(-0.5 * m), torch.zeros_like(m))
            img = img + (rho[sl, None] * e).sum(0)
        out.append(img.reshape(cone.nv, cone.nu) if pixels is None else img)
    return torch.stack(out)


def _tensors(gs):
    f = lambda a: torch.tensor(np.asarray(a, np.float64), dtype=torch.float64, requires_grad=True)
    return f(gs.mean), f(gs.scale), f(gs.quat), f(gs.value)


def rasterize(gs, cone, angles, k: float = 3.0, pixels=None) -> np.ndarray:
    """Eq. 9 projections of GaussSet gs, [V][nv][nu] float64 (or [V][P] at
    the given (iu, iv) pixels)."""
    with torch.no_grad():
        t = _tensors(gs)
        return rasterize_t(*t, cone, angles, k, pixels=pixels).numpy()


def rasterize_bwd(gs, cone, angles, k: float, g_proj) -> Dict[str, np.ndarray]:
    """Gradients of sum(g_proj * rasterize(gs)) with respect to the Gaussian
    parameters (mean, scale, quat, value), by autograd in float64."""
    t = _tensors(gs)
    p = rasterize_t(*t, cone, angles, k)
    (p * torch.tensor(np.asarray(g_proj, np.float64))).sum().backward()
    return {n: x.grad.numpy() for n, x in zip(("mean", "scale", "quat", "value"), t)}


def line_integral(mean, scale, quat, rho, cone, theta: float) -> np.ndarray:
    """Exact (untruncated, unbounded) line integral of one 3-D Gaussian along
    every pixel's ray: rho sqrt(2 pi / d^T A d) exp(-(w^T A w - (d^T A w)^2 /
    d^T A d) / 2), A = Sigma^-1, w = source - mean, d the unit ray direction.
    Closed form used to pin the rasterizer."""
    ct, st = math.cos(theta), math.sin(theta)
    o = np.array([cone.sad * ct, cone.sad * st, 0.0])
    eu = np.array([-st, ct, 0.0])
    ez = np.array([0.0, 0.0, 1.0])
    c_det = -(cone.sdd - cone.sad) * np.array([ct, st, 0.0])
    with torch.no_grad():
        R = _rotation(torch.tensor(np.asarray(quat, np.float64)[None]))[0].numpy()
    A = R @ np.diag(1.0 / np.asarray(scale, np.float64) ** 2) @ R.T
    w = o - np.asarray(mean, np.float64)
    out = np.zeros((cone.nv, cone.nu))
    for iv in range(cone.nv):
        for iu in range(cone.nu):
            a = (iu - 0.5 * (cone.nu - 1) + cone.off_u) * cone.du
            b = (iv - 0.5 * (cone.nv - 1) + cone.off_v) * cone.dv
            d = c_det + a * eu + b * ez - o
            d /= np.linalg.norm(d)
            dad, daw, waw = d @ A @ d, d @ A @ w, w @ A @ w
            out[iv, iu] = rho * math.sqrt(2 * math.pi / dad) * math.exp(-0.5 * (waw - daw * daw / dad))
    return out
