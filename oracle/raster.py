"""FP64 oracle of the soft silhouette renderer (test infrastructure only).

The paper renders its simulated meshes with a differentiable soft rasterizer
(SoftRas, DIB-R: Sec. 3 and App. on rendering) so that losses sit on pixels.  The
reading built here is SoftRas's silhouette: each vertex X is projected by a 3x4
camera matrix P to pixel coordinates u = (P0 . [X, 1]) / (P2 . [X, 1]),
v = (P1 . [X, 1]) / (P2 . [X, 1]); each triangle j covers pixel p (centre
(col + 0.5, row + 0.5)) with probability D_j(p) = sigmoid(delta_j(p) d_j(p)^2 / sigma),
d_j the distance from p to the triangle's boundary in pixels, delta_j = +1 inside,
-1 outside; the silhouette is I(p) = 1 - prod_j (1 - D_j(p)).  Terms with p outside
and d^2 > CUT sigma (D < 1e-6) are dropped, as the kernels do.  Plain float64 PyTorch
on the CPU; its gradients come from torch's autograd.  Nothing here is shared with
the HIP path.
"""
from __future__ import annotations

import math

import torch

CUT = -math.log(1e-6)  # outside terms with d^2 / sigma above this are dropped


def project(X, P):
    """X [n, 3] -> pixel coordinates [n, 2] under the 3x4 camera matrix P."""
    Xh = torch.cat([X, torch.ones(X.shape[0], 1, dtype=X.dtype)], 1)
    q = Xh @ P.T
    return q[:, :2] / q[:, 2:3]


def _seg_dist2(p, a, b):
    """Squared distance from points p [M, 1, 2] to segments a -> b [1, N, 2]."""
    e = b - a
    w = p - a
    t = ((w * e).sum(-1) / (e * e).sum(-1)).clamp(0.0, 1.0)
    q = a + t.unsqueeze(-1) * e
    return ((p - q) ** 2).sum(-1)


def silhouette(X, tris, P, height, width, sigma):
    """Soft silhouette image [height, width] of the triangle mesh (X [n, 3] world
    positions, tris [nt, 3]) seen through P; differentiable in X."""
    uv = project(X, P)
    A, B, C = uv[tris[:, 0]], uv[tris[:, 1]], uv[tris[:, 2]]
    rows, cols = torch.meshgrid(torch.arange(height, dtype=X.dtype), torch.arange(width, dtype=X.dtype),
                                indexing="ij")
    p = torch.stack([cols.reshape(-1) + 0.5, rows.reshape(-1) + 0.5], -1)[:, None, :]  # [M, 1, 2]
    a, b, c = A[None], B[None], C[None]
    cr = lambda s, t: s[..., 0] * t[..., 1] - s[..., 1] * t[..., 0]
    e0, e1, e2 = cr(b - a, p - a), cr(c - b, p - b), cr(a - c, p - c)
    area = cr(b - a, c - a)
    inside = ((e0 >= 0) & (e1 >= 0) & (e2 >= 0) & (area > 0)) | ((e0 <= 0) & (e1 <= 0) & (e2 <= 0) & (area < 0))
    d2 = torch.minimum(torch.minimum(_seg_dist2(p, a, b), _seg_dist2(p, b, c)), _seg_dist2(p, c, a))
    x = torch.where(inside, d2, -d2) / sigma
    keep = inside | (d2 <= CUT * sigma)
    log1m = torch.where(keep, -torch.nn.functional.softplus(x), torch.zeros_like(x))  # log(1 - D)
    return (1.0 - torch.exp(log1m.sum(1))).reshape(height, width)
