"""Pins of the soft silhouette oracle (SoftRas-style renderer used for pixel losses).

Closed forms: pinhole projection; a pixel centre on a triangle edge has coverage
exactly 1/2; a pixel at distance d outside one triangle sees sigmoid(-d^2/sigma); two
triangles compose as 1 - (1 - D1)(1 - D2); far pixels are exactly 0 and deep inside
pixels are 1 to rounding.  The image does not depend on the winding.  The autograd
gradient with respect to the vertices matches central differences.
"""
import math

import numpy as np
import torch

from oracle import raster as R

F64 = torch.float64


def pinhole(f, cx, cy):
    """Camera at the origin looking along +z: u = f X/Z + cx, v = f Y/Z + cy."""
    return torch.tensor([[f, 0, cx, 0], [0, f, cy, 0], [0, 0, 1, 0]], dtype=F64)


def screen_mesh(uv, z=2.0, f=10.0):
    """World vertices that project exactly to the pixel coordinates uv under
    pinhole(f, 0, 0) at depth z."""
    uv = torch.as_tensor(uv, dtype=F64)
    return torch.cat([uv * z / f, torch.full((uv.shape[0], 1), z, dtype=F64)], 1)


def sig(x):
    return 1.0 / (1.0 + math.exp(-x))


def test_projection():
    P = pinhole(100.0, 32.0, 16.0)
    X = torch.tensor([[0.5, -0.25, 2.0], [0.0, 0.0, 5.0]], dtype=F64)
    uv = R.project(X, P)
    assert torch.allclose(uv, torch.tensor([[57.0, 3.5], [32.0, 16.0]], dtype=F64), atol=1e-12)


def test_edge_distance_and_composition():
    sigma = 2.0
    P = pinhole(10.0, 0.0, 0.0)
    # triangle with its left edge on u = 4.5 (through pixel centres of column 4)
    tri = screen_mesh([[4.5, 0.0], [20.0, 10.0], [4.5, 20.0]])
    img = R.silhouette(tri, torch.tensor([[0, 1, 2]]), P, 12, 12, sigma)
    assert abs(float(img[10, 4]) - 0.5) < 1e-12          # on the edge: D = 1/2
    assert abs(float(img[10, 3]) - sig(-1.0 / sigma)) < 1e-12  # 1 pixel outside
    assert abs(float(img[10, 2]) - sig(-4.0 / sigma)) < 1e-12  # 2 pixels outside
    assert abs(float(img[10, 0]) - sig(-16.0 / sigma)) < 1e-12  # 4 pixels outside (16 / sigma < CUT: kept)
    assert abs(float(img[10, 8]) - sig(16.0 / sigma)) < 1e-12   # inside, 4 pixels from the nearest edge
    # a second triangle to the left with its right edge on u = 1: pixel (10, 2) (centre
    # u = 2.5) is 2 from the first and 1.5 from the second
    tri2 = screen_mesh([[4.5, 0.0], [20.0, 10.0], [4.5, 20.0], [1.0, 0.0], [-9.0, 10.0], [1.0, 20.0]])
    img2 = R.silhouette(tri2, torch.tensor([[0, 1, 2], [3, 4, 5]]), P, 12, 12, sigma)
    d_right, d_left = 2.0, 1.5
    expect = 1 - (1 - sig(-d_right ** 2 / sigma)) * (1 - sig(-d_left ** 2 / sigma))
    assert abs(float(img2[10, 2]) - expect) < 1e-12


def test_far_pixels_are_dropped_and_winding_does_not_matter():
    sigma = 1.0
    P = pinhole(10.0, 0.0, 0.0)
    X = screen_mesh([[3.2, 2.1], [9.7, 4.4], [5.1, 8.8]])
    a = R.silhouette(X, torch.tensor([[0, 1, 2]]), P, 16, 16, sigma)
    b = R.silhouette(X, torch.tensor([[0, 2, 1]]), P, 16, 16, sigma)
    assert torch.allclose(a, b, rtol=0, atol=1e-15)  # same up to the rounding of reversed segments
    assert float(a[15, 15]) == 0.0  # > sqrt(CUT sigma) away: term dropped


def test_gradient_against_central_differences():
    rng = np.random.default_rng(0)
    sigma = 1.5
    P = pinhole(12.0, 8.0, 8.0)
    X = torch.tensor(rng.uniform(-0.5, 0.5, (6, 3)) + [0, 0, 2.0], dtype=F64)
    tris = torch.tensor([[0, 1, 2], [3, 4, 5], [1, 3, 5]])
    Wt = torch.tensor(rng.normal(size=(16, 16)), dtype=F64)
    Xg = X.clone().requires_grad_(True)
    (R.silhouette(Xg, tris, P, 16, 16, sigma) * Wt).sum().backward()
    d = torch.tensor(rng.normal(size=X.shape), dtype=F64)
    h = 1e-6
    fp = (R.silhouette(X + h * d, tris, P, 16, 16, sigma) * Wt).sum()
    fm = (R.silhouette(X - h * d, tris, P, 16, 16, sigma) * Wt).sum()
    num = float(fp - fm) / (2 * h)
    ana = float((Xg.grad * d).sum())
    assert abs(num - ana) < 1e-6 * abs(ana)
