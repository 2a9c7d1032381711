"""Test-side helpers: build the oracle and the HIP model from the same seeded bodies,
and compare results.  (Tests only; the product path never imports this.)"""
import numpy as np

from paper_2104_02646_amd import workloads as W


def oracle_for(o, body):
    return o.Oracle(body.X, tets=body.tets, tris=body.tris, hinges=body.hinges, pinned=body.pinned,
                    gravity=body.gravity, ground=body.ground, plane=body.plane, dt=body.dt, air=body.air)


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    d = np.linalg.norm((a - b).ravel())
    n = np.linalg.norm(b.ravel())
    return d / n if n > 0 else d


def maxrel(a, b):
    """Largest element-wise difference relative to the largest reference magnitude:
    a localized error that the norm ratio would average away shows here."""
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    if a.size == 0:
        return 0.0
    d = np.abs(a - b).max()
    n = np.abs(b).max()
    return d / n if n > 0 else d


def mixed_body(seed=0):
    """Tet cube in sliding contact + small pinned cloth with bending (every force term)."""
    tet = W.tiny_cube(seed)
    cl = W.cloth(seed + 11, n=6, size=0.25, height=0.5)
    off = tet.np
    X = np.concatenate([tet.X, cl.X])
    v0 = np.concatenate([tet.v0, np.zeros_like(cl.X)])
    return W.Body(X=X, tets=tet.tets, tris=cl.tris + off, hinges=cl.hinges + off,
                  pinned=np.concatenate([tet.pinned, cl.pinned]), mu=tet.mu, lam=tet.lam, ktri=cl.ktri,
                  mass=np.concatenate([tet.mass, np.full(cl.np, 0.1)]), kb=0.05, ke=1e4, kd=3.0, kf=100.0,
                  muf=0.5, ground=True, dt=1.0 / 600, x0=X.copy(), v0=v0)


def perturbed_state(body, seed, depth=0.01):
    """A state with deformation, some particles below the ground, mixed stick/slip."""
    rng = np.random.default_rng(seed)
    x = body.x0 + rng.normal(0, 0.002, body.X.shape)
    if body.ground:
        low = np.argsort(x[:, 1])[: max(1, body.np // 4)]
        x[low, 1] -= depth
    v = body.v0 + rng.normal(0, 0.3, body.X.shape)
    v[rng.random(body.np) < 0.3] *= 0.01  # slow particles: stick branch
    return x, v
