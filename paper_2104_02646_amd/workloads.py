"""Seeded synthetic inputs: meshes, material parameters, initial states, targets.

This module produces inputs only.  It holds none of the simulation's arithmetic
(no rest-shape precompute, no forces, no integration), so both the HIP path and
the FP64 oracle may consume what it generates.  Every generator takes an
explicit ``numpy.random.Generator`` seed; the same seed yields the same bytes.

Geometry conventions: y is up, the ground is the plane y = 0.  Arrays are numpy,
AoS ``[n, 3]`` float64 for positions, int32 for topology.

Workload recipes (the paper's deformable / thin-shell settings, App. A.1 and
App. B, with every constant the paper leaves open written out here):

* ``tiny_cube``      3x3x3 hexes, 6 tets each (162 tets, 64 particles)
* ``cloth``          64x64 particle grid, 7938 triangles, 11781 bending hinges
* ``batch_bodies``   256 tet bodies, counts log-uniform in [500, 20000]
* ``large_blob``     ~200k tets voxelised from a sum-of-5-spheres implicit blob
* ``serving_trace``  Poisson stream of tet / cloth gradient queries
* ``gear``, ``walker``  actuated bodies of the control tasks (1152 / 168 tets)
* ``control_cloth``  free cloth under lift/drag (72 .. 2048 triangles)
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import permutations

import numpy as np

GRAVITY = (0.0, -9.81, 0.0)
GROUND = (0.0, 1.0, 0.0, 0.0)  # plane n.x = d with n = +y, d = 0

# ----------------------------------------------------------------------------------
# Mesh generators
# ----------------------------------------------------------------------------------

# Kuhn / Freudenthal split of the unit cube into 6 tets around the (0,0,0)-(1,1,1)
# diagonal: for each axis permutation p the tet is 0, e_p0, e_p0+e_p1, (1,1,1).
# The orientation of such a simplex equals the sign of the permutation, so odd
# permutations have two corners swapped to make every tet positively oriented.
_KUHN = []
for _perm in permutations(range(3)):
    _c = [(0, 0, 0)]
    _p = [0, 0, 0]
    for _a in _perm:
        _p[_a] = 1
        _c.append(tuple(_p))
    _inv = sum(1 for i in range(3) for j in range(i + 1, 3) if _perm[i] > _perm[j])
    if _inv % 2 == 1:
        _c[1], _c[2] = _c[2], _c[1]
    _KUHN.append(_c)


def voxel_tets(mask: np.ndarray, h: float, origin=(0.0, 0.0, 0.0)):
    """Tetrahedralise the occupied voxels of a boolean grid ``mask[nx, ny, nz]``.

    Each voxel becomes 6 Kuhn tets (conforming across faces because every voxel uses
    the same diagonal).  Particles are the voxel corners that are used, numbered in
    lexicographic (x, y, z) order; tets are listed voxel by voxel in the same order.
    Returns ``X [np, 3]``, ``tets [ne, 4]``.
    """
    mask = np.asarray(mask, bool)
    nx, ny, nz = mask.shape
    vox = np.argwhere(mask)  # lexicographic order
    corner_id = -np.ones((nx + 1, ny + 1, nz + 1), np.int64)
    offs = np.array([[a, b, c] for a in (0, 1) for b in (0, 1) for c in (0, 1)])
    used = np.zeros((nx + 1, ny + 1, nz + 1), bool)
    for o in offs:
        used[vox[:, 0] + o[0], vox[:, 1] + o[1], vox[:, 2] + o[2]] = True
    cid = np.argwhere(used)
    corner_id[cid[:, 0], cid[:, 1], cid[:, 2]] = np.arange(len(cid))
    X = cid.astype(np.float64) * h + np.asarray(origin, np.float64)
    tets = np.empty((len(vox) * 6, 4), np.int32)
    for k, simplex in enumerate(_KUHN):
        for j, c in enumerate(simplex):
            tets[k::6, j] = corner_id[vox[:, 0] + c[0], vox[:, 1] + c[1], vox[:, 2] + c[2]]
    return X, tets


def box_tets(nx: int, ny: int, nz: int, h: float, origin=(0.0, 0.0, 0.0)):
    return voxel_tets(np.ones((nx, ny, nz), bool), h, origin)


def cloth_grid(n: int, spacing: float, height: float):
    """``n x n`` particles in the x-z plane at y = height; each quad split along the
    same diagonal.  Returns X, tris [2(n-1)^2, 3], hinges [n_interior_edges, 4] with
    hinge = (wing0, wing1, edge0, edge1)."""
    ii, kk = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    X = np.stack([ii.ravel() * spacing, np.full(n * n, height), kk.ravel() * spacing], 1).astype(np.float64)
    pid = (ii * n + kk).astype(np.int32)
    a = pid[:-1, :-1].ravel(); b = pid[1:, :-1].ravel(); c = pid[1:, 1:].ravel(); d = pid[:-1, 1:].ravel()
    tris = np.empty((2 * len(a), 3), np.int32)
    tris[0::2] = np.stack([a, b, c], 1)
    tris[1::2] = np.stack([a, c, d], 1)
    hinges = hinges_from_tris(tris)
    return X, tris, hinges


def hinges_from_tris(tris: np.ndarray) -> np.ndarray:
    """Interior edges shared by exactly two triangles, as (wing0, wing1, e0, e1) with
    e0 < e1, sorted by edge; wing0 belongs to the triangle listed first."""
    t = np.asarray(tris, np.int64).reshape(-1, 3)
    if len(t) == 0:
        return np.zeros((0, 4), np.int32)
    u = np.concatenate([t[:, 0], t[:, 1], t[:, 2]])
    v = np.concatenate([t[:, 1], t[:, 2], t[:, 0]])
    w = np.concatenate([t[:, 2], t[:, 0], t[:, 1]])
    tri = np.concatenate([np.arange(len(t))] * 3)
    lo, hi = np.minimum(u, v), np.maximum(u, v)
    order = np.lexsort((tri, hi, lo))
    lo, hi, w = lo[order], hi[order], w[order]
    same = (lo[1:] == lo[:-1]) & (hi[1:] == hi[:-1])
    first = np.nonzero(same)[0]
    # an edge shared by three or more triangles is not a hinge
    bad = np.zeros(len(lo) + 1, bool)
    bad[first[1:][first[1:] - 1 == first[:-1]]] = True
    bad[first[:-1][first[1:] - 1 == first[:-1]]] = True
    keep = first[~bad[first]]
    return np.stack([w[keep], w[keep + 1], lo[keep], hi[keep]], 1).astype(np.int32)


def sphere_mask(r_vox: float):
    n = int(np.ceil(2 * r_vox)) + 1
    c = (np.arange(n) + 0.5) - n / 2.0
    gx, gy, gz = np.meshgrid(c, c, c, indexing="ij")
    return gx ** 2 + gy ** 2 + gz ** 2 <= r_vox ** 2


def _largest_component(mask: np.ndarray) -> np.ndarray:
    """Largest face-connected component of a boolean grid (iterative flood fill)."""
    lab = np.zeros(mask.shape, np.int32)
    best, best_n, cur = 0, 0, 0
    for start in map(tuple, np.argwhere(mask)):
        if lab[start]:
            continue
        cur += 1
        stack = [start]
        lab[start] = cur
        n = 0
        while stack:
            p = stack.pop()
            n += 1
            for ax in range(3):
                for s in (-1, 1):
                    q = list(p); q[ax] += s; q = tuple(q)
                    if 0 <= q[ax] < mask.shape[ax] and mask[q] and not lab[q]:
                        lab[q] = cur
                        stack.append(q)
        if n > best_n:
            best, best_n = cur, n
    return lab == best


def blob_mask(rng: np.random.Generator, target_voxels: int, tol: float = 0.02):
    """Sum-of-5-spheres implicit blob sum_i (r_i/|x-c_i|)^2 >= 1, centres U(-0.3,0.3)^3 m,
    radii U(0.15, 0.3) m, voxelised on a grid whose spacing is bisected until the
    largest face-connected component holds ``target_voxels`` (+-tol)."""
    cen = rng.uniform(-0.3, 0.3, (5, 3))
    rad = rng.uniform(0.15, 0.3, 5)
    lo_b = (cen - 3 * rad[:, None]).min(0)
    hi_b = (cen + 3 * rad[:, None]).max(0)

    def vox(h):
        n = np.ceil((hi_b - lo_b) / h).astype(int)
        axes = [lo_b[a] + (np.arange(n[a]) + 0.5) * h for a in range(3)]
        g = np.stack(np.meshgrid(*axes, indexing="ij"), -1)
        fld = np.zeros(g.shape[:3])
        for c, r in zip(cen, rad):
            d2 = ((g - c) ** 2).sum(-1)
            fld += r * r / np.maximum(d2, 1e-12)
        m = fld >= 1.0
        nz = np.argwhere(m)
        lo, hi = nz.min(0), nz.max(0) + 1
        m = m[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        return m

    h_lo, h_hi = 0.002, 0.2  # more voxels at h_lo
    m = None
    for _ in range(40):
        h = 0.5 * (h_lo + h_hi)
        m = vox(h)
        cnt = int(m.sum())
        if abs(cnt - target_voxels) <= tol * target_voxels:
            break
        if cnt > target_voxels:
            h_lo = h
        else:
            h_hi = h
    m = _largest_component(m)
    return m, h


# ----------------------------------------------------------------------------------
# Bodies
# ----------------------------------------------------------------------------------

@dataclass
class Body:
    """One simulated body: topology, rest shape, parameters, environment, start state."""
    X: np.ndarray
    tets: np.ndarray = field(default_factory=lambda: np.zeros((0, 4), np.int32))
    tris: np.ndarray = field(default_factory=lambda: np.zeros((0, 3), np.int32))
    hinges: np.ndarray = field(default_factory=lambda: np.zeros((0, 4), np.int32))
    pinned: np.ndarray | None = None
    mu: np.ndarray | None = None
    lam: np.ndarray | None = None
    ktri: np.ndarray | None = None
    mass: np.ndarray | None = None
    kb: float = 0.0
    ke: float = 0.0
    kd: float = 0.0
    kf: float = 0.0
    muf: float = 0.0
    air: bool = False        # lift/drag on the triangles
    kdrag: float = 0.0
    klift: float = 0.0
    gravity: tuple = GRAVITY
    ground: bool = False
    plane: tuple = GROUND
    dt: float = 1.0 / 600.0
    x0: np.ndarray | None = None
    v0: np.ndarray | None = None
    target: np.ndarray | None = None

    def __post_init__(self):
        n = len(self.X)
        if self.pinned is None:
            self.pinned = np.zeros(n, np.uint8)
        if self.x0 is None:
            self.x0 = self.X.copy()
        if self.v0 is None:
            self.v0 = np.zeros_like(self.X)

    @property
    def np(self):
        return len(self.X)

    @property
    def ne(self):
        return len(self.tets)

    @property
    def nt(self):
        return len(self.tris)

    @property
    def nh(self):
        return len(self.hinges)

    def params(self):
        """Parameter dict (the keys the oracle and the binding both accept)."""
        p = {"mass": self.mass, "kb": self.kb, "ke": self.ke, "kd": self.kd, "kf": self.kf, "muf": self.muf}
        if self.air:
            p["kdrag"] = self.kdrag
            p["klift"] = self.klift
        if self.ne:
            p["mu"] = self.mu
            p["lam"] = self.lam
        if self.nt:
            p["ktri"] = self.ktri
        return p

    def with_params(self, **kw):
        import copy
        b = copy.copy(self)
        for k, v in kw.items():
            setattr(b, k, v)
        return b

    def round_to(self, dtype):
        """Round every floating input to ``dtype`` (and back to float64), so an FP32 run
        and the FP64 oracle see identical inputs."""
        import copy
        b = copy.copy(self)
        r = lambda a: None if a is None else np.asarray(a, dtype).astype(np.float64)
        for k in ("X", "mu", "lam", "ktri", "mass", "x0", "v0", "target"):
            setattr(b, k, r(getattr(self, k)))
        for k in ("kb", "ke", "kd", "kf", "muf", "kdrag", "klift", "dt"):
            setattr(b, k, float(np.asarray(getattr(self, k), dtype)))
        b.gravity = tuple(float(np.asarray(g, dtype)) for g in self.gravity)
        b.plane = tuple(float(np.asarray(g, dtype)) for g in self.plane)
        return b


def _tet_materials(rng, ne, lo=1e4, hi=1e5, log=False):
    if log:
        return (np.exp(rng.uniform(np.log(lo), np.log(hi), ne)), np.exp(rng.uniform(np.log(lo), np.log(hi), ne)))
    return rng.uniform(lo, hi, ne), rng.uniform(lo, hi, ne)


def _place_on_ground(X, clearance):
    X = X.copy()
    X[:, 1] += clearance - X[:, 1].min()
    return X


def tiny_cube(seed: int = 0, h: float = 0.05):
    """Cube of 3x3x3 hexes (edge h) split into 6 tets each: 162 tets, 64 particles.
    mu, lambda ~ U(1e4, 1e5) per tet, mass ~ U(0.5, 1.5) per particle, gravity,
    ground contact k_e = 1e4, mu_f = 0.5, k_d = 0, k_f = 100, dt = 1/600.  Start:
    bottom face 0.02 m above the ground, v0 = (1, -0.5, 0) m/s."""
    rng = np.random.default_rng(seed)
    X, tets = box_tets(3, 3, 3, h)
    X = _place_on_ground(X, 0.02)
    mu, lam = _tet_materials(rng, len(tets))
    mass = rng.uniform(0.5, 1.5, len(X))
    v0 = np.tile([1.0, -0.5, 0.0], (len(X), 1))
    return Body(X=X, tets=tets, mu=mu, lam=lam, mass=mass, ke=1e4, kd=0.0, kf=100.0, muf=0.5,
                ground=True, dt=1.0 / 600.0, x0=X.copy(), v0=v0)


def redraw_tet_params(body: Body, seed: int, log=False, lo=1e4, hi=1e5):
    """An independent parameter draw theta* for the same body (system-ID target)."""
    rng = np.random.default_rng(seed)
    mu, lam = _tet_materials(rng, body.ne, lo, hi, log)
    mass = rng.uniform(0.5, 1.5, body.np)
    return body.with_params(mu=mu, lam=lam, mass=mass)


def cloth(seed: int = 10, n: int = 64, size: float = 2.0, height: float = 1.0, mass: float = 0.1,
          kb: float = 0.01):
    """n x n cloth grid (spacing size/(n-1)) at y = height; membrane k_t ~ U(1e3, 1e4) per
    triangle (mu = lambda = k_t), bending k_b, particle mass uniform, corners (0,0) and
    (n-1,0) pinned, gravity, no ground, dt = 1e-3."""
    rng = np.random.default_rng(seed)
    X, tris, hinges = cloth_grid(n, size / (n - 1), height)
    pinned = np.zeros(len(X), np.uint8)
    pinned[0] = 1                      # grid (0, 0)
    pinned[(n - 1) * n] = 1            # grid (n-1, 0)
    ktri = rng.uniform(1e3, 1e4, len(tris))
    return Body(X=X, tris=tris, hinges=hinges, pinned=pinned, ktri=ktri, mass=np.full(len(X), mass), kb=kb,
                ground=False, dt=1e-3)


def control_cloth(seed: int = 60, n: int | None = None, kdrag: float = 2.0, klift: float = 2.0):
    """Free cloth under lift/drag for the control-cloth task (Sec. 5.3: a random cloth
    of 64 to 2048 triangles is thrown towards a target; its initial velocity is
    optimised under nonlinear lift/drag).  n x n grid, n ~ U{7..33} unless given
    (2 (n-1)^2 = 72 .. 2048 triangles), side 0.5 m, 1.5 m above the ground plane
    (no contact: the task ends in the air), membrane k_t ~ U(1e3, 1e4), bending
    k_b = 0.01, particle mass 0.1 kg, gravity, air k_drag, k_lift, dt = 1e-3.
    Start: tilted 20 degrees about x, thrown with v0 = (2, 3, 0) m/s plus a seeded
    per-particle perturbation N(0, 0.1^2)."""
    rng = np.random.default_rng(seed)
    if n is None:
        n = int(rng.integers(7, 34))
    X, tris, hinges = cloth_grid(n, 0.5 / (n - 1), 0.0)
    a = np.deg2rad(20.0)
    X = X - X.mean(0)
    X = X @ np.array([[1, 0, 0], [0, np.cos(a), -np.sin(a)], [0, np.sin(a), np.cos(a)]]).T
    X[:, 1] += 1.5
    ktri = rng.uniform(1e3, 1e4, len(tris))
    v0 = np.tile([2.0, 3.0, 0.0], (len(X), 1)) + rng.normal(0.0, 0.1, X.shape)
    return Body(X=X, tris=tris, hinges=hinges, ktri=ktri, mass=np.full(len(X), 0.1), kb=0.01, ground=False,
                air=True, kdrag=kdrag, klift=klift, dt=1e-3, x0=X.copy(), v0=v0)


def redraw_cloth_params(body: Body, seed: int):
    rng = np.random.default_rng(seed)
    return body.with_params(ktri=rng.uniform(1e3, 1e4, body.nt))


def batch_body(seed: int, h: float = 0.05, lo: int = 500, hi: int = 20000):
    """One body of the multi-body batch: tet count log-uniform in [lo, hi]; box (side
    ratios U(1,2)) or grid-in-sphere with equal probability; materials, contact and
    start as ``tiny_cube``."""
    rng = np.random.default_rng(seed)
    n_target = float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
    vox_target = n_target / 6.0
    if rng.uniform() < 0.5:
        ratios = rng.uniform(1.0, 2.0, 3)
        s = (vox_target / ratios.prod()) ** (1.0 / 3.0)
        dims = np.maximum(1, np.round(ratios * s).astype(int))
        mask = np.ones(tuple(dims), bool)
    else:
        r_lo, r_hi = 0.5, 40.0
        for _ in range(60):
            r = 0.5 * (r_lo + r_hi)
            cnt = sphere_mask(r).sum()
            if cnt > vox_target:
                r_hi = r
            else:
                r_lo = r
        mask = sphere_mask(0.5 * (r_lo + r_hi))
        nz = np.argwhere(mask)
        lo_i, hi_i = nz.min(0), nz.max(0) + 1
        mask = mask[lo_i[0]:hi_i[0], lo_i[1]:hi_i[1], lo_i[2]:hi_i[2]]
    X, tets = voxel_tets(mask, h)
    X = _place_on_ground(X, 0.02)
    mu, lam = _tet_materials(rng, len(tets))
    mass = rng.uniform(0.5, 1.5, len(X))
    v0 = np.tile([1.0, -0.5, 0.0], (len(X), 1))
    return Body(X=X, tets=tets, mu=mu, lam=lam, mass=mass, ke=1e4, kd=0.0, kf=100.0, muf=0.5, ground=True,
                dt=1.0 / 600.0, x0=X.copy(), v0=v0)


def batch_bodies(seed: int = 20, n_bodies: int = 256, **kw):
    """The multi-body batch; body b draws from seed ``1000*seed + b``."""
    return [batch_body(1000 * seed + b, **kw) for b in range(n_bodies)]


def large_blob(seed: int = 30, target_tets: int = 200_000):
    """~200k-tet blob (sum of 5 spheres), mu, lambda log-uniform in [1e4, 1e6],
    mass U(0.5, 1.5), ground k_e = 1e5, mu_f = 0.5, k_d = 0, k_f = 100, dt = 1e-3,
    start 0.01 m above the ground with v0 = (1, -0.5, 0), no gravity: the body
    reaches the ground by its initial velocity (with 1 kg particles at ~3 cm
    spacing its own weight would crush the soft elements)."""
    rng = np.random.default_rng(seed)
    mask, h = blob_mask(rng, target_tets // 6)
    X, tets = voxel_tets(mask, h)
    X = _place_on_ground(X, 0.01)
    mu, lam = _tet_materials(rng, len(tets), 1e4, 1e6, log=True)
    mass = rng.uniform(0.5, 1.5, len(X))
    v0 = np.tile([1.0, -0.5, 0.0], (len(X), 1))
    return Body(X=X, tets=tets, mu=mu, lam=lam, mass=mass, ke=1e5, kd=0.0, kf=100.0, muf=0.5, ground=True,
                gravity=(0.0, 0.0, 0.0), dt=1e-3, x0=X.copy(), v0=v0)


def gear(seed: int = 50, n_teeth: int = 16, layers: int = 4, r_in: float = 0.06, dr: float = 0.03,
         dz: float = 0.02):
    """Soft gear for the actuated-locomotion control task (Sec. 5.3 control-fem: a
    gear of 1152 tets driven by per-tet actuation).  A ring of 2 n_teeth angular hex
    segments one hex deep (radii r_in .. r_in + dr) with a tooth hex (out to
    r_in + 2 dr) on every other segment, `layers` hexes thick along z; each hex is 6
    Kuhn tets: (32 + 16) x 4 = 192 hexes = 1152 tets and 480 particles for the
    defaults.  The axis is horizontal (z), so the gear stands on its teeth on the
    ground.  Rubber-like: mu, lambda ~ U(5e4, 1.5e5) Pa per tet, particle mass
    4.5 g (about 1100 kg/m^3), gravity, ground k_e = 1e4, k_d = 0, k_f = 100,
    mu_f = 0.5, dt = 5e-4 (explicit-stable for these elements), at rest 5 mm above
    the ground."""
    rng = np.random.default_rng(seed)
    na = 2 * n_teeth
    mask = np.zeros((na, 2, layers), bool)
    mask[:, 0, :] = True
    mask[0::2, 1, :] = True
    G, tets = voxel_tets(mask, 1.0)
    g = np.rint(G).astype(np.int64)
    g[:, 0] %= na  # angular index na is index 0: close the ring
    key = (g[:, 0] * 8 + g[:, 1]) * (layers + 1) + g[:, 2]
    uniq, first, inv = np.unique(key, return_index=True, return_inverse=True)
    tets = inv[tets].astype(np.int32)
    g = g[first]
    theta = 2.0 * np.pi * g[:, 0] / na
    r = r_in + dr * g[:, 1]
    X = np.stack([r * np.cos(theta), r * np.sin(theta), dz * g[:, 2]], 1)
    # (angle, radius) -> (x, y) reverses orientation: swap two corners of every tet
    tets = tets[:, [0, 2, 1, 3]].copy()
    X = _place_on_ground(X, 0.005)
    mu, lam = _tet_materials(rng, len(tets), 5e4, 1.5e5)
    mass = np.full(len(X), 0.0045)
    return Body(X=X, tets=tets, mu=mu, lam=lam, mass=mass, ke=1e4, kd=0.0, kf=100.0, muf=0.5,
                ground=True, dt=5e-4, x0=X.copy())


def walker(seed: int = 51, h: float = 0.02):
    """Planar two-legged walker for the control-walker task (Sec. 5.3: a 2D walker
    actuated per element), one voxel thick: a 10 x 2 voxel torso on two 2 x 2 voxel
    legs, 28 voxels = 168 tets.  Materials, mass and contact as for the gear; stands
    on its feet 2 mm above the ground."""
    rng = np.random.default_rng(seed)
    mask = np.zeros((10, 4, 1), bool)
    mask[:, 2:4, 0] = True
    mask[0:2, 0:2, 0] = True
    mask[8:10, 0:2, 0] = True
    X, tets = voxel_tets(mask, h)
    X = _place_on_ground(X, 0.002)
    mu, lam = _tet_materials(rng, len(tets), 5e4, 1.5e5)
    mass = np.full(len(X), 0.0045)
    return Body(X=X, tets=tets, mu=mu, lam=lam, mass=mass, ke=1e4, kd=0.0, kf=100.0, muf=0.5,
                ground=True, dt=5e-4, x0=X.copy())


def controller_weights(seed: int, n_signals: int, n: int, std: float = 0.5):
    """Initial controller weights W[n_signals, n] ~ N(0, std^2)."""
    return np.random.default_rng(seed).normal(0.0, std, (n_signals, n))


def synthetic_target(body: Body, seed: int, drop: float = 0.05, noise: float = 0.005):
    """A seeded target shape for benchmarks: the start shape lowered by ``drop`` and
    perturbed by Gaussian noise (no simulation involved)."""
    rng = np.random.default_rng(seed)
    t = body.x0.copy()
    t[:, 1] -= drop
    return t + rng.normal(0.0, noise, t.shape)


# ----------------------------------------------------------------------------------
# Serving trace
# ----------------------------------------------------------------------------------

@dataclass
class Query:
    arrival: float  # seconds from trace start
    kind: str       # "tet" or "cloth"
    size: int       # tets, or cloth side length in particles
    steps: int
    seed: int


def serving_trace(seed: int = 40, n: int = 2200, rate: float = 200.0):
    """Poisson arrivals (exponential gaps, mean rate req/s); half tet bodies with
    log-uniform [1e3, 5e4] tets, half cloth grids with side U{32..128}; steps U{50..400}."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n)
    t = np.cumsum(gaps)
    out = []
    for i in range(n):
        if rng.uniform() < 0.5:
            size = int(np.exp(rng.uniform(np.log(1e3), np.log(5e4))))
            kind = "tet"
        else:
            size = int(rng.integers(32, 129))
            kind = "cloth"
        out.append(Query(float(t[i]), kind, size, int(rng.integers(50, 401)), int(rng.integers(0, 2 ** 31 - 1))))
    return out


def query_body(q: Query) -> Body:
    if q.kind == "tet":
        b = batch_body(q.seed, lo=q.size, hi=q.size)
    else:
        b = cloth(q.seed, n=q.size)
    b.target = synthetic_target(b, q.seed + 1)
    return b


# ----------------------------------------------------------------------------------
# Rigid bodies
# ----------------------------------------------------------------------------------

@dataclass
class RigidBody:
    """One rigid body: body-frame vertices about the centre of mass, mass, body-frame
    inertia [Ixx, Iyy, Izz, Ixy, Ixz, Iyz], vertex contact [k_e, k_d, k_f, mu_f],
    environment, and the start state s0 = [x, quaternion (w first), v, omega]."""
    verts: np.ndarray
    mass: float
    inertia: np.ndarray
    ke: float = 300.0
    kd: float = 1.0
    kf: float = 100.0
    muf: float = 0.5
    gravity: tuple = GRAVITY
    ground: bool = True
    plane: tuple = GROUND
    dt: float = 1.0 / 600.0
    s0: np.ndarray = field(default_factory=lambda: np.array([0, 0, 0, 1, 0, 0, 0, 0, 0, 0, 0, 0, 0], float))

    @property
    def nv(self):
        return len(self.verts)

    def contact(self):
        return np.array([self.ke, self.kd, self.kf, self.muf], np.float64)

    def round_to(self, dtype):
        import copy
        b = copy.copy(self)
        r = lambda a: np.asarray(a, dtype).astype(np.float64)
        b.verts, b.inertia, b.s0 = r(self.verts), r(self.inertia), r(self.s0)
        for k in ("mass", "ke", "kd", "kf", "muf", "dt"):
            setattr(b, k, float(np.asarray(getattr(self, k), dtype)))
        b.gravity = tuple(float(np.asarray(g, dtype)) for g in self.gravity)
        b.plane = tuple(float(np.asarray(g, dtype)) for g in self.plane)
        return b


def _box_surface(a, b, c, n):
    """Vertices on the surface of an a x b x c box (n points per edge), centred."""
    t = np.linspace(-0.5, 0.5, n)
    g = np.array(np.meshgrid(t, t, t, indexing="ij")).reshape(3, -1).T
    on = (np.abs(g) == 0.5).any(1)
    return g[on] * np.array([a, b, c])


def _cylinder_surface(r, h, n_around, n_rings):
    """Vertices on two rims and intermediate rings of a cylinder along y, plus the
    two cap centres, centred."""
    th = 2 * np.pi * np.arange(n_around) / n_around
    ys = np.linspace(-h / 2, h / 2, n_rings)
    pts = [np.stack([r * np.cos(th), np.full(n_around, y), r * np.sin(th)], 1) for y in ys]
    return np.concatenate(pts + [np.array([[0, -h / 2, 0], [0, h / 2, 0]])])


def _sphere_surface(r, n_lat, n_lon):
    """Latitude-longitude vertices of a sphere plus its poles."""
    lat = np.pi * (np.arange(1, n_lat + 1) / (n_lat + 1) - 0.5)
    lon = 2 * np.pi * np.arange(n_lon) / n_lon
    la, lo = np.meshgrid(lat, lon, indexing="ij")
    pts = np.stack([r * np.cos(la) * np.cos(lo), r * np.sin(la), r * np.cos(la) * np.sin(lo)], -1).reshape(-1, 3)
    return np.concatenate([pts, [[0, -r, 0], [0, r, 0]]])


def _random_quaternion(rng):
    q = rng.normal(size=4)
    return q / np.linalg.norm(q)


def rigid_body(seed: int, kind: str | None = None):
    """A seeded rigid body for the rigid parameter-estimation task (Sec. 5.1 rigid;
    App. "Dataset": primitive shapes of at most 250 vertices with sampled sizes,
    densities, contact parameters, poses and initial velocities).  Shapes: box,
    cylinder or sphere (solid, uniform density; analytic inertia), scale U(0.5, 1.5)
    m per axis, density U(2, 12) kg/m^3, k_e U(100, 500), k_d U(0, 5) (the paper's
    1 .. 500 range for k_d is not stable with explicit steps at these masses),
    k_f U(1, 500), mu_f U(0.2, 1.0); start 0.2 .. 1 m above the ground in a random
    orientation with v0 ~ U(-2, 2)^3 (plus 1 m/s downwards) and omega0 ~ U(-3, 3)^3;
    gravity, dt = 1/600."""
    rng = np.random.default_rng(seed)
    kind = kind or ["box", "cylinder", "sphere"][int(rng.integers(3))]
    rho = rng.uniform(2.0, 12.0)
    if kind == "box":
        a, b, c = rng.uniform(0.5, 1.5, 3)
        verts = _box_surface(a, b, c, int(rng.integers(2, 7)))
        m = rho * a * b * c
        inertia = np.array([m * (b * b + c * c) / 12, m * (a * a + c * c) / 12, m * (a * a + b * b) / 12, 0, 0, 0])
    elif kind == "cylinder":
        r, h = rng.uniform(0.25, 0.75), rng.uniform(0.5, 1.5)
        verts = _cylinder_surface(r, h, int(rng.integers(8, 33)), int(rng.integers(2, 7)))
        m = rho * np.pi * r * r * h
        inertia = np.array([m * (3 * r * r + h * h) / 12, m * r * r / 2, m * (3 * r * r + h * h) / 12, 0, 0, 0])
    else:
        r = rng.uniform(0.25, 0.75)
        verts = _sphere_surface(r, int(rng.integers(4, 12)), int(rng.integers(6, 20)))
        m = rho * 4 / 3 * np.pi * r ** 3
        inertia = np.array([0.4 * m * r * r] * 3 + [0, 0, 0])
    verts = verts[:250]
    q = _random_quaternion(rng)
    s0 = np.zeros(13)
    s0[3:7] = q
    lowest = -(np.abs(verts).sum(1)).max()  # bound on the lowest point in any orientation
    s0[1] = -lowest + rng.uniform(0.2, 1.0)
    s0[7:10] = rng.uniform(-2, 2, 3) + np.array([0.0, -1.0, 0.0])
    s0[10:13] = rng.uniform(-3, 3, 3)
    return RigidBody(verts=verts, mass=m, inertia=inertia, ke=rng.uniform(100, 500), kd=rng.uniform(0, 5),
                     kf=rng.uniform(1, 500), muf=rng.uniform(0.2, 1.0), s0=s0)


def rigid_batch(seed: int = 80, n: int = 1024):
    """n seeded rigid bodies (box / cylinder / sphere, 8 .. 250 vertices each)."""
    return [rigid_body(seed * 100000 + i) for i in range(n)]
