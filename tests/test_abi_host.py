"""Host-only checks of the C-ABI library (no GPU needed): it loads, exports every
function the header declares, and its planner validates descriptions."""
import os
import re

import numpy as np
import pytest

from paper_2104_02646_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def gs():
    from paper_2104_02646_amd import gsim
    if not os.path.exists(gsim.LIB_PATH):
        from paper_2104_02646_amd import build
        build.build()
    gsim.load()
    return gsim


def declared_functions():
    src = open(os.path.join(ROOT, "include", "gsim.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gsim_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(gs):
    import ctypes
    lib = ctypes.CDLL(gs.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(gs.ABI_SYMBOLS)


def test_version(gs):
    import ctypes
    a, b = ctypes.c_int(), ctypes.c_int()
    assert gs.load().gsim_version(ctypes.byref(a), ctypes.byref(b)) == 0
    assert (a.value, b.value) >= (0, 1)


def test_plan_counts_and_sizes(gs):
    p = gs.Plan([W.tiny_cube(0), W.cloth(1, n=8)])
    assert (p.np, p.ne, p.nt, p.nh, p.nb) == (128, 162, 98, 133, 2)
    w1, c1, s1 = p.sizes(100, 10)
    w2, c2, s2 = p.sizes(400, 10)
    assert w2 > w1 and c2 > c1 and s2 == s1
    assert c1 == 10 * 6 * 128 * 4 and s1 == 10 * 6 * 128 * 4
    p64 = gs.Plan([W.tiny_cube(0)], dtype=__import__("torch").float64)
    assert p64.sizes(100, 10)[1] == 10 * 6 * 64 * 8


def _expect(gs, code, bodies):
    with pytest.raises(gs.GsimError) as ei:
        gs.Plan(bodies)
    assert ei.value.code == code, str(ei.value)


def test_rejects_out_of_range_index(gs):
    b = W.tiny_cube(0)
    b.tets = b.tets.copy()
    b.tets[5, 1] = 64
    _expect(gs, gs.GSIM_E_TOPOLOGY, [b])


def test_rejects_element_crossing_bodies(gs):
    a, b = W.tiny_cube(0), W.tiny_cube(1)
    pk = gs.pack([a, b])
    # an element of body 1 that points into body 0 after packing
    b2 = W.tiny_cube(1)
    b2.tets = b2.tets.copy()
    b2.tets[0, 0] = -3
    _expect(gs, gs.GSIM_E_TOPOLOGY, [a, b2])
    assert pk.poff[-1] == 128


def test_rejects_repeated_corner(gs):
    """Every element's corners are distinct particles (tet, triangle, hinge)."""
    b = W.tiny_cube(0)
    b.tets = b.tets.copy()
    b.tets[3, 2] = b.tets[3, 0]
    _expect(gs, gs.GSIM_E_TOPOLOGY, [b])
    c = W.cloth(1, n=6)
    c.hinges = c.hinges.copy()
    c.hinges[4, 1] = c.hinges[4, 0]   # both wing tips the same particle: not caught by geometry
    _expect(gs, gs.GSIM_E_TOPOLOGY, [c])


def test_rejects_degenerate_tet(gs):
    b = W.tiny_cube(0)
    b.X = b.X.copy()
    t = b.tets[7]
    b.X[t[3]] = b.X[t[0]] + 0.5 * (b.X[t[1]] - b.X[t[0]])  # collapse onto an edge
    _expect(gs, gs.GSIM_E_DEGENERATE, [b])


def test_rejects_nonfinite_and_bad_dt(gs):
    b = W.tiny_cube(0)
    b.X = b.X.copy()
    b.X[3, 1] = np.nan
    _expect(gs, gs.GSIM_E_NONFINITE, [b])
    c = W.tiny_cube(0)
    c.dt = 0.0
    _expect(gs, gs.GSIM_E_INVALID, [c])


def test_orients_negative_tets(gs):
    """A tet given with negative orientation is accepted (corners reordered)."""
    b = W.tiny_cube(0)
    b.tets = b.tets.copy()
    b.tets[:, [1, 2]] = b.tets[:, [2, 1]]
    p = gs.Plan([b])
    assert p.ne == 162


@pytest.mark.parametrize("which", ["batch", "cloth"])
def test_colouring_classes_are_particle_disjoint(gs, which):
    """Fused-path colouring: a permutation of each kind's elements; within every colour
    class of every body no two elements share a particle."""
    bodies = [W.batch_body(20000 + i, lo=500, hi=3000) for i in range(3)] if which == "batch" else \
        [W.cloth(3, n=20), W.cloth(4, n=9)]
    p = gs.Plan(bodies)
    pk = gs.pack(bodies)
    for kind, idx in ((0, pk.tets), (1, pk.tris), (2, pk.hinges)):
        n = len(idx)
        if n == 0:
            continue
        order, bounds = p.colouring(kind)
        assert np.array_equal(np.sort(order), np.arange(n))
        ncol = 0
        for b0, b1 in zip(bounds[:-1], bounds[1:]):
            if b1 < b0:   # next body's list starts
                continue
            cls = idx[order[b0:b1]].ravel()
            assert len(np.unique(cls)) == len(cls), "colour class shares a particle"
            ncol += 1
        assert ncol <= 128 * len(bodies) * 3


@pytest.mark.parametrize("which", ["mixed", "batch", "air"])
def test_element_tiles_and_partials(gs, which):
    """Two-pass element tiles: they partition each body's elements of each kind into
    runs of consecutive elements (at most 256, adjoint LDS within 16384 words); each
    tile's particle list is exactly the sorted set of particles its elements touch;
    corner codes point at the right tile particle and the sorted positions form one
    contiguous run per tile particle, ordered by (element, corner); partial slots
    are a bijection onto the sliced-ELL table (slot = slice base + 64 k + lane,
    k < degree, k increasing in tile order)."""
    bodies = ([W.tiny_cube(0), W.cloth(5, n=30), W.batch_body(20001, lo=700, hi=900)] if which == "mixed" else
              [W.tiny_cube(1), W.control_cloth(62, n=33), W.cloth(6, n=40)] if which == "air" else
              [W.batch_body(20000 + i, lo=3000, hi=20000) for i in range(3)])
    p = gs.Plan(bodies)
    pk = gs.pack(bodies)
    tiles, tp, run, slot = p.tiles()
    base, deg, nslot = p.partials()
    offs = {0: pk.eoff, 1: pk.toff, 2: pk.hoff}
    idxs = {0: pk.tets, 1: pk.tris, 2: pk.hinges}
    codes = {k: p.codes(k) for k in range(3) if len(idxs[k])}
    covered = {k: np.zeros(len(idxs[k]), int) for k in range(3)}
    seen_k = {}
    ends = list(tiles[1:, 4]) + [len(tp)]
    for i, (kind, body, e0, cnt, t0) in enumerate(tiles):
        kind, body, e0, cnt, t0 = map(int, (kind, body, e0, cnt, t0))
        idx, nc = idxs[kind], (3 if kind == 1 else 4)
        assert 1 <= cnt <= 256 and offs[kind][body] <= e0 and e0 + cnt <= offs[kind][body + 1]
        covered[kind][e0:e0 + cnt] += 1
        parts = tp[t0:ends[i]]
        m = len(parts)
        assert np.array_equal(parts, np.unique(idx[e0:e0 + cnt].ravel()))
        air = kind == 1 and bodies[body].air
        # adjoint LDS words: triangles of bodies with air also stage velocities and keep
        # a velocity adjoint per corner
        assert (12 * m + 8 * nc * cnt if air else 8 * m + 4 * nc * cnt) <= 16384
        cd = codes[kind][:, e0:e0 + cnt]
        lj, pos = cd & 0xFFFF, cd >> 16
        assert np.array_equal(parts[lj], idx[e0:e0 + cnt].T)
        assert np.array_equal(np.sort(pos.ravel()), np.arange(nc * cnt))
        r0, rn = run[t0:ends[i]] & 0xFFFF, run[t0:ends[i]] >> 16
        for j in range(m):
            # the run of tile particle j: its corners, in (element, corner) order
            mine = [(l, c) for l in range(cnt) for c in range(nc) if lj[c, l] == j]
            assert rn[j] == len(mine)
            assert [int(pos[c, l]) for l, c in mine] == list(range(r0[j], r0[j] + rn[j]))
        for j, q in enumerate(parts):
            q = int(q)
            b = int(np.searchsorted(pk.poff, q, side="right") - 1)
            li = q - int(pk.poff[b])
            g = int(np.sum([-(-int(pk.poff[r + 1] - pk.poff[r]) // 64) for r in range(b)])) + li // 64
            k, lane = divmod(int(slot[t0 + j]) - int(base[g]), 64)
            assert lane == li % 64 and k == seen_k.get(q, 0) and k < deg[q]
            seen_k[q] = k + 1
    for k in range(3):
        assert (covered[k] == 1).all()
    assert len(set(slot.tolist())) == len(slot) and slot.max() < nslot
    assert all(seen_k.get(q, 0) == deg[q] for q in range(len(deg)))


def test_ctypes_structs_match_header(gs, tmp_path):
    """Every struct the Python binding mirrors has the header's size and field
    offsets (compiled against include/gsim.h with the host C compiler)."""
    import ctypes
    import subprocess
    from paper_2104_02646_amd import serve
    mirrors = {"gsim_model_desc": gs._Desc, "gsim_state": gs._State, "gsim_params": gs._Params,
               "gsim_grads": gs._Grads, "gsim_query": serve._Query, "gsim_result": serve._Result,
               "gsim_controller": gs._Ctrl, "gsim_rigid_desc": gs._RigidDesc, "gsim_rigid_params": gs._RigidParams,
               "gsim_rigid_grads": gs._RigidGrads, "gsim_camera": gs._Camera}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gsim.h"', "int main(void) {"]
    expect = []
    for cname, cls in mirrors.items():
        lines.append('printf("%%zu\\n", sizeof(%s));' % cname)
        expect.append(ctypes.sizeof(cls))
        for fname, _ in cls._fields_:
            lines.append('printf("%%zu\\n", offsetof(%s, %s));' % (cname, fname))
            expect.append(getattr(cls, fname).offset)
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(s) for s in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got == expect


def test_rigid_description_validation(gs):
    """gsim_rigid_sizes validates on the host: vertex counts 1..256 per body,
    finite vertices, dt > 0; the workspace size grows with the vertex count."""
    import ctypes as C
    lib = gs.load()

    def sizes(nv_per_body, verts_fill=0.1, dt=1e-3):
        off = np.cumsum([0] + list(nv_per_body)).astype(np.int64)
        verts = np.full((int(off[-1]), 3), verts_fill, np.float64)
        nb = len(nv_per_body)
        grav = np.zeros((nb, 3))
        dts = np.full(nb, dt)
        d = gs._RigidDesc()
        d.dtype, d.n_bodies = 32, nb
        d.vert_off, d.verts, d.gravity, d.dt = off.ctypes.data, verts.ctypes.data, grav.ctypes.data, dts.ctypes.data
        out = C.c_size_t()
        rc = lib.gsim_rigid_sizes(C.byref(d), C.byref(out))
        return rc, out.value
    rc, small = sizes([8, 250])
    assert rc == 0
    rc, big = sizes([8, 250, 256])
    assert rc == 0 and big > small
    assert sizes([257])[0] == -7          # GSIM_E_UNSUPPORTED
    assert sizes([8], verts_fill=float("nan"))[0] == -6
    assert sizes([8], dt=0.0)[0] == -1


def test_raster_sizes_validation(gs):
    """gsim_raster_sizes validates on the host (dtype, counts, image size) and its
    workspace grows with the triangles and the pixels; FP64 needs more than FP32."""
    import ctypes as C
    lib = gs.load()

    def sizes(dtype, nv, nt, h, w):
        out = C.c_size_t()
        rc = lib.gsim_raster_sizes(dtype, C.c_int64(nv), C.c_int64(nt), h, w, C.byref(out))
        return rc, out.value
    rc, base = sizes(gs.GSIM_F32, 100, 150, 64, 64)
    assert rc == 0 and base > 0 and base % 256 == 0
    assert sizes(gs.GSIM_F32, 100, 1500, 64, 64)[1] > base
    assert sizes(gs.GSIM_F32, 100, 150, 256, 256)[1] > base
    assert sizes(gs.GSIM_F64, 100, 150, 64, 64)[1] > base
    assert sizes(7, 100, 150, 64, 64)[0] == -1         # dtype
    assert sizes(gs.GSIM_F32, 100, 0, 64, 64)[0] == -1  # no triangles
    assert sizes(gs.GSIM_F32, 0, 150, 64, 64)[0] == -1  # no vertices
    assert sizes(gs.GSIM_F32, 100, 150, 0, 64)[0] == -1  # empty image
    assert sizes(gs.GSIM_F32, 100, 150, 1 << 15, 1 << 15)[0] == -1  # image beyond 2^28 pixels
