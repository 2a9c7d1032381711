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
