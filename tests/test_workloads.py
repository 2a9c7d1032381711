"""Seeded input generators: exact counts, reproducibility, mesh validity."""
import numpy as np
import pytest

from paper_2104_02646_amd import workloads as W


def test_tiny_cube_counts_and_orientation():
    b = W.tiny_cube(0)
    assert (b.np, b.ne) == (64, 162)
    D = np.stack([b.X[b.tets[:, k]] - b.X[b.tets[:, 0]] for k in (1, 2, 3)], -1)
    assert np.all(np.linalg.det(D) > 0)
    assert abs(b.X[:, 1].min() - 0.02) < 1e-15


def test_cloth_counts():
    c = W.cloth(10)
    assert (c.np, c.nt, c.nh) == (4096, 7938, 11781)
    assert c.pinned.sum() == 2
    # hinges: wings are the third vertices of the two triangles sharing the edge
    tri_sets = {frozenset(t) for t in c.tris.tolist()}
    for w0, w1, e0, e1 in c.hinges[:200].tolist():
        assert frozenset((w0, e0, e1)) in tri_sets and frozenset((w1, e0, e1)) in tri_sets


def test_conforming_tets():
    """Each interior face shared by exactly two tets, boundary faces by one."""
    b = W.batch_body(20003)
    faces = {}
    for t in b.tets.tolist():
        for skip in range(4):
            f = tuple(sorted(t[:skip] + t[skip + 1:]))
            faces[f] = faces.get(f, 0) + 1
    assert set(faces.values()) <= {1, 2}
    D = np.stack([b.X[b.tets[:, k]] - b.X[b.tets[:, 0]] for k in (1, 2, 3)], -1)
    assert np.all(np.linalg.det(D) > 0)


def test_seeded_reproducible():
    a, b = W.batch_body(20007), W.batch_body(20007)
    assert np.array_equal(a.X, b.X) and np.array_equal(a.tets, b.tets) and np.array_equal(a.mu, b.mu)
    c = W.batch_body(20008)
    assert a.ne != c.ne or not np.array_equal(a.mu, c.mu)


@pytest.mark.parametrize("seed", range(20000, 20010))
def test_batch_body_size_range(seed):
    b = W.batch_body(seed)
    assert 400 <= b.ne <= 24000


def test_serving_trace():
    tr = W.serving_trace(40, n=400)
    gaps = np.diff([q.arrival for q in tr])
    assert np.all(gaps > 0)
    assert 150 < 1.0 / gaps.mean() < 260
    assert {q.kind for q in tr} == {"tet", "cloth"}
    assert all(50 <= q.steps <= 400 for q in tr)
