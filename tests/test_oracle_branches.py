"""Pins of the oracle's contact-branch classifier (App. A.1 "Contact"; R4-R6, R15):
closed-form cases, the tie, and agreement with the branch the oracle's own contact
force takes (its tangential part is -k_f u_t when sticking and -mu_f |lambda_n| u_t/|u_t|
when slipping)."""
import numpy as np

import oracle.oracle as O


def _points(n, ground=True):
    O.build(force=False)
    return O.Oracle(np.zeros((n, 3)), gravity=(0.0, -9.81, 0.0), ground=ground, dt=1e-3)


P = {"mass": None, "ke": 1e4, "kd": 0.0, "kf": 100.0, "muf": 0.5}


def test_closed_form_cases():
    o = _points(4)
    x = np.array([[0.0, 0.01, 0.0], [0.0, -0.01, 0.0], [0.0, -0.01, 0.0], [0.0, -0.01, 0.0]])
    # lambda_n = 1e4 * 0.01 = 100, mu_f lambda_n = 50: stick iff 100 |u_t| <= 50
    v = np.array([[3.0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.2, -1.0, 0.3], [2.0, 0.0, 0.0]])
    p = dict(P, mass=np.ones(4))
    assert o.contact_branches(p, x, v).tolist() == [0, 1, 1, 2]
    # exactly at the tie (|u_t| = 0.5): stick
    assert o.contact_branches(p, x[1:2].repeat(4, 0), np.array([[0.5, 0.0, 0.0]] * 4))[0] == 1
    # no ground: never in contact
    assert not _points(4, ground=False).contact_branches(p, x, v).any()


def test_branches_match_the_contact_force():
    rng = np.random.default_rng(4)
    n = 400
    o = _points(n)
    x = rng.normal(0, 0.01, (n, 3))
    v = rng.normal(0, 0.6, (n, 3))
    p = dict(P, mass=np.ones(n), kd=3.0)
    code = o.contact_branches(p, x, v)
    f = o.forces(p, x, v)
    assert (code == 0).any() and (code == 1).any() and (code == 2).any()
    ut = v.copy()
    ut[:, 1] = 0.0
    s = np.linalg.norm(ut, axis=1)
    lam = p["ke"] * np.maximum(-x[:, 1], 0.0) - p["kd"] * v[:, 1]
    ft = f.copy()
    ft[:, 1] = 0.0
    assert np.all(f[code == 0] == 0.0)
    st, sl = code == 1, code == 2
    np.testing.assert_allclose(ft[st], -p["kf"] * ut[st], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(ft[sl], -(p["muf"] * np.abs(lam[sl]) / s[sl])[:, None] * ut[sl], rtol=1e-12, atol=1e-15)
