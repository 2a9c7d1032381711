"""Pins of the oracle's lift/drag force on cloth triangles (App. A.1 thin shells; the
model is the flat-plate reading of a lift/drag force the paper names without a
formula).

Closed forms (still cloth, motion along the normal, motion in the plane, lift at 45
degrees), exact symmetries (odd in the velocity, covariant under rotation,
invariant under translation), the work done (lift does none, drag dissipates at
the rate k_d A |n.u| |u|^2), the force Jacobian's dot test with velocity
directions, and central differences of a rollout loss for the initial velocity
and both coefficients.
"""
import numpy as np

from helpers import oracle_for
from oracle import oracle as O
from paper_2104_02646_amd import workloads as W

TRI = np.array([[0.0, 0.0, 0.0], [0.6, 0.0, 0.0], [0.1, 0.5, 0.0]])  # area 0.15, normal +z


def total(f):
    return f.sum(0)


def test_still_and_in_plane_motion_feel_no_air():
    assert np.all(O.air_force(TRI, np.zeros((3, 3)), 2.0, 3.0) == 0.0)
    v = np.array([[1.0, 2.0, 0.0], [0.5, -1.0, 0.0], [3.0, 0.0, 0.0]])
    assert np.all(O.air_force(TRI, v, 2.0, 3.0) == 0.0)


def test_motion_along_the_normal_is_pure_quadratic_drag():
    """u = (0, 0, w): F = -k_d A |w| w e_z, split equally over the corners."""
    w = -2.5
    f = O.air_force(TRI, np.tile([0.0, 0.0, w], (3, 1)), 2.0, 3.0)
    A = 0.15
    assert np.allclose(total(f), [0.0, 0.0, -2.0 * A * abs(w) * w], rtol=1e-14, atol=1e-15)
    assert np.allclose(f[0], f[1]) and np.allclose(f[1], f[2])


def test_lift_at_45_degrees():
    """u at 45 degrees to the plate: lift = k_l A |u|^2 / 2, perpendicular to u, in the
    plane of n and u, turning the flow away from the normal side it hits."""
    A, kl = 0.15, 3.0
    u = np.array([1.0, 0.0, -1.0]) * 2.0  # |u|^2 = 8, n.u = -2
    lift = total(O.air_force(TRI, np.tile(u, (3, 1)), 0.0, kl))
    assert abs(np.linalg.norm(lift) - 0.5 * kl * A * 8.0) < 1e-13
    assert abs(lift @ u) < 1e-13
    assert abs(lift[1]) < 1e-15
    assert lift[2] > 0  # the plate hit from above (n.u < 0) is pushed up


def test_odd_in_velocity_and_power():
    rng = np.random.default_rng(0)
    for _ in range(20):
        x = rng.normal(size=(3, 3))
        v = rng.normal(size=(3, 3))
        kd, kl = rng.uniform(0.5, 3.0, 2)
        f = O.air_force(x, v, kd, kl)
        assert np.array_equal(O.air_force(x, -v, kd, kl), -f)
        u = v.mean(0)
        N = np.cross(x[1] - x[0], x[2] - x[0])
        A = 0.5 * np.linalg.norm(N)
        s = N @ u / np.linalg.norm(N)
        # lift does no work; drag removes k_d A |s| |u|^2
        assert abs(total(f) @ u + kd * A * abs(s) * (u @ u)) < 1e-12 * kd * A * (u @ u) * np.linalg.norm(u)
        assert abs(total(O.air_force(x, v, 0.0, kl)) @ u) < 1e-12 * kl * A * np.linalg.norm(u) ** 3


def test_rotation_covariance_and_translation_invariance():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(3, 3))
    v = rng.normal(size=(3, 3))
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    f = O.air_force(x, v, 1.3, 0.7)
    assert np.allclose(O.air_force(x @ Q.T, v @ Q.T, 1.3, 0.7), f @ Q.T, rtol=1e-12, atol=1e-13)
    assert np.allclose(O.air_force(x + [3.0, -2.0, 5.0], v, 1.3, 0.7), f, rtol=1e-12, atol=1e-13)
    # reversing the winding flips n but not the force
    assert np.allclose(O.air_force(x[[0, 2, 1]], v[[0, 2, 1]], 1.3, 0.7), f[[0, 2, 1]], rtol=1e-12, atol=1e-13)


def _air_cloth():
    return W.control_cloth(61, n=6)


def test_force_adjoint_dot_test_with_air(oracle_lib):
    """<fbar, J d> = <J^T fbar, d> for position, velocity and coefficient directions
    with the air force on; J d along velocities matches central differences."""
    body = _air_cloth()
    orc = oracle_for(oracle_lib, body)
    rng = np.random.default_rng(2)
    p = body.params()
    x = body.X + rng.normal(0, 0.01, body.X.shape)
    v = body.v0 + rng.normal(0, 0.5, body.X.shape)
    dx, dv = rng.normal(size=x.shape), rng.normal(size=x.shape)
    dp = {"ktri": rng.normal(size=body.nt), "kb": rng.normal(), "kdrag": rng.normal(), "klift": rng.normal(),
          "mass": np.zeros(body.np)}
    jd = orc.force_jvp(p, dp, x, v, dx, dv)
    fbar = rng.normal(size=x.shape)
    xb, vb, g = orc.force_vjp(p, x, v, fbar, want=("ktri",))
    lhs = (fbar * jd).sum()
    rhs = (xb * dx).sum() + (vb * dv).sum() + g["ktri"] @ dp["ktri"] + g["kb"] * dp["kb"] \
        + g["air"] @ np.array([dp["kdrag"], dp["klift"]])
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)
    assert np.abs(vb).max() > 0  # the velocity adjoint is not vacuous
    # (h = 1e-4: the membrane forces, up to ~800 N here and independent of v, put
    # eps |f| / h of cancellation into smaller steps)
    h = 1e-4
    fd = (orc.forces(p, x, v + h * dv) - orc.forces(p, x, v - h * dv)) / (2 * h)
    jv = orc.force_jvp(p, {"mass": np.zeros(body.np)}, x, v, np.zeros_like(x), dv)
    assert np.linalg.norm(fd - jv) < 1e-7 * np.linalg.norm(jv)


def test_rollout_gradients_with_air_central_fd(oracle_lib):
    """Control-cloth gradient: d loss / d v0 (the optimised quantity), and d loss /
    d k_drag, d k_lift, against central differences of a 60-step rollout."""
    body = _air_cloth()
    orc = oracle_for(oracle_lib, body)
    rng = np.random.default_rng(3)
    T = 60
    p = body.params()
    target = body.x0 + np.array([0.2, 0.1, 0.0]) + rng.normal(0, 0.01, body.X.shape)
    L, g, _, _ = orc.loss_and_grad(p, body.x0, body.v0, T, target, want=("ktri",))

    def loss(pp, v0):
        xT, _ = orc.rollout_final(pp, body.x0, v0, T)
        return orc.loss(xT, target)
    d = rng.normal(size=body.v0.shape)
    h = 1e-6
    num = (loss(p, body.v0 + h * d) - loss(p, body.v0 - h * d)) / (2 * h)
    assert abs(num - (g["v0"] * d).sum()) < 1e-6 * abs(num)
    for k, name in enumerate(("kdrag", "klift")):
        hp = 1e-4 * p[name]  # the loss moves by ~1e-11 per 1e-6 here: a larger step beats its rounding
        num = (loss(dict(p, **{name: p[name] + hp}), body.v0) - loss(dict(p, **{name: p[name] - hp}), body.v0)) / (2 * hp)
        assert abs(num - g["air"][k]) < 1e-6 * abs(num), (name, num, g["air"][k])
    # the air force matters here: without it the cloth ends elsewhere
    x_air, _ = orc.rollout_final(p, body.x0, body.v0, T)
    x_no, _ = oracle_for(oracle_lib, body.with_params(air=False)).rollout_final(p, body.x0, body.v0, T)
    assert np.abs(x_air - x_no).max() > 1e-3
