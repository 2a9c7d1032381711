"""Pins of the FP64 rigid-body oracle (App. A.1 "Rigid bodies", "Contact"; App. A.2).

Closed forms: the quaternion's rotation matrix on known rotations; free flight
(x_n = x0 + n dt v0 + g dt^2 n(n+1)/2); spin about a principal axis (omega constant,
each step turns by exactly 2 atan(|omega| dt / 2)); a box resting at its static depth
m g / (4 k_e) stays at rest; the first step of a box sliding at that depth loses
dt mu_f g of speed and gains the friction torque's spin.  Unit quaternions stay unit.
The reverse pass (forward-mode duals, two seed passes) against central differences
of a rollout loss for every parameter and initial-state component.
"""
import numpy as np

from oracle.oracle import RigidOracle

BOX = np.array([[a, b, c] for a in (-0.1, 0.1) for b in (-0.05, 0.05) for c in (-0.08, 0.08)])


def box_inertia(m, hx, hy, hz):
    a, b, c = 2 * hx, 2 * hy, 2 * hz
    return np.array([m * (b * b + c * c) / 12, m * (a * a + c * c) / 12, m * (a * a + b * b) / 12, 0.0, 0.0, 0.0])


def test_rotation_of_known_quaternions():
    """90 degrees about z maps e_x to e_y; 180 about x maps e_y to -e_y; the loss of
    the identity pose against the rotated vertices is 0 only for the same rotation."""
    o = RigidOracle(np.eye(3), gravity=(0, 0, 0), ground=False)
    c45 = np.sqrt(0.5)
    s = np.zeros(13)
    s[3:7] = [c45, 0, 0, c45]
    L, _ = o.loss(s, np.array([[0.0, 1, 0], [-1, 0, 0], [0, 0, 1]]))
    assert L < 1e-30
    s[3:7] = [0, 1, 0, 0]
    L, _ = o.loss(s, np.array([[1.0, 0, 0], [0, -1, 0], [0, 0, -1]]))
    assert L < 1e-30


def test_free_flight_closed_form():
    o = RigidOracle(BOX, ground=False, dt=1.0 / 600)
    s0 = np.zeros(13)
    s0[0:3] = [0.3, 2.0, -0.1]
    s0[3] = 1.0
    s0[7:10] = [1.0, 2.0, -0.5]
    st = o.rollout(s0, 2.0, box_inertia(2.0, 0.1, 0.05, 0.08), [1e4, 0, 100, 0.5], 50)
    n = np.arange(51)[:, None]
    g = np.array([0.0, -9.81, 0.0])
    dt = 1.0 / 600
    assert np.allclose(st[:, 0:3], s0[0:3] + n * dt * s0[7:10] + g * dt * dt * n * (n + 1) / 2, rtol=0, atol=1e-13)
    assert np.allclose(st[:, 7:10], s0[7:10] + n * dt * g, rtol=0, atol=1e-13)


def test_principal_axis_spin():
    """Diagonal inertia, omega along a principal axis: no gyroscopic torque, omega
    constant, and the normalised update turns by 2 atan(|omega| dt / 2) per step."""
    o = RigidOracle(BOX, gravity=(0, 0, 0), ground=False, dt=1e-2)
    for axis in range(3):
        s0 = np.zeros(13)
        s0[3] = 1.0
        s0[10 + axis] = 7.0
        st = o.rollout(s0, 2.0, box_inertia(2.0, 0.1, 0.05, 0.08), [0, 0, 0, 0], 40)
        assert np.all(st[:, 10 + axis] == 7.0)
        half = 40 * np.arctan(7.0 * 1e-2 / 2)
        assert abs(st[-1, 3] - np.cos(half)) < 1e-13 and abs(st[-1, 4 + axis] - np.sin(half)) < 1e-13
        assert np.abs(np.linalg.norm(st[:, 3:7], axis=1) - 1).max() < 1e-14


def test_box_at_static_depth_stays_at_rest():
    m, ke = 2.0, 1e4
    depth = m * 9.81 / (4 * ke)
    o = RigidOracle(BOX, dt=1.0 / 600)
    s0 = np.zeros(13)
    s0[1] = 0.05 - depth
    s0[3] = 1.0
    st = o.rollout(s0, m, box_inertia(m, 0.1, 0.05, 0.08), [ke, 0.0, 100.0, 0.5], 200)
    assert np.abs(st[:, 7:13]).max() < 1e-12
    assert np.abs(st[-1, 0:3] - s0[0:3]).max() < 1e-14


def test_first_step_of_a_sliding_box():
    """At the static depth, sliding along x: every bottom vertex slips, so the step
    removes dt mu_f g of speed, and the friction forces (mu_f m g / 4 each, at
    height -hy below the centre) add the spin dt (hy mu_f m g) / I_zz about -z."""
    m, ke, muf, dt = 2.0, 1e4, 0.5, 1.0 / 600
    depth = m * 9.81 / (4 * ke)
    I = box_inertia(m, 0.1, 0.05, 0.08)
    o = RigidOracle(BOX, dt=dt)
    s0 = np.zeros(13)
    s0[1] = 0.05 - depth
    s0[3] = 1.0
    s0[7] = 1.0
    s1 = o.step(s0, m, I, [ke, 0.0, 100.0, muf])
    assert abs(s1[7] - (1.0 - dt * muf * 9.81)) < 1e-13
    assert abs(s1[8]) < 1e-13
    assert abs(s1[12] - (-dt * 0.05 * muf * m * 9.81 / I[2])) < 1e-12
    assert abs(s1[10]) < 1e-13 and abs(s1[11]) < 1e-13


def _tumbling_box():
    rng = np.random.default_rng(0)
    o = RigidOracle(BOX, dt=1.0 / 600)
    q = rng.normal(size=4)
    s0 = np.zeros(13)
    s0[0:3] = [0.0, 0.13, 0.0]
    s0[3:7] = q / np.linalg.norm(q)
    s0[7:10] = [1.0, -1.5, 0.3]
    s0[10:13] = [2.0, -1.0, 3.0]
    I = box_inertia(2.0, 0.1, 0.05, 0.08) + np.array([0, 0, 0, 0.001, -0.0005, 0.0008])
    return o, s0, 2.0, I, np.array([2e4, 5.0, 100.0, 0.5])


def test_rollout_gradients_central_fd():
    o, s0, m, I, c = _tumbling_box()
    T = 80
    target = BOX + np.array([0.2, 0.05, 0.1])
    L, g, st = o.loss_and_grad(s0, m, I, c, T, target)
    assert (st[:, 1] < 0.13).any()
    contact_steps = sum(1 for s in st if (s[1] - 0.11) < 0)  # the box reaches the ground
    assert contact_steps > 0

    def loss(s0_, m_, I_, c_):
        return o.loss(o.rollout(s0_, m_, I_, c_, T)[-1], target)[0]
    rng = np.random.default_rng(1)
    h = 1e-6
    num = (loss(s0, m + h, I, c) - loss(s0, m - h, I, c)) / (2 * h)
    assert abs(num - g["m"]) < 1e-5 * abs(num)
    for name, vec, key in (("I", I, "I"), ("c", c, "c"), ("s0", s0, "s0")):
        d = rng.normal(size=vec.shape)
        scale = h * np.abs(vec).max()
        args = lambda sgn: {"I": (s0, m, vec + sgn * scale * d, c), "c": (s0, m, I, vec + sgn * scale * d),
                            "s0": (vec + sgn * scale * d, m, I, c)}[name]
        num = (loss(*args(1)) - loss(*args(-1))) / (2 * scale)
        ana = float(g[key] @ d)
        assert abs(num - ana) < 1e-5 * abs(ana), (name, num, ana)
