"""Pins of the oracle's element models against mathematics the paper fixes.

Each pin is independent of the formula it checks: energies are differentiated by
central finite differences, rest states and rigid motions must give zero force,
closed forms under uniform scaling come from the scalar energy, translation and
rotation invariance fix the force and torque sums, and the bending direction must
equal the finite-difference gradient of the dihedral angle.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore")


def rand_rot(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q @ np.diag(np.sign(np.diag(r)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def rest_tet(rng):
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float) * 0.05
    return X + rng.normal(0, 0.005, X.shape)


def rest_tri(rng):
    X = np.array([[0, 0, 0], [1, 0, 0], [0.3, 0, 0.9]], float) * 0.05
    return X @ rand_rot(rng).T + rng.normal(0, 0.002, X.shape)


def fd_grad(fun, x, h):
    g = np.zeros_like(x)
    for idx in np.ndindex(x.shape):
        xp = x.copy(); xp[idx] += h
        xm = x.copy(); xm[idx] -= h
        g[idx] = (fun(xp) - fun(xm)) / (2 * h)
    return g


# ---------------------------------------------------------------- tetrahedron

@pytest.mark.parametrize("seed", range(4))
def test_tet_zero_force_at_rest_and_rigid(oracle_lib, seed):
    """App. A.1 stable Neo-Hookean: with alpha = 1 + 3mu/(4lambda) (reading R1) the rest
    state and every rigid motion carry zero force."""
    o = oracle_lib
    rng = np.random.default_rng(seed)
    X = rest_tet(rng)
    mu, lam = rng.uniform(1e4, 1e5, 2)
    f, V = o.tet_force(X, X, mu, lam)
    assert V > 0
    scale = mu * V / 0.05
    assert np.abs(f).max() < 1e-10 * scale
    R = rand_rot(rng)
    x = X @ R.T + rng.normal(0, 1, 3)
    f, _ = o.tet_force(x, X, mu, lam)
    assert np.abs(f).max() < 1e-9 * scale


@pytest.mark.parametrize("seed", range(4))
def test_tet_force_is_negative_energy_gradient(oracle_lib, seed):
    o = oracle_lib
    rng = np.random.default_rng(10 + seed)
    X = rest_tet(rng)
    x = X + rng.normal(0, 0.006, X.shape)
    mu, lam = rng.uniform(1e4, 1e5, 2)
    act = [0.0, 0.1, -0.05, 0.0][seed]
    f, _ = o.tet_force(x, X, mu, lam, act)
    g = fd_grad(lambda y: o.tet_energy(y, X, mu, lam, act), x, 1e-7)
    assert np.linalg.norm(f + g) < 1e-6 * np.linalg.norm(f)


@pytest.mark.parametrize("seed", range(3))
def test_tet_force_and_torque_balance(oracle_lib, seed):
    """Translation / rotation invariance of the energy: sum f = 0, sum x x f = 0."""
    o = oracle_lib
    rng = np.random.default_rng(20 + seed)
    X = rest_tet(rng)
    x = X + rng.normal(0, 0.01, X.shape)
    f, _ = o.tet_force(x, X, 3e4, 7e4, 0.05)
    s = np.abs(f).max()
    assert np.abs(f.sum(0)).max() < 1e-12 * s * 4
    assert np.abs(np.cross(x, f).sum(0)).max() < 1e-12 * s * 4


@pytest.mark.parametrize("s", [0.7, 0.95, 1.0, 1.2, 1.5])
def test_tet_uniform_scaling_closed_form(oracle_lib, s):
    """Under x = s X (F = sI): Ic = 3s^2, J = s^3, cof F = s^2 I, so
    Psi(s) = mu/2 (3s^2-3) + lambda/2 (s^3-alpha)^2 - mu/2 log(3s^2+1), and
    (i) P = [mu s (1 - 1/(3s^2+1)) + lambda (s^3-alpha) s^2] I, f_{1..3} = -V P Dm^-T;
    (ii) the virtual power sum_i f_i . X_i equals -V dPsi/ds."""
    o = oracle_lib
    rng = np.random.default_rng(3)
    X = rest_tet(rng)
    mu, lam = 2e4, 8e4
    alpha = 1 + 0.75 * mu / lam
    f, V = o.tet_force(s * X, X, mu, lam)
    Dm = (X[1:] - X[0]).T
    p = mu * s * (1 - 1 / (3 * s * s + 1)) + lam * (s ** 3 - alpha) * s * s
    H = -V * p * np.linalg.inv(Dm).T
    fscale = abs(p) * V / 0.05 + 1e-30
    assert np.abs(f[1:] - H.T).max() <= 1e-9 * max(fscale, mu * V / 0.05)
    dpsi = 3 * mu * s + 3 * lam * s * s * (s ** 3 - alpha) - 3 * mu * s / (3 * s * s + 1)
    power = (f * X).sum()
    assert abs(power + V * dpsi) <= 1e-9 * V * (mu + lam)


# ---------------------------------------------------------------- membrane

@pytest.mark.parametrize("seed", range(4))
def test_tri_zero_force_rest_rigid(oracle_lib, seed):
    o = oracle_lib
    rng = np.random.default_rng(30 + seed)
    X = rest_tri(rng)
    k = rng.uniform(1e3, 1e4)
    f, A = o.tri_force(X, X, k)
    assert A > 0
    assert np.abs(f).max() < 1e-10 * k * A / 0.05
    x = X @ rand_rot(rng).T + rng.normal(0, 1, 3)
    f, _ = o.tri_force(x, X, k)
    assert np.abs(f).max() < 1e-9 * k * A / 0.05


@pytest.mark.parametrize("seed", range(4))
def test_tri_force_is_negative_energy_gradient(oracle_lib, seed):
    o = oracle_lib
    rng = np.random.default_rng(40 + seed)
    X = rest_tri(rng)
    x = X + rng.normal(0, 0.005, X.shape)
    k = rng.uniform(1e3, 1e4)
    f, _ = o.tri_force(x, X, k)
    g = fd_grad(lambda y: o.tri_energy(y, X, k), x, 1e-7)
    assert np.linalg.norm(f + g) < 1e-6 * np.linalg.norm(f)
    assert np.abs(f.sum(0)).max() < 1e-11 * np.abs(f).max()
    assert np.abs(np.cross(x, f).sum(0)).max() < 1e-11 * np.abs(f).max()


@pytest.mark.parametrize("s", [0.8, 1.0, 1.1, 1.3])
def test_tri_uniform_scaling_closed_form(oracle_lib, s):
    """In-plane scaling x = s X: Ic = 2 s^2, J = s^2; with mu = lambda = k and
    alpha2 = 5/3, Psi2(s) = k/2 (2s^2-2) + k/2 (s^2-5/3)^2 - k/2 log(2s^2+1) and the
    virtual power sum_i f_i . X_i = -A dPsi2/ds."""
    o = oracle_lib
    rng = np.random.default_rng(5)
    X = rest_tri(rng)
    X = X - X[0]
    k = 4e3
    f, A = o.tri_force(s * X, X, k)
    dpsi = 2 * k * s + 2 * k * s * (s * s - 5.0 / 3.0) - 2 * k * s / (2 * s * s + 1)
    assert abs((f * X).sum() + A * dpsi) <= 1e-9 * A * k


# ---------------------------------------------------------------- bending

def folded_hinge(theta, L=1.0, h1=1.0, h2=1.0):
    """Edge from (0,0,0) to (L,0,0); wing 0 at distance h1 in the +z direction; wing 1
    at distance h2 rotated by theta about the edge from the flat position (-z)."""
    x0 = np.array([0.4 * L, 0.0, h1])
    x1 = np.array([0.6 * L, h2 * np.sin(theta), -h2 * np.cos(theta)])
    return np.array([x0, x1, [0.0, 0.0, 0.0], [L, 0.0, 0.0]])


@pytest.mark.parametrize("theta", [0.0, 0.3, -0.5, 1.2])
def test_hinge_angle_brute_force(oracle_lib, theta):
    """The dihedral angle of a hand-built hinge folded by theta has magnitude |theta|
    (0 when flat); the sign flips with the fold direction."""
    o = oracle_lib
    phi = o.hinge_angle(folded_hinge(theta))
    assert abs(abs(phi) - abs(theta)) < 1e-12
    if theta != 0:
        assert np.sign(o.hinge_angle(folded_hinge(-theta))) == -np.sign(phi)


@pytest.mark.parametrize("theta", [0.2, -0.7, 1.0])
def test_hinge_force_magnitude_hand_built(oracle_lib, theta):
    """Two wings of height 1 on a unit edge: |N1| = |N2| = 1, s = 1/2, |u0| = 1, so
    |f0| = k_b |sin(theta/2)| / 2 (App. A.1 bending model, reading R3)."""
    o = oracle_lib
    kb = 3.0
    f = o.hinge_force(folded_hinge(theta), 0.0, kb)
    assert abs(np.linalg.norm(f[0]) - kb * abs(np.sin(theta / 2)) / 2) < 1e-12


def test_hinge_flat_zero_and_actuation(oracle_lib):
    o = oracle_lib
    x = folded_hinge(0.0)
    assert np.abs(o.hinge_force(x, 0.0, 1.0)).max() < 1e-15
    # per-edge actuation alpha moves the rest fold to phi = phi0 - 2 alpha
    xf = folded_hinge(0.4)
    phi = o.hinge_angle(xf)
    assert np.abs(o.hinge_force(xf, 0.0, 1.0, act=-phi / 2)).max() < 1e-14


@pytest.mark.parametrize("seed", range(5))
def test_hinge_direction_is_angle_gradient_and_restoring(oracle_lib, seed):
    """f_i = -k_b s sin((phi-phi0)/2) dphi/dx_i: compare with the FD gradient of the
    dihedral angle; sum f = 0 and zero torque; a small move along f reduces
    |phi - phi0|."""
    o = oracle_lib
    rng = np.random.default_rng(50 + seed)
    x = folded_hinge(rng.uniform(-1, 1), L=rng.uniform(0.5, 2), h1=rng.uniform(0.3, 1), h2=rng.uniform(0.3, 1))
    x = x @ rand_rot(rng).T + rng.normal(0, 0.05, x.shape)
    phi0 = rng.uniform(-0.2, 0.2)
    kb = 2.0
    f = o.hinge_force(x, phi0, kb)
    gphi = fd_grad(o.hinge_angle, x, 1e-6)
    phi = o.hinge_angle(x)
    E = x[3] - x[2]
    N1 = np.cross(x[0] - x[2], x[0] - x[3]); N2 = np.cross(x[1] - x[3], x[1] - x[2])
    s = E @ E / (np.linalg.norm(N1) + np.linalg.norm(N2))
    expect = -kb * s * np.sin((phi - phi0) / 2) * gphi
    assert np.abs(f - expect).max() < 1e-7 * np.abs(f).max()
    assert np.abs(f.sum(0)).max() < 1e-12 * np.abs(f).max() * 10
    assert np.abs(np.cross(x, f).sum(0)).max() < 1e-11 * np.abs(f).max() * 10
    eps = 1e-4 / np.abs(f).max()
    assert abs(o.hinge_angle(x + eps * f) - phi0) < abs(phi - phi0)


# ---------------------------------------------------------------- contact

def test_contact_normal_is_negative_penalty_gradient(oracle_lib):
    """Elastic normal force = -grad of the one-sided potential k_e C^2/2; zero above
    the plane; pushes out along +n (reading R4)."""
    o = oracle_lib
    pl = [0.0, 1.0, 0.0, 0.0]
    ke = 1e4
    for y in (-0.01, -0.002):
        x = np.array([0.3, y, -0.1])
        f = o.contact_force(x, np.zeros(3), pl, ke, 0.0, 100.0, 0.5)
        assert np.allclose(f, [0, -ke * y, 0], rtol=0, atol=1e-12)
    f = o.contact_force(np.array([0, 1e-9, 0]), np.array([3.0, -1, 0]), pl, ke, 10.0, 100.0, 0.5)
    assert np.all(f == 0)
    # tilted plane: force along its unit normal
    n = np.array([0.0, 0.8, 0.6])
    f = o.contact_force(np.array([0.0, -0.01, 0.0]), np.zeros(3), [*n, 0.0], ke, 0, 100, 0.5)
    assert np.allclose(f, ke * 0.008 * n, atol=1e-12)


def test_contact_damping_and_friction_branches(oracle_lib):
    """Relaxed Coulomb (App. A.1, App. B.2): stick gives -k_f u_t; slip gives
    -mu |lambda_n| u_t/|u_t|; the switch is at k_f |u_t| = mu |lambda_n|; k_d adds
    k_d Cdot with Cdot = -n.v."""
    o = oracle_lib
    pl = [0.0, 1.0, 0.0, 0.0]
    ke, kd, kf, muf = 1e4, 0.0, 100.0, 0.5
    x = np.array([0.0, -0.004, 0.0])  # lambda_n = 40
    v_slip = np.array([1.0, 0.0, 0.0])  # k_f |u| = 100 > 20
    f = o.contact_force(x, v_slip, pl, ke, kd, kf, muf)
    assert np.allclose(f, [-muf * 40, 40, 0], atol=1e-12)
    v_stick = np.array([0.1, 0.0, 0.05])  # k_f |u| = 11.2 < 20
    f = o.contact_force(x, v_stick, pl, ke, kd, kf, muf)
    assert np.allclose(f, [-kf * 0.1, 40, -kf * 0.05], atol=1e-12)
    f = o.contact_force(x, np.array([0.0, -0.3, 0.0]), pl, ke, 50.0, kf, muf)
    assert np.allclose(f, [0, 40 + 50 * 0.3, 0], atol=1e-12)
