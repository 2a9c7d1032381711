"""Pins of the FP64 controller oracle (App. "MPC controller architecture").

Values fixed by trigonometry (the phase grid at t = 0, sums over evenly spaced
phases, periodicity in time), properties of tanh (zero, odd symmetry,
saturation, bound), the backward against central differences of the forward,
and the whole control-task gradient (controller -> per-step actuation ->
rollout -> loss) against central differences of the oracle rollout.
"""
import numpy as np

from helpers import oracle_for
from oracle import controller as OC
from paper_2104_02646_amd import workloads as W


def test_signal_phase_grid_at_time_zero():
    """At t = 0 the N signals are sin(2 pi k / N): for N = 4 exactly 0, 1, 0, -1;
    for N = 8 the values are multiples of sqrt(2)/2."""
    s4 = OC.signals(4, 3.0, 0.01, 0, 1)[0]
    assert np.allclose(s4, [0.0, 1.0, 0.0, -1.0], atol=1e-15)
    r = np.sqrt(0.5)
    s8 = OC.signals(8, 3.0, 0.01, 0, 1)[0]
    assert np.allclose(s8, [0, r, 1, r, 0, -r, -1, -r], atol=1e-15)


def test_signal_sums_over_evenly_spaced_phases():
    """For N >= 2, sum_k sin(x + 2 pi k / N) = 0 at every x, and for N >= 3
    sum_k sin^2(x + 2 pi k / N) = N / 2: a wrong phase spacing breaks both."""
    for n in (2, 3, 5, 8, 16):
        S = OC.signals(n, 7.3, 1e-3, 11, 50)
        assert np.abs(S.sum(1)).max() < 1e-13
        if n >= 3:
            assert np.abs((S ** 2).sum(1) - n / 2).max() < 1e-13


def test_signals_periodic_in_time_and_shifted_by_t0():
    """omega = 2 pi / (P dt) repeats every P steps; starting at t0 equals dropping
    the first t0 rows."""
    P, dt = 25, 2e-3
    S = OC.signals(8, 2 * np.pi / (P * dt), dt, 0, 3 * P)
    assert np.abs(S[P:] - S[:-P]).max() < 1e-12
    S7 = OC.signals(8, 5.0, dt, 7, 30)
    assert np.array_equal(S7, OC.signals(8, 5.0, dt, 0, 37)[7:])


def test_forward_tanh_properties():
    """Zero weights give zero actuation; the layer is odd in W; large weights
    saturate at +-scale with the sign of the pre-activation; |act| <= scale."""
    rng = np.random.default_rng(0)
    Wt = rng.normal(0, 1.0, (8, 40))
    assert np.all(OC.forward(np.zeros((8, 40)), 3.0, 1e-3, 0, 20, scale=0.3) == 0)
    a = OC.forward(Wt, 3.0, 1e-3, 5, 20, scale=0.3)
    assert np.array_equal(OC.forward(-Wt, 3.0, 1e-3, 5, 20, scale=0.3), -a)
    assert np.abs(a).max() <= 0.3
    big = OC.forward(1e4 * Wt, 3.0, 1e-3, 5, 20, scale=0.3)
    z = OC.signals(8, 3.0, 1e-3, 5, 20) @ Wt
    assert np.allclose(big[np.abs(z) > 1e-2], 0.3 * np.sign(z[np.abs(z) > 1e-2]), atol=1e-12)


def test_backward_against_central_differences():
    """<G, d act> along a random weight direction, by central differences of the
    forward, equals <backward(G), dW>."""
    rng = np.random.default_rng(1)
    Wt = rng.normal(0, 0.7, (6, 30))
    G = rng.normal(size=(45, 30))
    dW = rng.normal(size=Wt.shape)
    h = 1e-6
    num = ((G * OC.forward(Wt + h * dW, 4.0, 2e-3, 3, 45, 0.25)).sum()
           - (G * OC.forward(Wt - h * dW, 4.0, 2e-3, 3, 45, 0.25)).sum()) / (2 * h)
    ana = (OC.backward(Wt, G, 4.0, 2e-3, 3, 0.25) * dW).sum()
    assert abs(num - ana) < 1e-8 * abs(ana)


def test_control_task_gradient_central_fd(oracle_lib):
    """Walker, 40 steps: L(W) = loss(rollout with act rows = controller(W)).  The chain
    controller backward o (per-step actuation gradients from the step adjoint) equals
    central differences of L along a random weight direction."""
    body = W.walker()
    orc = oracle_for(oracle_lib, body)
    T, omega, scale = 40, 2 * np.pi * 4.0, 0.2
    Wt = W.controller_weights(3, 8, body.ne)
    rng = np.random.default_rng(4)
    target = body.X + np.array([0.01, 0.0, 0.0]) + rng.normal(0, 0.001, body.X.shape)
    p = body.params()

    def loss_of(Wm, grad=False):
        act = OC.forward(Wm, omega, body.dt, 0, T, scale)
        xs, vs = [body.x0], [body.v0]
        for t in range(T):
            q = dict(p, act=act[t])
            xn, vn = orc.step(q, xs[-1], vs[-1])
            xs.append(xn)
            vs.append(vn)
        L, xb = orc.loss(xs[-1], target, with_grad=True)
        if not grad:
            return L
        vb = np.zeros_like(xb)
        gact = np.zeros_like(act)
        for t in range(T - 1, -1, -1):
            xb, vb, g = orc.step_vjp(dict(p, act=act[t]), xs[t], vs[t], xb, vb, want=("act",))
            gact[t] = g["act"]
        return L, OC.backward(Wm, gact, omega, body.dt, 0, scale)

    L, gW = loss_of(Wt, True)
    d = rng.normal(size=Wt.shape)
    h = 1e-6
    num = (loss_of(Wt + h * d) - loss_of(Wt - h * d)) / (2 * h)
    ana = float((gW * d).sum())
    assert abs(num - ana) <= 1e-5 * abs(ana), (num, ana)
