"""FP64 oracle of the open-loop actuation controller (test infrastructure only).

App. "MPC controller architecture" (used by the control-walker and control-fem
tasks of Sec. 5.3): the simulation time feeds N sinusoids with evenly spaced
phases, a fully connected layer without bias maps them to one value per
actuated element, and a tanh bounds the result.  Reading taken where the paper
is silent: the phases are 2 pi k / N, the time of step t is t * dt (the start of
the step), and an output amplitude `scale` multiplies the tanh (1 = the plain
layer).  Weights are ``W[N, n]``; actuation rows are ``act[T, n]`` (row t drives
step t0 + t).  Plain numpy in float64; nothing here is shared with the HIP path.
"""
from __future__ import annotations

import numpy as np


def signals(n_signals, omega, dt, t0, n_steps):
    """s[t, k] = sin(omega (t0 + t) dt + 2 pi k / N): the controller's inputs."""
    tau = (t0 + np.arange(n_steps, dtype=np.float64))[:, None] * dt
    phase = 2.0 * np.pi * np.arange(n_signals, dtype=np.float64)[None, :] / n_signals
    return np.sin(omega * tau + phase)


def forward(W, omega, dt, t0, n_steps, scale=1.0):
    """act[t, e] = scale tanh(sum_k s[t, k] W[k, e])."""
    W = np.asarray(W, np.float64)
    S = signals(W.shape[0], omega, dt, t0, n_steps)
    return scale * np.tanh(S @ W)


def backward(W, act_grad, omega, dt, t0, scale=1.0):
    """Gradient of sum(act_grad * forward(W)) with respect to W: the chain rule through
    the tanh (derivative 1 - tanh^2) and the linear layer (S^T)."""
    W = np.asarray(W, np.float64)
    G = np.asarray(act_grad, np.float64)
    S = signals(W.shape[0], omega, dt, t0, G.shape[0])
    y = np.tanh(S @ W)
    return S.T @ (G * scale * (1.0 - y * y))
