"""SimRollout (torch.autograd.Function over the checkpointed HIP adjoint)."""
import numpy as np
import pytest

from helpers import mixed_body, oracle_for, rel
from paper_2104_02646_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2104_02646_amd import gsim
    gsim.load()
    return gsim


def test_simrollout_matches_oracle(gs, oracle_lib):
    """Loss written in torch on the rollout output; backward through SimRollout
    reproduces the oracle's discrete-adjoint gradient for every parameter group."""
    from paper_2104_02646_amd.autograd import rollout
    body = mixed_body(6).round_to(np.float32)
    rng = np.random.default_rng(1)
    target = (body.X + rng.normal(0, 0.02, body.X.shape)).astype(np.float32).astype(np.float64)
    T = 50
    m = gs.Model([body], torch.float32, max_steps=T, ckpt_every=8)
    p = {k: v.clone().requires_grad_(True) for k, v in m.params_from_bodies().items()}
    x0 = gs.soa(body.x0).requires_grad_(True)
    v0 = gs.soa(body.v0).requires_grad_(True)
    xT, vT = rollout(m, p, x0, v0, T)
    loss = ((xT - gs.soa(target)) ** 2).sum() / body.np
    loss.backward()
    orc = oracle_for(oracle_lib, body)
    L_ref, g_ref, _, _ = orc.loss_and_grad(body.params(), body.x0, body.v0, T, target,
                                           want=("mu", "lam", "ktri", "mass"))
    np_ = lambda t: t.detach().double().cpu().numpy()
    errs = {"loss": abs(float(loss) - L_ref) / L_ref, "mu": rel(np_(p["mu"].grad), g_ref["mu"]),
            "lam": rel(np_(p["lam"].grad), g_ref["lam"]), "ktri": rel(np_(p["ktri"].grad), g_ref["ktri"]),
            "mass": rel(np_(p["mass"].grad), g_ref["mass"]), "contact": rel(np_(p["contact"].grad)[0], g_ref["contact"]),
            "x0": rel(gs.aos(x0.grad), g_ref["x0"]), "v0": rel(gs.aos(v0.grad), g_ref["v0"])}
    print("SimRollout errors", {k: "%.2e" % v for k, v in errs.items()})
    for k, v in errs.items():
        assert v < 1e-3, (k, v)


def test_two_rollouts_in_flight(gs):
    """Each forward owns its checkpoints: two rollouts, then both backwards, give the
    same gradients as running them one at a time."""
    from paper_2104_02646_amd.autograd import rollout
    body = W.tiny_cube(2)
    tgt = gs.soa(W.synthetic_target(body, 4))
    m = gs.Model([body], torch.float32, max_steps=40, ckpt_every=10)
    base = m.params_from_bodies()

    def run(scale, do_backward=True):
        p = {k: (v * scale if k == "mu" else v).clone().requires_grad_(True) for k, v in base.items()}
        xT, _ = rollout(m, p, gs.soa(body.x0), gs.soa(body.v0), 40)
        loss = ((xT - tgt) ** 2).sum()
        if do_backward:
            loss.backward()
        return loss, p
    la, pa = run(1.0)
    lb, pb = run(1.3)
    l1, q1 = run(1.0, False)
    l2, q2 = run(1.3, False)
    (l1 + l2).backward()
    assert torch.equal(pa["mu"].grad, q1["mu"].grad)
    assert torch.equal(pb["mu"].grad, q2["mu"].grad)
