"""Actuation inputs and their gradients on the HIP path vs the FP64 oracle (needs an MI355X).

Tet actuation shifts the Neo-Hookean rest-volume target (alpha = 1 + 3mu/(4lambda) + a);
hinge actuation shifts each hinge's rest fold (sin((phi - phi0)/2 + a)).  Both are
control inputs whose gradients drive the paper's control experiments (Sec. 5.3,
App. A).  Cases: one FP64 adjoint step; rollouts with one actuation for all steps
on the two-pass path (plain launches and graphs) and the fused path; per-step
actuation ([T, n] arrays) whose per-step gradients come from the oracle's
step adjoint at each step; a batch with two launch lanes; the autograd Function.
"""
import numpy as np
import pytest

from helpers import mixed_body, oracle_for, perturbed_state, rel
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


def _acts(body, seed, T=None, dtype=np.float64):
    """Seeded actuation: tet ~ N(0, 0.02), hinge ~ N(0, 0.1) rad; [n] or [T, n]."""
    rng = np.random.default_rng(seed)
    shape = (lambda n: (n,)) if T is None else (lambda n: (T, n))
    a = {}
    if body.ne:
        a["act"] = rng.normal(0, 0.02, shape(body.ne)).astype(dtype).astype(np.float64)
    if body.nh:
        a["hact"] = rng.normal(0, 0.1, shape(body.nh)).astype(dtype).astype(np.float64)
    return a


def _dev(a, tdt):
    return {k: torch.as_tensor(v).to("cuda", tdt).contiguous() for k, v in a.items()}


def _np(t):
    return t.detach().double().cpu().numpy()


def test_fp64_step_backward_actuation(gs, oracle_lib):
    """One FP64 step and its adjoint with tet and hinge actuation: state, position and
    velocity adjoints and both actuation gradients against the oracle."""
    body = mixed_body(1)
    x, v = perturbed_state(body, 8)
    rng = np.random.default_rng(9)
    xbp, vbp = rng.normal(size=x.shape), rng.normal(size=x.shape)
    acts = _acts(body, 10)
    orc = oracle_for(oracle_lib, body)
    p_ref = dict(body.params(), **acts)
    xo_ref, vo_ref = orc.step(p_ref, x, v)
    xbm_ref, vbm_ref, g_ref = orc.step_vjp(p_ref, x, v, xbp, vbp, want=("act", "hact", "mu"))
    m = gs.Model([body], torch.float64, max_steps=4, ckpt_every=2)
    p = dict(m.params_from_bodies(), **_dev(acts, torch.float64))
    xs, vs = gs.soa(x, torch.float64), gs.soa(v, torch.float64)
    xo, vo = m.step(p, xs, vs)
    g = m.zero_grads(("act", "hact", "mu"))
    xbm, vbm = m.step_backward(p, xs, vs, gs.soa(xbp, torch.float64), gs.soa(vbp, torch.float64), g)
    torch.cuda.synchronize()
    assert rel(gs.aos(vo) - v, vo_ref - v) < 1e-11
    assert rel(gs.aos(xbm) - xbp, xbm_ref - xbp) < 1e-10
    assert rel(gs.aos(vbm), vbm_ref) < 1e-11
    for k in ("act", "hact", "mu"):
        assert rel(_np(g[k]), g_ref[k]) < 1e-10, k
    # actuation changes the step (the test is not vacuous)
    xo0, vo0 = orc.step(body.params(), x, v)
    assert rel(vo_ref - v, vo0 - v) > 1e-4


@pytest.mark.parametrize("dtype,exec_mode,pos_tol,grad_tol", [
    ("f64", 0, 1e-10, 1e-8), ("f64", 2, 1e-10, 1e-8), ("f32", 1, 1e-4, 1e-3), ("f32", 2, 1e-4, 1e-3)])
def test_constant_actuation_rollout_gradients(gs, oracle_lib, dtype, exec_mode, pos_tol, grad_tol):
    """60 steps of the mixed body with one actuation held throughout: final positions,
    loss and the tet/hinge actuation gradients (summed over steps) vs the oracle."""
    T, K = 60, 7
    tdt = torch.float64 if dtype == "f64" else torch.float32
    npdt = np.float64 if dtype == "f64" else np.float32
    body = mixed_body(2)
    if dtype == "f32":
        body = body.round_to(np.float32)
    acts = _acts(body, 20, dtype=npdt)
    rng = np.random.default_rng(3)
    target = (body.X + rng.normal(0, 0.02, body.X.shape)).astype(npdt).astype(np.float64)
    orc = oracle_for(oracle_lib, body)
    L_ref, g_ref, xs, _ = orc.loss_and_grad(dict(body.params(), **acts), body.x0, body.v0, T, target,
                                            want=("act", "hact", "mu"))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        m = gs.Model([body], tdt, max_steps=T, ckpt_every=K)
        m.set_exec(exec_mode)
        p = dict(m.params_from_bodies(), **_dev(acts, tdt))
        xT, vT = m.rollout(p, gs.soa(body.x0, tdt), gs.soa(body.v0, tdt), T)
        loss, xb, vb = m.loss_mse(xT, gs.soa(target, tdt))
        g = m.zero_grads(("act", "hact", "mu"))
        m.rollout_backward(p, T, xb, vb, g)
    stream.synchronize()
    errs = {"x": rel(gs.aos(xT), xs[-1]), "loss": abs(float(loss[0]) - L_ref) / L_ref}
    errs.update({k: rel(_np(g[k]), g_ref[k]) for k in ("act", "hact", "mu")})
    print("constant actuation %s exec %d errors:" % (dtype, exec_mode), {k: "%.2e" % v for k, v in errs.items()})
    assert errs["x"] < pos_tol
    for k in ("act", "hact", "mu"):
        assert errs[k] < grad_tol, (k, errs[k])


def _oracle_per_step(orc, params, acts, x0, v0, target):
    """Rollout whose step t reads row t of each actuation array, the loss, and the
    per-step actuation gradients from the step adjoint at each step."""
    T = len(next(iter(acts.values())))
    xs, vs = [x0], [v0]
    for t in range(T):
        q = dict(params, **{k: a[t] for k, a in acts.items()})
        xn, vn = orc.step(q, xs[-1], vs[-1])
        xs.append(xn)
        vs.append(vn)
    L, xb = orc.loss(xs[-1], target, with_grad=True)
    vb = np.zeros_like(xb)
    per = {k: np.zeros_like(a) for k, a in acts.items()}
    for t in range(T - 1, -1, -1):
        q = dict(params, **{k: a[t] for k, a in acts.items()})
        xb, vb, gt = orc.step_vjp(q, xs[t], vs[t], xb, vb, want=tuple(acts))
        for k in acts:
            per[k][t] = gt[k]
    return xs[-1], L, per, xb


@pytest.mark.parametrize("dtype,exec_mode,pos_tol,grad_tol", [
    ("f64", 0, 1e-10, 1e-8), ("f64", 1, 1e-10, 1e-8), ("f32", 1, 1e-4, 1e-3)])
def test_per_step_actuation_gradients(gs, oracle_lib, dtype, exec_mode, pos_tol, grad_tol):
    """[T, n] actuation (row t drives step t), 30 steps with checkpoints every 7 (so
    segments are recomputed with their own rows): final positions and the [T, n]
    per-step gradients vs the oracle's step-by-step adjoint."""
    T, K = 30, 7
    tdt = torch.float64 if dtype == "f64" else torch.float32
    npdt = np.float64 if dtype == "f64" else np.float32
    body = mixed_body(4)
    if dtype == "f32":
        body = body.round_to(np.float32)
    acts = _acts(body, 30, T=T, dtype=npdt)
    rng = np.random.default_rng(31)
    target = (body.X + rng.normal(0, 0.02, body.X.shape)).astype(npdt).astype(np.float64)
    orc = oracle_for(oracle_lib, body)
    xT_ref, L_ref, per_ref, xb0_ref = _oracle_per_step(orc, body.params(), acts, body.x0, body.v0, target)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        m = gs.Model([body], tdt, max_steps=T, ckpt_every=K)
        m.set_exec(exec_mode)
        p = dict(m.params_from_bodies(), **_dev(acts, tdt))
        xT, vT = m.rollout(p, gs.soa(body.x0, tdt), gs.soa(body.v0, tdt), T)
        loss, xb, vb = m.loss_mse(xT, gs.soa(target, tdt))
        g = m.zero_grads(("act", "hact"), steps=T)
        xb0, _ = m.rollout_backward(p, T, xb, vb, g)
    stream.synchronize()
    errs = {"x": rel(gs.aos(xT), xT_ref), "x0": rel(gs.aos(xb0), xb0_ref)}
    errs.update({k: rel(_np(g[k]), per_ref[k]) for k in ("act", "hact")})
    # every step's row on its own (a row mixed up with another step's fails here)
    errs.update({k + "_row": max(rel(_np(g[k][t]), per_ref[k][t]) for t in range(T)) for k in ("act", "hact")})
    print("per-step actuation %s errors:" % dtype, {k: "%.2e" % v for k, v in errs.items()})
    assert errs["x"] < pos_tol
    for k in ("act", "hact", "x0"):
        assert errs[k] < grad_tol, (k, errs[k])
    for k in ("act_row", "hact_row"):
        assert errs[k] < 10 * grad_tol, (k, errs[k])


def test_per_step_actuation_batch_with_lanes(gs, oracle_lib):
    """Three bodies (tet cube, mixed, cloth) in one model with two launch lanes and
    per-step actuation: each body's slice of the per-step gradients vs the oracle."""
    T, K = 20, 6
    bodies = [W.tiny_cube(5), mixed_body(5), W.cloth(15, n=10, size=0.5)]
    bodies[2].v0 = np.zeros_like(bodies[2].X)
    acts = [_acts(b, 40 + i, T=T) for i, b in enumerate(bodies)]
    rng = np.random.default_rng(41)
    targets = [b.X + rng.normal(0, 0.02, b.X.shape) for b in bodies]
    m = gs.Model(bodies, torch.float64, max_steps=T, ckpt_every=K)
    m.set_lanes(2)
    cat = {}
    for k, n in (("act", "ne"), ("hact", "nh")):
        cat[k] = np.concatenate([a.get(k, np.zeros((T, getattr(b, n)))) for a, b in zip(acts, bodies)], axis=1)
    p = dict(m.params_from_bodies(), **_dev(cat, torch.float64))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        x0 = gs.soa(np.concatenate([b.x0 for b in bodies]), torch.float64)
        v0 = gs.soa(np.concatenate([b.v0 for b in bodies]), torch.float64)
        xT, vT = m.rollout(p, x0, v0, T)
        loss, xb, vb = m.loss_mse(xT, gs.soa(np.concatenate(targets), torch.float64))
        g = m.zero_grads(("act", "hact"), steps=T)
        m.rollout_backward(p, T, xb, vb, g)
    stream.synchronize()
    e0 = h0 = 0
    for b, a, tgt in zip(bodies, acts, targets):
        orc = oracle_for(oracle_lib, b)
        _, _, per, _ = _oracle_per_step(orc, b.params(), a, b.x0, b.v0, tgt)
        if b.ne:
            assert rel(_np(g["act"][:, e0:e0 + b.ne]), per["act"]) < 1e-8
        if b.nh:
            assert rel(_np(g["hact"][:, h0:h0 + b.nh]), per["hact"]) < 1e-8
        e0 += b.ne
        h0 += b.nh


def test_fused_rejects_per_step_actuation(gs):
    """The fused path takes one actuation for all steps: [T, n] arrays are refused
    with an error, before anything is launched."""
    body = mixed_body(1)
    m = gs.Model([body], torch.float32, max_steps=8, ckpt_every=4)
    m.set_exec(gs.EXEC_FUSED)
    p = dict(m.params_from_bodies(), **_dev(_acts(body, 1, T=8), torch.float32))
    with pytest.raises(gs.GsimError, match="strides"):
        m.rollout(p, gs.soa(body.x0), gs.soa(body.v0), 8)
    p["act"] = p["act"][:3]
    m.set_exec(gs.EXEC_GRAPH)
    with pytest.raises(ValueError, match="rows"):
        m.rollout(p, gs.soa(body.x0), gs.soa(body.v0), 8)


def test_simrollout_actuation_grad(gs, oracle_lib):
    """Per-step actuation through the autograd Function: act.grad and hact.grad ([T, n])
    equal the oracle's per-step gradients (FP32, 1e-3)."""
    from paper_2104_02646_amd.autograd import rollout
    T = 24
    body = mixed_body(6).round_to(np.float32)
    acts = _acts(body, 50, T=T, dtype=np.float32)
    rng = np.random.default_rng(51)
    target = (body.X + rng.normal(0, 0.02, body.X.shape)).astype(np.float32).astype(np.float64)
    m = gs.Model([body], torch.float32, max_steps=T, ckpt_every=5)
    p = m.params_from_bodies()
    p.update({k: v.requires_grad_(True) for k, v in _dev(acts, torch.float32).items()})
    xT, _ = rollout(m, p, gs.soa(body.x0), gs.soa(body.v0), T)
    loss = ((xT - gs.soa(target)) ** 2).sum() / body.np
    loss.backward()
    orc = oracle_for(oracle_lib, body)
    _, L_ref, per, _ = _oracle_per_step(orc, body.params(), acts, body.x0, body.v0, target)
    assert abs(float(loss.detach()) - L_ref) / L_ref < 1e-3
    for k in ("act", "hact"):
        assert p[k].grad.shape == (T, per[k].shape[1])
        assert rel(_np(p[k].grad), per[k]) < 1e-3, k


def test_aliased_tet_gradient_buffers_are_refused(gs):
    """The adjoint element pass reads each per-tet gradient before adding to it, so
    the mu, lam and act gradient buffers must be distinct: one buffer passed twice is
    refused before anything is launched."""
    body = mixed_body(1)
    m = gs.Model([body], torch.float32, max_steps=4, ckpt_every=2)
    p = m.params_from_bodies()
    xT, vT = m.rollout(p, gs.soa(body.x0), gs.soa(body.v0), 4)
    xb = torch.ones_like(xT)
    g = m.zero_grads(("mu", "lam"))
    g["lam"] = g["mu"]
    with pytest.raises(gs.GsimError, match="distinct"):
        m.rollout_backward(p, 4, xb, torch.zeros_like(xb), g)
    torch.cuda.synchronize()
    assert not g["mu"].any()
