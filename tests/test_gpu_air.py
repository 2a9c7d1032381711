"""Lift/drag on cloth (control-cloth task, Sec. 5.3) on the HIP path vs the FP64 oracle
(needs an MI355X).

The air force depends on the corner velocities, so its adjoint reaches the velocity
adjoint: the two-pass adjoint keeps a second per-(tile, particle) partial for it.
Cases: one FP64 step and adjoint step (every output, the velocity adjoint above
all); 120-step rollouts of free cloths of 72 and 2048 triangles with the gradient of
the loss with respect to the initial velocity (the quantity the task optimises), in
FP64 and FP32, plain launches and graphs; a batch mixing an air cloth, a cloth
without air and a tet body on two launch lanes (each body as alone); the autograd
Function; the fused path refusing air.
"""
import numpy as np
import pytest

from helpers import oracle_for, perturbed_state, rel
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


def test_fp64_step_and_adjoint_with_air(gs, oracle_lib):
    body = W.control_cloth(70, n=9)
    x, v = perturbed_state(body, 3)
    rng = np.random.default_rng(4)
    xbp, vbp = rng.normal(size=x.shape), rng.normal(size=x.shape)
    orc = oracle_for(oracle_lib, body)
    xo_ref, vo_ref = orc.step(body.params(), x, v)
    xbm_ref, vbm_ref, g_ref = orc.step_vjp(body.params(), x, v, xbp, vbp, want=("ktri", "mass"))
    # the part of the velocity adjoint that the air force contributes
    nb = body.with_params(air=False)
    _, vbm_noair, _ = oracle_for(oracle_lib, nb).step_vjp(nb.params(), x, v, xbp, vbp, want=())
    m = gs.Model([body], torch.float64, max_steps=4, ckpt_every=2)
    p = m.params_from_bodies()
    xs, vs = gs.soa(x, torch.float64), gs.soa(v, torch.float64)
    xo, vo = m.step(p, xs, vs)
    g = m.zero_grads(("ktri", "mass"))
    xbm, vbm = m.step_backward(p, xs, vs, gs.soa(xbp, torch.float64), gs.soa(vbp, torch.float64), g)
    torch.cuda.synchronize()
    assert rel(gs.aos(vo) - v, vo_ref - v) < 1e-11
    assert rel(gs.aos(xbm) - xbp, xbm_ref - xbp) < 1e-10
    assert rel(gs.aos(vbm) - vbm_noair, vbm_ref - vbm_noair) < 1e-10
    assert np.abs(vbm_ref - vbm_noair).max() > 1e-6 * np.abs(vbm_ref).max()
    assert rel(g["ktri"].cpu().numpy(), g_ref["ktri"]) < 1e-10
    assert rel(g["mass"].cpu().numpy(), g_ref["mass"]) < 1e-10


@pytest.mark.parametrize("n,dtype,exec_mode,pos_tol,grad_tol", [
    (7, "f64", 0, 1e-10, 1e-8), (33, "f64", 1, 1e-10, 1e-8), (7, "f32", 1, 1e-4, 1e-3), (33, "f32", 1, 1e-4, 1e-3)])
def test_control_cloth_v0_gradient(gs, oracle_lib, n, dtype, exec_mode, pos_tol, grad_tol):
    T, K = 120, 16
    tdt = torch.float64 if dtype == "f64" else torch.float32
    npdt = np.float64 if dtype == "f64" else np.float32
    body = W.control_cloth(71, n=n)
    if dtype == "f32":
        body = body.round_to(np.float32)
    rng = np.random.default_rng(72)
    target = (body.x0 + np.array([0.3, 0.2, 0.0]) + rng.normal(0, 0.01, body.X.shape)).astype(npdt).astype(np.float64)
    orc = oracle_for(oracle_lib, body)
    L_ref, g_ref, xs, _ = orc.loss_and_grad(body.params(), body.x0, body.v0, T, target, want=("ktri", "mass"))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        m = gs.Model([body], tdt, max_steps=T, ckpt_every=K)
        m.set_exec(exec_mode)
        p = m.params_from_bodies()
        xT, vT = m.rollout(p, gs.soa(body.x0, tdt), gs.soa(body.v0, tdt), T)
        loss, xb, vb = m.loss_mse(xT, gs.soa(target, tdt))
        g = m.zero_grads(("ktri", "mass"))
        xb0, vb0 = m.rollout_backward(p, T, xb, vb, g)
    stream.synchronize()
    errs = {"x": rel(gs.aos(xT), xs[-1]), "v0": rel(gs.aos(vb0), g_ref["v0"]), "x0": rel(gs.aos(xb0), g_ref["x0"]),
            "ktri": rel(g["ktri"].double().cpu().numpy(), g_ref["ktri"]),
            "mass": rel(g["mass"].double().cpu().numpy(), g_ref["mass"])}
    print("control cloth n=%d %s exec %d errors:" % (n, dtype, exec_mode), {k: "%.2e" % v for k, v in errs.items()})
    assert errs["x"] < pos_tol
    for k in ("v0", "x0", "ktri", "mass"):
        assert errs[k] < grad_tol, (k, errs[k])


def test_air_batch_with_lanes_bitwise_as_alone(gs):
    """An air cloth, a cloth without air and a tet body in one model on two lanes: each
    body's state and gradients are bitwise those of the body alone."""
    T, K = 40, 8
    bodies = [W.control_cloth(73, n=20), W.cloth(74, n=16, size=0.5), W.tiny_cube(75)]
    bodies[1].v0 = np.zeros_like(bodies[1].X)

    def run(bs, lanes):
        m = gs.Model(bs, torch.float32, max_steps=T, ckpt_every=K)
        if len(bs) > 1:
            m.set_lanes(lanes)
        p = m.params_from_bodies()
        x0 = gs.soa(np.concatenate([b.x0 for b in bs]))
        v0 = gs.soa(np.concatenate([b.v0 for b in bs]))
        xT, vT = m.rollout(p, x0, v0, T)
        tgt = gs.soa(np.concatenate([b.x0 + 0.05 for b in bs]))
        loss, xb, vb = m.loss_mse(xT, tgt)
        g = m.zero_grads(("ktri", "mass"))
        xb0, vb0 = m.rollout_backward(p, T, xb, vb, g)
        torch.cuda.synchronize()
        return xT.cpu(), vb0.cpu(), g["mass"].cpu()
    xa, va, ma = run(bodies, 2)
    p0 = 0
    for b in bodies:
        xs, vs, ms = run([b], 1)
        assert torch.equal(xa[:, p0:p0 + b.np], xs)
        assert torch.equal(va[:, p0:p0 + b.np], vs)
        assert torch.equal(ma[p0:p0 + b.np], ms)
        p0 += b.np


def test_simrollout_with_air_and_v0(gs, oracle_lib):
    from paper_2104_02646_amd.autograd import rollout
    T = 60
    body = W.control_cloth(76, n=12).round_to(np.float32)
    target = (body.x0 + 0.1).astype(np.float32).astype(np.float64)
    m = gs.Model([body], torch.float32, max_steps=T, ckpt_every=10)
    p = m.params_from_bodies()
    v0 = gs.soa(body.v0).requires_grad_(True)
    xT, _ = rollout(m, p, gs.soa(body.x0), v0, T)
    loss = ((xT - gs.soa(target)) ** 2).sum() / body.np
    loss.backward()
    orc = oracle_for(oracle_lib, body)
    L_ref, g_ref, _, _ = orc.loss_and_grad(body.params(), body.x0, body.v0, T, target, want=())
    assert abs(float(loss.detach()) - L_ref) / L_ref < 1e-4
    assert rel(gs.aos(v0.grad), g_ref["v0"]) < 1e-3


def test_fused_refuses_air(gs):
    m = gs.Model([W.control_cloth(77, n=8)], torch.float32, max_steps=8, ckpt_every=4)
    with pytest.raises(gs.GsimError, match="lift/drag"):
        m.set_exec(gs.EXEC_FUSED)


def test_control_cloth_bench_batch_sampled(gs, oracle_lib):
    """The bench's lift/drag workload in its launch configuration (64 control cloths,
    seeds 900 .. 963, FP32, 100 steps, checkpoints every 10, graph execution on the
    default lanes; target x0 + 0.3 m): four cloths of different sizes against the FP64
    oracle (final positions, loss, initial-velocity, initial-position, stiffness and
    mass gradients)."""
    T, K = 100, 10
    bodies = [W.control_cloth(900 + i).round_to(np.float32) for i in range(64)]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        m = gs.Model(bodies, torch.float32, max_steps=T, ckpt_every=K)
        p = m.params_from_bodies()
        x0 = gs.soa(np.concatenate([b.x0 for b in bodies]))
        v0 = gs.soa(np.concatenate([b.v0 for b in bodies]))
        tgt = np.concatenate([b.x0 + 0.3 for b in bodies]).astype(np.float32)
        xT, vT = m.rollout(p, x0, v0, T)
        loss, xb, vb = m.loss_mse(xT, gs.soa(tgt))
        g = m.zero_grads(("ktri", "mass"))
        xb0, vb0 = m.rollout_backward(p, T, xb, vb, g)
    stream.synchronize()
    po = np.cumsum([0] + [b.np for b in bodies])
    to = np.cumsum([0] + [b.nt for b in bodies])
    xT, xb0, vb0 = gs.aos(xT), gs.aos(xb0), gs.aos(vb0)
    loss, gk, gm = loss.double().cpu().numpy(), g["ktri"].double().cpu().numpy(), g["mass"].double().cpu().numpy()
    sizes = [b.nt for b in bodies]
    picks = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 17, 40})
    worst = {}
    for i in picks:
        b = bodies[i]
        ps, ts = slice(po[i], po[i + 1]), slice(to[i], to[i + 1])
        L, gr, xs, _ = oracle_for(oracle_lib, b).loss_and_grad(b.params(), b.x0, b.v0, T,
                                                             tgt[ps].astype(np.float64), want=("ktri", "mass"))
        errs = {"x": rel(xT[ps], xs[-1]), "loss": abs(loss[i] - L) / L, "v0": rel(vb0[ps], gr["v0"]),
                "x0": rel(xb0[ps], gr["x0"]), "ktri": rel(gk[ts], gr["ktri"]), "mass": rel(gm[ps], gr["mass"])}
        print("control cloth %d (%d triangles):" % (i, b.nt), {k: "%.2e" % v for k, v in errs.items()})
        for k, v in errs.items():
            worst[k] = max(worst.get(k, 0.0), v)
    assert worst["x"] < 1e-4
    for k in ("loss", "v0", "x0", "ktri", "mass"):
        assert worst[k] < 1e-3, (k, worst[k])
