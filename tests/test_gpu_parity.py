"""HIP path vs the FP64 oracle (needs an MI355X).

FP64 kernels check the algorithm (agreement to ~1e-12); FP32 kernels check the
production precision against the stated tolerances: 1e-4 relative on positions
after 100 steps, 1e-3 relative on parameter gradients.  Inputs are rounded to
FP32 before the oracle sees them, so the errors measure arithmetic only.
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


def np_params(body):
    return body.params()


def grads_to_np(g):
    return {k: v.detach().double().cpu().numpy() for k, v in g.items()}


CASES = ["cube", "mixed", "cloth"]


def make_case(name):
    if name == "cube":
        return W.tiny_cube(3)
    if name == "mixed":
        return mixed_body(1)
    b = W.cloth(12, n=12, size=0.6)
    b.v0 = np.zeros_like(b.X)
    return b


# ----------------------------------------------------------------- one step

@pytest.mark.parametrize("case", CASES)
def test_fp64_step_forces(gs, oracle_lib, case):
    """One FP64 step: the velocity change (dt * acceleration) matches the oracle."""
    body = make_case(case)
    x, v = perturbed_state(body, 7)
    orc = oracle_for(oracle_lib, body)
    xo_ref, vo_ref = orc.step(body.params(), x, v)
    m = gs.Model([body], torch.float64, max_steps=4, ckpt_every=2)
    p = m.params_from_bodies()
    xo, vo = m.step(p, gs.soa(x, torch.float64), gs.soa(v, torch.float64))
    torch.cuda.synchronize()
    dv_ref = vo_ref - v
    assert rel(gs.aos(vo) - v, dv_ref) < 1e-11
    assert rel(gs.aos(xo), xo_ref) < 1e-14


@pytest.mark.parametrize("case", CASES)
def test_fp64_step_backward(gs, oracle_lib, case):
    """One FP64 adjoint step against the oracle's dual-number adjoint, every output."""
    body = make_case(case)
    x, v = perturbed_state(body, 8)
    rng = np.random.default_rng(9)
    xbp, vbp = rng.normal(size=x.shape), rng.normal(size=x.shape)
    orc = oracle_for(oracle_lib, body)
    xbm_ref, vbm_ref, g_ref = orc.step_vjp(body.params(), x, v, xbp, vbp, want=("mu", "lam", "ktri", "mass"))
    m = gs.Model([body], torch.float64, max_steps=4, ckpt_every=2)
    p = m.params_from_bodies()
    g = m.zero_grads()
    xbm, vbm = m.step_backward(p, gs.soa(x, torch.float64), gs.soa(v, torch.float64),
                               gs.soa(xbp, torch.float64), gs.soa(vbp, torch.float64), g)
    torch.cuda.synchronize()
    g = grads_to_np(g)
    assert rel(gs.aos(xbm), xbm_ref) < 1e-11
    assert rel(gs.aos(vbm), vbm_ref) < 1e-11
    assert rel(gs.aos(xbm) - xbp, xbm_ref - xbp) < 1e-10  # the force-Jacobian part alone
    assert rel(g["mass"], g_ref["mass"]) < 1e-10
    if body.ne:
        assert rel(g["mu"], g_ref["mu"]) < 1e-10
        assert rel(g["lam"], g_ref["lam"]) < 1e-10
    if body.nt:
        assert rel(g["ktri"], g_ref["ktri"]) < 1e-10
    if body.ground:
        assert rel(g["contact"][0], g_ref["contact"]) < 1e-10


# -------------------------------------------------------------- rollouts

def _system_id_target(o, body, T):
    """Target = oracle final positions under an independent parameter draw (seed+1)."""
    if body.ne:
        star = W.redraw_tet_params(body, 1)
    else:
        star = W.redraw_cloth_params(body, 11)
    orc = oracle_for(o, star)
    xT, _ = orc.rollout_final(star.params(), star.x0, star.v0, T)
    return xT


def _gpu_loss_grad(gs, body, T, K, dtype, target, exec_mode=0):
    if exec_mode == 1:  # graphs are captured on a non-default stream
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            out = _gpu_loss_grad(gs, body, T, K, dtype, target, exec_mode=2)
        s.synchronize()
        return out
    m = gs.Model([body], dtype, max_steps=T, ckpt_every=K)
    exec_mode = 1 if exec_mode == 2 else exec_mode
    m.set_exec(exec_mode)
    p = m.params_from_bodies()
    x0, v0 = gs.soa(body.x0, dtype), gs.soa(body.v0, dtype)
    xT, vT = m.rollout(p, x0, v0, T)
    loss, xb, vb = m.loss_mse(xT, gs.soa(target, dtype))
    g = m.zero_grads()
    xb0, vb0 = m.rollout_backward(p, T, xb, vb, g)
    torch.cuda.synchronize()
    return gs.aos(xT), float(loss[0]), grads_to_np(g), gs.aos(xb0), gs.aos(vb0)


@pytest.mark.parametrize("dtype,pos_tol,grad_tol", [("f64", 1e-10, 1e-8), ("f32", 1e-4, 1e-3)])
def test_tiny_cube_rollout_and_gradients(gs, oracle_lib, dtype, pos_tol, grad_tol):
    """162-tet cube, 100 steps with ground contact and friction, gradients w.r.t. mu,
    lambda, mass and mu_f (and the contact stiffness) against the oracle."""
    T, K = 100, 10
    tdt = torch.float64 if dtype == "f64" else torch.float32
    body = W.tiny_cube(0)
    if dtype == "f32":
        body = body.round_to(np.float32)
    target = _system_id_target(oracle_lib, body, T)
    if dtype == "f32":
        target = target.astype(np.float32).astype(np.float64)
    orc = oracle_for(oracle_lib, body)
    L_ref, g_ref, xs, vs = orc.loss_and_grad(body.params(), body.x0, body.v0, T, target, want=("mu", "lam", "mass"))
    xT, L, g, xb0, vb0 = _gpu_loss_grad(gs, body, T, K, tdt, target)
    errs = {"x": rel(xT, xs[-1]), "loss": abs(L - L_ref) / L_ref, "mu": rel(g["mu"], g_ref["mu"]),
            "lam": rel(g["lam"], g_ref["lam"]), "mass": rel(g["mass"], g_ref["mass"]),
            "muf": abs(g["contact"][0, 3] - g_ref["contact"][3]) / abs(g_ref["contact"][3]),
            "ke": abs(g["contact"][0, 0] - g_ref["contact"][0]) / abs(g_ref["contact"][0]),
            "x0": rel(xb0, g_ref["x0"]), "v0": rel(vb0, g_ref["v0"])}
    print("tiny cube %s errors:" % dtype, {k: "%.2e" % v for k, v in errs.items()})
    assert (xs[-1][:, 1] < 0).any(), "contact must be active"
    assert errs["x"] < pos_tol
    for k in ("mu", "lam", "mass", "muf", "ke", "x0", "v0"):
        assert errs[k] < grad_tol, (k, errs[k])


@pytest.mark.parametrize("dtype,pos_tol,grad_tol", [("f64", 1e-10, 1e-8), ("f32", 1e-4, 1e-3)])
def test_mixed_rollout_and_gradients(gs, oracle_lib, dtype, pos_tol, grad_tol):
    """Tets + membrane + bending + pins + contact with damping in one body, 60 steps."""
    T, K = 60, 7
    tdt = torch.float64 if dtype == "f64" else torch.float32
    body = mixed_body(2)
    if dtype == "f32":
        body = body.round_to(np.float32)
    rng = np.random.default_rng(3)
    target = body.X + rng.normal(0, 0.02, body.X.shape)
    if dtype == "f32":
        target = target.astype(np.float32).astype(np.float64)
    orc = oracle_for(oracle_lib, body)
    L_ref, g_ref, xs, vs = orc.loss_and_grad(body.params(), body.x0, body.v0, T, target,
                                             want=("mu", "lam", "ktri", "mass"))
    xT, L, g, xb0, vb0 = _gpu_loss_grad(gs, body, T, K, tdt, target)
    errs = {"x": rel(xT, xs[-1]), "mu": rel(g["mu"], g_ref["mu"]), "lam": rel(g["lam"], g_ref["lam"]),
            "ktri": rel(g["ktri"], g_ref["ktri"]), "mass": rel(g["mass"], g_ref["mass"]),
            "contact": rel(g["contact"][0], g_ref["contact"]), "x0": rel(xb0, g_ref["x0"])}
    print("mixed %s errors:" % dtype, {k: "%.2e" % v for k, v in errs.items()})
    assert errs["x"] < pos_tol
    for k in ("mu", "lam", "ktri", "mass", "contact", "x0"):
        assert errs[k] < grad_tol, (k, errs[k])


def test_cloth_64x64_fp32(gs, oracle_lib):
    """64x64 cloth (7938 triangles, 11781 hinges), two pinned corners, 400 steps, FP32:
    positions after 100 and 400 steps, and the per-triangle stiffness gradient."""
    T = 400
    body = W.cloth(10).round_to(np.float32)
    orc = oracle_for(oracle_lib, body)
    target = _system_id_target(oracle_lib, body, T).astype(np.float32).astype(np.float64)
    L_ref, g_ref, xs, vs = orc.loss_and_grad(body.params(), body.x0, body.v0, T, target, want=("ktri",))
    m = gs.Model([body], torch.float32, max_steps=T, ckpt_every=20)
    p = m.params_from_bodies()
    x0, v0 = gs.soa(body.x0), gs.soa(body.v0)
    x100, _ = m.rollout(p, x0, v0, 100, checkpoint=False)
    xT, L, g, xb0, vb0 = _gpu_loss_grad(gs, body, T, 20, torch.float32, target)
    errs = {"x100": rel(gs.aos(x100), xs[100]), "x400": rel(xT, xs[-1]), "ktri": rel(g["ktri"], g_ref["ktri"]),
            "loss": abs(L - L_ref) / L_ref}
    print("cloth 64x64 f32 errors:", {k: "%.2e" % v for k, v in errs.items()})
    assert errs["x100"] < 1e-4
    assert errs["x400"] < 1e-4
    assert errs["ktri"] < 1e-3


# ------------------------------------------------------ structural checks

def test_batch_alone_equals_in_mix_bitwise(gs):
    """A body's arithmetic and reduction order do not depend on the batch: each body
    stepped alone gives the same bits as inside a multi-body launch."""
    bodies = [W.batch_body(20000 + i, lo=300, hi=3000) for i in range(5)] + [W.cloth(4, n=10, size=0.5)]
    for b in bodies:
        b.target = W.synthetic_target(b, 1)
    T, K = 30, 7
    mb = gs.Model(bodies, torch.float32, max_steps=T, ckpt_every=K)
    p = mb.params_from_bodies()
    x0 = gs.soa(np.concatenate([b.x0 for b in bodies]))
    v0 = gs.soa(np.concatenate([b.v0 for b in bodies]))
    xT, vT = mb.rollout(p, x0, v0, T)
    loss, xb, vb = mb.loss_mse(xT, gs.soa(np.concatenate([b.target for b in bodies])))
    g = mb.zero_grads()
    xb0, vb0 = mb.rollout_backward(p, T, xb, vb, g)
    torch.cuda.synchronize()
    p0 = e0 = t0 = 0
    for i, b in enumerate(bodies):
        m1 = gs.Model([b], torch.float32, max_steps=T, ckpt_every=K)
        p1 = m1.params_from_bodies()
        x1, v1 = m1.rollout(p1, gs.soa(b.x0), gs.soa(b.v0), T)
        l1, xb1, vb1 = m1.loss_mse(x1, gs.soa(b.target))
        g1 = m1.zero_grads()
        xb01, _ = m1.rollout_backward(p1, T, xb1, vb1, g1)
        torch.cuda.synchronize()
        sl = slice(p0, p0 + b.np)
        assert torch.equal(xT[:, sl], x1)
        assert torch.equal(loss[i:i + 1], l1)
        assert torch.equal(xb0[:, sl], xb01)
        assert torch.equal(g["mass"][sl], g1["mass"])
        assert torch.equal(g["contact"][i], g1["contact"][0])
        if b.ne:
            assert torch.equal(g["mu"][e0:e0 + b.ne], g1["mu"])
        if b.nt:
            assert torch.equal(g["ktri"][t0:t0 + b.nt], g1["ktri"])
        p0 += b.np
        e0 += b.ne
        t0 += b.nt


def test_graph_and_launch_shapes_bitwise(gs):
    """hipGraph replay and every launch shape give the same bits as plain launches;
    checkpoint interval does not change the gradient bits (recompute is exact)."""
    body = W.tiny_cube(5)
    target = W.synthetic_target(body, 2)
    ref = _gpu_loss_grad(gs, body, 50, 10, torch.float32, target, exec_mode=0)
    for mode, K in ((1, 10), (0, 1), (0, 50), (1, 7)):
        out = _gpu_loss_grad(gs, body, 50, K, torch.float32, target, exec_mode=mode)
        for a, b in zip(out, ref):
            if isinstance(a, dict):
                for k in a:
                    assert np.array_equal(a[k], b[k]), (mode, K, k)
            else:
                assert np.array_equal(np.asarray(a), np.asarray(b)), (mode, K)
    m = gs.Model([body], torch.float32, max_steps=50, ckpt_every=10)
    p = m.params_from_bodies()
    x0, v0 = gs.soa(body.x0), gs.soa(body.v0)
    base, _ = m.rollout(p, x0, v0, 50)
    for block, items in ((64, 1), (128, 4), (512, 2)):
        m.set_exec(0, block, items)
        x, _ = m.rollout(p, x0, v0, 50)
        assert torch.equal(x, base), (block, items)


def test_repeat_runs_bitwise(gs):
    """Run-to-run determinism (no atomics): two rollouts + backward give identical bits."""
    body = mixed_body(4)
    target = W.synthetic_target(body, 3)
    a = _gpu_loss_grad(gs, body, 40, 8, torch.float32, target)
    b = _gpu_loss_grad(gs, body, 40, 8, torch.float32, target)
    assert np.array_equal(a[0], b[0])
    for k in a[2]:
        assert np.array_equal(a[2][k], b[2][k])

@pytest.mark.parametrize("with_air", [False, True])
def test_lanes_bitwise(gs, with_air):
    """Two, three and four launch lanes (bodies split into concurrently running groups, plain
    and graph execution) and kernel-timing mode (every pass on the caller's stream, with
    events around each launch) give the same bits as one lane; also for a batch with
    a lift/drag cloth, whose tiles run the air kernel variant."""
    bodies = [W.batch_body(21000 + i, lo=300, hi=4000) for i in range(7)] + [W.cloth(8, n=12, size=0.5)]
    if with_air:
        bodies.insert(3, W.control_cloth(9, n=14))
    for b in bodies:
        b.target = W.synthetic_target(b, 2)
    T, K = 24, 5
    stream = torch.cuda.Stream()
    out = {}
    with torch.cuda.stream(stream):
        m = gs.Model(bodies, torch.float32, max_steps=T, ckpt_every=K)
        assert m.get_lanes() == 2
        p = m.params_from_bodies()
        x0 = gs.soa(np.concatenate([b.x0 for b in bodies]))
        v0 = gs.soa(np.concatenate([b.v0 for b in bodies]))
        tgt = gs.soa(np.concatenate([b.target for b in bodies]))
        for lanes in (1, 2, 3, 4):
            for mode in (gs.EXEC_PLAIN, gs.EXEC_GRAPH, "timing"):
                m.set_lanes(lanes)
                m.set_exec(gs.EXEC_PLAIN if mode == "timing" else mode)
                if mode == "timing":
                    m.set_timing()
                for rep in range(2):
                    xT, vT = m.rollout(p, x0, v0, T, stream=stream)
                    loss, xb, vb = m.loss_mse(xT, tgt, stream=stream)
                    g = m.zero_grads()
                    xb0, vb0 = m.rollout_backward(p, T, xb, vb, g, stream=stream)
                    torch.cuda.synchronize()
                    out[(lanes, mode, rep)] = [xT.clone(), loss.clone(), xb0.clone(), vb0.clone()] + \
                        [v.clone() for v in g.values()]
                if mode == "timing":
                    launches = m.read_timing()
                    m.set_timing(())
                    assert launches["element_fwd"][0] > 0
    ref = out[(1, gs.EXEC_PLAIN, 0)]
    for key, val in out.items():
        for a, b in zip(val, ref):
            assert torch.equal(a, b), key
    single = gs.Model([bodies[0]], torch.float32, max_steps=T, ckpt_every=K)
    assert single.get_lanes() == 1
    with pytest.raises(gs.GsimError):
        single.set_lanes(2)


def test_tiny_cube_against_stored_oracle_results(gs):
    """FP64 HIP path against the stored oracle results of tests/golden (written from
    the oracle alone): the tiny cube, 40 steps, loss and the first gradient entries."""
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_golden.json")) as fh:
        ref = json.load(fh)["tiny_cube"]
    b = W.tiny_cube(0)
    xT, L, g, xb0, vb0 = _gpu_loss_grad(gs, b, ref["steps"], 8, torch.float64, W.synthetic_target(b, 1))
    assert abs(L - ref["loss"]) < 1e-12 * abs(ref["loss"])
    assert rel(xT[:4], ref["x_final_first4"]) < 1e-12
    for key, name in (("mu", "grad_mu_first6"), ("lam", "grad_lam_first6"), ("mass", "grad_mass_first6")):
        assert rel(g[key][:6], ref[name]) < 1e-9, key
    assert rel(np.ravel(g["contact"]), ref["grad_contact"]) < 1e-9
    assert rel(xb0[:2], ref["grad_x0_first2"]) < 1e-9 and rel(vb0[:2], ref["grad_v0_first2"]) < 1e-9
