"""Device-side failure detection (needs an MI355X): per-body status flags raised by the
kernels and read by gsim_model_check; the serving engine's per-query status and its
submit-time validation.  Non-finite values never steer an index or a loop bound, so a
NaN or infinite value only propagates through the arithmetic of its own body."""
import numpy as np
import pytest

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


def _bodies():
    return [W.tiny_cube(s).round_to(np.float32) for s in (0, 1, 2)]


def _gradient(gs, bodies, mass, exec_mode, T=60, K=10):
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        m = gs.Model(bodies, torch.float32, max_steps=T, ckpt_every=K)
        m.set_exec(exec_mode)
        if exec_mode != gs.EXEC_FUSED:
            m.set_lanes(2)
        p = m.params_from_bodies()
        p["mass"] = mass.clone()
        x0 = gs.soa(np.concatenate([b.x0 for b in bodies]))
        v0 = gs.soa(np.concatenate([b.v0 for b in bodies]))
        xT, vT = m.rollout(p, x0, v0, T, stream=stream)
        loss, xb, vb = m.loss_mse(xT, x0 + 0.01, stream=stream)
        g = m.zero_grads(("mu", "lam", "mass", "contact"))
        m.rollout_backward(p, T, xb, vb, g, stream=stream)
    torch.cuda.synchronize()
    return m, xT, loss, g, stream


@pytest.mark.parametrize("exec_name", ["graph", "fused"])
def test_nan_mass_flags_its_body_only(gs, exec_name):
    bodies = _bodies()
    ex = {"graph": gs.EXEC_GRAPH, "fused": gs.EXEC_FUSED}[exec_name]
    good = torch.as_tensor(np.concatenate([b.mass for b in bodies]), dtype=torch.float32, device="cuda")
    bad = good.clone()
    bad[bodies[0].np + 5] = float("nan")  # one particle of body 1
    m0, x0, l0, g0, s0 = _gradient(gs, bodies, good, ex)
    # (the landing compresses these soft cubes by about half an element: some tets invert,
    # which is reported in the other bit and is not a failure)
    assert (m0.check(stream=s0) & gs.FLAG_NONFINITE).tolist() == [0, 0, 0]
    m1, x1, l1, g1, s1 = _gradient(gs, bodies, bad, ex)
    with pytest.raises(gs.GsimError) as e:
        m1.check(stream=s1)
    assert e.value.code == gs.GSIM_E_NONFINITE
    assert (e.value.flags & gs.FLAG_NONFINITE).tolist() == [0, 1, 0]
    # the other bodies' results are the same bits
    p0, p1 = bodies[0].np, bodies[0].np + bodies[1].np
    e0, e1 = bodies[0].ne, bodies[0].ne + bodies[1].ne
    for sl_p, sl_e, b in ((slice(0, p0), slice(0, e0), 0), (slice(p1, None), slice(e1, None), 2)):
        assert torch.equal(x1[:, sl_p], x0[:, sl_p])
        assert torch.equal(l1[b], l0[b])
        assert torch.equal(g1["mu"][sl_e], g0["mu"][sl_e]) and torch.equal(g1["lam"][sl_e], g0["lam"][sl_e])
        assert torch.equal(g1["mass"][sl_p], g0["mass"][sl_p]) and torch.equal(g1["contact"][b], g0["contact"][b])
    assert not torch.isfinite(l1[1])
    # cleared flags stay clear on a clean run of the same model
    with pytest.raises(gs.GsimError):
        m1.check(clear=True, stream=s1)
    assert m1.check(stream=s1).tolist() == [0, 0, 0]  # cleared


def test_inverted_tet_is_reported_not_failed(gs):
    """A state with one corner pushed through its tet's opposite face: the step raises
    the body's inversion flag only (the stable energy is defined there)."""
    bodies = _bodies()[:2]
    m = gs.Model(bodies, torch.float32, max_steps=4, ckpt_every=2)
    p = m.params_from_bodies()
    X = np.concatenate([b.X for b in bodies])
    t = bodies[1].tets[0] + bodies[0].np
    x = X.copy()
    # move corner 0 of that tet to the far side of the face (1, 2, 3)
    c = x[t[1:]].mean(0)
    x[t[0]] = c + 1.5 * (c - X[t[0]])
    xo, vo = m.step(p, gs.soa(x), gs.soa(np.zeros_like(x)), 1)
    torch.cuda.synchronize()
    f = m.check()
    assert f.tolist() == [0, gs.FLAG_INVERTED]
    assert torch.isfinite(xo).all()


def test_engine_refuses_invalid_queries(gs):
    from paper_2104_02646_amd import serve as sv
    eng = sv.Engine(pool_bytes=256 << 20, max_live=4)
    b = W.tiny_cube(0).round_to(np.float32)
    b.target = W.synthetic_target(b, 1)
    for field, value, code in (("mass", np.nan, gs.GSIM_E_NONFINITE), ("mass", 0.0, gs.GSIM_E_INVALID),
                               ("mu", -1.0, gs.GSIM_E_INVALID), ("lam", np.inf, gs.GSIM_E_NONFINITE)):
        qb = sv.QueryBuffers(b, 20, 5)
        qb.inp[field][3] = value
        with pytest.raises(gs.GsimError) as e:
            eng.submit(qb)
        assert e.value.code == code, (field, value)
    assert eng.stats()["admitted"] == 0


def test_engine_fails_a_diverging_query_alone(gs):
    """A query whose particles are so light that the first ground contact makes the
    explicit step diverge (mass 1e-9 kg) completes with GSIM_E_NONFINITE and frees its
    slot; the queries beside it give the same bits as alone."""
    from paper_2104_02646_amd import serve as sv
    T, K = 60, 10
    bodies = [W.tiny_cube(s).round_to(np.float32) for s in (0, 1, 2)]
    for i, b in enumerate(bodies):
        b.target = W.synthetic_target(b, 10 + i).astype(np.float32).astype(np.float64)
    bodies[1] = bodies[1].with_params(mass=np.full(bodies[1].np, 1e-9))
    eng = sv.Engine(pool_bytes=512 << 20, max_live=8)
    free0 = eng.stats()["pool_free"]
    qbs = [sv.QueryBuffers(b, T, K) for b in bodies]
    for qb in qbs:
        eng.submit(qb)
    done = eng.run_until_idle()
    assert len(done) == 3 and eng.stats()["pool_free"] == free0  # every slot freed
    st = {qid: qb.status for qid, qb, *_ in done}
    assert [qb.status for qb in qbs] == [gs.GSIM_OK, gs.GSIM_E_NONFINITE, gs.GSIM_OK], st
    for i in (0, 2):
        loss, g = sv.solve_alone(qbs[i])
        assert np.float32(loss) == np.float32(qbs[i].loss)
        for k in ("mu", "lam", "mass", "contact"):
            assert np.array_equal(g[k], qbs[i].out[k]), (i, k)


def test_binding_rejects_mismatched_tensors(gs):
    """The binding checks every caller tensor against what the library will assume (dtype,
    device, contiguity, size) before any launch: a float32 state handed to an FP64 model
    would otherwise be read as doubles past its end."""
    b = W.tiny_cube(0)
    m = gs.Model([b], torch.float64, max_steps=4, ckpt_every=2)
    p = m.params_from_bodies()
    x64, v64 = gs.soa(b.x0, torch.float64), gs.soa(b.v0, torch.float64)
    with pytest.raises(TypeError):
        m.rollout(p, gs.soa(b.x0), v64, 4)
    with pytest.raises(ValueError):
        m.rollout(p, x64[:, :-1].contiguous(), v64, 4)
    with pytest.raises(ValueError):
        m.rollout(p, x64.t().contiguous().t(), v64, 4)
    with pytest.raises(TypeError):
        m.rollout(dict(p, mu=p["mu"].float()), x64, v64, 4)
    with pytest.raises(ValueError):
        m.rollout(dict(p, mass=p["mass"][:-1]), x64, v64, 4)
    with pytest.raises(TypeError):
        m.loss_mse(x64, gs.soa(b.x0))
    g = m.zero_grads(("mu",))
    xT, vT = m.rollout(p, x64, v64, 4)
    loss, xb, vb = m.loss_mse(xT, x64)
    with pytest.raises(TypeError):
        m.rollout_backward(p, 4, xb, vb, {"mu": g["mu"].float()})
    m.rollout_backward(p, 4, xb, vb, g)  # the matching call still runs
    torch.cuda.synchronize()
    assert torch.isfinite(g["mu"]).all()
    rb = [W.rigid_body(700, "box")]
    rm = gs.RigidModel(rb, torch.float64)
    with pytest.raises(TypeError):
        rm.rollout(rm.params_from_bodies(), rm.initial_state().float(), 3)
    r = gs.Renderer(np.array([[0, 1, 2]], np.int32), 3, 8, 8, torch.float32)
    with pytest.raises(ValueError):
        r.forward(torch.zeros(3, 2, device="cuda"), np.eye(3, 4), 1e-3)
