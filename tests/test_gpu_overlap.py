"""Overlapped recompute (gsim_model_set_overlap): the checkpointed backward recomputes
segment s - 1 in the same element and particle launches as the adjoint steps of segment
s, alternating two segment buffers.  Each tile's arithmetic is unchanged, so every output
is bitwise that of the backward without overlap: checked over ragged and single-step
segments, one to four launch lanes, plain and graph execution, FP32 and FP64, and a
model with lift/drag (which keeps the sequential backward)."""
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


def gradient(gs, bodies, dtype, T, K, overlap, exec_mode, lanes=1):
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        m = gs.Model(bodies, dtype, max_steps=T, ckpt_every=K, overlap=overlap)
        m.set_exec(exec_mode)
        m.set_lanes(min(lanes, len(bodies)))
        p = m.params_from_bodies()
        x0 = gs.soa(np.concatenate([b.x0 for b in bodies]), dtype=dtype)
        v0 = gs.soa(np.concatenate([b.v0 for b in bodies]), dtype=dtype)
        tg = gs.soa(np.concatenate([W.synthetic_target(b, 40 + i) for i, b in enumerate(bodies)]), dtype=dtype)
        xT, vT = m.rollout(p, x0, v0, T, stream=stream)
        loss, xb, vb = m.loss_mse(xT, tg, stream=stream)
        g = m.zero_grads(("mu", "lam", "ktri", "mass", "contact"))
        out = {}
        for rep in range(2):  # twice: the second call replays a captured graph
            for t in g.values():
                t.zero_()
            xb0, vb0 = m.rollout_backward(p, T, xb, vb, g, stream=stream)
            stream.synchronize()
            out[rep] = {k: v.detach().cpu().numpy().copy() for k, v in g.items()}
            out[rep]["xb0"], out[rep]["vb0"] = xb0.cpu().numpy(), vb0.cpu().numpy()
    for k in out[0]:
        assert np.array_equal(out[0][k], out[1][k]), k
    return out[0]


def batch6(dtype):
    bodies = [W.tiny_cube(3), mixed_body(5), W.cloth(7, n=20, size=0.8)]
    bodies += [W.batch_body(61000 + i, lo=700, hi=3000) for i in range(3)]
    return [b.round_to(np.float32) for b in bodies] if dtype == torch.float32 else bodies


CASES = [  # (bodies, T, K): ragged last segment, one-step segments, one segment, K = T - 1
    ("cube", 40, 7), ("cube", 12, 1), ("cube", 9, 10), ("mixed", 30, 29), ("batch", 40, 7), ("batch", 23, 4),
]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-T%d-K%d" % c)
def test_overlap_bitwise_equals_sequential(gs, case, dtype):
    dt = torch.float32 if dtype == "f32" else torch.float64
    name, T, K = case
    bodies = {"cube": [W.tiny_cube(4)], "mixed": [mixed_body(5)], "batch": batch6(dt)}[name]
    if dt == torch.float32 and name != "batch":
        bodies = [b.round_to(np.float32) for b in bodies]
    for exec_mode in (gs.EXEC_PLAIN, gs.EXEC_GRAPH):
        for lanes in ((1, 2, 4) if name == "batch" else (1,)):
            a = gradient(gs, bodies, dt, T, K, False, exec_mode, lanes)
            b = gradient(gs, bodies, dt, T, K, True, exec_mode, lanes)
            for k in a:
                assert np.array_equal(a[k], b[k]), (k, exec_mode, lanes)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_paired_layout_bitwise_equals_sequential(gs, dtype):
    """A model with at least 2048 element tiles (here 32-element tiles over ~70k tets)
    runs each shared element launch in the paired layout (one workgroup per tile, adjoint
    pass then forward pass): bitwise the sequential backward, on 1 and 4 lanes."""
    dt = torch.float32 if dtype == "f32" else torch.float64
    bodies = [W.batch_body(62000 + i, lo=2000, hi=5000) for i in range(20)]
    if dt == torch.float32:
        bodies = [b.round_to(np.float32) for b in bodies]
    from paper_2104_02646_amd import gsim
    assert len(gsim.Plan(bodies, tile_elems=32).tiles()[0]) >= 2048
    for lanes in (1, 4):
        outs = []
        for overlap in (False, True):
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                m = gs.Model(bodies, dt, max_steps=12, ckpt_every=4, overlap=overlap, tile_elems=32)
                m.set_exec(gs.EXEC_GRAPH)
                m.set_lanes(lanes)
                p = m.params_from_bodies()
                x0 = gs.soa(np.concatenate([b.x0 for b in bodies]), dtype=dt)
                v0 = gs.soa(np.concatenate([b.v0 for b in bodies]), dtype=dt)
                tg = gs.soa(np.concatenate([W.synthetic_target(b, 80 + i) for i, b in enumerate(bodies)]), dtype=dt)
                xT, _ = m.rollout(p, x0, v0, 12, stream=stream)
                loss, xb, vb = m.loss_mse(xT, tg, stream=stream)
                g = m.zero_grads(("mu", "lam", "mass", "contact"))
                xb0, vb0 = m.rollout_backward(p, 12, xb, vb, g, stream=stream)
                stream.synchronize()
                outs.append([t.cpu().numpy().copy() for t in list(g.values()) + [xb0, vb0]])
        for a, b in zip(*outs):
            assert np.array_equal(a, b), lanes


def test_overlap_with_lift_drag_keeps_the_sequential_backward(gs):
    bodies = [W.control_cloth(5, n=12), W.tiny_cube(2)]
    a = gradient(gs, bodies, torch.float64, 30, 7, False, gs.EXEC_GRAPH, 2)
    b = gradient(gs, bodies, torch.float64, 30, 7, True, gs.EXEC_GRAPH, 2)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("exec_name", ["graph", "persist"])
@pytest.mark.parametrize("T,K", [(40, 7), (9, 10)])
def test_kept_last_segment_follows_its_checkpoints(gs, T, K, exec_name):
    """A checkpointed rollout (graph or persistent execution) leaves its last segment's
    states for the next backward with the same checkpoints: that backward equals, bitwise, one without the second buffer, also
    when a forward-only rollout from another state ran in between; a checkpointed rollout
    into other checkpoints in between, or a toggle of the buffer, makes the backward
    recompute the segment and it still equals the reference."""
    bodies = [W.tiny_cube(6).round_to(np.float32), mixed_body(7).round_to(np.float32)]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        m = gs.Model(bodies, torch.float32, max_steps=T, ckpt_every=K)
        m.set_exec({"graph": gs.EXEC_GRAPH, "persist": gs.EXEC_PERSIST}[exec_name])
        p = m.params_from_bodies()
        x0 = gs.soa(np.concatenate([b.x0 for b in bodies]))
        v0 = gs.soa(np.concatenate([b.v0 for b in bodies]))
        x0b, v0b = x0 + 0.003, v0 * 0.5
        tg = gs.soa(np.concatenate([W.synthetic_target(b, 60 + i) for i, b in enumerate(bodies)]))
        ck_other = m.new_checkpoints()

        def grad(between=None, overlap=True):
            m.set_overlap(overlap)
            xT, _ = m.rollout(p, x0, v0, T, stream=stream)
            loss, xb, vb = m.loss_mse(xT, tg, stream=stream)
            if between:
                between()
            g = m.zero_grads(("mu", "lam", "ktri", "mass", "contact"))
            xb0, vb0 = m.rollout_backward(p, T, xb, vb, g, stream=stream)
            stream.synchronize()
            return [t.cpu().numpy().copy() for t in list(g.values()) + [xb0, vb0]]

        ref = grad(overlap=False)
        cases = {
            "kept": grad(),
            "forward-only rollout between": grad(lambda: m.rollout(p, x0b, v0b, T, checkpoint=False, stream=stream)),
            "checkpointed rollout into other checkpoints between":
                grad(lambda: m.rollout(p, x0b, v0b, T, ckpt=ck_other, stream=stream)),
            "buffer toggled between": grad(lambda: (m.set_overlap(False), m.set_overlap(True))),
        }
    for name, out in cases.items():
        for a, b in zip(ref, out):
            assert np.array_equal(a, b), name


def test_overlap_needs_a_large_enough_buffer(gs):
    m = gs.Model([W.tiny_cube(0)], torch.float32, max_steps=20, ckpt_every=5, overlap=False)
    small = torch.empty(4 * 6 * m.np - 1, dtype=torch.float32, device="cuda")  # K - 1 = 4 states, one value short
    with pytest.raises(gs.GsimError) as e:
        gs._check(gs.load().gsim_model_set_overlap(m._h, small.data_ptr(), small.numel() * 4))
    assert e.value.code == gs.GSIM_E_WORKSPACE
    m.set_overlap(True)  # the binding's own buffer: max(K - 1, 1) states
    m.set_overlap(False)


def test_overlapped_tiny_cube_against_oracle(oracle_lib, gs):
    """The tiny cube (162 tets), FP32, 100 steps, checkpoints every 10, graph execution
    with the overlapped backward: positions within 1e-4 and gradients within 1e-3 of the
    FP64 oracle."""
    body = W.tiny_cube(0).round_to(np.float32)
    tgt = W.synthetic_target(body, 1).astype(np.float32).astype(np.float64)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        m = gs.Model([body], torch.float32, max_steps=100, ckpt_every=10)
        m.set_exec(gs.EXEC_GRAPH)
        p = m.params_from_bodies()
        xT, _ = m.rollout(p, gs.soa(body.x0), gs.soa(body.v0), 100, stream=stream)
        loss, xb, vb = m.loss_mse(xT, gs.soa(tgt), stream=stream)
        g = m.zero_grads(("mu", "lam", "mass", "contact"))
        m.rollout_backward(p, 100, xb, vb, g, stream=stream)
        stream.synchronize()
    L, go, xs, _ = oracle_for(oracle_lib, body).loss_and_grad(body.params(), body.x0, body.v0, 100, tgt,
                                                               want=("mu", "lam", "mass"))
    errs = {"x": rel(gs.aos(xT), xs[-1]), "mu": rel(g["mu"].double().cpu().numpy(), go["mu"]),
            "lam": rel(g["lam"].double().cpu().numpy(), go["lam"]),
            "mass": rel(g["mass"].double().cpu().numpy(), go["mass"]),
            "contact": rel(g["contact"][0].double().cpu().numpy(), go["contact"])}
    print("overlapped backward, tiny cube against the oracle:", {k: "%.2e" % v for k, v in errs.items()})
    assert errs["x"] < 1e-4 and all(errs[k] < 1e-3 for k in ("mu", "lam", "mass", "contact")), errs
