"""Persistent execution (one workgroup per body runs a call's whole run of steps through
the two-pass tiles, barriers in place of launch boundaries): bitwise the two-pass
results, since the tiles, their partial slots and the particle passes' thread mapping
are the same; against the oracle through that identity and directly."""
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


def run(gs, bodies, T, K, exec_mode, targets, tile=0, pshape=None):
    m = gs.Model(bodies, torch.float32, max_steps=T, ckpt_every=K, tile_elems=tile)
    if pshape:
        m.set_launch(1, *pshape)
    m.set_exec(exec_mode)
    p = m.params_from_bodies()
    x0 = gs.soa(np.concatenate([b.x0 for b in bodies]))
    v0 = gs.soa(np.concatenate([b.v0 for b in bodies]))
    xT, vT = m.rollout(p, x0, v0, T)
    loss, xb, vb = m.loss_mse(xT, gs.soa(np.concatenate(targets)))
    g = m.zero_grads()
    xb0, vb0 = m.rollout_backward(p, T, xb, vb, g)
    x1, v1 = m.step(p, x0, v0)
    xbm, vbm = m.step_backward(p, x0, v0, xb, vb)
    torch.cuda.synchronize()
    out = {k: v.detach().cpu().numpy() for k, v in g.items()}
    for k, t in (("xT", xT), ("vT", vT), ("xb0", xb0), ("vb0", vb0), ("loss", loss), ("x1", x1), ("v1", v1),
                 ("xbm", xbm), ("vbm", vbm)):
        out[k] = t.detach().cpu().numpy()
    return out


def batch6():
    bodies = [W.tiny_cube(3).round_to(np.float32), mixed_body(5).round_to(np.float32),
              W.cloth(7, n=20, size=0.8).round_to(np.float32)]
    bodies += [W.batch_body(60000 + i, lo=700, hi=3000).round_to(np.float32) for i in range(3)]
    return bodies


@pytest.mark.parametrize("case", ["cube", "mixed", "batch"])
def test_persist_bitwise_equals_two_pass(gs, case):
    """Rollout with checkpoints, loss, checkpointed backward, one step and one backward
    step: every output bitwise equal between plain two-pass launches and persistent
    execution (the batch: six bodies of 1 to 12 element tiles)."""
    bodies = {"cube": [W.tiny_cube(4).round_to(np.float32)], "mixed": [mixed_body(5).round_to(np.float32)],
              "batch": batch6()}[case]
    tg = [W.synthetic_target(b, 9 + i).astype(np.float32).astype(np.float64) for i, b in enumerate(bodies)]
    a = run(gs, bodies, 40, 7, gs.EXEC_PLAIN, tg)
    b = run(gs, bodies, 40, 7, gs.EXEC_PERSIST, tg)
    assert a.keys() == b.keys()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_persist_follows_the_particle_pass_shape(gs):
    """With a particle-pass shape of 128 threads x 2 particles the two-pass contact sums
    change their tree; persistent execution takes the same shape and stays bitwise equal."""
    bodies = batch6()[:4]
    tg = [W.synthetic_target(b, 30 + i).astype(np.float32).astype(np.float64) for i, b in enumerate(bodies)]
    a = run(gs, bodies, 25, 5, gs.EXEC_PLAIN, tg, tile=128, pshape=(128, 2))
    b = run(gs, bodies, 25, 5, gs.EXEC_PERSIST, tg, tile=128, pshape=(128, 2))
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_persist_tiny_cube_against_oracle(oracle_lib, gs):
    """The tiny cube (162 tets), 100 steps, checkpoints every 10, persistent execution:
    positions within 1e-4 and the mu, lambda, mass and contact gradients within 1e-3 of
    the FP64 oracle."""
    body = W.tiny_cube(0).round_to(np.float32)
    tgt = W.synthetic_target(body, 1).astype(np.float32).astype(np.float64)
    o = run(gs, [body], 100, 10, gs.EXEC_PERSIST, [tgt])
    L, g, xs, _ = oracle_for(oracle_lib, body).loss_and_grad(body.params(), body.x0, body.v0, 100, tgt,
                                                             want=("mu", "lam", "mass"))
    errs = {"x": rel(o["xT"].T, xs[-1]), "mu": rel(o["mu"], g["mu"]), "lam": rel(o["lam"], g["lam"]),
            "mass": rel(o["mass"], g["mass"]), "contact": rel(o["contact"][0], g["contact"])}
    print("persistent tiny cube against the oracle:", {k: "%.2e" % v for k, v in errs.items()})
    assert errs["x"] < 1e-4 and all(errs[k] < 1e-3 for k in ("mu", "lam", "mass", "contact")), errs


def test_persist_refusals(gs):
    cube = W.tiny_cube(0)
    m64 = gs.Model([cube], torch.float64, max_steps=4, ckpt_every=2)
    with pytest.raises(gs.GsimError) as e:
        m64.set_exec(gs.EXEC_PERSIST)
    assert e.value.code == gs.GSIM_E_UNSUPPORTED
    air = W.control_cloth(3, n=6) if hasattr(W, "control_cloth") else None
    if air is not None and getattr(air, "air", False):
        ma = gs.Model([air], torch.float32, max_steps=4, ckpt_every=2)
        with pytest.raises(gs.GsimError) as e:
            ma.set_exec(gs.EXEC_PERSIST)
        assert e.value.code == gs.GSIM_E_UNSUPPORTED
    m = gs.Model([cube], torch.float32, max_steps=4, ckpt_every=2)
    m.set_exec(gs.EXEC_PERSIST)
    with pytest.raises(gs.GsimError):
        m.set_timing()
