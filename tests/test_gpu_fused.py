"""Fused execution (one workgroup per body, LDS-resident, whole segments per launch)
against the oracle and against the two-pass path."""
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


def run(gs, bodies, T, K, dtype, exec_mode, targets):
    m = gs.Model(bodies, dtype, max_steps=T, ckpt_every=K)
    m.set_exec(exec_mode)
    p = m.params_from_bodies()
    x0 = gs.soa(np.concatenate([b.x0 for b in bodies]), dtype)
    v0 = gs.soa(np.concatenate([b.v0 for b in bodies]), dtype)
    xT, vT = m.rollout(p, x0, v0, T)
    loss, xb, vb = m.loss_mse(xT, gs.soa(np.concatenate(targets), dtype))
    g = m.zero_grads()
    xb0, vb0 = m.rollout_backward(p, T, xb, vb, g)
    torch.cuda.synchronize()
    out = {k: v.detach().double().cpu().numpy() for k, v in g.items()}
    out["x"] = gs.aos(xT)
    out["xb0"] = gs.aos(xb0)
    out["loss"] = loss.double().cpu().numpy()
    return out


@pytest.mark.parametrize("case", ["cube", "mixed", "cloth"])
def test_fused_fp64_matches_two_pass(gs, case):
    """Same arithmetic, different summation order: FP64 agreement ~1e-12."""
    b = {"cube": W.tiny_cube(4), "mixed": mixed_body(5), "cloth": W.cloth(7, n=20, size=0.8)}[case]
    tgt = W.synthetic_target(b, 9)
    a = run(gs, [b], 40, 7, torch.float64, gs.EXEC_PLAIN, [tgt])
    f = run(gs, [b], 40, 7, torch.float64, gs.EXEC_FUSED, [tgt])
    for k in a:
        if np.abs(a[k]).max() > 0:
            assert rel(f[k], a[k]) < 1e-11, (k, rel(f[k], a[k]))


def test_fused_fp32_cube_against_oracle(gs, oracle_lib):
    T = 100
    b = W.tiny_cube(0).round_to(np.float32)
    tgt = W.synthetic_target(b, 1).astype(np.float32).astype(np.float64)
    f = run(gs, [b], T, 10, torch.float32, gs.EXEC_FUSED, [tgt])
    orc = oracle_for(oracle_lib, b)
    L, g, xs, _ = orc.loss_and_grad(b.params(), b.x0, b.v0, T, tgt, want=("mu", "lam", "mass"))
    errs = {"x": rel(f["x"], xs[-1]), "mu": rel(f["mu"], g["mu"]), "lam": rel(f["lam"], g["lam"]),
            "mass": rel(f["mass"], g["mass"]), "contact": rel(f["contact"][0], g["contact"])}
    print("fused f32 cube errors", {k: "%.2e" % v for k, v in errs.items()})
    assert errs["x"] < 1e-4
    for k in ("mu", "lam", "mass", "contact"):
        assert errs[k] < 1e-3


def test_fused_cloth_60_fp32_against_oracle(gs, oracle_lib):
    """60x60 cloth (the largest square grid whose adjoint state fits in 160 KB of LDS),
    400 steps."""
    T = 400
    b = W.cloth(10, n=60).round_to(np.float32)
    orc = oracle_for(oracle_lib, b)
    tgt = (b.X + np.random.default_rng(2).normal(0, 0.05, b.X.shape)).astype(np.float32).astype(np.float64)
    L, g, xs, _ = orc.loss_and_grad(b.params(), b.x0, b.v0, T, tgt, want=("ktri",))
    f = run(gs, [b], T, 20, torch.float32, gs.EXEC_FUSED, [tgt])
    errs = {"x": rel(f["x"], xs[-1]), "ktri": rel(f["ktri"], g["ktri"])}
    print("fused f32 cloth errors", {k: "%.2e" % v for k, v in errs.items()})
    assert errs["x"] < 1e-4 and errs["ktri"] < 1e-3


def test_fused_batch_alone_vs_mix_and_determinism(gs):
    bodies = [W.batch_body(20000 + i, lo=500, hi=4000) for i in range(6)]
    tgts = [W.synthetic_target(b, 3 + i) for i, b in enumerate(bodies)]
    mix = run(gs, bodies, 30, 10, torch.float32, gs.EXEC_FUSED, tgts)
    again = run(gs, bodies, 30, 10, torch.float32, gs.EXEC_FUSED, tgts)
    for k in mix:
        assert np.array_equal(mix[k], again[k]), k
    p0 = e0 = 0
    for i, b in enumerate(bodies):
        one = run(gs, [b], 30, 10, torch.float32, gs.EXEC_FUSED, [tgts[i]])
        assert np.array_equal(one["x"], mix["x"][p0:p0 + b.np])
        assert np.array_equal(one["mu"], mix["mu"][e0:e0 + b.ne])
        assert np.array_equal(one["mass"], mix["mass"][p0:p0 + b.np])
        assert np.array_equal(one["contact"][0], mix["contact"][i])
        p0 += b.np
        e0 += b.ne
    # checkpoint interval does not change the bits
    k7 = run(gs, bodies, 30, 7, torch.float32, gs.EXEC_FUSED, tgts)
    assert np.array_equal(k7["mu"], mix["mu"]) and np.array_equal(k7["xb0"], mix["xb0"])


def test_fused_rejects_oversized_body(gs):
    b = W.large_blob(30)
    m = gs.Model([b], torch.float32, max_steps=10, ckpt_every=5)
    with pytest.raises(gs.GsimError) as ei:
        m.set_exec(gs.EXEC_FUSED)
    assert ei.value.code == gs.GSIM_E_UNSUPPORTED
