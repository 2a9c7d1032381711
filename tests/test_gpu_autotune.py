"""Launch-shape autotuner: picks a shape per pass, caches it, changes no results."""
import numpy as np
import pytest

from paper_2104_02646_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_autotune_picks_caches_and_preserves_results(tmp_path, monkeypatch):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2104_02646_amd import autotune, gsim
    monkeypatch.setenv("GSIM_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    bodies = [W.batch_body(20000 + i, lo=1000, hi=6000) for i in range(6)]
    m = gsim.Model(bodies, torch.float32, max_steps=20, ckpt_every=5)
    p = m.params_from_bodies()
    x0 = gsim.soa(np.concatenate([b.x0 for b in bodies]))
    v0 = gsim.soa(np.concatenate([b.v0 for b in bodies]))
    ref, _ = m.rollout(p, x0, v0, 20)
    rep = autotune.tune(m, p, x0, v0, steps=3)
    assert len(rep) == 2 and all(not r["cached"] for r in rep.values())
    for r in rep.values():
        assert r["ms_per_step"] == min(r["candidates"].values())
    out, _ = m.rollout(p, x0, v0, 20)
    assert torch.equal(out, ref)  # forward positions do not depend on the launch shape
    m2 = gsim.Model(bodies, torch.float32, max_steps=20, ckpt_every=5)
    rep2 = autotune.tune(m2, p, x0, v0)
    assert all(r["cached"] for r in rep2.values())
    assert m2.get_launch(0) == m.get_launch(0) and m2.get_launch(1) == m.get_launch(1)


@pytest.mark.parametrize("tile", [32, 128, 512, 2048])
def test_tile_sizes_match_oracle(oracle_lib, tile):
    """Every element-tile size the planner accepts gives the oracle's gradients (FP32, 40
    steps, checkpoints every 8): the tile size only reorders the scatter's sums."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from helpers import oracle_for, rel
    from paper_2104_02646_amd import gsim
    T, K = 40, 8
    bodies = [W.batch_body(20000 + i, lo=600, hi=4000).round_to(np.float32) for i in (3, 4)]
    targets = [W.synthetic_target(b, 70 + i).astype(np.float32).astype(np.float64) for i, b in enumerate(bodies)]
    m = gsim.Model(bodies, torch.float32, max_steps=T, ckpt_every=K, tile_elems=tile)
    tiles = m.plan.tiles()[0]
    assert tiles[:, 3].max() <= tile
    p = m.params_from_bodies()
    xT, _ = m.rollout(p, gsim.soa(np.concatenate([b.x0 for b in bodies])),
                      gsim.soa(np.concatenate([b.v0 for b in bodies])), T)
    loss, xb, vb = m.loss_mse(xT, gsim.soa(np.concatenate(targets)))
    g = m.zero_grads(("mu", "lam", "mass", "contact"))
    m.rollout_backward(p, T, xb, vb, g)
    torch.cuda.synchronize()
    e0 = 0
    p0 = 0
    for i, b in enumerate(bodies):
        L, go, xs, _ = oracle_for(oracle_lib, b).loss_and_grad(b.params(), b.x0, b.v0, T, targets[i],
                                                               want=("mu", "lam", "mass"))
        sl_e, sl_p = slice(e0, e0 + b.ne), slice(p0, p0 + b.np)
        errs = {"x": rel(gsim.aos(xT)[sl_p], xs[-1]), "mu": rel(g["mu"][sl_e].double().cpu().numpy(), go["mu"]),
                "lam": rel(g["lam"][sl_e].double().cpu().numpy(), go["lam"]),
                "mass": rel(g["mass"][sl_p].double().cpu().numpy(), go["mass"]),
                "contact": rel(g["contact"][i].double().cpu().numpy(), go["contact"])}
        print("tile %d body %d:" % (tile, i), {k: "%.2e" % v for k, v in errs.items()})
        assert errs["x"] < 1e-4 and all(errs[k] < 1e-3 for k in ("mu", "lam", "mass", "contact")), errs
        e0 += b.ne
        p0 += b.np


def test_tune_model_picks_a_measured_configuration(tmp_path, monkeypatch):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2104_02646_amd import autotune, gsim
    monkeypatch.setenv("GSIM_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    bodies = [W.batch_body(20000 + i, lo=1000, hi=3000) for i in range(4)]
    m, rep = autotune.tune_model(bodies, torch.float32, 10, 5, tiles=(128, 512), lanes=(1, 2))
    assert not rep["cached"] and rep["ms_per_gradient"] == min(rep["candidates_ms"].values())
    c = rep["choice"]
    assert m.get_exec()[0] == c["exec"] and (c["exec"] == gsim.EXEC_FUSED or m.get_lanes() == c["lanes"])
    assert (m.plan.tile_elems or gsim.TILE_DEFAULT) == c["tile_elems"]
    m2, rep2 = autotune.tune_model(bodies, torch.float32, 10, 5, tiles=(128, 512), lanes=(1, 2))
    assert rep2["cached"] and rep2["choice"] == c
