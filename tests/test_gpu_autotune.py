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
