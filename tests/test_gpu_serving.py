"""Continuous-batching engine: every query's answer is bit-for-bit the answer it
gets alone, queries that arrive while others run are admitted as memory frees up,
and admission respects the device pool (FIFO)."""
import numpy as np
import pytest

from paper_2104_02646_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2104_02646_amd import serve
    serve.gsim.load()
    return serve


def _table_bytes(sv, max_live, max_tiles):
    """Pool bytes the engine keeps for its own per-tick tables."""
    probe = sv.Engine(pool_bytes=64 << 20, max_live=max_live, max_tiles=max_tiles)
    return (64 << 20) - probe.stats()["pool_free"]


def mixed_queries():
    qs = []
    for i, (kind, size, T, K) in enumerate([("tet", 800, 60, 10), ("cloth", 16, 45, 7), ("tet", 3000, 80, 20),
                                            ("cloth", 24, 30, 30), ("tet", 1500, 25, 4), ("tet", 500, 90, 9),
                                            ("cloth", 12, 70, 10), ("tet", 5000, 40, 10)]):
        b = W.batch_body(50000 + i, lo=size, hi=size) if kind == "tet" else W.cloth(60 + i, n=size, size=0.5)
        b.target = W.synthetic_target(b, 70 + i)
        qs.append((b, T, K))
    return qs


@pytest.mark.parametrize("rounds", [1, 3])
def test_alone_equals_in_mix_bitwise(sv, rounds):
    qs = mixed_queries()
    eng = sv.Engine(pool_bytes=1 << 30, max_live=16, micro_steps=rounds)
    qbs = [sv.QueryBuffers(b, T, K) for b, T, K in qs]
    # half now, the rest while the first half is in flight
    for qb in qbs[:4]:
        eng.submit(qb)
    done = []
    for _ in range(20):
        eng.tick()
        done += eng.poll()
    for qb in qbs[4:]:
        eng.submit(qb)
    done += eng.run_until_idle()
    assert len(done) == len(qbs)
    st = eng.stats()
    assert st["mean_live"] > 1.5, st
    times = {qid: (ta, td) for qid, qb, ts, ta, td in done}
    late = [times[q] for q in list(times)[4:]]
    early_done = max(td for ta, td in list(times.values())[:4])
    assert any(ta < early_done for ta, td in late), "late queries must be admitted while early ones run"
    for qb in qbs:
        loss, g = sv.solve_alone(qb)
        assert np.float32(loss) == np.float32(qb.loss), (loss, qb.loss)
        b = qb.body
        assert np.array_equal(g["mass"], qb.out["mass"])
        if b.ne:
            assert np.array_equal(g["mu"], qb.out["mu"])
            assert np.array_equal(g["lam"], qb.out["lam"])
            assert np.array_equal(g["contact"], qb.out["contact"])
        if b.nt:
            assert np.array_equal(g["ktri"], qb.out["k_tri"])


def test_admission_by_footprint_fifo(sv):
    """A pool that holds only two of the queries at once: the rest wait, admission
    follows submission order, everything completes with the right answers."""
    qs = [(W.batch_body(51000 + i, lo=2000, hi=2000), 40, 10) for i in range(5)]
    for i, (b, T, K) in enumerate(qs):
        b.target = W.synthetic_target(b, 90 + i)
    qbs = [sv.QueryBuffers(b, T, K) for b, T, K in qs]
    need = max(qb.bytes() for qb in qbs)
    tables = _table_bytes(sv, 16, 1 << 14)
    eng = sv.Engine(pool_bytes=int(2.5 * need) + tables, max_live=16, max_tiles=1 << 14)
    for qb in qbs:
        eng.submit(qb)
    peak = 0
    done = []
    while True:
        nl, nq = eng.tick()
        peak = max(peak, nl)
        done += eng.poll()
        if nl == 0 and nq == 0:
            break
    assert peak == 2
    admits = [ta for qid, qb, ts, ta, td in sorted(done, key=lambda r: r[0])]
    assert admits == sorted(admits)
    for qb in qbs:
        loss, g = sv.solve_alone(qb)
        assert np.array_equal(g["mu"], qb.out["mu"])


def test_rejects_query_larger_than_pool(sv):
    from paper_2104_02646_amd import gsim
    b = W.batch_body(52000, lo=4000, hi=4000)
    b.target = W.synthetic_target(b, 1)
    qb = sv.QueryBuffers(b, 100, 10)
    eng = sv.Engine(pool_bytes=qb.bytes() // 2 + _table_bytes(sv, 4, 1 << 14), max_live=4, max_tiles=1 << 14)
    with pytest.raises(gsim.GsimError) as ei:
        eng.submit(qb)
    assert ei.value.code == gsim.GSIM_E_WORKSPACE


def test_served_answers_match_the_oracle(sv, oracle_lib):
    """A tet query and a cloth query served together with two more queries in the mix:
    each answer (loss, and the gradients w.r.t. its own parameters) against the FP64
    oracle's discrete adjoint of the same rollout: loss within 1e-4, gradients within
    1e-3 (norm-relative, R16; the largest element-wise error printed)."""
    from helpers import maxrel, oracle_for, rel
    T, K = 60, 10
    tet = W.batch_body(50100, lo=1200, hi=1200).round_to(np.float32)
    cloth = W.cloth(61, n=20, size=0.5).round_to(np.float32)
    extra = [W.batch_body(50101, lo=3000, hi=3000).round_to(np.float32), W.cloth(62, n=12, size=0.5).round_to(np.float32)]
    bodies = [tet, cloth] + extra
    for i, b in enumerate(bodies):
        b.target = W.synthetic_target(b, 80 + i).astype(np.float32).astype(np.float64)
    eng = sv.Engine(pool_bytes=1 << 30, max_live=8)
    qbs = [sv.QueryBuffers(b, T, K) for b in bodies]
    for qb in qbs:
        eng.submit(qb)
    done = eng.run_until_idle()
    assert len(done) == len(qbs) and eng.stats()["mean_live"] > 2
    for qb, b in zip(qbs[:2], bodies[:2]):
        assert qb.status == 0
        want = ("mu", "lam", "mass") if b.ne else ("ktri", "mass")
        L, g, xs, _ = oracle_for(oracle_lib, b).loss_and_grad(b.params(), b.x0, b.v0, T, b.target, want=want)
        errs = {"loss": abs(qb.loss - L) / abs(L)}
        for k in want:
            errs[k] = rel(qb.out["k_tri" if k == "ktri" else k], g[k])
            errs[k + " max"] = maxrel(qb.out["k_tri" if k == "ktri" else k], g[k])
        if b.ground:
            errs["contact"] = rel(qb.out["contact"], g["contact"])
        print("served %s (%d elements): %s" % ("tet" if b.ne else "cloth", b.ne or b.nt,
                                              {k: "%.2e" % v for k, v in errs.items()}))
        assert errs["loss"] < 1e-4
        for k, v in errs.items():
            if k != "loss" and not k.endswith(" max"):
                assert v < 1e-3, (k, v)


def test_store_every_state_is_bitwise_the_checkpointed_answer(sv):
    """The same queries with their own checkpoint intervals (store limit 0) and with
    every state stored (a limit above every footprint): bitwise the same losses and
    gradients, in fewer micro-step rounds (no recomputed segments)."""
    qs = mixed_queries()
    runs = []
    for limit in (0, 1 << 40):
        qbs = [sv.QueryBuffers(b, T, K) for b, T, K in qs]
        eng = sv.Engine(pool_bytes=1 << 30, max_live=16)
        eng.set_store_limit(limit)
        for qb in qbs:
            eng.submit(qb)
        eng.run_until_idle()
        runs.append((qbs, eng.stats()["ticks"]))
    (a, ticks_a), (b, ticks_b) = runs
    for qa, qb in zip(a, b):
        assert qa.status == 0 and qb.status == 0
        assert np.float32(qa.loss) == np.float32(qb.loss)
        for k in qa.out:
            assert np.array_equal(qa.out[k], qb.out[k]), k
    assert ticks_b < ticks_a


def test_more_segments_than_one_lookup_holds(sv):
    """300 small queries live at once: every round's launches hold 300 segments, beyond
    one wavefront's 64 and beyond the 256 begins each workgroup loads at once, so the
    tile lookup takes its chunked path; every answer is bitwise that of the query alone
    (sampled) and the first rounds run all 300 together."""
    qs = []
    for s in range(300):
        b = W.tiny_cube(s)
        b.target = W.synthetic_target(b, 1000 + s)
        qs.append(b)
    qbs = [sv.QueryBuffers(b, 12, 4) for b in qs]
    eng = sv.Engine(pool_bytes=1 << 30, max_live=300, max_tiles=1 << 12)
    for qb in qbs:
        eng.submit(qb)
    nl, nq = eng.tick()
    assert nl == 300 and nq == 0
    done = eng.poll() + eng.run_until_idle()
    assert len(done) == 300
    for qb in qbs[::23] + [qbs[-1]]:
        assert qb.status == 0
        loss, g = sv.solve_alone(qb)
        assert np.float32(loss) == np.float32(qb.loss)
        for k in ("mu", "lam", "mass", "contact"):
            assert np.array_equal(g[k], qb.out[k]), k


def test_prepared_on_threads_equals_submit(sv):
    """Queries prepared concurrently on worker threads (gsim_engine_prepare) and then
    submitted in order: bitwise the answers of plain submission; a handle that is not
    submitted is freed; a query that cannot fit is refused at submission (the handle is
    consumed either way)."""
    from concurrent.futures import ThreadPoolExecutor
    from paper_2104_02646_amd import gsim
    qs = mixed_queries()
    ref = [sv.QueryBuffers(b, T, K) for b, T, K in qs]
    eng = sv.Engine(pool_bytes=1 << 30, max_live=16)
    for qb in ref:
        eng.submit(qb)
    eng.run_until_idle()
    qbs = [sv.QueryBuffers(b, T, K) for b, T, K in qs]
    with ThreadPoolExecutor(4) as pool:
        handles = list(pool.map(sv.Engine.prepare, qbs))
    eng2 = sv.Engine(pool_bytes=1 << 30, max_live=16)
    for qb, h in zip(qbs, handles):
        eng2.submit_prepared(qb, h)
    eng2.run_until_idle()
    for a, b in zip(ref, qbs):
        assert a.status == 0 and b.status == 0
        assert np.float32(a.loss) == np.float32(b.loss)
        for k in a.out:
            assert np.array_equal(a.out[k], b.out[k]), k
    spare = sv.Engine.prepare(qbs[0])
    sv._load().gsim_prepared_destroy(spare)
    big = W.batch_body(52000, lo=4000, hi=4000)
    big.target = W.synthetic_target(big, 1)
    qb = sv.QueryBuffers(big, 100, 10)
    small = sv.Engine(pool_bytes=qb.bytes() // 2 + _table_bytes(sv, 4, 1 << 14), max_live=4, max_tiles=1 << 14)
    small.set_store_limit(0)
    with pytest.raises(gsim.GsimError) as ei:
        small.submit_prepared(qb, sv.Engine.prepare(qb))
    assert ei.value.code == gsim.GSIM_E_WORKSPACE
