"""Every body of the 256-body batch (1,367,346 tets) against the FP64 oracle, in the
launch configuration the benchmark times (graph-captured two-pass path, 512-element
tiles, four launch lanes, overlapped backward; FP32, 100 steps, checkpoints every 10)
and through the fused path.
Per body: positions and loss within 1e-4, gradients w.r.t. mu, lambda, mass and the
contact parameters within 1e-3 (norm-relative, R16), with the largest element-wise
error printed beside each.

Branch flips (R15): the contact model has two kinks (contact on/off, stick/slip).  For
every body the oracle also runs with its state stored the way the kernels store it
(displacement from rest and velocity rounded to FP32 after each step), and the
particle-steps whose branch differs from the FP64 run's are counted and printed.  A
body with such a flip has a loss whose derivative is one-sided there, and the
FP64 run and the FP32 run take different sides; its gradients are checked, at the
same 1e-3, against the oracle's exact discrete adjoint along the run that takes the
FP32 side.  The oracle runs on the host's cores in threads (its ctypes calls release
the interpreter lock; each thread owns its oracle objects)."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from helpers import maxrel, oracle_for, rel
from paper_2104_02646_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

T, K, N = 100, 10, 256
WORKERS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def gs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2104_02646_amd import gsim
    gsim.load()
    return gsim


@pytest.fixture(scope="module")
def batch():
    bodies = [b.round_to(np.float32) for b in W.batch_bodies(20, N)]
    targets = [W.synthetic_target(b, 7000 + i).astype(np.float32).astype(np.float64) for i, b in enumerate(bodies)]
    return bodies, targets


@pytest.fixture(scope="module")
def reference(oracle_lib, batch):
    bodies, targets = batch
    want = ("mu", "lam", "mass")

    def one(i):
        b = bodies[i]
        o = oracle_for(oracle_lib, b)
        p = b.params()
        L, g, xs, vs = o.loss_and_grad(p, b.x0, b.v0, T, targets[i], want=want)
        # the same run with the state stored as the kernels store it
        f32 = lambda a: a.astype(np.float32).astype(np.float64)
        xq, vq = [b.x0], [b.v0]
        for _ in range(T):
            x1, v1 = o.step(p, xq[-1], vq[-1])
            xq.append(b.X + f32(x1 - b.X))
            vq.append(f32(v1))
        flips = []
        for t in range(T):
            ca, cb = o.contact_branches(p, xs[t], vs[t]), o.contact_branches(p, xq[t], vq[t])
            flips += [(t, int(j), int(ca[j]), int(cb[j])) for j in np.nonzero(ca != cb)[0]]
        matched = None
        if flips:
            Lq, xbq = o.loss(xq[-1], targets[i], with_grad=True)
            _, _, gq = o.backward(p, np.array(xq), np.array(vq), xbq, None, want=want)
            matched = (Lq, gq)
        return L, g, xs[-1], flips, matched

    ref = []
    with ThreadPoolExecutor(WORKERS) as pool:
        for i, r in enumerate(pool.map(one, range(N))):
            ref.append(r)
            if (i + 1) % 32 == 0:
                print("oracle: %d of %d bodies" % (i + 1, N), flush=True)
    nflip = sum(len(r[3]) for r in ref)
    print("branch flips between the FP64 run and the FP32-stored run: %d particle-steps in %d bodies %s"
          % (nflip, sum(1 for r in ref if r[3]), {i: r[3] for i, r in enumerate(ref) if r[3]}), flush=True)
    return ref


@pytest.mark.parametrize("exec_name", ["graph", "fused"])
def test_every_body_against_oracle(gs, batch, reference, exec_name):
    from test_gpu_batch import run_batch
    bodies, targets = batch
    x, loss, g = run_batch(gs, bodies, targets, {"graph": gs.EXEC_GRAPH, "fused": gs.EXEC_FUSED}[exec_name])
    poff = np.concatenate([[0], np.cumsum([b.np for b in bodies])])
    eoff = np.concatenate([[0], np.cumsum([b.ne for b in bodies])])
    errs = {k: np.zeros(N) for k in ("x", "loss", "mu", "lam", "mass", "contact")}
    emax = {k: np.zeros(N) for k in ("mu", "lam", "mass")}
    for i, (L, go, xT, flips, matched) in enumerate(reference):
        pe, ee = slice(poff[i], poff[i + 1]), slice(eoff[i], eoff[i + 1])
        errs["x"][i] = rel(x[pe], xT)
        errs["loss"][i] = abs(loss[i] - L) / abs(L)
        gref = go
        if flips:  # one-sided derivative at a flipped kink: the branch-matched adjoint
            gref = matched[1]
            print("%s body %d: %d flipped particle-steps %s; against the FP64 run: %s" % (
                exec_name, i, len(flips), flips,
                {k: "%.2e" % rel(g[k][sl], go[k]) for k, sl in (("mu", ee), ("lam", ee), ("mass", pe))}
                | {"contact": "%.2e" % rel(g["contact"][i], go["contact"])}))
        for k, sl in (("mu", ee), ("lam", ee), ("mass", pe)):
            errs[k][i] = rel(g[k][sl], gref[k])
            emax[k][i] = maxrel(g[k][sl], gref[k])
        errs["contact"][i] = rel(g["contact"][i], gref["contact"])
    for k, v in errs.items():
        extra = "  max element %.2e" % emax[k].max() if k in emax else ""
        print("%s %-7s max %.2e (body %3d)  median %.2e%s" % (exec_name, k, v.max(), v.argmax(), np.median(v), extra))
    assert errs["x"].max() < 1e-4 and errs["loss"].max() < 1e-4
    for k in ("mu", "lam", "mass", "contact"):
        assert errs[k].max() < 1e-3, (k, errs[k].max(), int(errs[k].argmax()))
