"""Every body of the 256-body batch against the FP64 oracle (not collected by pytest:
~2.5 minutes of oracle time on 8 cores).  Runs the batch on the GPU through the
graph-captured two-pass path and the fused path (FP32, 100 steps, checkpoints every
10), then the oracle on every body in a process pool, and prints the per-body
norm-relative errors of positions, loss and the gradients w.r.t. mu, lambda, mass
and the contact parameters: maximum (and its body), median, and bodies above 1e-3.

    python tests/full_batch_parity.py [--workers 8]
"""
import argparse
import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

T, K, N = 100, 10, 256


def oracle_body(i):
    import oracle.oracle as O
    from helpers import oracle_for
    from paper_2104_02646_amd import workloads as W
    b = W.batch_body(1000 * 20 + i).round_to(np.float32)
    tgt = W.synthetic_target(b, 7000 + i).astype(np.float32).astype(np.float64)
    L, g, xs, _ = oracle_for(O, b).loss_and_grad(b.params(), b.x0, b.v0, T, tgt, want=("mu", "lam", "mass"))
    return L, g, xs[-1]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=8)
    args = ap.parse_args()
    import torch
    import oracle.oracle as O
    from helpers import rel
    from paper_2104_02646_amd import gsim, workloads as W
    from test_gpu_batch import run_batch
    O.build(force=False)
    gsim.load()
    bodies = [b.round_to(np.float32) for b in W.batch_bodies(20, N)]
    targets = [W.synthetic_target(b, 7000 + i).astype(np.float32).astype(np.float64) for i, b in enumerate(bodies)]
    gpu = {name: run_batch(gsim, bodies, targets, mode) for name, mode in
           (("graph", gsim.EXEC_GRAPH), ("fused", gsim.EXEC_FUSED))}
    ref = []
    with Pool(args.workers) as pool:
        for i, r in enumerate(pool.imap(oracle_body, range(N), chunksize=1)):
            ref.append(r)
            if (i + 1) % 32 == 0:
                print("oracle: %d of %d bodies done" % (i + 1, N), flush=True)
    poff = np.concatenate([[0], np.cumsum([b.np for b in bodies])])
    eoff = np.concatenate([[0], np.cumsum([b.ne for b in bodies])])
    for name, (x, loss, g) in gpu.items():
        errs = {k: [] for k in ("x", "loss", "mu", "lam", "mass", "contact")}
        for i, (L, go, xT) in enumerate(ref):
            pe, ee = slice(poff[i], poff[i + 1]), slice(eoff[i], eoff[i + 1])
            errs["x"].append(rel(x[pe], xT))
            errs["loss"].append(abs(loss[i] - L) / abs(L))
            errs["mu"].append(rel(g["mu"][ee], go["mu"]))
            errs["lam"].append(rel(g["lam"][ee], go["lam"]))
            errs["mass"].append(rel(g["mass"][pe], go["mass"]))
            errs["contact"].append(rel(g["contact"][i], go["contact"]))
        for k, v in errs.items():
            v = np.array(v)
            print("%s %-7s max %.2e (body %3d)  median %.2e  bodies > 1e-3: %d" %
                  (name, k, v.max(), v.argmax(), np.median(v), (v > 1e-3).sum()))


if __name__ == "__main__":
    main()
