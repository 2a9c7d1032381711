"""Writes the FP64 oracle's 1000-step discrete-adjoint gradient of the large blob
(App. A adjoint over App. A.2 semi-implicit Euler steps of the App. B.1 energy), so
that the GPU test can compare its checkpointed 1000-step gradient element by element
without running the oracle for half an hour.  Calls only oracle/ and the seeded input
generators.

    python tests/golden/make_blob_reference.py      (about 30 minutes on one core)

Writes tests/golden/blob_mu_1000.npy (float32 [n_tets]: d loss / d mu per element)
and tests/golden/blob_mu_1000.json (loss, sizes and input checksums)."""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle.oracle as O  # noqa: E402
from paper_2104_02646_amd import workloads as W  # noqa: E402

T = 1000


def blob():
    b = W.large_blob(30).round_to(np.float32)
    b.target = W.synthetic_target(b, 31).astype(np.float32).astype(np.float64)
    return b


def checksums(b):
    return {"X": float(b.X.sum()), "mu": float(b.mu.sum()), "lam": float(b.lam.sum()), "mass": float(b.mass.sum()),
            "target": float(b.target.sum()), "v0": float(b.v0.sum())}


def main():
    O.build(force=False)
    b = blob()
    t0 = time.time()
    o = O.Oracle(b.X, tets=b.tets, pinned=b.pinned, gravity=b.gravity, ground=b.ground, plane=b.plane, dt=b.dt)
    L, g, xs, _ = o.loss_and_grad(b.params(), b.x0, b.v0, T, b.target, want=("mu",))
    np.save(os.path.join(HERE, "blob_mu_1000.npy"), g["mu"].astype(np.float32))
    meta = {"steps": T, "n_tets": int(b.ne), "n_particles": int(b.np), "loss": float(L),
            "mu_grad_norm": float(np.linalg.norm(g["mu"])), "checksums": checksums(b),
            "oracle_seconds": time.time() - t0,
            "source": "tests/golden/make_blob_reference.py (FP64 oracle, seed 30 blob, target seed 31)"}
    with open(os.path.join(HERE, "blob_mu_1000.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(meta)


if __name__ == "__main__":
    main()
