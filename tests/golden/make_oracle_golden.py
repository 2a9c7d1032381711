"""Writes tests/golden/oracle_golden.json: FP64 oracle results on small fixed inputs,
so that any later change to the oracle's arithmetic shows up as a diff of this file
(the values come from oracle/ alone; nothing here runs the HIP path).

Cases (each value's definition in the paper):
  tiny_cube   - 162 Neo-Hookean tets in sliding ground contact (App. A.1 FEM and
                contact), 40 semi-implicit Euler steps (App. A.2), position loss and
                its discrete-adjoint gradients (App. A)
  mixed_body  - the same cube plus a pinned 6 x 6 cloth with membrane and bending
                (App. A.1 thin shells), 30 steps, every parameter gradient
  rigid_box   - one rigid box with vertex contact (App. A.1 rigid bodies), 120 steps
  silhouette  - soft silhouette of a 6 x 6 cloth at 12 x 14 pixels (the soft
                rasterizer used for pixel losses, Sec. 3) and its vertex gradient

    python tests/golden/make_oracle_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path[:0] = [ROOT, os.path.dirname(HERE)]

OUT = os.path.join(HERE, "oracle_golden.json")


def compute():
    import torch

    import oracle.oracle as O
    from helpers import mixed_body, oracle_for
    from oracle import raster as R
    from paper_2104_02646_amd import workloads as W

    out = {}
    # tiny cube: loss and gradients
    b = W.tiny_cube(0)
    tgt = W.synthetic_target(b, 1)
    L, g, xs, _ = oracle_for(O, b).loss_and_grad(b.params(), b.x0, b.v0, 40, tgt,
                                                 want=("mu", "lam", "mass", "contact"))
    out["tiny_cube"] = {"steps": 40, "loss": L, "x_final_first4": xs[-1][:4].tolist(),
                        "grad_mu_first6": g["mu"][:6].tolist(), "grad_lam_first6": g["lam"][:6].tolist(),
                        "grad_mass_first6": g["mass"][:6].tolist(), "grad_contact": np.ravel(g["contact"]).tolist(),
                        "grad_x0_first2": g["x0"][:2].tolist(), "grad_v0_first2": g["v0"][:2].tolist()}
    # mixed body: every force term
    b = mixed_body(0)
    tgt = W.synthetic_target(b, 2)
    L, g, xs, _ = oracle_for(O, b).loss_and_grad(b.params(), b.x0, b.v0, 30, tgt,
                                                 want=("mu", "lam", "ktri", "mass", "contact"))
    out["mixed_body"] = {"steps": 30, "loss": L, "grad_ktri_first6": g["ktri"][:6].tolist(),
                         "grad_mu_norm": float(np.linalg.norm(g["mu"])),
                         "grad_mass_norm": float(np.linalg.norm(g["mass"])),
                         "grad_contact": np.ravel(g["contact"]).tolist()}
    # rigid box
    rb = W.rigid_body(700, "box")
    o = O.RigidOracle(rb.verts, gravity=rb.gravity, ground=rb.ground, plane=rb.plane, dt=rb.dt)
    L, gr, st = o.loss_and_grad(rb.s0, rb.mass, rb.inertia, rb.contact(), 120, rb.verts + rb.s0[:3] + 0.1)
    out["rigid_box"] = {"steps": 120, "loss": float(L), "state_final": st[-1].tolist(), "grad_s0": gr["s0"].tolist(),
                        "grad_mass": float(gr["m"]), "grad_inertia": gr["I"].tolist(), "grad_contact": gr["c"].tolist()}
    # silhouette
    cl = W.cloth(31, n=6, size=1.0, height=1.0)
    P = np.array([[14.0, 0.0, 7.0, -7.0], [0.0, -14.0, 6.0, 8.0], [0.0, 0.0, 1.0, 2.5]])
    X = torch.tensor(cl.X, requires_grad=True)
    img = R.silhouette(X, torch.as_tensor(cl.tris, dtype=torch.long), torch.tensor(P), 12, 14, 1.5)
    w = torch.linspace(-1.0, 1.0, 12 * 14, dtype=torch.float64).reshape(12, 14)
    (img * w).sum().backward()
    img = img.detach()
    out["silhouette"] = {"P": P.tolist(), "sigma": 1.5, "height": 12, "width": 14,
                         "image_sum": float(img.sum()), "image_row6": img[6].tolist(),
                         "grad_first3": X.grad[:3].tolist()}
    return out


if __name__ == "__main__":
    with open(OUT, "w") as fh:
        json.dump(compute(), fh, indent=1)
    print("wrote", OUT)
