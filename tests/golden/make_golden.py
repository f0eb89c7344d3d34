"""Writes the oracle snapshots in this folder (calls only oracle/ and the seeded
input generators). The paper prints no worked numeric example of the simulator,
so these fix the oracle's own FP64 results for the 10x10 (C1) and 32x32 (C2)
workloads: the step and rollout of Sec. 3.1 (Eq. 1, 4, 5) and the adjoint of its
backward pass, under the readings listed in the oracle's header.

    python tests/golden/make_golden.py
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2203_11938_amd import workloads as W  # noqa: E402

SAMPLE_VERTS = 8


def snapshot(name, steps=None):
    w = W.workload(name) if steps is None else W.workload(name, steps=steps)
    inst = W.make_instances(w)[0]
    tgt_o = oracle.Oracle(inst.tris, inst.rest, inst.pins,
                          *(np.array(inst.material.as_tuple()) * inst.target_factors),
                          dt=w.dt, cg_tol=1e-12)
    frames = w.loss_frames()
    target, _, _, _ = tgt_o.rollout(w.steps, inst.x0, inst.v0, inst.forces, frames)
    o = oracle.Oracle(inst.tris, inst.rest, inst.pins, *inst.material.as_tuple(), dt=w.dt,
                      cg_tol=1e-12)
    xo, _, _, _ = o.rollout(w.steps, inst.x0, inst.v0, inst.forces, frames)
    g = o.gradient(w.steps, inst.x0, inst.v0, inst.forces, frames, 2.0 * (xo - target))
    verts = np.random.Generator(np.random.PCG64(99)).choice(inst.n_verts, SAMPLE_VERTS,
                                                          replace=False)
    verts = np.sort(verts)
    return {
        "workload": name, "steps": w.steps, "dt": w.dt, "n": w.n,
        "loss": float(np.sum((xo - target) ** 2)),
        "sample_vertices": verts.tolist(),
        "x_final": xo[-1][verts].tolist(),
        "dl_dmaterial": g["material"].tolist(),
        "dl_dx0": g["x0"][verts].tolist(),
        "dl_dv0": g["v0"][verts].tolist(),
        "dl_dforces_step1": g["forces"][0][verts].tolist(),
        "norms": {"x_final": float(np.linalg.norm(xo[-1])),
                  "dl_dx0": float(np.linalg.norm(g["x0"])),
                  "dl_dforces": float(np.linalg.norm(g["forces"]))},
    }


def main():
    for name, steps in (("C1", None), ("C2", 30)):
        d = snapshot(name, steps)
        d["source"] = ("FP64 oracle, CG tol 1e-12 (Sec. 3.1, Eq. 1-5 and the backward pass; "
                       "readings R1-R18); written by tests/golden/make_golden.py")
        path = os.path.join(HERE, f"{name.lower()}_oracle.json")
        with open(path, "w") as f:
            json.dump(d, f, indent=1)
        print("wrote", path)


if __name__ == "__main__":
    main()
