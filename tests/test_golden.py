"""Stored oracle snapshots (tests/golden/, written by tests/golden/make_golden.py):
the oracle must keep reproducing them (a change to its arithmetic shows here and
needs the passage that justifies it), and the GPU must match them within the
parity gates."""

import json
import os

import numpy as np
import pytest

from paper_2203_11938_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def load(name):
    with open(os.path.join(HERE, "golden", f"{name.lower()}_oracle.json")) as f:
        return json.load(f)


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("name", ["C1", "C2"])
def test_oracle_reproduces_snapshot(oracle_mod, name):
    d = load(name)
    w = W.workload(name, steps=d["steps"])
    inst = W.make_instances(w)[0]
    tgt_o = oracle_mod.Oracle(inst.tris, inst.rest, inst.pins,
                              *(np.array(inst.material.as_tuple()) * inst.target_factors),
                              dt=w.dt, cg_tol=1e-12)
    frames = w.loss_frames()
    target, _, _, _ = tgt_o.rollout(w.steps, inst.x0, inst.v0, inst.forces, frames)
    o = oracle_mod.Oracle(inst.tris, inst.rest, inst.pins, *inst.material.as_tuple(), dt=w.dt,
                          cg_tol=1e-12)
    xo, _, _, _ = o.rollout(w.steps, inst.x0, inst.v0, inst.forces, frames)
    g = o.gradient(w.steps, inst.x0, inst.v0, inst.forces, frames, 2.0 * (xo - target))
    v = d["sample_vertices"]
    assert abs(float(np.sum((xo - target) ** 2)) - d["loss"]) <= 1e-10 * abs(d["loss"])
    assert rel(xo[-1][v], d["x_final"]) <= 1e-12
    assert rel(g["material"], d["dl_dmaterial"]) <= 1e-9
    assert rel(g["x0"][v], d["dl_dx0"]) <= 1e-9
    assert rel(g["forces"][0][v], d["dl_dforces_step1"]) <= 1e-9


@pytest.mark.gpu
def test_gpu_matches_c1_snapshot():
    import torch
    from gpu_common import make_sim, targets
    d = load("C1")
    w = W.workload("C1")
    inst = W.make_instances(w)[0]
    s = make_sim(w, [inst])
    dev = torch.device("cuda:0")
    x0 = torch.tensor(W.to_soa(inst.x0), dtype=torch.float64, device=dev)
    frames = w.loss_frames()
    # the target rollout (scaled material) from the oracle, as in the snapshot
    tgt = torch.tensor(W.to_soa(targets(w)), dtype=torch.float64, device=dev)
    xo = s.rollout(w.steps, x0, None, None, None, frames)
    g = s.adjoint((2.0 * (xo - tgt)).contiguous())
    s.sync()
    x = W.from_soa(xo.cpu().numpy())
    v = d["sample_vertices"]
    loss = float(((xo - tgt) ** 2).sum())
    print(f"C1 snapshot: loss {loss:.9e} vs {d['loss']:.9e}", flush=True)
    assert abs(loss - d["loss"]) <= 1e-6 * d["loss"]
    assert rel(x[-1][v], d["x_final"]) <= 1e-9
    assert rel(g["material"].cpu().numpy()[0], d["dl_dmaterial"]) <= 1e-6
    assert rel(W.from_soa(g["x0"].cpu().numpy())[v], d["dl_dx0"]) <= 1e-6
    s.close()
