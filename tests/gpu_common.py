"""Shared helpers of the GPU tests: build a library handle for a workload, run the
rollout + adjoint through the C ABI, and compute the FP64 oracle's reference."""

from __future__ import annotations

import functools

import numpy as np

import oracle
from paper_2203_11938_amd import workloads as W


def note(msg):
    print(msg, flush=True)


as_given = W.as_given


def make_sim(w, insts, **kw):
    from paper_2203_11938_amd import sim
    sheets = [sim.Sheet(i.tris, i.rest, i.pins, *i.material.as_tuple()) for i in insts]
    args = dict(dt=w.dt, precision=w.precision, cg_tol=w.cg_tol,
                checkpoint_every=w.checkpoint_every, max_steps=w.steps)
    args.update(kw)
    return sim.Simulator(sheets, **args)


def oracle_for(inst, w, tol=1e-12, factors=None):
    mat = np.array(inst.material.as_tuple())
    if factors is not None:
        mat = mat * factors
    return oracle.Oracle(inst.tris, inst.rest, inst.pins, *mat, dt=w.dt, cg_tol=tol)


@functools.lru_cache(maxsize=16)
def _targets_cached(name, steps, idx):
    w = W.workload(name, steps=steps)
    inst = W.make_instances(w)[idx]
    o = oracle_for(inst, w, factors=inst.target_factors)
    frames = w.loss_frames()
    xo, _, _, _ = o.rollout(w.steps, inst.x0, inst.v0, inst.forces, frames)
    return xo


def targets(w, idx=0):
    """Reading R13: the oracle's rollout with (k_s, k_b, d) scaled by seeded U[0.5, 2]."""
    return _targets_cached(w.name, w.steps, idx)


def oracle_reference(w, inst, target, tol=1e-12):
    """Oracle positions at the loss frames and gradients of L = sum |x - target|^2."""
    o = oracle_for(inst, w, tol=tol)
    frames = w.loss_frames()
    xo, _, _, _ = o.rollout(w.steps, inst.x0, inst.v0, inst.forces, frames)
    g = o.gradient(w.steps, inst.x0, inst.v0, inst.forces, frames, 2.0 * (xo - target))
    g["x"] = xo
    g["loss"] = float(np.sum((xo - target) ** 2))
    return g


def gpu_run(sim, w, insts, targets_list, adjoint=True):
    """Rollout (+ adjoint) through the library for the concatenated instances."""
    import torch
    dev = torch.device("cuda:0")
    dt = sim.dtype
    x0 = torch.tensor(W.to_soa(np.concatenate([i.x0 for i in insts])), dtype=dt, device=dev)
    v0 = torch.tensor(W.to_soa(np.concatenate([i.v0 for i in insts])), dtype=dt, device=dev)
    F = None
    if insts[0].forces is not None:
        F = torch.tensor(W.to_soa(np.concatenate([i.forces for i in insts], axis=1)), dtype=dt,
                         device=dev)
    frames = w.loss_frames()
    xo = sim.rollout(w.steps, x0, v0, F, None, frames)
    out = dict(x=W.from_soa(xo.cpu().numpy().astype(np.float64)))
    if adjoint:
        tgt = torch.tensor(W.to_soa(np.concatenate(targets_list, axis=1)), dtype=dt, device=dev)
        g = sim.adjoint((2.0 * (xo - tgt)).contiguous())
        out.update({k: (None if v is None else v.cpu().numpy().astype(np.float64))
                    for k, v in g.items()})
        out["forces"] = W.from_soa(out["forces"]) if out["forces"] is not None else None
        out["x0"] = W.from_soa(out["x0"])
        out["v0"] = W.from_soa(out["v0"])
    st = sim.sync()
    out["status"] = st
    out["stats"] = sim.stats()
    return out


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))
