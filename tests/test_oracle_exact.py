"""Pins of the oracle's exact-solve driver (the golden-file generator's path).

The driver solves each step of Eq. 4-5 with scipy's sparse LU instead of the
oracle's CG, then runs the oracle's own backward step (orc_adjoint_rhs,
orc_adjoint_update) around an exact solve of A(x_{s-1}) mu = u. It must agree
with the CG-based oracle, which the brute-force finite differences of
test_oracle_adjoint.py pin, and its assembled system must be the dense one.
"""

import numpy as np

from paper_2203_11938_amd import workloads as W


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def test_sparse_system_equals_dense_system(oracle_mod):
    rest, tris = W.grid_sheet(5)
    o = oracle_mod.Oracle(tris, rest, W.pin_set(5, "top2"), 300.0, 1e-3, 0.2, dt=0.01)
    g = np.random.default_rng(3)
    x = rest + 0.02 * g.normal(size=rest.shape)
    v = 0.1 * g.normal(size=rest.shape)
    F = 0.01 * g.normal(size=rest.shape)
    A, b = o.system_sparse(x, v, F)
    Ad, bd = o.system(x, v, F)
    assert np.array_equal(A.toarray(), Ad)
    assert np.array_equal(b, bd)


def test_exact_driver_matches_cg_oracle_on_3x3(oracle_mod):
    rest, tris = W.grid_sheet(3)
    o = oracle_mod.Oracle(tris, rest, W.pin_set(3, "top2"), 60.0, 2e-3, 0.2, dt=0.01,
                          cg_tol=1e-14)
    g = np.random.default_rng(0)
    steps = 6
    x0 = rest + 0.02 * g.normal(size=rest.shape)
    v0 = 0.2 * g.normal(size=rest.shape)
    F = 0.02 * g.normal(size=(steps, 9, 3))
    frames = np.array([2, 4, 6], np.int32)
    target = x0[None] + 0.05 * g.normal(size=(3, 9, 3))
    xo, _, _, _ = o.rollout(steps, x0, v0, F, frames)
    ref = o.gradient(steps, x0, v0, F, frames, 2.0 * (xo - target))
    ex = o.gradient_exact(steps, x0, v0, F, frames, target)
    assert rel(ex["x"], xo) <= 1e-13
    for k in ("material", "forces", "x0", "v0"):
        assert rel(ex[k], ref[k]) <= 1e-10, k


def test_exact_driver_matches_cg_oracle_on_32x32_prefix(oracle_mod):
    w = W.workload("C2", steps=12)
    inst = W.make_instances(w)[0]
    o = oracle_mod.Oracle(inst.tris, inst.rest, inst.pins, *inst.material.as_tuple(), dt=w.dt,
                          cg_tol=1e-13)
    frames = np.array([4, 8, 12], np.int32)
    target = W.loss_targets(w, inst, frames)
    xo, _, _, _ = o.rollout(w.steps, inst.x0, inst.v0, inst.forces, frames)
    ref = o.gradient(w.steps, inst.x0, inst.v0, inst.forces, frames, 2.0 * (xo - target))
    ex = o.gradient_exact(w.steps, inst.x0, inst.v0, inst.forces, frames, target)
    assert rel(ex["x"], xo) <= 1e-11
    for k in ("material", "forces", "x0", "v0"):
        assert rel(ex[k], ref[k]) <= 1e-8, k
