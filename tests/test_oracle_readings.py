"""Evidence for the readings of the synthetic force recipes (the oracle, CPU only).

The 32x32 recipe gives per-vertex, per-step forces N(0, 0.05^2). Taken literally as
nodal forces in N they push each 24 mg vertex at ~2000 m/s^2: after one 10 ms step
vertices move a quarter of the sheet's side, and by the third step the step matrix
with the exact membrane block is no longer positive definite (the oracle's CG breaks
down). Read as a load in N/m^2 on each vertex's area share (the reading the workloads
use), the same draws give a sheet that runs all 100 steps.
"""

import numpy as np

from paper_2203_11938_amd import workloads as W


def test_literal_nodal_forces_break_the_32x32_workload(oracle_mod):
    w = W.workload("C2")
    inst = W.make_instances(w)[0]
    literal = W.rng(w.number, 1).normal(0.0, w.force_sigma, size=(w.steps, inst.n_verts, 3))
    o = oracle_mod.Oracle(inst.tris, inst.rest, inst.pins, *inst.material.as_tuple(), dt=w.dt,
                          cg_tol=1e-10)
    xo, _, _, st = o.rollout(1, inst.x0, inst.v0, literal[:1], check=False)
    assert st == oracle_mod.ORC_OK
    assert np.abs(xo[-1] - inst.x0).max() > 0.25 * W.SHEET_SIDE / 2
    _, _, _, st = o.rollout(3, inst.x0, inst.v0, literal[:3], check=False)
    assert st == oracle_mod.ORC_E_INDEFINITE
    # the area-share reading of the same draws: a first step of about a millimetre (the
    # sheet starts to fall), and the whole rollout runs (the sheet swings down from its
    # two pinned corners, no vertex farther from its start than the sheet's diagonal)
    xo, _, _, st = o.rollout(1, inst.x0, inst.v0, inst.forces[:1], check=False)
    assert st == oracle_mod.ORC_OK and np.abs(xo[-1] - inst.x0).max() < 2e-3
    xo, _, _, st = o.rollout(w.steps, inst.x0, inst.v0, inst.forces, check=False)
    assert st == oracle_mod.ORC_OK and np.isfinite(xo).all()
    assert np.linalg.norm(xo[-1] - inst.x0, axis=1).max() < np.sqrt(2.0) * W.SHEET_SIDE
