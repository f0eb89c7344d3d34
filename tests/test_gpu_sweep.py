"""Seeded parity sweep against the FP64 oracle over shapes and launch options.

Each case draws, from its seed: a sheet side n (5..30, so the sheets end in ragged
solver workgroups of 64..256 rows and in ragged coarse aggregates), a pin set, the
material (each scalar x U[0.5, 2] around the workload's) and the initial velocity
scale; the seed also picks the coarse aggregate size, rows per workgroup and the
matrix home the solver may use (the library's choice where that home cannot hold
the sheet's rows). Forces follow the 32x32 workload's recipe. Gates as for that
workload in FP64: positions 1e-9, gradients 1e-6 (relative, per block).
"""

import numpy as np
import pytest

from gpu_common import gpu_run, make_sim, note, oracle_for, rel
from paper_2203_11938_amd import workloads as W

pytestmark = pytest.mark.gpu


def case(seed):
    g = np.random.default_rng(1000 + seed)
    n = int(g.integers(5, 31))
    steps = 10
    rest, tris = W.grid_sheet(n)
    pins = W.pin_set(n, ["top2", "corner", "topedge"][seed % 3])
    base = np.array(W.Material().as_tuple())
    mat = W.Material(*(base * g.uniform(0.5, 2.0, size=3)))
    V = n * n
    forces = g.normal(0.0, 0.05, size=(steps, V, 3)) * (W.SHEET_SIDE ** 2 / V)
    v0 = g.normal(0.0, 0.02 * g.uniform(0.0, 1.0), size=(V, 3))
    v0[pins] = 0.0
    inst = W.Instance(rest, tris, pins, mat, rest.copy(), v0, forces, g.uniform(0.5, 2.0, size=3))
    # options by seed, so that the cases cover every aggregate size and home; a
    # workgroup may overlap at most four aggregates: rows <= 4 x the aggregate size
    coarse = [64, 32, 16, 0][seed % 4]
    rows = [r for r in (64, 128, 192, 256) if coarse == 0 or r <= 4 * coarse]
    opts = dict(rows_per_block=rows[(seed // 4 + seed) % len(rows)],
                matrix_home=["registers", "lds", "streamed"][(seed // 4) % 3],
                coarse_size=coarse)
    return inst, steps, opts


@pytest.mark.parametrize("seed", range(12))
def test_seeded_sweep_matches_oracle(seed):
    inst, steps, opts = case(seed)
    w = W.workload("C2", steps=steps, precision="fp64", cg_tol=1e-10)
    frames = w.loss_frames()
    o_t = oracle_for(inst, w, factors=inst.target_factors)
    tgt, _, _, _ = o_t.rollout(steps, inst.x0, inst.v0, inst.forces, frames)
    o = oracle_for(inst, w)
    xo, _, _, _ = o.rollout(steps, inst.x0, inst.v0, inst.forces, frames)
    ref = o.gradient(steps, inst.x0, inst.v0, inst.forces, frames, 2.0 * (xo - tgt))
    from paper_2203_11938_amd import sim
    try:
        s = make_sim(w, [inst], **opts)
    except sim.SimError as e:   # a home no launch shape of this sheet can use
        assert e.code == sim.SIM_E_INVALID, e
        opts["matrix_home"] = None
        s = make_sim(w, [inst], **opts)
    st = s.stats()
    out = gpu_run(s, w, [inst], [tgt])
    errs = dict(x=rel(out["x"], xo), forces=rel(out["forces"], ref["forces"]),
                x0=rel(out["x0"], ref["x0"]), v0=rel(out["v0"], ref["v0"]))
    for k in range(3):
        errs[f"mat{k}"] = abs(out["material"][0][k] - ref["material"][k]) / abs(ref["material"][k])
    note(f"sweep {seed}: {inst.n_verts} vertices, pins {len(inst.pins)}, options {opts}, "
         f"workgroups {st['blocks']}, home {st['solver_matrix_home']}: " +
         ", ".join(f"{k} {v:.1e}" for k, v in errs.items()))
    assert errs.pop("x") <= 1e-9
    for k, v in errs.items():
        assert v <= 1e-6, (seed, k, v)
    s.close()
