"""GPU parity on edge cases and options, against the FP64 oracle on the same inputs.

Inputs are seeded and synthetic: caller vertex orders that are random permutations,
an irregular sheet (jittered rest positions, random cell diagonals), the smallest
meshes (one triangle, a 2x2 grid), a fully pinned sheet, a one-step rollout, a
rollout with no loss frames, a sheet whose rows fill the last workgroup only in part,
and the handle options (FP32 stored matrix, other aggregate sizes, the tension
membrane system, the solver's matrix homes). Gates: FP64 handles 1e-9 on
positions and 1e-6 on gradients (relative, per block), as for the 32x32 workload;
the FP32 stored matrix is held to the FP32 workload's 1e-5 and 1e-4.
"""

import dataclasses

import numpy as np
import pytest

from gpu_common import gpu_run, make_sim, note, oracle_for, rel
from paper_2203_11938_amd import workloads as W

pytestmark = pytest.mark.gpu


def relabel(inst, perm):
    """The same sheet with vertex i renamed perm[i]."""
    inv = np.argsort(perm)
    return dataclasses.replace(
        inst, rest=inst.rest[inv], x0=inst.x0[inv], v0=inst.v0[inv],
        tris=perm[inst.tris].astype(np.int32), pins=np.sort(perm[inst.pins]).astype(np.int32),
        forces=None if inst.forces is None else inst.forces[:, inv])


def irregular_sheet(n, seed):
    """An n x n sheet with rest positions jittered in the plane (0.2 of the spacing)
    and each cell split along a random diagonal (consistent orientation)."""
    g = np.random.default_rng(seed)
    rest, _ = W.grid_sheet(n)
    a = W.SHEET_SIDE / (n - 1)
    inner = np.ones(n * n, bool)
    idx = np.arange(n * n).reshape(n, n)
    inner[idx[0]] = inner[idx[-1]] = inner[idx[:, 0]] = inner[idx[:, -1]] = False
    rest = rest.copy()
    rest[inner, :2] += g.uniform(-0.2 * a, 0.2 * a, size=(inner.sum(), 2))
    tris = []
    for r in range(n - 1):
        for c in range(n - 1):
            v00, v01, v10, v11 = idx[r, c], idx[r, c + 1], idx[r + 1, c], idx[r + 1, c + 1]
            if g.random() < 0.5:
                tris += [(v00, v01, v11), (v00, v11, v10)]
            else:
                tris += [(v00, v01, v10), (v01, v11, v10)]
    return rest, np.array(tris, dtype=np.int32)


def instance(rest, tris, pins, steps, seed, sigma=0.05, material=W.Material()):
    g = np.random.default_rng(seed)
    V = rest.shape[0]
    forces = g.normal(0.0, sigma, size=(steps, V, 3)) * (W.SHEET_SIDE ** 2 / V)
    return W.Instance(rest, tris, np.asarray(pins, np.int32), material, rest.copy(),
                      np.zeros((V, 3)), forces, g.uniform(0.5, 2.0, size=3))


def reference(w, inst, membrane=None):
    """Oracle target (material scaled by the instance's factors), frames, gradients."""
    frames = w.loss_frames()
    o_t = oracle_for(inst, w, factors=inst.target_factors)
    o = oracle_for(inst, w)
    if membrane is not None:
        o_t.set_membrane_system(membrane)
        o.set_membrane_system(membrane)
    tgt, _, _, _ = o_t.rollout(w.steps, inst.x0, inst.v0, inst.forces, frames)
    xo, _, _, _ = o.rollout(w.steps, inst.x0, inst.v0, inst.forces, frames)
    g = o.gradient(w.steps, inst.x0, inst.v0, inst.forces, frames, 2.0 * (xo - tgt))
    g["x"] = xo
    return tgt, g


def check(out, ref, tol_x, tol_g, label):
    errs = dict(x=rel(out["x"], ref["x"]), forces=rel(out["forces"], ref["forces"]),
                x0=rel(out["x0"], ref["x0"]), v0=rel(out["v0"], ref["v0"]))
    for k in range(3):
        errs[f"mat{k}"] = (abs(out["material"][0][k] - ref["material"][k]) /
                           max(abs(ref["material"][k]), 1e-300))
    note(f"{label}: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()) +
         f"; cg iters fwd {out['stats']['cg_iters_forward']}")
    assert errs["x"] <= tol_x, (label, errs)
    for k, v in errs.items():
        if k != "x":
            assert v <= tol_g, (label, k, v)


def fp64(steps, **kw):
    return W.workload("C2", steps=steps, precision="fp64", cg_tol=1e-10, **kw)


def test_shuffled_caller_order():
    w = fp64(20)
    base = dataclasses.replace(W.make_instances(w)[0])
    perm = np.random.default_rng(11).permutation(base.n_verts).astype(np.int32)
    inst = relabel(base, perm)
    tgt, ref = reference(w, inst)
    out = gpu_run(make_sim(w, [inst]), w, [inst], [tgt])
    check(out, ref, 1e-9, 1e-6, "32x32 sheet, caller order a random permutation")


def test_irregular_sheet():
    w = fp64(25)
    rest, tris = irregular_sheet(14, 5)
    inst = instance(rest, tris, [13 * 14, 14 * 14 - 1], w.steps, 6)
    tgt, ref = reference(w, inst)
    out = gpu_run(make_sim(w, [inst]), w, [inst], [tgt])
    check(out, ref, 1e-9, 1e-6, "14x14 irregular sheet")


@pytest.mark.parametrize("kind", ["triangle", "grid2"])
def test_smallest_meshes(kind):
    w = fp64(15)
    if kind == "triangle":
        rest = np.array([[0.0, 0.0, 0.0], [0.3, 0.0, 0.0], [0.1, 0.25, 0.0]])
        tris = np.array([[0, 1, 2]], np.int32)
        pins = [0]
    else:
        rest, tris = W.grid_sheet(2)
        pins = []
    inst = instance(rest, tris, pins, w.steps, 7)
    tgt, ref = reference(w, inst)
    out = gpu_run(make_sim(w, [inst]), w, [inst], [tgt])
    check(out, ref, 1e-9, 1e-6, f"smallest mesh: {kind}")


def test_fully_pinned_sheet():
    w = fp64(10)
    rest, tris = W.grid_sheet(6)
    inst = instance(rest, tris, np.arange(36), w.steps, 8)
    inst = dataclasses.replace(inst, x0=inst.x0 + 0.01)
    tgt = inst.x0[None].repeat(w.steps, axis=0) + 0.003
    out = gpu_run(make_sim(w, [inst]), w, [inst], [tgt])
    # pins hold their start: every frame is x0, dL/dx0 sums the frames' gradients,
    # nothing else reaches the loss
    assert np.array_equal(out["x"], np.broadcast_to(inst.x0, out["x"].shape))
    assert np.allclose(out["x0"], (2.0 * (out["x"] - tgt)).sum(axis=0), rtol=1e-14, atol=0)
    assert np.all(out["v0"] == 0) and np.all(out["forces"] == 0)
    assert np.all(out["material"] == 0)


def test_one_step_and_no_loss_frames():
    import torch
    w = fp64(1)
    inst = W.make_instances(w)[0]
    tgt, ref = reference(w, inst)
    s = make_sim(w, [inst])
    out = gpu_run(s, w, [inst], [tgt])
    check(out, ref, 1e-9, 1e-6, "one step")
    # a rollout with no loss frames: the loss is zero, so is every gradient
    dev = torch.device("cuda:0")
    x0 = torch.tensor(W.to_soa(inst.x0), dtype=s.dtype, device=dev)
    F = torch.tensor(W.to_soa(inst.forces), dtype=s.dtype, device=dev)
    xo = s.rollout(1, x0, None, F, None, [])
    assert tuple(xo.shape) == (0, 3, inst.n_verts)
    g = s.adjoint(xo.clone())
    s.sync()
    for k, v in g.items():
        if v is not None:
            assert torch.count_nonzero(v).item() == 0, k


def test_fp32_stored_matrix():
    """The FP32 copy of A perturbs the solved system by ~6e-8 relative, the
    solution by up to cond(A) times that; on this sheet it still meets the FP32
    workload's gates (1e-5 positions, 1e-4 gradients; measured 1e-7 and 4e-5)."""
    w = W.workload("C2", steps=30)
    inst = W.make_instances(w)[0]
    inst = dataclasses.replace(inst, x0=inst.x0.astype(np.float32).astype(np.float64),
                               forces=inst.forces.astype(np.float32).astype(np.float64))
    tgt, ref = reference(w, inst)
    out = gpu_run(make_sim(w, [inst], matrix_precision="fp32"), w, [inst], [tgt])
    check(out, ref, 1e-5, 1e-4, "32x32 sheet, FP32 stored matrix")


@pytest.mark.parametrize("agg", [16, 32, 128])
def test_other_aggregate_sizes(agg):
    w = fp64(20)
    inst = W.make_instances(w)[0]
    tgt, ref = reference(w, inst)
    s = make_sim(w, [inst], coarse_size=agg)
    note(f"aggregates of {agg}: {s.stats()['coarse_aggregates']} aggregates")
    out = gpu_run(s, w, [inst], [tgt])
    check(out, ref, 1e-9, 1e-6, f"aggregates of {agg}")


def test_tension_membrane_system():
    """The tension-clamped membrane block is not differentiable where a principal
    strain is zero, which every strain of the flat rest state is, and its derivatives
    are ill-conditioned where the two principal strains coincide: the start is the
    rest shape stretched by 0.1% along x and 0.2% along y, so the clamp starts on its
    smooth side with distinct principal strains."""
    import oracle
    w = fp64(25)
    inst = W.make_instances(w)[0]
    x0 = inst.x0.copy()
    x0[:, 0] *= 1.001
    x0[:, 1] *= 1.002
    inst = dataclasses.replace(inst, x0=x0)
    tgt, ref = reference(w, inst, membrane=oracle.Oracle.MEMBRANE_TENSION)
    out = gpu_run(make_sim(w, [inst], membrane="tension"), w, [inst], [tgt])
    check(out, ref, 1e-9, 1e-6, "tension membrane system")


def test_matrix_home_on_rows_of_more_than_13_blocks():
    """The irregular sheet couples up to 17 vertices in a row: the register-resident
    home is refused at creation (SIM_E_INVALID), the library's choice falls back to
    another home, and the streamed and LDS homes agree bit for bit and with the
    oracle."""
    from paper_2203_11938_amd import sim
    w = fp64(15)
    rest, tris = irregular_sheet(14, 5)
    inst = instance(rest, tris, [13 * 14, 14 * 14 - 1], w.steps, 6)
    with pytest.raises(sim.SimError) as err:
        make_sim(w, [inst], matrix_home="registers")
    assert err.value.code == sim.SIM_E_INVALID
    s = make_sim(w, [inst])
    assert s.stats()["solver_matrix_home"] in (1, 2)
    s.close()
    tgt, ref = reference(w, inst)
    outs = {h: gpu_run(make_sim(w, [inst], matrix_home=h, rows_per_block=64), w, [inst], [tgt])
            for h in ("streamed", "lds")}
    for k in ("x", "forces", "x0", "v0", "material"):
        assert np.array_equal(outs["lds"][k], outs["streamed"][k]), k
    check(outs["lds"], ref, 1e-9, 1e-6, "14x14 irregular sheet, LDS and streamed homes")


@pytest.mark.parametrize("rows,matrix", [(64, "fp64"), (128, "fp64"), (128, "fp32")])
def test_split_register_rows_on_a_ragged_sheet(rows, matrix):
    """A 27x27 sheet (729 vertices): the last workgroup holds only part of its rows
    and the last run of the middle level is short. Register rows on two wavefront
    teams (the second team's threads of missing rows hold nothing) agree bit for bit
    with streamed rows at the same launch shape, and with the oracle (an FP32 stored
    matrix at the FP32 matrix's gates, 1e-5 and 1e-4)."""
    w = fp64(15)
    rest, tris = W.grid_sheet(27)
    inst = instance(rest, tris, [26 * 27, 27 * 27 - 1], w.steps, 8)
    tgt, ref = reference(w, inst)
    outs = {}
    for h in ("streamed", "registers"):
        s = make_sim(w, [inst], matrix_home=h, rows_per_block=rows, matrix_precision=matrix)
        st = s.stats()
        assert st["rows_per_block"] == rows
        assert st["solver_row_teams"] == (2 if h == "registers" else 1)
        outs[h] = gpu_run(s, w, [inst], [tgt])
    for k in ("x", "forces", "x0", "v0", "material"):
        assert np.array_equal(outs["registers"][k], outs["streamed"][k]), (rows, matrix, k)
    tol_x, tol_g = (1e-9, 1e-6) if matrix == "fp64" else (1e-5, 1e-4)
    check(outs["registers"], ref, tol_x, tol_g,
          f"27x27 sheet, {rows} register rows on two teams, {matrix} matrix")


def test_rows_per_block_the_coarse_space_cannot_use():
    """A workgroup may overlap at most four coarse aggregates: 256 rows per workgroup
    with 16-vertex aggregates is refused at creation (SIM_E_INVALID), and the same
    aggregates with 64 rows work."""
    from paper_2203_11938_amd import sim
    w = fp64(5)
    inst = W.make_instances(w)[0]
    with pytest.raises(sim.SimError) as err:
        make_sim(w, [inst], rows_per_block=256, coarse_size=16)
    assert err.value.code == sim.SIM_E_INVALID
    s = make_sim(w, [inst], rows_per_block=64, coarse_size=16)
    assert s.stats()["rows_per_block"] == 64
    s.close()
