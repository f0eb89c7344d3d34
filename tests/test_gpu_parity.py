"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (stated per test): positions after the full rollout <= 1e-5 relative
and gradients <= 1e-4 relative per block for FP32 (CG tol 1e-7, FP64 solver
vectors and reductions); the FP64 build is held to tighter bounds, which
separates arithmetic from bugs.
"""

import numpy as np
import pytest

from gpu_common import as_given, gpu_run, make_sim, note, oracle_reference, rel, targets
from paper_2203_11938_amd import workloads as W

pytestmark = pytest.mark.gpu


def check_grads(g, ref, tol, label):
    errs = {}
    for k in range(3):
        errs[f"mat{k}"] = abs(g["material"][0][k] - ref["material"][k]) / abs(ref["material"][k])
    errs["forces"] = rel(g["forces"], ref["forces"]) if ref.get("forces") is not None else 0.0
    errs["x0"] = rel(g["x0"], ref["x0"])
    errs["v0"] = rel(g["v0"], ref["v0"])
    note(f"{label}: gradient rel errors " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= tol, (label, k, v)


def test_c1_fp64_rollout():
    w = W.workload("C1")
    inst = W.make_instances(w)[0]
    note("C1: 10x10, 50 steps, fp64, tol 1e-10")
    tgt = targets(w)
    ref = oracle_reference(w, inst, tgt)
    s = make_sim(w, [inst])
    out = gpu_run(s, w, [inst], [tgt])
    e = rel(out["x"][-1], ref["x"][-1])
    loss = float(np.sum((out["x"] - tgt) ** 2))
    note(f"C1: final position rel err {e:.2e}, loss {loss:.6e} vs {ref['loss']:.6e}, "
         f"cg iters fwd {out['stats']['cg_iters_forward']}")
    assert e <= 1e-9
    assert abs(loss - ref["loss"]) <= 1e-8 * ref["loss"]
    check_grads(out, ref, 1e-7, "C1 fp64")


@pytest.mark.parametrize("precision,tol_x,tol_g", [("fp64", 1e-9, 1e-7), ("fp32", 1e-5, 1e-4)])
def test_c2_parity(precision, tol_x, tol_g):
    w = W.workload("C2", precision=precision)
    inst = as_given(W.make_instances(w)[0], precision)
    note(f"C2: 32x32, 100 steps, {precision}")
    tgt = targets(w)
    ref = oracle_reference(w, inst, tgt)
    s = make_sim(w, [inst], cg_tol=1e-10 if precision == "fp64" else 1e-7)
    out = gpu_run(s, w, [inst], [tgt])
    e = rel(out["x"][-1], ref["x"][-1])
    disp = rel(out["x"][-1], ref["x"][-1]) * np.linalg.norm(ref["x"][-1]) / np.linalg.norm(
        ref["x"][-1] - inst.x0)
    note(f"C2 {precision}: final position rel err {e:.2e} (vs displacement {disp:.2e}), "
         f"cg iters fwd {out['stats']['cg_iters_forward']} adj {out['stats']['cg_iters_adjoint']}")
    assert e <= tol_x
    check_grads(out, ref, tol_g, f"C2 {precision}")


def test_determinism_bitwise():
    w = W.workload("C2", steps=30)
    inst = W.make_instances(w)[0]
    note("determinism: C2 shape, 30 steps, two runs")
    tgt = inst.x0[None].repeat(30, axis=0)
    s = make_sim(w, [inst])
    a = gpu_run(s, w, [inst], [tgt])
    b = gpu_run(s, w, [inst], [tgt])
    for k in ("x", "forces", "x0", "v0", "material"):
        assert np.array_equal(a[k], b[k]), k


def test_checkpoint_recompute_is_bitwise_store_all():
    w = W.workload("C3", steps=40, checkpoint_every=0)
    inst = W.make_instances(w)[0]
    note("checkpoint: 64x64, 40 steps, store-all vs every 20 vs every 7")
    tgt = inst.x0[None].repeat(len(w.loss_frames()), axis=0) + 0.01
    a = gpu_run(make_sim(w, [inst]), w, [inst], [tgt])
    for k in (20, 7):
        b = gpu_run(make_sim(w, [inst], checkpoint_every=k), w, [inst], [tgt])
        assert b["stats"]["cg_iters_recompute"] > 0
        for key in ("x", "forces", "x0", "v0", "material"):
            assert np.array_equal(a[key], b[key]), (k, key)


def test_batch_matches_single_instances():
    w = W.workload("C4", steps=15, batch=4, batch_n_range=(16, 40))
    insts = W.make_instances(w)
    note("batch: 4 sheets (16..40 per side), 15 steps, batched vs one by one")
    tgts = [i.x0[None].repeat(w.steps, axis=0) + 0.02 for i in insts]
    # the same rows per solver workgroup on both sides, so that every reduction of a
    # sheet runs over the same partition
    batched = gpu_run(make_sim(w, insts, rows_per_block=128), w, insts, tgts)
    off = np.concatenate([[0], np.cumsum([i.n_verts for i in insts])])
    for b, inst in enumerate(insts):
        single = gpu_run(make_sim(w, [inst], rows_per_block=128), w, [inst], [tgts[b]])
        sl = slice(off[b], off[b + 1])
        assert np.array_equal(batched["x"][:, sl], single["x"]), b
        assert np.array_equal(batched["forces"][:, sl], single["forces"]), b
        assert np.array_equal(batched["x0"][sl], single["x0"]), b
        assert np.array_equal(batched["material"][b], single["material"][0]), b


@pytest.mark.parametrize("coarse_size,rows", [(64, 128), (0, 128), (64, 256)])
def test_matrix_homes_are_bitwise_equal(coarse_size, rows):
    """Streamed, LDS-resident and register-resident matrix rows feed the same
    products in the same order: at the same launch shape (rows per workgroup, one
    workgroup per CU) the rollout and every gradient agree bit for bit; the
    register-resident run also meets the FP64 gates against the oracle. Register
    rows of 128-row workgroups run over two wavefront teams (each multiplies one of
    the row's two slot ranges); those of 256-row workgroups on one (whose FP64 rows do
    not fit in LDS: streamed and registers only)."""
    w = W.workload("C2", steps=20, precision="fp64", cg_tol=1e-10)
    inst = W.make_instances(w)[0]
    tgt = inst.x0[None].repeat(w.steps, axis=0) + 0.01
    outs = {}
    homes = ("streamed", "lds", "registers") if rows <= 128 else ("streamed", "registers")
    for home in homes:
        s = make_sim(w, [inst], rows_per_block=rows, matrix_home=home, coarse_size=coarse_size)
        st = s.stats()
        assert st["solver_matrix_home"] == ("auto", "streamed", "lds", "registers").index(home)
        assert st["rows_per_block"] == rows
        assert st["solver_row_teams"] == (2 if home == "registers" and rows <= 128 else 1)
        outs[home] = gpu_run(s, w, [inst], [tgt])
        note(f"matrix home {home} (coarse {coarse_size}, rows {rows}): workgroups per CU "
             f"{st['solver_wg_per_cu']}, row teams {st['solver_row_teams']}, "
             f"cg iters fwd {outs[home]['stats']['cg_iters_forward']}")
    for home in homes[1:]:
        for k in ("x", "forces", "x0", "v0", "material"):
            assert np.array_equal(outs[home][k], outs["streamed"][k]), (home, k)
    ref = oracle_reference(w, inst, tgt)
    assert rel(outs["registers"]["x"][-1], ref["x"][-1]) <= 1e-9
    check_grads(outs["registers"], ref, 1e-6, f"registers (coarse {coarse_size}, rows {rows})")


def test_autotuned_handle_matches_oracle():
    """The measuring autotuner only changes the solver's launch shape: results stay
    within the parity gates of the 32x32 workload."""
    w = W.workload("C2", steps=30)
    inst = as_given(W.make_instances(w)[0], w.precision)
    tgt = targets(w)
    s = make_sim(w, [inst], autotune=True)
    st = s.stats()
    note(f"autotune: {st['autotune_candidates']} launch shapes timed, chose rows "
         f"{st['rows_per_block']} (matrix home {st['solver_matrix_home']}), "
         f"{1e3 * st['autotune_ms_per_iter']:.1f} us per CG iteration")
    assert st["autotuned"] == 1 and st["autotune_candidates"] > 1
    out = gpu_run(s, w, [inst], [tgt])
    ref = oracle_reference(w, inst, tgt)
    assert rel(out["x"][-1], ref["x"][-1]) <= 1e-5
    assert rel(out["forces"], ref["forces"]) <= 1e-4
    assert rel(out["x0"], ref["x0"]) <= 1e-4
    s.close()


def test_block_jacobi_only_matches_oracle():
    """The solver without its coarse space (coarse_size 0) meets the same gates."""
    w = W.workload("C2", steps=30)
    inst = as_given(W.make_instances(w)[0], w.precision)
    tgt = targets(w)
    s = make_sim(w, [inst], coarse_size=0)
    assert s.stats()["coarse_aggregates"] == 0
    out = gpu_run(s, w, [inst], [tgt])
    ref = oracle_reference(w, inst, tgt)
    note(f"block-Jacobi only: cg iters fwd {out['stats']['cg_iters_forward']}")
    assert rel(out["x"][-1], ref["x"][-1]) <= 1e-5
    assert rel(out["forces"], ref["forces"]) <= 1e-4
    assert rel(out["x0"], ref["x0"]) <= 1e-4
    s.close()


def test_coarse_space_cuts_iterations():
    """The coarse level, whose inverse the one-launch sweep forms every step, is what
    takes a 64x64 step from ~1,300 block-Jacobi CG iterations to ~110: a wrong,
    inaccurate or disabled coarse inverse shows up as several times more iterations
    (the true-residual test keeps the answers right either way, so parity alone would
    not see it)."""
    import torch
    w = W.workload("H", steps=8)
    inst = W.make_instances(w)[0]
    dev = torch.device("cuda:0")
    its = {}
    for cs in (64, 0):
        s = make_sim(w, [inst], coarse_size=cs)
        x0 = torch.tensor(W.to_soa(inst.x0), dtype=s.dtype, device=dev)
        F = torch.tensor(W.to_soa(inst.forces[:w.steps]), dtype=s.dtype, device=dev)
        s.rollout(w.steps, x0, None, F, None, np.array([w.steps], np.int32))
        assert s.status() == 0
        its[cs] = float(s.cg_iters()[0].mean())
        s.close()
    note(f"64x64 sheet, {w.steps} steps: CG iterations per solve {its[64]:.0f} with the coarse "
         f"space, {its[0]:.0f} block-Jacobi only")
    assert its[64] <= 150
    assert its[0] >= 5 * its[64]
