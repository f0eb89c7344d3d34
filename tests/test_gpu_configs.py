"""Full-size GPU checks of the checkpointed, batched and large workloads.

The oracle cannot run these rollouts end to end in seconds, so they are checked
through outputs the oracle computes one by one and through identities that hold
at any size:
  * single steps: the GPU state after step s-1 (read back through extra output
    frames, FP64 I/O so that v = (x_s - x_{s-1})/h is the state's own velocity)
    is advanced by the oracle and compared with the GPU's step s;
  * segment adjoint: dL/dF of the last steps depends only on those steps, so it
    must equal the oracle's adjoint of that segment started from the GPU state;
  * scale homogeneity: scaling (k_s, k_b, d, F) by c scales both sides of the
    step's linear system (Eq. 4) by c, so the trajectory does not change and
    k_s dL/dk_s + k_b dL/dk_b + d dL/dd + <F, dL/dF> = 0;
  * translation: moving x0 (pins included) by c moves every frame by c, so
    sum_i dL/dx0_i = sum over frames and vertices of dL/dx_s.
Members of the batch are compared with the oracle end to end.
"""

import time

import numpy as np
import pytest

import oracle
from gpu_common import as_given, gpu_run, make_sim, note, oracle_for, oracle_reference, rel
from paper_2203_11938_amd import workloads as W

pytestmark = pytest.mark.gpu


def random_targets(w, inst, frames):
    g = W.rng(w.number, 4)
    return inst.x0[None] + 0.01 * g.normal(size=(len(frames),) + inst.x0.shape)


def run_with_frames(w, inst, extra, target, **kw):
    """GPU rollout + adjoint of L = sum over the loss frames of |x - target|^2, with
    extra output frames (zero loss gradient) from which states are read back."""
    import torch
    tf = list(w.loss_frames())
    frames = np.unique(np.concatenate([tf, np.asarray(extra, np.int32)])).astype(np.int32)
    s = make_sim(w, [inst], **kw)
    dev = torch.device("cuda:0")
    dt = s.dtype
    x0 = torch.tensor(W.to_soa(inst.x0), dtype=dt, device=dev)
    v0 = torch.tensor(W.to_soa(inst.v0), dtype=dt, device=dev)
    F = None if inst.forces is None else torch.tensor(W.to_soa(inst.forces), dtype=dt, device=dev)
    t0 = time.time()
    xo = s.rollout(w.steps, x0, v0, F, None, frames)
    s.sync()
    note(f"{w.name}: GPU rollout of {w.steps} steps took {time.time() - t0:.1f} s "
         f"({s.stats()['cg_iters_forward']} CG iterations)")
    x = W.from_soa(xo.cpu().numpy().astype(np.float64))
    dl = np.zeros_like(x)
    for k, f in enumerate(frames):
        if f in tf:
            dl[k] = 2.0 * (x[k] - target[tf.index(f)])
    t0 = time.time()
    g = s.adjoint(torch.tensor(W.to_soa(dl), dtype=dt, device=dev))
    s.sync()
    note(f"{w.name}: GPU adjoint took {time.time() - t0:.1f} s")
    out = dict(x={int(f): x[k] for k, f in enumerate(frames)}, dl=dl, stats=s.stats(),
               material=g["material"].cpu().numpy()[0],
               forces=W.from_soa(g["forces"].cpu().numpy().astype(np.float64)),
               x0=W.from_soa(g["x0"].cpu().numpy().astype(np.float64)))
    s.close()
    return out


def state_at(out, inst, s, h):
    """(x_s, v_s) from the output frames (s = 0: the initial state)."""
    if s == 0:
        return inst.x0, inst.v0
    xp = out["x"][s - 1] if s > 1 else inst.x0
    return out["x"][s], (out["x"][s] - xp) / h


def check_single_steps(w, inst, out, samples, cg_tol, oracle_tol):
    """The GPU's increment dv of step s solves the oracle's step system to the
    GPU's CG tolerance (convergence is accepted on the true residual), and the
    GPU's x_s agrees with the oracle's own step from the same state."""
    o = oracle_for(inst, w, tol=oracle_tol)
    for s in samples:
        x, v = state_at(out, inst, s - 1, w.dt)
        F = None if inst.forces is None else inst.forces[s - 1]
        _, v_s = state_at(out, inst, s, w.dt)
        r, bn, st = o.step_residual(x, v, F, v_s - v)
        assert st == oracle.ORC_OK
        res = np.linalg.norm(r) / bn
        xs, _, _, it, st = o.step(x, v, F)
        assert st == oracle.ORC_OK
        e_inc = rel(out["x"][s] - x, xs - x)
        e_pos = rel(out["x"][s], xs)
        note(f"{w.name} step {s}: relative residual of the GPU increment in the oracle's "
             f"system {res:.2e} (CG tol {cg_tol:.0e}); position rel err {e_pos:.2e}, "
             f"increment rel err {e_inc:.2e} (oracle CG iters {it})")
        assert res <= 1.5 * cg_tol
        assert e_pos <= 1e-6
        assert e_inc <= 1e-3


def check_identities(w, inst, out, tol):
    terms = list(np.array(inst.material.as_tuple()) * out["material"])
    if inst.forces is not None:
        terms.append(float(np.sum(inst.forces * out["forces"])))
    terms = np.array(terms)
    hom = abs(terms.sum()) / np.abs(terms).max()
    tr = rel(out["x0"].sum(axis=0), out["dl"].sum(axis=(0, 1)))
    note(f"{w.name}: homogeneity residual {hom:.2e} (terms {np.array2string(terms, precision=3)}), "
         f"translation identity rel err {tr:.2e}")
    assert hom <= tol
    assert tr <= tol


def check_segment_adjoint(w, inst, out, k, target, tol, oracle_tol):
    """dL/dF of the last k steps against the oracle's adjoint of that segment."""
    s0 = w.steps - k
    x, v = state_at(out, inst, s0, w.dt)
    tf = list(w.loss_frames())
    seg = [f for f in tf if f > s0]
    dl = np.array([2.0 * (out["x"][f] - target[tf.index(f)]) for f in seg])
    o = oracle_for(inst, w, tol=oracle_tol)
    F = None if inst.forces is None else inst.forces[s0:]
    g = o.gradient(k, x, v, F, np.array(seg, np.int32) - s0, dl)
    e = rel(out["forces"][s0:], g["forces"])
    note(f"{w.name}: dL/dF of the last {k} steps vs the oracle's segment adjoint: rel err {e:.2e}")
    assert e <= tol


def test_c3_checkpointed_full_size():
    w = W.workload("C3")
    inst = W.make_instances(w)[0]
    target = random_targets(w, inst, w.loss_frames())
    note("C3: 64x64, 200 steps of 5 ms, corner pin, checkpoint every 20, loss every 10th frame")
    samples = [1, 2, 100, 161, 200]
    # step s is checked from (x_{s-1}, v_{s-1}), and v_{s-1} needs x_{s-2}
    extra = sorted({q for s in samples for q in (s - 2, s - 1, s) if q >= 1} | {194, 195})
    out = run_with_frames(w, inst, extra, target, precision="fp64")
    st = out["stats"]
    note(f"C3: cg iters fwd {st['cg_iters_forward']} recompute {st['cg_iters_recompute']} "
         f"adj {st['cg_iters_adjoint']}")
    assert st["cg_iters_recompute"] > 0
    check_single_steps(w, inst, out, samples, w.cg_tol, oracle_tol=1e-10)
    check_identities(w, inst, out, tol=1e-4)
    check_segment_adjoint(w, inst, out, 5, target, tol=1e-4, oracle_tol=1e-10)


def test_c4_batched_members_match_oracle():
    w = W.workload("C4")
    insts = [as_given(i, w.precision) for i in W.make_instances(w)]
    nv = [i.n_verts for i in insts]
    note(f"C4: {len(insts)} sheets ({min(nv)}..{max(nv)} vertices, {sum(nv)} in all), "
         f"{w.steps} steps, one handle")
    # the two smallest sheets and the one nearest 30x30 (the oracle runs them in seconds)
    members = [int(b) for b in np.argsort(nv)[:2]] + [int(np.argmin(np.abs(np.array(nv) - 900)))]
    tgts = []
    for b, inst in enumerate(insts):
        if b in members:
            o = oracle_for(inst, w, factors=inst.target_factors)
            xo, _, _, _ = o.rollout(w.steps, inst.x0, inst.v0, inst.forces)
            tgts.append(xo)
        else:
            tgts.append(inst.x0[None].repeat(w.steps, axis=0) + 0.01)
    s = make_sim(w, insts)
    import torch
    dev = torch.device("cuda:0")
    dt = s.dtype
    x0 = torch.tensor(W.to_soa(np.concatenate([i.x0 for i in insts])), dtype=dt, device=dev)
    F = torch.tensor(W.to_soa(np.concatenate([i.forces for i in insts], axis=1)), dtype=dt,
                     device=dev)
    xo = s.rollout(w.steps, x0, None, F)
    tgt = torch.tensor(W.to_soa(np.concatenate(tgts, axis=1)), dtype=dt, device=dev)
    g = s.adjoint((2.0 * (xo - tgt)).contiguous())
    status = s.status()
    inst_status = s.instance_status()
    st = s.stats()
    note(f"C4: handle status {status}, solver launches per solve "
         f"{st['solver_launches_per_solve']}, blocks {st['blocks']}, rows {st['rows_per_block']}, "
         f"matrix home {st['solver_matrix_home']}")
    broken = [b for b in range(len(insts)) if inst_status[b] != 0]
    note(f"C4: sheets whose step matrix stopped being positive definite: {broken}")
    # a breakdown is the method's own (the exact membrane block is indefinite under
    # compression): the oracle must report it for the same sheet
    for b in broken:
        o = oracle_for(insts[b], w, tol=w.cg_tol)
        _, _, _, ost = o.rollout(w.steps, insts[b].x0, None, insts[b].forces, check=False)
        assert ost in (oracle.ORC_E_INDEFINITE, oracle.ORC_E_NOT_CONVERGED), (b, ost)
    x = W.from_soa(xo.cpu().numpy().astype(np.float64))
    gm = g["material"].cpu().numpy()
    gF = W.from_soa(g["forces"].cpu().numpy().astype(np.float64))
    gx0 = W.from_soa(g["x0"].cpu().numpy().astype(np.float64))
    off = np.concatenate([[0], np.cumsum(nv)])
    healthy = np.ones(off[-1], dtype=bool)
    for b in broken:
        healthy[off[b]:off[b + 1]] = False
    assert np.isfinite(x[:, healthy]).all() and np.isfinite(gF[:, healthy]).all()
    for b in members:
        assert inst_status[b] == 0
        inst = insts[b]
        ref = oracle_reference(w, inst, tgts[b])
        sl = slice(off[b], off[b + 1])
        ex = rel(x[:, sl], ref["x"])
        em = np.abs(gm[b] - ref["material"]) / np.abs(ref["material"])
        eF = rel(gF[:, sl], ref["forces"])
        ex0 = rel(gx0[sl], ref["x0"])
        note(f"C4 sheet {b} ({inst.n_verts} vertices): positions {ex:.2e}, material "
             f"{np.array2string(em, precision=2)}, forces {eF:.2e}, x0 {ex0:.2e}")
        assert ex <= 1e-6
        assert em.max() <= 1e-4 and eF <= 1e-4 and ex0 <= 1e-4
    s.close()


def test_c4_tension_variant_runs_every_sheet():
    w = W.workload("C4", steps=30)
    insts = [as_given(i, w.precision) for i in W.make_instances(w)]
    note(f"C4 (tension-clamped membrane block): {len(insts)} sheets, {w.steps} steps")
    s = make_sim(w, insts, membrane="tension")
    tgts = [i.x0[None].repeat(w.steps, axis=0) + 0.01 for i in insts]
    out = gpu_run(s, w, insts, tgts)
    assert out["status"] == 0
    assert (s.instance_status() == 0).all()
    assert np.isfinite(out["x"]).all() and np.isfinite(out["forces"]).all()
    s.close()


def test_c5_large_sheet_full_size():
    w = W.workload("C5")
    inst = W.make_instances(w)[0]
    target = random_targets(w, inst, w.loss_frames())
    note("C5: 200x200, 300 steps of 5 ms, top edge pinned, Fourier wind, checkpoint every 30")
    out = run_with_frames(w, inst, [1, 298, 299, 300], target, precision="fp64")
    st = out["stats"]
    note(f"C5: cg iters fwd {st['cg_iters_forward']} recompute {st['cg_iters_recompute']} "
         f"adj {st['cg_iters_adjoint']}, blocks {st['blocks']}, rows {st['rows_per_block']}, "
         f"matrix home {st['solver_matrix_home']}")
    check_single_steps(w, inst, out, [1, 300], w.cg_tol, oracle_tol=1e-9)
    check_identities(w, inst, out, tol=1e-4)
    check_segment_adjoint(w, inst, out, 1, target, tol=1e-4, oracle_tol=1e-9)
