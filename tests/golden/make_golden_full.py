"""Writes the full-size oracle golden files of the 64x64 checkpointed (C3), batched (C4)
and 200x200 (C5) workloads. Calls only oracle/ and the seeded input generators.

Each step of Eq. 4-5 is solved exactly (sparse LU with one refinement step, the
oracle's exact-solve driver) instead of by the oracle's CG, whose block-Jacobi
iterations would take hours on the 200x200 sheet; the backward sweep is the
oracle's own (implicit differentiation of Eq. 4). Inputs are the FP32-rounded
arrays an FP32 handle receives; the loss is L = sum over the loss frames of
|x_s - target_s|^2 with seeded targets (workloads.loss_targets).

    python tests/golden/make_golden_full.py c3
    python tests/golden/make_golden_full.py c4 --workers 4
    python tests/golden/make_golden_full.py c4t --workers 4
    python tests/golden/make_golden_full.py c5 --workers 6

Large intermediates (the 200x200 trajectory) go to --scratch (default
/tmp/phisft_golden), never into the repository.
"""

import argparse
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2203_11938_amd import workloads as W  # noqa: E402

SOLVER = ("FP64 oracle, each step solved exactly (scipy sparse LU + one refinement "
          "step), backward sweep orc_adjoint_rhs / orc_adjoint_update (Sec. 3.1, Eq. 1-5 "
          "and the backward pass; readings R1-R18)")


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def f32(a):
    return np.asarray(a, dtype=np.float32)


def make_oracle(inst, w):
    return oracle.Oracle(inst.tris, inst.rest, inst.pins, *inst.material.as_tuple(), dt=w.dt)


# ------------------------------------------------------------------ one sheet
def sheet_gradient(w, inst, targets, frames):
    o = make_oracle(inst, w)
    t0 = time.time()
    g = o.gradient_exact(w.steps, inst.x0, inst.v0, inst.forces, frames, targets)
    g["seconds"] = time.time() - t0
    return g


def c3(args):
    w = W.workload("C3")
    inst = W.as_given(W.make_instances(w)[0], w.precision)
    frames = w.loss_frames()
    targets = W.loss_targets(w, inst, frames)
    log(f"C3: 64x64, {w.steps} steps")
    g = sheet_gradient(w, inst, targets, frames)
    keep_frames = np.array([10, 100, 200], np.int32)
    keep_steps = np.array([1, 20, 21, 100, 181, 200], np.int32)
    out = dict(source=SOLVER, workload="C3", steps=w.steps, seconds=g["seconds"],
               loss_frames=frames, x_frames=keep_frames,
               x=f32(g["x"][[list(frames).index(f) for f in keep_frames]]),
               loss=g["loss"], material=g["material"], dl_dx0=f32(g["x0"]),
               dl_dv0=f32(g["v0"]), dl_dF_steps=keep_steps,
               dl_dF=f32(g["forces"][keep_steps - 1]),
               dl_dF_norms=np.linalg.norm(g["forces"].reshape(w.steps, -1), axis=1))
    path = os.path.join(HERE, "c3_oracle.npz")
    np.savez_compressed(path, **out)
    log(f"wrote {path} ({g['seconds']:.0f} s of oracle time)")


# ------------------------------------------------------------- batched sheets
def c4t_sheet(b):
    """A sheet of the batched workload under the tension-clamped membrane system
    (the recorded variant of reading R9, SPD in every state)."""
    w = W.workload("C4")
    inst = W.as_given(W.make_instances(w)[b], w.precision)
    frames = w.loss_frames()
    o = make_oracle(inst, w)
    o.set_membrane_system(oracle.Oracle.MEMBRANE_TENSION)
    t0 = time.time()
    g = o.gradient_exact(w.steps, inst.x0, inst.v0, inst.forces, frames,
                         W.loss_targets(w, inst, frames, sheet=b))
    return dict(sheet=b, nv=inst.n_verts, x=g["x"][-1], material=g["material"], dl_dx0=g["x0"],
                dl_dF_norm=float(np.linalg.norm(g["forces"])), loss=g["loss"],
                seconds=time.time() - t0)


def c4t(args):
    w = W.workload("C4")
    n = len(W.make_instances(w))
    log(f"C4 (tension membrane system): {n} sheets, {w.steps} steps, {args.workers} processes")
    t0 = time.time()
    with mp.get_context("fork").Pool(args.workers) as pool:
        res = sorted(pool.imap_unordered(c4t_sheet, range(n)), key=lambda r: r["sheet"])
    nv = np.array([r["nv"] for r in res])
    out = dict(source=SOLVER + "; tension-clamped membrane block in the step matrix",
               workload="C4 tension", steps=w.steps, seconds=time.time() - t0, sheet_nv=nv,
               x=f32(np.concatenate([r["x"] for r in res])),
               dl_dx0=f32(np.concatenate([r["dl_dx0"] for r in res])),
               material=np.array([r["material"] for r in res]),
               dl_dF_norm=np.array([r["dl_dF_norm"] for r in res]),
               loss=np.array([r["loss"] for r in res]))
    path = os.path.join(HERE, "c4_tension_oracle.npz")
    np.savez_compressed(path, **out)
    log(f"wrote {path}")


def c4_sheet(b):
    w = W.workload("C4")
    inst = W.as_given(W.make_instances(w)[b], w.precision)
    frames = w.loss_frames()
    # the configured CG (tolerance 1e-7, block Jacobi) decides whether the step matrix
    # stays positive definite: the exact membrane block may not (reading R9)
    o = oracle.Oracle(inst.tris, inst.rest, inst.pins, *inst.material.as_tuple(), dt=w.dt,
                      cg_tol=w.cg_tol)
    _, _, iters, st = o.rollout(w.steps, inst.x0, inst.v0, inst.forces, check=False)
    res = dict(sheet=b, nv=inst.n_verts, cg_status=int(st))
    if st in (oracle.ORC_OK, oracle.ORC_E_NOT_CONVERGED):
        g = sheet_gradient(w, inst, W.loss_targets(w, inst, frames, sheet=b), frames)
        res.update(x=g["x"][-1], material=g["material"], dl_dx0=g["x0"],
                   dl_dF_norm=float(np.linalg.norm(g["forces"])), loss=g["loss"],
                   seconds=g["seconds"])
    return res


def c4(args):
    w = W.workload("C4")
    n = len(W.make_instances(w))
    log(f"C4: {n} sheets, {w.steps} steps, {args.workers} processes")
    t0 = time.time()
    with mp.get_context("fork").Pool(args.workers) as pool:
        res = []
        for r in pool.imap_unordered(c4_sheet, range(n)):
            log(f"C4 sheet {r['sheet']} ({r['nv']} vertices): CG status {r['cg_status']}")
            res.append(r)
    res.sort(key=lambda r: r["sheet"])
    nv = np.array([r["nv"] for r in res])
    off = np.concatenate([[0], np.cumsum(nv)])
    V = off[-1]
    x = np.full((V, 3), np.nan)
    gx0 = np.full((V, 3), np.nan)
    mat = np.full((n, 3), np.nan)
    fn = np.full(n, np.nan)
    loss = np.full(n, np.nan)
    for r in res:
        if "x" in r:
            sl = slice(off[r["sheet"]], off[r["sheet"] + 1])
            x[sl], gx0[sl] = r["x"], r["dl_dx0"]
            mat[r["sheet"]] = r["material"]
            fn[r["sheet"]] = r["dl_dF_norm"]
            loss[r["sheet"]] = r["loss"]
    out = dict(source=SOLVER + "; breakdown status from the oracle's CG at tolerance 1e-7",
               workload="C4", steps=w.steps, seconds=time.time() - t0, sheet_nv=nv,
               cg_status=np.array([r["cg_status"] for r in res]), x=f32(x), dl_dx0=f32(gx0),
               material=mat, dl_dF_norm=fn, loss=loss)
    path = os.path.join(HERE, "c4_oracle.npz")
    np.savez_compressed(path, **out)
    log(f"wrote {path}")


# ------------------------------------------------------------ 200x200 sheet
def c5_worker(wid, nwork, steps, scratch, qin, qout):
    """Factors A(x_{s-1}) for its steps s (s = steps - wid, steps - wid - nwork, ...),
    one ahead of the sweep, and solves the adjoint system when u_s arrives."""
    w = W.workload("C5")
    inst = W.as_given(W.make_instances(w)[0], w.precision)
    o = make_oracle(inst, w)
    X = np.load(os.path.join(scratch, "c5_X.npy"), mmap_mode="r")
    Vv = np.load(os.path.join(scratch, "c5_V.npy"), mmap_mode="r")
    for s in range(steps - wid, 0, -nwork):
        F = inst.forces[s - 1]
        solver, _ = o._exact_solver(np.array(X[s - 1]), np.array(Vv[s - 1]), F)
        s_got, u = qin.get()
        assert s_got == s
        qout.put((s, solver.solve(u)))
        del solver


def c5(args):
    w = W.workload("C5")
    if args.steps:
        w = W.workload("C5", steps=args.steps)
    inst = W.as_given(W.make_instances(w)[0], w.precision)
    frames = w.loss_frames()
    targets = W.loss_targets(w, inst, frames)
    o = make_oracle(inst, w)
    os.makedirs(args.scratch, exist_ok=True)
    xp = os.path.join(args.scratch, "c5_X.npy")
    t0 = time.time()
    if args.reuse and os.path.exists(xp):
        X = np.load(xp)
        Vv = np.load(os.path.join(args.scratch, "c5_V.npy"))
        DV = np.load(os.path.join(args.scratch, "c5_DV.npy"))
        log("C5: forward states reused from the scratch folder")
    else:
        n = inst.n_verts
        X = np.zeros((w.steps + 1, n, 3))
        Vv = np.zeros_like(X)
        DV = np.zeros_like(X)
        X[0] = inst.x0
        pinned = np.zeros(n, bool)
        pinned[inst.pins] = True
        for s in range(1, w.steps + 1):
            solver, b = o._exact_solver(X[s - 1], Vv[s - 1], inst.forces[s - 1])
            dv = solver.solve(b).reshape(n, 3)
            dv[pinned] = 0.0
            DV[s] = dv
            Vv[s] = Vv[s - 1] + dv
            X[s] = X[s - 1] + w.dt * Vv[s]
            if s % 10 == 0 or s == 1:
                log(f"C5 forward step {s}/{w.steps} ({time.time() - t0:.0f} s)")
        for name, a in (("X", X), ("V", Vv), ("DV", DV)):
            np.save(os.path.join(args.scratch, f"c5_{name}.npy"), a)
    t_fwd = time.time() - t0
    # backward sweep: the oracle's own backward step around exact solves that worker
    # processes factor ahead
    lib = oracle._load()
    ctx = mp.get_context("fork")
    qin = [ctx.Queue() for _ in range(args.workers)]
    qout = ctx.Queue()
    procs = [ctx.Process(target=c5_worker, args=(k, args.workers, w.steps, args.scratch, qin[k],
                                                 qout)) for k in range(args.workers)]
    for p in procs:
        p.start()
    n = inst.n_verts
    xo = X[frames]
    dl = 2.0 * (xo - targets)
    gx = np.zeros((n, 3))
    gv = np.zeros((n, 3))
    u = np.zeros((n, 3))
    gm = np.zeros(3)
    gF = np.zeros((w.steps, n, 3))
    fi = len(frames) - 1
    d = oracle._d
    t1 = time.time()
    for s in range(w.steps, 0, -1):
        if fi >= 0 and frames[fi] == s:
            gx += dl[fi]
            fi -= 1
        lib.orc_adjoint_rhs(o._h, d(gx), d(gv), d(u))
        qin[(w.steps - s) % args.workers].put((s, u.ravel().copy()))
        s_got, mu = qout.get()
        assert s_got == s
        mu = np.ascontiguousarray(mu.reshape(n, 3))
        gF[s - 1] = w.dt * mu
        xs = np.ascontiguousarray(X[s - 1])
        vs = np.ascontiguousarray(Vv[s])
        dvs = np.ascontiguousarray(DV[s])
        vp = np.ascontiguousarray(Vv[s - 1])
        gw = np.zeros(3)
        lib.orc_adjoint_update(o._h, d(xs), d(vp), d(vs), d(dvs), d(mu), d(u), d(gx), d(gv), d(gm),
                               d(gw))
        if s % 10 == 0:
            log(f"C5 backward step {s} ({time.time() - t1:.0f} s)")
    for p in procs:
        p.join()
    keep_frames = np.array([f for f in (30, w.steps) if f in set(frames.tolist())], np.int32)
    keep_steps = np.array(sorted({1, min(31, w.steps), w.steps}), np.int32)
    out = dict(source=SOLVER, workload="C5", steps=w.steps, seconds_forward=t_fwd,
               seconds_backward=time.time() - t1, loss_frames=frames, x_frames=keep_frames,
               x=f32(xo[[list(frames).index(f) for f in keep_frames]]),
               loss=float(np.sum((xo - targets) ** 2)), material=gm, dl_dx0=f32(gx),
               dl_dv0=f32(gv), dl_dF_steps=keep_steps, dl_dF=f32(gF[keep_steps - 1]),
               dl_dF_norms=np.linalg.norm(gF.reshape(w.steps, -1), axis=1))
    path = os.path.join(HERE, "c5_oracle.npz" if not args.steps else f"c5_{w.steps}_oracle.npz")
    np.savez_compressed(path, **out)
    log(f"wrote {path} (forward {t_fwd:.0f} s, backward {time.time() - t1:.0f} s)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["c3", "c4", "c4t", "c5"])
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--steps", type=int, default=0, help="C5: a shorter rollout (test runs)")
    ap.add_argument("--scratch", default="/tmp/phisft_golden")
    ap.add_argument("--reuse", action="store_true", help="C5: reuse stored forward states")
    args = ap.parse_args()
    dict(c3=c3, c4=c4, c4t=c4t, c5=c5)[args.which](args)


if __name__ == "__main__":
    main()
