"""Benchmark: one full gradient (rollout + adjoint) of the differentiable cloth step.

Workload (headline): a 64x64-vertex sheet (0.5 m, 7938 triangles), 100 steps of
0.01 s, top corners pinned, per-step Gaussian load 0.05 N/m^2 on each vertex's area
share, material k_s 1e3 N/m, k_b 1e-4 N m, d 0.1 kg/m^2, FP32 arrays at the
boundary with FP64 state, element arithmetic and solver vectors, CG tolerance 1e-7,
every state stored. Loss: summed squared distance to a target rollout (material
scaled by seeded factors). A benchmark "step" is one gradient.

Prints one JSON line with the throughput in vertex-steps/s (vertices x simulated
steps / wall time of rollout + adjoint, inputs resident on the GPU), the roofline
of the dominant kernel (the persistent PCG), the 200x200 sheet's gradient with its
own roofline (sub-object "c5"), and the FP64 CPU oracle timed on a bounded sample
of the same workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def solver_source_hash() -> str:
    p = os.path.join(ROOT, "paper_2203_11938_amd", "csrc", "kernels.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def measured_traffic(workload: str):
    """Per-launch HBM bytes of the solver from the committed rocprofv3 counter
    summary, or None if absent or taken on a different kernel source."""
    p = os.path.join(ROOT, "profiles", f"k_pcg_{workload}_counters.txt")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_sha256_16") != solver_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def block_pattern_size(tris, nv: int) -> int:
    """Non-zero 3x3 blocks of a sheet's step matrix: vertex pairs sharing a triangle,
    the two wing vertices of every interior edge, and the diagonal."""
    import numpy as np
    t = np.asarray(tris, dtype=np.int64)
    pairs = [t[:, [a, b]] for a in range(3) for b in range(3)]
    # interior edges: directed edge (i, j) of one triangle and (j, i) of another
    e = np.concatenate([t[:, [0, 1, 2]], t[:, [1, 2, 0]], t[:, [2, 0, 1]]])  # (i, j, opposite)
    key = e[:, 0] * nv + e[:, 1]
    rev = e[:, 1] * nv + e[:, 0]
    order = np.argsort(key)
    pos = np.searchsorted(key[order], rev)
    pos = np.minimum(pos, len(key) - 1)
    hit = key[order][pos] == rev
    wings = np.stack([e[hit, 2], e[order][pos][hit, 2]], axis=1)
    pairs += [wings, wings[:, ::-1]]
    allp = np.concatenate(pairs)
    return int(np.unique(allp[:, 0] * nv + allp[:, 1]).size)


def host_cpu() -> dict:
    """The host's CPU model and core counts (the oracle runs on one of them)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return dict(model=model, logical_cpus=os.cpu_count(), usable_cpus=usable)


def cpu_baseline(w, inst, sample_steps: int, gpu_iters_per_solve: float):
    import numpy as np
    import oracle
    o = oracle.Oracle(inst.tris, inst.rest, inst.pins, *inst.material.as_tuple(), dt=w.dt,
                      cg_tol=w.cg_tol)
    frames = np.arange(1, sample_steps + 1, dtype=np.int32)
    F = inst.forces[:sample_steps] if inst.forces is not None else None
    xo, _, _, _ = o.rollout(sample_steps, inst.x0, inst.v0, F, frames)
    tgt = inst.x0[None] + 0.01
    t0 = time.perf_counter()
    g = o.gradient(sample_steps, inst.x0, inst.v0, F, frames, 2.0 * (xo - tgt))
    dt = time.perf_counter() - t0
    its = float(np.mean(np.concatenate([g["iters_fwd"], g["iters_adj"]])))
    return dict(value=inst.n_verts * sample_steps / dt, unit="vertex-steps/s", cores=1,
                kind="oracle", host=host_cpu(),
                sample=f"first {sample_steps} of the {w.steps} steps of the same sheet, rollout "
                       f"+ adjoint in one single-threaded FP64 call ({dt:.1f} s)",
                solver=f"the oracle solves each step by block-Jacobi CG ({its:.0f} iterations "
                       f"per solve); the GPU by pipelined CG with a three-level preconditioner "
                       f"({gpu_iters_per_solve:.0f} per solve): the ratio mixes algorithm and "
                       "hardware")


def sequential_comparison(w, insts, batched_ms, steps, membrane, autotune):
    """The same gradient with one handle per sheet, launched one after the other
    on the same stream (warm-up excluded); returns the wall times and the ratio."""
    import numpy as np
    import torch
    from paper_2203_11938_amd import sim as S, workloads as W
    dev = torch.device("cuda:0")
    runs = []
    for inst in insts:
        sim = S.Simulator([S.Sheet(inst.tris, inst.rest, inst.pins, *inst.material.as_tuple())],
                          dt=w.dt, precision=w.precision, cg_tol=w.cg_tol,
                          checkpoint_every=w.checkpoint_every, max_steps=w.steps,
                          membrane=membrane, autotune=autotune)
        dt = sim.dtype
        x0 = torch.tensor(W.to_soa(inst.x0), dtype=dt, device=dev)
        F = torch.tensor(W.to_soa(inst.forces), dtype=dt, device=dev)
        tgt = (x0[None].repeat(len(w.loss_frames()), 1, 1) + 0.01).contiguous()
        runs.append((sim, x0, F, tgt))

    def all_gradients():
        for sim, x0, F, tgt in runs:
            xo = sim.rollout(w.steps, x0, None, F, None, w.loss_frames())
            sim.adjoint((2.0 * (xo - tgt)).contiguous())
        for sim, *_ in runs:
            sim.status()

    all_gradients()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        all_gradients()
    torch.cuda.synchronize()
    seq_ms = 1e3 * (time.perf_counter() - t0) / steps
    for sim, *_ in runs:
        sim.close()
    return dict(sheets=len(insts), batched_ms=round(batched_ms, 3), sequential_ms=round(seq_ms, 3),
                speedup=round(seq_ms / batched_ms, 2))


def variant_timing(w, sheets, x0, v0, F, tgt, frames, steps, warmup, membrane, autotune,
                   graph=False, checkpoint_every=None):
    """The same gradient on another handle: in graph mode (rollout and adjoint
    captured once and replayed; fixed input, output and loss-gradient arrays) and/or
    with another checkpoint interval; returns the wall time per gradient."""
    import torch
    from paper_2203_11938_amd import sim as S
    ck = w.checkpoint_every if checkpoint_every is None else checkpoint_every
    sim = S.Simulator(sheets, dt=w.dt, precision=w.precision, cg_tol=w.cg_tol,
                      checkpoint_every=ck, max_steps=w.steps,
                      membrane=membrane, autotune=autotune, graph=graph)
    xo = torch.empty((len(frames), 3, sim.n_verts), dtype=sim.dtype, device=x0.device)
    dl = torch.empty_like(xo)
    V, nb = sim.n_verts, sim.n_instances
    outs = dict(material=torch.empty((nb, 3), dtype=torch.float64, device=x0.device),
                forces=torch.empty((w.steps, 3, V), dtype=sim.dtype, device=x0.device),
                x0=torch.empty((3, V), dtype=sim.dtype, device=x0.device),
                v0=torch.empty((3, V), dtype=sim.dtype, device=x0.device))

    def gradient():
        sim.rollout(w.steps, x0, v0, F, None, frames, x_out=xo)
        torch.sub(xo, tgt, out=dl).mul_(2.0)
        sim.adjoint(dl, out=outs)

    for _ in range(max(warmup, 1)):
        gradient()
        sim.status()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        gradient()
        sim.status()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    st = sim.stats()
    sim.close()
    out = dict(ms_per_gradient=round(ms, 3),
               value=round(sim.n_verts * w.steps / (ms * 1e-3), 1))
    if graph:
        out.update(captures=int(st["graph_captures"]), replays=int(st["graph_replays"]))
    if ck:
        out.update(checkpoint_every=ck, cg_iters_recompute=int(st["cg_iters_recompute"]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed gradients")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="H")
    ap.add_argument("--cpu-sample-steps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the rule-based solver launch shape instead of timing the candidates")
    ap.add_argument("--membrane", default="exact", choices=["exact", "tension"],
                    help="membrane block of the step matrix")
    ap.add_argument("--checkpoint-report", type=int, default=10, metavar="K",
                    help="store-all workloads: also time the gradient with a state "
                         "checkpoint every K steps (0: skip)")
    ap.add_argument("--coarse-size", type=int, default=None, metavar="N",
                    help="vertices per aggregate of the solver's coarse space (library "
                         "default 64; 0: block-Jacobi only)")
    ap.add_argument("--graph", action="store_true",
                    help="also time the same gradients on a handle in HIP-graph mode")
    ap.add_argument("--sequential", action="store_true",
                    help="batched workloads: also time one handle per sheet, run back to back, "
                         "and report the batched speed-up")
    ap.add_argument("--c5-steps", type=int, default=3, metavar="K",
                    help="also time K gradients of the 200x200 sheet (C5) after one warm-up, "
                         "reported in the 'c5' sub-object with its own roofline (0: skip)")
    ap.add_argument("--chamfer-steps", type=int, default=10, metavar="K",
                    help="also time K Chamfer-distance calls (Eq. 10) of 65,536 x 40,000 points, "
                         "reported in the 'chamfer' sub-object (0: skip)")
    ap.add_argument("--window-iters", type=int, default=10, metavar="K",
                    help="also time K iterations of the adaptive-window Adam loop on a 17x17 "
                         "sheet with all 40 frames active, reported in the 'window' "
                         "sub-object (0: skip)")
    ap.add_argument("--wang-steps", type=int, default=2, metavar="K",
                    help="also time K gradients of the headline sheet with the anisotropic "
                         "strain-dependent material, reported in the 'wang' sub-object (0: skip)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run three plain device copies of MIB MiB (untimed), the "
                         "known-size reference for scaling HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the simulator has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2203_11938_amd import sim as S, workloads as W

    w = W.workload(args.workload)
    insts = W.make_instances(w)
    dev = torch.device("cuda:0")
    if args.calibrate_copy > 0:
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"bench: calibration copies of {args.calibrate_copy} MiB done", file=sys.stderr,
              flush=True)
        del a, b
    print(f"bench: workload {w.name}, {len(insts)} sheet(s), {w.steps} steps", file=sys.stderr,
          flush=True)
    run = timed_gradients(w, insts, args.steps, args.warmup, args.membrane,
                          not args.no_autotune, args.coarse_size)
    sim, st, ms, value = run["sim"], run["stats"], run["ms"], run["value"]
    sides = [int(round(np.sqrt(i.n_verts))) for i in insts]
    roof = roofline(sim, insts, st, run["sheet_iters"], run["iters"], run["wall"],
                    measured_traffic(w.name))
    lib = S.library_identity()
    out = dict(metric="vertex-steps/s forward+adjoint (ms per gradient, 100-step 64\u00d764 "
                      "sheet); % HBM peak",
               value=round(value, 1), unit="vertex-steps/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(ms, 3), higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
               config=dict(workload=(f"{w.name}: {w.n}x{w.n} sheet" if len(insts) == 1 else
                                     f"{w.name}: {len(insts)} sheets of {min(sides)}..{max(sides)} per side") +
                           f", {w.steps} steps of {w.dt} s, rollout + adjoint",
                           sheets=len(insts), vertices=sim.n_verts, sim_steps=w.steps,
                           cg_tol=w.cg_tol, cg_iters_per_gradient=run["iters"] // args.steps,
                           solver_blocks=st["blocks"], rows_per_block=st["rows_per_block"],
                           matrix_precision=sim.matrix_precision, membrane=args.membrane,
                           forces="N(0, 0.05^2) N/m^2 per vertex times its area share"
                           if w.forces == "gauss" else w.forces,
                           coarse_aggregates=st["coarse_aggregates"],
                           coarse_max_dim=st["coarse_max_dim"],
                           autotuned=bool(st["autotuned"]),
                           autotune_candidates=st["autotune_candidates"],
                           solver_matrix=S.MATRIX_HOMES[st["solver_matrix_home"]],
                           solver_launches_per_solve=st["solver_launches_per_solve"],
                           solver_wg_per_cu=st["solver_wg_per_cu"],
                           solver_row_teams=st["solver_row_teams"],
                           coarse_rows_lds=bool(st["coarse_rows_lds"]),
                           device_bytes=int(st["device_bytes"]),
                           device_status=S.status_name(sim.status()),
                           library=lib),
               roofline=roof)
    sheets = [S.Sheet(i.tris, i.rest, i.pins, *i.material.as_tuple()) for i in insts]
    if args.graph:
        print("bench: graph-mode handle", file=sys.stderr, flush=True)
        out["graph_mode"] = variant_timing(w, sheets, run["x0"], run["v0"], run["F"], run["tgt"],
                                           w.loss_frames(), args.steps, args.warmup,
                                           args.membrane, not args.no_autotune, graph=True)
    if args.checkpoint_report > 0 and w.checkpoint_every == 0:
        print(f"bench: checkpoint every {args.checkpoint_report}", file=sys.stderr, flush=True)
        out["checkpointed"] = variant_timing(w, sheets, run["x0"], run["v0"], run["F"], run["tgt"],
                                             w.loss_frames(), args.steps, args.warmup,
                                             args.membrane, not args.no_autotune,
                                             checkpoint_every=args.checkpoint_report)
    if args.sequential and len(insts) > 1:
        out["batched_vs_sequential"] = sequential_comparison(w, insts, ms, args.steps,
                                                             args.membrane, not args.no_autotune)
    gpu_ips = run["iters"] / max(1, args.steps * w.steps * 2 * len(insts))
    sim.close()
    del run
    if args.c5_steps > 0 and w.name != "C5":
        # the 200x200 sheet (300 steps, checkpoint every 30): its own timed gradients and
        # solver roofline, next to the headline
        w5 = W.workload("C5")
        insts5 = W.make_instances(w5)
        print(f"bench: C5, 200x200 sheet, {w5.steps} steps", file=sys.stderr, flush=True)
        r5 = timed_gradients(w5, insts5, args.c5_steps, 1, args.membrane, not args.no_autotune,
                             args.coarse_size)
        st5 = r5["stats"]
        out["c5"] = dict(workload="C5: 200x200 sheet, 300 steps of 0.005 s, checkpoint every 30, "
                                  "rollout + adjoint",
                         steps=args.c5_steps, warmup=1, ms_per_gradient=round(r5["ms"], 3),
                         value=round(r5["value"], 1), unit="vertex-steps/s",
                         cg_iters_per_gradient=r5["iters"] // args.c5_steps,
                         cg_iters_recompute=int(st5["cg_iters_recompute"]),
                         device_bytes=int(st5["device_bytes"]),
                         coarse_store_slots=int(st5["coarse_store_slots"]),
                         solver_blocks=st5["blocks"], rows_per_block=st5["rows_per_block"],
                         roofline=roofline(r5["sim"], insts5, st5, r5["sheet_iters"],
                                           r5["iters"], r5["wall"], measured_traffic("C5")))
        r5["sim"].close()
        del r5
    if args.chamfer_steps > 0:
        print("bench: Chamfer distance", file=sys.stderr, flush=True)
        out["chamfer"] = chamfer_timing(65536, 40000, args.chamfer_steps, 3)
    if args.wang_steps > 0 and len(insts) == 1:
        print("bench: anisotropic material", file=sys.stderr, flush=True)
        out["wang"] = wang_timing(w, insts, args.wang_steps, 1, not args.no_autotune)
    if args.window_iters > 0:
        print("bench: adaptive-window Adam loop", file=sys.stderr, flush=True)
        out["window"] = window_timing(args.window_iters, 2)
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, insts[0], args.cpu_sample_steps, gpu_ips)
    print(json.dumps(out), flush=True)


FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X


def chamfer_timing(n_g: int, n_m: int, steps: int, warmup: int):
    """The Chamfer distance (Eq. 10) of a 65,536-point scan against the 40,000 points of
    a 200x200 reconstruction (seeded synthetic clouds), timed with HIP events around
    every call on its stream. Roofline: ALU-bound; 8 FLOP per point pair and direction
    (3 differences, 3 squares, 2 additions), 2 n_g n_m pairs per call."""
    import numpy as np
    import torch
    from paper_2203_11938_amd import sim as S, workloads as W
    g, m = W.chamfer_points(n_g, n_m)
    dev = torch.device("cuda:0")
    gt = torch.tensor(np.ascontiguousarray(g.T), dtype=torch.float32, device=dev)
    mt = torch.tensor(np.ascontiguousarray(m.T), dtype=torch.float32, device=dev)
    ws = torch.empty(S.load_library().sim_chamfer_workspace_bytes(n_g, n_m), dtype=torch.uint8,
                     device=dev)
    for _ in range(warmup):
        S.chamfer(gt, mt, workspace=ws)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        ch = S.chamfer(gt, mt, workspace=ws)
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    flops = 8.0 * 2.0 * n_g * n_m
    achieved = flops / (ms * 1e-3) / 1e12
    return dict(workload=f"Chamfer distance (Eq. 10): {n_g} scan points vs {n_m} "
                         "reconstruction points, both directions, FP32 distances, FP64 means",
                steps=steps, warmup=warmup, ms_per_call=round(ms, 4),
                wall_ms_per_call=round(1e3 * wall / steps, 4),
                value=round(2.0 * n_g * n_m / (ms * 1e-3), 1), unit="point pairs/s",
                chamfer=float(ch.item()),
                roofline=dict(bound="alu", achieved=round(achieved, 2),
                              peak=FP32_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                              frac=round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4), traffic=None,
                              kernel="k_chamfer_nn (HIP events around the whole call: "
                                     "the fill, unpack and sum launches around it included)"))


def window_timing(iters: int, warmup: int):
    """Iterations of the outer loop (Sec. 3.3-3.4) on the paper's sequence size (a
    289-vertex sheet, 40 frames), every frame active: each is a rollout over the 40
    frames, the frame energies, the adjoint and the Adam steps, plus the host's read of
    the energies that decides the window. The observed frames are the library's own
    rollout under the hidden parameters of the seeded problem (FP64, CG tolerance 1e-10).
    Wall clock per iteration."""
    import numpy as np
    import torch
    from paper_2203_11938_amd import sim as S, workloads as W
    from paper_2203_11938_amd.optimize import AdaptiveWindowAdam
    p = W.window_problem()
    w, i = p.workload, p.instance
    dev = torch.device("cuda:0")
    s = S.Simulator([S.Sheet(i.tris, i.rest, i.pins, *i.material.as_tuple())], dt=w.dt,
                    precision=w.precision, cg_tol=w.cg_tol, max_steps=w.steps)
    x0 = torch.tensor(W.to_soa(i.x0), dtype=s.dtype, device=dev)
    truth = torch.tensor(np.array(p.true_material)[None], device=dev)
    tgt = s.rollout(w.steps, x0, None, None, truth, None,
                    wind=torch.tensor(p.true_wind[None], device=dev)).clone()
    s.sync()
    drv = AdaptiveWindowAdam(s, tgt, x0, torch.tensor(np.array(p.guess_material)[None], device=dev),
                             wind=torch.tensor(p.guess_wind[None], device=dev), first=w.steps)
    drv.run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = drv.run(iters)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / iters
    st = s.stats()
    out = dict(workload=f"adaptive-window Adam loop: {w.n}x{w.n} sheet ({i.n_verts} vertices), "
                        f"{w.steps} frames of {w.dt} s all active, material + wind + forces, "
                        "lr 1e-3, FP64",
               iterations=iters, warmup=warmup, ms_per_iteration=round(ms, 3),
               value=round(1e3 / ms, 2), unit="iterations/s",
               loss_first=recs[0].loss, loss_last=recs[-1].loss,
               cg_iters_last_gradient=int(st["cg_iters_forward"] + st["cg_iters_adjoint"]))
    s.close()
    return out


def wang_timing(w, insts, steps, warmup, autotune):
    """The headline gradient with the anisotropic strain-dependent material (stretch
    table S [4][6], bend table B [3][5]): seeded tables of factors U[0.5, 2] around the
    workload's (k_s, k_b), an area term of 0.3 k_s; the target rollout scales S, B and d
    by the workload's target factors. Same timing as the headline."""
    import numpy as np
    import torch
    from paper_2203_11938_amd import sim as S, workloads as W
    dev = torch.device("cuda:0")
    g = np.random.default_rng(9001)
    ks, kb, d = insts[0].material.as_tuple()
    St = np.exp(g.uniform(np.log(0.5), np.log(2.0), size=(4, 6))) * ks
    St[3] *= 0.3
    Bt = np.exp(g.uniform(np.log(0.5), np.log(2.0), size=(3, 5))) * kb
    f = insts[0].target_factors
    mat = torch.tensor(S.wang_material(St, Bt, d)[None], device=dev)
    mat_t = torch.tensor(S.wang_material(St * f[0], Bt * f[1], d * f[2])[None], device=dev)
    sheets = [S.Sheet(i.tris, i.rest, i.pins, *i.material.as_tuple()) for i in insts]
    sim = S.Simulator(sheets, dt=w.dt, precision=w.precision, cg_tol=w.cg_tol,
                      max_steps=w.steps, autotune=autotune, material_model="wang")
    dt = sim.dtype
    x0 = torch.tensor(W.to_soa(insts[0].x0), dtype=dt, device=dev)
    F = torch.tensor(W.to_soa(insts[0].forces), dtype=dt, device=dev)
    frames = w.loss_frames()
    tgt = sim.rollout(w.steps, x0, None, F, mat_t, frames).clone()
    sim.status()

    def gradient():
        xo = sim.rollout(w.steps, x0, None, F, mat, frames)
        return sim.adjoint((2.0 * (xo - tgt)).contiguous())

    for _ in range(warmup):
        gradient()
        sim.status()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    for _ in range(steps):
        gradient()
        sim.status()
        st = sim.stats()
        iters += st["cg_iters_forward"] + st["cg_iters_adjoint"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = dict(workload=f"{w.name}: {w.n}x{w.n} sheet, {w.steps} steps of {w.dt} s, rollout + "
                        "adjoint, anisotropic material (40 material gradient entries)",
               steps=steps, warmup=warmup, ms_per_gradient=round(1e3 * wall / steps, 3),
               value=round(sim.n_verts * w.steps * steps / wall, 1), unit="vertex-steps/s",
               cg_iters_per_gradient=iters // steps, device_status=S.status_name(sim.status()))
    sim.close()
    return out


def timed_gradients(w, insts, steps, warmup, membrane, autotune, coarse_size):
    """A handle over the workload's sheets, warm-up gradients, then `steps` timed
    gradients (rollout + adjoint, inputs resident on the device) with solver timing on."""
    import numpy as np
    import torch
    from paper_2203_11938_amd import sim as S, workloads as W
    dev = torch.device("cuda:0")
    sheets = [S.Sheet(i.tris, i.rest, i.pins, *i.material.as_tuple()) for i in insts]
    sim = S.Simulator(sheets, dt=w.dt, precision=w.precision, cg_tol=w.cg_tol,
                      checkpoint_every=w.checkpoint_every, max_steps=w.steps,
                      membrane=membrane, autotune=autotune, coarse_size=coarse_size)
    dt = sim.dtype
    x0 = torch.tensor(W.to_soa(np.concatenate([i.x0 for i in insts])), dtype=dt, device=dev)
    v0 = torch.tensor(W.to_soa(np.concatenate([i.v0 for i in insts])), dtype=dt, device=dev)
    F = torch.tensor(W.to_soa(np.concatenate([i.forces for i in insts], axis=1)), dtype=dt,
                     device=dev)
    frames = w.loss_frames()
    # target: rollout of the same sheets with the seeded material factors (untimed)
    mat_t = torch.tensor(np.array([np.array(i.material.as_tuple()) * i.target_factors
                                   for i in insts]), dtype=torch.float64, device=dev)
    tgt = sim.rollout(w.steps, x0, v0, F, mat_t, frames).clone()
    sim.status()

    def gradient():
        xo = sim.rollout(w.steps, x0, v0, F, None, frames)
        return sim.adjoint((2.0 * (xo - tgt)).contiguous())

    for _ in range(warmup):
        gradient()
        sim.status()
    sim.set_timing(True)
    iters = 0
    sheet_iters = np.zeros(len(insts))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        gradient()
        sim.status()
        st = sim.stats()
        iters += st["cg_iters_forward"] + st["cg_iters_adjoint"] + st["cg_iters_recompute"]
        fwd, adj = sim.cg_iters()
        sheet_iters += fwd.sum(axis=0) + adj.sum(axis=0)
        if len(insts) == 1:
            sheet_iters += st["cg_iters_recompute"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = 1e3 * wall / steps
    return dict(sim=sim, stats=sim.stats(), wall=wall, ms=ms, iters=int(iters),
                sheet_iters=sheet_iters, value=sim.n_verts * w.steps * steps / wall,
                x0=x0, v0=v0, F=F, tgt=tgt)


def roofline(sim, insts, st, sheet_iters, iters, wall, traffic):
    """Roofline of the persistent solver: algorithmic bytes per CG iteration are the
    operator read once (9 entries in the stored precision + a 4-byte column index per
    non-zero 3x3 block) plus one pass over each solver vector: 336 B per vertex with the
    solver's FP64 vectors (p 24, A p 48, x 48, r 48, block-Jacobi inverse 72, z 48, the
    p update 48), 192 B with FP32 ones (the FP32 yardstick, reported beside it). A batched
    launch iterates every sheet on its own, so each sheet's iterations are weighted with
    its own bytes per iteration."""
    import numpy as np
    msize = 8 if sim.matrix_precision == "fp64" else 4
    nnz = np.array([block_pattern_size(i.tris, i.n_verts) for i in insts], dtype=np.float64)
    nv = np.array([i.n_verts for i in insts], dtype=np.float64)
    b64 = (9 * msize + 4) * nnz + 336 * nv
    b32 = 40 * nnz + 192 * nv
    launches = max(st["solver_launches"], 1)
    avg_ms = st["solver_ms"] / launches
    per_launch = float(np.dot(b64, sheet_iters)) / launches
    per_launch32 = float(np.dot(b32, sheet_iters)) / launches
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    achieved32 = per_launch32 / (avg_ms * 1e-3) / 1e9
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4),
                traffic=None if traffic is None else round(traffic, 1),
                kernel="k_pcg", avg_launch_ms=round(avg_ms, 4),
                cg_iters_per_launch=round(iters / launches, 1),
                bytes_per_cg_iter=int(b64.sum()) if len(insts) == 1 else None,
                frac_fp32_yardstick=round(achieved32 / HBM_PEAK_GBS, 4),
                solver_share_of_wall=round(st["solver_ms"] / (wall * 1e3), 3))


if __name__ == "__main__":
    main()
