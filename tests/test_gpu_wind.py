"""GPU parity of the velocity-dependent wind (Eq. 2's w; the aerodynamic force of
reading R19 with the paper's air density, Sec. 3.4) against the FP64 oracle, through
the C ABI: the force in the step's right-hand side, its velocity Jacobian in the step
matrix, and the adjoint's gradients including dL/dw.

Gates: FP64 handles 1e-9 on positions and 1e-7 on every gradient block (relative, as
for the 32x32 workload); FP32 handles 1e-5 and 1e-4. The full-size closed form (a
flat sheet falling through still air moves as one body, its vertical velocity
following v <- v + h (rho |s| s + d g) / (d + 2 h rho |s|), s = -v) needs no oracle.
"""

import numpy as np
import pytest

from gpu_common import make_sim, note, oracle_for, rel
from paper_2203_11938_amd import sim as S, workloads as W

pytestmark = pytest.mark.gpu

WIND = (0.5, 0.2, -1.5)


def run(s, w, insts, winds, targets):
    import torch
    dev = torch.device("cuda:0")
    dt = s.dtype
    x0 = torch.tensor(W.to_soa(np.concatenate([i.x0 for i in insts])), dtype=dt, device=dev)
    F = torch.tensor(W.to_soa(np.concatenate([i.forces for i in insts], axis=1)), dtype=dt,
                     device=dev)
    wt = torch.tensor(np.asarray(winds, np.float64).reshape(-1, 3), device=dev)
    frames = w.loss_frames()
    xo = s.rollout(w.steps, x0, None, F, None, frames, wind=wt)
    tgt = torch.tensor(W.to_soa(np.concatenate(targets, axis=1)), dtype=dt, device=dev)
    g = s.adjoint((2.0 * (xo - tgt)).contiguous())
    st = s.status()
    out = dict(status=st, x=W.from_soa(xo.cpu().numpy().astype(np.float64)))
    for k, v in g.items():
        out[k] = v.cpu().numpy().astype(np.float64)
    for k in ("forces", "x0", "v0"):
        out[k] = W.from_soa(out[k])
    return out


def oracle_ref(w, inst, wind, target, rho=1.0):
    o = oracle_for(inst, w)
    o.set_wind(wind, rho)
    frames = w.loss_frames()
    xo, _, _, _ = o.rollout(w.steps, inst.x0, inst.v0, inst.forces, frames)
    g = o.gradient(w.steps, inst.x0, inst.v0, inst.forces, frames, 2.0 * (xo - target))
    g["x"] = xo
    return g


def errors(out, ref, sl=slice(None), b=0):
    e = dict(x=rel(out["x"][-1][sl], ref["x"][-1]))
    for k, name in enumerate(("k_s", "k_b", "d")):
        e[name] = abs(out["material"][b][k] - ref["material"][k]) / abs(ref["material"][k])
    e["wind"] = rel(out["wind"][b], ref["wind"])
    e["forces"] = rel(out["forces"][:, sl], ref["forces"])
    e["x0"] = rel(out["x0"][sl], ref["x0"])
    e["v0"] = rel(out["v0"][sl], ref["v0"])
    return e


@pytest.mark.parametrize("precision,tol_x,tol_g", [("fp64", 1e-9, 1e-7), ("fp32", 1e-5, 1e-4)])
def test_wind_parity_32x32(precision, tol_x, tol_g):
    w = W.workload("C2", steps=30, precision=precision,
                   cg_tol=1e-10 if precision == "fp64" else 1e-7)
    inst = W.as_given(W.make_instances(w)[0], precision)
    target = W.loss_targets(w, inst, w.loss_frames())
    s = make_sim(w, [inst])
    out = run(s, w, [inst], [WIND], [target])
    assert out["status"] == 0
    ref = oracle_ref(w, inst, WIND, target)
    e = errors(out, ref)
    note(f"wind {precision}: " + ", ".join(f"{k} {v:.1e}" for k, v in e.items()) +
         f"; dL/dw {np.array2string(out['wind'][0], precision=4)}")
    assert e.pop("x") <= tol_x
    for k, v in e.items():
        assert v <= tol_g, (k, v)
    s.close()


def test_wind_batch_each_sheet_its_own_wind():
    w = W.workload("C4", steps=12, batch=3, batch_n_range=(10, 20), precision="fp64",
                   cg_tol=1e-10)
    insts = W.make_instances(w)
    winds = [(0.3, -0.4, 1.2), (0.0, 0.0, 0.0), (-1.0, 0.5, -0.8)]
    frames = w.loss_frames()
    targets = [W.loss_targets(w, i, frames, sheet=b) for b, i in enumerate(insts)]
    s = make_sim(w, insts)
    out = run(s, w, insts, winds, targets)
    assert out["status"] == 0
    off = np.concatenate([[0], np.cumsum([i.n_verts for i in insts])])
    for b, inst in enumerate(insts):
        ref = oracle_ref(w, inst, winds[b], targets[b])
        e = errors(out, ref, slice(off[b], off[b + 1]), b)
        note(f"wind batch sheet {b} ({inst.n_verts} vertices, w {winds[b]}): " +
             ", ".join(f"{k} {v:.1e}" for k, v in e.items()))
        assert e.pop("x") <= 1e-9
        for k, v in e.items():
            assert v <= 1e-7, (b, k, v)
    s.close()


def test_wind_checkpoint_recompute_is_bitwise_store_all():
    w = W.workload("C2", steps=24, precision="fp64", cg_tol=1e-10)
    inst = W.make_instances(w)[0]
    target = W.loss_targets(w, inst, w.loss_frames())
    a = run(make_sim(w, [inst]), w, [inst], [WIND], [target])
    b = run(make_sim(w, [inst], checkpoint_every=7), w, [inst], [WIND], [target])
    for k in ("x", "material", "wind", "forces", "x0", "v0"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("wind", [(0.0, 0.0, 0.0), (1.0, -0.6, 0.0)])
def test_flat_sheet_falls_through_air_full_size(wind):
    """200x200 unpinned flat sheet from rest, still air or a wind in its plane."""
    import torch
    n, steps, h, d, rho = 200, 8, 0.01, 0.1, 1.0
    rest, tris = W.grid_sheet(n)
    s = S.Simulator([S.Sheet(tris, rest, [], 1e3, 1e-4, d)], dt=h, precision="fp64",
                    cg_tol=1e-12, max_steps=steps, air_density=rho)
    dev = torch.device("cuda:0")
    x0 = torch.tensor(W.to_soa(rest), dtype=torch.float64, device=dev)
    wt = torch.tensor([wind], dtype=torch.float64, device=dev)
    xo = s.rollout(steps, x0, wind=wt)
    st = s.sync(allow_not_converged=True)
    if st == S.SIM_E_NOT_CONVERGED:   # a tolerance at the unpinned sheet's attainable floor
        assert s.stats()["max_rel_residual"] <= 1e-9
    x = W.from_soa(xo.cpu().numpy())
    vz, z, err = 0.0, 0.0, 0.0
    for k in range(steps):
        sn = -vz
        vz += h * (rho * abs(sn) * sn + d * (-9.81)) / (d + 2.0 * h * rho * abs(sn))
        z += h * vz
        err = max(err, np.abs(x[k][:, 2] - z).max(), np.abs(x[k][:, :2] - rest[:, :2]).max())
    note(f"falling through air {n}x{n}, wind {wind}: max position error {err:.2e} m "
         f"(fall {-z:.3e} m)")
    assert err <= 1e-10
    s.close()


def test_autograd_wind_gradient():
    import torch
    w = W.workload("C2", n=12, steps=10, precision="fp64", cg_tol=1e-10)
    inst = W.make_instances(w)[0]
    s = make_sim(w, [inst])
    dev = torch.device("cuda:0")
    mat = torch.tensor([inst.material.as_tuple()], dtype=torch.float64, device=dev)
    x0 = torch.tensor(inst.x0, dtype=torch.float64, device=dev)
    F = torch.tensor(inst.forces, dtype=torch.float64, device=dev)
    wind = torch.tensor([WIND], dtype=torch.float64, device=dev, requires_grad=True)
    xo = S.rollout(s, w.steps, mat, x0, forces=F, wind=wind)
    tgt = torch.tensor(W.loss_targets(w, inst, w.loss_frames()), device=dev)
    loss = ((xo - tgt) ** 2).sum()
    loss.backward()
    ref = oracle_ref(w, inst, WIND, W.loss_targets(w, inst, w.loss_frames()))
    e = rel(wind.grad.cpu().numpy()[0], ref["wind"])
    note(f"autograd dL/dw rel err {e:.1e}")
    assert e <= 1e-7
    s.close()
