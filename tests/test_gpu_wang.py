"""GPU parity of the anisotropic strain-dependent material (the paper's S in R^24 and
B in R^15, readings R20/R21 of Wang et al.'s model) against the FP64 oracle, through
the C ABI: forces and stiffness blocks of the step, and the adjoint's 40 material
gradient entries (24 stretch, 15 bend, density) with the other gradient blocks.

The sheets are soft (stretch tables around 30 N/m) so that their strains cross every
strain segment within the rollout. Gates as for the isotropic 32x32 workload: FP64
handles 1e-9 on positions and 1e-7 on every gradient block (relative to the block's
largest entry), FP32 handles 1e-5 and 1e-4.
"""

import numpy as np
import pytest

from gpu_common import make_sim, note, oracle_for, rel
from paper_2203_11938_amd import sim as S, workloads as W

pytestmark = pytest.mark.gpu

KS, KB = 30.0, 3e-6


def tables(seed, ks=KS, kb=KB):
    g = np.random.default_rng(seed)
    St = np.exp(g.uniform(np.log(0.5), np.log(2.0), size=(4, 6))) * ks
    St[3] *= 0.3
    Bt = np.exp(g.uniform(np.log(0.5), np.log(2.0), size=(3, 5))) * kb
    return St, Bt


def workload(n, steps, precision, **kw):
    return W.workload("C2", n=n, steps=steps, precision=precision,
                      cg_tol=1e-11 if precision == "fp64" else 1e-7, **kw)


def gpu_run(s, w, insts, mats, winds, targets):
    import torch
    dev = torch.device("cuda:0")
    dt = s.dtype
    x0 = torch.tensor(W.to_soa(np.concatenate([i.x0 for i in insts])), dtype=dt, device=dev)
    F = torch.tensor(W.to_soa(np.concatenate([i.forces for i in insts], axis=1)), dtype=dt,
                     device=dev)
    mt = torch.tensor(np.stack(mats), device=dev)
    wt = None if winds is None else torch.tensor(np.asarray(winds, np.float64), device=dev)
    frames = w.loss_frames()
    xo = s.rollout(w.steps, x0, None, F, mt, frames, wind=wt)
    tgt = torch.tensor(W.to_soa(np.concatenate(targets, axis=1)), dtype=dt, device=dev)
    g = s.adjoint((2.0 * (xo - tgt)).contiguous())
    out = dict(status=s.status(), x=W.from_soa(xo.cpu().numpy().astype(np.float64)))
    for k, v in g.items():
        out[k] = None if v is None else v.cpu().numpy().astype(np.float64)
    for k in ("forces", "x0", "v0"):
        out[k] = W.from_soa(out[k])
    return out


def oracle_ref(w, inst, St, Bt, d, target, wind=None):
    o = oracle_for(inst, w)
    o.set_params(density=d)
    o.set_material_wang(St, Bt)
    if wind is not None:
        o.set_wind(wind)
    frames = w.loss_frames()
    xo, _, _, _ = o.rollout(w.steps, inst.x0, inst.v0, inst.forces, frames)
    g = o.gradient(w.steps, inst.x0, inst.v0, inst.forces, frames, 2.0 * (xo - target))
    g["x"] = xo
    return g


def errors(out, ref, b=0, sl=slice(None)):
    m = out["material"][b]
    e = dict(x=rel(out["x"][-1][sl], ref["x"][-1]),
             stretch=rel(m[:24], ref["material"][:24]), bend=rel(m[24:39], ref["material"][24:39]),
             density=abs(m[39] - ref["material"][39]) / abs(ref["material"][39]),
             forces=rel(out["forces"][:, sl], ref["forces"]), x0=rel(out["x0"][sl], ref["x0"]),
             v0=rel(out["v0"][sl], ref["v0"]))
    if out.get("wind") is not None:
        e["wind"] = rel(out["wind"][b], ref["wind"])
    return e


@pytest.mark.parametrize("precision,tol_x,tol_g", [("fp64", 1e-9, 1e-7), ("fp32", 1e-5, 1e-4)])
def test_wang_parity_16x16(precision, tol_x, tol_g):
    w = workload(16, 40, precision)
    inst = W.as_given(W.make_instances(w)[0], precision)
    St, Bt = tables(21)
    d = 0.1
    target = W.loss_targets(w, inst, w.loss_frames())
    s = make_sim(w, [inst], material_model="wang")
    out = gpu_run(s, w, [inst], [S.wang_material(St, Bt, d)], None, [target])
    assert out["status"] == 0, S.status_name(out["status"])
    ref = oracle_ref(w, inst, St, Bt, d, target)
    e = errors(out, ref)
    note(f"wang {precision} 16x16: " + ", ".join(f"{k} {v:.1e}" for k, v in e.items()))
    assert e.pop("x") <= tol_x
    for k, v in e.items():
        assert v <= tol_g, (k, v)
    s.close()


def test_wang_with_wind_in_a_batch():
    """Two sheets of different sizes and tables in one handle, one wind each; every
    sheet against its own oracle."""
    w = workload(12, 30, "fp64")
    wb = workload(16, 30, "fp64")
    insts = [W.make_instances(w)[0], W.make_instances(wb)[0]]
    tabs = [tables(31), tables(32)]
    dens = [0.1, 0.14]
    winds = [(0.4, -0.2, 1.0), (-0.3, 0.5, -0.8)]
    targets = [W.loss_targets(w, insts[0], w.loss_frames()),
               W.loss_targets(w, insts[1], w.loss_frames(), sheet=1)]
    s = make_sim(w, insts, material_model="wang")
    out = gpu_run(s, w, insts, [S.wang_material(*tabs[b], dens[b]) for b in range(2)], winds,
                  targets)
    assert out["status"] == 0, S.status_name(out["status"])
    off = np.cumsum([0] + [i.n_verts for i in insts])
    for b in range(2):
        ref = oracle_ref(w, insts[b], *tabs[b], dens[b], targets[b], wind=winds[b])
        e = errors(out, ref, b=b, sl=slice(off[b], off[b + 1]))
        note(f"wang batch sheet {b}: " + ", ".join(f"{k} {v:.1e}" for k, v in e.items()))
        assert e.pop("x") <= 1e-9
        for k, v in e.items():
            assert v <= 1e-7, (b, k, v)
    s.close()


def test_wang_isotropic_tables_match_the_isotropic_handle():
    """Tables that encode (k_s, k_b) reproduce an isotropic handle: positions to 1e-12,
    and the stretch and bend gradient sums are dL/dk_s and dL/dk_b."""
    w = workload(16, 30, "fp64")
    inst = W.make_instances(w)[0]
    ks, kb, d = 400.0, 2e-4, 0.1
    target = W.loss_targets(w, inst, w.loss_frames())
    si = make_sim(w, [inst])
    oi = gpu_run(si, w, [inst], [np.array([ks, kb, d])], None, [target])
    sw = make_sim(w, [inst], material_model="wang")
    St = np.full((4, 6), ks)
    St[3] = 0.0
    ow = gpu_run(sw, w, [inst], [S.wang_material(St, np.full((3, 5), kb), d)], None, [target])
    assert oi["status"] == 0 and ow["status"] == 0
    gi, gw = oi["material"][0], ow["material"][0]
    e = dict(x=rel(ow["x"], oi["x"]), k_s=abs(gw[:18].sum() - gi[0]) / abs(gi[0]),
             k_b=abs(gw[24:39].sum() - gi[1]) / abs(gi[1]), d=abs(gw[39] - gi[2]) / abs(gi[2]),
             forces=rel(ow["forces"], oi["forces"]), x0=rel(ow["x0"], oi["x0"]))
    note("wang iso tables vs isotropic handle: " + ", ".join(f"{k} {v:.1e}" for k, v in e.items()))
    assert e.pop("x") <= 1e-10
    for k, v in e.items():
        assert v <= 1e-8, (k, v)
    si.close()
    sw.close()


def test_wang_checkpointed_equals_store_all():
    w = workload(16, 30, "fp64")
    inst = W.make_instances(w)[0]
    St, Bt = tables(41)
    mat = [S.wang_material(St, Bt, 0.1)]
    target = W.loss_targets(w, inst, w.loss_frames())
    a = gpu_run(make_sim(w, [inst], material_model="wang"), w, [inst], mat, None, [target])
    b = gpu_run(make_sim(w, [inst], material_model="wang", checkpoint_every=7), w, [inst], mat,
                None, [target])
    for k in ("x", "material", "forces", "x0", "v0"):
        assert np.array_equal(a[k], b[k]), k


def test_wang_refuses_the_tension_membrane():
    w = workload(8, 5, "fp64")
    inst = W.make_instances(w)[0]
    with pytest.raises(S.SimError) as e:
        make_sim(w, [inst], material_model="wang", membrane="tension")
    assert "status -1" in str(e.value)
