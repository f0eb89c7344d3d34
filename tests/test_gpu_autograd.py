"""The torch.autograd path (ClothRollout / sim.rollout): vertex-major tensors in and out,
the library's adjoint as the backward pass; gradients of a squared-distance loss
against the FP64 oracle's (gates 1e-9 positions, 1e-6 gradients, as for the 32x32
workload in FP64)."""

import numpy as np
import pytest
import torch

from gpu_common import make_sim, note, oracle_for, rel
from paper_2203_11938_amd import sim as S, workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("with_v0", [True, False])
def test_autograd_matches_oracle(with_v0):
    w = W.workload("C2", steps=20, precision="fp64", cg_tol=1e-10)
    inst = W.make_instances(w)[0]
    frames = w.loss_frames()
    o_t = oracle_for(inst, w, factors=inst.target_factors)
    tgt, _, _, _ = o_t.rollout(w.steps, inst.x0, inst.v0, inst.forces, frames)
    o = oracle_for(inst, w)
    xo, _, _, _ = o.rollout(w.steps, inst.x0, inst.v0, inst.forces, frames)
    ref = o.gradient(w.steps, inst.x0, inst.v0, inst.forces, frames, 2.0 * (xo - tgt))

    s = make_sim(w, [inst])
    dev = torch.device("cuda:0")
    f64 = dict(dtype=torch.float64, device=dev)
    material = torch.tensor([inst.material.as_tuple()], **f64, requires_grad=True)
    forces = torch.tensor(inst.forces, **f64, requires_grad=True)
    x0 = torch.tensor(inst.x0, **f64, requires_grad=True)
    v0 = torch.tensor(inst.v0, **f64, requires_grad=True) if with_v0 else None
    x = S.rollout(s, w.steps, material, x0, v0, forces, frames)
    assert tuple(x.shape) == (len(frames), inst.n_verts, 3)
    loss = ((x - torch.tensor(tgt, **f64)) ** 2).sum()
    loss.backward()
    errs = dict(x=rel(x.detach().cpu().numpy(), xo),
                material=rel(material.grad.cpu().numpy()[0], ref["material"]),
                forces=rel(forces.grad.cpu().numpy(), ref["forces"]),
                x0=rel(x0.grad.cpu().numpy(), ref["x0"]))
    if with_v0:
        errs["v0"] = rel(v0.grad.cpu().numpy(), ref["v0"])
    note("autograd: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    assert errs["x"] <= 1e-9
    for k, v in errs.items():
        if k != "x":
            assert v <= 1e-6, (k, v)
    s.close()


def test_backward_refuses_a_later_rollout_on_the_handle():
    """Two forward passes on one handle, then the first one's backward: the handle's
    adjoint belongs to the second rollout, so the backward raises instead of returning
    the wrong trajectory's gradients; the second graph's backward still works."""
    w = W.workload("C2", n=8, steps=5, precision="fp64", cg_tol=1e-10)
    inst = W.make_instances(w)[0]
    s = make_sim(w, [inst])
    f64 = dict(dtype=torch.float64, device=torch.device("cuda:0"))
    mat = torch.tensor([inst.material.as_tuple()], **f64, requires_grad=True)
    x0 = torch.tensor(inst.x0, **f64)
    F1 = torch.tensor(inst.forces, **f64, requires_grad=True)
    F2 = torch.tensor(2.0 * inst.forces, **f64, requires_grad=True)
    x1 = S.rollout(s, w.steps, mat, x0, None, F1)
    x2 = S.rollout(s, w.steps, mat, x0, None, F2)
    with pytest.raises(RuntimeError, match="another rollout"):
        x1.sum().backward()
    x2.sum().backward()
    assert F2.grad is not None and torch.isfinite(F2.grad).all()
    s.close()


def test_unconverged_forward_raises_unless_allowed():
    """A solve capped at one iteration does not converge: the autograd path raises by
    default and warns when the handle allows it."""
    w = W.workload("C2", n=8, steps=3, precision="fp64", cg_tol=1e-12)
    inst = W.make_instances(w)[0]
    s = make_sim(w, [inst], cg_max_iter=1)
    f64 = dict(dtype=torch.float64, device=torch.device("cuda:0"))
    mat = torch.tensor([inst.material.as_tuple()], **f64, requires_grad=True)
    x0 = torch.tensor(inst.x0, **f64)
    with pytest.raises(S.SimError):
        S.rollout(s, w.steps, mat, x0)
    s.allow_not_converged = True
    with pytest.warns(RuntimeWarning):
        x = S.rollout(s, w.steps, mat, x0)
    assert torch.isfinite(x).all()
    s.close()
