"""The allocation-free rollout (sim_rollout_noalloc) against sim_rollout through the C
ABI: the same kernels on the same inputs, with the solver's exchange buffers in the
library's static device array instead of the handle's workspace, so every output is
bitwise equal. Two calls in a row share that array, the second on a smaller sheet;
the adjoint after each is the same as after sim_rollout; a handle whose buffers do
not fit the array is refused."""

import numpy as np
import pytest

from gpu_common import make_sim, note
from paper_2203_11938_amd import sim as S, workloads as W

pytestmark = pytest.mark.gpu


def run(s, w, inst, noalloc):
    import torch
    dev = torch.device("cuda:0")
    x0 = torch.tensor(W.to_soa(inst.x0), dtype=s.dtype, device=dev)
    F = torch.tensor(W.to_soa(inst.forces), dtype=s.dtype, device=dev)
    frames = w.loss_frames()
    xo = torch.empty((len(frames), 3, inst.n_verts), dtype=s.dtype, device=dev)
    s.rollout(w.steps, x0, None, F, None, frames, x_out=xo, noalloc=noalloc)
    assert s.status() == S.SIM_OK
    tgt = x0[None] + 0.01
    g = s.adjoint((2.0 * (xo - tgt)).contiguous())
    assert s.status() == S.SIM_OK
    out = dict(x=xo.cpu().numpy())
    out.update({k: v.cpu().numpy() for k, v in g.items() if v is not None})
    return out


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_rollout_is_bitwise_the_rollout(precision):
    # the second call runs a smaller sheet on the same scratch array
    for n, steps in ((32, 20), (12, 8)):
        w = W.workload("C2", n=n, steps=steps, precision=precision)
        inst = W.make_instances(w)[0]
        s = make_sim(w, [inst])
        ref = run(s, w, inst, noalloc=False)
        got = run(s, w, inst, noalloc=True)
        note(f"noalloc {precision}: {n}x{n} sheet, {steps} steps, "
             f"{s.stats()['blocks']} solver workgroups")
        for k in ref:
            assert np.array_equal(ref[k], got[k]), (n, k)
        s.close()


def test_noalloc_refuses_handles_beyond_the_array():
    import torch
    w = W.workload("C2", n=256, steps=1)
    rest, tris = W.grid_sheet(256)
    s = S.Simulator([S.Sheet(tris, rest, W.pin_set(256, "top2"), 1e3, 1e-4, 0.1)], dt=0.01,
                    max_steps=1)
    x0 = torch.tensor(W.to_soa(rest), dtype=torch.float32, device="cuda:0")
    with pytest.raises(S.SimError) as e:
        s.rollout(1, x0, noalloc=True)
    assert e.value.code == S.SIM_E_INVALID
    note(f"noalloc: 256x256 sheet refused ({e.value})")
    s.close()
