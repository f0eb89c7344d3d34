"""HIP graph capture and replay of the rollout and adjoint (the handle's graph option).

Each replay is compared bit for bit with direct launches of the same handle shape on
the same inputs, with unrelated eager GPU work and synchronisations between replays,
and after the inputs' contents change in place (a replay reads the arrays anew).
Parity with the oracle follows from the direct-launch tests.
"""

import numpy as np
import pytest
import torch

from gpu_common import make_sim, note
from paper_2203_11938_amd import workloads as W

pytestmark = pytest.mark.gpu


def _inputs(w, inst, dev, dt):
    x0 = torch.tensor(W.to_soa(inst.x0), dtype=dt, device=dev)
    F = torch.tensor(W.to_soa(inst.forces), dtype=dt, device=dev)
    return x0, F


def _run(s, steps, x0, F, x_out, dl, outs):
    s.rollout(steps, x0, None, F, x_out=x_out)
    g = s.adjoint(dl, out=outs)
    s.sync()
    return x_out.cpu().numpy().copy(), {k: v.cpu().numpy().copy() for k, v in g.items() if v is not None}


@pytest.mark.parametrize("checkpoint", [0, 7])
def test_graph_replays_match_direct_launches(checkpoint):
    w = W.workload("C2", steps=30, precision="fp64")
    inst = W.make_instances(w)[0]
    dev = torch.device("cuda:0")
    note(f"graph: C2 sheet, 30 steps, fp64, checkpoint {checkpoint}")
    kw = dict(rows_per_block=128, checkpoint_every=checkpoint)
    direct = make_sim(w, [inst], **kw)
    graph = make_sim(w, [inst], graph=True, **kw)
    dt = direct.dtype
    x0, F = _inputs(w, inst, dev, dt)
    V = x0.shape[1]
    dl = torch.linspace(-1e-3, 1e-3, 30 * 3 * V, dtype=dt, device=dev).reshape(30, 3, V)
    xo_d = torch.empty((30, 3, V), dtype=dt, device=dev)
    xo_g = torch.empty((30, 3, V), dtype=dt, device=dev)
    # the same result arrays on every call (a replay needs the captured pointers)
    def outs():
        return dict(material=torch.empty((1, 3), dtype=torch.float64, device=dev),
                    forces=torch.empty((30, 3, V), dtype=dt, device=dev),
                    x0=torch.empty((3, V), dtype=dt, device=dev),
                    v0=torch.empty((3, V), dtype=dt, device=dev))
    out_d, out_g = outs(), outs()
    ref_x, ref_g = _run(direct, 30, x0, F, xo_d, dl, out_d)
    for rep in range(3):
        x, g = _run(graph, 30, x0, F, xo_g, dl, out_g)
        st = graph.stats()
        note(f"graph rep {rep}: captures {st['graph_captures']}, replays {st['graph_replays']}")
        assert np.array_equal(x, ref_x), rep
        for k in ref_g:
            assert np.array_equal(g[k], ref_g[k]), (rep, k)
        assert st["graph_captures"] == 2 and st["graph_replays"] == 2 * rep
        # unrelated eager work and a synchronisation between replays
        a = torch.randn(512, 512, device=dev)
        (a @ a).sum().item()
        torch.cuda.synchronize()
    # new input values in the same arrays (a lifted start, half the load): the replay
    # reads them
    x0[2].add_(0.01)
    F.mul_(0.5)
    ref_x, ref_g = _run(direct, 30, x0, F, xo_d, dl, out_d)
    x, g = _run(graph, 30, x0, F, xo_g, dl, out_g)
    assert np.array_equal(x, ref_x)
    for k in ref_g:
        assert np.array_equal(g[k], ref_g[k]), k
    assert graph.stats()["graph_replays"] == 6
    # another output array: a new capture
    xo_2 = torch.empty_like(xo_g)
    x, g = _run(graph, 30, x0, F, xo_2, dl, out_g)
    assert np.array_equal(x, ref_x)
    assert graph.stats()["graph_captures"] == 4
    direct.close()
    graph.close()
