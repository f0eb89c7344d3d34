"""Device memory of checkpointed handles (state checkpoint every k steps, recompute in
the adjoint): it must grow with the rollout's capacity only through the checkpoints
(48 B per vertex each, x and v in FP64), never through per-step storage. With the
default store, the solver's coarse operators are kept for one checkpoint segment
(k slots); coarse_keep_all keeps one per step. A handle that stores every state grows
by a full state per step.

Checked on the 200x200 sheet (V = 40,000) with k = 30, comparing the device bytes the
library reports (sim_stats.device_bytes) for capacities of 300 and 600 steps: the
difference may hold the 10 extra checkpoints and the per-step statistics arrays
(iteration counts and residuals, 36 B per step and sheet), plus allocation rounding.
"""

import pytest

from gpu_common import note
from paper_2203_11938_amd import sim as S, workloads as W

pytestmark = pytest.mark.gpu


def handle_bytes(n, k, steps, **kw):
    rest, tris = W.grid_sheet(n)
    s = S.Simulator([S.Sheet(tris, rest, W.pin_set(n, "topedge"), 1e3, 1e-4, 0.1)], dt=0.005,
                    checkpoint_every=k, max_steps=steps, **kw)
    st = s.stats()
    s.close()
    return st["device_bytes"], st["coarse_store_slots"]


def test_checkpointed_memory_grows_only_with_checkpoints():
    n, k = 200, 30
    V = n * n
    b300, slots300 = handle_bytes(n, k, 300)
    b600, slots600 = handle_bytes(n, k, 600)
    state = 48 * V
    growth = b600 - b300
    bound = (600 // k - 300 // k) * state + 300 * 36 + 64 * 1024
    note(f"memory: 200x200, checkpoint every {k}: {b300 / 2**20:.1f} MiB for 300 steps, "
         f"{b600 / 2**20:.1f} MiB for 600 (growth {growth / 2**20:.2f} MiB, bound "
         f"{bound / 2**20:.2f}); coarse slots {slots300}, {slots600}")
    assert slots300 == k and slots600 == k
    assert growth <= bound
    # (T/k + k + 3) states, the rest is the steps-independent workspace
    fixed = b300 - (300 // k + 1 + k + 3) * state
    note(f"memory: steps-independent part {fixed / 2**20:.1f} MiB "
         f"({fixed / V:.0f} B per vertex)")
    # keeping every step's coarse operators is the opt-in that grows with the steps
    bk, slotsk = handle_bytes(n, k, 300, coarse_keep_all=True)
    note(f"memory: coarse_keep_all: {bk / 2**20:.1f} MiB, {slotsk} coarse slots")
    assert slotsk == 300 and bk > b300


def test_store_all_grows_by_a_state_per_step():
    n = 64
    V = n * n
    b100, _ = handle_bytes(n, 0, 100)
    b200, _ = handle_bytes(n, 0, 200)
    per_step = (b200 - b100) / 100
    note(f"memory: 64x64, every state stored: {per_step:.0f} B per step of capacity "
         f"({48 * V} B per state)")
    # a state, the step's statistics, and the step's coarse operators (kept per step
    # when every state is stored): an FP32 coarse inverse of 384^2 entries and the
    # aggregate and run offsets and 6x6 inverses, about 0.86 MB on this sheet
    assert 48 * V <= per_step <= 48 * V + 36 + 0.9e6
