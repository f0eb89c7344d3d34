"""Adaptive temporal-window Adam driver of phi-SfT's outer optimisation (Sec. 3.3 and
3.4), over the library's C ABI.

Each iteration re-simulates the active frames 1..t_a (sim_rollout), evaluates the
per-frame energies E_t = sum_i |x_t,i - target_t,i|^2 and their gradient
(sim_frame_loss), back-propagates through the simulator (sim_adjoint) and takes one
Adam step per parameter group (sim_adam_step). All arithmetic runs in the library's
kernels; this module holds the host-side control: which frames are active.

The window (Sec. 3.3): it starts with the first `first` frames (five in the paper). A
frame is added when the energy of the latest active frame falls below the threshold
b, or after `max_iters` iterations on the current window. b is the energy of frame
`first` at the moment frame `first` + 1 is added, so the first addition always
happens at the iteration cap (reading of the paper's definition, where b is not yet
known while only the first frames are active). The decision for the next iteration
uses the energies of the current iteration's rollout, taken before its Adam step;
for a batch handle the sheets' energies of a frame are added up.

Parameters (the paper's phi without the unused ones): the material of each sheet
((k_s, k_b, d), or the anisotropic tables and d) in log space, the wind velocity w,
and the per-step forces F_t read as loads on each vertex's area share (the optimised
variable is F / vertex area). Adam uses one step counter for all groups (the
iteration number); forces of frames that were never active keep zero moments and do
not move.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import sim as S


@dataclass
class Record:
    iteration: int
    active: int                 # frames simulated in this iteration
    energies: np.ndarray        # [active] energy of each active frame (sheets added up)
    loss: float                 # their sum


@dataclass
class WindowState:
    active: int
    iters_in_window: int = 0
    threshold: Optional[float] = None


def next_window(state: WindowState, energies: np.ndarray, n_frames: int, first: int,
                max_iters: int) -> WindowState:
    """The window after an iteration whose active frames had these energies."""
    s = WindowState(state.active, state.iters_in_window + 1, state.threshold)
    if s.active >= n_frames:
        return s
    latest = float(energies[s.active - 1])
    below = s.threshold is not None and latest < s.threshold
    if below or s.iters_in_window >= max_iters:
        if s.threshold is None and s.active == first:
            s.threshold = float(energies[first - 1])
        s.active += 1
        s.iters_in_window = 0
    return s


@dataclass
class AdaptiveWindowAdam:
    """Optimises material, wind and forces of `sim`'s sheets against target positions.

    targets [n_frames, 3, V] and x0 [3, V] (v0 optional) in the handle's precision;
    material [n_instances, n_material] (positive entries: it is optimised through its
    logarithm) and wind [n_instances, 3] float64 initial guesses
    (wind None: no aerodynamic force, not optimised); forces [n_frames, 3, V] initial
    guess (None: zero). Learning rates per group (the paper uses 1e-3 for all)."""
    sim: S.Simulator
    targets: torch.Tensor
    x0: torch.Tensor
    material: torch.Tensor
    wind: Optional[torch.Tensor] = None
    forces: Optional[torch.Tensor] = None
    v0: Optional[torch.Tensor] = None
    first: int = 5
    max_iters: int = 50
    lr_material: float = 1e-3
    lr_wind: float = 1e-3
    lr_forces: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    optimise: tuple = ("material", "wind", "forces")
    history: List[Record] = field(default_factory=list)

    def __post_init__(self):
        sim = self.sim
        self.n_frames = int(self.targets.shape[0])
        if self.n_frames > sim.max_steps:
            raise ValueError("the handle's max_steps is shorter than the sequence")
        dev, dt, V, nb = self.x0.device, sim.dtype, sim.n_verts, sim.n_instances
        self.material = self.material.clone().contiguous()
        if "material" in self.optimise and not bool((self.material > 0).all()):
            raise ValueError("the material is optimised in log space: every entry must be "
                             "positive (an anisotropic table without an area term has zeros)")
        if self.wind is not None:
            self.wind = self.wind.clone().contiguous()
        self.forces = (torch.zeros((self.n_frames, 3, V), dtype=dt, device=dev)
                       if self.forces is None else self.forces.clone().contiguous())
        z = lambda t: torch.zeros(t.numel(), dtype=torch.float64, device=dev)
        self._m = {k: (z(t), z(t)) for k, t in (("material", self.material),
                                                 ("forces", self.forces))}
        if self.wind is not None:
            self._m["wind"] = (z(self.wind), z(self.wind))
        self._area = torch.tensor(sim.vertex_areas(), dtype=torch.float64, device=dev)
        self._xo = torch.empty((self.n_frames, 3, V), dtype=dt, device=dev)
        self._dl = torch.empty_like(self._xo)
        self._energy = torch.empty((self.n_frames, nb), dtype=torch.float64, device=dev)
        self._g = dict(material=torch.empty((nb, sim.n_material), dtype=torch.float64,
                                            device=dev),
                       forces=torch.empty((self.n_frames, 3, V), dtype=dt, device=dev),
                       x0=torch.empty((3, V), dtype=dt, device=dev),
                       v0=torch.empty((3, V), dtype=dt, device=dev))
        if self.wind is not None:
            self._g["wind"] = torch.empty((nb, 3), dtype=torch.float64, device=dev)
        self.window = WindowState(min(self.first, self.n_frames))
        self.iteration = 0

    def step(self) -> Record:
        sim, ta = self.sim, self.window.active
        frames = np.arange(1, ta + 1, dtype=np.int32)
        xo, dl, en = self._xo[:ta], self._dl[:ta], self._energy[:ta]
        sim.rollout(ta, self.x0, self.v0, self.forces[:ta], self.material, frames, x_out=xo,
                    wind=self.wind)
        sim.frame_loss(xo, self.targets[:ta], en, dl)
        out = {k: (v[:ta] if k == "forces" else v) for k, v in self._g.items()}
        g = sim.adjoint(dl, out=out, want_wind=self.wind is not None)
        energies = en.sum(dim=1).cpu().numpy()   # waits for the step's work
        st = sim.status()
        if st not in (S.SIM_OK, S.SIM_E_NOT_CONVERGED):
            raise S.SimError(st, "optimisation step: " + S.status_name(st))
        self.iteration += 1
        t = self.iteration
        if "material" in self.optimise:
            m1, m2 = self._m["material"]
            S.adam_step(self.material, g["material"], m1, m2, t, self.lr_material, self.beta1,
                        self.beta2, self.eps, log_space=True)
        if "wind" in self.optimise and self.wind is not None:
            m1, m2 = self._m["wind"]
            S.adam_step(self.wind, g["wind"], m1, m2, t, self.lr_wind, self.beta1, self.beta2,
                        self.eps)
        if "forces" in self.optimise:
            m1, m2 = self._m["forces"]
            S.adam_step(self.forces, g["forces"], m1, m2, t, self.lr_forces, self.beta1,
                        self.beta2, self.eps, scale=self._area, n=ta * 3 * sim.n_verts)
        rec = Record(t, ta, energies, float(energies.sum()))
        self.history.append(rec)
        self.window = next_window(self.window, energies, self.n_frames, self.first,
                                  self.max_iters)
        return rec

    def run(self, iterations: int) -> List[Record]:
        return [self.step() for _ in range(iterations)]
