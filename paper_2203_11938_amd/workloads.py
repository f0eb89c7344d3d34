"""Seeded synthetic inputs for the cloth simulator: sheets, pins, forces, states.

This module holds input recipes only -- no simulator arithmetic. Both the GPU
library's tests/benchmark and the FP64 oracle read the arrays it produces.

The paper measures on captured sequences (~300-vertex templates, ~40 frames;
Sec. 4) that are not available here; these seeded sheets stand in for them.

Conventions (readings of details the paper leaves open):
  * square sheet of side L = 0.5 m with n x n vertices, vertex id j*n + i at
    rest position (i*L/(n-1), j*L/(n-1), 0); horizontal start, gravity along -z;
  * each grid quad (a=(i,j), b=(i+1,j), c=(i,j+1), d=(i+1,j+1)) is split along
    a-d into the counter-clockwise triangles (a, b, d) and (a, d, c);
  * "top" is the row j = n-1;
  * all randomness is numpy PCG64 seeded with 1000*c + stream, c the workload
    number, streams: 0 target material factors, 1 forces, 2 initial
    perturbation, 3 batch sizes and materials, 4 finite-difference directions.

Arrays are vertex-major ``[V, 3]`` float64 here; the library boundary is
``[3, V]`` (see ``to_soa``).
"""

from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

SHEET_SIDE = 0.5
GRAVITY = (0.0, 0.0, -9.81)


def rng(workload: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * workload + stream))


def grid_sheet(n: int, side: float = SHEET_SIDE):
    """Rest positions [n*n, 3] and triangles [2(n-1)^2, 3] of a regular sheet."""
    if n < 2:
        raise ValueError("a sheet needs at least 2x2 vertices")
    a = side / (n - 1)
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    rest = np.stack([i.ravel() * a, j.ravel() * a, np.zeros(n * n)], axis=1).astype(np.float64)
    tris = []
    for jj in range(n - 1):
        for ii in range(n - 1):
            va = jj * n + ii
            vb = va + 1
            vc = va + n
            vd = vc + 1
            tris.append((va, vb, vd))
            tris.append((va, vd, vc))
    return rest, np.asarray(tris, dtype=np.int32)


def pin_set(n: int, kind: str) -> np.ndarray:
    top = (n - 1) * n
    if kind == "top2":
        return np.array([top, top + n - 1], dtype=np.int32)
    if kind == "corner":
        return np.array([top], dtype=np.int32)
    if kind == "topedge":
        return np.arange(top, top + n, dtype=np.int32)
    if kind == "none":
        return np.zeros(0, dtype=np.int32)
    raise ValueError(kind)


def grid_vertex_area(n: int, side: float = SHEET_SIDE) -> np.ndarray:
    """Area share of each grid vertex, a^2 * (incident triangles) / 6 -- used only
    to turn the wind pressure recipe of the 200x200 workload into nodal forces."""
    a = side / (n - 1)
    _, tris = grid_sheet(n, side)
    cnt = np.bincount(tris.ravel(), minlength=n * n)
    return a * a * cnt / 6.0


def fourier_wind(n: int, generator: np.random.Generator, amplitude: float = 0.1,
                 modes: int = 8, side: float = SHEET_SIDE) -> np.ndarray:
    """Spatially smooth wind pressure field [V, 3] in N/m^2: the mean of ``modes``
    random Fourier modes d_k cos(2 pi kappa_k . X / L + phase_k), kappa_k drawn from
    {-3..3}^2 without 0, d_k uniform on the unit sphere, scaled by ``amplitude``."""
    rest, _ = grid_sheet(n, side)
    kap = []
    while len(kap) < modes:
        k = generator.integers(-3, 4, size=2)
        if k[0] != 0 or k[1] != 0:
            kap.append(k)
    kap = np.asarray(kap, dtype=np.float64)
    d = generator.normal(size=(modes, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    ph = generator.uniform(0.0, 2.0 * np.pi, size=modes)
    arg = 2.0 * np.pi * (rest[:, :2] @ kap.T) / side + ph[None, :]
    return amplitude * (np.cos(arg) @ d) / modes


@dataclass
class Material:
    stretch: float = 1e3   # k_s [N/m]
    bend: float = 1e-4     # k_b [N m]
    density: float = 0.1   # d [kg/m^2]

    def as_tuple(self):
        return (self.stretch, self.bend, self.density)


@dataclass
class Workload:
    name: str
    number: int            # seed family
    n: int                 # vertices per side
    steps: int
    dt: float
    pins: str
    material: Material = field(default_factory=Material)
    forces: str = "zero"   # zero | gauss | wind
    force_sigma: float = 0.05
    perturb_sigma: float = 0.0   # normal displacement of free vertices [m]
    precision: str = "fp32"
    cg_tol: float = 1e-7
    checkpoint_every: int = 0    # 0 = store every state
    loss_every: int = 1          # loss on frames loss_every, 2*loss_every, ...
    batch: int = 1               # independent instances (sizes drawn when > 1)
    batch_n_range: tuple = (16, 64)

    @property
    def n_verts(self):
        return self.n * self.n

    def loss_frames(self) -> np.ndarray:
        return np.arange(self.loss_every, self.steps + 1, self.loss_every, dtype=np.int32)


WORKLOADS = {
    # 10x10 plain forward sheet, FP64 both sides, CG tol 1e-10, 50 steps.
    "C1": Workload("C1", 1, 10, 50, 0.01, "top2", precision="fp64", cg_tol=1e-10),
    # 32x32 forward + adjoint, per-vertex per-step Gaussian wind load N(0, 0.05^2) N/m^2
    # times the vertex's area share.
    "C2": Workload("C2", 2, 32, 100, 0.01, "top2", forces="gauss"),
    # 64x64, 200 steps of 5 ms, one corner pinned, 1 mm normal perturbation,
    # checkpoint every 20 steps, loss on every 10th frame.
    "C3": Workload("C3", 3, 64, 200, 0.005, "corner", perturb_sigma=1e-3, checkpoint_every=20,
                   loss_every=10),
    # 64 independent sheets, sizes 16..64 per side, log-uniform materials.
    "C4": Workload("C4", 4, 64, 100, 0.01, "top2", forces="gauss", batch=64),
    # 200x200, 300 steps of 5 ms, top edge pinned, Fourier wind, checkpoint 30.
    "C5": Workload("C5", 5, 200, 300, 0.005, "topedge", forces="wind", checkpoint_every=30,
                   loss_every=10),
    # Headline: 100-step 64x64 sheet, C2 force recipe, store-all.
    "H": Workload("H", 6, 64, 100, 0.01, "top2", forces="gauss"),
}


def workload(name: str, **overrides) -> Workload:
    w = WORKLOADS[name]
    return replace(w, **overrides) if overrides else w


@dataclass
class Instance:
    """One sheet's inputs, vertex-major float64."""
    rest: np.ndarray
    tris: np.ndarray
    pins: np.ndarray
    material: Material
    x0: np.ndarray
    v0: np.ndarray
    forces: Optional[np.ndarray]   # [steps, V, 3] or None
    target_factors: np.ndarray     # multipliers of (k_s, k_b, d) for the target rollout

    @property
    def n_verts(self):
        return self.rest.shape[0]


def _instance(w: Workload, n: int, material: Material, force_rng, perturb_rng,
              factor_rng) -> Instance:
    rest, tris = grid_sheet(n)
    pins = pin_set(n, w.pins)
    V = n * n
    x0 = rest.copy()
    if w.perturb_sigma > 0:
        free = np.ones(V, dtype=bool)
        free[pins] = False
        xi = perturb_rng.normal(0.0, w.perturb_sigma, size=V)
        x0[free, 2] += xi[free]
    v0 = np.zeros((V, 3))
    if w.forces == "zero":
        forces = None
    elif w.forces == "gauss":
        # sigma read as a wind load in N/m^2 on each vertex's area share: taken as a
        # nodal force in N (0.05 N on a ~24 mg vertex, ~200 g) the linearised step
        # diverges within a few frames.
        xi = force_rng.normal(0.0, w.force_sigma, size=(w.steps, V, 3))
        forces = xi * grid_vertex_area(n)[None, :, None]
    elif w.forces == "wind":
        f = fourier_wind(n, force_rng) * grid_vertex_area(n)[:, None]
        forces = np.broadcast_to(f, (w.steps, V, 3)).copy()
    else:
        raise ValueError(w.forces)
    factors = factor_rng.uniform(0.5, 2.0, size=3)
    return Instance(rest, tris, pins, material, x0, v0, forces, factors)


def make_instances(w: Workload) -> list:
    """The workload's instances (one unless ``w.batch`` > 1)."""
    fr, pr, tr = rng(w.number, 1), rng(w.number, 2), rng(w.number, 0)
    if w.batch == 1:
        return [_instance(w, w.n, w.material, fr, pr, tr)]
    br = rng(w.number, 3)
    lo, hi = w.batch_n_range
    out = []
    for _ in range(w.batch):
        n = int(br.integers(lo, hi + 1))
        mat = Material(stretch=float(np.exp(br.uniform(np.log(1e2), np.log(1e4)))),
                       bend=float(np.exp(br.uniform(np.log(1e-5), np.log(1e-3)))),
                       density=float(np.exp(br.uniform(np.log(0.05), np.log(0.3)))))
        out.append(_instance(w, n, mat, fr, pr, tr))
    return out


def loss_targets(w: Workload, inst: Instance, frames, scale: float = 0.01,
                 sheet: int = 0) -> np.ndarray:
    """Seeded target positions [n_frames, V, 3] for the full-size parity runs: the
    initial positions plus N(0, scale^2) m offsets per frame (stream 4, jumped ahead
    by the sheet's index in a batch). A cheap stand-in for the scaled-material target
    rollout, which on the largest sheets would cost as much oracle time as the
    gradient itself."""
    g = np.random.Generator(np.random.PCG64(1000 * w.number + 4).jumped(sheet))
    frames = np.asarray(frames)
    return inst.x0[None] + scale * g.normal(size=(frames.size,) + inst.x0.shape)


def fd_directions(w: Workload, count: int, shape) -> np.ndarray:
    """Seeded unit directions for finite-difference checks."""
    g = rng(w.number, 4)
    d = g.normal(size=(count,) + tuple(shape))
    d /= np.linalg.norm(d.reshape(count, -1), axis=1).reshape((count,) + (1,) * len(shape))
    return d


def chamfer_points(n_g: int, n_m: int, seed: int = 7000):
    """Point sets for the Chamfer distance (Eq. 10), vertex-major float64: G, a noisy
    scan of a folded sheet (uniform samples of a smooth height field over the 0.5 m
    square plus N(0, (1 mm)^2) noise per coordinate, like a depth camera's point cloud),
    and M, points sampled from a reconstruction of it that is off by a smooth 3 mm
    misfit. Seeded (PCG64); the paper's captured clouds are not available."""
    g_rng = np.random.Generator(np.random.PCG64(seed))

    def surface(u, v, misfit):
        z = 0.04 * np.sin(3.0 * np.pi * u / SHEET_SIDE) * np.cos(2.0 * np.pi * v / SHEET_SIDE) \
            + 0.02 * np.sin(np.pi * (u + v) / SHEET_SIDE)
        z = z + misfit * np.sin(5.0 * np.pi * u / SHEET_SIDE + 1.0) * np.sin(4.0 * np.pi * v / SHEET_SIDE)
        return np.stack([u, v, z], axis=1)

    ug, vg = g_rng.uniform(0.0, SHEET_SIDE, size=(2, n_g))
    g = surface(ug, vg, 0.0) + g_rng.normal(0.0, 1e-3, size=(n_g, 3))
    um, vm = g_rng.uniform(0.0, SHEET_SIDE, size=(2, n_m))
    m = surface(um, vm, 3e-3)
    return g, m


@dataclass
class WindowProblem:
    """Inputs of the outer-loop (window + Adam) workload: a sheet, the hidden parameters
    that produced its observed sequence, and the optimiser's starting guess."""
    workload: Workload
    instance: Instance
    true_material: tuple
    true_wind: np.ndarray        # [3] m/s
    guess_material: tuple
    guess_wind: np.ndarray       # [3] m/s (zero, as the paper initialises it)


def window_problem(n: int = 17, frames: int = 40, precision: str = "fp64",
                   cg_tol: float = 1e-10) -> WindowProblem:
    """A stand-in for one of the paper's sequences (~300-vertex template, ~40 frames,
    Sec. 4): an n x n sheet hanging from its two top corners, 10 ms steps. The observed
    frames are a rollout under hidden parameters: (k_s, k_b, d) of the default material
    times seeded U[0.5, 2] factors (stream 0) and a wind of seeded direction and speed
    U[1, 3] m/s (stream 5). The optimiser starts from the default material, zero wind
    and zero forces. Seeds: workload number 7."""
    w = Workload("N3", 7, n, frames, 0.01, "top2", precision=precision, cg_tol=cg_tol)
    inst = _instance(w, n, w.material, rng(7, 1), rng(7, 2), rng(7, 0))
    g = rng(7, 5)
    d = g.normal(size=3)
    wind = d / np.linalg.norm(d) * g.uniform(1.0, 3.0)
    true_mat = tuple(np.array(w.material.as_tuple()) * inst.target_factors)
    return WindowProblem(w, inst, true_mat, wind, w.material.as_tuple(), np.zeros(3))


def as_given(inst: Instance, precision: str) -> Instance:
    """The instance's inputs as a handle of the given precision receives them: an FP32
    handle takes x0, v0 and the forces as float32, so a reference fed the same rounded
    values sees the same problem (rest positions stay float64: sim_create takes them
    in double)."""
    if precision != "fp32":
        return inst
    q = lambda a: None if a is None else a.astype(np.float32).astype(np.float64)
    return replace(inst, x0=q(inst.x0), v0=q(inst.v0), forces=q(inst.forces))


def to_soa(a: np.ndarray) -> np.ndarray:
    """[..., V, 3] -> [..., 3, V] (the library's coalesced layout)."""
    return np.ascontiguousarray(np.swapaxes(a, -1, -2))


def from_soa(a: np.ndarray) -> np.ndarray:
    """[..., 3, V] -> [..., V, 3]."""
    return np.ascontiguousarray(np.swapaxes(a, -1, -2))
