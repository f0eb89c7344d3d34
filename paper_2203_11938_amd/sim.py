"""ctypes binding of ``libphisft_sim.so`` (C ABI in ``include/phisft_sim.h``).

Argument marshalling only: every step of the rollout and of the adjoint runs in
the HIP kernels of the library. PyTorch supplies device memory and the stream.
If the library is missing this module raises -- there is no CPU fallback.

Device tensors at the boundary are structure-of-arrays ``[..., 3, V]`` in the
handle's precision (float32 for FP32, float64 for FP64); material arrays are
float64 ``[n_instances, n_material]``: (k_s, k_b, d) for the isotropic model, or the
anisotropic stretch table S [4, 6], bend table B [3, 5] and d (40 entries, see
``wang_material``).
"""

from __future__ import annotations

import ctypes
import hashlib
import os
import warnings
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libphisft_sim.so")

SIM_OK = 0
SIM_E_INVALID = -1
SIM_E_MESH = -2
SIM_E_NOMEM = -3
SIM_E_HIP = -4
SIM_E_NOT_CONVERGED = -5
SIM_E_INDEFINITE = -6
SIM_E_NONFINITE = -7
SIM_E_STATE = -8
SIM_FP32 = 0
SIM_FP64 = 1
SIM_MEMBRANE_EXACT = 0
SIM_MEMBRANE_TENSION = 1
SIM_MATERIAL_ISOTROPIC = 0
SIM_MATERIAL_WANG = 1
SIM_WANG_PARAMS = 40


def wang_material(stretch, bend, density) -> np.ndarray:
    """The 40 material entries of one sheet for the anisotropic model: stretch table
    [4, 6] (warp, weft, shear, area measures x strain segments) in N/m, bend table
    [3, 5] (0, 45, 90 degree directions x angle segments) in N m, density in kg/m^2."""
    S = np.asarray(stretch, dtype=np.float64).reshape(4, 6)
    B = np.asarray(bend, dtype=np.float64).reshape(3, 5)
    return np.concatenate([S.ravel(), B.ravel(), [float(density)]])


class SimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class _Mesh(ctypes.Structure):
    _fields_ = [("n_verts", ctypes.c_int32), ("n_tris", ctypes.c_int32),
                ("tris", ctypes.POINTER(ctypes.c_int32))]


class _Material(ctypes.Structure):
    _fields_ = [("stretch", ctypes.c_double), ("bend", ctypes.c_double),
                ("density", ctypes.c_double)]


# sim_matrix_home values by index (0: the library's choice)
MATRIX_HOMES = ("auto", "streamed", "lds", "registers")


class _Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("cg_tol", ctypes.c_double),
                ("cg_max_iter", ctypes.c_int32), ("checkpoint_every", ctypes.c_int32),
                ("gravity", ctypes.c_double * 3), ("max_steps", ctypes.c_int32),
                ("rows_per_block", ctypes.c_int32), ("membrane_system", ctypes.c_int32),
                ("matrix_precision", ctypes.c_int32), ("coarse_size", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("matrix_home", ctypes.c_int32), ("air_density", ctypes.c_double),
                ("coarse_keep_all", ctypes.c_int32), ("material_model", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("n_steps", ctypes.c_int32), ("n_instances", ctypes.c_int32),
                ("cg_iters_forward", ctypes.c_int64), ("cg_iters_recompute", ctypes.c_int64),
                ("cg_iters_adjoint", ctypes.c_int64), ("cg_iters_max", ctypes.c_int32),
                ("max_rel_residual", ctypes.c_double), ("device_status", ctypes.c_int32),
                ("rows_per_block", ctypes.c_int32), ("blocks", ctypes.c_int32),
                ("solver_matrix_home", ctypes.c_int32), ("solver_launches_per_solve", ctypes.c_int32),
                ("nnz_blocks", ctypes.c_int64), ("solver_launches", ctypes.c_int64),
                ("solver_ms", ctypes.c_double), ("coarse_aggregates", ctypes.c_int32),
                ("coarse_max_dim", ctypes.c_int32), ("autotuned", ctypes.c_int32),
                ("autotune_candidates", ctypes.c_int32), ("autotune_ms_per_iter", ctypes.c_double),
                ("solver_wg_per_cu", ctypes.c_int32), ("coarse_rows_lds", ctypes.c_int32),
                ("graph_captures", ctypes.c_int64), ("graph_replays", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("coarse_store_slots", ctypes.c_int32),
                ("material_params", ctypes.c_int32), ("solver_row_teams", ctypes.c_int32)]


_lib = None

EXPORTS = ("sim_default_options", "sim_create", "sim_create_batch", "sim_rollout",
           "sim_rollout_noalloc", "sim_adjoint",
           "sim_sync_status", "sim_set_timing", "sim_get_stats", "sim_get_cg_iters",
           "sim_get_instance_status", "sim_frame_loss", "sim_get_vertex_areas",
           "sim_adam_step", "sim_chamfer_workspace_bytes", "sim_chamfer",
           "sim_status_string", "sim_last_error", "sim_destroy")


def load_library(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(the simulator has no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    sig = {
        "sim_default_options": (None, [ctypes.POINTER(_Options)]),
        "sim_create": (i32, [ctypes.POINTER(_Mesh), ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(i32), i32, ctypes.POINTER(_Material), ctypes.c_double,
                             ctypes.POINTER(_Options), ctypes.POINTER(vp)]),
        "sim_create_batch": (i32, [i32, ctypes.POINTER(_Mesh),
                                   ctypes.POINTER(ctypes.POINTER(ctypes.c_double)),
                                   ctypes.POINTER(ctypes.POINTER(i32)), ctypes.POINTER(i32),
                                   ctypes.POINTER(_Material), ctypes.c_double,
                                   ctypes.POINTER(_Options), ctypes.POINTER(vp)]),
        "sim_rollout": (i32, [vp, i32, vp, vp, vp, vp, vp, ctypes.POINTER(i32), i32, vp, vp]),
        "sim_rollout_noalloc": (i32, [vp, i32, vp, vp, vp, vp, vp, ctypes.POINTER(i32), i32, vp,
                                      vp]),
        "sim_adjoint": (i32, [vp, vp, vp, vp, vp, vp, vp, vp]),
        "sim_sync_status": (i32, [vp]),
        "sim_set_timing": (i32, [vp, i32]),
        "sim_get_stats": (i32, [vp, ctypes.POINTER(_Stats)]),
        "sim_get_cg_iters": (i32, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "sim_get_instance_status": (i32, [vp, ctypes.POINTER(i32)]),
        "sim_frame_loss": (i32, [vp, i32, vp, vp, vp, vp, vp]),
        "sim_get_vertex_areas": (i32, [vp, ctypes.POINTER(ctypes.c_double)]),
        "sim_adam_step": (i32, [vp, i32, vp, vp, vp, ctypes.c_int64, vp, i32, i32, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double, i32, vp]),
        "sim_chamfer_workspace_bytes": (ctypes.c_size_t, [i32, i32]),
        "sim_chamfer": (i32, [vp, i32, vp, i32, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]),
        "sim_status_string": (ctypes.c_char_p, [i32]),
        "sim_last_error": (ctypes.c_char_p, [vp]),
        "sim_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def library_identity(path: str = LIB_PATH) -> dict:
    """Path and content hash of the library this process loads (recorded by the
    benchmark so that a measurement names the exact build it ran)."""
    with open(path, "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()[:16]
    return dict(path=os.path.relpath(path, os.path.dirname(HERE)), sha256_16=digest)


def status_name(code: int) -> str:
    """The library's name for a status code."""
    return load_library().sim_status_string(int(code)).decode()


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def adam_step(param: torch.Tensor, grad: torch.Tensor, m1: torch.Tensor, m2: torch.Tensor,
              t: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8, log_space: bool = False, scale: Optional[torch.Tensor] = None,
              n: Optional[int] = None):
    """One Adam step in place on the first n entries of param (sim_adam_step); m1, m2
    float64 moments of param's size; scale [period] float64 or None."""
    lib = load_library()
    if param.dtype not in (torch.float32, torch.float64) or grad.dtype != param.dtype:
        raise ValueError("param and grad must share a float32 or float64 dtype")
    for t_, name in ((param, "param"), (grad, "grad"), (m1, "m1"), (m2, "m2")):
        if not t_.is_cuda or not t_.is_contiguous():
            raise ValueError(f"{name}: expected a contiguous CUDA tensor")
    n = param.numel() if n is None else int(n)
    prec = SIM_FP64 if param.dtype == torch.float64 else SIM_FP32
    st = lib.sim_adam_step(_ptr(param), prec, _ptr(grad), _ptr(m1), _ptr(m2), n, _ptr(scale),
                           0 if scale is None else int(scale.numel()), 1 if log_space else 0,
                           lr, beta1, beta2, eps, int(t), _stream())
    if st != SIM_OK:
        raise SimError(st, "sim_adam_step: " + lib.sim_status_string(st).decode())


def chamfer(g: torch.Tensor, m: torch.Tensor, nearest: bool = False,
            workspace: Optional[torch.Tensor] = None):
    """Chamfer distance (Eq. 10) of the point sets g [3, n_g] and m [3, n_m] (float32
    CUDA tensors, SoA) through sim_chamfer. Returns a float64 tensor [1]; with
    ``nearest`` also each point's smallest squared distance and nearest index in the
    other set (d_g, i_g, d_m, i_m). ``workspace``: a uint8 CUDA tensor of at least
    sim_chamfer_workspace_bytes bytes, reused across calls (allocated here if None)."""
    lib = load_library()
    for t, name in ((g, "g"), (m, "m")):
        if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous() or t.dim() != 2 \
                or t.shape[0] != 3:
            raise ValueError(f"{name}: expected a contiguous float32 CUDA tensor [3, N]")
    ng, nm = int(g.shape[1]), int(m.shape[1])
    need = lib.sim_chamfer_workspace_bytes(ng, nm)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=g.device)
    ch = torch.empty(1, dtype=torch.float64, device=g.device)
    out = {}
    if nearest:
        out = dict(d_g=torch.empty(ng, dtype=torch.float32, device=g.device),
                   i_g=torch.empty(ng, dtype=torch.int32, device=g.device),
                   d_m=torch.empty(nm, dtype=torch.float32, device=g.device),
                   i_m=torch.empty(nm, dtype=torch.int32, device=g.device))
    st = lib.sim_chamfer(_ptr(g), ng, _ptr(m), nm, _ptr(ch), _ptr(out.get("d_g")),
                         _ptr(out.get("i_g")), _ptr(out.get("d_m")), _ptr(out.get("i_m")),
                         _ptr(workspace), workspace.numel(), _stream())
    if st != SIM_OK:
        raise SimError(st, "sim_chamfer: " + lib.sim_status_string(st).decode())
    return (ch, out) if nearest else ch


@dataclass
class Sheet:
    """One sheet's host description: triangles [T,3], rest positions [V,3], pins."""
    tris: np.ndarray
    rest: np.ndarray
    pins: Sequence[int]
    stretch: float
    bend: float
    density: float


class Simulator:
    """A handle of the library over one or several sheets (batched when several).

    ``dt`` is the step h [s]; ``precision`` "fp32" or "fp64"; ``cg_tol`` the
    relative residual at which each CG solve stops; ``checkpoint_every`` k > 0
    keeps every k-th state and recomputes the rest in the adjoint; ``membrane``
    selects the system matrix's membrane block ("exact" Hessian or "tension");
    ``coarse_size`` sets the vertices per aggregate of the solver's coarse space
    (0: block-Jacobi only); ``autotune`` times the feasible solver launch shapes at
    creation and keeps the fastest; ``graph`` captures rollout and adjoint into HIP
    graphs that later calls with the same arrays replay; ``matrix_home`` pins where
    the solver keeps its matrix rows ("streamed", "lds" or "registers"; None: the
    library's choice); ``air_density`` is the aerodynamic force's rho_air [kg/m^3]
    (acting in rollouts given a wind velocity); ``coarse_keep_all`` keeps every
    step's coarse operators under checkpointing (faster, memory not bounded by the
    checkpoint interval); ``material_model`` "wang" selects the anisotropic
    strain-dependent material (material arrays of 40 entries per sheet).
    """

    def __init__(self, sheets: Sequence[Sheet], dt: float, precision: str = "fp32",
                 cg_tol: float = 1e-7, cg_max_iter: int = 20000, checkpoint_every: int = 0,
                 max_steps: int = 1000, gravity=(0.0, 0.0, -9.81), rows_per_block: int = 0,
                 membrane: str = "exact", matrix_precision: str = "fp64",
                 coarse_size: Optional[int] = None, autotune: bool = False,
                 graph: bool = False, matrix_home: Optional[str] = None,
                 air_density: float = 1.0, coarse_keep_all: bool = False,
                 material_model: str = "isotropic"):
        lib = load_library()
        self._lib = lib
        self._h = None
        opt = _Options()
        lib.sim_default_options(ctypes.byref(opt))
        opt.precision = SIM_FP64 if precision == "fp64" else SIM_FP32
        opt.cg_tol = cg_tol
        opt.cg_max_iter = cg_max_iter
        opt.checkpoint_every = checkpoint_every
        opt.max_steps = max_steps
        opt.gravity[:] = list(gravity)
        opt.rows_per_block = rows_per_block
        if membrane not in ("exact", "tension"):
            raise ValueError("membrane must be 'exact' or 'tension'")
        opt.membrane_system = SIM_MEMBRANE_TENSION if membrane == "tension" else SIM_MEMBRANE_EXACT
        opt.matrix_precision = SIM_FP32 if matrix_precision == "fp32" else SIM_FP64
        if coarse_size is not None:
            opt.coarse_size = coarse_size
        opt.autotune = 1 if autotune else 0
        opt.graph = 1 if graph else 0
        opt.air_density = air_density
        opt.coarse_keep_all = 1 if coarse_keep_all else 0
        if material_model not in ("isotropic", "wang"):
            raise ValueError("material_model must be 'isotropic' or 'wang'")
        opt.material_model = SIM_MATERIAL_WANG if material_model == "wang" else SIM_MATERIAL_ISOTROPIC
        self.material_model = material_model
        self.n_material = SIM_WANG_PARAMS if material_model == "wang" else 3
        if matrix_home is not None:
            if matrix_home not in MATRIX_HOMES[1:]:
                raise ValueError(f"matrix_home must be one of {MATRIX_HOMES[1:]}")
            opt.matrix_home = MATRIX_HOMES.index(matrix_home)
        self.matrix_precision = matrix_precision
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        n = len(sheets)
        keep = []
        meshes = (_Mesh * n)()
        rests = (ctypes.POINTER(ctypes.c_double) * n)()
        pins = (ctypes.POINTER(ctypes.c_int32) * n)()
        npins = (ctypes.c_int32 * n)()
        mats = (_Material * n)()
        self.sizes = []
        for b, s in enumerate(sheets):
            tr = np.ascontiguousarray(s.tris, dtype=np.int32).reshape(-1, 3)
            rp = np.ascontiguousarray(s.rest, dtype=np.float64).reshape(-1, 3)
            pn = np.ascontiguousarray(np.asarray(s.pins, dtype=np.int32).reshape(-1))
            keep += [tr, rp, pn]
            meshes[b].n_verts = rp.shape[0]
            meshes[b].n_tris = tr.shape[0]
            meshes[b].tris = tr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            rests[b] = rp.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            pins[b] = pn.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if pn.size else None
            npins[b] = pn.size
            mats[b] = _Material(s.stretch, s.bend, s.density)
            self.sizes.append(rp.shape[0])
        h = ctypes.c_void_p()
        st = lib.sim_create_batch(n, meshes, rests, pins, npins, mats, dt, ctypes.byref(opt),
                                  ctypes.byref(h))
        if st != SIM_OK:
            raise SimError(st, "sim_create_batch: " + lib.sim_status_string(st).decode())
        self._h = h
        self.n_instances = n
        self.n_verts = int(sum(self.sizes))
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(int)
        self.dt = dt
        self.max_steps = max_steps
        self.n_steps = 0
        self.n_loss = 0
        # rollouts run on this handle so far: the autograd path checks that a backward
        # pass still refers to the rollout of its own forward pass
        self.generation = 0
        # ClothRollout: accept SIM_E_NOT_CONVERGED (with a warning) instead of raising
        self.allow_not_converged = False

    def close(self):
        if self._h is not None:
            self._lib.sim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, what: str):
        if st != SIM_OK:
            msg = self._lib.sim_last_error(self._h).decode() if self._h else ""
            raise SimError(st, f"{what}: {self._lib.sim_status_string(st).decode()} {msg}")

    def _need(self, t: Optional[torch.Tensor], shape, name: str, dtype=None):
        if t is None:
            return None
        dtype = dtype or self.dtype
        if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name}: expected a contiguous {dtype} CUDA tensor of shape "
                             f"{tuple(shape)}, got {t.dtype} {tuple(t.shape)} "
                             f"{'cuda' if t.is_cuda else 'cpu'}")
        return t

    def rollout(self, n_steps: int, x0: torch.Tensor, v0: Optional[torch.Tensor] = None,
                forces: Optional[torch.Tensor] = None, material: Optional[torch.Tensor] = None,
                loss_frames: Optional[Sequence[int]] = None, x_out: Optional[torch.Tensor] = None,
                wind: Optional[torch.Tensor] = None, noalloc: bool = False):
        """Run ``n_steps`` steps. Returns positions at the loss frames [n_loss, 3, V].
        ``wind`` [n_instances, 3] float64 is each sheet's wind velocity (None: no
        aerodynamic force). ``noalloc`` calls the allocation-free entry point
        (sim_rollout_noalloc); pass ``x_out`` too so that nothing is allocated."""
        V = self.n_verts
        frames = np.arange(1, n_steps + 1, dtype=np.int32) if loss_frames is None else \
            np.ascontiguousarray(loss_frames, dtype=np.int32)
        self._need(x0, (3, V), "x0")
        self._need(v0, (3, V), "v0")
        self._need(forces, (n_steps, 3, V), "forces")
        self._need(material, (self.n_instances, self.n_material), "material", torch.float64)
        self._need(wind, (self.n_instances, 3), "wind", torch.float64)
        if x_out is None:
            x_out = torch.empty((frames.size, 3, V), dtype=self.dtype, device=x0.device)
        self._need(x_out, (frames.size, 3, V), "x_out")
        fn = self._lib.sim_rollout_noalloc if noalloc else self._lib.sim_rollout
        st = fn(self._h, int(n_steps), _ptr(x0), _ptr(v0), _ptr(forces), _ptr(material),
                _ptr(wind), frames.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                int(frames.size), _ptr(x_out), _stream())
        self._check(st, "sim_rollout_noalloc" if noalloc else "sim_rollout")
        # the adjoint re-reads these; keep them alive
        self._keep = (forces, material, wind)
        self.has_wind = wind is not None
        self.n_steps = n_steps
        self.n_loss = int(frames.size)
        self.loss_frames = frames
        self.generation += 1
        return x_out

    def adjoint(self, dl_dx: torch.Tensor, want_forces: bool = True, want_x0: bool = True,
                want_v0: bool = True, want_material: bool = True, out: Optional[dict] = None,
                want_wind: Optional[bool] = None):
        """Gradients of the loss whose frame gradients are ``dl_dx`` [n_loss, 3, V].

        ``out`` may hold preallocated result tensors (keys material, wind, forces, x0,
        v0); passing the same ones on every call lets a graph-mode handle replay. The
        wind gradient is returned when the rollout had a wind (``want_wind`` None)."""
        V = self.n_verts
        self._need(dl_dx, (self.n_loss, 3, V), "dl_dx")
        dev = dl_dx.device
        out = out or {}
        def buf(key, want, shape, dtype):
            if not want:
                return None
            t = out.get(key)
            if t is None:
                return torch.empty(shape, dtype=dtype, device=dev)
            self._need(t, shape, key, dtype)
            return t
        g_mat = buf("material", want_material, (self.n_instances, self.n_material), torch.float64)
        if want_wind is None:
            want_wind = getattr(self, "has_wind", False)
        g_w = buf("wind", want_wind, (self.n_instances, 3), torch.float64)
        g_F = buf("forces", want_forces, (self.n_steps, 3, V), self.dtype)
        g_x0 = buf("x0", want_x0, (3, V), self.dtype)
        g_v0 = buf("v0", want_v0, (3, V), self.dtype)
        st = self._lib.sim_adjoint(self._h, _ptr(dl_dx), _ptr(g_mat), _ptr(g_w), _ptr(g_F),
                                   _ptr(g_x0), _ptr(g_v0), _stream())
        self._check(st, "sim_adjoint")
        return dict(material=g_mat, wind=g_w, forces=g_F, x0=g_x0, v0=g_v0)

    def sync(self, allow_not_converged: bool = False) -> int:
        """Wait for the stream; raise on a sticky device error."""
        st = self._lib.sim_sync_status(self._h)
        if st == SIM_E_NOT_CONVERGED and allow_not_converged:
            return st
        self._check(st, "device status")
        return st

    def set_timing(self, enable: bool):
        self._check(self._lib.sim_set_timing(self._h, 1 if enable else 0), "sim_set_timing")

    def status(self) -> int:
        return self._lib.sim_sync_status(self._h)

    def stats(self) -> dict:
        s = _Stats()
        self._check(self._lib.sim_get_stats(self._h, ctypes.byref(s)), "sim_get_stats")
        return {k: getattr(s, k) for k, _ in _Stats._fields_}

    def instance_status(self) -> np.ndarray:
        out = np.zeros(self.n_instances, dtype=np.int32)
        self._check(self._lib.sim_get_instance_status(self._h, out.ctypes.data_as(
            ctypes.POINTER(ctypes.c_int32))), "sim_get_instance_status")
        return out

    def frame_loss(self, x: torch.Tensor, target: torch.Tensor, energy: torch.Tensor,
                   dl_dx: Optional[torch.Tensor] = None):
        """Per frame and sheet, sum |x - target|^2 into energy [n_frames, n_instances]
        (float64) and 2 (x - target) into dl_dx (sim_frame_loss); x, target, dl_dx
        [n_frames, 3, V] in the handle's precision."""
        nf = int(x.shape[0])
        self._need(x, (nf, 3, self.n_verts), "x")
        self._need(target, (nf, 3, self.n_verts), "target")
        self._need(energy, (nf, self.n_instances), "energy", torch.float64)
        self._need(dl_dx, (nf, 3, self.n_verts), "dl_dx")
        self._check(self._lib.sim_frame_loss(self._h, nf, _ptr(x), _ptr(target), _ptr(energy),
                                             _ptr(dl_dx), _stream()), "sim_frame_loss")

    def vertex_areas(self) -> np.ndarray:
        """Lumped vertex areas [V] (caller's order)."""
        out = np.zeros(self.n_verts)
        self._check(self._lib.sim_get_vertex_areas(
            self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "sim_get_vertex_areas")
        return out

    def cg_iters(self):
        n = self.n_steps * self.n_instances
        f = np.zeros(n, dtype=np.int32)
        a = np.zeros(n, dtype=np.int32)
        self._check(self._lib.sim_get_cg_iters(self._h, f.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                               a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
                    "sim_get_cg_iters")
        return f.reshape(self.n_steps, self.n_instances), a.reshape(self.n_steps, self.n_instances)


def _sync_checked(sim: Simulator, what: str):
    st = sim.sync(allow_not_converged=sim.allow_not_converged)
    if st == SIM_E_NOT_CONVERGED:
        warnings.warn(f"{what}: a CG solve did not converge (cg_max_iter or unverified "
                      "residual); results use the last iterate", RuntimeWarning)


class ClothRollout(torch.autograd.Function):
    """Differentiable rollout: (material, forces, x0, v0, wind) -> positions at the loss
    frames.

    User-facing layout is vertex-major: forces [n_steps, V, 3], x0/v0 [V, 3],
    output [n_loss, V, 3]; material [n_instances, n_material] and wind [n_instances, 3]
    float64 (wind None:
    no aerodynamic force). The backward pass is the library's adjoint of the
    handle's most recent rollout, so it raises if another rollout ran on the same
    handle in between; a solve that did not converge raises too unless
    ``sim.allow_not_converged`` is set (then it warns). Double backward is not
    supported.
    """

    @staticmethod
    def forward(ctx, sim: Simulator, n_steps: int, loss_frames, material, forces, x0, v0,
                wind=None):
        soa = lambda t: None if t is None else t.transpose(-1, -2).contiguous()
        xo = sim.rollout(n_steps, soa(x0), soa(v0), soa(forces), material.contiguous(),
                         loss_frames, wind=None if wind is None else wind.contiguous())
        _sync_checked(sim, "rollout")
        ctx.sim = sim
        ctx.generation = sim.generation
        ctx.has_forces = forces is not None
        ctx.has_v0 = v0 is not None
        ctx.has_wind = wind is not None
        return xo.transpose(-1, -2).contiguous()

    @staticmethod
    def backward(ctx, g):
        sim = ctx.sim
        if sim.generation != ctx.generation:
            raise RuntimeError("the simulator handle has run another rollout since this "
                               "forward pass; its adjoint would belong to that rollout "
                               "(use one handle per pending backward pass)")
        r = sim.adjoint(g.transpose(-1, -2).contiguous(), want_forces=ctx.has_forces,
                        want_wind=ctx.has_wind)
        _sync_checked(sim, "adjoint")
        aos = lambda t: None if t is None else t.transpose(-1, -2).contiguous()
        return (None, None, None, r["material"], aos(r["forces"]), aos(r["x0"]),
                aos(r["v0"]) if ctx.has_v0 else None, r["wind"] if ctx.has_wind else None)


def rollout(sim: Simulator, n_steps: int, material, x0, v0=None, forces=None, loss_frames=None,
            wind=None):
    """Differentiable rollout through the library (see ClothRollout)."""
    return ClothRollout.apply(sim, n_steps, loss_frames, material, forces, x0, v0, wind)
