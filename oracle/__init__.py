"""FP64 CPU oracle of the phi-SfT cloth step and its adjoint -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never loads it and shares
no code with it.

The arithmetic lives in ``phisft_oracle.cpp`` (plain single-threaded C++17,
FP64); this module is argument marshalling through ctypes. Arrays are
vertex-major ``[V, 3]`` float64 (the GPU library's boundary uses ``[3, V]``).
Every function cites the part of the paper it follows (Sec. 3.1, Eq. 1-5, and
the backward pass by implicit differentiation).
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import build_oracle, library_path

ORC_OK = 0
ORC_E_INVALID = -1
ORC_E_MESH = -2
ORC_E_NOT_CONVERGED = -5
ORC_E_INDEFINITE = -6
ORC_E_NONFINITE = -7

_lib = None


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        build_oracle()
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    D = ctypes.POINTER(ctypes.c_double)
    I = ctypes.POINTER(ctypes.c_int)
    c_int, c_double = ctypes.c_int, ctypes.c_double
    sig = {
        "orc_create": (P, [c_int, c_int, I, D, I, c_int, I]),
        "orc_destroy": (None, [P]),
        "orc_set_params": (c_int, [P] + [c_double] * 8 + [c_int]),
        "orc_set_membrane_system": (c_int, [P, c_int]),
        "orc_num_hinges": (c_int, [P]),
        "orc_num_blocks": (c_int, [P]),
        "orc_get_geometry": (None, [P, D, D, D, I, D, D]),
        "orc_energy": (c_double, [P, D, D, D]),
        "orc_internal_force": (None, [P, D, D]),
        "orc_ksys_apply": (None, [P, D, D, D]),
        "orc_kexact_apply": (None, [P, D, D, D]),
        "orc_ksys_assembled_apply": (None, [P, D, D, D]),
        "orc_third": (None, [P, D, D, D, D]),
        "orc_hinge_theta": (c_double, [D]),
        "orc_hinge_theta_grad": (None, [D, D]),
        "orc_system": (c_int, [P, D, D, D, D, D]),
        "orc_solve_step": (c_int, [P, D, D, D, D, I]),
        "orc_step_residual": (c_int, [P, D, D, D, D, D, D]),
        "orc_step": (c_int, [P, D, D, D, D, D, D, I]),
        "orc_rollout": (c_int, [P, c_int, D, D, D, I, c_int, D, D, I]),
        "orc_gradient": (c_int, [P, c_int, D, D, D, I, c_int, D, D, D, D, D, D, I, I]),
        "orc_pattern": (None, [P, I, I]),
        "orc_system_blocks": (c_int, [P, D, D, D, D, D]),
        "orc_adjoint_rhs": (None, [P, D, D, D]),
        "orc_adjoint_update": (None, [P, D, D, D, D, D, D, D, D, D, D]),
        "orc_set_wind": (c_int, [P, c_int, c_double, c_double, c_double, c_double]),
        "orc_wind_force": (None, [P, D, D, D]),
        "orc_set_material": (c_int, [P, c_int, D, D]),
        "orc_num_material": (c_int, [P]),
        "orc_get_material_frames": (None, [P, D, D]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _d(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def hinge_theta(x4):
    """Dihedral angle of one hinge (x0, x1 | x2, x3), bending model reading R8."""
    x4 = _f64(x4, (4, 3))
    return _load().orc_hinge_theta(_d(x4))


def hinge_theta_grad(x4):
    """Closed-form gradient of the dihedral angle, shape [4, 3]."""
    x4 = _f64(x4, (4, 3))
    g = np.zeros((4, 3))
    _load().orc_hinge_theta_grad(_d(x4), _d(g))
    return g


class ExactSolve:
    """Sparse LU of one step matrix A with one step of iterative refinement per
    solve. The factorisation first runs without pivoting on the symmetric structure
    (the matrix is symmetric and, away from breakdowns, positive definite); if a
    solve's refined residual is not at rounding level it refactors with partial
    pivoting."""

    def __init__(self, A):
        import scipy.sparse.linalg as spla
        self.A = A
        self._spla = spla
        self._csc = A.tocsc()
        self.lu = spla.splu(self._csc, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                            options=dict(SymmetricMode=True))
        self.pivoted = False

    def _solve(self, rhs):
        x = self.lu.solve(rhs)
        return x + self.lu.solve(rhs - self.A @ x)

    def solve(self, rhs):
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        x = self._solve(rhs)
        nb = np.linalg.norm(rhs)
        if nb > 0 and not np.linalg.norm(self.A @ x - rhs) <= 1e-9 * nb and not self.pivoted:
            self.lu = self._spla.splu(self._csc, permc_spec="MMD_AT_PLUS_A")
            self.pivoted = True
            x = self._solve(rhs)
        return x


class Oracle:
    """One cloth sheet: topology, rest state, pins (Sec. 3.1 'Deformation Model').

    Parameters mirror the GPU library's ``sim_create``: a triangle mesh with
    fixed topology, rest positions [V, 3], pinned vertex ids, material
    (k_s [N/m], k_b [N m], d [kg/m^2]), time step h [s], gravity and the CG
    tolerance of the oracle's own solver.
    """

    def __init__(self, tris, rest, pins=(), ks=1e3, kb=1e-4, density=0.1, dt=0.01,
                 gravity=(0.0, 0.0, -9.81), cg_tol=1e-12, cg_max_iter=100000):
        lib = _load()
        self.tris = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
        self.rest = _f64(rest).reshape(-1, 3)
        self.pins = np.ascontiguousarray(pins, dtype=np.int32).reshape(-1)
        self.nv = self.rest.shape[0]
        self.nt = self.tris.shape[0]
        st = ctypes.c_int(0)
        self._h = lib.orc_create(self.nv, self.nt, _i(self.tris), _d(self.rest),
                                 _i(self.pins) if self.pins.size else None,
                                 int(self.pins.size), ctypes.byref(st))
        if not self._h:
            raise OracleError(st.value, "create")
        self.set_params(ks, kb, density, dt, gravity, cg_tol, cg_max_iter)
        self.nh = lib.orc_num_hinges(self._h)
        self.nnzb = lib.orc_num_blocks(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_destroy(h)
            self._h = None

    def set_params(self, ks=None, kb=None, density=None, dt=None, gravity=None, cg_tol=None,
                   cg_max_iter=None):
        self.ks = self.__dict__.get("ks", 0.0) if ks is None else float(ks)
        self.kb = self.__dict__.get("kb", 0.0) if kb is None else float(kb)
        self.density = self.__dict__.get("density", 0.0) if density is None else float(density)
        self.dt = self.__dict__.get("dt", 0.01) if dt is None else float(dt)
        if gravity is not None:
            self.gravity = tuple(float(g) for g in gravity)
        if cg_tol is not None:
            self.cg_tol = float(cg_tol)
        if cg_max_iter is not None:
            self.cg_max_iter = int(cg_max_iter)
        st = _load().orc_set_params(self._h, self.ks, self.kb, self.density, self.dt,
                                    *self.gravity, self.cg_tol, self.cg_max_iter)
        if st != ORC_OK:
            raise OracleError(st, "set_params")

    MEMBRANE_GAUSS_NEWTON = 0
    MEMBRANE_EXACT = 1
    MEMBRANE_TENSION = 2

    def set_wind(self, wind=None, air_density=1.0):
        """Wind velocity w [m/s] (Eq. 2's w) and air density [kg/m^3] of the
        aerodynamic force (reading R19; the paper fixes the density at 1 kg/m^3,
        Sec. 3.4). None switches the force off."""
        on = wind is not None
        w = (0.0, 0.0, 0.0) if wind is None else tuple(float(c) for c in wind)
        st = _load().orc_set_wind(self._h, 1 if on else 0, *w, float(air_density))
        if st != ORC_OK:
            raise OracleError(st, "set_wind")
        self.wind = None if wind is None else np.array(w)

    def set_material_wang(self, stretch=None, bend=None):
        """Anisotropic strain-dependent material (readings R20, R21): stretch table
        [4, 6] (warp, weft, shear, area measures x strain segments) in N/m and bend table
        [3, 5] (0, 45, 90 degree directions x angle segments) in N m. None: the
        isotropic model (k_s, k_b of set_params). Density stays that of set_params."""
        lib = _load()
        if stretch is None:
            st = lib.orc_set_material(self._h, 0, None, None)
            self.wang = None
        else:
            S = _f64(stretch, (4, 6)).ravel()
            B = _f64(bend, (3, 5)).ravel()
            st = lib.orc_set_material(self._h, 1, _d(S), _d(B))
            self.wang = (S.reshape(4, 6).copy(), B.reshape(3, 5).copy())
        if st != ORC_OK:
            raise OracleError(st, "set_material")

    @property
    def nmat(self):
        """Entries of the material gradient: 3 (k_s, k_b, d) or 40 (S, B, d)."""
        return _load().orc_num_material(self._h)

    def material_frames(self):
        """Measure tensors N_1..N_4 of every triangle (local frame; N_00, N_01, N_11)
        [nt, 4, 3] and every hinge's direction weights [nh, 3] (readings R20, R21)."""
        N = np.zeros((self.nt, 4, 3))
        w = np.zeros((self.nh, 3))
        _load().orc_get_material_frames(self._h, _d(N), _d(w))
        return N, w

    def wind_force(self, x, v):
        """The aerodynamic force alone at (x, v) [V, 3] (reading R19)."""
        x = _f64(x, (self.nv, 3))
        v = _f64(v, (self.nv, 3))
        f = np.zeros((self.nv, 3))
        _load().orc_wind_force(self._h, _d(x), _d(v), _d(f))
        return f

    def set_membrane_system(self, mode: int):
        """Stress term of the system matrix's membrane block (reading R9):
        MEMBRANE_EXACT (default; true Hessian, can be indefinite under
        compression), MEMBRANE_TENSION (tension part of the strain only) or
        MEMBRANE_GAUSS_NEWTON."""
        st = _load().orc_set_membrane_system(self._h, int(mode))
        if st != ORC_OK:
            raise OracleError(st, "set_membrane_system")

    # ---------------------------------------------------------------- geometry
    def geometry(self):
        """Rest precompute: B = D_m^-1 [T,2,2], triangle areas, lumped vertex areas
        (reading R6), hinges [H,4], c_e and rest angles (reading R8)."""
        B = np.zeros((self.nt, 4))
        at = np.zeros(self.nt)
        av = np.zeros(self.nv)
        hv = np.zeros((self.nh, 4), dtype=np.int32)
        ce = np.zeros(self.nh)
        th0 = np.zeros(self.nh)
        _load().orc_get_geometry(self._h, _d(B), _d(at), _d(av), _i(hv), _d(ce), _d(th0))
        return dict(B=B.reshape(-1, 2, 2), tri_area=at, vert_area=av, hinges=hv, c_e=ce,
                    theta_rest=th0)

    # ----------------------------------------------------- element-level probes
    def energy(self, x):
        """Internal energy E_m + E_b at positions x (Sec. 3.1, readings R7, R8)."""
        x = _f64(x, (self.nv, 3))
        em = ctypes.c_double(0)
        eb = ctypes.c_double(0)
        e = _load().orc_energy(self._h, _d(x), ctypes.byref(em), ctypes.byref(eb))
        return e, em.value, eb.value

    def internal_force(self, x):
        """f = -dE/dx (Sec. 3.1, Eq. 3 right-hand side, internal part)."""
        x = _f64(x, (self.nv, 3))
        f = np.zeros((self.nv, 3))
        _load().orc_internal_force(self._h, _d(x), _d(f))
        return f

    def _apply(self, fn, x, u):
        x = _f64(x, (self.nv, 3))
        u = _f64(u, (self.nv, 3))
        o = np.zeros((self.nv, 3))
        fn(self._h, _d(x), _d(u), _d(o))
        return o

    def ksys_apply(self, x, u):
        """K_sys u: configured membrane block + Gauss-Newton bending (reading R9)."""
        return self._apply(_load().orc_ksys_apply, x, u)

    def kexact_apply(self, x, u):
        """K_exact u: the true Hessian of E (= -df/dx) along u."""
        return self._apply(_load().orc_kexact_apply, x, u)

    def ksys_assembled_apply(self, x, u):
        """K_sys u through the assembled block matrix the solver uses."""
        return self._apply(_load().orc_ksys_assembled_apply, x, u)

    def third(self, x, mu, w):
        """grad_x [mu^T K_sys(x) w] (the state derivative of the system matrix)."""
        x = _f64(x, (self.nv, 3))
        mu = _f64(mu, (self.nv, 3))
        w = _f64(w, (self.nv, 3))
        o = np.zeros((self.nv, 3))
        _load().orc_third(self._h, _d(x), _d(mu), _d(w), _d(o))
        return o

    # --------------------------------------------------------------- the step
    def system(self, x, v, F=None):
        """Dense A = M + h^2 K_sys (pins eliminated) and b of one step (Eq. 4-5)."""
        n = 3 * self.nv
        x = _f64(x, (self.nv, 3))
        v = _f64(v, (self.nv, 3))
        F = _f64(F, (self.nv, 3)) if F is not None else None
        A = np.zeros((n, n))
        b = np.zeros(n)
        _load().orc_system(self._h, _d(x), _d(v), _d(F), _d(A), _d(b))
        return A, b

    def solve_step(self, x, v, F=None):
        """Delta v of one step from the oracle's block-Jacobi PCG."""
        x = _f64(x, (self.nv, 3))
        v = _f64(v, (self.nv, 3))
        F = _f64(F, (self.nv, 3)) if F is not None else None
        dv = np.zeros((self.nv, 3))
        it = ctypes.c_int(0)
        st = _load().orc_solve_step(self._h, _d(x), _d(v), _d(F), _d(dv), ctypes.byref(it))
        return dv, it.value, st

    def step_residual(self, x, v, F, dv):
        """r = b - A dv of the step from (x, v) (Eq. 4-5), and ||b||. Returns (r, ||b||, status)."""
        x = _f64(x, (self.nv, 3))
        v = _f64(v, (self.nv, 3))
        F = _f64(F, (self.nv, 3)) if F is not None else None
        dv = _f64(dv, (self.nv, 3))
        r = np.zeros((self.nv, 3))
        bn = ctypes.c_double(0.0)
        st = _load().orc_step_residual(self._h, _d(x), _d(v), _d(F), _d(dv), _d(r),
                                       ctypes.byref(bn))
        return r, bn.value, st

    def step(self, x, v, F=None):
        """One step S_t = PS(S_{t-1}; phi_{t-1}) (Eq. 1, 4, 5). Returns (x, v, dv, iters, status)."""
        x = _f64(x, (self.nv, 3))
        v = _f64(v, (self.nv, 3))
        F = _f64(F, (self.nv, 3)) if F is not None else None
        xo = np.zeros((self.nv, 3))
        vo = np.zeros((self.nv, 3))
        dvo = np.zeros((self.nv, 3))
        it = ctypes.c_int(0)
        st = _load().orc_step(self._h, _d(x), _d(v), _d(F), _d(xo), _d(vo), _d(dvo),
                              ctypes.byref(it))
        return xo, vo, dvo, it.value, st

    def rollout(self, n_steps, x0, v0=None, forces=None, loss_frames=None, check=True):
        """Positions at the loss frames [n_loss, V, 3], final velocity, CG iterations."""
        x0 = _f64(x0, (self.nv, 3))
        v0 = np.zeros((self.nv, 3)) if v0 is None else _f64(v0, (self.nv, 3))
        forces = _f64(forces, (n_steps, self.nv, 3)) if forces is not None else None
        frames = np.arange(1, n_steps + 1, dtype=np.int32) if loss_frames is None else \
            np.ascontiguousarray(loss_frames, dtype=np.int32)
        xo = np.zeros((frames.size, self.nv, 3))
        vf = np.zeros((self.nv, 3))
        iters = np.zeros(n_steps, dtype=np.int32)
        st = _load().orc_rollout(self._h, int(n_steps), _d(x0), _d(v0), _d(forces), _i(frames),
                                 int(frames.size), _d(xo), _d(vf), _i(iters))
        if check and st not in (ORC_OK,):
            raise OracleError(st, "rollout")
        return xo, vf, iters, st

    def gradient(self, n_steps, x0, v0, forces, loss_frames, dl_dx, check=True):
        """Rollout + adjoint: the material gradient (dL/d(k_s, k_b, d), or dL/d(S, B, d)
        [40] with the anisotropic model), dL/dF [n_steps, V, 3], dL/dx0, dL/dv0."""
        x0 = _f64(x0, (self.nv, 3))
        v0 = np.zeros((self.nv, 3)) if v0 is None else _f64(v0, (self.nv, 3))
        forces = _f64(forces, (n_steps, self.nv, 3)) if forces is not None else None
        frames = np.ascontiguousarray(loss_frames, dtype=np.int32)
        dl_dx = _f64(dl_dx, (frames.size, self.nv, 3))
        gm = np.zeros(self.nmat)
        gw = np.zeros(3)
        gF = np.zeros((n_steps, self.nv, 3))
        gx0 = np.zeros((self.nv, 3))
        gv0 = np.zeros((self.nv, 3))
        itf = np.zeros(n_steps, dtype=np.int32)
        ita = np.zeros(n_steps, dtype=np.int32)
        st = _load().orc_gradient(self._h, int(n_steps), _d(x0), _d(v0), _d(forces), _i(frames),
                                  int(frames.size), _d(dl_dx), _d(gm), _d(gw), _d(gF), _d(gx0),
                                  _d(gv0), _i(itf), _i(ita))
        if check and st != ORC_OK:
            raise OracleError(st, "gradient")
        return dict(material=gm, wind=gw, forces=gF, x0=gx0, v0=gv0, iters_fwd=itf,
                    iters_adj=ita, status=st)

    # ------------------------------------------- exact-solve driver (golden files)
    def pattern(self):
        """CSR block pattern of the step matrix: (rowptr [V+1], col [nnzb])."""
        rp = np.zeros(self.nv + 1, dtype=np.int32)
        col = np.zeros(self.nnzb, dtype=np.int32)
        _load().orc_pattern(self._h, _i(rp), _i(col))
        return rp, col

    def system_sparse(self, x, v, F=None):
        """The step's system (Eq. 4-5, pins eliminated) as a scipy CSR matrix A
        [3V, 3V] and b [3V] (vertex-major unknowns)."""
        import scipy.sparse as sp
        if not hasattr(self, "_csr"):
            rp, col = self.pattern()
            # block (i, j) at slot s expands to rows 3i+k, columns 3j+m
            rows = np.repeat(np.arange(self.nv), np.diff(rp))
            r = (3 * rows[:, None, None] + np.arange(3)[None, :, None]).repeat(3, axis=2)
            c = (3 * col[:, None, None] + np.arange(3)[None, None, :]).repeat(3, axis=1)
            self._csr = (r.ravel(), c.ravel())
        x = _f64(x, (self.nv, 3))
        v = _f64(v, (self.nv, 3))
        F = _f64(F, (self.nv, 3)) if F is not None else None
        blocks = np.zeros((self.nnzb, 3, 3))
        b = np.zeros(3 * self.nv)
        st = _load().orc_system_blocks(self._h, _d(x), _d(v), _d(F), _d(blocks), _d(b))
        if st != ORC_OK:
            raise OracleError(st, "system_blocks")
        n = 3 * self.nv
        A = sp.csr_matrix((blocks.ravel(), self._csr), shape=(n, n))
        return A, b

    def _exact_solver(self, x, v, F):
        """Exact solver of the step matrix A(x) (scipy's sparse LU, a library routine
        standing for 'solve A dv = b' of Eq. 4) and the step's b."""
        A, b = self.system_sparse(x, v, F)
        return ExactSolve(A), b

    def rollout_exact(self, n_steps, x0, v0=None, forces=None):
        """Every state of a rollout whose steps are solved exactly (sparse LU instead of
        CG): returns X, V, DV [n_steps + 1, V, 3]."""
        x0 = _f64(x0, (self.nv, 3))
        v0 = np.zeros((self.nv, 3)) if v0 is None else _f64(v0, (self.nv, 3))
        X = np.zeros((n_steps + 1, self.nv, 3))
        Vv = np.zeros_like(X)
        DV = np.zeros_like(X)
        X[0] = x0
        Vv[0] = v0
        Vv[0][self.pins] = 0.0
        pinned = np.zeros(self.nv, dtype=bool)
        pinned[self.pins] = True
        for s in range(1, n_steps + 1):
            F = None if forces is None else forces[s - 1]
            lu, b = self._exact_solver(X[s - 1], Vv[s - 1], F)
            dv = lu.solve(b).reshape(self.nv, 3)
            dv[pinned] = 0.0
            DV[s] = dv
            Vv[s] = Vv[s - 1] + dv
            Vv[s][pinned] = 0.0
            X[s] = X[s - 1] + self.dt * Vv[s]
        return X, Vv, DV

    def gradient_exact(self, n_steps, x0, v0, forces, loss_frames, targets, states=None):
        """Rollout + adjoint with exact step solves, for the loss
        L = sum over the loss frames of |x_s - target_s|^2 (dL/dx_s = 2 (x_s - target_s)).
        The backward sweep is the oracle's own (orc_adjoint_rhs, orc_adjoint_update)
        around an exact solve of A(x_{s-1}) mu = u. Returns the positions at the loss
        frames, the loss and the material gradient (3 or 40 entries), dL/dF, dL/dx0,
        dL/dv0."""
        frames = [int(f) for f in loss_frames]
        X, Vv, DV = states if states is not None else self.rollout_exact(n_steps, x0, v0, forces)
        targets = np.asarray(targets, dtype=np.float64)
        xo = X[frames]
        dl = 2.0 * (xo - targets)
        gx = np.zeros((self.nv, 3))
        gv = np.zeros((self.nv, 3))
        u = np.zeros((self.nv, 3))
        gm = np.zeros(self.nmat)
        gw = np.zeros(3)
        gF = np.zeros((n_steps, self.nv, 3))
        lib = _load()
        fi = len(frames) - 1
        for s in range(n_steps, 0, -1):
            if fi >= 0 and frames[fi] == s:
                gx += dl[fi]
                fi -= 1
            lib.orc_adjoint_rhs(self._h, _d(gx), _d(gv), _d(u))
            F = None if forces is None else forces[s - 1]
            lu, _ = self._exact_solver(X[s - 1], Vv[s - 1], F)
            mu = np.ascontiguousarray(lu.solve(u.ravel()).reshape(self.nv, 3))
            gF[s - 1] = self.dt * mu
            xp = np.ascontiguousarray(X[s - 1])
            vp = np.ascontiguousarray(Vv[s - 1])
            vs = np.ascontiguousarray(Vv[s])
            dvs = np.ascontiguousarray(DV[s])
            lib.orc_adjoint_update(self._h, _d(xp), _d(vp), _d(vs), _d(dvs), _d(mu), _d(u),
                                   _d(gx), _d(gv), _d(gm), _d(gw))
        return dict(x=xo, loss=float(np.sum((xo - targets) ** 2)), material=gm, wind=gw,
                    forces=gF, x0=gx, v0=gv)
