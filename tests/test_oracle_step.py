"""Pins of the oracle's time step and rollout (Sec. 3.1, Eq. 1, 4, 5; readings R1-R4, R9, R11).

Closed forms (free fall, the 'only F' model of the paper's ablation with no
material forces), a conservation law, and a library linear solve.
"""

import numpy as np
import pytest

from paper_2203_11938_amd import workloads as W

G = np.array(W.GRAVITY)


def test_pcg_matches_library_solve(oracle_mod):
    # the step's system at a deformed, moving state of the 10x10 workload
    w = W.workload("C1")
    inst = W.make_instances(w)[0]
    o = oracle_mod.Oracle(inst.tris, inst.rest, inst.pins, *inst.material.as_tuple(), dt=w.dt,
                          cg_tol=1e-13)
    xo, vf, _, _ = o.rollout(12, inst.x0)
    x = xo[-1]
    F = np.random.default_rng(1).normal(0.0, 1e-3, size=x.shape)
    A, b = o.system(x, vf, F)
    assert np.allclose(A, A.T, rtol=0, atol=1e-14 * np.abs(A).max())
    assert np.linalg.eigvalsh(A).min() > 0  # SPD (R9)
    ref = np.linalg.solve(A, b)
    dv, iters, st = o.solve_step(x, vf, F)
    assert st == 0 and iters > 10
    assert np.linalg.norm(dv.ravel() - ref) <= 1e-10 * np.linalg.norm(ref)
    # pinned rows are Dirichlet: zero increment
    assert np.abs(dv[inst.pins]).max() == 0.0
    # the sparse step residual: b - A dv for the library's solution is at rounding
    # level, for zero it is b, and it is affine in dv with slope -A
    r, bn, st = o.step_residual(x, vf, F, ref.reshape(-1, 3))
    assert st == 0 and abs(bn - np.linalg.norm(b)) <= 1e-14 * bn
    assert np.linalg.norm(r) <= 1e-12 * bn
    r0, _, _ = o.step_residual(x, vf, F, np.zeros_like(x))
    assert np.array_equal(r0.ravel(), b)
    d = np.random.default_rng(2).normal(size=x.shape)
    r1, _, _ = o.step_residual(x, vf, F, d)
    assert np.allclose(r1.ravel(), b - A @ d.ravel(), rtol=0, atol=1e-12 * np.abs(A @ d.ravel()).max())


@pytest.mark.parametrize("n,steps", [(3, 30), (9, 20)])
def test_free_fall_closed_form(oracle_mod, n, steps):
    # no pins, no forces, start at rest shape: x_s = X + g h^2 s(s+1)/2, v_s = s h g
    rest, tris = W.grid_sheet(n)
    h = 0.01
    o = oracle_mod.Oracle(tris, rest, (), 1e3, 1e-4, 0.1, dt=h, cg_tol=1e-13)
    xo, vf, iters, st = o.rollout(steps, rest)
    for k, s in enumerate(range(1, steps + 1)):
        ref = rest + G * h * h * s * (s + 1) / 2
        assert np.abs(xo[k] - ref).max() <= 1e-12
    assert np.abs(vf - steps * h * G).max() <= 1e-11


def test_only_forces_closed_form(oracle_mod):
    # k_s = k_b = 0, g = 0 (the paper's 'only F' model): v_s = v_0 + h sum_{r<s} F_r / m,
    # x_s = x_0 + h sum_{q<=s} v_q; pinned vertices stay put
    n, steps, h, d = 5, 12, 0.02, 0.3
    rest, tris = W.grid_sheet(n)
    pins = W.pin_set(n, "top2")
    o = oracle_mod.Oracle(tris, rest, pins, 0.0, 0.0, d, dt=h, gravity=(0, 0, 0), cg_tol=1e-14)
    m = d * o.geometry()["vert_area"][:, None]
    g = np.random.default_rng(2)
    F = g.normal(size=(steps, n * n, 3))
    x0 = rest + 0.01 * g.normal(size=rest.shape)
    v0 = g.normal(size=rest.shape)
    xo, vf, _, _ = o.rollout(steps, x0, v0, F)
    free = np.ones(n * n, bool); free[pins] = False
    v = v0.copy(); v[~free] = 0
    x = x0.copy()
    for s in range(steps):
        v = v + h * F[s] / m
        v[~free] = 0
        x = x + h * v
        assert np.allclose(xo[s], x, rtol=0, atol=1e-12)
    assert np.allclose(vf, v, rtol=0, atol=1e-11)


def test_momentum_conserved_without_pins_and_gravity(oracle_mod):
    n, steps = 7, 15
    rest, tris = W.grid_sheet(n)
    o = oracle_mod.Oracle(tris, rest, (), 500.0, 1e-3, 0.1, dt=0.01, gravity=(0, 0, 0),
                          cg_tol=1e-14)
    o.set_membrane_system(o.MEMBRANE_TENSION)  # crumpled start: keep the system SPD
    m = 0.1 * o.geometry()["vert_area"][:, None]
    g = np.random.default_rng(3)
    x0 = rest + 0.005 * g.normal(size=rest.shape)
    v0 = 0.3 * g.normal(size=rest.shape)
    x, v = x0, v0
    p0 = (m * v0).sum(axis=0)
    for _ in range(steps):
        x, v, dv, it, st = o.step(x, v)
        assert st == 0
        assert np.abs((m * v).sum(axis=0) - p0).max() <= 1e-11 * np.abs(m * v0).sum()


def test_exact_membrane_system_breaks_down_on_stiff_light_sheet(oracle_mod):
    # Reading R9: a 40x40 sheet of the batched workload (k_s ~ 8.8e3 N/m, d ~ 0.089 kg/m^2)
    # makes M + h^2 K indefinite with the exact membrane Hessian within ten steps; the
    # tension-clamped system matrix runs the same steps.
    w = W.workload("C4")
    inst = W.make_instances(w)[8]
    assert int(np.sqrt(inst.n_verts)) == 40 and inst.material.stretch > 8e3
    o = oracle_mod.Oracle(inst.tris, inst.rest, inst.pins, *inst.material.as_tuple(), dt=w.dt,
                          cg_tol=1e-7)
    o.set_membrane_system(o.MEMBRANE_EXACT)
    _, _, _, st = o.rollout(12, inst.x0, None, inst.forces[:12], check=False)
    assert st == oracle_mod.ORC_E_INDEFINITE
    o.set_membrane_system(o.MEMBRANE_TENSION)
    _, _, _, st = o.rollout(12, inst.x0, None, inst.forces[:12], check=False)
    assert st == oracle_mod.ORC_OK


def test_mesh_errors(oracle_mod):
    rest, tris = W.grid_sheet(4)
    bad = rest.copy()
    bad[1] = bad[0]  # collapses triangles touching vertices 0 and 1
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.Oracle(tris, bad, ())
    assert e.value.code == oracle_mod.ORC_E_MESH
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.Oracle(tris, rest, (99,))
    assert e.value.code == oracle_mod.ORC_E_INVALID
    flipped = tris.copy()
    flipped[0] = flipped[0][::-1]  # same directed edge used twice
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.Oracle(flipped, rest, ())
    assert e.value.code == oracle_mod.ORC_E_MESH


def test_not_converged_is_reported(oracle_mod):
    w = W.workload("C1")
    inst = W.make_instances(w)[0]
    o = oracle_mod.Oracle(inst.tris, inst.rest, inst.pins, *inst.material.as_tuple(), dt=w.dt,
                          cg_tol=1e-10, cg_max_iter=3)
    _, _, iters, st = o.rollout(3, inst.x0, check=False)
    assert st == oracle_mod.ORC_E_NOT_CONVERGED
    assert (iters == 3).all()
