"""Pins of the oracle's aerodynamic force (Eq. 2's wind velocity w, reading R19: per
triangle rho_air * rest area * |s| s n with s = n . (w - mean vertex velocity), a third
to each vertex) and of the step and adjoint with it.

* closed forms on a flat sheet: a uniform normal wind gives a total force
  rho L^2 |w_n| w_n n; a wind in the sheet's plane gives none;
* the step matrix's wind block h D equals -h df/dv by central differences and is
  symmetric positive semi-definite;
* a flat unpinned sheet falling through still air (or through a wind in its plane)
  moves as one body: its vertical velocity follows the scalar recursion
  v <- v + h (rho |s| s + d g) / (d + 2 h rho |s|), s = -v, exactly as the step defines it;
* the adjoint's gradients, the wind gradient dL/dw included, against brute-force
  central differences of every input of a 3x3 sheet.
"""

import numpy as np
import pytest

from paper_2203_11938_amd import workloads as W

RHO = 1.2


def test_uniform_normal_wind_on_flat_sheet(oracle_mod):
    n = 6
    rest, tris = W.grid_sheet(n)
    o = oracle_mod.Oracle(tris, rest, [], 1e3, 1e-4, 0.1)
    L2 = W.SHEET_SIDE ** 2
    for wz in (2.0, -3.0):
        o.set_wind((0.0, 0.0, wz), RHO)
        f = o.wind_force(rest, np.zeros_like(rest))
        assert np.allclose(f.sum(axis=0), [0.0, 0.0, RHO * L2 * abs(wz) * wz], rtol=1e-13, atol=1e-15)
        # a third of each incident triangle's share: proportional to the lumped area
        va = o.geometry()["vert_area"]
        assert np.allclose(f[:, 2], RHO * abs(wz) * wz * va, rtol=1e-13)
    # in the sheet's plane: no normal component, no force
    o.set_wind((1.5, -0.7, 0.0), RHO)
    assert np.abs(o.wind_force(rest, np.zeros_like(rest))).max() == 0.0
    # the sheet's own motion: moving with the wind gives no force
    v = np.tile([0.3, 0.1, -0.4], (rest.shape[0], 1))
    o.set_wind((0.3, 0.1, -0.4), RHO)
    assert np.abs(o.wind_force(rest, v)).max() <= 1e-17


def test_wind_block_of_step_matrix_is_minus_h_dfdv(oracle_mod):
    rest, tris = W.grid_sheet(4)
    pins = W.pin_set(4, "top2")
    o = oracle_mod.Oracle(tris, rest, pins, 300.0, 1e-3, 0.2, dt=0.01)
    g = np.random.default_rng(5)
    x = rest + 0.03 * g.normal(size=rest.shape)
    v = 0.4 * g.normal(size=rest.shape)
    v[pins] = 0.0
    o.set_wind(None)
    A0, _ = o.system(x, v)
    o.set_wind((0.4, -0.2, 1.1), RHO)
    A1, _ = o.system(x, v)
    hD = A1 - A0
    # central differences of the wind force in every velocity coordinate
    n = 3 * rest.shape[0]
    J = np.zeros((n, n))
    eps = 1e-6
    for c in range(n):
        vp, vm = v.copy(), v.copy()
        vp.flat[c] += eps
        vm.flat[c] -= eps
        J[:, c] = (o.wind_force(x, vp) - o.wind_force(x, vm)).ravel() / (2 * eps)
    free = np.repeat(~np.isin(np.arange(rest.shape[0]), pins), 3)
    ref = -0.01 * J[np.ix_(free, free)]
    assert np.linalg.norm(hD[np.ix_(free, free)] - ref) <= 1e-7 * np.linalg.norm(ref)
    # symmetric and positive semi-definite up to the rounding of A1 - A0
    assert np.abs(hD - hD.T).max() <= 1e-12 * np.abs(hD).max()
    assert np.linalg.eigvalsh(0.5 * (hD + hD.T)).min() >= -1e-12 * np.abs(hD).max()
    # pinned rows and columns stay the identity's
    assert np.abs(hD[~free]).max() == 0.0 and np.abs(hD[:, ~free]).max() == 0.0


@pytest.mark.parametrize("wind", [(0.0, 0.0, 0.0), (0.8, -0.5, 0.0)])
def test_flat_sheet_falls_through_air_as_one_body(oracle_mod, wind):
    n, steps, h, d = 8, 25, 0.01, 0.1
    rest, tris = W.grid_sheet(n)
    o = oracle_mod.Oracle(tris, rest, [], 1e3, 1e-4, d, dt=h, cg_tol=1e-14)
    o.set_wind(wind, RHO)
    xo, vf, _, st = o.rollout(steps, rest)
    assert st == oracle_mod.ORC_OK
    vz, z = 0.0, 0.0
    for k in range(steps):
        s = -vz
        vz += h * (RHO * abs(s) * s + d * (-9.81)) / (d + 2.0 * h * RHO * abs(s))
        z += h * vz
        assert np.allclose(xo[k][:, 2], z, rtol=0, atol=1e-13), k
        assert np.allclose(xo[k][:, :2], rest[:, :2], rtol=0, atol=1e-13), k
    assert np.allclose(vf[:, 2], vz, rtol=0, atol=1e-12)
    # air drag slows the fall below the vacuum value
    assert z > -9.81 * h * h * steps * (steps + 1) / 2


def test_adjoint_with_wind_matches_bruteforce_fd_on_3x3(oracle_mod):
    """Every input entry: 3 material + 3 wind + 27 x0 + 27 v0 + 135 forces."""
    rest, tris = W.grid_sheet(3)
    pins = W.pin_set(3, "top2")
    ks, kb, d = 60.0, 2e-3, 0.2
    wind = np.array([0.3, -0.2, 1.0])
    o = oracle_mod.Oracle(tris, rest, pins, ks, kb, d, dt=0.01, cg_tol=1e-14)
    o.set_wind(wind, RHO)
    g = np.random.default_rng(7)
    steps = 5
    x0 = rest + 0.02 * g.normal(size=rest.shape)
    v0 = 0.2 * g.normal(size=rest.shape)
    F = 0.02 * g.normal(size=(steps, 9, 3))
    frames = np.arange(1, steps + 1, dtype=np.int32)
    target = x0[None] + 0.05 * g.normal(size=(steps, 9, 3))

    def L(mat=(ks, kb, d), w=wind, x0_=x0, v0_=v0, F_=F):
        o.set_params(*mat)
        o.set_wind(w, RHO)
        xo, _, _, _ = o.rollout(steps, x0_, v0_, F_, frames)
        return np.sum((xo - target) ** 2)

    xo, _, _, _ = o.rollout(steps, x0, v0, F, frames)
    gr = o.gradient(steps, x0, v0, F, frames, 2.0 * (xo - target))

    fd_m = np.zeros(3)
    for k in range(3):
        hs = 1e-6 * (ks, kb, d)[k]
        mp, mm = [ks, kb, d], [ks, kb, d]
        mp[k] += hs
        mm[k] -= hs
        fd_m[k] = (L(mat=mp) - L(mat=mm)) / (2 * hs)
    fd_w = np.zeros(3)
    for k in range(3):
        wp, wm = wind.copy(), wind.copy()
        wp[k] += 1e-6
        wm[k] -= 1e-6
        fd_w[k] = (L(w=wp) - L(w=wm)) / 2e-6
    o.set_params(ks, kb, d)
    o.set_wind(wind, RHO)
    assert np.allclose(gr["material"], fd_m, rtol=1e-6, atol=0)
    assert np.linalg.norm(gr["wind"] - fd_w) <= 1e-6 * np.linalg.norm(fd_w)
    assert np.abs(gr["wind"]).max() > 0.0

    for name, base, key in [("x0_", x0, "x0"), ("v0_", v0, "v0"), ("F_", F, "forces")]:
        fd = np.zeros_like(base)
        for idx in np.ndindex(base.shape):
            p, m = base.copy(), base.copy()
            p[idx] += 1e-7
            m[idx] -= 1e-7
            fd[idx] = (L(**{name: p}) - L(**{name: m})) / 2e-7
        assert np.linalg.norm(gr[key] - fd) <= 1e-6 * np.linalg.norm(fd), key


def test_exact_driver_matches_cg_oracle_with_wind(oracle_mod):
    w = W.workload("C2", steps=8)
    inst = W.make_instances(w)[0]
    o = oracle_mod.Oracle(inst.tris, inst.rest, inst.pins, *inst.material.as_tuple(), dt=w.dt,
                          cg_tol=1e-13)
    o.set_wind((0.5, 0.2, -1.5), 1.0)
    frames = np.array([4, 8], np.int32)
    target = W.loss_targets(w, inst, frames)
    xo, _, _, _ = o.rollout(w.steps, inst.x0, inst.v0, inst.forces, frames)
    ref = o.gradient(w.steps, inst.x0, inst.v0, inst.forces, frames, 2.0 * (xo - target))
    ex = o.gradient_exact(w.steps, inst.x0, inst.v0, inst.forces, frames, target)
    rel = lambda a, b: np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b)
    assert rel(ex["x"], xo) <= 1e-11
    for k in ("material", "wind", "forces", "x0", "v0"):
        assert rel(ex[k], ref[k]) <= 1e-8, k
