"""Pins of the oracle's adjoint (the paper's backward pass: implicit differentiation of Eq. 4).

Brute-force central differences of every input entry on a 3x3 sheet, random
directions on a larger one, the closed-form gradient of the 'only F' model and
the scale-homogeneity identity of the step.
"""

import numpy as np
import pytest

from paper_2203_11938_amd import workloads as W


def loss_and_grad(o, steps, x0, v0, F, frames, target):
    xo, _, _, _ = o.rollout(steps, x0, v0, F, frames)
    loss = np.sum((xo - target) ** 2)
    g = o.gradient(steps, x0, v0, F, frames, 2.0 * (xo - target))
    return loss, g


def loss_only(o, steps, x0, v0, F, frames, target):
    xo, _, _, _ = o.rollout(steps, x0, v0, F, frames)
    return np.sum((xo - target) ** 2)


def small_problem(oracle_mod, n=3, steps=5, seed=0, pins="top2", amp=0.02, membrane=1):
    rest, tris = W.grid_sheet(n)
    p = W.pin_set(n, pins)
    ks, kb, d = 60.0, 2e-3, 0.2
    o = oracle_mod.Oracle(tris, rest, p, ks, kb, d, dt=0.01, cg_tol=1e-14)
    o.set_membrane_system(membrane)
    g = np.random.default_rng(seed)
    V = n * n
    x0 = rest + amp * g.normal(size=rest.shape)
    v0 = 0.2 * g.normal(size=rest.shape)
    F = 0.02 * g.normal(size=(steps, V, 3))
    frames = np.arange(1, steps + 1, dtype=np.int32)
    target = x0[None] + 0.05 * g.normal(size=(steps, V, 3))
    return o, (ks, kb, d), x0, v0, F, frames, target


@pytest.mark.parametrize("membrane", [1, 2])
def test_adjoint_matches_bruteforce_fd_on_3x3(oracle_mod, membrane):
    # every input entry: 3 material + 27 x0 + 27 v0 + 135 forces, rel <= 1e-6, for the
    # exact (1) and the tension-clamped (2) system membrane block; the crumpled start keeps
    # principal strains away from the clamp's kink
    o, mat, x0, v0, F, frames, target = small_problem(oracle_mod, membrane=membrane)
    steps = F.shape[0]
    _, g = loss_and_grad(o, steps, x0, v0, F, frames, target)

    def L_with(mat_=mat, x0_=x0, v0_=v0, F_=F):
        o.set_params(*mat_)
        return loss_only(o, steps, x0_, v0_, F_, frames, target)

    fd_m = np.zeros(3)
    for k in range(3):
        hstep = 1e-6 * mat[k]
        mp = list(mat); mp[k] += hstep
        mm = list(mat); mm[k] -= hstep
        fd_m[k] = (L_with(mat_=mp) - L_with(mat_=mm)) / (2 * hstep)
    o.set_params(*mat)
    assert np.allclose(g["material"], fd_m, rtol=1e-6, atol=0)

    def fd_array(name, base):
        out = np.zeros_like(base)
        hstep = 1e-7
        for idx in np.ndindex(base.shape):
            p = base.copy(); p[idx] += hstep
            m = base.copy(); m[idx] -= hstep
            kw = {name: p}
            lp = L_with(**kw)
            kw = {name: m}
            lm = L_with(**kw)
            out[idx] = (lp - lm) / (2 * hstep)
        return out

    for name, base, key in [("x0_", x0, "x0"), ("v0_", v0, "v0"), ("F_", F, "forces")]:
        fd = fd_array(name, base)
        an = g[key]
        assert np.linalg.norm(an - fd) <= 1e-6 * np.linalg.norm(fd), key
    # pinned vertices: no velocity gradient, no force gradient
    assert np.abs(g["v0"][o.pins]).max() == 0.0
    assert np.abs(g["forces"][:, o.pins]).max() == 0.0


@pytest.mark.parametrize("seed,membrane,amp", [(1, 1, 0.003), (2, 1, 0.003), (1, 2, 0.02),
                                               (2, 2, 0.02)])
def test_adjoint_random_directions_fd(oracle_mod, seed, membrane, amp):
    # exact block from a mildly perturbed start (a strongly crumpled 7x7 sheet makes the
    # exact system indefinite), tension-clamped block from a crumpled one
    o, mat, x0, v0, F, frames, target = small_problem(oracle_mod, n=7, steps=12, seed=seed,
                                                      amp=amp, membrane=membrane)
    steps = F.shape[0]
    frames = np.array([4, 8, 12], dtype=np.int32)
    target = target[frames - 1]
    _, g = loss_and_grad(o, steps, x0, v0, F, frames, target)
    gen = np.random.default_rng(seed + 10)
    hstep = 1e-7
    for _ in range(3):
        dx, dv, dF = (gen.normal(size=x0.shape), gen.normal(size=v0.shape),
                      gen.normal(size=F.shape))
        dm = gen.normal(size=3) * np.array(mat)
        pred = (np.sum(g["x0"] * dx) + np.sum(g["v0"] * dv) + np.sum(g["forces"] * dF)
                + np.sum(g["material"] * dm))

        def at(t):
            o.set_params(*(np.array(mat) + t * dm))
            return loss_only(o, steps, x0 + t * dx, v0 + t * dv, F + t * dF, frames, target)

        fd = (at(hstep) - at(-hstep)) / (2 * hstep)
        o.set_params(*mat)
        assert np.isclose(pred, fd, rtol=1e-6)


def test_only_forces_gradient_closed_form(oracle_mod):
    # k_s = k_b = 0, g = 0: dx_s / dF_r = (h^2 / m)(s - r) I for r < s (0-based force index)
    n, steps, h, d = 4, 8, 0.01, 0.2
    rest, tris = W.grid_sheet(n)
    pins = W.pin_set(n, "corner")
    o = oracle_mod.Oracle(tris, rest, pins, 0.0, 0.0, d, dt=h, gravity=(0, 0, 0), cg_tol=1e-14)
    m = d * o.geometry()["vert_area"]
    s = 6
    c = np.random.default_rng(4).normal(size=(1, n * n, 3))
    g = o.gradient(steps, rest, None, np.zeros((steps, n * n, 3)), np.array([s], np.int32), c)
    free = np.ones(n * n, bool); free[pins] = False
    for r in range(steps):
        ref = c[0] * (h * h / m[:, None]) * max(s - r, 0)
        ref[~free] = 0.0
        assert np.allclose(g["forces"][r], ref, rtol=1e-12, atol=1e-15)
    assert np.allclose(g["material"][:2], 0.0, atol=1e-15)


def test_only_forces_initial_state_and_density_gradients_closed_form(oracle_mod):
    # k_s = k_b = 0, g = 0, pinned vertices held: x_s = x_0 + s h v_0 + (h^2 / m) sum_{r<s}
    # (s - r) F_r on free vertices, m = d * (incident rest area) / 3, so for
    # L = sum_s <c_s, x_s>: dL/dx_0 = sum_s c_s, dL/dv_0 = sum_s s h c_s (free rows) and
    # dL/dd = -sum_s <c_s, x_s - x_0 - s h v_0> / d (the force term scales with 1 / d)
    n, steps, h, d = 5, 12, 0.02, 0.3
    rest, tris = W.grid_sheet(n)
    pins = W.pin_set(n, "top2")
    V = n * n
    o = oracle_mod.Oracle(tris, rest, pins, 0.0, 0.0, d, dt=h, gravity=(0, 0, 0), cg_tol=1e-14)
    g = np.random.default_rng(12)
    F = g.normal(size=(steps, V, 3))
    x0 = rest + 0.01 * g.normal(size=rest.shape)
    v0 = 0.1 * g.normal(size=rest.shape)
    frames = np.array([3, 7, 12], np.int32)
    c = g.normal(size=(len(frames), V, 3))
    gr = o.gradient(steps, x0, v0, F, frames, c)
    free = np.ones(V, bool)
    free[pins] = False
    e1, e2 = rest[tris[:, 1]] - rest[tris[:, 0]], rest[tris[:, 2]] - rest[tris[:, 0]]
    area = 0.5 * np.linalg.norm(np.cross(e1, e2), axis=1)
    m = np.zeros(V)
    for k in range(3):
        np.add.at(m, tris[:, k], d * area / 3.0)
    # the force part of x_s on free rows: (h^2 / m) sum_{r<s} (s - r) F_r
    disp = [h * h * sum((f - r) * F[r] for r in range(f)) / m[:, None] for f in frames]
    gx0 = c.sum(axis=0)
    gv0 = sum(f * h * c[k] for k, f in enumerate(frames)) * free[:, None]
    gd = -sum(np.sum((c[k] * disp[k])[free]) for k in range(len(frames))) / d
    assert np.allclose(gr["x0"], gx0, rtol=1e-12, atol=1e-14)
    assert np.allclose(gr["v0"], gv0, rtol=1e-12, atol=1e-14)
    assert np.isclose(gr["material"][2], gd, rtol=1e-10)


def test_homogeneity_identity(oracle_mod):
    # (k_s, k_b, d, F) -> c (k_s, k_b, d, F) scales A and b alike, so the trajectory is
    # unchanged: k_s dL/dk_s + k_b dL/dk_b + d dL/dd + <F, dL/dF> = 0
    o, mat, x0, v0, F, frames, target = small_problem(oracle_mod, n=6, steps=10, seed=5,
                                                      amp=0.003)
    _, g = loss_and_grad(o, F.shape[0], x0, v0, F, frames, target)
    terms = np.array([mat[0] * g["material"][0], mat[1] * g["material"][1],
                      mat[2] * g["material"][2], np.sum(F * g["forces"])])
    assert abs(terms.sum()) <= 1e-9 * np.abs(terms).max()
    assert np.abs(terms).max() > 1e-6
