"""Pins of the oracle's element physics (Sec. 3.1 force model, readings R6-R9).

Each test checks the oracle against something other than itself: closed forms,
invariants of any internal force, and central finite differences.
"""

import numpy as np
import pytest

from paper_2203_11938_amd import workloads as W

L = W.SHEET_SIDE


def sheet(oracle_mod, n=6, pins=(), ks=1e3, kb=1e-4, d=0.1, dt=0.01):
    rest, tris = W.grid_sheet(n)
    return oracle_mod.Oracle(tris, rest, pins, ks, kb, d, dt=dt), rest


def random_state(rest, amp, seed):
    g = np.random.default_rng(seed)
    return rest + amp * g.normal(size=rest.shape)


def rotation(seed):
    g = np.random.default_rng(seed)
    q, _ = np.linalg.qr(g.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


# ------------------------------------------------------------------ geometry
@pytest.mark.parametrize("n", [3, 10, 32])
def test_areas_sum_to_sheet_area(oracle_mod, n):
    o, _ = sheet(oracle_mod, n)
    geo = o.geometry()
    assert np.isclose(geo["tri_area"].sum(), L * L, rtol=1e-13)
    assert np.isclose(geo["vert_area"].sum(), L * L, rtol=1e-13)
    # lumped mass (R6): sum m_i = d L^2
    assert np.isclose(0.1 * geo["vert_area"].sum(), 0.1 * L * L, rtol=1e-13)
    # regular grid: every triangle has area a^2 / 2
    a = L / (n - 1)
    assert np.allclose(geo["tri_area"], a * a / 2, rtol=1e-12)


@pytest.mark.parametrize("n", [3, 10, 64])
def test_hinge_and_block_counts(oracle_mod, n):
    o, _ = sheet(oracle_mod, n)
    # interior edges of the split grid: 3(n-1)^2 + 2(n-1) edges minus 4(n-1) boundary ones
    assert o.nh == 3 * (n - 1) ** 2 - 2 * (n - 1)
    geo = o.geometry()
    assert np.allclose(geo["theta_rest"], 0.0, atol=1e-12)   # flat sheet
    # c_e = 3 |e|^2 / (A1 + A2): axis edges a^2, diagonals 2 a^2; A1 + A2 = a^2
    e2 = np.array([np.sum((o.rest[h[1]] - o.rest[h[0]]) ** 2) for h in geo["hinges"]])
    a = L / (n - 1)
    assert np.allclose(geo["c_e"], 3 * e2 / (a * a), rtol=1e-12)
    assert set(np.round(e2 / (a * a), 9)) <= {1.0, 2.0}


# ---------------------------------------------------------------- invariants
def test_rest_state_is_force_free(oracle_mod):
    o, rest = sheet(oracle_mod, 8)
    f = o.internal_force(rest)
    assert np.abs(f).max() < 1e-12
    e, em, eb = o.energy(rest)
    assert abs(e) < 1e-20


def test_rigid_motion_is_force_free(oracle_mod):
    o, rest = sheet(oracle_mod, 8)
    x = rest @ rotation(1).T + np.array([0.3, -1.2, 2.0])
    f = o.internal_force(x)
    assert np.abs(f).max() < 1e-10
    assert abs(o.energy(x)[0]) < 1e-18


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_net_force_and_torque_vanish(oracle_mod, seed):
    o, rest = sheet(oracle_mod, 7, kb=3e-3)
    x = random_state(rest, 0.01, seed)
    f = o.internal_force(x)
    scale = np.abs(f).max()
    assert scale > 1e-3
    assert np.abs(f.sum(axis=0)).max() < 1e-11 * scale * len(x)
    torque = np.cross(x, f).sum(axis=0)
    assert np.abs(torque).max() < 1e-11 * scale * len(x)


# ------------------------------------------------------------- closed forms
@pytest.mark.parametrize("s", [0.97, 1.0, 1.05, 1.3])
def test_uniform_stretch_energy(oracle_mod, s):
    # x = diag(s, 1, 1) X: G = diag((s^2 - 1)/2, 0) -> E_m = L^2 k_s (s^2 - 1)^2 / 8
    ks = 850.0
    o, rest = sheet(oracle_mod, 9, ks=ks)
    x = rest * np.array([s, 1.0, 1.0])
    e, em, eb = o.energy(x)
    assert np.isclose(em, L * L * ks * (s * s - 1) ** 2 / 8, rtol=1e-12, atol=1e-18)
    assert abs(eb) < 1e-20


@pytest.mark.parametrize("alpha", [0.1, 0.7, 2.0, -1.1])
def test_dihedral_fold(oracle_mod, alpha):
    # two triangles (0,1,2) and (1,0,3) sharing edge 0->1 along x; wing 3 rotated
    # about the edge by alpha: theta = -alpha, E_b = k_b * 3|e|^2/(A1+A2) * alpha^2
    x = np.array([[0, 0, 0], [1, 0, 0], [0.5, 1, 0], [0.5, -np.cos(alpha), np.sin(alpha)]],
                 dtype=float)
    assert np.isclose(oracle_mod.hinge_theta(x), -alpha, atol=1e-14)
    rest = x.copy()
    rest[3] = [0.5, -1.0, 0.0]
    kb = 2e-3
    o = oracle_mod.Oracle(np.array([[0, 1, 2], [1, 0, 3]]), rest, (), 0.0, kb, 0.1)
    assert o.nh == 1
    e, em, eb = o.energy(x)
    assert np.isclose(eb, kb * 3.0 * alpha * alpha, rtol=1e-12)
    assert abs(em) < 1e-20  # rotation about the shared edge is an isometry of each triangle


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_theta_gradient_matches_fd(oracle_mod, seed):
    g = np.random.default_rng(seed)
    x = np.array([[0, 0, 0], [1, 0, 0], [0.4, 0.9, 0.1], [0.6, -0.8, 0.3]]) + 0.05 * g.normal(size=(4, 3))
    grad = oracle_mod.hinge_theta_grad(x)
    eps = 1e-6
    fd = np.zeros((4, 3))
    for a in range(4):
        for k in range(3):
            xp = x.copy(); xp[a, k] += eps
            xm = x.copy(); xm[a, k] -= eps
            fd[a, k] = (oracle_mod.hinge_theta(xp) - oracle_mod.hinge_theta(xm)) / (2 * eps)
    assert np.allclose(grad, fd, rtol=1e-7, atol=1e-8)
    # the closed form is translation- and rotation-free
    assert np.abs(grad.sum(axis=0)).max() < 1e-12
    assert np.abs(np.cross(x, grad).sum(axis=0)).max() < 1e-12


@pytest.mark.parametrize("seed", [6, 7])
def test_force_is_negative_energy_gradient(oracle_mod, seed):
    o, rest = sheet(oracle_mod, 6, kb=5e-3)
    x = random_state(rest, 0.01, seed)
    f = o.internal_force(x)
    g = np.random.default_rng(seed + 100)
    for _ in range(4):
        d = g.normal(size=x.shape)
        eps = 1e-6
        de = (o.energy(x + eps * d)[0] - o.energy(x - eps * d)[0]) / (2 * eps)
        assert np.isclose(-np.sum(f * d), de, rtol=1e-7)


# ------------------------------------------------------------------ Hessians
@pytest.mark.parametrize("seed", [8, 9])
def test_kexact_is_force_jacobian(oracle_mod, seed):
    o, rest = sheet(oracle_mod, 6, kb=5e-3)
    x = random_state(rest, 0.01, seed)
    g = np.random.default_rng(seed)
    for _ in range(3):
        u = g.normal(size=x.shape)
        eps = 1e-6
        fd = -(o.internal_force(x + eps * u) - o.internal_force(x - eps * u)) / (2 * eps)
        k = o.kexact_apply(x, u)
        assert np.linalg.norm(k - fd) <= 1e-6 * np.linalg.norm(k)


@pytest.mark.parametrize("which", ["kexact_apply", "ksys_apply", "ksys_assembled_apply"])
def test_stiffness_symmetric(oracle_mod, which):
    o, rest = sheet(oracle_mod, 6, kb=5e-3)
    x = random_state(rest, 0.01, 11)
    g = np.random.default_rng(12)
    u, w = g.normal(size=x.shape), g.normal(size=x.shape)
    ap = getattr(o, which)
    a, b = np.sum(u * ap(x, w)), np.sum(w * ap(x, u))
    assert np.isclose(a, b, rtol=1e-11)


def test_ksys_assembled_equals_element_route(oracle_mod):
    o, rest = sheet(oracle_mod, 7, kb=5e-3)
    x = random_state(rest, 0.01, 13)
    u = np.random.default_rng(14).normal(size=x.shape)
    a = o.ksys_apply(x, u)
    b = o.ksys_assembled_apply(x, u)
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a)


@pytest.mark.parametrize("seed", [15, 16, 17])
def test_tension_ksys_positive_semidefinite(oracle_mod, seed):
    # compressed, crumpled states (the exact Hessian's indefiniteness under compression is
    # pinned in closed form by test_tension_clamp_closed_form)
    o, rest = sheet(oracle_mod, 6, kb=1e-4)
    o.set_membrane_system(o.MEMBRANE_TENSION)
    x = 0.97 * random_state(rest, 0.01, seed)
    g = np.random.default_rng(seed)
    for _ in range(20):
        u = g.normal(size=x.shape)
        assert np.sum(u * o.ksys_apply(x, u)) >= -1e-12 * np.sum(u * u)


@pytest.mark.parametrize("s", [0.99, 1.02])
def test_tension_clamp_closed_form(oracle_mod, s):
    # x = s X: G = (s^2-1)/2 I. For u = (0, 0, X_x): u^T K_exact u = k_s L^2 (s^2-1)/2, and
    # K_sys keeps it only in tension (s > 1); in compression its membrane block gives 0.
    ks, kb = 700.0, 1e-3
    o, rest = sheet(oracle_mod, 9, ks=ks, kb=kb)
    x = s * rest
    u = np.zeros_like(rest); u[:, 2] = rest[:, 0]
    ue = np.sum(u * o.kexact_apply(x, u))
    assert np.isclose(np.sum(u * o.ksys_apply(x, u)), ue, rtol=1e-12)  # default: exact block
    o.set_membrane_system(o.MEMBRANE_TENSION)
    us = np.sum(u * o.ksys_apply(x, u))
    assert np.isclose(ue, ks * L * L * (s * s - 1) / 2, rtol=1e-10)
    if s > 1:
        assert np.isclose(us, ue, rtol=1e-10)
    else:
        assert abs(us) < 1e-10 * abs(ue)


def test_tension_ksys_is_exact_hessian_in_pure_tension(oracle_mod):
    o, rest = sheet(oracle_mod, 6, ks=1e3, kb=0.0)
    o.set_membrane_system(o.MEMBRANE_TENSION)
    x = 1.03 * rest + 1e-4 * np.random.default_rng(18).normal(size=rest.shape)
    u = np.random.default_rng(19).normal(size=rest.shape)
    a, b = o.ksys_apply(x, u), o.kexact_apply(x, u)
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("seed,scale", [(20, 1.0), (21, 0.985), (22, 1.02)])
def test_third_contraction_matches_fd(oracle_mod, seed, scale, mode):
    # grad_x [mu^T K_sys(x) w] against central differences of the element route
    o, rest = sheet(oracle_mod, 5, kb=5e-3)
    o.set_membrane_system(mode)
    x = scale * random_state(rest, 0.01, seed)
    g = np.random.default_rng(seed + 7)
    mu, w = g.normal(size=x.shape), g.normal(size=x.shape)
    t = o.third(x, mu, w)
    for _ in range(3):
        d = g.normal(size=x.shape)
        eps = 1e-7
        fd = (np.sum(mu * o.ksys_apply(x + eps * d, w)) - np.sum(mu * o.ksys_apply(x - eps * d, w))) / (2 * eps)
        assert np.isclose(np.sum(t * d), fd, rtol=1e-6)
