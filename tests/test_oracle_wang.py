"""Pins of the oracle's anisotropic strain-dependent material (readings R20, R21 of the
paper's S in R^24 and B in R^15, taken from Wang et al.; the paper gives no formulas,
so the model itself is parity unpinned against the paper). Checked against what the
readings and the mathematics fix:

* isotropic reduction: stretch tables S[0..2][j] = k_s, S[3][j] = 0 and bend tables
  B[a][j] = k_b give the isotropic R7/R8 model exactly (energy, force, both stiffness
  products, the third-derivative contraction and the whole rollout + adjoint, whose
  parameter sums are dL/dk_s and dL/dk_b);
* constant tables with an area term lambda are St.Venant-Kirchhoff with Lame lambda:
  W = (mu_s / 2) ||G||^2 + (lambda / 2) tr(G)^2;
* the piecewise response: a triangle stretched along the warp axis by Green strain e
  stores area * (psi_warp(|e|) + psi_area(|e|)), psi the double integral of the
  piecewise-constant stiffness, integrated here numerically across the breaks;
* the frames: on a grid sheet the bending-direction weights are (0, 0, 1) for edges
  along x, (1, 0, 0) along y and (0, 1, 0) on the diagonals; a sheet turned by 90
  degrees in its plane with warp and weft tables swapped (and the 0 / 90 degree bend
  tables) stores the same energy in the turned state;
* central differences: force = -dE/dx, K_exact u = directional derivative of -f, the
  third contraction = derivative of mu^T K_sys(x) w, and every one of the 40 material
  gradient entries of an exact-solve rollout's loss.
"""

import numpy as np
import pytest

from paper_2203_11938_amd import workloads as W

STRAIN_BREAKS = [0.0, 0.0025, 0.005, 0.01, 0.02, 0.04]
BEND_BREAKS = [0.0, 0.05, 0.1, 0.2, 0.4]


def tables(seed, ks=1e3, kb=1e-4, lam=0.3):
    g = np.random.default_rng(seed)
    S = np.exp(g.uniform(np.log(0.5), np.log(2.0), size=(4, 6))) * ks
    S[3] *= lam
    B = np.exp(g.uniform(np.log(0.5), np.log(2.0), size=(3, 5))) * kb
    return S, B


def iso_tables(ks, kb, lam=0.0):
    S = np.full((4, 6), ks)
    S[3] = lam
    return S, np.full((3, 5), kb)


def sheet(oracle_mod, n=5, pins=(), ks=1e3, kb=1e-4, d=0.1, dt=0.01, rest=None):
    r, tris = W.grid_sheet(n)
    if rest is not None:
        r = rest
    return oracle_mod.Oracle(tris, r, pins, ks, kb, d, dt=dt), r, tris


def state(rest, amp, seed):
    g = np.random.default_rng(seed)
    return rest + amp * g.normal(size=rest.shape)


def test_isotropic_tables_reduce_to_the_isotropic_model(oracle_mod):
    ks, kb = 700.0, 3e-4
    o, rest, _ = sheet(oracle_mod, 6, ks=ks, kb=kb)
    x = state(rest, 0.02, 1)
    u = np.random.default_rng(2).normal(size=rest.shape)
    w = np.random.default_rng(3).normal(size=rest.shape)
    ref = (o.energy(x), o.internal_force(x), o.ksys_apply(x, u), o.kexact_apply(x, u),
           o.third(x, u, w))
    o.set_material_wang(*iso_tables(ks, kb))
    got = (o.energy(x), o.internal_force(x), o.ksys_apply(x, u), o.kexact_apply(x, u),
           o.third(x, u, w))
    for k, (a, b) in enumerate(zip(ref[1:], got[1:])):
        assert np.abs(a - b).max() <= 1e-11 * np.abs(a).max(), k
    assert np.allclose(ref[0][0], got[0][0], rtol=1e-12, atol=0)


def test_isotropic_tables_reduce_the_gradient(oracle_mod):
    ks, kb, d = 400.0, 2e-4, 0.15
    o, rest, _ = sheet(oracle_mod, 5, pins=W.pin_set(5, "top2"), ks=ks, kb=kb, d=d)
    T = 4
    F = 0.01 * np.random.default_rng(4).normal(size=(T, rest.shape[0], 3))
    target = state(rest, 0.01, 5)
    r0 = o.gradient_exact(T, rest, None, F, [T], target[None])
    o.set_material_wang(*iso_tables(ks, kb))
    assert o.nmat == 40
    r1 = o.gradient_exact(T, rest, None, F, [T], target[None])
    g = r1["material"]
    assert abs(g[:18].sum() - r0["material"][0]) <= 1e-10 * abs(r0["material"][0])
    assert abs(g[24:39].sum() - r0["material"][1]) <= 1e-10 * abs(r0["material"][1])
    assert abs(g[39] - r0["material"][2]) <= 1e-10 * abs(r0["material"][2])
    for k in ("x", "forces", "x0", "v0"):
        assert np.abs(r1[k] - r0[k]).max() <= 1e-10 * np.abs(r0[k]).max(), k


def test_lame_lambda(oracle_mod):
    mu_s, lam = 800.0, 250.0
    o, rest, tris = sheet(oracle_mod, 4)
    o.set_material_wang(*iso_tables(mu_s, 1e-4, lam))
    x = state(rest, 0.03, 6)
    geo = o.geometry()
    # W = (mu_s / 2) ||G||_F^2 + (lambda / 2) tr(G)^2 per unit rest area, summed
    e = 0.0
    for t, (a, b, c) in enumerate(tris):
        B = geo["B"][t]
        F = np.stack([x[b] - x[a], x[c] - x[a]], axis=1) @ B
        G = 0.5 * (F.T @ F - np.eye(2))
        e += geo["tri_area"][t] * (0.5 * mu_s * np.sum(G * G) + 0.5 * lam * np.trace(G) ** 2)
    assert np.isclose(o.energy(x)[1], e, rtol=1e-12)


def psi_numeric(k, breaks, t):
    """Double integral of the piecewise-constant stiffness from 0 to t on a grid with the
    breaks as nodes: the stress by summing stiffness x width, the energy by trapezoids
    (exact for the piecewise-linear stress)."""
    grid = np.unique(np.concatenate([np.linspace(0.0, t, 2001), [b for b in breaks if b < t]]))
    mid = 0.5 * (grid[1:] + grid[:-1])
    stiff = np.asarray(k)[np.searchsorted(breaks, mid, side="right") - 1]
    sigma = np.concatenate([[0.0], np.cumsum(stiff * np.diff(grid))])
    return float(np.sum(0.5 * (sigma[1:] + sigma[:-1]) * np.diff(grid)))


@pytest.mark.parametrize("e", [0.001, 0.004, 0.012, 0.033, 0.07, -0.006])
def test_uniaxial_warp_response(oracle_mod, e):
    # one triangle in the xy plane, rest edges along x and y
    rest = np.array([[0.0, 0.0, 0.0], [0.1, 0.0, 0.0], [0.0, 0.1, 0.0]])
    o = oracle_mod.Oracle(np.array([[0, 1, 2]]), rest, [], 1e3, 1e-4, 0.1)
    S, B = tables(7)
    o.set_material_wang(S, B)
    x = rest.copy()
    x[:, 0] *= np.sqrt(1.0 + 2.0 * e)      # G_uu = e, G_vv = G_uv = 0
    area = 0.005
    want = area * (psi_numeric(S[0], STRAIN_BREAKS, abs(e)) + psi_numeric(S[3], STRAIN_BREAKS, abs(e)))
    assert np.isclose(o.energy(x)[1], want, rtol=2e-7)


def test_grid_bending_directions(oracle_mod):
    o, rest, _ = sheet(oracle_mod, 4)
    _, w = o.material_frames()
    hv = o.geometry()["hinges"]
    e = rest[hv[:, 1]] - rest[hv[:, 0]]
    along_x = np.abs(e[:, 1]) < 1e-12
    along_y = np.abs(e[:, 0]) < 1e-12
    diag = ~(along_x | along_y)
    assert np.allclose(w[along_x], [0, 0, 1], atol=1e-12)
    assert np.allclose(w[along_y], [1, 0, 0], atol=1e-12)
    assert np.allclose(w[diag], [0, 1, 0], atol=1e-12)


def test_turned_sheet_with_swapped_tables(oracle_mod):
    o, rest, tris = sheet(oracle_mod, 5)
    S, B = tables(8)
    o.set_material_wang(S, B)
    x = state(rest, 0.01, 9)
    x[:, 2] += 0.05 * np.sin(6.0 * rest[:, 0])   # folds for the hinges
    R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    o2 = oracle_mod.Oracle(tris, rest @ R.T, [], 1e3, 1e-4, 0.1)
    S2 = S[[1, 0, 2, 3]]
    B2 = B[[2, 1, 0]]
    o2.set_material_wang(S2, B2)
    e1, e2 = o.energy(x), o2.energy(x @ R.T)
    assert np.isclose(e1[1], e2[1], rtol=1e-12) and np.isclose(e1[2], e2[2], rtol=1e-12)
    # with the tables not swapped the turned sheet differs (the model is anisotropic)
    o2.set_material_wang(S, B)
    assert abs(o2.energy(x @ R.T)[1] - e1[1]) > 1e-3 * e1[1]


@pytest.mark.parametrize("seed", [10, 11])
def test_force_and_stiffness_against_differences(oracle_mod, seed):
    o, rest, _ = sheet(oracle_mod, 4)
    S, B = tables(seed)
    o.set_material_wang(S, B)
    x = state(rest, 0.01, seed)
    x[:, 2] += 0.08 * np.cos(5.0 * rest[:, 1])
    f = o.internal_force(x)
    h = 1e-7
    fd = np.zeros_like(x)
    for i in range(x.shape[0]):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, c] += h
            xm[i, c] -= h
            fd[i, c] = -(o.energy(xp)[0] - o.energy(xm)[0]) / (2 * h)
    assert np.abs(f - fd).max() <= 1e-5 * np.abs(f).max()
    u = np.random.default_rng(seed + 1).normal(size=x.shape)
    Ku = o.kexact_apply(x, u)
    fdk = -(o.internal_force(x + h * u) - o.internal_force(x - h * u)) / (2 * h)
    assert np.abs(Ku - fdk).max() <= 1e-5 * np.abs(Ku).max()
    mu = np.random.default_rng(seed + 2).normal(size=x.shape)
    t3 = o.third(x, mu, u)
    fd3 = np.zeros_like(x)
    for i in range(x.shape[0]):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, c] += h
            xm[i, c] -= h
            fd3[i, c] = (np.sum(mu * o.ksys_apply(xp, u)) - np.sum(mu * o.ksys_apply(xm, u))) / (2 * h)
    assert np.abs(t3 - fd3).max() <= 1e-5 * np.abs(t3).max()


def test_material_gradient_against_differences(oracle_mod):
    # a soft sheet so that the strains cross several breaks within a few steps
    o, rest, _ = sheet(oracle_mod, 4, pins=W.pin_set(4, "top2"), ks=20.0, kb=2e-5, d=0.1,
                       dt=0.02)
    S, B = tables(12, ks=20.0, kb=2e-5)
    T = 4
    F = 0.02 * np.random.default_rng(13).normal(size=(T, rest.shape[0], 3))
    target = state(rest, 0.02, 14)

    def loss(S, B):
        o.set_material_wang(S, B)
        X, _, _ = o.rollout_exact(T, rest, None, F)
        return float(np.sum((X[T] - target) ** 2))

    o.set_material_wang(S, B)
    g = o.gradient_exact(T, rest, None, F, [T], target[None])["material"]
    X, _, _ = o.rollout_exact(T, rest, None, F)
    reached = False
    for k in range(4):
        for j in range(6):
            dS = np.zeros_like(S)
            hstep = 1e-6 * S[k, j]
            dS[k, j] = hstep
            fd = (loss(S + dS, B) - loss(S - dS, B)) / (2 * hstep)
            assert abs(g[6 * k + j] - fd) <= 1e-6 * np.abs(g[:24]).max() + 1e-4 * abs(fd), (k, j)
            reached = reached or (j >= 2 and abs(fd) > 0)
    for a in range(3):
        for j in range(5):
            dB = np.zeros_like(B)
            hstep = 1e-6 * B[a, j]
            dB[a, j] = hstep
            fd = (loss(S, B + dB) - loss(S, B - dB)) / (2 * hstep)
            assert abs(g[24 + 5 * a + j] - fd) <= 1e-6 * np.abs(g[24:39]).max() + 1e-4 * abs(fd), (a, j)
    # the rollout reaches the later strain segments (the test exercises more than the first)
    assert reached
