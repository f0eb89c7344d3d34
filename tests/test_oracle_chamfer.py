"""Pins of the Chamfer-distance oracle (Sec. 4.2, Eq. 10) against what the definition
fixes: pure-Python loops on tiny sets, identical sets, single points, a translated
copy of a well-separated set, and the symmetry of the two terms."""

import numpy as np

from oracle import chamfer as C


def loops(g, m):
    """Eq. 10 with plain loops (tiny sets only)."""
    def term(a, b):
        s = 0.0
        for p in a:
            s += min(sum((p[k] - q[k]) ** 2 for k in range(3)) for q in b)
        return s / len(a)
    return term(g, m) + term(m, g)


def test_matches_plain_loops():
    r = np.random.default_rng(0)
    g, m = r.normal(size=(7, 3)), r.normal(size=(5, 3))
    assert abs(C.chamfer(g, m)[0] - loops(g.tolist(), m.tolist())) <= 1e-14


def test_closed_forms():
    r = np.random.default_rng(1)
    g = r.uniform(size=(50, 3))
    assert C.chamfer(g, g)[0] == 0.0
    p, q = np.array([[0.1, 0.2, 0.3]]), np.array([[0.4, -0.1, 0.7]])
    assert abs(C.chamfer(p, q)[0] - 2 * np.sum((p - q) ** 2)) <= 1e-16
    # a grid of spacing 1 and its copy moved by t (|t| << 1/2): each point's nearest
    # neighbour is its own copy, so Ch = 2 |t|^2
    gx = np.stack(np.meshgrid(np.arange(6.0), np.arange(5.0), np.arange(4.0)), -1).reshape(-1, 3)
    t = np.array([0.05, -0.02, 0.03])
    ch, nn = C.chamfer(gx, gx + t)
    assert abs(ch - 2 * t @ t) <= 1e-15
    assert np.array_equal(nn["i_g"], np.arange(len(gx)))


def test_symmetric_and_first_index_on_ties():
    r = np.random.default_rng(2)
    g, m = r.normal(size=(40, 3)), r.normal(size=(33, 3))
    assert abs(C.chamfer(g, m)[0] - C.chamfer(m, g)[0]) <= 1e-15
    m2 = np.concatenate([m, m[:5]])     # duplicates: the first copy is the nearest index
    _, nn = C.chamfer(g, m2)
    assert nn["i_g"].max() < 33
