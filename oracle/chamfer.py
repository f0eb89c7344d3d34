"""FP64 CPU oracle of the Chamfer distance -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module; the GPU library never loads it.

The paper evaluates reconstructions by the Chamfer distance between a point cloud
G and points M sampled from the reconstructed mesh (Sec. 4.2, Eq. 10):
  Ch(G, M) = 1/|G| sum_{g in G} min_{m in M} |g - m|^2 + 1/|M| sum_{m in M} min_{g in G} |m - g|^2.
This is that definition written out: every squared distance in FP64, the minimum
over the other set, the two means. Points are vertex-major [N, 3].
"""

from __future__ import annotations

import numpy as np


def nearest(q, db, chunk: int = 1024):
    """For every point of q [Nq, 3]: the smallest squared distance to db [Nd, 3] and the
    index of the first point of db that attains it (Eq. 10's inner minimum)."""
    q = np.asarray(q, dtype=np.float64)
    db = np.asarray(db, dtype=np.float64)
    d = np.empty(q.shape[0])
    idx = np.empty(q.shape[0], dtype=np.int64)
    for a in range(0, q.shape[0], chunk):
        diff = q[a:a + chunk, None, :] - db[None, :, :]
        sq = np.einsum("ijk,ijk->ij", diff, diff)
        idx[a:a + chunk] = np.argmin(sq, axis=1)
        d[a:a + chunk] = sq[np.arange(sq.shape[0]), idx[a:a + chunk]]
    return d, idx


def chamfer(g, m):
    """Ch(G, M) of Eq. 10, with the per-point minima of both directions."""
    dg, ig = nearest(g, m)
    dm, im = nearest(m, g)
    return float(dg.mean() + dm.mean()), dict(d_g=dg, i_g=ig, d_m=dm, i_m=im)
