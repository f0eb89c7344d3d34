"""Oracle of phi-SfT's outer optimisation loop (Sec. 3.3 'Adaptive Optimisation Scheme'
and Sec. 3.4): Adam over the physical parameters with a growing active window of frames.
Test infrastructure only: the product path never imports this module.

Written from the paper, independent of the GPU library's driver:
  * each iteration simulates frames 1..t_a from the template and evaluates the energy of
    every active frame (Sec. 3.4: the objective is recomputed for all active frames in
    every iteration); here the energy of frame t is E_t = sum_i |x_t,i - target_t,i|^2,
    the 3D stand-in for the image energies, and the gradient comes from the oracle's
    exact-solve rollout and adjoint (Oracle.gradient_exact);
  * Adam (Kingma and Ba, 'Adam: A Method for Stochastic Optimization', Algorithm 1):
    m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2, theta <- theta - lr (m / (1-b1^t)) /
    (sqrt(v / (1-b2^t)) + eps), learning rate 1e-3 (Sec. 3.4);
  * the window (Sec. 3.3): five active frames at the start; the next frame joins when
    the latest active frame's energy is below b or after an iteration cap on the current
    window. b is what the fifth frame's energy is when the sixth joins; before that
    moment b does not exist, so that first join comes from the cap (reading).

Parameters: the material (k_s, k_b, d) through its logarithm, the wind velocity, and the
per-step forces F_t through F_t / (vertex area): the paper adds the optimised corrective
term to the vertex velocity (mass and step constant), and with lumped masses
proportional to the vertex areas that velocity increment is F_t / area up to a constant.
"""

from __future__ import annotations

import numpy as np


class Adam:
    """Adam on a flat float64 vector theta (Algorithm 1 of Kingma and Ba)."""

    def __init__(self, n, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, theta, g, t):
        """theta after step t (t = 1, 2, ...) with gradient g."""
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mhat = self.m / (1.0 - self.b1 ** t)
        vhat = self.v / (1.0 - self.b2 ** t)
        return theta - self.lr * mhat / (np.sqrt(vhat) + self.eps)


class Window:
    """The active window t_a of Sec. 3.3 and its threshold b."""

    def __init__(self, n_frames, first=5, max_iters=50):
        self.n_frames, self.first, self.max_iters = n_frames, first, max_iters
        self.t_a = min(first, n_frames)
        self.b = None
        self.since = 0

    def update(self, E):
        """After an iteration whose active frames 1..t_a had energies E."""
        self.since += 1
        if self.t_a == self.n_frames:
            return
        reached = self.b is not None and E[self.t_a - 1] < self.b
        if reached or self.since == self.max_iters:
            if self.t_a == self.first and self.b is None:
                self.b = E[self.first - 1]     # frame five's energy as frame six joins
            self.t_a += 1
            self.since = 0


def window_schedule(energies_of, n_frames, iterations, first=5, max_iters=50):
    """Active window per iteration for an energy source energies_of(it, t_a) -> the
    energies of frames 1..t_a at iteration it. Returns the list of t_a and b."""
    w = Window(n_frames, first, max_iters)
    out = []
    for it in range(iterations):
        out.append(w.t_a)
        w.update(energies_of(it, w.t_a))
    return out, w.b


def optimise(oracle, targets, x0, material, wind=None, forces=None, iterations=20, first=5,
             max_iters=50, lr=(1e-3, 1e-3, 1e-3), beta1=0.9, beta2=0.999, eps=1e-8,
             optimise=("material", "wind", "forces")):
    """Runs the loop on one sheet. targets [T, V, 3]; x0 [V, 3]; material (k_s, k_b, d);
    wind [3] or None (no aerodynamic force, not optimised); forces [T, V, 3] or None
    (zero). lr: learning rates of (material, wind, forces). Returns the history
    (t_a, per-frame energies) and the final parameters."""
    T, V = targets.shape[0], targets.shape[1]
    p_mat = np.array(material, dtype=np.float64)
    p_w = None if wind is None else np.array(wind, dtype=np.float64)
    F = np.zeros((T, V, 3)) if forces is None else np.array(forces, dtype=np.float64)
    area = oracle.geometry()["vert_area"]
    opt_m = Adam(3, lr[0], beta1, beta2, eps)
    opt_w = Adam(3, lr[1], beta1, beta2, eps)
    opt_f = Adam(T * V * 3, lr[2], beta1, beta2, eps)
    win = Window(T, first, max_iters)
    history = []
    for it in range(1, iterations + 1):
        t_a = win.t_a
        oracle.set_params(ks=p_mat[0], kb=p_mat[1], density=p_mat[2])
        oracle.set_wind(p_w)
        frames = list(range(1, t_a + 1))
        r = oracle.gradient_exact(t_a, x0, None, F[:t_a], frames, targets[:t_a])
        E = np.sum((r["x"] - targets[:t_a]) ** 2, axis=(1, 2))
        history.append((t_a, E))
        if "material" in optimise:
            th = opt_m.step(np.log(p_mat), r["material"] * p_mat, it)
            p_mat = np.exp(th)
        if "wind" in optimise and p_w is not None:
            p_w = opt_w.step(p_w, r["wind"], it)
        if "forces" in optimise:
            # a frame that has never been active has zero gradient and zero moments,
            # so Adam leaves it where it is (0 / (0 + eps))
            g = np.zeros((T, V, 3))
            g[:t_a] = r["forces"] * area[None, :, None]
            th_new = opt_f.step((F / area[None, :, None]).ravel(), g.ravel(), it)
            F = th_new.reshape(T, V, 3) * area[None, :, None]
        win.update(E)
    return dict(history=history, material=p_mat, wind=p_w, forces=F, threshold=win.b)
