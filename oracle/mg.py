"""Geometric multigrid V-cycle, Algorithm 1 of the paper (oracle, FP64).

MGV(w, b, level, nu1, nu2):
  coarsest level: w <- A^{-1} b (exact solve);
  otherwise: nu1 pre-smoothing sweeps; r_{2h} <- I_{2h<-h}(b - A w);
  e_{2h} <- MGV(0, r_{2h}, next level); w <- w + I_{h<-2h} e_{2h};
  nu2 post-smoothing sweeps.

Reading for the periodic problem: the pressure is defined up to a constant,
so the "exact" coarsest solve is the bordered system
[[A_c, e_p], [e_p^T, 0]] [w; lam] = [b; 0] with e_p the indicator of the
pressure unknowns (zero-mean pressure).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .smoother import BoxSmoother


class VCycle:
    def __init__(self, levels, box=4, nu1=2, nu2=2, mode="colour2", omega=1.0):
        """levels: list of system.Level, finest first.  mode: the box order of
        every smoothed level (a string), or one order per smoothed level (a
        sequence; Algorithm 1 fixes no order, so levels may differ).  omega:
        the box correction's weight (1 = the paper's undamped boxes)."""
        self.levels = levels
        self.nu1, self.nu2 = nu1, nu2
        self.omega = omega
        nsm = len(levels) - 1
        self.modes = [mode] * nsm if isinstance(mode, str) else list(mode)[:nsm]
        if len(self.modes) != nsm:
            raise ValueError("one box order per smoothed level")
        self.mode = mode
        self.smoothers = [BoxSmoother(lv.A, lv.N, box) for lv in levels[:-1]]
        Ac = levels[-1].A.toarray()
        Nc = levels[-1].N
        n = Ac.shape[0]
        B = np.zeros((n + 1, n + 1))
        B[:n, :n] = Ac
        B[2 * Nc * Nc:n, n] = 1.0
        B[n, 2 * Nc * Nc:n] = 1.0
        self.coarse_matrix = B
        self.coarse_lu = sla.lu_factor(B)

    def coarse_solve(self, b):
        n = b.shape[0]
        sol = sla.lu_solve(self.coarse_lu, np.concatenate([b, [0.0]]))
        return sol[:n]

    def mgv(self, w, b, l=0):
        lv = self.levels[l]
        if l == len(self.levels) - 1:
            return self.coarse_solve(b)
        sm = self.smoothers[l]
        for _ in range(self.nu1):
            w = sm.sweep(w, b, self.modes[l], self.omega)
        r2 = lv.R @ (b - lv.A @ w)
        e2 = self.mgv(np.zeros_like(r2), r2, l + 1)
        w = w + lv.P @ e2
        for _ in range(self.nu2):
            w = sm.sweep(w, b, self.modes[l], self.omega)
        return w

    def __call__(self, r):
        """Preconditioner z = MGV(0, r) on the finest level."""
        return self.mgv(np.zeros_like(r), r, 0)


def mg_solve(A, b, vcycle, x0=None, rtol=1e-8, maxit=100):
    """Multigrid as the solver (Sec. 5.1): x <- x + MGV(0, b - A x) until
    ||b - A x|| <= rtol ||b|| or maxit V-cycles (stopping early once the
    residual has grown by 1e12: the iteration diverges).  Returns
    (x, V-cycles applied, converged, relative residual history)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, float)
    bnorm = float(np.linalg.norm(b))
    hist = []
    if bnorm == 0.0:
        return np.zeros_like(b), 0, True, hist
    its = 0
    while True:
        r = b - A @ x
        beta = float(np.linalg.norm(r))
        hist.append(beta / bnorm)
        if beta <= rtol * bnorm:
            return x, its, True, hist
        if its >= maxit or beta > 1e12 * bnorm:
            return x, its, False, hist
        x = x + vcycle(r)
        its += 1


def iteration_matrix(A, vcycle, n):
    """The multigrid iteration matrix T = I - M A (M the V-cycle as a linear
    map, the error propagator of one mg_solve step), column by column."""
    T = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        T[:, k] = e - vcycle(A @ e)
    return T
