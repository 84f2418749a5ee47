"""Explicit-time stability limit (oracle; sets dt for the workloads).

Sec. 4.1: the explicit method is forward Euler on dX/dt = gamma S^* L_h^{-1} S A_f X,
stable iff alpha * rho <= 2, with rho the spectral radius of S^* L_h^{-1} S A_f
(real, non-positive eigenvalues: S^* L^{-1} S is symmetric positive
semidefinite and A_f negative semidefinite).

Reading for the nodal-spring workloads (force K L X with unit spreading
weight): lambda_max = spectral radius of E = S^* L_0^{-1} S (-L), L_0 the
steady periodic MAC Stokes operator (mu = 1, zero-mean gauge), evaluated at
the initial configuration; dt_exp = 2 / (K lambda_max).  The eigenvalue is
found with Lanczos (scipy eigsh) on the symmetrised form H A H,
H = (-L)^{1/2}, A = S^* L_0^{-1} S, which has the same non-zero spectrum.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import ib, stokes_fft


def _half_power(fiber_offsets, M):
    """Dense (-L)^{1/2} per fibre, block-diagonal, via symmetric eigensolve."""
    L = ib.fiber_laplacian(fiber_offsets, M).toarray()
    blocks = []
    offs = np.asarray(fiber_offsets)
    for f in range(len(offs) - 1):
        a, b = int(offs[f]), int(offs[f + 1])
        ev, Q = np.linalg.eigh(-L[a:b, a:b])
        ev = np.maximum(ev, 0.0)
        blocks.append((a, b, (Q * np.sqrt(ev)) @ Q.T))
    return blocks


def _apply_blocks(blocks, x):
    y = np.zeros_like(x)
    for a, b, Hb in blocks:
        y[a:b] = Hb @ x[a:b]
    return y


def stokes_coupling(X, N, mu=1.0, kind=ib.DELTA_IB4):
    """Returns a function F (M,2) -> U (M,2) applying S^* L_0^{-1} S."""
    Su = ib.spread_matrix(X, N, 0, kind)
    Sv = ib.spread_matrix(X, N, 1, kind)
    h2 = (1.0 / N) ** 2

    def apply(F):
        fu = (Su @ F[:, 0]).reshape(N, N)
        fv = (Sv @ F[:, 1]).reshape(N, N)
        u, v, _ = stokes_fft.solve(fu, fv, 0.0, mu)
        U = np.empty_like(F)
        U[:, 0] = h2 * (Su.T @ u.reshape(-1))
        U[:, 1] = h2 * (Sv.T @ v.reshape(-1))
        return U
    return apply


def lambda_max(X, fiber_offsets, N, mu=1.0, kind=ib.DELTA_IB4, tol=1e-10):
    M = X.shape[0]
    A = stokes_coupling(X, N, mu, kind)
    blocks = _half_power(fiber_offsets, M)

    def mv(x):
        x = x.reshape(M, 2)
        hx = np.stack([_apply_blocks(blocks, x[:, 0]), _apply_blocks(blocks, x[:, 1])], 1)
        y = A(hx)
        return np.stack([_apply_blocks(blocks, y[:, 0]), _apply_blocks(blocks, y[:, 1])], 1).reshape(-1)

    op = spla.LinearOperator((2 * M, 2 * M), matvec=mv, dtype=float)
    v0 = np.random.default_rng(0).standard_normal(2 * M)
    val = spla.eigsh(op, k=1, which="LA", tol=tol, v0=v0, return_eigenvectors=False)
    return float(val[0])


def lambda_max_dense(X, fiber_offsets, N, mu=1.0, kind=ib.DELTA_IB4):
    """Brute force for tiny cases: assemble E = S^* L_0^{-1} S (-L) column by
    column and take the largest eigenvalue magnitude."""
    M = X.shape[0]
    A = stokes_coupling(X, N, mu, kind)
    L = ib.fiber_laplacian(fiber_offsets, M).toarray()
    E = np.zeros((2 * M, 2 * M))
    for col in range(2 * M):
        e = np.zeros(2 * M)
        e[col] = 1.0
        F = e.reshape(M, 2)
        F = np.stack([-L @ F[:, 0], -L @ F[:, 1]], 1)
        E[:, col] = A(F).reshape(-1)
    return float(np.max(np.abs(np.linalg.eigvals(E))))


def dt_explicit(X, fiber_offsets, N, K, mu=1.0, kind=ib.DELTA_IB4):
    return 2.0 / (K * lambda_max(X, fiber_offsets, N, mu, kind))
