"""Right-preconditioned flexible GMRES (oracle, FP64).

The paper uses multigrid as a right preconditioner for GMRES (Sec. 3.3) with
an iteration cap of 100 (Sec. 5.1).  The flexible variant (Saad, 1993) stores
the preconditioned vectors z_j and forms x = x0 + Z y; for a fixed linear
preconditioner it produces the same iterates as right-preconditioned GMRES.

Reading of the stopping rule: stop when the Arnoldi residual estimate
|g_{j+1}| <= rtol * ||b||_2 (relative to b, not r0, so warm starts are judged
on the same scale), then confirm with the true residual; if the true residual
misses the target, restart from the current iterate.  Iterations count
preconditioner applications.  Orthogonalisation: "mgs" (modified
Gram-Schmidt) or "cgs2" (classical Gram-Schmidt applied twice).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np


@dataclass
class FGMRESResult:
    x: np.ndarray
    iters: int
    converged: bool
    rel_resid_est: float
    rel_resid_true: float
    history: list = field(default_factory=list)


def fgmres(A, b, precond, x0=None, rtol=1e-8, maxit=100, restart=None, orth="cgs2"):
    """Solve A x = b.  A: callable or matrix; precond: callable r -> z."""
    mv = A if callable(A) else (lambda x: A @ x)
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, float)
    bnorm = float(np.linalg.norm(b))
    m = maxit if restart is None else restart
    hist = []
    if bnorm == 0.0:
        return FGMRESResult(np.zeros(n), 0, True, 0.0, 0.0, hist)
    target = rtol * bnorm
    total = 0
    est = np.inf
    while True:
        r = b - mv(x)
        beta = float(np.linalg.norm(r))
        if beta <= target:
            return FGMRESResult(x, total, True, beta / bnorm, beta / bnorm, hist)
        if total >= maxit:
            return FGMRESResult(x, total, False, est, beta / bnorm, hist)
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(m):
            if total >= maxit:
                break
            Z[j] = precond(V[j])
            w = mv(Z[j])
            total += 1
            if orth == "mgs":
                for i in range(j + 1):
                    H[i, j] = np.dot(V[i], w)
                    w = w - H[i, j] * V[i]
            else:
                h1 = V[:j + 1] @ w
                w = w - V[:j + 1].T @ h1
                h2 = V[:j + 1] @ w
                w = w - V[:j + 1].T @ h2
                H[:j + 1, j] = h1 + h2
            H[j + 1, j] = float(np.linalg.norm(w))
            breakdown = H[j + 1, j] == 0.0
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            # apply the previous rotations to the new column
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / d
            sn[j] = H[j + 1, j] / d
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            est = abs(g[j + 1]) / bnorm
            hist.append(est)
            j_done = j + 1
            if abs(g[j + 1]) <= target or breakdown:
                break
        k = j_done
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Z[:k].T @ y
        r = b - mv(x)
        true = float(np.linalg.norm(r)) / bnorm
        if true * bnorm <= target:
            return FGMRESResult(x, total, True, est, true, hist)
        if total >= maxit:
            return FGMRESResult(x, total, False, est, true, hist)
