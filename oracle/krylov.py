"""Right-preconditioned flexible GMRES (oracle, FP64).

The paper uses multigrid as a right preconditioner for GMRES (Sec. 3.3) with
an iteration cap of 100 (Sec. 5.1).  The flexible variant (Saad, 1993) stores
the preconditioned vectors z_j and forms x = x0 + Z y; for a fixed linear
preconditioner it produces the same iterates as right-preconditioned GMRES.

Reading of the stopping rule: stop when the Arnoldi residual estimate
|g_{j+1}| <= rtol * ||b||_2 (relative to b, not r0, so warm starts are judged
on the same scale), then confirm with the true residual; if the true residual
misses the target, restart from the current iterate.  Iterations count
preconditioner applications.  Orthogonalisation (the paper does not fix
one): "mgs" (modified Gram-Schmidt), "cgs2" (classical Gram-Schmidt applied
twice), or "dcgs2", classical Gram-Schmidt twice with the second pass delayed
by one iteration (the low-synchronisation form of Swirydowicz, Langou,
Ananthan, Yang and Thomas, 2021).  dcgs2 is cgs2 reordered; in exact
arithmetic both build the same basis and Hessenberg matrix:

  * iteration j projects w = A z_j once against the final v_0 .. v_{j-1}
    and the not yet final u_j (the once-projected, normalised vector of the
    previous iteration): w' = w - sum_k v_k s_k - v_j s_j, norm nu_j,
    u_{j+1} = w' / nu_j;
  * the products <v_k, u_j> and <v_k, w> come from one pass over the basis;
    with t = <v_k, u_j> (k < j) the second projection of u_j is
    v_j = (u_j - sum_k v_k t_k) / rho, rho = sqrt(<u_j, u_j> - |t|^2), and
    s_j = <v_j, w> = (<u_j, w> - t . s) / rho;
  * column j - 1 of H becomes final once t and rho are known, because
    A z_{j-1} = sum_k v_k h_{k,j-1} + nu_{j-1} u_j: h_{k,j-1} += nu_{j-1} t_k,
    h_{j,j-1} = nu_{j-1} rho;
  * the stopping test of iteration j uses column j with its first-pass
    values (a rotated copy); the column is made final (the same second
    projection, of u_{j+1}) before the solution is formed.

z_j is the preconditioner applied to u_j rather than to v_j; the flexible
form only needs A Z = V H with orthonormal V, which holds for whatever z_j
were used.
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
        if orth == "dcgs2":
            x, total, est, done = _cycle_dcgs2(mv, precond, b, x, r, beta, m, maxit, total, target, bnorm, hist)
            r = b - mv(x)
            true = float(np.linalg.norm(r)) / bnorm
            if true * bnorm <= target:
                return FGMRESResult(x, total, True, est, true, hist)
            if total >= maxit:
                return FGMRESResult(x, total, False, est, true, hist)
            continue
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


def _rotate(H, cs, sn, g, j):
    """Apply rotations 0 .. j-1 to column j of H, form rotation j, update g."""
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


def _second_pass(V, j):
    """Products of v_0 .. v_j with u_{j+1}: returns (t, rho), the delayed
    second projection of u_{j+1} (rho^2 = <u, u> - |t|^2)."""
    a = V[:j + 2] @ V[j + 1]
    t = a[:j + 1]
    return t, float(np.sqrt(a[j + 1] - t @ t))


def _cycle_dcgs2(mv, precond, b, x, r, beta, m, maxit, total, target, bnorm, hist):
    """One FGMRES(m) cycle with delayed classical Gram-Schmidt twice.
    Returns (x, total, estimate, stopped on the estimate)."""
    n = b.shape[0]
    V = np.zeros((m + 1, n))
    Z = np.zeros((m, n))
    H = np.zeros((m + 1, m))
    cs = np.zeros(m)
    sn = np.zeros(m)
    g = np.zeros(m + 1)
    g[0] = beta
    V[0] = r / beta
    nu = 0.0          # first-pass norm of the vector now held (as u_j) in V[j]
    est = np.inf
    k = 0
    done = False
    for j in range(m):
        if total >= maxit:
            break
        Z[j] = precond(V[j])
        w = mv(Z[j])
        total += 1
        a = V[:j + 1] @ V[j]       # <v_k, u_j>, <u_j, u_j>
        c = V[:j + 1] @ w          # <v_k, w>, <u_j, w>
        if j > 0:
            t = a[:j]
            rho = float(np.sqrt(a[j] - t @ t))
            H[:j, j - 1] += nu * t
            H[j, j - 1] = nu * rho
            _rotate(H, cs, sn, g, j - 1)
            s_j = (c[j] - t @ c[:j]) / rho
            V[j] = (V[j] - V[:j].T @ t) / rho
        else:
            s_j = c[0]
        H[:j, j] = c[:j]
        H[j, j] = s_j
        w = w - V[:j].T @ c[:j] - s_j * V[j]
        nu = float(np.linalg.norm(w))
        H[j + 1, j] = nu
        if nu != 0.0:
            V[j + 1] = w / nu
        # stopping test on a rotated copy of the first-pass column
        Ht, cst, snt, gt = H.copy(), cs.copy(), sn.copy(), g.copy()
        _rotate(Ht, cst, snt, gt, j)
        est = abs(gt[j + 1]) / bnorm
        hist.append(est)
        k = j + 1
        if abs(gt[j + 1]) <= target or nu == 0.0:
            done = True
            break
    if k == 0:
        return x, total, est, done
    # make column k - 1 final
    j = k - 1
    if nu != 0.0:
        t, rho = _second_pass(V, j)
        H[:j + 1, j] += nu * t
        H[j + 1, j] = nu * rho
    _rotate(H, cs, sn, g, j)
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
    return x + Z[:k].T @ y, total, est, done
