"""The implicit-step linear system and its multigrid hierarchy (oracle, FP64).

Implicit time step (Sec. 2.3.2): forces at the new positions, spreading and
interpolation lagged at X^n.  Eliminating F^{n+1} and X^{n+1} (substituting
X^{n+1} = X^n + dt S^* u^{n+1} into F^{n+1} = K L X^{n+1}) gives the Eulerian
saddle system of Sec. 3; with the unsteady Stokes form of the discussion
(Sec. 8, operator I - dt Lap - dt^2 gamma S A_f S^*, here divided by dt and
scaled by rho, mu):

  (rho/dt) u - mu Lap_h u + G p + M_0 u = (rho/dt) u^n + S_0 (K L X^n) + g
  -D u = 0,        M_0 = -dt K S_0 L S^*,  S^* = h^2 S_0^T.

Readings: the printed right-hand side lacks the stiffness factor that the
substitution produces; it is restored (S A_f X^n carries gamma).  The system
is kept in this form, not multiplied by dt, and continuity is written as
-D u so that the matrix is symmetric (D = -G^T); residual norms are taken in
this scaling.

Coarse operators (Sec. 3.2, hybrid): the Stokes part is re-discretised with
h_l = 2^l h, the same rho/dt and mu; the elasticity part is Galerkin,
M_{l+1} = R_l M_l P_l with the velocity transfers of Sec. 3.1, recursively.
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np
import scipy.sparse as sp

from . import mac, ib


@dataclass
class Level:
    N: int
    A: sp.csr_matrix          # 3N^2 x 3N^2 level operator
    M_u: sp.csr_matrix        # elasticity block on u faces
    M_v: sp.csr_matrix        # elasticity block on v faces
    R: sp.csr_matrix | None   # restriction to the next level (None on the coarsest)
    P: sp.csr_matrix | None   # prolongation from the next level


def stokes_blocks(N, c, mu):
    """Blocks of the re-discretised unsteady Stokes operator on an N^2 grid:
    returns (Auu, Gx, Gy, Dx, Dy) with Auu = c I - mu Lap."""
    Lap = mac.laplacian(N)
    Gx, Gy = mac.gradient(N)
    Dx, Dy = mac.divergence(N)
    Auu = c * sp.identity(N * N, format="csr") - mu * Lap
    return Auu, Gx, Gy, Dx, Dy


def assemble(N, c, mu, M_u, M_v):
    """Level matrix [[cI - mu Lap + M_u, 0, Gx], [0, cI - mu Lap + M_v, Gy],
    [-Dx, -Dy, 0]]."""
    Auu, Gx, Gy, Dx, Dy = stokes_blocks(N, c, mu)
    Z = None
    return sp.bmat([[Auu + M_u, Z, Gx],
                    [Z, Auu + M_v, Gy],
                    [-Dx, -Dy, Z]], format="csr")


def ib_operator_fine(X, fiber_offsets, N, dt, K, kind=ib.DELTA_IB4):
    """M_0 = -dt K S_0 L S^* per velocity component (sparse, N^2 x N^2)."""
    L = ib.fiber_laplacian(fiber_offsets, X.shape[0])
    out = []
    for comp in (0, 1):
        S = ib.spread_matrix(X, N, comp, kind)
        Sstar = ib.interp_matrix(X, N, comp, kind)
        out.append((-dt * K) * (S @ L @ Sstar).tocsr())
    return out


def hierarchy(N, levels, rho, mu, dt, X=None, fiber_offsets=None, K=0.0,
              kind=ib.DELTA_IB4):
    """Operators on levels 0..levels-1 (N_l = N / 2^l)."""
    c = rho / dt
    n = N * N
    if X is not None and K != 0.0 and len(X) > 0:
        M_u, M_v = ib_operator_fine(X, fiber_offsets, N, dt, K, kind)
    else:
        M_u = sp.csr_matrix((n, n))
        M_v = sp.csr_matrix((n, n))
    out = []
    Nl = N
    for l in range(levels):
        A = assemble(Nl, c, mu, M_u, M_v)
        if l < levels - 1:
            R = mac.restrict_w(Nl)
            P = mac.prolong_w(Nl)
            lv = Level(Nl, A, M_u, M_v, R, P)
            # Galerkin coarsening of the elasticity part, per component
            M_u = (mac.restrict_u(Nl) @ M_u @ mac.prolong_u(Nl)).tocsr()
            M_v = (mac.restrict_v(Nl) @ M_v @ mac.prolong_v(Nl)).tocsr()
        else:
            lv = Level(Nl, A, M_u, M_v, None, None)
        out.append(lv)
        Nl //= 2
    return out


def rhs(u_n, v_n, X, fiber_offsets, K, dt, rho, g_u=None, g_v=None, kind=ib.DELTA_IB4):
    """b = [(rho/dt) u^n + S_0 (K L X^n) + g_u; (rho/dt) v^n + ... ; 0]."""
    N = u_n.shape[0]
    c = rho / dt
    bu = c * u_n.copy()
    bv = c * v_n.copy()
    if X is not None and len(X) > 0 and K != 0.0:
        G = ib.fiber_force(X, fiber_offsets, K)
        fu, fv = ib.spread(X, G, N, kind)
        bu += fu
        bv += fv
    if g_u is not None:
        bu += g_u
    if g_v is not None:
        bv += g_v
    return np.concatenate([bu.reshape(-1), bv.reshape(-1), np.zeros(N * N)])


def split(w, N):
    n = N * N
    return (w[:n].reshape(N, N), w[n:2 * n].reshape(N, N), w[2 * n:].reshape(N, N))
