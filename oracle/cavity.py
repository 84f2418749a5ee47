"""The paper's test problem with walls (oracle, FP64): lid-driven cavity,
thick annulus, steady Stokes (Sec. 4), its explicit stability limit
(Sec. 4.1, Table 1) and the multigrid hierarchy with walls (Sec. 3 on this
domain).  Test infrastructure only, like the rest of this package.

Domain and walls (Sec. 4): the unit square with the velocity prescribed on
the boundary, zero except the tangential velocity on the top wall,
u(x, 1) = (1 - cos 2 pi x) / 2.

Layout: the periodic module's N x N arrays.  u[j][i] sits at (i h, (j+1/2) h),
so the faces i = 0 lie on the walls x = 0 (and, in storage, stand for the
faces on x = 1 as well); v[j][i] at ((i+1/2) h, j h), the faces j = 0 on
y = 0 (and y = 1).  These wall faces carry prescribed normal velocity zero:
they stay in the unknown vector w = [u; v; p] as identity rows that no other
row references, so every iterate keeps them at zero and the remaining rows
are the walled discretisation.

Readings taken (the paper gives the stencils as "standard second-order
finite differences" and no boundary detail):
  * a face next to a wall parallel to it sees the ghost value 2 g - u across
    the wall (g the wall's tangential velocity), so the wall value is the
    average of the face and its ghost; the g term moves to the right-hand
    side;
  * transfers (Sec. 3.1) are the periodic stencils with the wall faces
    removed: restriction rows of coarse wall faces are zero, and the
    bilinear prolongation takes the ghost of the coarse field across a
    tangential wall (-e, homogeneous for an error), which weights the
    coarse face next to the wall by 1/2 for the fine face next to the wall;
    coarse wall faces contribute nothing;
  * the thick annulus (Sec. 4): M1 = 19 N / 8 points along each of M2 =
    3 N / 32 + 1 concentric rings, s1 spacing ds1 = 2 pi r / M1 and s2
    spacing ds2 = w / (M2 - 1); the force density gamma A_f X takes the
    second difference along each ring only, A_f = L / ds^2 (Sec. 2.2), and
    is spread with the printed weight ds^2.  The text sets ds1 = ds2 = ds
    while the sizes give ds1 = 0.661 h and ds2 = 0.667 h; Table 1 decides:
    ds = ds1 in both places reproduces its alpha_exp to the printed digits
    (6.09, 3.93, 2.82, 2.28), the node area ds1 ds2 as weight gives values
    0.8 % lower.  The weights cancel: S A_f X = S_0 L X, the nodal spring
    form of the periodic modules (G = K L X with unit spreading weight) with
    K = gamma.
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import ib, mac

LID = "(1 - cos 2 pi x) / 2"


def wall_u(N):
    """Boolean N x N mask of the u faces on the walls x = 0 (and x = 1)."""
    m = np.zeros((N, N), bool)
    m[:, 0] = True
    return m


def wall_v(N):
    """Boolean N x N mask of the v faces on the walls y = 0 (and y = 1)."""
    m = np.zeros((N, N), bool)
    m[0, :] = True
    return m


def _coo(rows, cols, vals, shape):
    return sp.csr_matrix((np.asarray(vals, float), (np.asarray(rows), np.asarray(cols))), shape=shape)


def laplacian_face(N, comp):
    """5-point Laplacian on the u (comp 0) or v (comp 1) faces with walls.
    Normal direction (x for u): the neighbours across i = 0 / i = N are wall
    faces of value zero and drop out.  Tangential direction: the ghost across
    the wall is -u (homogeneous part; the lid's 2 g term is in lid_rhs).
    Wall-face rows are zero here (the operator adds their identity)."""
    h = 1.0 / N
    r, c, v = [], [], []
    for j in range(N):
        for i in range(N):
            a, t = (i, j) if comp == 0 else (j, i)   # a: normal index, t: tangential index
            if a == 0:
                continue
            k = j * N + i
            diag = -4.0
            for da, dt in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                na, nt = a + da, t + dt
                if na == 0 or na == N:          # wall face: value zero
                    continue
                if nt < 0 or nt >= N:           # across a tangential wall: ghost -u
                    diag -= 1.0
                    continue
                ii, jj = (na, nt) if comp == 0 else (nt, na)
                r.append(k); c.append(jj * N + ii); v.append(1.0 / h**2)
            r.append(k); c.append(k); v.append(diag / h**2)
    return _coo(r, c, v, (N * N, N * N))


def gradient(N):
    """(Gp)^u_{i,j} = (p_{i,j} - p_{i-1,j}) / h for i >= 1, (Gp)^v likewise
    for j >= 1; zero on wall faces.  Returns (Gx, Gy)."""
    h = 1.0 / N
    rx, cx, vx, ry, cy, vy = [], [], [], [], [], []
    for j in range(N):
        for i in range(N):
            k = j * N + i
            if i >= 1:
                rx += [k, k]; cx += [k, k - 1]; vx += [1 / h, -1 / h]
            if j >= 1:
                ry += [k, k]; cy += [k, k - N]; vy += [1 / h, -1 / h]
    n = N * N
    return _coo(rx, cx, vx, (n, n)), _coo(ry, cy, vy, (n, n))


def divergence(N):
    """(Du)_{i,j} = (u_{i+1,j} - u_{i,j}) / h + (v_{i,j+1} - v_{i,j}) / h with
    the wall faces (i = 0, i + 1 = N; j = 0, j + 1 = N) of value zero.
    Returns (Dx, Dy)."""
    h = 1.0 / N
    rx, cx, vx, ry, cy, vy = [], [], [], [], [], []
    for j in range(N):
        for i in range(N):
            k = j * N + i
            if i + 1 < N:
                rx.append(k); cx.append(k + 1); vx.append(1 / h)
            if i >= 1:
                rx.append(k); cx.append(k); vx.append(-1 / h)
            if j + 1 < N:
                ry.append(k); cy.append(k + N); vy.append(1 / h)
            if j >= 1:
                ry.append(k); cy.append(k); vy.append(-1 / h)
    n = N * N
    return _coo(rx, cx, vx, (n, n)), _coo(ry, cy, vy, (n, n))


def wall_identity(N):
    """Diagonal matrix with 1 on the wall faces of w = [u; v; p]."""
    d = np.concatenate([wall_u(N).ravel(), wall_v(N).ravel(), np.zeros(N * N, bool)]).astype(float)
    return sp.diags(d, format="csr")


def assemble(N, c, mu, M_u, M_v):
    """Level matrix with walls: [[c I - mu Lap_u + M_u, 0, Gx], [0, c I -
    mu Lap_v + M_v, Gy], [-Dx, -Dy, 0]] on the interior faces, identity rows
    on the wall faces (c I acts on interior faces only)."""
    n = N * N
    Gx, Gy = gradient(N)
    Dx, Dy = divergence(N)
    iu = sp.diags((~wall_u(N)).ravel().astype(float), format="csr")
    iv = sp.diags((~wall_v(N)).ravel().astype(float), format="csr")
    Auu = c * iu - mu * laplacian_face(N, 0) + M_u
    Avv = c * iv - mu * laplacian_face(N, 1) + M_v
    A = sp.bmat([[Auu, None, Gx], [None, Avv, Gy], [-Dx, -Dy, None]], format="csr")
    return (A + wall_identity(N)).tocsr()


def lid_rhs(N, mu):
    """Right-hand side of the lid (top wall tangential velocity g(x)): the
    ghost 2 g - u of the top row of u faces puts mu 2 g / h^2 on that row."""
    h = 1.0 / N
    bu = np.zeros((N, N))
    x = np.arange(N) * h
    g = 0.5 * (1.0 - np.cos(2.0 * np.pi * x))
    bu[N - 1, 1:] = mu * 2.0 * g[1:] / h**2
    return np.concatenate([bu.ravel(), np.zeros(N * N), np.zeros(N * N)])


# ---------------------------------------------------------------- transfers with walls

def restrict_u(N):
    """R_u of Sec. 3.1 with the coarse wall faces' rows removed."""
    Nc = N // 2
    R = mac.restrict_u(N).tolil()
    for J in range(Nc):
        R.rows[J * Nc], R.data[J * Nc] = [], []
    return R.tocsr()


def restrict_v(N):
    Nc = N // 2
    R = mac.restrict_v(N).tolil()
    for I in range(Nc):
        R.rows[I], R.data[I] = [], []
    return R.tocsr()


def _lin_tangent_wall(j, Nc):
    """Bilinear weights along the tangential direction with the ghost -e
    across a wall: the fine row next to a wall takes 3/4 - 1/4 of its
    coarse row."""
    J = j // 2
    if j % 2 == 0:
        return [(J, 0.75), (J - 1, 0.25)] if J >= 1 else [(J, 0.5)]
    return [(J, 0.75), (J + 1, 0.25)] if J + 1 < Nc else [(J, 0.5)]


def _lin_normal_wall(i, Nc):
    """Bilinear weights along the normal direction; coarse wall faces
    (index 0 or Nc) are zero and drop out."""
    if i % 2 == 0:
        return [] if i == 0 else [(i // 2, 1.0)]
    return [(I, 0.5) for I in ((i - 1) // 2, (i + 1) // 2) if 0 < I < Nc]


def prolong_u(N):
    Nc = N // 2
    r, c, v = [], [], []
    for j in range(N):
        for i in range(N):
            for I, wx in _lin_normal_wall(i, Nc):
                for J, wy in _lin_tangent_wall(j, Nc):
                    r.append(j * N + i); c.append(J * Nc + I); v.append(wx * wy)
    return _coo(r, c, v, (N * N, Nc * Nc))


def prolong_v(N):
    Nc = N // 2
    r, c, v = [], [], []
    for j in range(N):
        for i in range(N):
            for J, wy in _lin_normal_wall(j, Nc):
                for I, wx in _lin_tangent_wall(i, Nc):
                    r.append(j * N + i); c.append(J * Nc + I); v.append(wx * wy)
    return _coo(r, c, v, (N * N, Nc * Nc))


def restrict_w(N):
    return sp.block_diag([restrict_u(N), restrict_v(N), mac.restrict_p(N)], format="csr")


def prolong_w(N):
    return sp.block_diag([prolong_u(N), prolong_v(N), mac.prolong_p(N)], format="csr")


# ---------------------------------------------------------------- structure

@dataclass
class Annulus:
    X: np.ndarray             # (M1 M2, 2) node positions, ring by ring
    fiber_offsets: np.ndarray  # M2 + 1 offsets, one closed ring each
    M1: int
    M2: int
    ds1: float
    ds2: float


def annulus(N, xc=0.5, yc=0.5, r=0.25, width=1.0 / 16):
    """Thick annulus of Sec. 4: X(s1, s2) = (xc + (r + s2) cos(s1 / r),
    yc + (r + s2) sin(s1 / r)), s1 = k ds1 (k < M1), s2 = l ds2 (l < M2)."""
    if N % 32:
        raise ValueError("N must be a multiple of 32 (M1 = 19 N / 8, M2 = 3 N / 32 + 1)")
    M1, M2 = 19 * N // 8, 3 * N // 32 + 1
    ds1, ds2 = 2.0 * np.pi * r / M1, width / (M2 - 1)
    s1 = np.arange(M1) * ds1
    X = []
    for l in range(M2):
        rad = r + l * ds2
        X.append(np.stack([xc + rad * np.cos(s1 / r), yc + rad * np.sin(s1 / r)], 1))
    return Annulus(np.concatenate(X), np.arange(M2 + 1) * M1, M1, M2, ds1, ds2)


def nodal_stiffness(a: Annulus, gamma):
    """K of the nodal form G = K L X for the force density gamma A_f X,
    A_f = L / ds1^2, spread with weight ds1^2: K = gamma."""
    return gamma


# ---------------------------------------------------------------- hierarchy and explicit limit

@dataclass
class Level:
    N: int
    A: sp.csr_matrix
    M_u: sp.csr_matrix
    M_v: sp.csr_matrix
    R: sp.csr_matrix | None
    P: sp.csr_matrix | None


def ib_operator(a: Annulus, N, alpha, kind=ib.DELTA_COS4):
    """alpha S A_f S^* per velocity component as the matrix M_0 of the
    system (the periodic modules' sign: M_0 = -alpha S A_f S^*, positive
    semidefinite); S A_f = S_0 L (weights as in the module header)."""
    L = ib.fiber_laplacian(a.fiber_offsets, a.X.shape[0])
    out = []
    for comp in (0, 1):
        S = ib.spread_matrix(a.X, N, comp, kind)
        Ss = ib.interp_matrix(a.X, N, comp, kind)
        out.append((-alpha) * (S @ L @ Ss).tocsr())
    return out


def hierarchy(N, levels, alpha, a: Annulus | None = None, c=0.0, mu=1.0, kind=ib.DELTA_COS4):
    """Levels 0 .. levels-1 of the walled problem: Stokes re-discretised with
    walls on every level, the elasticity part Galerkin with the walled
    transfers (Sec. 3.2).  c = rho / dt (0: the steady form of Sec. 4)."""
    n = N * N
    if a is not None and alpha != 0.0:
        M_u, M_v = ib_operator(a, N, alpha, kind)
    else:
        M_u = sp.csr_matrix((n, n))
        M_v = sp.csr_matrix((n, n))
    out = []
    Nl = N
    for l in range(levels):
        A = assemble(Nl, c, mu, M_u, M_v)
        if l < levels - 1:
            lv = Level(Nl, A, M_u, M_v, restrict_w(Nl), prolong_w(Nl))
            M_u = (restrict_u(Nl) @ M_u @ prolong_u(Nl)).tocsr()
            M_v = (restrict_v(Nl) @ M_v @ prolong_v(Nl)).tocsr()
        else:
            lv = Level(Nl, A, M_u, M_v, None, None)
        out.append(lv)
        Nl //= 2
    return out


def rhs(N, a: Annulus | None, gamma, mu=1.0, kind=ib.DELTA_COS4):
    """b of the steady cavity system: the lid plus the spread force
    gamma S A_f X^n (the elastic force of the configuration X^n)."""
    b = lid_rhs(N, mu)
    if a is not None and gamma != 0.0:
        G = ib.fiber_force(a.X, a.fiber_offsets, nodal_stiffness(a, gamma))
        fu, fv = ib.spread(a.X, G, N, kind)
        b[:N * N] += np.where(wall_u(N), 0.0, fu).ravel()
        b[N * N:2 * N * N] += np.where(wall_v(N), 0.0, fv).ravel()
    return b


def stokes_solver(N, mu=1.0):
    """Steady walled Stokes solve f -> (u, v) through a sparse LU of the
    system bordered by the constant-pressure constraint."""
    A = assemble(N, 0.0, mu, sp.csr_matrix((N * N, N * N)), sp.csr_matrix((N * N, N * N)))
    n = A.shape[0]
    e = np.zeros(n)
    e[2 * N * N:] = 1.0
    B = sp.bmat([[A, sp.csr_matrix(e[:, None])], [sp.csr_matrix(e[None, :]), None]], format="csc")
    lu = spla.splu(B)

    def solve(fu, fv):
        fu = np.asarray(fu).reshape(N, N)
        fv = np.asarray(fv).reshape(N, N)
        rhs_ = np.concatenate([np.where(wall_u(N), 0.0, fu).ravel(), np.where(wall_v(N), 0.0, fv).ravel(),
                               np.zeros(N * N + 1)])
        x = lu.solve(rhs_)
        return x[:N * N], x[N * N:2 * N * N]
    return solve


def alpha_exp(N, kind=ib.DELTA_COS4, tol=1e-10, a: Annulus | None = None):
    """alpha_exp = 2 / rho(S^* L_h^{-1} S A_f) (Sec. 4.1) for the annulus in
    the walled cavity, L_h the steady Stokes solve (mu = 1).  With S A_f =
    S_0 L and -L = D^T D (D the forward difference along each ring), the
    non-zero spectrum is that of the symmetric D P D^T, P = h^2 S_0^T
    L_h^{-1} S_0; its largest eigenvalue by Lanczos."""
    a = annulus(N) if a is None else a
    M = a.X.shape[0]
    h2 = (1.0 / N) ** 2
    Su = ib.spread_matrix(a.X, N, 0, kind)
    Sv = ib.spread_matrix(a.X, N, 1, kind)
    solve = stokes_solver(N)
    r, c, v = [], [], []
    for f in range(a.M2):
        o = f * a.M1
        for k in range(a.M1):
            r += [o + k, o + k]; c += [o + (k + 1) % a.M1, o + k]; v += [1.0, -1.0]
    D = _coo(r, c, v, (M, M))

    def mv(y):
        y = y.reshape(2, M)
        F = np.stack([D.T @ y[0], D.T @ y[1]])
        u, vv = solve(Su @ F[0], Sv @ F[1])
        U = h2 * np.stack([Su.T @ u, Sv.T @ vv])
        return np.concatenate([D @ U[0], D @ U[1]])

    op = spla.LinearOperator((2 * M, 2 * M), matvec=mv, dtype=float)
    v0 = np.random.default_rng(0).standard_normal(2 * M)
    lam = float(spla.eigsh(op, k=1, which="LA", tol=tol, v0=v0, return_eigenvectors=False)[0])
    return 2.0 / lam
