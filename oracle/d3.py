"""The method in three space dimensions (oracle, FP64).  Test infrastructure:
only the tests, the smoke check and the benchmark's CPU baseline use it.

The paper states its tests in two dimensions and says the formulation, the
hybrid multigrid and the big-box smoother carry over to three (Sec. 2.1,
Sec. 6, and the cost remark of the discussion: a box of n^3 cells holds
d (n + 1) n^(d-1) velocities and n^d pressures, 304 unknowns for n = 4).
This module writes that extension out with the paper's two-dimensional
definitions taken axis by axis:

  * MAC grid (Sec. 2.2) on the periodic unit cube, N cells per side,
    h = 1/N: u[k][j][i] at (i h, (j+1/2) h, (k+1/2) h), v at
    ((i+1/2) h, j h, (k+1/2) h), w at ((i+1/2) h, (j+1/2) h, k h), p at the
    cell centre; flat index (k N + j) N + i; x = [u; v; w; p].
  * 7-point Laplacian, one-sided gradient and divergence (Sec. 2.2).
  * Level system of the implicit step (Sec. 2.3.2 and the unsteady operator
    of the discussion, divided by dt): per component a,
    (c - mu Lap) u_a + G_a p + M_a u_a, continuity -D u, c = rho / dt,
    M_a = -dt K S_a L J_a with S_a the spread matrix (tensor-product delta
    divided by h^3) and J_a = h^3 S_a^T the interpolation.
  * Transfers (Sec. 3.1) per face family: full weighting (1, 2, 1)/4 along
    the face normal and two-point averages along both tangential axes for
    the restriction; linear along the normal and (3/4, 1/4) along each
    tangential axis for the prolongation; pressure by the average of eight
    and by constant prolongation.
  * Coarse levels (Sec. 3.2): Stokes re-discretised, elasticity Galerkin
    M_{l+1} = R M_l P.
  * Box relaxation (Sec. 5-6): boxes of n^3 cells with every face of their
    cells (faces on box sides shared with the neighbour box), the box block
    of the level matrix solved exactly; checkerboard order by
    (bx + by + bz) mod 2, Jacobi within a colour (boxes of one colour share
    no unknowns); optional weight omega.
  * V-cycle (Algorithm 1) with the bordered coarsest solve (zero-mean
    pressure), FGMRES from the two-dimensional oracle (it is dimension free).
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import ib, krylov

E = ((1, 0, 0), (0, 1, 0), (0, 0, 1))


def fidx(i, j, k, N):
    """Flat index of cell or face (i, j, k), periodic."""
    return ((k % N) * N + (j % N)) * N + (i % N)


def _coo(rows, cols, vals, shape):
    return sp.csr_matrix((np.asarray(vals, float), (np.asarray(rows), np.asarray(cols))), shape=shape)


def _cells(N):
    for k in range(N):
        for j in range(N):
            for i in range(N):
                yield i, j, k


def laplacian(N):
    """7-point periodic Laplacian, the same for every face family and p."""
    h2 = (1.0 / N) ** 2
    r, c, v = [], [], []
    for i, j, k in _cells(N):
        a = fidx(i, j, k, N)
        r.append(a); c.append(a); v.append(-6.0 / h2)
        for e in E:
            for s in (1, -1):
                r.append(a); c.append(fidx(i + s * e[0], j + s * e[1], k + s * e[2], N)); v.append(1.0 / h2)
    n = N ** 3
    return _coo(r, c, v, (n, n))


def gradient(N):
    """(G_a p) on face family a: (p(cell) - p(cell - e_a)) / h.  Three
    N^3 x N^3 matrices (faces x cells)."""
    h = 1.0 / N
    out = []
    for e in E:
        r, c, v = [], [], []
        for i, j, k in _cells(N):
            a = fidx(i, j, k, N)
            r += [a, a]; c += [a, fidx(i - e[0], j - e[1], k - e[2], N)]; v += [1.0 / h, -1.0 / h]
        out.append(_coo(r, c, v, (N ** 3, N ** 3)))
    return out


def divergence(N):
    """(D u)(cell) = sum over a of (u_a(cell + e_a) - u_a(cell)) / h.  Three
    N^3 x N^3 matrices (cells x faces of family a)."""
    h = 1.0 / N
    out = []
    for e in E:
        r, c, v = [], [], []
        for i, j, k in _cells(N):
            a = fidx(i, j, k, N)
            r += [a, a]; c += [fidx(i + e[0], j + e[1], k + e[2], N), a]; v += [1.0 / h, -1.0 / h]
        out.append(_coo(r, c, v, (N ** 3, N ** 3)))
    return out


def assemble(N, c, mu, Ms):
    """Level matrix [[cI - mu Lap + M_a, G_a] per component; [-D_a, 0]]."""
    n = N ** 3
    Lap = laplacian(N)
    G = gradient(N)
    D = divergence(N)
    I = sp.identity(n, format="csr")
    blocks = [[None] * 4 for _ in range(4)]
    for a in range(3):
        blocks[a][a] = c * I - mu * Lap + (Ms[a] if Ms is not None else sp.csr_matrix((n, n)))
        blocks[a][3] = G[a]
        blocks[3][a] = -D[a]
    blocks[3][3] = sp.csr_matrix((n, n))
    return sp.bmat(blocks, format="csr")


# ---------------------------------------------------------------- transfers (Sec. 3.1)

def _lin_normal(i):
    """Fine face i along its normal: on coarse face i/2 (i even) or midway
    between (i-1)/2 and (i+1)/2."""
    if i % 2 == 0:
        return [(i // 2, 1.0)]
    return [((i - 1) // 2, 0.5), ((i + 1) // 2, 0.5)]


def _lin_tangent(j):
    """Fine index j along a tangential axis: h/2 below coarse J = j // 2
    for even j (3/4 on J, 1/4 on J - 1), h/2 above for odd j (3/4 on J,
    1/4 on J + 1)."""
    J = j // 2
    return [(J, 0.75), (J - 1, 0.25)] if j % 2 == 0 else [(J, 0.75), (J + 1, 0.25)]


def restrict_face(N, a):
    """R_a: coarse face (I, J, K) of family a = (1/4)(1, 2, 1) over fine faces
    2 I_a - 1, 2 I_a, 2 I_a + 1 along the normal times two-point averages
    over 2 I_t, 2 I_t + 1 along both tangential axes."""
    Nc = N // 2
    r, c, v = [], [], []
    for I in _cells(Nc):
        row = fidx(*I, Nc)
        for d, wd in ((-1, 0.25), (0, 0.5), (1, 0.25)):
            for s1 in (0, 1):
                for s2 in (0, 1):
                    f = [0, 0, 0]
                    t = [b for b in range(3) if b != a]
                    f[a] = 2 * I[a] + d
                    f[t[0]] = 2 * I[t[0]] + s1
                    f[t[1]] = 2 * I[t[1]] + s2
                    r.append(row); c.append(fidx(*f, N)); v.append(wd * 0.25)
    return _coo(r, c, v, (Nc ** 3, N ** 3))


def prolong_face(N, a):
    """P_a: fine face of family a from the coarse faces, linear along the
    normal and (3/4, 1/4) along each tangential axis."""
    Nc = N // 2
    r, c, v = [], [], []
    for f in _cells(N):
        row = fidx(*f, N)
        w = [_lin_normal(f[b]) if b == a else _lin_tangent(f[b]) for b in range(3)]
        for ci, wi in w[0]:
            for cj, wj in w[1]:
                for ck, wk in w[2]:
                    r.append(row); c.append(fidx(ci, cj, ck, Nc)); v.append(wi * wj * wk)
    return _coo(r, c, v, (N ** 3, Nc ** 3))


def restrict_p(N):
    Nc = N // 2
    r, c, v = [], [], []
    for I in _cells(Nc):
        for s in _cells(2):
            r.append(fidx(*I, Nc)); c.append(fidx(2 * I[0] + s[0], 2 * I[1] + s[1], 2 * I[2] + s[2], N))
            v.append(0.125)
    return _coo(r, c, v, (Nc ** 3, N ** 3))


def prolong_p(N):
    Nc = N // 2
    r, c, v = [], [], []
    for f in _cells(N):
        r.append(fidx(*f, N)); c.append(fidx(f[0] // 2, f[1] // 2, f[2] // 2, Nc)); v.append(1.0)
    return _coo(r, c, v, (N ** 3, Nc ** 3))


def restrict_w(N):
    return sp.block_diag([restrict_face(N, 0), restrict_face(N, 1), restrict_face(N, 2), restrict_p(N)],
                         format="csr")


def prolong_w(N):
    return sp.block_diag([prolong_face(N, 0), prolong_face(N, 1), prolong_face(N, 2), prolong_p(N)],
                         format="csr")


# ---------------------------------------------------------------- immersed structure (Sec. 2.2)

def spread_matrix(X, N, comp, kind=ib.DELTA_IB4):
    """S_a: (N^3 x M), entry (face, k) = phi(rx) phi(ry) phi(rz) / h^3, r the
    wrapped offset in grid units from point k to the face of family comp."""
    X = np.asarray(X, float)
    h = 1.0 / N
    off = [0.5, 0.5, 0.5]
    off[comp] = 0.0
    rows, cols, vals = [], [], []
    for k in range(X.shape[0]):
        idx, wts = [], []
        for b in range(3):
            s = X[k, b] / h
            ii = np.floor(s - off[b]).astype(int) + np.arange(-2, 3)
            idx.append(ii)
            wts.append(ib.phi(ib.wrap(ii + off[b] - s, N), kind))
        for a0, i0 in enumerate(idx[0]):
            if wts[0][a0] == 0.0:
                continue
            for a1, i1 in enumerate(idx[1]):
                if wts[1][a1] == 0.0:
                    continue
                for a2, i2 in enumerate(idx[2]):
                    if wts[2][a2] == 0.0:
                        continue
                    rows.append(fidx(i0, i1, i2, N)); cols.append(k)
                    vals.append(wts[0][a0] * wts[1][a1] * wts[2][a2] / h ** 3)
    return sp.csr_matrix((vals, (rows, cols)), shape=(N ** 3, X.shape[0]))


def interp_matrix(X, N, comp, kind=ib.DELTA_IB4):
    """J_a = h^3 S_a^T."""
    return ((1.0 / N) ** 3 * spread_matrix(X, N, comp, kind).T).tocsr()


def ib_operator(X, fiber_offsets, N, dt, K, kind=ib.DELTA_IB4):
    """M_a = -dt K S_a L J_a for a = 0, 1, 2."""
    L = ib.fiber_laplacian(fiber_offsets, X.shape[0])
    return [(-dt * K) * (spread_matrix(X, N, a, kind) @ L @ interp_matrix(X, N, a, kind)).tocsr()
            for a in range(3)]


def spread_force(X, G, N, kind=ib.DELTA_IB4):
    """f_a = S_a G[:, a] as flat N^3 arrays."""
    return [spread_matrix(X, N, a, kind) @ G[:, a] for a in range(3)]


def interp(X, u, kind=ib.DELTA_IB4):
    """U = J u, (M, 3), u a list of three flat face arrays."""
    N = round(len(u[0]) ** (1.0 / 3.0))
    return np.stack([interp_matrix(X, N, a, kind) @ u[a] for a in range(3)], axis=1)


@dataclass
class Level:
    N: int
    A: sp.csr_matrix
    Ms: list
    R: sp.csr_matrix | None
    P: sp.csr_matrix | None


def hierarchy(N, levels, rho, mu, dt, X=None, fiber_offsets=None, K=0.0, kind=ib.DELTA_IB4):
    """Level operators, finest first (N_l = N / 2^l)."""
    c = rho / dt
    n = N ** 3
    if X is not None and K != 0.0 and len(X) > 0:
        Ms = ib_operator(X, fiber_offsets, N, dt, K, kind)
    else:
        Ms = [sp.csr_matrix((n, n)) for _ in range(3)]
    out = []
    Nl = N
    for l in range(levels):
        A = assemble(Nl, c, mu, Ms)
        if l < levels - 1:
            out.append(Level(Nl, A, Ms, restrict_w(Nl), prolong_w(Nl)))
            Ms = [(restrict_face(Nl, a) @ Ms[a] @ prolong_face(Nl, a)).tocsr() for a in range(3)]
        else:
            out.append(Level(Nl, A, Ms, None, None))
        Nl //= 2
    return out


# ---------------------------------------------------------------- box relaxation (Sec. 5-6)

def box_dofs(b, N, n):
    """Indices into x = [u; v; w; p] of box b = (bx, by, bz): for face family
    a every face whose index lies in [b_a n, b_a n + n] along a and in
    [b_t n, b_t n + n - 1] along the other axes (x fastest), then the n^3
    pressures.  d (n + 1) n^(d-1) + n^d unknowns."""
    n3 = N ** 3
    out = []
    for a in range(4):
        ext = [n + 1 if bb == a else n for bb in range(3)]
        for k in range(ext[2]):
            for j in range(ext[1]):
                for i in range(ext[0]):
                    out.append(a * n3 + fidx(b[0] * n + i, b[1] * n + j, b[2] * n + k, N))
    return np.array(out, dtype=np.int64)


class BoxSmoother:
    """Checkerboard box relaxation on one level: every box block extracted
    from the level matrix and inverted (numpy's LU-based inverse); a colour's
    boxes are solved together, each with its own inverse, from the residual
    at the start of the colour."""

    def __init__(self, A, N, n):
        if N % n or (N // n) % 2:
            raise ValueError("N / n must be even")
        self.A = A.tocsr()
        self.N, self.n, self.nb = N, n, N // n
        self.boxes = [b for b in _cells(self.nb)]
        self.D = np.stack([box_dofs(b, N, n) for b in self.boxes])
        self.inv = np.stack([np.linalg.inv(self.A[d][:, d].toarray()) for d in self.D])
        par = np.array([sum(b) % 2 for b in self.boxes])
        self.classes = [np.nonzero(par == c)[0] for c in (0, 1)]
        self.index = {b: q for q, b in enumerate(self.boxes)}

    def box_matrix(self, b):
        d = self.D[self.index[tuple(b)]]
        return self.A[d][:, d].toarray()

    def solve_box(self, b, w, rhs, omega=1.0):
        """w[box] += omega A_box^{-1} (rhs - A w)[box] (a dense solve of the
        extracted block, independent of the stored inverse)."""
        d = self.D[self.index[tuple(b)]]
        r = rhs - self.A @ w
        w = w.copy()
        w[d] += omega * sla.solve(self.A[d][:, d].toarray(), r[d])
        return w

    def sweep(self, w, rhs, omega=1.0):
        w = w.copy()
        for cls in self.classes:
            r = rhs - self.A @ w
            D = self.D[cls]
            w[D] += omega * np.einsum("bij,bj->bi", self.inv[cls], r[D])
        return w


class VCycle:
    """Algorithm 1 on the three-dimensional hierarchy; coarsest level solved
    exactly through the system bordered by the pressure constant."""

    def __init__(self, levels, n=4, nu1=1, nu2=1, omega=1.0):
        self.levels = levels
        self.nu1, self.nu2, self.omega = nu1, nu2, omega
        self.smoothers = [BoxSmoother(lv.A, lv.N, n) for lv in levels[:-1]]
        Nc = levels[-1].N
        A = levels[-1].A.toarray()
        m = A.shape[0]
        B = np.zeros((m + 1, m + 1))
        B[:m, :m] = A
        B[3 * Nc ** 3:m, m] = 1.0
        B[m, 3 * Nc ** 3:m] = 1.0
        self.coarse_matrix = B
        self.coarse_lu = sla.lu_factor(B)

    def coarse_solve(self, b):
        return sla.lu_solve(self.coarse_lu, np.concatenate([b, [0.0]]))[:b.shape[0]]

    def mgv(self, w, b, l=0):
        if l == len(self.levels) - 1:
            return self.coarse_solve(b)
        lv, sm = self.levels[l], self.smoothers[l]
        for _ in range(self.nu1):
            w = sm.sweep(w, b, self.omega)
        r2 = lv.R @ (b - lv.A @ w)
        e = self.mgv(np.zeros_like(r2), r2, l + 1)
        w = w + lv.P @ e
        for _ in range(self.nu2):
            w = sm.sweep(w, b, self.omega)
        return w

    def __call__(self, r):
        return self.mgv(np.zeros_like(r), r, 0)


def bordered_solve(A, b, N):
    """Direct solve of A x = b with zero-mean pressure (reference for tests)."""
    m = A.shape[0]
    e = np.zeros(m)
    e[3 * N ** 3:] = 1.0
    B = sp.bmat([[A, sp.csr_matrix(e[:, None])], [sp.csr_matrix(e[None, :]), None]], format="csc")
    return spla.spsolve(B, np.concatenate([b, [0.0]]))[:m]


def rhs(N, c, u, X=None, fiber_offsets=None, K=0.0, kind=ib.DELTA_IB4):
    """Right-hand side of the implicit step: c u^n + S (K L X^n) per
    component, 0 for continuity.  u: list of three flat face arrays."""
    b = np.zeros(4 * N ** 3)
    for a in range(3):
        b[a * N ** 3:(a + 1) * N ** 3] = c * np.asarray(u[a], float)
    if X is not None and K != 0.0 and len(X) > 0:
        G = ib.fiber_force(X, fiber_offsets, K)
        f = spread_force(X, G, N, kind)
        for a in range(3):
            b[a * N ** 3:(a + 1) * N ** 3] += f[a]
    return b


def step(u, X, fiber_offsets, N, levels, rho, mu, dt, K, n=4, nu=(1, 1), rtol=1e-10, maxit=100,
         kind=ib.DELTA_IB4):
    """One implicit step (Sec. 2.3.2 in three dimensions): solve the level-0
    system with FGMRES preconditioned by the V-cycle, then move the points
    X^{n+1} = X^n + dt J u^{n+1}.  Returns (u, p, X, FGMRES result)."""
    lv = hierarchy(N, levels, rho, mu, dt, X, fiber_offsets, K, kind)
    b = rhs(N, rho / dt, u, X, fiber_offsets, K, kind)
    V = VCycle(lv, n, nu[0], nu[1])
    res = krylov.fgmres(lv[0].A, b, V, rtol=rtol, maxit=maxit)
    n3 = N ** 3
    un = [res.x[a * n3:(a + 1) * n3] for a in range(3)]
    Xn = np.asarray(X, float) + dt * interp(X, un, kind) if X is not None and len(X) else X
    return un, res.x[3 * n3:], Xn, res
