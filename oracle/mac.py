"""MAC staggered-grid operators and multigrid transfers (oracle, FP64).

Paper Sec. 2.2 (staggered grid, second-order Laplacian, gradient and
divergence) and Sec. 3.1 (pressure averaging / constant prolongation;
u restricted by full weighting in x and two-point averaging in y, v the
transpose; bilinear velocity prolongation).

Layout: periodic unit square, N cells per side, h = 1/N; u[j][i] at
(i h, (j+1/2) h), v[j][i] at ((i+1/2) h, j h), p[j][i] at the cell centre.
Flat index j*N + i.  Every matrix here is built entry by entry from its
stencil; nothing is derived from another operator, so identities such as
D = -G^T are genuine checks.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def fidx(i, j, N):
    """Flat index of (i, j) with periodic wrap."""
    return (j % N) * N + (i % N)


def _coo(rows, cols, vals, shape):
    return sp.csr_matrix((np.asarray(vals, float), (np.asarray(rows), np.asarray(cols))),
                         shape=shape)


def laplacian(N):
    """5-point periodic Laplacian (u_E + u_W + u_N + u_S - 4 u)/h^2 on one
    face (or cell) family; identical for u, v and p (Sec. 2.2)."""
    h = 1.0 / N
    r, c, v = [], [], []
    for j in range(N):
        for i in range(N):
            k = fidx(i, j, N)
            r.append(k); c.append(k); v.append(-4.0 / h**2)
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                r.append(k); c.append(fidx(i + di, j + dj, N)); v.append(1.0 / h**2)
    return _coo(r, c, v, (N * N, N * N))


def gradient(N):
    """(Gp)^u_{i,j} = (p_{i,j} - p_{i-1,j})/h,  (Gp)^v_{i,j} = (p_{i,j} - p_{i,j-1})/h.
    Returns (Gx, Gy), each N^2 x N^2 (faces x cells)."""
    h = 1.0 / N
    rx, cx, vx, ry, cy, vy = [], [], [], [], [], []
    for j in range(N):
        for i in range(N):
            k = fidx(i, j, N)
            rx += [k, k]; cx += [fidx(i, j, N), fidx(i - 1, j, N)]; vx += [1 / h, -1 / h]
            ry += [k, k]; cy += [fidx(i, j, N), fidx(i, j - 1, N)]; vy += [1 / h, -1 / h]
    n = N * N
    return _coo(rx, cx, vx, (n, n)), _coo(ry, cy, vy, (n, n))


def divergence(N):
    """(Du)_{i,j} = (u_{i+1,j} - u_{i,j})/h + (v_{i,j+1} - v_{i,j})/h.
    Returns (Dx, Dy), each N^2 x N^2 (cells x faces)."""
    h = 1.0 / N
    rx, cx, vx, ry, cy, vy = [], [], [], [], [], []
    for j in range(N):
        for i in range(N):
            k = fidx(i, j, N)
            rx += [k, k]; cx += [fidx(i + 1, j, N), fidx(i, j, N)]; vx += [1 / h, -1 / h]
            ry += [k, k]; cy += [fidx(i, j + 1, N), fidx(i, j, N)]; vy += [1 / h, -1 / h]
    n = N * N
    return _coo(rx, cx, vx, (n, n)), _coo(ry, cy, vy, (n, n))


# ---------------------------------------------------------------- transfers (Sec. 3.1)

def restrict_p(N):
    """R_p: coarse cell = average of its four fine cells.  (N/2)^2 x N^2."""
    Nc = N // 2
    r, c, v = [], [], []
    for J in range(Nc):
        for I in range(Nc):
            for a in (0, 1):
                for b in (0, 1):
                    r.append(fidx(I, J, Nc)); c.append(fidx(2 * I + a, 2 * J + b, N)); v.append(0.25)
    return _coo(r, c, v, (Nc * Nc, N * N))


def restrict_u(N):
    """R_u = (1/8)[1 2 1; * ; 1 2 1]: full weighting over fine faces
    2I-1, 2I, 2I+1 in x, two-point average over fine rows 2J, 2J+1 in y."""
    Nc = N // 2
    w = {-1: 1.0, 0: 2.0, 1: 1.0}
    r, c, v = [], [], []
    for J in range(Nc):
        for I in range(Nc):
            for d, wd in w.items():
                for jj in (2 * J, 2 * J + 1):
                    r.append(fidx(I, J, Nc)); c.append(fidx(2 * I + d, jj, N)); v.append(wd / 8.0)
    return _coo(r, c, v, (Nc * Nc, N * N))


def restrict_v(N):
    """R_v: the transpose rule of R_u (two-point average in x, full weighting in y)."""
    Nc = N // 2
    w = {-1: 1.0, 0: 2.0, 1: 1.0}
    r, c, v = [], [], []
    for J in range(Nc):
        for I in range(Nc):
            for d, wd in w.items():
                for ii in (2 * I, 2 * I + 1):
                    r.append(fidx(I, J, Nc)); c.append(fidx(ii, 2 * J + d, N)); v.append(wd / 8.0)
    return _coo(r, c, v, (Nc * Nc, N * N))


def prolong_p(N):
    """P_p: each fine cell takes the value of its coarse cell.  N^2 x (N/2)^2."""
    Nc = N // 2
    r, c, v = [], [], []
    for j in range(N):
        for i in range(N):
            r.append(fidx(i, j, N)); c.append(fidx(i // 2, j // 2, Nc)); v.append(1.0)
    return _coo(r, c, v, (N * N, Nc * Nc))


def _lin_normal(i):
    """Bilinear weights along the face-normal direction: fine face i lies on
    coarse face i/2 (i even) or midway between (i-1)/2 and (i+1)/2."""
    if i % 2 == 0:
        return [(i // 2, 1.0)]
    return [((i - 1) // 2, 0.5), ((i + 1) // 2, 0.5)]


def _lin_tangent(j):
    """Bilinear weights along the tangential direction: fine row j = 2J sits
    h/2 below coarse row J (weights 3/4 on J, 1/4 on J-1); j = 2J+1 sits h/2
    above (3/4 on J, 1/4 on J+1)."""
    J = j // 2
    if j % 2 == 0:
        return [(J, 0.75), (J - 1, 0.25)]
    return [(J, 0.75), (J + 1, 0.25)]


def prolong_u(N):
    """P_u: bilinear interpolation of coarse u faces to fine u faces."""
    Nc = N // 2
    r, c, v = [], [], []
    for j in range(N):
        for i in range(N):
            for I, wx in _lin_normal(i):
                for J, wy in _lin_tangent(j):
                    r.append(fidx(i, j, N)); c.append(fidx(I, J, Nc)); v.append(wx * wy)
    return _coo(r, c, v, (N * N, Nc * Nc))


def prolong_v(N):
    """P_v: bilinear interpolation with the roles of x and y exchanged."""
    Nc = N // 2
    r, c, v = [], [], []
    for j in range(N):
        for i in range(N):
            for J, wy in _lin_normal(j):
                for I, wx in _lin_tangent(i):
                    r.append(fidx(i, j, N)); c.append(fidx(I, J, Nc)); v.append(wx * wy)
    return _coo(r, c, v, (N * N, Nc * Nc))


def restrict_w(N):
    """Block restriction of w = [u; v; p]."""
    return sp.block_diag([restrict_u(N), restrict_v(N), restrict_p(N)], format="csr")


def prolong_w(N):
    """Block prolongation of w = [u; v; p]."""
    return sp.block_diag([prolong_u(N), prolong_v(N), prolong_p(N)], format="csr")
