"""Generalised (big-)box relaxation (oracle, FP64).

Paper Sec. 5 (Vanka-type box relaxation: per cell, solve the local system
of its four velocities and one pressure) and Sec. 6 (big boxes: n x n cells
updated together; velocities on box edges belong to both neighbouring boxes
and are updated twice; no further overlap).  The local matrix is the
restriction of the full level operator, elasticity term included, to the
box's unknowns; each box update is w[box] += A_box^{-1} (b - A w)[box], with
no damping (none is stated).

Orderings:
  * paper mode: boxes in lexicographic order, block Gauss-Seidel (Sec. 5, 6);
  * colour2 mode: two colours, (bx + by) mod 2 (checkerboard), colour 0
    first; within a colour every box solves from the residual at the start
    of that colour (Jacobi within a colour).  Boxes of one colour share no
    unknowns (diagonal neighbours touch only at a corner).  This is the GPU
    path's default ordering;
  * colour mode: four colours by (bx mod 2, by mod 2) in the order (0,0),
    (1,0), (0,1), (1,1), with the same within-colour rule.
The coloured orderings are different (equally valid) smoothers from the
paper's lexicographic one.

The local solve uses a pivoted dense LU of the extracted block.

Damping: the paper states none (omega = 1, every default here).  An optional
omega scales each box correction, w[box] += omega A_box^{-1} (b - A w)[box]
-- the damped block relaxation that weights a smoother's correction, an
option of this build (a schedule parameter), not the paper's method.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

COLOURS = ((0, 0), (1, 0), (0, 1), (1, 1))
MODES = ("colour2", "colour", "paper")


def box_dofs(bx, by, N, n):
    """Indices into w = [u; v; p] of the unknowns of box (bx, by): all u faces
    i in [bx n, bx n + n], j in [by n, by n + n - 1]; all v faces
    i in [bx n, bx n + n - 1], j in [by n, by n + n]; the n^2 pressures."""
    NN = N * N
    u = [((j % N) * N + (i % N)) for j in range(by * n, by * n + n)
         for i in range(bx * n, bx * n + n + 1)]
    v = [NN + ((j % N) * N + (i % N)) for j in range(by * n, by * n + n + 1)
         for i in range(bx * n, bx * n + n)]
    p = [2 * NN + ((j % N) * N + (i % N)) for j in range(by * n, by * n + n)
         for i in range(bx * n, bx * n + n)]
    return np.array(u + v + p, dtype=np.int64)


def box_dof_table(N, n):
    """box_dofs of every box as one (nb^2, ndof) array, row by * nb + bx."""
    nb = N // n
    NN = N * N
    by, bx = np.divmod(np.arange(nb * nb), nb)
    bx, by = bx[:, None], by[:, None]
    lu_j, lu_i = np.divmod(np.arange(n * (n + 1)), n + 1)   # u faces: n rows of n + 1
    lv_j, lv_i = np.divmod(np.arange(n * (n + 1)), n)       # v faces: n + 1 rows of n
    lp_j, lp_i = np.divmod(np.arange(n * n), n)
    u = ((by * n + lu_j) % N) * N + (bx * n + lu_i) % N
    v = NN + ((by * n + lv_j) % N) * N + (bx * n + lv_i) % N
    p = 2 * NN + ((by * n + lp_j) % N) * N + (bx * n + lp_i) % N
    return np.concatenate([u, v, p], axis=1).astype(np.int64)


def sweep_shared(A, N, n, w, b, mode="colour2", omega=1.0):
    """One coloured sweep (Jacobi within a colour, colour order as
    BoxSmoother.sweep_colour2 / sweep_colour) on a level without elastic
    rows.  The periodic Stokes operator is invariant under translation, so
    every box block is the same matrix: the block of box (0, 0) is factored
    once and all boxes of a colour are solved together from the residual at
    the start of that colour.  Boxes of one colour share no unknowns, so the
    scatter of their updates has no repeated index."""
    A = A.tocsr()
    D = box_dof_table(N, n)
    lu = sla.lu_factor(A[D[0]][:, D[0]].toarray())
    nb = N // n
    by, bx = np.divmod(np.arange(nb * nb), nb)
    if mode == "colour2":
        classes = [(bx + by) % 2 == par for par in (0, 1)]
    elif mode == "colour":
        classes = [(bx % 2 == cx) & (by % 2 == cy) for cx, cy in COLOURS]
    else:
        raise ValueError(mode)
    w = w.copy()
    for sel in classes:
        r = b - A @ w
        Dc = D[sel]
        w[Dc] += omega * sla.lu_solve(lu, r[Dc].T).T
    return w


class BoxSmoother:
    """Box relaxation on one level: extracts and factors every box block."""

    def __init__(self, A, N, n):
        if N % n != 0 or N < 2 * n:
            raise ValueError("box size must divide N and N >= 2n")
        self.A = A.tocsr()
        self.N, self.n = N, n
        self.nb = N // n
        self.dofs = {}
        self.lu = {}
        for by in range(self.nb):
            for bx in range(self.nb):
                d = box_dofs(bx, by, N, n)
                self.dofs[(bx, by)] = d
                Ab = self.A[d][:, d].toarray()
                self.lu[(bx, by)] = sla.lu_factor(Ab)

    def box_matrix(self, bx, by):
        d = self.dofs[(bx, by)]
        return self.A[d][:, d].toarray()

    def sweep_colour(self, w, b, omega=1.0):
        """One sweep in colour order with Jacobi-within-colour semantics."""
        w = w.copy()
        for cx, cy in COLOURS:
            r = b - self.A @ w
            upd = []
            for by in range(cy, self.nb, 2):
                for bx in range(cx, self.nb, 2):
                    d = self.dofs[(bx, by)]
                    upd.append((d, sla.lu_solve(self.lu[(bx, by)], r[d])))
            for d, z in upd:
                w[d] += omega * z
        return w

    def sweep_colour2(self, w, b, omega=1.0):
        """One checkerboard sweep: colour (bx + by) mod 2 = 0, then 1, each
        from the residual at the start of the colour."""
        w = w.copy()
        for par in (0, 1):
            r = b - self.A @ w
            upd = []
            for by in range(self.nb):
                for bx in range(self.nb):
                    if (bx + by) % 2 != par:
                        continue
                    d = self.dofs[(bx, by)]
                    upd.append((d, sla.lu_solve(self.lu[(bx, by)], r[d])))
            for d, z in upd:
                w[d] += omega * z
        return w

    def sweep_paper(self, w, b, omega=1.0):
        """One lexicographic block Gauss-Seidel sweep (the paper's order)."""
        w = w.copy()
        for by in range(self.nb):
            for bx in range(self.nb):
                d = self.dofs[(bx, by)]
                r = b[d] - self.A[d] @ w
                w[d] += omega * sla.lu_solve(self.lu[(bx, by)], r)
        return w

    def sweep(self, w, b, mode="colour2", omega=1.0):
        if mode == "colour2":
            return self.sweep_colour2(w, b, omega)
        if mode == "colour":
            return self.sweep_colour(w, b, omega)
        if mode == "paper":
            return self.sweep_paper(w, b, omega)
        raise ValueError(mode)
