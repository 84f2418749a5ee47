"""Pins of the three-dimensional oracle (oracle/d3.py) to what the paper and
the mathematics fix: the box size the paper counts (304 unknowns, about
750 KB dense for n = 4), the reduction of every operator to the pinned
two-dimensional oracle on fields that do not depend on one coordinate, the
cyclic symmetry of the axes, closed-form Stokes solutions, the structure of
the elastic operator, exact box solves, and the multigrid-preconditioned
solve against a direct one."""
import numpy as np
import pytest

import ibgen
from oracle import d3, ib, krylov, mac, smoother


def test_box_unknowns_and_dense_size():
    """Discussion of solver performance: a box of n^d cells holds
    d (n + 1) n^(d-1) velocities and n^d pressures: 56 unknowns (about
    25 KB dense) for d = 2, n = 4, and 304 (about 750 KB) for d = 3, n = 4."""
    N = 16
    for n in (1, 2, 4):
        assert len(d3.box_dofs((1, 0, 1), N, n)) == 3 * (n + 1) * n * n + n ** 3
        assert len(smoother.box_dofs(1, 0, N, n)) == 2 * (n + 1) * n + n * n
    assert len(d3.box_dofs((0, 0, 0), N, 4)) == 304
    assert len(smoother.box_dofs(0, 0, N, 4)) == 56
    assert round(304 ** 2 * 8 / 1000, -1) == 740.0          # "approximately 750 KB"
    assert round(56 ** 2 * 8 / 1000) == 25                   # "approximately 25 KB"
    d = d3.box_dofs((1, 1, 0), N, 4)
    assert len(np.unique(d)) == len(d)


def _lift(f2, N):
    """z-invariant 3-D field from a 2-D (N, N) array [j][i]."""
    return np.broadcast_to(f2.reshape(1, N, N), (N, N, N)).reshape(-1)


def test_operators_reduce_to_two_dimensions():
    """On fields that do not depend on z, with w = 0, the 3-D Laplacian,
    gradient and divergence equal the pinned 2-D ones in every z plane."""
    N = 8
    rng = np.random.default_rng(1)
    u2, v2, p2 = (rng.standard_normal((N, N)) for _ in range(3))
    L3, L2 = d3.laplacian(N), mac.laplacian(N)
    assert np.allclose(L3 @ _lift(u2, N), _lift((L2 @ u2.ravel()).reshape(N, N), N), atol=1e-10)
    G3 = d3.gradient(N)
    Gx, Gy = mac.gradient(N)
    assert np.allclose(G3[0] @ _lift(p2, N), _lift((Gx @ p2.ravel()).reshape(N, N), N))
    assert np.allclose(G3[1] @ _lift(p2, N), _lift((Gy @ p2.ravel()).reshape(N, N), N))
    assert np.allclose(G3[2] @ _lift(p2, N), 0.0)
    D3 = d3.divergence(N)
    Dx, Dy = mac.divergence(N)
    div3 = D3[0] @ _lift(u2, N) + D3[1] @ _lift(v2, N)
    assert np.allclose(div3, _lift((Dx @ u2.ravel() + Dy @ v2.ravel()).reshape(N, N), N))


def test_transfers_reduce_to_two_dimensions():
    """Restriction and prolongation of z-invariant u, v and p fields equal the
    pinned 2-D transfers plane by plane; w's (normal z) transfers act on
    z-invariant fields as the 2-D pressure-like tangential rules do."""
    N = 8
    Nc = N // 2
    rng = np.random.default_rng(2)
    u2, v2, p2 = (rng.standard_normal((N, N)) for _ in range(3))
    uc, vc, pc = (rng.standard_normal((Nc, Nc)) for _ in range(3))
    assert np.allclose(d3.restrict_face(N, 0) @ _lift(u2, N),
                       _lift((mac.restrict_u(N) @ u2.ravel()).reshape(Nc, Nc), Nc))
    assert np.allclose(d3.restrict_face(N, 1) @ _lift(v2, N),
                       _lift((mac.restrict_v(N) @ v2.ravel()).reshape(Nc, Nc), Nc))
    assert np.allclose(d3.restrict_p(N) @ _lift(p2, N),
                       _lift((mac.restrict_p(N) @ p2.ravel()).reshape(Nc, Nc), Nc))
    assert np.allclose(d3.prolong_face(N, 0) @ _lift(uc, Nc),
                       _lift((mac.prolong_u(N) @ uc.ravel()).reshape(N, N), N))
    assert np.allclose(d3.prolong_face(N, 1) @ _lift(vc, Nc),
                       _lift((mac.prolong_v(N) @ vc.ravel()).reshape(N, N), N))
    assert np.allclose(d3.prolong_p(N) @ _lift(pc, Nc),
                       _lift((mac.prolong_p(N) @ pc.ravel()).reshape(N, N), N))
    # constants are kept by every transfer
    for a in range(3):
        assert np.allclose(d3.restrict_face(N, a) @ np.ones(N ** 3), 1.0)
        assert np.allclose(d3.prolong_face(N, a) @ np.ones(Nc ** 3), 1.0)


def test_axis_symmetry():
    """Rotating the axes maps face family a onto family a + 1: the gradient,
    divergence and transfers of family a + 1 act on rotated fields as those
    of family a on the original (catches an axis-specific index error in
    the family the 2-D reduction does not see)."""
    N = 8
    rng = np.random.default_rng(3)
    p = rng.standard_normal(N ** 3)
    f = rng.standard_normal(N ** 3)
    G, D = d3.gradient(N), d3.divergence(N)
    # rotation R: new (i', j', k') = (k, i, j)  i.e.  x' = z, y' = x, z' = y
    def R(x, n=N):
        a = x.reshape(n, n, n)                      # [k][j][i]
        out = np.empty_like(a)
        for k in range(n):
            for j in range(n):
                for i in range(n):
                    out[j, i, k] = a[k, j, i]       # new [k'=j][j'=i][i'=k]
        return out.reshape(-1)
    # family a along axis a becomes family along the rotated axis: x -> y, y -> z, z -> x
    for a, b in ((0, 1), (1, 2), (2, 0)):
        assert np.allclose(R(G[a] @ p), G[b] @ R(p))
        assert np.allclose(R(D[a] @ f), D[b] @ R(f))
        rf = d3.restrict_face(N, a) @ f
        assert np.allclose(R(rf, N // 2), d3.restrict_face(N, b) @ R(f))
        pc = rng.standard_normal((N // 2) ** 3)
        assert np.allclose(R(d3.prolong_face(N, a) @ pc), d3.prolong_face(N, b) @ R(pc, N // 2))


def test_delta_reduces_to_two_dimensions():
    """Summing the 3-D spread of a point over a z column times h gives the
    2-D spread (the 1-D kernels sum to one over the grid), for both kernels;
    the interpolation is h^3 times the transposed spread."""
    N = 16
    rng = np.random.default_rng(4)
    X = rng.uniform(0.0, 1.0, (5, 3))
    h = 1.0 / N
    for kind in (ib.DELTA_IB4, ib.DELTA_COS4):
        for a in (0, 1):
            S3 = d3.spread_matrix(X, N, a, kind).toarray().reshape(N, N * N, -1)
            S2 = ib.spread_matrix(X[:, :2], N, a, kind).toarray()
            assert np.allclose(S3.sum(axis=0) * h, S2)
        # w faces: summed over x they are the 2-D v faces of the (y, z) plane
        S3w = d3.spread_matrix(X, N, 2, kind).toarray().reshape(N, N, N, -1)     # [k][j][i]
        S2v = ib.spread_matrix(X[:, 1:], N, 1, kind).toarray().reshape(N, N, -1)  # [z][y]
        assert np.allclose(S3w.sum(axis=2) * h, S2v)
        S3 = d3.spread_matrix(X, N, 2, kind)
        assert np.allclose(np.asarray(S3.sum(axis=0)).ravel() * h ** 3, 1.0)
        assert np.allclose(d3.interp_matrix(X, N, 2, kind).toarray(), h ** 3 * S3.toarray().T)


def test_stokes_closed_forms():
    """Unsteady periodic Stokes (K = 0): a shear force (sin 2 pi y, 0, 0) on
    u faces gives u = f / (c + mu lambda), lambda = (4 / h^2) sin^2(pi h), and
    p = 0; a gradient force G phi gives u = 0 and p = phi (zero mean)."""
    N, c, mu = 8, 3.0, 0.7
    h = 1.0 / N
    A = d3.assemble(N, c, mu, None)
    n3 = N ** 3
    k, j, i = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    f = np.sin(2 * np.pi * (j + 0.5) * h).reshape(-1)
    b = np.zeros(4 * n3)
    b[:n3] = f
    x = d3.bordered_solve(A, b, N)
    lam = 4.0 / h ** 2 * np.sin(np.pi * h) ** 2
    assert np.allclose(x[:n3], f / (c + mu * lam), atol=1e-12)
    assert np.allclose(x[n3:], 0.0, atol=1e-12)
    phi = (np.cos(2 * np.pi * (i + 0.5) * h) * np.cos(2 * np.pi * (k + 0.5) * h)).reshape(-1)
    G = d3.gradient(N)
    b = np.concatenate([G[0] @ phi, G[1] @ phi, G[2] @ phi, np.zeros(n3)])
    x = d3.bordered_solve(A, b, N)
    assert np.allclose(x[:3 * n3], 0.0, atol=1e-11)
    assert np.allclose(x[3 * n3:], phi - phi.mean(), atol=1e-11)


def test_elastic_operator_structure():
    """M_a = -dt K S L J: symmetric positive semidefinite on the finest level
    (J = h^3 S^T, -L positive semidefinite), zero on constants (the delta
    interpolates constants exactly and L annihilates them), and the
    Galerkin coarse blocks keep constants in their kernel."""
    N = 16
    X, offs = ibgen.sphere_rings(N)
    lv = d3.hierarchy(N, 3, 1.0, 1.0, 0.01, X, offs, 1e3)
    for a in range(3):
        M = lv[0].Ms[a]
        assert abs(M - M.T).max() < 1e-9 * abs(M).max()
        ev = np.linalg.eigvalsh(M.toarray())
        assert ev.min() > -1e-9 * abs(ev).max()
        for l in range(3):
            Ml = lv[l].Ms[a]
            assert abs(Ml @ np.ones(Ml.shape[0])).max() < 1e-9 * abs(Ml).max()
    # Galerkin identity on one coarse block, entry by entry
    M1 = d3.restrict_face(N, 1) @ lv[0].Ms[1] @ d3.prolong_face(N, 1)
    assert abs(M1 - lv[1].Ms[1]).max() <= 1e-13 * abs(M1).max()


def test_box_solve_is_exact_and_sweep_reduces_error():
    """A box update zeroes the residual on that box's rows; checkerboard
    sweeps contract the error of a random start."""
    N = 8
    X, offs = ibgen.sphere_rings(N, r=0.3, spacing=0.5)
    lv = d3.hierarchy(N, 1, 1.0, 1.0, 0.02, X, offs, 200.0)   # dt K = 4 (coloured sweeps diverge near 40)
    A = lv[0].A
    sm = d3.BoxSmoother(A, N, 2)
    rng = np.random.default_rng(5)
    b = rng.standard_normal(A.shape[0])
    b[3 * N ** 3:] -= b[3 * N ** 3:].mean()          # consistent: continuity rows sum to zero
    w = rng.standard_normal(A.shape[0])
    w1 = sm.solve_box((1, 0, 1), w, b)
    d = d3.box_dofs((1, 0, 1), N, 2)
    assert np.abs((b - A @ w1)[d]).max() < 1e-10 * np.abs(b).max()
    other = np.setdiff1d(np.arange(A.shape[0]), d)
    assert np.array_equal(w1[other], w[other])
    x = d3.bordered_solve(A, b, N)
    e0 = w - x
    e0[3 * N ** 3:] -= e0[3 * N ** 3:].mean()
    wk = w
    for _ in range(4):
        wk = sm.sweep(wk, b)
    e = wk - x
    e[3 * N ** 3:] -= e[3 * N ** 3:].mean()
    assert np.linalg.norm(e) < 0.5 * np.linalg.norm(e0)


@pytest.mark.parametrize("n", [2, 4])
def test_vcycle_fgmres_reaches_rtol(n):
    """MG-preconditioned FGMRES on the 3-D level-0 system of the sphere's
    rings reaches rtol in the assembled operator, and the V-cycle
    alone contracts (spectral radius of I - M A estimated by power steps)."""
    N = 16
    levels = 3 if n == 2 else 2
    X, offs = ibgen.sphere_rings(N)
    lv = d3.hierarchy(N, levels, 1.0, 1.0, 0.01, X, offs, 1e3)    # dt K = 10
    V = d3.VCycle(lv, n, 1, 1)
    rng = np.random.default_rng(6)
    A = lv[0].A
    b = rng.standard_normal(A.shape[0])
    b[3 * N ** 3:] -= b[3 * N ** 3:].mean()
    res = krylov.fgmres(A, b, V, rtol=1e-10, maxit=60)
    assert res.converged
    assert np.linalg.norm(b - A @ res.x) <= 1e-10 * np.linalg.norm(b)
    e = rng.standard_normal(A.shape[0])
    for _ in range(6):
        e1 = e - V(A @ e)
        e1[3 * N ** 3:] -= e1[3 * N ** 3:].mean()
        ratio = np.linalg.norm(e1) / np.linalg.norm(e)
        e = e1
    assert ratio < 0.5


def test_step_without_structure_is_the_stokes_step():
    """K = 0: one implicit step of a shear mode is u^{n+1} = c u^n /
    (c + mu lambda) (closed form), the points move with the interpolated
    velocity."""
    N, rho, mu, dt = 8, 1.0, 1.0, 0.01
    h = 1.0 / N
    k, j, i = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    u0 = np.sin(2 * np.pi * (k + 0.5) * h).reshape(-1)           # u varies along z
    X, offs = ibgen.sphere_rings(N, r=0.3, spacing=1.0)
    un, p, Xn, res = d3.step([u0, np.zeros(N ** 3), np.zeros(N ** 3)], X, offs, N, 2, rho, mu, dt, 0.0, n=2)
    c = rho / dt
    lam = 4.0 / h ** 2 * np.sin(np.pi * h) ** 2
    assert np.allclose(un[0], c * u0 / (c + mu * lam), atol=1e-9)
    assert np.allclose(un[1], 0.0, atol=1e-9) and np.allclose(un[2], 0.0, atol=1e-9)
    U = d3.interp(X, un)
    assert np.allclose(Xn, X + dt * U)
    assert np.allclose(U[:, 1:], 0.0, atol=1e-9)


def test_rings_generator_inputs():
    X, offs = ibgen.sphere_rings(32)
    assert X.shape == (offs[-1], 3) and offs[0] == 0 and np.all(np.diff(offs) >= 8)
    X2, _ = ibgen.sphere_rings(32)
    assert np.array_equal(X, X2)
