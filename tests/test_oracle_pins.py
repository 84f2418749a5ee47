"""Pins of the CPU oracle against what the mathematics fixes.

Each test ties one oracle function to a closed form, an invariant, a
textbook special case or brute force on a tiny input, chosen so that a
dropped term, a wrong sign or index, or a transposed operand fails at least
one of them.  No value here comes from the GPU path.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import ibgen
from oracle import mac, ib, system, smoother, mg, krylov, stokes_fft, dtexp, step

rng = np.random.default_rng(2024)


# ---------------------------------------------------------------- delta kernels (Sec. 2.2)

@pytest.mark.parametrize("kind", [ib.DELTA_IB4, ib.DELTA_COS4])
def test_delta_moment_identities(kind):
    """sum_i phi(r - i) = 1, even and odd sums = 1/2, sum phi^2 = 3/8."""
    r = np.linspace(0.0, 1.0, 2001)
    ii = np.arange(-3, 4)[:, None]
    w = ib.phi(r[None, :] - ii, kind)
    assert np.max(np.abs(w.sum(0) - 1.0)) < 1e-14
    even = w[(ii[:, 0] % 2) == 0].sum(0)
    assert np.max(np.abs(even - 0.5)) < 1e-14
    assert np.max(np.abs((w**2).sum(0) - 3.0 / 8.0)) < 1e-14
    # support: |r| < 2
    assert ib.phi(2.0, kind) == 0.0 and ib.phi(-2.5, kind) == 0.0
    assert ib.phi(0.0, kind) > 0.0


def test_delta_first_moment():
    """IB4 has zero first moment; the cosine kernel does not (max ~0.021)."""
    r = np.linspace(0.0, 1.0, 2001)
    ii = np.arange(-3, 4)[:, None]
    m_ib4 = ((r[None, :] - ii) * ib.phi(r[None, :] - ii, ib.DELTA_IB4)).sum(0)
    m_cos = ((r[None, :] - ii) * ib.phi(r[None, :] - ii, ib.DELTA_COS4)).sum(0)
    assert np.max(np.abs(m_ib4)) < 1e-14
    assert 0.015 < np.max(np.abs(m_cos)) < 0.03


def test_delta_ib4_closed_values():
    """Peskin's kernel: phi(0) = 1/2, phi(1) = 1/4, phi(1/2) = (2 + sqrt 2)/8."""
    assert abs(ib.phi(0.0) - 0.5) < 1e-16
    assert abs(ib.phi(1.0) - 0.25) < 1e-16
    assert abs(ib.phi(0.5) - (2.0 + np.sqrt(2.0)) / 8.0) < 1e-15
    assert abs(ib.phi(1.0, ib.DELTA_COS4) - 0.25) < 1e-16


# ---------------------------------------------------------------- MAC operators (Sec. 2.2)

@pytest.mark.parametrize("N", [4, 8, 16])
def test_mac_div_is_minus_grad_transpose(N):
    Gx, Gy = mac.gradient(N)
    Dx, Dy = mac.divergence(N)
    assert abs(Dx + Gx.T).max() < 1e-12 * N
    assert abs(Dy + Gy.T).max() < 1e-12 * N


def test_mac_div_grad_is_cell_laplacian():
    N = 16
    Gx, Gy = mac.gradient(N)
    Dx, Dy = mac.divergence(N)
    assert abs(Dx @ Gx + Dy @ Gy - mac.laplacian(N)).max() < 1e-9


def test_mac_div_curl_zero():
    """A discrete stream function psi on nodes gives u = (psi_{i,j+1} - psi_{i,j})/h,
    v = -(psi_{i+1,j} - psi_{i,j})/h with D(u, v) = 0 exactly."""
    N = 16
    h = 1.0 / N
    psi = rng.standard_normal((N, N))  # psi[j][i] at node (i h, j h)
    u = (np.roll(psi, -1, axis=0) - psi) / h
    v = -(np.roll(psi, -1, axis=1) - psi) / h
    Dx, Dy = mac.divergence(N)
    div = Dx @ u.reshape(-1) + Dy @ v.reshape(-1)
    assert np.max(np.abs(div)) < 1e-11 * np.max(np.abs(u))


def test_mac_laplacian_fourier_symbol():
    N = 16
    h = 1.0 / N
    kx, ky = 3, 5
    j, i = np.mgrid[0:N, 0:N]
    tx, ty = 2 * np.pi * kx / N, 2 * np.pi * ky / N
    e = np.exp(1j * (tx * i + ty * j)).reshape(-1)
    lam = -(4.0 / h**2) * (np.sin(tx / 2) ** 2 + np.sin(ty / 2) ** 2)
    Le = mac.laplacian(N) @ e
    assert np.max(np.abs(Le - lam * e)) < 1e-10 * abs(lam)


# ---------------------------------------------------------------- transfers (Sec. 3.1)

@pytest.mark.parametrize("N", [8, 16])
def test_transfer_identities(N):
    Rp, Pp = mac.restrict_p(N), mac.prolong_p(N)
    assert abs(Rp @ Pp - sp.identity((N // 2) ** 2)).max() < 1e-15
    for R in (mac.restrict_u(N), mac.restrict_v(N), Rp):
        assert np.allclose(np.asarray(R.sum(1)).ravel(), 1.0, atol=1e-15)
    for P in (mac.prolong_u(N), mac.prolong_v(N), Pp):
        assert np.allclose(P @ np.ones((N // 2) ** 2), 1.0, atol=1e-15)


def test_prolong_u_bilinear_exact_on_linear_fields():
    """P_u reproduces a field linear in x and y at fine faces whose bilinear
    stencil does not wrap (u at (i h, (j + 1/2) h))."""
    N = 16
    Nc = N // 2
    H = 2.0 / N
    J, I = np.mgrid[0:Nc, 0:Nc]
    f = lambda x, y: 0.3 + 1.7 * x - 2.1 * y
    uc = f(I * H, (J + 0.5) * H).reshape(-1)
    uf = (mac.prolong_u(N) @ uc).reshape(N, N)
    j, i = np.mgrid[0:N, 0:N]
    ex = f(i / N, (j + 0.5) / N)
    inner = (i < N - 2) & (j >= 1) & (j < N - 1)
    assert np.max(np.abs(uf - ex)[inner]) < 1e-13
    vc = f((I + 0.5) * H, J * H).reshape(-1)
    vf = (mac.prolong_v(N) @ vc).reshape(N, N)
    exv = f((i + 0.5) / N, j / N)
    innerv = (j < N - 2) & (i >= 1) & (i < N - 1)
    assert np.max(np.abs(vf - exv)[innerv]) < 1e-13


def test_restrict_u_full_weighting_weights():
    """R_u rows: weights 1/8 * [1 2 1] on fine rows 2J and 2J+1 (Sec. 3.1)."""
    N = 8
    R = mac.restrict_u(N).toarray()
    row = R[mac.fidx(1, 1, N // 2)]
    expect = np.zeros(N * N)
    for d, wd in ((-1, 1), (0, 2), (1, 1)):
        for jj in (2, 3):
            expect[mac.fidx(2 + d, jj, N)] = wd / 8
    assert np.array_equal(row, expect)


def _swap_axes(N):
    """Permutation T with (T f)[j][i] = f[i][j] on an N x N field: the
    reflection x <-> y of the periodic square.  It maps the v faces
    ((i + 1/2) h, j h) onto the u faces (j h, (i + 1/2) h) and back, so the
    MAC discretisation is invariant under it with u and v exchanged."""
    idx = np.arange(N * N).reshape(N, N).T.ravel()
    return sp.csr_matrix((np.ones(N * N), (np.arange(N * N), idx)), shape=(N * N, N * N))


@pytest.mark.parametrize("N", [8, 16])
def test_restrict_v_is_the_reflection_of_restrict_u(N):
    """Sec. 3.1 gives R_v as R_u with the roles of x and y exchanged: under
    the reflection x <-> y, restricting a v field equals restricting the
    reflected field as u and reflecting back.  Together with the explicit
    R_u weights above this fixes every weight of R_v; R_u's own rule applied
    to v faces fails it."""
    T, Tc = _swap_axes(N), _swap_axes(N // 2)
    assert abs(mac.restrict_v(N) - Tc @ mac.restrict_u(N) @ T).max() == 0.0
    assert abs(mac.prolong_v(N) - T @ mac.prolong_u(N) @ Tc).max() == 0.0
    assert abs(mac.restrict_u(N) - Tc @ mac.restrict_u(N) @ T).max() > 0.1   # u's rule is not symmetric


@pytest.mark.parametrize("comp", ["u", "v"])
def test_restriction_exact_on_linear_fields(comp):
    """Each face restriction is a weighted mean of fine faces whose centroid is
    the coarse face centre, so a field linear in x and y, sampled at the fine
    faces of its family, restricts to its values at the coarse faces (away
    from the periodic seam).  A rule centred on the wrong face family (R_u's
    stencil on v faces, or a shifted row pair) misses the coarse centre."""
    N = 16
    Nc, h, H = N // 2, 1.0 / N, 2.0 / N
    f = lambda x, y: 0.3 + 1.7 * x - 2.1 * y
    j, i = np.mgrid[0:N, 0:N]
    J, I = np.mgrid[0:Nc, 0:Nc]
    if comp == "u":
        R = mac.restrict_u(N)
        fine = f(i * h, (j + 0.5) * h)
        ex = f(I * H, (J + 0.5) * H)
        inner = (I >= 1) & (I < Nc - 1)
    else:
        R = mac.restrict_v(N)
        fine = f((i + 0.5) * h, j * h)
        ex = f((I + 0.5) * H, J * H)
        inner = (J >= 1) & (J < Nc - 1)
    out = (R @ fine.ravel()).reshape(Nc, Nc)
    assert np.max(np.abs(out - ex)[inner]) < 1e-13


# ---------------------------------------------------------------- spreading / interpolation

def _pts(M=30, N=16, seed=3):
    r = np.random.default_rng(seed)
    return r.uniform(-0.2, 1.2, size=(M, 2))   # unwrapped positions on purpose


@pytest.mark.parametrize("kind", [ib.DELTA_IB4, ib.DELTA_COS4])
def test_spread_window_equals_brute_force(kind):
    N = 16
    X = _pts(N=N)
    for comp in (0, 1):
        A = ib.spread_matrix(X, N, comp, kind)
        B = ib.spread_matrix(X, N, comp, kind, brute=True)
        assert abs(A - B).max() < 1e-14 * N * N


@pytest.mark.parametrize("kind", [ib.DELTA_IB4, ib.DELTA_COS4])
def test_spread_interp_adjoint_and_partition(kind):
    N = 16
    X = _pts(N=N)
    G = rng.standard_normal(X.shape)
    u = rng.standard_normal((N, N))
    v = rng.standard_normal((N, N))
    fu, fv = ib.spread(X, G, N, kind)
    U = ib.interp(X, u, v, kind)
    h2 = 1.0 / N**2
    lhs = h2 * (np.sum(fu * u) + np.sum(fv * v))
    rhs = np.sum(G * U)
    assert abs(lhs - rhs) < 1e-13 * max(1.0, abs(rhs))
    assert abs(h2 * fu.sum() - G[:, 0].sum()) < 1e-13
    assert abs(h2 * fv.sum() - G[:, 1].sum()) < 1e-13
    c = ib.interp(X, np.full((N, N), 2.5), np.full((N, N), -1.5), kind)
    assert np.max(np.abs(c - [2.5, -1.5])) < 1e-14


def test_interp_linear_exact_ib4():
    """IB4 interpolates linear fields exactly (zero first moment); the field
    is linear over the 4x4 support of a point away from the periodic seam."""
    N = 32
    X = np.random.default_rng(1).uniform(0.3, 0.7, size=(20, 2))
    j, i = np.mgrid[0:N, 0:N]
    f = lambda x, y: 1.0 + 2.0 * x - 3.0 * y
    u = f(i / N, (j + 0.5) / N)
    v = f((i + 0.5) / N, j / N)
    U = ib.interp(X, u, v, ib.DELTA_IB4)
    ex = f(X[:, 0], X[:, 1])
    assert np.max(np.abs(U[:, 0] - ex)) < 1e-13
    assert np.max(np.abs(U[:, 1] - ex)) < 1e-13


def test_spread_first_moment_ib4():
    """Spread force carries the point's first moment (IB4)."""
    N = 32
    X = np.array([[0.43, 0.57]])
    G = np.array([[1.0, 0.0]])
    fu, _ = ib.spread(X, G, N, ib.DELTA_IB4)
    j, i = np.mgrid[0:N, 0:N]
    h2 = 1.0 / N**2
    assert abs(h2 * np.sum(fu * (i / N)) - X[0, 0]) < 1e-14
    assert abs(h2 * np.sum(fu * ((j + 0.5) / N)) - X[0, 1]) < 1e-14


def test_fiber_force_conserves_force_and_torque():
    w = ibgen.small_case(N=16, M=50, n_fibers=2)
    G = ib.fiber_force(w.X, w.fiber_offsets, 7.0)
    assert np.max(np.abs(G.sum(0))) < 1e-12
    torque = np.sum(w.X[:, 0] * G[:, 1] - w.X[:, 1] * G[:, 0])
    assert abs(torque) < 1e-11
    # second difference of a closed polygon: the hand value at one node
    X = w.X
    k = 3
    assert np.allclose(G[k], 7.0 * (X[k - 1] - 2 * X[k] + X[k + 1]), rtol=0, atol=1e-13)


# ---------------------------------------------------------------- system and coarse operators

def _small(N=16, K=2e3, levels=3, seed=5, dt=None):
    w = ibgen.small_case(N=N, M=48, K=K, seed=seed, levels=levels)
    if dt is None:
        dt = 5.0 * dtexp.dt_explicit(w.X, w.fiber_offsets, N, K)
    lv = system.hierarchy(N, levels, 1.0, 1.0, dt, w.X, w.fiber_offsets, K)
    return w, dt, lv


def test_level0_symmetric_with_pressure_nullspace():
    w, dt, lv = _small()
    A = lv[0].A
    assert abs(A - A.T).max() < 1e-9 * abs(A).max()
    N = lv[0].N
    e = np.zeros(3 * N * N)
    e[2 * N * N:] = 1.0
    assert np.max(np.abs(A @ e)) < 1e-9
    # M_0 is symmetric positive semidefinite
    Mu = lv[0].M_u.toarray()
    ev = np.linalg.eigvalsh(0.5 * (Mu + Mu.T))
    assert ev.min() > -1e-9 * ev.max() and ev.max() > 0


def test_galerkin_kills_constants_all_levels():
    """M_l 1 = 0 and 1^T M_l = 0 on every level (interpolation of constants is
    exact, L 1 = 0, R and P preserve constants)."""
    w, dt, lv = _small(levels=3)
    for l in lv:
        n = l.N * l.N
        for M in (l.M_u, l.M_v):
            assert np.max(np.abs(M @ np.ones(n))) < 1e-10 * abs(M).max()
            assert np.max(np.abs(M.T @ np.ones(n))) < 1e-10 * abs(M).max()


def test_galerkin_footprint_is_local():
    """Coarse elasticity rows are nonzero only within a few coarse cells of
    the structure."""
    w, dt, lv = _small(N=32, levels=3)
    for l in lv:
        N = l.N
        rows = np.unique(l.M_u.nonzero()[0])
        i, j = rows % N, rows // N
        x, y = i / N, (j + 0.5) / N
        d = np.min(np.hypot(*[np.minimum(np.abs(a[:, None] - b[None, :]),
                                          1 - np.abs(a[:, None] - b[None, :]))
                              for a, b in ((x, w.X[:, 0] % 1), (y, w.X[:, 1] % 1))]), axis=1)
        assert d.max() < 4.5 / N


def test_coarse_stokes_rediscretised():
    """With K = 0 every level operator equals the Stokes operator assembled
    directly on that grid (hybrid coarsening, Sec. 3.2)."""
    lv = system.hierarchy(16, 3, 1.0, 1.0, 0.1)
    for l in lv:
        Z = sp.csr_matrix((l.N**2, l.N**2))
        assert abs(l.A - system.assemble(l.N, 10.0, 1.0, Z, Z)).max() < 1e-12 * abs(l.A).max()


# ---------------------------------------------------------------- box relaxation (Sec. 5, 6)

def test_box_dof_count():
    for n, ndof in ((1, 5), (2, 16), (4, 56)):
        assert len(smoother.box_dofs(0, 0, 16, n)) == ndof
        assert len(set(smoother.box_dofs(1, 1, 16, n))) == ndof


def test_same_colour_boxes_disjoint():
    N, n = 16, 4
    for cx, cy in smoother.COLOURS:
        seen = set()
        for by in range(cy, N // n, 2):
            for bx in range(cx, N // n, 2):
                d = set(smoother.box_dofs(bx, by, N, n))
                assert not (seen & d)
                seen |= d
    for n in (1, 2, 4):          # checkerboard: diagonal neighbours share no unknown
        for par in (0, 1):
            seen = set()
            for by in range(N // n):
                for bx in range(N // n):
                    if (bx + by) % 2 != par:
                        continue
                    d = set(smoother.box_dofs(bx, by, N, n))
                    assert not (seen & d)
                    seen |= d


def test_colour_orders_cover_every_unknown():
    """Each sweep ordering updates every unknown at least once."""
    N, n = 16, 4
    allu = set(range(3 * N * N))
    for par_sets in ([[(bx, by) for by in range(4) for bx in range(4) if (bx + by) % 2 == p] for p in (0, 1)],):
        cov = set()
        for boxes in par_sets:
            for bx, by in boxes:
                cov |= set(smoother.box_dofs(bx, by, N, n))
        assert cov == allu


def test_paper_mode_box_residual_zero_after_update():
    w, dt, lv = _small(N=16)
    sm = smoother.BoxSmoother(lv[0].A, 16, 4)
    b = rng.standard_normal(3 * 256)
    x = rng.standard_normal(3 * 256)
    A = lv[0].A
    # one box update by hand through the smoother's LU
    d = sm.dofs[(1, 2)]
    import scipy.linalg as sla
    x2 = x.copy()
    x2[d] += sla.lu_solve(sm.lu[(1, 2)], (b - A @ x)[d])
    r = (b - A @ x2)[d]
    assert np.max(np.abs(r)) < 1e-11 * np.max(np.abs(b - A @ x))


@pytest.mark.parametrize("mode", ["paper", "colour", "colour2"])
def test_damped_box_correction(mode):
    """A right-hand side carried only by unknowns that belong to the last box
    alone (its interior pressures) leaves every earlier box with a zero
    residual, so one damped sweep updates that box once: the iterate is omega
    times the undamped one and the box's residual drops to (1 - omega) of
    the right-hand side there, for omega = 0.6."""
    N, n = 8, 4
    lv = system.hierarchy(N, 2, 1.0, 1.0, 0.05)
    A = lv[0].A
    sm = smoother.BoxSmoother(A, N, n)
    b = np.zeros(3 * N * N)
    last = (1, 0) if mode == "colour2" else (1, 1)     # a box of the sweep's last colour
    d = sm.dofs[last]
    interior = [k for k in d if k >= 2 * N * N]          # the box's pressures
    b[interior] = rng.standard_normal(len(interior))
    x1 = sm.sweep(np.zeros_like(b), b, mode)
    xw = sm.sweep(np.zeros_like(b), b, mode, omega=0.6)
    assert np.max(np.abs(xw - 0.6 * x1)) < 1e-14 * np.max(np.abs(x1))
    r = (b - A @ xw)[d]
    assert np.max(np.abs(r - 0.4 * b[d])) < 1e-12 * np.max(np.abs(b))


@pytest.mark.parametrize("n", [2, 4])
def test_colour_phase_exact_without_elasticity(n):
    """Without the elastic term, same-colour boxes do not couple for n >= 2,
    so after a colour phase the residual vanishes on every box of that colour."""
    N = 16
    lv = system.hierarchy(N, 2, 1.0, 1.0, 0.05)
    A = lv[0].A
    sm = smoother.BoxSmoother(A, N, n)
    b = rng.standard_normal(3 * N * N)
    x = np.zeros(3 * N * N)
    import scipy.linalg as sla
    r = b - A @ x
    for by in range(0, N // n, 2):
        for bx in range(0, N // n, 2):
            d = sm.dofs[(bx, by)]
            x[d] += sla.lu_solve(sm.lu[(bx, by)], r[d])
    r2 = b - A @ x
    for by in range(0, N // n, 2):
        for bx in range(0, N // n, 2):
            assert np.max(np.abs(r2[sm.dofs[(bx, by)]])) < 1e-10 * np.max(np.abs(b))


@pytest.mark.parametrize("n,mode", [(1, "colour2"), (2, "colour"), (4, "colour2"), (4, "colour")])
def test_shared_block_sweep_equals_per_box_sweep(n, mode):
    """Without elastic rows the one-factorisation sweep reproduces the
    per-box sweep (each box's own block and LU) on random data, and the box
    table lists each box's unknowns in box_dofs order."""
    N = 16
    lv = system.hierarchy(N, 2, 1.0, 1.0, 0.05)
    A = lv[0].A
    sm = smoother.BoxSmoother(A, N, n)
    D = smoother.box_dof_table(N, n)
    for by in range(N // n):
        for bx in range(N // n):
            assert np.array_equal(D[by * (N // n) + bx], sm.dofs[(bx, by)])
    b = rng.standard_normal(3 * N * N)
    x = rng.standard_normal(3 * N * N)
    ref = sm.sweep(x, b, mode)
    got = smoother.sweep_shared(A, N, n, x, b, mode)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


def test_box_matrix_is_restriction_of_operator():
    """A_box entries equal the level operator's entries (spot check against
    the stencil: diagonal c + 4 mu / h^2 plus the elastic diagonal)."""
    w, dt, lv = _small(N=16)
    sm = smoother.BoxSmoother(lv[0].A, 16, 4)
    Ab = sm.box_matrix(0, 0)
    c = 1.0 / dt
    h = 1.0 / 16
    d = sm.dofs[(0, 0)]
    Mu = lv[0].M_u.toarray()
    for a in range(20):  # u rows
        assert abs(Ab[a, a] - (c + 4.0 / h**2 + Mu[d[a], d[a]])) < 1e-9 * abs(Ab[a, a])


# ---------------------------------------------------------------- coarse solve, V-cycle

def test_coarse_bordered_solve():
    w, dt, lv = _small(N=16, levels=3)
    V = mg.VCycle(lv, 4, 1, 1)
    Nc = lv[-1].N
    b = rng.standard_normal(3 * Nc * Nc)
    b[2 * Nc * Nc:] -= b[2 * Nc * Nc:].mean()
    x = V.coarse_solve(b)
    assert np.max(np.abs(lv[-1].A @ x - b)) < 1e-11 * np.max(np.abs(b))
    assert abs(x[2 * Nc * Nc:].mean()) < 1e-13


def test_vcycle_box_order_per_level():
    """A box order given per level applies level by level: one order for every
    level repeats the single-order V-cycle bit for bit, and a mixed one equals
    the V-cycle assembled from the two by hand (level 0's sweeps of the first
    order around a coarse correction whose sweeps take the second)."""
    w, dt, lv = _small(N=16, levels=3)
    r = rng.standard_normal(3 * 256)
    r[512:] -= r[512:].mean()
    a = mg.VCycle(lv, 2, 1, 1, "colour")(r)
    b = mg.VCycle(lv, 2, 1, 1, ["colour", "colour"])(r)
    assert np.array_equal(a, b)
    mixed = mg.VCycle(lv, 2, 1, 1, ["colour", "colour2"])
    one = mg.VCycle(lv, 2, 1, 1, "colour")
    two = mg.VCycle(lv, 2, 1, 1, "colour2")
    w0 = one.smoothers[0].sweep(np.zeros_like(r), r, "colour")
    r1 = lv[0].R @ (r - lv[0].A @ w0)
    e1 = two.mgv(np.zeros_like(r1), r1, 1)
    ref = one.smoothers[0].sweep(w0 + lv[0].P @ e1, r, "colour")
    assert np.array_equal(mixed(r), ref)
    with pytest.raises(ValueError):
        mg.VCycle(lv, 2, 1, 1, ["colour"])


@pytest.mark.parametrize("mode", ["colour2", "colour", "paper"])
def test_mg_iteration_matrix_contracts(mode):
    """Spectral radius of the V-cycle iteration matrix on the mean-zero
    pressure space is < 1; at K = 0 it is of the size the paper reports for
    its (Dirichlet) Stokes case, ~0.2-0.3 (parity unpinned for periodic)."""
    N = 16
    lv = system.hierarchy(N, 2, 1.0, 1.0, 1e3)   # nearly steady Stokes, K = 0
    V = mg.VCycle(lv, 1, 1, 1, mode)
    n = 3 * N * N
    A = lv[0].A
    T = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        T[:, k] = V.mgv(e, np.zeros(n))
    # project out the constant-pressure mode
    q = np.zeros(n)
    q[2 * N * N:] = 1.0 / N
    Pm = np.eye(n) - np.outer(q, q)
    ev = np.abs(np.linalg.eigvals(Pm @ T @ Pm))
    rho = np.sort(ev)[-1]
    assert rho < 0.6
    assert 0.05 < rho


# ---------------------------------------------------------------- FGMRES and full solves

def test_fgmres_matches_dense_direct_stiff():
    """Tiny stiff problem: MG-FGMRES at rtol 1e-13 against a bordered dense LU."""
    for N, K in ((8, 1e5), (16, 1e6)):
        w = ibgen.small_case(N=N, M=24 if N == 8 else 48, K=K, seed=11, levels=2)
        dt = 50 * dtexp.dt_explicit(w.X, w.fiber_offsets, N, K)
        lv, V = step.build(N, 2, 1.0, 1.0, dt, w.X, w.fiber_offsets, K, box=2, nu1=1, nu2=1)
        b = system.rhs(rng.standard_normal((N, N)), rng.standard_normal((N, N)), w.X,
                       w.fiber_offsets, K, dt, 1.0)
        res = krylov.fgmres(lv[0].A, b, V, rtol=1e-13, maxit=100)
        assert res.converged
        A = lv[0].A.toarray()
        n = A.shape[0]
        B = np.zeros((n + 1, n + 1))
        B[:n, :n] = A
        B[2 * N * N:n, n] = 1
        B[n, 2 * N * N:n] = 1
        xd = np.linalg.solve(B, np.concatenate([b, [0]]))[:n]
        x = res.x.copy()
        x[2 * N * N:] -= x[2 * N * N:].mean()
        kappa = np.linalg.cond(B)
        err = np.linalg.norm(x - xd) / np.linalg.norm(xd)
        assert err < max(1e-10, 1e-13 * kappa)


def test_fgmres_mgs_and_cgs2_agree():
    w, dt, lv = _small(N=16)
    V = mg.VCycle(lv, 4, 1, 1)
    b = system.rhs(np.zeros((16, 16)), np.zeros((16, 16)), w.X, w.fiber_offsets, w.K, dt, 1.0)
    r1 = krylov.fgmres(lv[0].A, b, V, rtol=1e-10, orth="mgs")
    r2 = krylov.fgmres(lv[0].A, b, V, rtol=1e-10, orth="cgs2")
    assert abs(r1.iters - r2.iters) <= 1
    assert r1.rel_resid_true < 1e-10 and r2.rel_resid_true < 1e-10


def test_fgmres_dcgs2_equals_cgs2():
    """The delayed second Gram-Schmidt pass is a reordering of CGS2: after the
    same number of iterations the iterates agree to rounding (stiff 16^2 case,
    500 x dt_exp, pressure compared without its mean), converged solves take
    the same count, and so do restarted ones."""
    N, K = 16, 1e6
    w = ibgen.small_case(N=N, M=48, K=K, seed=11, levels=2)
    dt = 500 * dtexp.dt_explicit(w.X, w.fiber_offsets, N, K)
    lv, V = step.build(N, 3, 1.0, 1.0, dt, w.X, w.fiber_offsets, K, box=2, nu1=1, nu2=1)
    b = system.rhs(rng.standard_normal((N, N)), rng.standard_normal((N, N)), w.X, w.fiber_offsets, K, dt, 1.0)
    n2 = 2 * N * N
    for k in (1, 2, 9, 30):
        r1 = krylov.fgmres(lv[0].A, b, V, rtol=1e-30, maxit=k, orth="cgs2")
        r2 = krylov.fgmres(lv[0].A, b, V, rtol=1e-30, maxit=k, orth="dcgs2")
        assert r1.iters == r2.iters == k
        x1, x2 = r1.x.copy(), r2.x.copy()
        x1[n2:] -= x1[n2:].mean()
        x2[n2:] -= x2[n2:].mean()
        assert np.linalg.norm(x1 - x2) <= 1e-10 * np.linalg.norm(x1)
        assert np.allclose(r1.history, r2.history, rtol=1e-8, atol=0)
    r1 = krylov.fgmres(lv[0].A, b, V, rtol=1e-10, maxit=200, orth="cgs2")
    r2 = krylov.fgmres(lv[0].A, b, V, rtol=1e-10, maxit=200, orth="dcgs2")
    assert r1.converged and r2.converged and r1.iters == r2.iters
    assert r2.rel_resid_true <= 1e-10
    r1 = krylov.fgmres(lv[0].A, b, V, rtol=1e-6, maxit=400, restart=20, orth="cgs2")
    r2 = krylov.fgmres(lv[0].A, b, V, rtol=1e-6, maxit=400, restart=20, orth="dcgs2")
    assert r1.iters == r2.iters and abs(r1.rel_resid_true - r2.rel_resid_true) <= 1e-6 * r1.rel_resid_true


def test_fgmres_zero_rhs_and_maxit():
    lv = system.hierarchy(8, 2, 1.0, 1.0, 0.1)
    V = mg.VCycle(lv, 2, 1, 1)
    res = krylov.fgmres(lv[0].A, np.zeros(192), V)
    assert res.iters == 0 and res.converged and np.all(res.x == 0)
    b = rng.standard_normal(192)
    b[128:] -= b[128:].mean()
    res = krylov.fgmres(lv[0].A, b, V, rtol=1e-30, maxit=2)
    assert res.iters == 2 and not res.converged


def test_stokes_mg_matches_fft():
    """K = 0: periodic unsteady Stokes is diagonalised by the DFT; MG-FGMRES
    must match the spectral solution."""
    N = 32
    c, mu = 7.0, 1.0
    fu = rng.standard_normal((N, N))
    fv = rng.standard_normal((N, N))
    uf, vf, pf = stokes_fft.solve(fu, fv, c, mu)
    lv = system.hierarchy(N, 3, 1.0, mu, 1.0 / c)
    V = mg.VCycle(lv, 4, 2, 2)
    b = np.concatenate([fu.ravel(), fv.ravel(), np.zeros(N * N)])
    res = krylov.fgmres(lv[0].A, b, V, rtol=1e-13)
    u, v, p = system.split(res.x, N)
    ref = np.concatenate([uf.ravel(), vf.ravel(), pf.ravel()])
    got = np.concatenate([u.ravel(), v.ravel(), (p - p.mean()).ravel()])
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-9


def test_fft_stokes_satisfies_assembled_operator():
    N = 16
    c = 3.0
    fu = rng.standard_normal((N, N))
    fv = rng.standard_normal((N, N))
    u, v, p = stokes_fft.solve(fu, fv, c, 1.0)
    A = system.hierarchy(N, 1, 1.0, 1.0, 1.0 / c)[0].A
    w = np.concatenate([u.ravel(), v.ravel(), p.ravel()])
    b = np.concatenate([fu.ravel(), fv.ravel(), np.zeros(N * N)])
    assert np.max(np.abs(A @ w - b)) < 1e-11 * np.max(np.abs(b))


@pytest.mark.parametrize("N", [16, 32])
def test_manufactured_solution_second_order(N):
    """Continuum periodic Stokes solution (stream function sin sin, pressure
    cos cos) sampled at face centres; discretisation error O(h^2)."""
    errs = []
    for n in (N, 2 * N):
        h = 1.0 / n
        c, mu = 2.0, 1.0
        j, i = np.mgrid[0:n, 0:n]
        k = 2 * np.pi
        U = lambda x, y: np.sin(k * x) * np.cos(k * y)
        Vf = lambda x, y: -np.cos(k * x) * np.sin(k * y)
        P = lambda x, y: np.cos(k * x) * np.cos(k * y)
        # f = c u - mu Lap u + grad p, Lap u = -2 k^2 u
        fu = lambda x, y: (c + 2 * mu * k * k) * U(x, y) - k * np.sin(k * x) * np.cos(k * y)
        fv = lambda x, y: (c + 2 * mu * k * k) * Vf(x, y) - k * np.cos(k * x) * np.sin(k * y)
        xu, yu = i * h, (j + 0.5) * h
        xv, yv = (i + 0.5) * h, j * h
        lv = system.hierarchy(n, 3, 1.0, mu, 1.0 / c)
        V = mg.VCycle(lv, 4, 2, 2)
        b = np.concatenate([fu(xu, yu).ravel(), fv(xv, yv).ravel(), np.zeros(n * n)])
        res = krylov.fgmres(lv[0].A, b, V, rtol=1e-12)
        u, v, p = system.split(res.x, n)
        pe = P((i + 0.5) * h, (j + 0.5) * h)
        e = max(np.max(np.abs(u - U(xu, yu))), np.max(np.abs(v - Vf(xv, yv))),
                np.max(np.abs((p - p.mean()) - pe)))
        errs.append(e)
    ratio = errs[0] / errs[1]
    assert 3.5 < ratio < 4.5


# ---------------------------------------------------------------- explicit limit

def test_lambda_max_lanczos_matches_dense():
    w = ibgen.small_case(N=16, M=40, seed=9)
    a = dtexp.lambda_max(w.X, w.fiber_offsets, 16)
    b = dtexp.lambda_max_dense(w.X, w.fiber_offsets, 16)
    assert abs(a - b) < 1e-8 * b


def test_explicit_limit_is_a_stability_boundary():
    """Forward Euler on dX/dt = K S^* L_0^{-1} S L X is stable just below
    dt_exp and unstable just above (Sec. 4.1)."""
    w = ibgen.small_case(N=16, M=40, seed=9)
    K = 1e3
    dt = dtexp.dt_explicit(w.X, w.fiber_offsets, 16, K)
    A = dtexp.stokes_coupling(w.X, 16)
    L = ib.fiber_laplacian(w.fiber_offsets, w.M)

    def grow(dtf):
        x = np.random.default_rng(0).standard_normal((w.M, 2))
        for _ in range(400):
            x = x + dtf * K * A(np.stack([L @ x[:, 0], L @ x[:, 1]], 1))
        return np.linalg.norm(x)
    assert grow(0.98 * dt) < 1e3
    assert grow(1.05 * dt) > 1e3


# ---------------------------------------------------------------- time step invariants

def _energy(u, v, X, offs, K, rho, h):
    L = ib.fiber_laplacian(offs, X.shape[0])
    e_el = -0.5 * K * (np.sum(X[:, 0] * (L @ X[:, 0])) + np.sum(X[:, 1] * (L @ X[:, 1])))
    return 0.5 * rho * h * h * (np.sum(u * u) + np.sum(v * v)) + e_el


def test_step_energy_identity_and_momentum():
    """Discrete energy identity of the lagged implicit scheme (unconditional
    stability, Sec. 2.3.2):
    E' - E = dt mu h^2 (u', Lap u') - rho/2 h^2 |u' - u|^2
             - K/2 (d, -L d) + dt h^2 (g, u'),  d = X' - X;
    and rho (mean u' - mean u) / dt = mean g."""
    N = 16
    w = ibgen.small_case(N=N, M=48, K=3e3, seed=4, with_force=True)
    dt = 20 * dtexp.dt_explicit(w.X, w.fiber_offsets, N, w.K)
    h = 1.0 / N
    r0 = np.random.default_rng(1)
    u = 0.1 * r0.standard_normal((N, N))
    v = 0.1 * r0.standard_normal((N, N))
    p = np.zeros((N, N))
    s = step.step(u, v, p, w.X, w.fiber_offsets, w.K, dt, 2, rtol=1e-13,
                  g_u=w.g_u, g_v=w.g_v, box=4)
    assert s.converged
    E0 = _energy(u, v, w.X, w.fiber_offsets, w.K, 1.0, h)
    E1 = _energy(s.u, s.v, s.X, w.fiber_offsets, w.K, 1.0, h)
    Lap = mac.laplacian(N)
    Lf = ib.fiber_laplacian(w.fiber_offsets, w.M)
    d = s.X - w.X
    visc = dt * h * h * (s.u.ravel() @ (Lap @ s.u.ravel()) + s.v.ravel() @ (Lap @ s.v.ravel()))
    kin = 0.5 * h * h * (np.sum((s.u - u) ** 2) + np.sum((s.v - v) ** 2))
    el = 0.5 * w.K * (d[:, 0] @ (-Lf @ d[:, 0]) + d[:, 1] @ (-Lf @ d[:, 1]))
    work = dt * h * h * (np.sum(w.g_u * s.u) + np.sum(w.g_v * s.v))
    pred = visc - kin - el + work
    scale = abs(E0) + abs(visc) + abs(el) + abs(work)
    assert abs((E1 - E0) - pred) < 1e-9 * scale
    # momentum
    assert abs((s.u.mean() - u.mean()) / dt - w.g_u.mean()) < 1e-9
    assert abs((s.v.mean() - v.mean()) / dt - w.g_v.mean()) < 1e-9
    # divergence-free to solve tolerance
    Dx, Dy = mac.divergence(N)
    div = Dx @ s.u.ravel() + Dy @ s.v.ravel()
    assert np.linalg.norm(div) < 1e-10 * np.linalg.norm(s.b)


def test_step_energy_decays_without_forcing():
    N = 16
    w = ibgen.small_case(N=N, M=48, K=3e3, seed=6)
    dt = 100 * dtexp.dt_explicit(w.X, w.fiber_offsets, N, w.K)
    h = 1.0 / N
    u = np.zeros((N, N)); v = np.zeros((N, N)); p = np.zeros((N, N))
    X = w.X.copy()
    E = [_energy(u, v, X, w.fiber_offsets, w.K, 1.0, h)]
    for _ in range(3):
        s = step.step(u, v, p, X, w.fiber_offsets, w.K, dt, 2, rtol=1e-12, box=4)
        u, v, p, X = s.u, s.v, s.p, s.X
        E.append(_energy(u, v, X, w.fiber_offsets, w.K, 1.0, h))
    assert all(E[k + 1] <= E[k] * (1 + 1e-10) for k in range(3))
    assert E[-1] < E[0]


# ---------------------------------------------------------------- explicit method (Sec. 2.3.1, Sec. 7)

def test_explicit_step_is_a_stokes_solve_with_the_force_at_x_n():
    """The explicit step's velocity is the periodic unsteady Stokes solution
    (an independent FFT solve) for the right-hand side (rho/dt) u^n + S_0 G^n
    + g, and the positions move with the interpolated new velocity."""
    N = 16
    w = ibgen.small_case(N=N, M=40, K=2e3, seed=4, with_force=True)
    dt = 0.5 * dtexp.dt_explicit(w.X, w.fiber_offsets, N, w.K)
    r = np.random.default_rng(12)
    u0, v0 = r.standard_normal((N, N)), r.standard_normal((N, N))
    o = step.step(u0, v0, np.zeros((N, N)), w.X, w.fiber_offsets, w.K, dt, 2, rtol=1e-13, g_u=w.g_u, g_v=w.g_v,
                  scheme="explicit")
    b = system.rhs(u0, v0, w.X, w.fiber_offsets, w.K, dt, 1.0, w.g_u, w.g_v)
    fu, fv, _ = system.split(b, N)
    uf, vf, pf = stokes_fft.solve(fu, fv, 1.0 / dt, 1.0)
    assert np.max(np.abs(o.u - uf)) < 1e-10 * np.max(np.abs(uf))
    assert np.max(np.abs(o.v - vf)) < 1e-10 * np.max(np.abs(vf))
    U = ib.interp(w.X, uf, vf)
    assert np.max(np.abs(o.X - (w.X + dt * U))) < 1e-12
    # with no springs the two schemes are the same step
    oi = step.step(u0, v0, np.zeros((N, N)), w.X, w.fiber_offsets, 0.0, dt, 2, rtol=1e-13)
    oe = step.step(u0, v0, np.zeros((N, N)), w.X, w.fiber_offsets, 0.0, dt, 2, rtol=1e-13, scheme="explicit")
    assert np.array_equal(oi.u, oe.u) and np.array_equal(oi.X, oe.X)


# ---------------------------------------------------------------- multigrid as the solver (Sec. 5.1-5.2)

def _mg_case(N=16, K=1e3, fac=5.0):
    w = ibgen.small_case(N=N, M=40, K=K, seed=9)
    dt = fac * dtexp.dt_explicit(w.X, w.fiber_offsets, N, K)
    lv = system.hierarchy(N, 2, 1.0, 1.0, dt, w.X, w.fiber_offsets, K)
    return lv, mg.VCycle(lv, 2, 1, 1, "colour")


def test_mg_iteration_matrix_is_the_error_propagator():
    """One multigrid step x1 = x0 + MGV(0, b - A x0) moves the error by the
    iteration matrix: x1 - x* = T (x0 - x*), with x* the exact solution (dense
    bordered solve; errors compared with their pressure means removed)."""
    lv, V = _mg_case()
    A = lv[0].A
    n = A.shape[0]
    N = lv[0].N
    T = mg.iteration_matrix(A, V, n)
    r = np.random.default_rng(31)
    b = r.standard_normal(n)
    b[2 * N * N:] -= b[2 * N * N:].mean()
    B = np.zeros((n + 1, n + 1))
    B[:n, :n] = A.toarray()
    B[2 * N * N:n, n] = 1.0
    B[n, 2 * N * N:n] = 1.0
    xs = np.linalg.solve(B, np.concatenate([b, [0.0]]))[:n]
    x0 = r.standard_normal(n)
    x1, its, _, _ = mg.mg_solve(A, b, V, x0=x0, rtol=0.0, maxit=1)
    assert its == 1

    def zm(e):
        e = e.copy()
        e[2 * N * N:] -= e[2 * N * N:].mean()
        return e
    e1, Te0 = zm(x1 - xs), zm(T @ (x0 - xs))
    assert np.max(np.abs(e1 - Te0)) < 1e-10 * np.max(np.abs(e1))


def test_mg_solver_converges_at_the_spectral_radius():
    """The residual of the multigrid solver falls, asymptotically, by the
    spectral radius of the iteration matrix per V-cycle (on the space of
    zero-mean pressure), and the solver meets its tolerance."""
    lv, V = _mg_case(K=1e3, fac=20.0)
    A = lv[0].A
    n = A.shape[0]
    N = lv[0].N
    T = mg.iteration_matrix(A, V, n)
    q = np.zeros(n)
    q[2 * N * N:] = 1.0 / N
    Pm = np.eye(n) - np.outer(q, q)
    rho = float(np.max(np.abs(np.linalg.eigvals(Pm @ T @ Pm))))
    assert 0.05 < rho < 0.9
    b = np.random.default_rng(32).standard_normal(n)
    b[2 * N * N:] -= b[2 * N * N:].mean()
    x, its, ok, hist = mg.mg_solve(A, b, V, rtol=1e-12, maxit=400)
    assert ok and np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b)
    late = [hist[k + 1] / hist[k] for k in range(len(hist) - 6, len(hist) - 1)]
    assert abs(np.exp(np.mean(np.log(late))) - rho) < 0.1 * rho, (late, rho)
