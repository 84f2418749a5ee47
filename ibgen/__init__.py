"""Seeded synthetic workload generator for the implicit immersed-boundary solve.

This module draws the inputs of the elastic-membrane workloads: Lagrangian
point positions of closed fibres (perturbed ellipses, rings), fibre offsets,
stiffness values and the smooth random body force.  It holds none of the
method's arithmetic (no operators, no spreading, no solves); both the CPU
oracle and the GPU path consume the arrays it returns.

Conventions: periodic unit square, N cells per side, h = 1/N.  Velocity
faces follow the MAC layout of the paper's spatial discretisation (Sec. 2.2):
u[j][i] sits at (i h, (j + 1/2) h), v[j][i] at ((i + 1/2) h, j h).  Arrays are
row-major with x fastest.  Seeds are 1311000 + 100 * config + instance.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

__all__ = [
    "Workload", "seed_for", "ellipse", "rings", "fourier_force",
    "config_c1", "config_c2_cases", "config_c3", "config_c4", "config_c5",
    "small_case", "cnn_init", "sphere_rings",
]


def seed_for(config: int, instance: int = 0) -> int:
    return 1311_000 + 100 * config + instance


@dataclass
class Workload:
    """One IB problem instance (inputs only)."""
    name: str
    N: int                      # cells per side
    levels: int                 # multigrid levels (coarsest N / 2**(levels-1))
    X: np.ndarray               # (M, 2) float64 Lagrangian positions (unwrapped)
    fiber_offsets: np.ndarray   # (F+1,) int32 CSR offsets of closed fibres
    K: float                    # nodal spring stiffness (G = K L X)
    dt_factor: float            # dt = dt_factor * explicit limit
    rho: float = 1.0
    mu: float = 1.0
    box: int = 4
    nu1: int = 2
    nu2: int = 2
    rtol: float = 1e-8
    steps: int = 1
    g_u: np.ndarray | None = None   # (N, N) body force on u faces, or None
    g_v: np.ndarray | None = None
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return int(self.X.shape[0])


def ellipse(rng: np.random.Generator, M: int, perturb: float = 0.02,
            centre=(0.5, 0.5), axes_range=(0.2, 0.3)):
    """Closed ellipse with semi-axes ~ U(axes_range) and a radial
    perturbation perturb*sin(m*theta + phi0), m ~ U{2..5}, phi0 ~ U(0, 2pi);
    theta_k = 2 pi k / M, axis-aligned."""
    a, b = rng.uniform(axes_range[0], axes_range[1], size=2)
    m = int(rng.integers(2, 6))
    phi0 = float(rng.uniform(0.0, 2.0 * np.pi))
    th = 2.0 * np.pi * np.arange(M) / M
    d = perturb * np.sin(m * th + phi0)
    X = np.empty((M, 2))
    X[:, 0] = centre[0] + (a + d) * np.cos(th)
    X[:, 1] = centre[1] + (b + d) * np.sin(th)
    return X, dict(a=float(a), b=float(b), m=m, phi0=phi0)


def _pdist(p, q):
    d = np.abs(np.asarray(p) - np.asarray(q))
    d = np.minimum(d, 1.0 - d)
    return float(np.hypot(d[0], d[1]))


def rings(rng: np.random.Generator, n_rings: int, M_each: int, N: int,
          r_range=(0.05, 0.1), gap_cells: float = 8.0, max_tries: int = 100000):
    """n_rings non-overlapping circles: radii ~ U(r_range), centres ~ U[0,1)^2
    by rejection with periodic centre distance >= r_i + r_j + gap_cells*h."""
    h = 1.0 / N
    radii = rng.uniform(r_range[0], r_range[1], size=n_rings)
    centres = []
    tries = 0
    for i in range(n_rings):
        while True:
            tries += 1
            if tries > max_tries:
                raise RuntimeError("ring placement failed")
            c = rng.uniform(0.0, 1.0, size=2)
            if all(_pdist(c, centres[j]) >= radii[i] + radii[j] + gap_cells * h
                   for j in range(len(centres))):
                centres.append(c)
                break
    th = 2.0 * np.pi * np.arange(M_each) / M_each
    X = np.concatenate([
        np.stack([c[0] + r * np.cos(th), c[1] + r * np.sin(th)], axis=1)
        for c, r in zip(centres, radii)])
    offs = np.arange(n_rings + 1, dtype=np.int32) * M_each
    return X, offs, dict(radii=radii.tolist(),
                         centres=[list(map(float, c)) for c in centres])


def fourier_force(rng: np.random.Generator, N: int, n_modes: int = 16, kmax: int = 4):
    """Smooth random body force: per component, sum of n_modes Fourier modes
    a cos(2 pi k.x) + b sin(2 pi k.x), k ~ U{-kmax..kmax}^2 minus 0,
    a, b ~ N(0, 1); sampled at the u and v face centres."""
    h = 1.0 / N
    out = []
    for comp in range(2):
        ks = []
        while len(ks) < n_modes:
            k = rng.integers(-kmax, kmax + 1, size=2)
            if k[0] == 0 and k[1] == 0:
                continue
            ks.append(k)
        ks = np.array(ks, dtype=np.float64)
        a = rng.standard_normal(n_modes)
        b = rng.standard_normal(n_modes)
        i = np.arange(N, dtype=np.float64)
        if comp == 0:   # u faces: (i h, (j+1/2) h)
            x = i[None, :] * h
            y = (i[:, None] + 0.5) * h
        else:           # v faces: ((i+1/2) h, j h)
            x = (i[None, :] + 0.5) * h
            y = i[:, None] * h
        g = np.zeros((N, N))
        for m in range(n_modes):
            ph = 2.0 * np.pi * (ks[m, 0] * x + ks[m, 1] * y)
            g += a[m] * np.cos(ph) + b[m] * np.sin(ph)
        out.append(g)
    return out[0], out[1]


def annulus(N: int, xc: float = 0.5, yc: float = 0.5, r: float = 0.25, width: float = 1.0 / 16):
    """The thick annulus of the paper's test problem (Sec. 4) as input
    positions: M2 = 3 N / 32 + 1 concentric rings of M1 = 19 N / 8 points,
    ring l at radius r + l width / (M2 - 1), point k at angle 2 pi k / M1.
    Returns (X of shape (M1 M2, 2), fibre offsets, M1, M2).  Deterministic."""
    if N % 32:
        raise ValueError("N must be a multiple of 32")
    M1, M2 = 19 * N // 8, 3 * N // 32 + 1
    th = 2.0 * np.pi * np.arange(M1) / M1
    X = np.concatenate([np.stack([xc + (r + l * width / (M2 - 1)) * np.cos(th),
                                  yc + (r + l * width / (M2 - 1)) * np.sin(th)], 1) for l in range(M2)])
    return X, np.arange(M2 + 1, dtype=np.int32) * M1, M1, M2


def config_c1() -> Workload:
    """32x32, 4 levels, one perturbed ellipse of 128 points, K=1e4,
    dt = 100 x explicit limit, V(2,2), box 4, rtol 1e-10, one step."""
    rng = np.random.default_rng(seed_for(1))
    X, meta = ellipse(rng, 128)
    return Workload("ellipse-32x32-M128-K1e4", 32, 4, X,
                    np.array([0, 128], np.int32), 1e4, 100.0, rtol=1e-10,
                    steps=1, seed=seed_for(1), meta=meta)


def config_c2_cases(N: int = 256, levels: int = 7, M: int = 1024):
    """256x256, one ellipse of 1024 points, smooth random body force;
    K in {1e2, 1e4, 1e6, 1e8} x dt in {100, 1000} x explicit limit; 20 steps
    each at rtol 1e-8.  Geometry and force shared by all 8 cases.  The level
    count is not fixed by the workload; 7 levels put the coarsest grid at
    4 x 4 = max(4, box), the paper's coarsest-grid rule."""
    rng = np.random.default_rng(seed_for(2))
    X, meta = ellipse(rng, M)
    gu, gv = fourier_force(rng, N)
    cases = []
    for K in (1e2, 1e4, 1e6, 1e8):
        for f in (100.0, 1000.0):
            cases.append(Workload(f"ellipse-{N}x{N}-M{M}-K{K:.0e}-dt{int(f)}x",
                                  N, levels, X.copy(), np.array([0, M], np.int32),
                                  K, f, rtol=1e-8, steps=20, g_u=gu, g_v=gv,
                                  seed=seed_for(2), meta=dict(meta)))
    return cases


def config_c3() -> Workload:
    """1024x1024, 7 levels, 8 rings of 2048 points, K=1e6, dt 500x."""
    rng = np.random.default_rng(seed_for(3))
    X, offs, meta = rings(rng, 8, 2048, 1024)
    return Workload("8rings-1024x1024-M16384-K1e6", 1024, 7, X, offs, 1e6, 500.0,
                    rtol=1e-8, steps=50, seed=seed_for(3), meta=meta)


def config_c4(n_problems: int = 64):
    """Batch of independent problems, N ~ U{64,128,256,512}, one ellipse of
    round(0.8 pi N) points, K = 10**U(3,7), dt 100x, 10 steps; levels down
    to a 4 x 4 coarsest grid (the paper's max(4, box) rule)."""
    out = []
    for inst in range(n_problems):
        rng = np.random.default_rng(seed_for(4, inst))
        N = int(rng.choice([64, 128, 256, 512]))
        M = int(round(0.8 * np.pi * N))
        X, meta = ellipse(rng, M)
        K = float(10.0 ** rng.uniform(3.0, 7.0))
        levels = int(np.log2(N // 4)) + 1
        out.append(Workload(f"batch{inst}-{N}x{N}-M{M}", N, levels, X,
                            np.array([0, M], np.int32), K, 100.0, rtol=1e-8,
                            steps=10, seed=seed_for(4, inst), meta=meta))
    return out


def config_c5() -> Workload:
    """512x512, 6 levels, one ellipse of 2048 points, K=1e5, dt 200x,
    smooth random body force, 400 steps."""
    rng = np.random.default_rng(seed_for(5))
    X, meta = ellipse(rng, 2048)
    gu, gv = fourier_force(rng, 512)
    return Workload("ellipse-512x512-M2048-K1e5", 512, 6, X,
                    np.array([0, 2048], np.int32), 1e5, 200.0, rtol=1e-8,
                    steps=400, g_u=gu, g_v=gv, seed=seed_for(5), meta=meta)


def small_case(N: int = 16, M: int = 40, K: float = 1e3, seed: int = 7,
               n_fibers: int = 1, levels: int = 2, box: int = 4,
               with_force: bool = False) -> Workload:
    """Tiny seeded problem for brute-force checks (ellipses of M points)."""
    rng = np.random.default_rng(seed)
    Xs, offs = [], [0]
    for f in range(n_fibers):
        c = (0.5, 0.5) if n_fibers == 1 else tuple(rng.uniform(0.3, 0.7, size=2))
        X, _ = ellipse(rng, M, centre=c, axes_range=(0.15, 0.3))
        Xs.append(X)
        offs.append(offs[-1] + M)
    X = np.concatenate(Xs)
    gu = gv = None
    if with_force:
        gu, gv = fourier_force(rng, N, n_modes=4, kmax=2)
    return Workload(f"small-{N}-M{M}", N, levels, X, np.array(offs, np.int32), K,
                    1.0, box=box, rtol=1e-12, g_u=gu, g_v=gv, seed=seed)


def cnn_init(seed: int, layers=((5, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 3))):
    """Initial parameters of the warm-start network, flat FP32 in layer
    order (per layer W [co, ci, 3, 3] row-major, then b [co]): W ~ N(0,
    2 / (9 ci)) (He), b = 0, and the last layer all zero, so that the
    untrained network proposes no change."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (ci, co) in enumerate(layers):
        if li == len(layers) - 1:
            W = np.zeros(co * ci * 9)
        else:
            W = rng.standard_normal(co * ci * 9) * np.sqrt(2.0 / (9 * ci))
        parts += [W, np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


def sphere_rings(N: int, seed: int = 0, r: float = 0.22, spacing: float = 1.0,
                 stretch=(1.15, 0.9, 0.95), centre=(0.5, 0.5, 0.5), jitter: float = 0.05):
    """Three-dimensional structure for the periodic unit cube: closed
    latitude rings on a stretched sphere (an ellipsoid with semi-axes
    r * stretch), rings `spacing` h apart in polar arc length, points about
    `spacing` h apart along each ring, each ring turned by a random phase and
    every point moved by up to jitter * h.  Returns (X (M, 3), fibre offsets)."""
    rng = np.random.default_rng(seed_for(6, seed))
    h = 1.0 / N
    n_lat = max(1, int(round(np.pi * r / (spacing * h))) - 1)
    pts, offs = [], [0]
    for i in range(n_lat):
        th = np.pi * (i + 1) / (n_lat + 1)
        m = max(8, int(round(2.0 * np.pi * r * np.sin(th) / (spacing * h))))
        ph = 2.0 * np.pi * np.arange(m) / m + rng.uniform(0.0, 2.0 * np.pi)
        ring = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.full(m, np.cos(th))], axis=1)
        ring = np.asarray(centre) + r * np.asarray(stretch) * ring
        ring += rng.uniform(-jitter * h, jitter * h, size=ring.shape)
        pts.append(ring)
        offs.append(offs[-1] + m)
    return np.concatenate(pts), np.asarray(offs, dtype=np.int32)
