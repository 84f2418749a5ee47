"""Helpers for the GPU parity tests: build oracle problems and GPU solvers on
the same seeded inputs.  The oracle supplies expected values; the GPU side
is called only through the C ABI (paper_1311_5614_amd.ibmg)."""
import numpy as np
import torch

import ibgen
from oracle import dtexp, step as ostep, system, mg

DEV = "cuda:0"


def tdev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def tnp(t):
    return t.detach().cpu().numpy()


def make(N=32, levels=3, M=64, K=1e4, dt_factor=20.0, seed=5, box=4, nu=(2, 2), prec=0, n_fibers=1,
         delta=0, maxit=100, rtol=1e-10, with_force=False, guess=0, colours=2, tail_max=0):
    from paper_1311_5614_amd import ibmg
    w = ibgen.small_case(N=N, M=M, K=K, seed=seed, n_fibers=n_fibers, levels=levels, box=box,
                         with_force=with_force)
    dt = dt_factor * dtexp.dt_explicit(w.X, w.fiber_offsets, N, K, kind=delta) if K > 0 else 0.05
    cfg = ibmg.Config(N=N, levels=levels, K=K, box=box, nu1=nu[0], nu2=nu[1], maxit=maxit, rtol=rtol,
                      prec=prec, delta=delta, guess=guess, colours=colours, tail_max=tail_max)
    s = ibmg.Solver(cfg, w.fiber_offsets, DEV)
    return w, dt, s


def oracle_levels(w, dt, levels, K, delta=0):
    return system.hierarchy(w.N, levels, 1.0, 1.0, dt, w.X, w.fiber_offsets, K, delta)


def rel(a, b):
    a = np.asarray(a, float).ravel()
    b = np.asarray(b, float).ravel()
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
