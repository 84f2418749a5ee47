"""GPU parity of the box smoother and the V-cycle on levels with elastic rows
at the sizes where the benchmark workloads run them, element by element
against the oracle's BoxSmoother and VCycle (Sec. 5-6 box relaxation,
Algorithm 1).

These sizes reach the kernel forms the small-grid parity tests do not:
  * four waves per workgroup in the box kernel (levels with at least 2048
    boxes per colour) on levels with elastic rows: the 256x256 single-ellipse
    sweep geometry (level 0, 2 colours) and the eight-ring 1024x1024 geometry
    on a 512x512 grid (levels 0 and 1);
  * the elastic-row pass striding over more than 8192 active rows per
    component (the eight rings at 512x512, 9170 active u rows);
  * 8x8 boxes on a level with elastic rows at 256x256.

Tolerances: FP64 one sweep and one V-cycle 1e-11 relative in max-norm (the
same bound as the small grids: explicit Gauss-Jordan inverses against the
oracle's pivoted LU, FMA contraction).  FP32 V-cycle fields (per-box FP64
inverses of boxes with elastic rows): the measured error is printed and
bounded by 1e-5 relative in max-norm for a sweep (measured up to 2.7e-6),
and for a V-cycle in 2-norm by 1e-5 at K = 1e4, 100 x dt_exp and 1e-4 at
K = 1e6, 1000 x dt_exp (measured 2.6e-5: float epsilon 6e-8 times the growth
of the stiffer box solves).
"""
import json
import os

import numpy as np
import pytest
import torch

from gpu_common import DEV, rel, tdev, tnp

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

import ibgen  # noqa: E402
from oracle import ib, mg, smoother, system  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1311_5614_amd import ibmg  # noqa: F401  (raises if the library is missing)


def _dt(key, k=0):
    with open(os.path.join(ROOT, "tests", "golden", "workload_dt.json")) as f:
        return json.load(f)[key][k]["dt"]


def _geometry(name):
    """(X, fiber_offsets, K, dt, N) of a workload geometry on the grid the test uses."""
    if name == "ellipse256-K1e4-100x":
        w = ibgen.config_c2_cases()[2]
        return w.X, w.fiber_offsets, w.K, _dt("c2", 2), 256
    if name == "ellipse256-K1e6-1000x":
        w = ibgen.config_c2_cases()[5]
        return w.X, w.fiber_offsets, w.K, _dt("c2", 5), 256
    if name == "rings512":
        # the eight rings of the 1024x1024 workload (K = 1e6) on a 512 x 512
        # grid, at the 1024 workload's time step
        w = ibgen.config_c3()
        return w.X, w.fiber_offsets, w.K, _dt("c3"), 512
    raise KeyError(name)


def _solver(N, levels, K, fo, box, colours, prec, nu=(2, 2)):
    from paper_1311_5614_amd import ibmg
    cfg = ibmg.Config(N=N, levels=levels, K=K, box=box, nu1=nu[0], nu2=nu[1], colours=colours, prec=prec,
                      maxit=50, rtol=1e-8)
    return ibmg.Solver(cfg, fo, DEV)


def _active_rows(X, N):
    S = ib.spread_matrix(X, N, 0, ib.DELTA_IB4)
    return int(np.count_nonzero(np.asarray(abs(S).sum(1)).ravel()))


SWEEPS = [
    # (geometry, box, colours, prec, levels checked)
    ("ellipse256-K1e4-100x", 4, 2, 0, (0, 1)),
    ("ellipse256-K1e6-1000x", 4, 2, 0, (0,)),
    ("ellipse256-K1e6-1000x", 4, 4, 0, (0,)),
    ("ellipse256-K1e6-1000x", 8, 2, 0, (0,)),
    ("ellipse256-K1e6-1000x", 4, 2, 1, (0,)),
    ("rings512", 4, 2, 0, (0, 1)),
    ("rings512", 4, 2, 1, (0, 1)),
]


@pytest.mark.parametrize("geom,box,colours,prec,check", SWEEPS)
def test_smooth_parity_elastic_levels(geom, box, colours, prec, check):
    X, fo, K, dt, N = _geometry(geom)
    if geom == "rings512":
        assert _active_rows(X, N) > 8192   # the elastic-row pass takes its grid-stride loop
    levels = int(np.log2(N // 16)) + 1          # coarsest 16 x 16
    s = _solver(N, levels, K, fo, box, colours, prec)
    try:
        s.setup(dt, tdev(X))
        lv = system.hierarchy(N, max(check) + 1, 1.0, 1.0, dt, X, fo, K)
        rng = np.random.default_rng(31)
        mode = "colour2" if colours == 2 else "colour"
        for l in check:
            Nl = lv[l].N
            b = rng.standard_normal(3 * Nl * Nl)
            x = rng.standard_normal(3 * Nl * Nl)
            sm = smoother.BoxSmoother(lv[l].A, Nl, box)
            xo = sm.sweep(x, b, mode)
            xg = tnp(s.smooth(l, tdev(b), tdev(x.copy()), 1))
            e = rel(xg, xo)
            print(f"{geom} box {box} colours {colours} prec {prec} level {l}: sweep error {e:.2e}")
            assert e < (1e-11 if prec == 0 else 1e-5), (l, e)
    finally:
        s.close()


@pytest.mark.parametrize("geom,box,prec", [("ellipse256-K1e4-100x", 4, 0), ("ellipse256-K1e6-1000x", 4, 0),
                                           ("ellipse256-K1e6-1000x", 8, 0), ("ellipse256-K1e4-100x", 4, 1),
                                           ("ellipse256-K1e6-1000x", 4, 1)])
def test_vcycle_parity_256_elastic(geom, box, prec):
    """One V(2,2) over 5 levels (coarsest 16 x 16) of the 256x256 sweep
    geometry, checkerboard boxes, against the oracle's VCycle."""
    X, fo, K, dt, N = _geometry(geom)
    s = _solver(N, 5, K, fo, box, 2, prec)
    try:
        s.setup(dt, tdev(X))
        lv = system.hierarchy(N, 5, 1.0, 1.0, dt, X, fo, K)
        V = mg.VCycle(lv, box, 2, 2, "colour2")
        r = np.random.default_rng(32).standard_normal(3 * N * N)
        r[2 * N * N:] -= r[2 * N * N:].mean()
        z = tnp(s.vcycle(tdev(r)))
        zo = V(r)
        if prec == 0:
            e = rel(z, zo)
            print(f"{geom} box {box}: fp64 V-cycle error (max-norm) {e:.2e}")
            assert e < 1e-11
        else:
            e = np.linalg.norm(z - zo) / np.linalg.norm(zo)
            print(f"{geom} box {box}: fp32 V-cycle error (2-norm) {e:.2e}")
            assert e < (1e-5 if geom == "ellipse256-K1e4-100x" else 1e-4)
    finally:
        s.close()
