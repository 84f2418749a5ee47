"""GPU parity of the batched form: problems of different grid sizes, point
counts, stiffness, time steps and options advanced together through
ibmg_batch_step must give, problem by problem, bitwise the same state and the
same iteration counts as ibmg_step on one handle per problem; one small
problem is also checked against the CPU oracle's step."""
import numpy as np
import pytest
import torch

from gpu_common import DEV, tdev, tnp

pytestmark = pytest.mark.gpu

import ibgen  # noqa: E402
from oracle import dtexp, step as ostep  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1311_5614_amd import ibmg  # noqa: F401  (raises if the library is missing)


# (N, levels, M, K, dt factor, box, (nu1, nu2), colours, seed, body force[, tail_max])
SPECS = [
    (32, 4, 64, 1e4, 50.0, 4, (2, 2), 2, 11, False),    # whole V-cycle in the LDS tail
    (64, 5, 120, 1e5, 100.0, 4, (2, 2), 2, 12, True),   # one big level
    (128, 6, 300, 1e3, 100.0, 4, (2, 2), 2, 13, False),  # two big levels
    (64, 4, 90, 1e6, 20.0, 2, (1, 1), 4, 14, False),    # 2x2 boxes, 4 colours, V(1,1), 8x8 coarsest
    (128, 6, 250, 0.0, 1.0, 4, (2, 1), 2, 15, True),    # no elastic coupling (K = 0)
    (64, 5, 160, 1e2, 10.0, 1, (2, 2), 2, 16, False),   # single-cell boxes (mild: weak smoother)
    (128, 6, 280, 1e4, 50.0, 4, (2, 2), 2, 17, False, 8),  # tail from 8^2 down: four big levels
    (64, 3, 140, 1e4, 50.0, 4, (2, 2), 2, 18, False, 1),   # 16^2 coarsest solved alone in the tail
    (64, 4, 150, 1e5, 100.0, 8, (2, 2), 2, 19, False),  # 8x8 boxes, 8^2 coarsest (register inverse)
    (128, 5, 300, 1e4, 50.0, 8, (1, 1), 4, 20, True),   # 8x8 boxes, 4 colours, 16^2 coarsest
]


def _inputs():
    out = []
    for (N, levels, M, K, fac, box, nu, col, seed, force, *tm) in SPECS:
        w = ibgen.small_case(N=N, M=M, K=max(K, 1.0), seed=seed, levels=levels, box=box, with_force=force)
        w.tail_max = tm[0] if tm else 0
        dt = fac * dtexp.dt_explicit(w.X, w.fiber_offsets, N, K) if K > 0 else 0.02
        out.append((w, K, dt, box, nu, col))
    return out


def _cfg(w, K, box, nu, col, prec):
    from paper_1311_5614_amd import ibmg
    return ibmg.Config(N=w.N, levels=w.levels, K=K, box=box, nu1=nu[0], nu2=nu[1], maxit=100, rtol=1e-9,
                       prec=prec, colours=col, tail_max=w.tail_max)


def _state(w):
    z = torch.zeros(w.N, w.N, dtype=torch.float64, device=DEV)
    g = (tdev(w.g_u), tdev(w.g_v)) if w.g_u is not None else (None, None)
    return [z.clone(), z.clone(), z.clone(), tdev(w.X), g[0], g[1]]


def _run_single(inp, prec, steps):
    from paper_1311_5614_amd import ibmg
    res = []
    for (w, K, dt, box, nu, col) in inp:
        s = ibmg.Solver(_cfg(w, K, box, nu, col, prec), w.fiber_offsets, DEV)
        u, v, p, X, gu, gv = _state(w)
        its = []
        for _ in range(steps):
            st = s.step(dt, u, v, p, X, gu, gv)
            its.append((st["iters"], st["converged"]))
        torch.cuda.synchronize()
        res.append(([u, v, p, X], its))
        s.close()
    return res


def _run_batch(inp, prec, steps, graph=True):
    from paper_1311_5614_amd import ibmg
    B = ibmg.Batch([_cfg(w, K, box, nu, col, prec) for (w, K, dt, box, nu, col) in inp],
                   [w.fiber_offsets for (w, *_) in inp], DEV)
    B.set_graph(graph)
    st = [_state(w) for (w, *_) in inp]
    dts = [dt for (_, _, dt, *_) in inp]
    its = [[] for _ in inp]
    for _ in range(steps):
        out = B.step(dts, [s[0] for s in st], [s[1] for s in st], [s[2] for s in st], [s[3] for s in st],
                     [s[4] for s in st], [s[5] for s in st])
        for i, o in enumerate(out):
            its[i].append((o["iters"], o["converged"]))
    torch.cuda.synchronize()
    rounds = B.rounds()
    B.close()
    return [(s[:4], it) for s, it in zip(st, its)], rounds


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_equals_single_bitwise(prec):
    inp = _inputs()
    single = _run_single(inp, prec, steps=2)
    batch, rounds = _run_batch(inp, prec, steps=2)
    print("iterations (single, batch):", [(a[1], b[1]) for a, b in zip(single, batch)])
    for i, ((ts, its), (tb, itb)) in enumerate(zip(single, batch)):
        assert its == itb, (i, its, itb)
        if inp[i][3] > 1:   # single-cell boxes are too weak a smoother to promise rtol in 100 steps
            assert all(c == 1 for _, c in its), (i, its)
        for a, b in zip(ts, tb):
            assert torch.equal(a, b), (i, float((a - b).abs().max()))
    # lockstep: the rounds of one step are bounded by the slowest problem's
    # iterations plus two rounds per Arnoldi cycle (start, end) and ||b||
    assert rounds <= sum(max(it[s][0] for _, it in single) + 4 for s in range(2))


def test_batch_of_coarsest_only_tails_equals_single_bitwise():
    """Every problem's LDS-resident tail is its coarsest level alone (tail
    size 1, and 8x8 boxes): the tail kernel's LDS is sized for that level."""
    inp = [i for i, spec in zip(_inputs(), SPECS) if spec[5] == 8 or spec[10:] == (1,)]
    assert len(inp) == 3
    single = _run_single(inp, 1, steps=1)
    batch, _ = _run_batch(inp, 1, steps=1)
    for (ts, its), (tb, itb) in zip(single, batch):
        assert its == itb
        for a, b in zip(ts, tb):
            assert torch.equal(a, b)


def test_batch_graph_equals_eager():
    inp = _inputs()[:4]
    g, _ = _run_batch(inp, 1, steps=1, graph=True)
    e, _ = _run_batch(inp, 1, steps=1, graph=False)
    for (ta, ia), (tb, ib_) in zip(g, e):
        assert ia == ib_
        for a, b in zip(ta, tb):
            assert torch.equal(a, b)


def test_batch_member_matches_oracle_step():
    inp = _inputs()[:2]
    batch, _ = _run_batch(inp, 0, steps=1)
    w, K, dt, box, nu, col = inp[0]
    z = np.zeros((w.N, w.N))
    o = ostep.step(z, z, z, w.X, w.fiber_offsets, K, dt, w.levels, 1.0, 1.0, box, nu[0], nu[1], 1e-12,
                   g_u=w.g_u, g_v=w.g_v)
    u, v, p, X = (tnp(t) for t in batch[0][0])
    scale = max(np.abs(o.u).max(), np.abs(o.v).max())
    du = max(np.abs(u - o.u).max(), np.abs(v - o.v).max())
    assert du / scale < 1e-8
    # interpolation weights are non-negative and sum to one per component, so
    # the position error is at most dt times the velocity error
    assert np.abs(X - o.X).max() <= dt * du * (1 + 1e-12) + 1e-15


def test_batch_iteration_cap_and_errors():
    from paper_1311_5614_amd import ibmg
    inp = _inputs()[:2]
    cfgs = [_cfg(w, K, box, nu, col, 0) for (w, K, dt, box, nu, col) in inp]
    cfgs[1].maxit = 2
    B = ibmg.Batch(cfgs, [w.fiber_offsets for (w, *_) in inp], DEV)
    st = [_state(w) for (w, *_) in inp]
    out = B.step([dt for (_, _, dt, *_) in inp], [s[0] for s in st], [s[1] for s in st], [s[2] for s in st],
                 [s[3] for s in st])
    assert out[0]["converged"] == 1 and out[1]["converged"] == 0 and out[1]["iters"] == 2
    assert out[1]["status"] == ibmg.IBMG_NOT_CONVERGED
    with pytest.raises(ibmg.IBMGError):
        B.step([0.0, 1.0], [s[0] for s in st], [s[1] for s in st], [s[2] for s in st], [s[3] for s in st])
    B.close()
