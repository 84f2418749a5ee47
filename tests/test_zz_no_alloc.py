"""ibmg_spread_noalloc (scratch in a static device array, no allocation)
against ibmg_spread on the same inputs, bit for bit: two calls in a row, the
second with a smaller grid and fewer points, then the empty structure."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_common import DEV, make, tdev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1311_5614_amd import ibmg  # noqa: F401  (raises if the library is missing)


def _noalloc(N, delta, X, G):
    from paper_1311_5614_amd import ibmg
    fu = torch.full((N, N), np.nan, dtype=torch.float64, device=DEV)
    fv = torch.full((N, N), np.nan, dtype=torch.float64, device=DEV)
    M = 0 if X is None else X.shape[0]
    stream = torch.cuda.current_stream(DEV).cuda_stream
    rc = ibmg.lib().ibmg_spread_noalloc(N, delta, M, C.c_void_p(X.data_ptr() if M else 0),
                                        C.c_void_p(G.data_ptr() if M else 0), C.c_void_p(fu.data_ptr()),
                                        C.c_void_p(fv.data_ptr()), C.c_void_p(stream))
    torch.cuda.synchronize()
    return rc, fu, fv


@pytest.mark.parametrize("delta", [0, 1])
def test_spread_noalloc_matches_spread(delta):
    rng = np.random.default_rng(50 + delta)
    for N, M, nf in ((256, 4000, 4), (64, 300, 2)):
        w, dt, s = make(N=N, levels=int(np.log2(N // 16)) + 1, M=M // nf, n_fibers=nf, delta=delta)
        X = w.X + rng.uniform(-1.5, 1.5, size=(1, 2))       # unwrapped positions
        G = rng.standard_normal(X.shape)
        fu, fv = s.spread(tdev(X), tdev(G))
        rc, gu, gv = _noalloc(N, delta, tdev(X), tdev(G))
        assert rc == 0
        assert torch.equal(gu, fu) and torch.equal(gv, fv), (N, M)
        s.close()
    rc, gu, gv = _noalloc(32, delta, None, None)
    assert rc == 0 and float(gu.abs().max()) == 0.0 and float(gv.abs().max()) == 0.0


def test_spread_noalloc_rejects_sizes_beyond_its_limit():
    from paper_1311_5614_amd import ibmg
    L = ibmg.lib()
    z = C.c_void_p(0)
    fu = torch.zeros(1, dtype=torch.float64, device=DEV)
    p = C.c_void_p(fu.data_ptr())
    assert L.ibmg_spread_noalloc(1024, 0, 10, p, p, p, p, z) == -1    # N above 512
    assert L.ibmg_spread_noalloc(48, 0, 10, p, p, p, p, z) == -1      # not a power of two
    assert L.ibmg_spread_noalloc(64, 0, 9000, p, p, p, p, z) == -1    # M above 8192
    assert L.ibmg_spread_noalloc(64, 2, 10, p, p, p, p, z) == -1      # bad delta
    assert L.ibmg_spread_noalloc(64, 0, 10, z, p, p, p, z) == -1      # null positions
