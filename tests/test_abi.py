"""The C ABI without a GPU: the library loads, exports every symbol the header
declares, the ctypes structs match the C layout, and host-side validation
(shapes, options, fibre offsets) behaves as documented.  No compute call."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ibmg.h")


def _lib():
    from paper_1311_5614_amd import ibmg
    return ibmg, ibmg.lib()


def header_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(ibmg_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    ibmg, L = _lib()
    syms = header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(ibmg.EXPORTS) == syms
    out = subprocess.run(["nm", "-D", "--defined-only", ibmg.LIB_PATH], capture_output=True, text=True).stdout
    for s in syms:
        assert re.search(rf"\bT {s}$", out, re.M), s


def test_struct_layout_matches_c():
    ibmg, _ = _lib()
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "ibmg.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(ibmg_problem), sizeof(ibmg_opts), sizeof(ibmg_stats),
         offsetof(ibmg_problem, fiber_offsets), offsetof(ibmg_problem, K), offsetof(ibmg_opts, rtol),
         offsetof(ibmg_stats, t_step_ms), offsetof(ibmg_opts, colours), offsetof(ibmg_opts, tail_max),
         offsetof(ibmg_stats, rel_resid_est), offsetof(ibmg_stats, guess_rejected), offsetof(ibmg_opts, restart),
         offsetof(ibmg_opts, colours_from), offsetof(ibmg_opts, scheme),
         offsetof(ibmg_opts, solver), offsetof(ibmg_opts, omega), offsetof(ibmg_opts, orth),
         offsetof(ibmg_problem, domain));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        got = list(map(int, subprocess.run([exe], capture_output=True, text=True).stdout.split()))
    want = [C.sizeof(ibmg.ibmg_problem), C.sizeof(ibmg.ibmg_opts), C.sizeof(ibmg.ibmg_stats),
            ibmg.ibmg_problem.fiber_offsets.offset, ibmg.ibmg_problem.K.offset, ibmg.ibmg_opts.rtol.offset,
            ibmg.ibmg_stats.t_step_ms.offset, ibmg.ibmg_opts.colours.offset,
            ibmg.ibmg_opts.tail_max.offset, ibmg.ibmg_stats.rel_resid_est.offset,
            ibmg.ibmg_stats.guess_rejected.offset, ibmg.ibmg_opts.restart.offset,
            ibmg.ibmg_opts.colours_from.offset, ibmg.ibmg_opts.scheme.offset,
            ibmg.ibmg_opts.solver.offset, ibmg.ibmg_opts.omega.offset, ibmg.ibmg_opts.orth.offset,
            ibmg.ibmg_problem.domain.offset]
    assert got == want


def _create(N=32, levels=3, box=4, offs=(0, 40), **kw):
    ibmg, L = _lib()
    o = (C.c_int32 * len(offs))(*offs)
    prob = ibmg.ibmg_problem(N, kw.get("rho", 1.0), kw.get("mu", 1.0), offs[-1], len(offs) - 1,
                             C.cast(o, C.POINTER(C.c_int32)), kw.get("K", 1e3), kw.get("delta", 0),
                             kw.get("domain", 0))
    opts = ibmg.ibmg_opts(levels, box, kw.get("nu1", 2), kw.get("nu2", 2), kw.get("maxit", 100),
                          kw.get("rtol", 1e-8), kw.get("prec", 0), kw.get("guess", 0), kw.get("colours", 2),
                          kw.get("tail_max", 0), kw.get("restart", 0), kw.get("colours_from", 0),
                          kw.get("scheme", 0), kw.get("solver", 0), kw.get("omega", 1.0), kw.get("orth", 0))
    h = C.c_void_p()
    rc = L.ibmg_create(C.byref(h), C.byref(prob), C.byref(opts), None)
    return rc, h, L


def test_create_validates_shapes_without_gpu():
    rc, h, L = _create()
    assert rc == 0
    n = C.c_size_t()
    assert L.ibmg_workspace_bytes(h, C.byref(n)) == 0 and n.value > 0
    # unbound workspace -> ENOMEM on every device call, before touching the GPU
    assert L.ibmg_setup(h, 0.1, None) == -4
    assert L.ibmg_vcycle(h, None, None) == -4
    assert L.ibmg_destroy(h) == 0
    assert _create(N=48)[0] == -2                     # not a power of two
    assert _create(N=32, levels=5)[0] == -2           # coarsest 2x2
    assert _create(N=16, levels=2, box=3)[0] == -2    # unsupported box
    assert _create(N=16, levels=2, box=16)[0] == -2   # unsupported box
    assert _create(N=8, levels=2, box=4)[0] == 0      # 8x8 holds two 4x4 boxes per side
    assert _create(N=16, levels=2, box=8)[0] == 0     # 16x16 holds two 8x8 boxes per side
    assert _create(N=16, levels=3, box=8)[0] == -2    # an 8x8 smoothed level holds one 8x8 box
    assert _create(N=64, levels=2)[0] == -2           # coarsest 32 > 16
    assert _create(offs=(0, 30, 20))[0] == -1         # decreasing offsets
    assert _create(offs=(5, 40))[0] == -1             # offsets must start at 0
    assert _create(rho=0.0)[0] == -1
    assert _create(maxit=0)[0] == -1
    assert _create(prec=3)[0] == -1
    assert _create(colours=3)[0] == -1
    assert _create(colours=4)[0] == 0
    assert _create(tail_max=16)[0] == 0 and _create(tail_max=1)[0] == 0
    assert _create(tail_max=12)[0] == -1 and _create(tail_max=64)[0] == -1
    # restart: basis of 1..200 vectors; the cap may then exceed 200
    assert _create(maxit=1001)[0] == -1 and _create(maxit=1000)[0] == 0
    assert _create(maxit=5000, restart=50)[0] == 0
    assert _create(maxit=5000, restart=1001)[0] == -1 and _create(restart=-1)[0] == -1
    rc, h, L = _create(maxit=5000, restart=50)
    n_r = C.c_size_t()
    L.ibmg_workspace_bytes(h, C.byref(n_r))
    L.ibmg_destroy(h)
    rc, h, L = _create(maxit=50)
    n_50 = C.c_size_t()
    L.ibmg_workspace_bytes(h, C.byref(n_50))
    L.ibmg_destroy(h)
    assert n_r.value == n_50.value      # the workspace holds the basis, not the cap
    assert _create(colours=4, colours_from=2)[0] == 0 and _create(colours_from=4)[0] == -1
    assert _create(scheme=1)[0] == 0 and _create(scheme=2)[0] == -1
    assert _create(solver=1)[0] == 0 and _create(solver=2)[0] == -1
    assert _create(omega=0.8)[0] == 0 and _create(omega=1.5)[0] == -1 and _create(omega=-0.1)[0] == -1
    assert _create(orth=1)[0] == 0 and _create(orth=2)[0] == -1 and _create(orth=-1)[0] == -1
    # the walled cavity: steady form allowed, grid-wide levels only
    assert _create(domain=1, tail_max=1)[0] == 0 and _create(domain=1, tail_max=1, rho=0.0)[0] == 0
    assert _create(domain=1)[0] == -1 and _create(domain=2, tail_max=1)[0] == -1
    assert _create(rho=0.0, tail_max=1)[0] == -1


def test_status_strings():
    _, L = _lib()
    for code in (0, 1, -1, -2, -3, -4, -5, -6, 99):
        assert L.ibmg_status_string(code).decode()


def test_batch_create_validates_without_gpu():
    ibmg, L = _lib()
    offs = [(C.c_int32 * 2)(0, 40), (C.c_int32 * 2)(0, 80)]

    def make(Ns, precs, levels, box=4):
        probs = (ibmg.ibmg_problem * len(Ns))(*[
            ibmg.ibmg_problem(N, 1.0, 1.0, o[1], 1, C.cast(o, C.POINTER(C.c_int32)), 1e3, 0)
            for N, o in zip(Ns, offs)])
        opts = (ibmg.ibmg_opts * len(Ns))(*[ibmg.ibmg_opts(lv, box, 2, 2, 100, 1e-8, pr, 0, 2, 0)
                                            for pr, lv in zip(precs, levels)])
        h = C.c_void_p()
        return L.ibmg_batch_create(C.byref(h), len(Ns), probs, opts, None), h

    rc, h = make([32, 64], [0, 0], [4, 5])
    assert rc == 0
    n = C.c_size_t()
    assert L.ibmg_batch_workspace_bytes(h, C.byref(n)) == 0
    # the batch holds at least the two problems' own workspaces
    need = 0
    for N, lv in ((32, 4), (64, 5)):
        rc1, h1, _ = _create(N=N, levels=lv, offs=(0, 40 if N == 32 else 80))
        n1 = C.c_size_t()
        L.ibmg_workspace_bytes(h1, C.byref(n1))
        need += n1.value
        L.ibmg_destroy(h1)
    assert n.value >= need
    # unbound -> ENOMEM before any device work
    one = (C.c_double * 2)(1e-3, 1e-3)
    ptrs = (C.c_void_p * 2)()
    assert L.ibmg_batch_step(h, one, ptrs, ptrs, ptrs, ptrs, None, None, None) == -4
    assert L.ibmg_batch_destroy(h) == 0
    assert make([32, 64], [0, 1], [4, 5])[0] == -1   # mixed V-cycle precision
    assert make([32, 48], [0, 0], [4, 5])[0] == -2   # one bad grid
    rc8, h8 = make([32, 64], [0, 0], [2, 3], box=8)          # 8x8 boxes
    assert rc8 == 0
    assert L.ibmg_batch_destroy(h8) == 0
    assert make([32, 64], [0, 0], [4, 3], box=8)[0] == -2    # an 8x8 level would hold one 8x8 box
    h = C.c_void_p()
    assert L.ibmg_batch_create(C.byref(h), 0, None, None, None) == -1



def test_cnn_create_validates_without_gpu():
    ibmg, L = _lib()
    h = C.c_void_p()
    assert L.ibmg_cnn_create(C.byref(h), 64, 4, None) == 0
    n = C.c_size_t()
    assert L.ibmg_cnn_workspace_bytes(h, C.byref(n)) == 0
    # parameters, moments, gradient (4 x 39331 FP32) and the pair store (4 x 8 x 64^2 FP32) at least
    assert n.value >= 4 * 39331 * 4 + 4 * 8 * 64 * 64 * 4
    assert L.ibmg_cnn_infer(h, None, None) == -4          # unbound
    assert L.ibmg_cnn_destroy(h) == 0
    assert L.ibmg_cnn_create(C.byref(h), 48, 4, None) == -2
    assert L.ibmg_cnn_create(C.byref(h), 8, 4, None) == -2
    assert L.ibmg_cnn_create(C.byref(h), 64, 0, None) == -1


HEADER3 = os.path.join(ROOT, "include", "ibmg3.h")


def test_three_dimensional_abi_exports_and_layout():
    """include/ibmg3.h: every declared symbol is exported and bound, and the
    ctypes structs match the C layout."""
    ibmg, L = _lib()
    syms = sorted(set(re.findall(r"^int\s+(ibmg3_\w+)\s*\(", open(HEADER3).read(), re.M)))
    assert syms == sorted(ibmg.EXPORTS3)
    out = subprocess.run(["nm", "-D", "--defined-only", ibmg.LIB_PATH], capture_output=True, text=True).stdout
    for s in syms:
        assert hasattr(L, s) and re.search(rf"\bT {s}$", out, re.M), s
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "ibmg3.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(ibmg3_problem), sizeof(ibmg3_opts),
         offsetof(ibmg3_problem, fiber_offsets), offsetof(ibmg3_problem, K), offsetof(ibmg3_problem, delta),
         offsetof(ibmg3_opts, rtol), offsetof(ibmg3_opts, omega));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        got = list(map(int, subprocess.run([exe], capture_output=True, text=True).stdout.split()))
    P, O = ibmg.ibmg3_problem, ibmg.ibmg3_opts
    assert got == [C.sizeof(P), C.sizeof(O), P.fiber_offsets.offset, P.K.offset, P.delta.offset, O.rtol.offset,
                   O.omega.offset]


def _create3(N=32, levels=4, box=4, offs=(0, 40, 80), **kw):
    ibmg, L = _lib()
    o = (C.c_int32 * len(offs))(*offs)
    prob = ibmg.ibmg3_problem(N, kw.get("rho", 1.0), kw.get("mu", 1.0), offs[-1], len(offs) - 1,
                              C.cast(o, C.POINTER(C.c_int32)), kw.get("K", 1e3), kw.get("delta", 0))
    opts = ibmg.ibmg3_opts(levels, box, kw.get("nu1", 1), kw.get("nu2", 1), kw.get("maxit", 100),
                           kw.get("rtol", 1e-8), kw.get("omega", 1.0))
    h = C.c_void_p()
    rc = L.ibmg3_create(C.byref(h), C.byref(prob), C.byref(opts), None)
    return rc, h, L


def test_three_dimensional_create_validation_and_workspace():
    """Shapes the 3-D handle accepts and rejects (no device work): N a power
    of two in 8..128, box 2 or 4 with an even number of boxes per side on
    every smoothed level, a coarsest grid of 2 to 8 cells, fibres of at least
    3 points; the workspace grows with the grid and holds one 304 x 304
    inverse per box of the smoothed levels with structure."""
    rc, h, L = _create3()
    assert rc == 0
    nb = C.c_size_t()
    assert L.ibmg3_workspace_bytes(h, C.byref(nb)) == 0
    boxes = 8 ** 3 + 4 ** 3 + 2 ** 3      # the three smoothed levels of 32^3 with 4^3 boxes
    assert nb.value > boxes * 304 * 304 * 8
    L.ibmg3_destroy(h)
    rc, h, L = _create3(K=0.0)
    nb0 = C.c_size_t()
    L.ibmg3_workspace_bytes(h, C.byref(nb0))
    assert nb0.value < nb.value
    L.ibmg3_destroy(h)
    invalid = (dict(N=24), dict(N=4, levels=2), dict(box=3),
               dict(levels=2), dict(levels=3),      # coarsest 16 and 8 cells (at most 4)
               dict(levels=5),                      # level 4 smoothed with one box per side
               dict(levels=6), dict(offs=(0, 2)), dict(offs=(0, 40, 30)), dict(rho=0.0), dict(omega=1.5),
               dict(maxit=0), dict(nu1=0, nu2=0), dict(delta=3))
    for kw in invalid:
        rc, h, L = _create3(**kw)
        assert rc == -1, kw
    valid = (dict(levels=4), dict(N=64, levels=5), dict(N=16, levels=3), dict(N=8, levels=2),
             dict(N=16, levels=3, box=2), dict(N=8, levels=2, box=2), dict(N=8, levels=2, box=4),
             dict(N=16, levels=4, box=2))
    for kw in valid:
        rc, h, L = _create3(**kw)
        assert rc == 0, kw
        L.ibmg3_destroy(h)
