"""Thin ctypes binding of libibmg.so (include/ibmg.h).

Argument marshalling only: every arithmetic step runs in the gfx950 kernels
of the library.  PyTorch supplies device memory (the workspace and the
caller's tensors) and the HIP stream.  The functions keep the C names; the
`Solver` class bundles a handle with its workspace tensor.

The library must be built (python -m paper_1311_5614_amd.build); importing
this module raises if libibmg.so is missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libibmg.so")

IBMG_OK, IBMG_NOT_CONVERGED = 0, 1
IBMG_EINVAL, IBMG_ESHAPE, IBMG_EHIP, IBMG_ENOMEM, IBMG_ENONFINITE, IBMG_ESTATE = -1, -2, -3, -4, -5, -6
IBMG_DELTA_IB4, IBMG_DELTA_COS4 = 0, 1
IBMG_FP64, IBMG_FP32 = 0, 1
IBMG_GUESS_ZERO, IBMG_GUESS_PREV = 0, 1
IBMG_IMPLICIT, IBMG_EXPLICIT = 0, 1
IBMG_SOLVER_FGMRES, IBMG_SOLVER_MG = 0, 1
IBMG_KERNEL_BOX, IBMG_KERNEL_RES, IBMG_KERNEL_MULTIDOT, IBMG_KERNEL_UPDATE = 0, 1, 2, 3
IBMG_KERNEL_DOT2, IBMG_KERNEL_UPDATE2 = 4, 5
IBMG_ORTH_CGS2, IBMG_ORTH_DCGS2 = 0, 1
IBMG_PERIODIC, IBMG_CAVITY = 0, 1
IBMG_GUESS_RECORD, IBMG_GUESS_EXTRAP, IBMG_GUESS_LEARNED = 0, 1, 2

EXPORTS = [
    "ibmg_create", "ibmg_workspace_bytes", "ibmg_bind_workspace", "ibmg_destroy",
    "ibmg_status_string", "ibmg_set_timing", "ibmg_phase_timing", "ibmg_box_bench", "ibmg_setup", "ibmg_step",
    "ibmg_rhs", "ibmg_solve", "ibmg_apply", "ibmg_residual", "ibmg_smooth", "ibmg_restrict",
    "ibmg_prolong_add", "ibmg_coarse_solve", "ibmg_vcycle", "ibmg_box_matrix",
    "ibmg_fiber_force", "ibmg_spread", "ibmg_interp",
    "ibmg_batch_create", "ibmg_batch_workspace_bytes", "ibmg_batch_bind_workspace", "ibmg_batch_step",
    "ibmg_batch_set_graph", "ibmg_batch_rounds", "ibmg_batch_destroy", "ibmg_step_x0",
    "ibmg_cnn_create", "ibmg_cnn_workspace_bytes", "ibmg_cnn_bind_workspace", "ibmg_cnn_set_params",
    "ibmg_cnn_get_params", "ibmg_cnn_set_scales", "ibmg_cnn_get_scales", "ibmg_cnn_record", "ibmg_cnn_pairs",
    "ibmg_cnn_train", "ibmg_cnn_infer", "ibmg_cnn_loss_grad", "ibmg_cnn_destroy", "ibmg_spread_noalloc",
    "ibmg_kernel_bench", "ibmg_guess_step", "ibmg_guess_reset", "ibmg_guess_get_increment",
    "ibmg_guess_set_increment",
]

EXPORTS3 = [
    "ibmg3_create", "ibmg3_workspace_bytes", "ibmg3_bind_workspace", "ibmg3_destroy", "ibmg3_setup",
    "ibmg3_apply", "ibmg3_restrict", "ibmg3_prolong_add", "ibmg3_box_matrix", "ibmg3_smooth", "ibmg3_vcycle",
    "ibmg3_rhs", "ibmg3_solve", "ibmg3_step", "ibmg3_box_counts",
]


class ibmg_problem(C.Structure):
    _fields_ = [("N", C.c_int32), ("rho", C.c_double), ("mu", C.c_double),
                ("n_points", C.c_int32), ("n_fibers", C.c_int32),
                ("fiber_offsets", C.POINTER(C.c_int32)), ("K", C.c_double), ("delta", C.c_int32),
                ("domain", C.c_int32)]


class ibmg_opts(C.Structure):
    _fields_ = [("levels", C.c_int32), ("box", C.c_int32), ("nu1", C.c_int32), ("nu2", C.c_int32),
                ("maxit", C.c_int32), ("rtol", C.c_double), ("vcycle_prec", C.c_int32),
                ("guess", C.c_int32), ("colours", C.c_int32), ("tail_max", C.c_int32),
                ("restart", C.c_int32), ("colours_from", C.c_int32), ("scheme", C.c_int32),
                ("solver", C.c_int32), ("omega", C.c_double), ("orth", C.c_int32)]


class ibmg_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("fallback", C.c_int32),
                ("guess_rejected", C.c_int32), ("rel_resid_est", C.c_double),
                ("rel_resid_true", C.c_double), ("bnorm", C.c_double), ("t_setup_ms", C.c_double),
                ("t_solve_ms", C.c_double), ("t_step_ms", C.c_double), ("guess_alpha", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ibmg3_problem(C.Structure):
    _fields_ = [("N", C.c_int32), ("rho", C.c_double), ("mu", C.c_double), ("M", C.c_int32),
                ("nfib", C.c_int32), ("fiber_offsets", C.POINTER(C.c_int32)), ("K", C.c_double),
                ("delta", C.c_int32)]


class ibmg3_opts(C.Structure):
    _fields_ = [("levels", C.c_int32), ("box", C.c_int32), ("nu1", C.c_int32), ("nu2", C.c_int32),
                ("maxit", C.c_int32), ("rtol", C.c_double), ("omega", C.c_double)]


def load(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_1311_5614_amd.build`")
    lib = C.CDLL(path)
    vp, i32, dbl, sz = C.c_void_p, C.c_int, C.c_double, C.c_size_t
    sig = {
        "ibmg_create": [C.POINTER(vp), C.POINTER(ibmg_problem), C.POINTER(ibmg_opts), vp],
        "ibmg_workspace_bytes": [vp, C.POINTER(sz)],
        "ibmg_bind_workspace": [vp, vp, sz],
        "ibmg_destroy": [vp],
        "ibmg_status_string": [i32],
        "ibmg_set_timing": [vp, i32],
        "ibmg_phase_timing": [vp, C.POINTER(dbl), C.POINTER(C.c_int64), C.POINTER(dbl)],
        "ibmg_box_bench": [vp, i32, i32, i32, C.POINTER(dbl), C.POINTER(dbl)],
        "ibmg_setup": [vp, dbl, vp],
        "ibmg_step": [vp, dbl, vp, vp, vp, vp, vp, vp, C.POINTER(ibmg_stats)],
        "ibmg_rhs": [vp, vp, vp, vp, vp, vp],
        "ibmg_solve": [vp, vp, vp, C.POINTER(ibmg_stats)],
        "ibmg_apply": [vp, i32, vp, vp],
        "ibmg_residual": [vp, i32, vp, vp, vp],
        "ibmg_smooth": [vp, i32, vp, vp, i32],
        "ibmg_restrict": [vp, i32, vp, vp],
        "ibmg_prolong_add": [vp, i32, vp, vp],
        "ibmg_coarse_solve": [vp, vp, vp],
        "ibmg_vcycle": [vp, vp, vp],
        "ibmg_box_matrix": [vp, i32, i32, i32, vp],
        "ibmg_fiber_force": [vp, vp, vp],
        "ibmg_spread": [vp, vp, vp, vp, vp],
        "ibmg_interp": [vp, vp, vp, vp, vp],
        "ibmg_batch_create": [C.POINTER(vp), i32, C.POINTER(ibmg_problem), C.POINTER(ibmg_opts), vp],
        "ibmg_batch_workspace_bytes": [vp, C.POINTER(sz)],
        "ibmg_batch_bind_workspace": [vp, vp, sz],
        "ibmg_batch_step": [vp, C.POINTER(dbl), C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                            C.POINTER(vp), C.POINTER(vp), C.POINTER(ibmg_stats)],
        "ibmg_batch_set_graph": [vp, i32],
        "ibmg_batch_rounds": [vp, C.POINTER(C.c_int64)],
        "ibmg_batch_destroy": [vp],
        "ibmg_step_x0": [vp, dbl, vp, vp, vp, vp, vp, vp, vp, C.POINTER(ibmg_stats)],
        "ibmg_cnn_create": [C.POINTER(vp), i32, i32, vp],
        "ibmg_cnn_workspace_bytes": [vp, C.POINTER(sz)],
        "ibmg_cnn_bind_workspace": [vp, vp, sz],
        "ibmg_cnn_set_params": [vp, C.POINTER(C.c_float)],
        "ibmg_cnn_get_params": [vp, C.POINTER(C.c_float)],
        "ibmg_cnn_set_scales": [vp, C.POINTER(C.c_float), C.POINTER(C.c_float)],
        "ibmg_cnn_get_scales": [vp, C.POINTER(C.c_float)],
        "ibmg_cnn_record": [vp, vp, vp],
        "ibmg_cnn_pairs": [vp, C.POINTER(C.c_int32)],
        "ibmg_cnn_train": [vp, i32, C.c_float, C.POINTER(C.c_float), C.POINTER(C.c_float)],
        "ibmg_cnn_infer": [vp, vp, vp],
        "ibmg_cnn_loss_grad": [vp, vp, vp, C.POINTER(C.c_float), C.POINTER(C.c_float)],
        "ibmg_cnn_destroy": [vp],
        "ibmg_spread_noalloc": [i32, i32, i32, vp, vp, vp, vp, vp],
        "ibmg_kernel_bench": [vp, i32, i32, i32, i32, C.POINTER(dbl), C.POINTER(dbl)],
        "ibmg_guess_step": [vp, vp, i32, dbl, vp, vp, vp, vp, vp, vp, C.POINTER(ibmg_stats)],
        "ibmg_guess_reset": [vp],
        "ibmg_guess_get_increment": [vp, vp],
        "ibmg_guess_set_increment": [vp, vp],
    }
    sig.update({
        "ibmg3_create": [C.POINTER(vp), C.POINTER(ibmg3_problem), C.POINTER(ibmg3_opts), vp],
        "ibmg3_workspace_bytes": [vp, C.POINTER(sz)],
        "ibmg3_bind_workspace": [vp, vp, sz],
        "ibmg3_destroy": [vp],
        "ibmg3_setup": [vp, dbl, vp],
        "ibmg3_apply": [vp, i32, vp, vp],
        "ibmg3_restrict": [vp, i32, vp, vp],
        "ibmg3_prolong_add": [vp, i32, vp, vp],
        "ibmg3_box_matrix": [vp, i32, i32, i32, i32, vp],
        "ibmg3_smooth": [vp, i32, vp, vp, i32],
        "ibmg3_vcycle": [vp, vp, vp],
        "ibmg3_rhs": [vp, vp, vp, vp],
        "ibmg3_solve": [vp, vp, vp, C.POINTER(ibmg_stats)],
        "ibmg3_step": [vp, dbl, vp, vp, vp, C.POINTER(ibmg_stats)],
        "ibmg3_box_counts": [vp, i32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)],
    })
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_char_p if name == "ibmg_status_string" else C.c_int
    return lib


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


class IBMGError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {lib().ibmg_status_string(code).decode()} ({code})")


def _check(code, where, allow_not_converged=True):
    if code < 0 or (code > 0 and not allow_not_converged):
        raise IBMGError(code, where)
    return code


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("contiguous float64 tensor expected")
    return C.c_void_p(t.data_ptr())


@dataclass
class Config:
    N: int
    levels: int
    K: float = 0.0
    rho: float = 1.0
    mu: float = 1.0
    delta: int = IBMG_DELTA_IB4
    box: int = 4
    nu1: int = 2
    nu2: int = 2
    maxit: int = 100
    rtol: float = 1e-8
    prec: int = IBMG_FP64
    guess: int = IBMG_GUESS_ZERO
    colours: int = 2
    tail_max: int = 0
    restart: int = 0
    colours_from: int = 0
    scheme: int = 0
    solver: int = 0
    omega: float = 1.0
    orth: int = 0
    domain: int = 0


def _problem(cfg: Config, fiber_offsets):
    """(ibmg_problem, ibmg_opts, keep-alive offsets array, M) of a config."""
    offs = [int(x) for x in (fiber_offsets if fiber_offsets is not None else [0])]
    M = offs[-1] if len(offs) > 1 else 0
    arr = (C.c_int32 * len(offs))(*offs)
    prob = ibmg_problem(cfg.N, cfg.rho, cfg.mu, M, max(0, len(offs) - 1),
                        C.cast(arr, C.POINTER(C.c_int32)), cfg.K, cfg.delta, cfg.domain)
    opts = ibmg_opts(cfg.levels, cfg.box, cfg.nu1, cfg.nu2, cfg.maxit, cfg.rtol, cfg.prec,
                     cfg.guess, cfg.colours, cfg.tail_max, cfg.restart, cfg.colours_from, cfg.scheme, cfg.solver, cfg.omega,
                     cfg.orth)
    return prob, opts, arr, M


class Solver:
    """One handle plus its torch-owned workspace on `device`."""

    def __init__(self, cfg: Config, fiber_offsets, device="cuda:0", stream=None):
        L = lib()
        self.cfg = cfg
        self.device = torch.device(device)
        prob, opts, self._offs, self.M = _problem(cfg, fiber_offsets)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(L.ibmg_create(C.byref(h), C.byref(prob), C.byref(opts),
                             C.c_void_p(self.stream.cuda_stream)), "ibmg_create")
        self.h = h
        nbytes = C.c_size_t()
        _check(L.ibmg_workspace_bytes(h, C.byref(nbytes)), "ibmg_workspace_bytes")
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        _check(L.ibmg_bind_workspace(h, C.c_void_p(self.workspace.data_ptr()), nbytes.value),
               "ibmg_bind_workspace")

    def close(self):
        if getattr(self, "h", None):
            lib().ibmg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- thin wrappers (same names as the C ABI without the prefix)
    def setup(self, dt, X):
        return _check(lib().ibmg_setup(self.h, float(dt), _ptr(X)), "ibmg_setup")

    def step(self, dt, u, v, p, X, g_u=None, g_v=None):
        st = ibmg_stats()
        code = _check(lib().ibmg_step(self.h, float(dt), _ptr(u), _ptr(v), _ptr(p), _ptr(X),
                                      _ptr(g_u), _ptr(g_v), C.byref(st)), "ibmg_step")
        d = st.as_dict()
        d["status"] = code
        return d

    def step_x0(self, dt, u, v, p, X, x0, g_u=None, g_v=None):
        st = ibmg_stats()
        code = _check(lib().ibmg_step_x0(self.h, float(dt), _ptr(u), _ptr(v), _ptr(p), _ptr(X),
                                         _ptr(g_u), _ptr(g_v), _ptr(x0), C.byref(st)), "ibmg_step_x0")
        d = st.as_dict()
        d["status"] = code
        return d

    def guess_step(self, net, mode, dt, u, v, p, X, g_u=None, g_v=None):
        """One step with the learned-iterate machinery of `net` (ibmg_guess_step;
        mode IBMG_GUESS_RECORD / _EXTRAP / _LEARNED)."""
        st = ibmg_stats()
        code = _check(lib().ibmg_guess_step(self.h, net.h, int(mode), float(dt), _ptr(u), _ptr(v), _ptr(p),
                                            _ptr(X), _ptr(g_u), _ptr(g_v), C.byref(st)), "ibmg_guess_step")
        d = st.as_dict()
        d["status"] = code
        return d

    def rhs(self, u, v, g_u=None, g_v=None):
        N = self.cfg.N
        b = torch.empty(3 * N * N, dtype=torch.float64, device=self.device)
        _check(lib().ibmg_rhs(self.h, _ptr(u), _ptr(v), _ptr(g_u), _ptr(g_v), _ptr(b)), "ibmg_rhs")
        return b

    def solve(self, b, w):
        st = ibmg_stats()
        code = _check(lib().ibmg_solve(self.h, _ptr(b), _ptr(w), C.byref(st)), "ibmg_solve")
        d = st.as_dict()
        d["status"] = code
        return d

    def _n3(self, level):
        Nl = self.cfg.N >> level
        return 3 * Nl * Nl

    def apply(self, level, w):
        y = torch.empty(self._n3(level), dtype=torch.float64, device=self.device)
        _check(lib().ibmg_apply(self.h, level, _ptr(w), _ptr(y)), "ibmg_apply")
        return y

    def residual(self, level, b, w):
        r = torch.empty(self._n3(level), dtype=torch.float64, device=self.device)
        _check(lib().ibmg_residual(self.h, level, _ptr(b), _ptr(w), _ptr(r)), "ibmg_residual")
        return r

    def smooth(self, level, b, w, sweeps=1):
        _check(lib().ibmg_smooth(self.h, level, _ptr(b), _ptr(w), sweeps), "ibmg_smooth")
        return w

    def restrict(self, level, fine):
        c = torch.empty(self._n3(level + 1), dtype=torch.float64, device=self.device)
        _check(lib().ibmg_restrict(self.h, level, _ptr(fine), _ptr(c)), "ibmg_restrict")
        return c

    def prolong_add(self, level, coarse, fine):
        _check(lib().ibmg_prolong_add(self.h, level, _ptr(coarse), _ptr(fine)), "ibmg_prolong_add")
        return fine

    def coarse_solve(self, b):
        w = torch.empty_like(b)
        _check(lib().ibmg_coarse_solve(self.h, _ptr(b), _ptr(w)), "ibmg_coarse_solve")
        return w

    def vcycle(self, r):
        z = torch.empty_like(r)
        _check(lib().ibmg_vcycle(self.h, _ptr(r), _ptr(z)), "ibmg_vcycle")
        return z

    def box_matrix(self, level, bx, by):
        n = self.cfg.box
        nd = 2 * n * (n + 1) + n * n
        out = torch.empty(nd * nd, dtype=torch.float64, device=self.device)
        _check(lib().ibmg_box_matrix(self.h, level, bx, by, _ptr(out)), "ibmg_box_matrix")
        return out.view(nd, nd)

    def fiber_force(self, X):
        G = torch.empty_like(X)
        _check(lib().ibmg_fiber_force(self.h, _ptr(X), _ptr(G)), "ibmg_fiber_force")
        return G

    def spread(self, X, G):
        N = self.cfg.N
        fu = torch.empty(N, N, dtype=torch.float64, device=self.device)
        fv = torch.empty(N, N, dtype=torch.float64, device=self.device)
        _check(lib().ibmg_spread(self.h, _ptr(X), _ptr(G), _ptr(fu), _ptr(fv)), "ibmg_spread")
        return fu, fv

    def interp(self, X, u, v):
        U = torch.empty_like(X)
        _check(lib().ibmg_interp(self.h, _ptr(X), _ptr(u), _ptr(v), _ptr(U)), "ibmg_interp")
        return U

    def box_bench(self, level, colour, reps):
        us, by = C.c_double(), C.c_double()
        _check(lib().ibmg_box_bench(self.h, level, colour, reps, C.byref(us), C.byref(by)), "ibmg_box_bench")
        return us.value, by.value

    def kernel_bench(self, kernel, level, arg, reps):
        """(mean microseconds per launch, algorithmic bytes per launch) of one
        hot-path kernel replayed `reps` times (ibmg_kernel_bench)."""
        us, by = C.c_double(), C.c_double()
        _check(lib().ibmg_kernel_bench(self.h, kernel, level, arg, reps, C.byref(us), C.byref(by)),
               "ibmg_kernel_bench")
        return us.value, by.value

    def set_timing(self, on=True):
        _check(lib().ibmg_set_timing(self.h, 1 if on else 0), "ibmg_set_timing")

    def phase_timing(self):
        ms, n, by = C.c_double(), C.c_int64(), C.c_double()
        _check(lib().ibmg_phase_timing(self.h, C.byref(ms), C.byref(n), C.byref(by)), "ibmg_phase_timing")
        return dict(total_ms=ms.value, launches=n.value, bytes=by.value)


class Batch:
    """A batch handle (ibmg_batch_*) over several problems plus its workspace."""

    def __init__(self, cfgs, fiber_offsets, device="cuda:0", stream=None):
        L = lib()
        self.cfgs = list(cfgs)
        self.device = torch.device(device)
        P = len(self.cfgs)
        parts = [_problem(c, o) for c, o in zip(self.cfgs, fiber_offsets)]
        self._keep = [pt[2] for pt in parts]
        self.M = [pt[3] for pt in parts]
        probs = (ibmg_problem * P)(*[pt[0] for pt in parts])
        opts = (ibmg_opts * P)(*[pt[1] for pt in parts])
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(L.ibmg_batch_create(C.byref(h), P, probs, opts, C.c_void_p(self.stream.cuda_stream)),
               "ibmg_batch_create")
        self.h = h
        nbytes = C.c_size_t()
        _check(L.ibmg_batch_workspace_bytes(h, C.byref(nbytes)), "ibmg_batch_workspace_bytes")
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        _check(L.ibmg_batch_bind_workspace(h, C.c_void_p(self.workspace.data_ptr()), nbytes.value),
               "ibmg_batch_bind_workspace")

    def close(self):
        if getattr(self, "h", None):
            lib().ibmg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _ptrs(ts, allow_none=False):
        arr = (C.c_void_p * len(ts))()
        for i, t in enumerate(ts):
            if t is None:
                if not allow_none:
                    raise ValueError("device tensor expected")
                arr[i] = None
            else:
                arr[i] = _ptr(t).value
        return arr

    def step(self, dts, us, vs, ps, Xs, g_us=None, g_vs=None):
        P = len(self.cfgs)
        dt = (C.c_double * P)(*[float(x) for x in dts])
        st = (ibmg_stats * P)()
        gu = self._ptrs(g_us, True) if g_us is not None else None
        gv = self._ptrs(g_vs, True) if g_vs is not None else None
        code = _check(lib().ibmg_batch_step(self.h, dt, self._ptrs(us), self._ptrs(vs), self._ptrs(ps),
                                            self._ptrs(Xs, True), gu, gv, st), "ibmg_batch_step")
        out = []
        for i in range(P):
            d = st[i].as_dict()
            d["status"] = code
            out.append(d)
        return out

    def set_graph(self, on=True):
        _check(lib().ibmg_batch_set_graph(self.h, 1 if on else 0), "ibmg_batch_set_graph")

    def rounds(self):
        n = C.c_int64()
        _check(lib().ibmg_batch_rounds(self.h, C.byref(n)), "ibmg_batch_rounds")
        return n.value


CNN_PARAMS = 39331


class Cnn:
    """The warm-start network (ibmg_cnn_*) plus its workspace."""

    def __init__(self, N, max_pairs, device="cuda:0", stream=None):
        L = lib()
        self.N = N
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(L.ibmg_cnn_create(C.byref(h), N, max_pairs, C.c_void_p(self.stream.cuda_stream)), "ibmg_cnn_create")
        self.h = h
        nbytes = C.c_size_t()
        _check(L.ibmg_cnn_workspace_bytes(h, C.byref(nbytes)), "ibmg_cnn_workspace_bytes")
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        _check(L.ibmg_cnn_bind_workspace(h, C.c_void_p(self.workspace.data_ptr()), nbytes.value),
               "ibmg_cnn_bind_workspace")

    def reset(self):
        """Forget the previous step increment (ibmg_guess_reset)."""
        _check(lib().ibmg_guess_reset(self.h), "ibmg_guess_reset")

    def get_increment(self):
        dw = torch.empty(3 * self.N * self.N, dtype=torch.float64, device=self.device)
        _check(lib().ibmg_guess_get_increment(self.h, _ptr(dw)), "ibmg_guess_get_increment")
        return dw

    def set_increment(self, dw):
        _check(lib().ibmg_guess_set_increment(self.h, _ptr(dw)), "ibmg_guess_set_increment")

    def close(self):
        if getattr(self, "h", None):
            lib().ibmg_cnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _f32(a, n):
        import numpy as np
        a = np.ascontiguousarray(a, dtype=np.float32)
        if a.size != n:
            raise ValueError(f"{n} values expected")
        return a, a.ctypes.data_as(C.POINTER(C.c_float))

    def set_params(self, params):
        a, ptr = self._f32(params, CNN_PARAMS)
        _check(lib().ibmg_cnn_set_params(self.h, ptr), "ibmg_cnn_set_params")

    def get_params(self):
        import numpy as np
        out = np.empty(CNN_PARAMS, dtype=np.float32)
        _check(lib().ibmg_cnn_get_params(self.h, out.ctypes.data_as(C.POINTER(C.c_float))), "ibmg_cnn_get_params")
        return out

    def set_scales(self, s_in, s_out):
        a, pa = self._f32(s_in, 5)
        b, pb = self._f32(s_out, 3)
        _check(lib().ibmg_cnn_set_scales(self.h, pa, pb), "ibmg_cnn_set_scales")

    def get_scales(self):
        import numpy as np
        out = np.empty(8, dtype=np.float32)
        _check(lib().ibmg_cnn_get_scales(self.h, out.ctypes.data_as(C.POINTER(C.c_float))), "ibmg_cnn_get_scales")
        return out

    def record(self, in5, dw3):
        _check(lib().ibmg_cnn_record(self.h, _ptr(in5), _ptr(dw3)), "ibmg_cnn_record")

    def pairs(self):
        n = C.c_int32()
        _check(lib().ibmg_cnn_pairs(self.h, C.byref(n)), "ibmg_cnn_pairs")
        return n.value

    def train(self, epochs, lr):
        lf, ll = C.c_float(), C.c_float()
        _check(lib().ibmg_cnn_train(self.h, int(epochs), float(lr), C.byref(lf), C.byref(ll)), "ibmg_cnn_train")
        return lf.value, ll.value

    def infer(self, in5):
        out = torch.empty(3, self.N, self.N, dtype=torch.float64, device=self.device)
        _check(lib().ibmg_cnn_infer(self.h, _ptr(in5), _ptr(out)), "ibmg_cnn_infer")
        return out

    def loss_grad(self, in5, dw3):
        import numpy as np
        g = np.empty(CNN_PARAMS, dtype=np.float32)
        loss = C.c_float()
        _check(lib().ibmg_cnn_loss_grad(self.h, _ptr(in5), _ptr(dw3), C.byref(loss),
                                        g.ctypes.data_as(C.POINTER(C.c_float))), "ibmg_cnn_loss_grad")
        return loss.value, g


@dataclass
class Config3:
    """Problem and options of the three-dimensional solver (include/ibmg3.h)."""
    N: int
    levels: int
    K: float = 0.0
    rho: float = 1.0
    mu: float = 1.0
    delta: int = IBMG_DELTA_IB4
    box: int = 4
    nu1: int = 1
    nu2: int = 1
    maxit: int = 100
    rtol: float = 1e-8
    omega: float = 1.0


class Solver3:
    """An ibmg3 handle plus its torch-owned workspace on `device`."""

    def __init__(self, cfg: Config3, fiber_offsets, device="cuda:0", stream=None):
        L = lib()
        self.cfg = cfg
        self.device = torch.device(device)
        offs = [int(x) for x in (fiber_offsets if fiber_offsets is not None else [0])]
        self.M = offs[-1] if len(offs) > 1 else 0
        self._offs = (C.c_int32 * len(offs))(*offs)
        prob = ibmg3_problem(cfg.N, cfg.rho, cfg.mu, self.M, max(0, len(offs) - 1),
                             C.cast(self._offs, C.POINTER(C.c_int32)), cfg.K, cfg.delta)
        opts = ibmg3_opts(cfg.levels, cfg.box, cfg.nu1, cfg.nu2, cfg.maxit, cfg.rtol, cfg.omega)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(L.ibmg3_create(C.byref(h), C.byref(prob), C.byref(opts), C.c_void_p(self.stream.cuda_stream)),
               "ibmg3_create")
        self.h = h
        nbytes = C.c_size_t()
        _check(L.ibmg3_workspace_bytes(h, C.byref(nbytes)), "ibmg3_workspace_bytes")
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        _check(L.ibmg3_bind_workspace(h, C.c_void_p(self.workspace.data_ptr()), nbytes.value),
               "ibmg3_bind_workspace")

    def close(self):
        if getattr(self, "h", None):
            lib().ibmg3_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def n(self, level=0):
        Nl = self.cfg.N >> level
        return 4 * Nl ** 3

    def setup(self, dt, X):
        return _check(lib().ibmg3_setup(self.h, float(dt), _ptr(X)), "ibmg3_setup")

    def apply(self, level, x):
        y = torch.empty(self.n(level), dtype=torch.float64, device=self.device)
        _check(lib().ibmg3_apply(self.h, level, _ptr(x), _ptr(y)), "ibmg3_apply")
        return y

    def restrict(self, level, rf):
        rc = torch.empty(self.n(level + 1), dtype=torch.float64, device=self.device)
        _check(lib().ibmg3_restrict(self.h, level, _ptr(rf), _ptr(rc)), "ibmg3_restrict")
        return rc

    def prolong_add(self, level, ec, wf):
        _check(lib().ibmg3_prolong_add(self.h, level, _ptr(ec), _ptr(wf)), "ibmg3_prolong_add")
        return wf

    def box_matrix(self, level, bx, by, bz):
        n = self.cfg.box
        nd = 3 * (n + 1) * n * n + n ** 3
        out = torch.empty(nd, nd, dtype=torch.float64, device=self.device)
        _check(lib().ibmg3_box_matrix(self.h, level, bx, by, bz, _ptr(out)), "ibmg3_box_matrix")
        return out

    def smooth(self, level, b, w, sweeps=1):
        _check(lib().ibmg3_smooth(self.h, level, _ptr(b), _ptr(w), sweeps), "ibmg3_smooth")
        return w

    def vcycle(self, r):
        z = torch.empty_like(r)
        _check(lib().ibmg3_vcycle(self.h, _ptr(r), _ptr(z)), "ibmg3_vcycle")
        return z

    def rhs(self, uvw, X=None):
        b = torch.empty(self.n(0), dtype=torch.float64, device=self.device)
        _check(lib().ibmg3_rhs(self.h, _ptr(uvw), _ptr(X), _ptr(b)), "ibmg3_rhs")
        return b

    def solve(self, b, x):
        st = ibmg_stats()
        code = _check(lib().ibmg3_solve(self.h, _ptr(b), _ptr(x), C.byref(st)), "ibmg3_solve")
        d = st.as_dict()
        d["status"] = code
        return d

    def step(self, dt, uvw, p, X):
        st = ibmg_stats()
        code = _check(lib().ibmg3_step(self.h, float(dt), _ptr(uvw), _ptr(p), _ptr(X), C.byref(st)), "ibmg3_step")
        d = st.as_dict()
        d["status"] = code
        return d

    def box_counts(self, level):
        own, total = C.c_int32(), C.c_int32()
        _check(lib().ibmg3_box_counts(self.h, level, C.byref(own), C.byref(total)), "ibmg3_box_counts")
        return own.value, total.value
