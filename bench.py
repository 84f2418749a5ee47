"""Benchmark: implicit IB time steps per second on one MI355X.

Headline workload (default, --workload c3): the 1024x1024 eight-ring
instance -- 8 elastic rings of 2048 points (16384 Lagrangian points), K = 1e6,
dt = 500 x the explicit stability limit, 7 multigrid levels, every solve to
relative residual 1e-8.  One bench step is one implicit time step of that
trajectory (setup, right-hand side, FGMRES solve, position update).  Two forms
are timed from the same initial state, each `--repeats` times (median
reported):

  plain   FP64 V-cycle inside FP64 FGMRES, default schedule (4x4 boxes,
          checkerboard order, V(2,2), no restart below the 200 cap);
  chosen  the schedule the autotuner table gives for this workload
          (schedules.json: FP32 V-cycle inside FP64 FGMRES, box order,
          sweeps, tail, restart), the value reported.

Inputs are resident in HBM before timing starts; every timed step includes
its setup.  Also reported: iterations per solve and steps that missed rtol
per form, the HIP-event roofline of the dominant kernel, the 4096x4096 plain
V-cycle bandwidth probe, the oracle timed on the host on a bounded sample of
the same workload, and (unless --no-extras) the 256x256 stiffness sweep and
the 64-problem batch as extra keys.

Other workloads: --workload c2 (256x256 sweep, forms concurrent / plain /
fp32 / tuned), c4 (64-problem batch), c5 (512x512 learned warm start), c1,
cavity (the walled test problem), mgsolver, efficiency, d3 (the
three-dimensional form).

python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--workload c3|c2|c4|c5|c1]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MAXIT = 200          # Krylov basis of the batch and the learned trajectory: FGMRES(200)
MAXIT_TOTAL = 1000   # iteration cap of every solve; the 256x256 sweep keeps a basis of this size (no
                     # restart: restarted FGMRES stagnates on its hardest steps)
C3_BASIS = 600       # Krylov basis of both 1024x1024 forms (30 GB with the preconditioned directions)
BOX_REPS = 200   # back-to-back box launches timed for the roofline
METRIC = "IB time-steps/sec and FGMRES iters/solve at rel resid 1e-8, plain vs chosen"


BOX_SOURCES = ("paper_1311_5614_amd/csrc/level_ops.h", "paper_1311_5614_amd/csrc/mg.hip",
               "paper_1311_5614_amd/csrc/common.h", "paper_1311_5614_amd/csrc/krylov.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_box_traffic.txt")


def box_source_hash():
    import hashlib
    h = hashlib.sha1()
    for f in BOX_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(launch):
    """HBM bytes per launch of the timed box launch from the committed
    rocprofv3 counter summary (FETCH_SIZE, WRITE_SIZE scaled by the copy
    calibration), or None if the summary is for another launch or the box
    kernel's sources changed since the counters were taken."""
    if not launch or not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.strip().split("=", 1)
                kv[k] = v
    if kv.get("kernel_source_sha1") != box_source_hash():
        return None
    if kv.get("launch") != f"k_box<{'float' if launch['prec'] == 'fp32' else 'double'}> level 0 grid {launch['grid']}":
        return None
    return float(kv["traffic_bytes"])


def load_dt(key):
    with open(os.path.join(ROOT, "tests", "golden", "workload_dt.json")) as f:
        return json.load(f)[key]


def workloads(name):
    import ibgen
    if name == "c2":
        cases = ibgen.config_c2_cases()
        dts = load_dt("c2")
        return cases, [d["dt"] for d in dts]
    if name == "c1":
        return [ibgen.config_c1()], [load_dt("c1")[0]["dt"]]
    if name == "c3":
        return [ibgen.config_c3()], [load_dt("c3")[0]["dt"]]
    if name == "c4":
        return ibgen.config_c4(), [d["dt"] for d in load_dt("c4")]
    raise SystemExit(f"unknown workload {name}")


def schedule_key(workload, w):
    return f"{w.K:.0e}-{int(w.dt_factor)}" if workload == "c2" else str(w.N)


def tuned(workload, cases):
    """Copies of the cases with the autotuned schedule of their class
    (paper_1311_5614_amd/schedules.json) and the V-cycle precision it chose."""
    import copy
    from paper_1311_5614_amd import autotune
    table = autotune.load().get(workload, {})
    out, precs = [], []
    for w in cases:
        sch = table.get(schedule_key(workload, w))
        c = copy.copy(w)
        if sch is None:
            out.append(c)
            precs.append(1)
            continue
        c.levels, c.tail_max, c.nu1, c.nu2, c.colours = (sch["levels"], sch["tail_max"], sch["nu1"], sch["nu2"],
                                                         sch["colours"])
        c.box = sch.get("box", 4)
        out.append(c)
        precs.append(sch.get("prec", 1))
    return out, precs


class Run:
    """Device state of one trajectory plus its solver handle."""

    def __init__(self, w, dt, prec, dev, stream=None):
        import torch
        from paper_1311_5614_amd import ibmg
        self.w, self.dt = w, dt
        cfg = ibmg.Config(N=w.N, levels=w.levels, K=w.K, rho=w.rho, mu=w.mu, box=w.box, nu1=w.nu1,
                          nu2=w.nu2, maxit=MAXIT_TOTAL, restart=0, rtol=w.rtol, prec=prec,
                          colours=getattr(w, "colours", 2), tail_max=getattr(w, "tail_max", 0),
                          colours_from=getattr(w, "colours_from", 0))
        self.s = ibmg.Solver(cfg, w.fiber_offsets, dev, stream=stream)
        t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev).contiguous()
        self.X0 = t(w.X)
        self.gu = t(w.g_u) if w.g_u is not None else None
        self.gv = t(w.g_v) if w.g_v is not None else None
        N = w.N
        self.u = torch.zeros(N, N, dtype=torch.float64, device=dev)
        self.v = torch.zeros_like(self.u)
        self.p = torch.zeros_like(self.u)
        self.X = self.X0.clone()

    def reset(self):
        self.u.zero_(); self.v.zero_(); self.p.zero_()
        self.X.copy_(self.X0)

    def step(self):
        return self.s.step(self.dt, self.u, self.v, self.p, self.X, self.gu, self.gv)


class BatchRun:
    """Every trajectory of the workload in one batch handle."""

    def __init__(self, ws, dts, prec, dev):
        import torch
        from paper_1311_5614_amd import ibmg
        self.ws, self.dts = ws, dts
        cfgs = [ibmg.Config(N=w.N, levels=w.levels, K=w.K, rho=w.rho, mu=w.mu, box=w.box, nu1=w.nu1,
                            nu2=w.nu2, maxit=MAXIT_TOTAL, restart=MAXIT, rtol=w.rtol, prec=prec,
                            colours=getattr(w, "colours", 2), tail_max=getattr(w, "tail_max", 0))
                for w in ws]
        self.b = ibmg.Batch(cfgs, [w.fiber_offsets for w in ws], dev)
        t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev).contiguous()
        self.X0 = [t(w.X) for w in ws]
        self.g = [(t(w.g_u), t(w.g_v)) if w.g_u is not None else (None, None) for w in ws]
        z = lambda w: torch.zeros(w.N, w.N, dtype=torch.float64, device=dev)
        self.u = [z(w) for w in ws]
        self.v = [z(w) for w in ws]
        self.p = [z(w) for w in ws]
        self.X = [x.clone() for x in self.X0]

    def reset(self):
        for a in self.u + self.v + self.p:
            a.zero_()
        for x, x0 in zip(self.X, self.X0):
            x.copy_(x0)

    def step(self):
        return self.b.step(self.dts, self.u, self.v, self.p, self.X, [g[0] for g in self.g],
                           [g[1] for g in self.g])


def timed_batch(br, steps, warmup):
    import torch
    br.reset()
    for _ in range(warmup):
        br.step()
    br.reset()
    torch.cuda.synchronize()
    its, conv = [], []
    r0 = br.b.rounds()
    phases = [0.0, 0.0, 0.0]
    t0 = time.perf_counter()
    for _ in range(steps):
        out = br.step()
        for st in out:
            its.append(st["iters"])
            conv.append(st["converged"])
        phases[0] += out[0]["t_setup_ms"]
        phases[1] += out[0]["t_solve_ms"]
        phases[2] += out[0]["t_step_ms"]
    torch.cuda.synchronize()
    print(f"[bench] batch host phases per step: setup {phases[0] / steps:.1f} ms, solve {phases[1] / steps:.1f} ms, "
          f"step {phases[2] / steps:.1f} ms", file=sys.stderr, flush=True)
    return time.perf_counter() - t0, its, conv, br.b.rounds() - r0


def timed_concurrent(runs, steps, warmup):
    """Like timed(), but every trajectory advances in a host thread of its own
    on a stream of its own (the library's calls release the interpreter, and
    each solve's small, latency-bound launches overlap with the others')."""
    import threading
    import torch
    from paper_1311_5614_amd.ibmg import IBMGError
    for r in runs:
        r.reset()
    for _ in range(warmup):          # graph capture, sequentially
        for r in runs:
            try:
                r.step()
            except IBMGError:
                pass
    for r in runs:
        r.reset()
    torch.cuda.synchronize()
    per_case = [[] for _ in runs]
    conv_case = [[] for _ in runs]
    failed = {}

    case_s = [0.0] * len(runs)

    def work(c, r):
        t_start = time.perf_counter()
        for s in range(steps):
            try:
                st = r.step()
            except IBMGError as e:
                failed[c] = f"step {s}: {e}"
                return
            per_case[c].append(st["iters"])
            conv_case[c].append(st["converged"])
        case_s[c] = time.perf_counter() - t_start

    threads = [threading.Thread(target=work, args=(c, r)) for c, r in enumerate(runs)]
    t0 = time.perf_counter()
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    its = [i for pc in per_case for i in pc]
    conv = [c for cc in conv_case for c in cc]
    if failed:
        conv.append(0)
        its.append(0)
    timed.per_case = per_case
    timed.failed = failed
    timed.case_s = case_s
    return t, its, conv, None


def timed(runs, steps, warmup, timing=False):
    """Warm up, reset every trajectory, then time `steps` steps of all of them.
    With timing set, the box kernels are event-timed (eager launches instead of
    the replayed V-cycle graph)."""
    import torch
    for r in runs:
        r.reset()
    from paper_1311_5614_amd.ibmg import IBMGError as _E
    for _ in range(warmup):
        for r in runs:
            try:
                r.step()
            except _E:
                pass
    for r in runs:
        r.reset()
        r.s.set_timing(timing)
    torch.cuda.synchronize()
    from paper_1311_5614_amd.ibmg import IBMGError
    its, conv = [], []
    per_case = [[] for _ in runs]
    failed = {}
    t0 = time.perf_counter()
    for s in range(steps):
        for c, r in enumerate(runs):
            if c in failed:
                continue
            try:
                st = r.step()
            except IBMGError as e:
                # e.g. a trajectory whose fibre neighbours drift apart beyond
                # the elasticity window: it stops here, reported as failed
                failed[c] = f"step {s}: {e}"
                print(f"[bench] trajectory {c} ({r.w.name}) stopped at step {s}: {e}", file=sys.stderr, flush=True)
                continue
            its.append(st["iters"])
            conv.append(st["converged"])
            per_case[c].append(st["iters"])
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    timed.per_case = per_case
    if failed:
        conv.append(0)   # a stopped trajectory counts as one unconverged step
        its.append(0)
    timed.failed = failed
    ph = None
    if timing:
        tot = dict(total_ms=0.0, launches=0, bytes=0.0)
        for r in runs:
            d = r.s.phase_timing()
            for k in tot:
                tot[k] += d[k]
            r.s.set_timing(False)
        ph = tot
    return t, its, conv, ph


def cpu_baseline(w, dt, budget_note, steps=3):
    """Oracle (plain numpy/scipy, FP64): `steps` time steps of one case."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import step as ostep
    N = w.N
    u = v = p = np.zeros((N, N))
    X = w.X
    its = []
    with threadpool_limits(1):
        t0 = time.perf_counter()
        for _ in range(steps):
            o = ostep.step(u, v, p, X, w.fiber_offsets, w.K, dt, w.levels, w.rho, w.mu, w.box, w.nu1,
                           w.nu2, w.rtol, g_u=w.g_u, g_v=w.g_v)
            u, v, p, X = o.u, o.v, o.p, o.X
            its.append(o.iters)
        t = time.perf_counter() - t0
    return {"value": steps / t, "unit": "time-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} implicit steps of {w.name} ({its} FGMRES iterations, {t:.1f} s); "
                      f"1 BLAS thread; {budget_note}"}


def run_learned(args, dev):
    """The 512x512 learned-warm-start trajectory.  Steps 1..H start from w^n
    and record (features, target) pairs in the network handle (the target
    being the change of the step increment, dw^n - dw^{n-1}); the network is
    trained on the GPU; then steps H+1..2H run four ways from the same state
    at step H: learned (x0 = w^n + dw^{n-1} + net(features), guarded by the
    minimal-residual weight alpha), extrapolation alone (x0 = w^n + dw^{n-1},
    same guard: what the network adds is the difference of the two), from
    w^n, and from zero.  Features, proposals, increments and targets are
    formed inside the library (ibmg_guess_step)."""
    import torch
    from paper_1311_5614_amd import ibmg
    import ibgen
    w = ibgen.config_c5()
    dt = load_dt("c5")[0]["dt"]
    H = args.steps or 200        # half-trajectory length (default 200 of 400)
    N = w.N
    # the V-cycle schedule tuned for the 1024x1024 rings (the default V(2,2) with the checkerboard
    # stalls on step 267 of this trajectory at 1000 iterations, FP32 and FP64 alike, as V(2,2) did on
    # the rings' calibration steps); no restart below the cap of 1000
    sch = c3_schedule()
    cfg = lambda guess: ibmg.Config(N=N, levels=7, K=w.K, rho=w.rho, mu=w.mu, box=sch["box"], nu1=sch["nu1"],
                                    nu2=sch["nu2"], maxit=MAXIT_TOTAL, restart=0, rtol=w.rtol, prec=sch["prec"],
                                    guess=guess, tail_max=sch["tail_max"], colours=sch["colours"],
                                    colours_from=sch.get("colours_from", 0), omega=sch.get("omega", 1.0),
                                    orth=sch.get("orth", 0))
    s = ibmg.Solver(cfg(ibmg.IBMG_GUESS_PREV), w.fiber_offsets, dev)
    s0 = ibmg.Solver(cfg(ibmg.IBMG_GUESS_ZERO), w.fiber_offsets, dev)
    net = ibmg.Cnn(N, H, dev)
    net.set_params(ibgen.cnn_init(ibgen.seed_for(5, 1)))
    t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev).contiguous()
    gu, gv = t(w.g_u), t(w.g_v)
    z = torch.zeros(N, N, dtype=torch.float64, device=dev)
    u, v, p, X = z.clone(), z.clone(), z.clone(), t(w.X)
    t0 = time.perf_counter()
    its_train = []
    net.reset()
    for n in range(H):
        st = s.guess_step(net, ibmg.IBMG_GUESS_RECORD, dt, u, v, p, X, gu, gv)
        its_train.append(st["iters"])
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    t0 = time.perf_counter()
    loss_first, loss_last = net.train(args.epochs, args.lr)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    # MFMA roofline of the network: one inference (six BF16 convolutions,
    # 2 x 9 x ci x co flop per pixel each) timed with HIP events on the
    # network's stream, 20 back to back
    G = s.fiber_force(X)
    fu, fv = s.spread(X, G)
    feats = torch.stack([u, v, p, fu, fv]).contiguous()
    net.infer(feats)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(net.stream)
    for _ in range(20):
        net.infer(feats)
    e1.record(net.stream)
    e1.synchronize()
    infer_ms = e0.elapsed_time(e1) / 20
    flop = 2.0 * 9 * N * N * sum(ci * co for ci, co in ((5, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 3)))
    conv_roof = {"kernel": "k_conv (six 3x3 convolutions, BF16 MFMA, FP32 accumulation), one inference",
                 "bound": "mfma", "achieved": flop / (infer_ms * 1e-3) / 1e12, "peak": 2500.0, "unit": "TFLOP/s",
                 "frac": flop / (infer_ms * 1e-3) / 1e12 / 2500.0, "flop": flop, "ms": infer_ms,
                 "note": "includes the input packing and output unpacking passes of the inference"}
    print(f"[bench] c5 network inference {infer_ms:.3f} ms, {conv_roof['achieved']:.1f} TFLOP/s", file=sys.stderr,
          flush=True)
    start = [a.clone() for a in (u, v, p, X)]
    dstart = net.get_increment()          # dw^{H-1}: every form starts from it
    res = {}
    for form in ("learned", "extrap", "prev", "zero"):
        u, v, p, X = (a.clone() for a in start)
        net.set_increment(dstart)
        its, conv, alphas = [], [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for n in range(H):
            if form in ("learned", "extrap"):
                mode = ibmg.IBMG_GUESS_LEARNED if form == "learned" else ibmg.IBMG_GUESS_EXTRAP
                st = s.guess_step(net, mode, dt, u, v, p, X, gu, gv)
                alphas.append(st["guess_alpha"])
            elif form == "prev":
                st = s.step(dt, u, v, p, X, gu, gv)
            else:
                st = s0.step(dt, u, v, p, X, gu, gv)
            its.append(st["iters"])
            conv.append(st["converged"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res[form] = dict(time_s=el, timesteps=H, rate=H / el, iters_mean=sum(its) / H, iters_max=max(its),
                         converged=sum(conv))
        if alphas:
            res[form]["alpha_mean"] = sum(alphas) / len(alphas)
        print(f"[bench] c5 {form}: {H} steps in {el:.3f} s -> {H / el:.2f} steps/s, iters mean "
              f"{res[form]['iters_mean']:.2f}, converged {sum(conv)}/{H}", file=sys.stderr, flush=True)
    out = {
        "metric": METRIC, "value": res["learned"]["rate"], "unit": "time-steps/s", "n_gpus": 1,
        "steps": H, "warmup": 0, "ms_per_step": 1e3 * res["learned"]["time_s"] / H,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": ("f64+f32" if sch["prec"] == ibmg.IBMG_FP32 else "f64") + "+bf16",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: steps 1-{H} record and train, steps {H + 1}-{2 * H} timed",
                   "grid": N, "points": w.M, "K": w.K, "dt_factor": w.dt_factor,
                   "chosen_form": "learned initial iterate w^n + alpha (Dw^{n-1} + net) in fp64 FGMRES; "
                                  + describe(cfg(ibmg.IBMG_GUESS_PREV))},
        "forms": res,
        "roofline": conv_roof,
        "training": {"pairs": H, "epochs": args.epochs, "lr": args.lr, "loss_first": loss_first,
                     "loss_last": loss_last, "train_s": t_train, "first_half_s": t_first,
                     "first_half_iters_mean": sum(its_train) / H},
    }
    print(json.dumps(out))

def c3_schedule():
    """The chosen schedule of the 1024x1024 eight-ring workload (autotuner table)."""
    from paper_1311_5614_amd import autotune
    return autotune.load()["c3"]["1024"]


C3_FORMS = ("chosen", "plain", "chosen_prev_start", "chosen_zero_start", "chosen_fp32")


def c3_start(form):
    """Initial iterate of a form: "extrap" (w^n plus the previous step's
    increment, through the solver's guard: ibmg_guess_step), "prev" (w^n) or
    "zero"."""
    if form in ("chosen", "chosen_fp32"):
        return c3_schedule().get("start", "prev")
    return {"chosen_prev_start": "prev", "chosen_zero_start": "zero"}.get(form, "zero")


def c3_config(form):
    """Solver options of a form on the 1024x1024 workload: plain (FP64 V-cycle,
    default schedule, zero start), chosen (the autotuned schedule and its
    start rule), and for attribution the chosen schedule from a zero start and
    with the FP32 V-cycle."""
    import dataclasses
    from paper_1311_5614_amd import ibmg
    import ibgen
    if form == "chosen_zero_start":
        return dataclasses.replace(c3_config("chosen"), guess=ibmg.IBMG_GUESS_ZERO)
    if form == "chosen_prev_start":
        return dataclasses.replace(c3_config("chosen"), guess=ibmg.IBMG_GUESS_PREV)
    if form == "chosen_fp32":
        return dataclasses.replace(c3_config("chosen"), prec=ibmg.IBMG_FP32)
    w = ibgen.config_c3()
    if form == "plain":
        return ibmg.Config(N=w.N, levels=w.levels, K=w.K, rho=w.rho, mu=w.mu, box=4, nu1=2, nu2=2,
                           maxit=MAXIT_TOTAL, restart=C3_BASIS, rtol=w.rtol, prec=ibmg.IBMG_FP64, colours=2,
                           tail_max=0)
    sch = c3_schedule()
    return ibmg.Config(N=w.N, levels=sch["levels"], K=w.K, rho=w.rho, mu=w.mu, box=sch["box"], nu1=sch["nu1"],
                       nu2=sch["nu2"], maxit=sch.get("maxit", MAXIT_TOTAL), restart=sch.get("restart", C3_BASIS), rtol=w.rtol,
                       prec=sch["prec"], colours=sch["colours"], tail_max=sch["tail_max"],
                       colours_from=sch.get("colours_from", 0), guess=sch.get("guess", 0),
                       omega=sch.get("omega", 1.0), orth=sch.get("orth", ibmg.IBMG_ORTH_CGS2))


def describe(cfg, start=None):
    from paper_1311_5614_amd import ibmg
    rs = f"FGMRES({cfg.restart}), cap {cfg.maxit}" if cfg.restart else f"FGMRES, cap {cfg.maxit}"
    order = (f"{cfg.colours} colours on levels 0-{cfg.colours_from - 1}, checkerboard below" if cfg.colours_from
             else f"{cfg.colours} colours")
    if start == "extrap":
        start = "previous step's solution plus its increment (guarded extrapolation)"
    else:
        start = "previous step's solution" if cfg.guess == ibmg.IBMG_GUESS_PREV else "zero"
    orth = "delayed CGS2" if cfg.orth == ibmg.IBMG_ORTH_DCGS2 else "CGS2"
    return (f"{'FP32' if cfg.prec == ibmg.IBMG_FP32 else 'FP64'} V({cfg.nu1},{cfg.nu2}) V-cycle, {cfg.levels} levels, "
            f"{cfg.box}x{cfg.box} boxes, {order}, box weight {cfg.omega:g}, tail {cfg.tail_max or 32}, {rs}, "
            f"FP64 Krylov ({orth}), initial iterate {start}")


def timed_trajectory(s, w, dt, dev, steps, warmup, repeats, net=None):
    """`warmup` untimed steps, then `repeats` runs of `steps` steps, each from
    the workload's initial state (u = v = p = 0, X^0), bracketed by device
    synchronisations.  net: a network handle whose trajectory state serves
    the extrapolated start (ibmg_guess_step, reset with the state).  Returns
    the per-run seconds and the per-step stats of every run."""
    import torch
    from paper_1311_5614_amd import ibmg
    t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev).contiguous()
    X0 = t(w.X)
    z = torch.zeros(w.N, w.N, dtype=torch.float64, device=dev)
    u, v, p, X = z.clone(), z.clone(), z.clone(), X0.clone()
    step = (lambda: s.step(dt, u, v, p, X)) if net is None else \
        (lambda: s.guess_step(net, ibmg.IBMG_GUESS_EXTRAP, dt, u, v, p, X))
    if net is not None:
        net.reset()
    for _ in range(warmup):
        step()
    times, stats = [], []
    for _ in range(repeats):
        u.zero_(); v.zero_(); p.zero_(); X.copy_(X0)
        if net is not None:
            net.reset()
        torch.cuda.synchronize()
        run = []
        t0 = time.perf_counter()
        for _ in range(steps):
            run.append(step())
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        stats.append(run)
    return times, stats


def form_summary(cfg, times, stats, steps, start=None):
    import statistics
    med = statistics.median(times)
    its = [st["iters"] for run in stats for st in run]
    res = [st["rel_resid_true"] for run in stats for st in run]
    conv = [st["converged"] for run in stats for st in run]
    return {"schedule": describe(cfg, start), "rate": steps / med, "ms_per_step": 1e3 * med / steps,
            "runs_s": [round(x, 4) for x in times], "iters_mean": sum(its) / len(its), "iters_max": max(its),
            "steps_timed": len(its), "converged": sum(conv), "missed_rtol": len(its) - sum(conv),
            "rel_resid_max": max(res), "fallbacks": sum(st["fallback"] for run in stats for st in run)}


def cpu_leg_c3(iters=2):
    """Oracle sample of the 1024x1024 workload (run in a child process): step
    1's setup (level hierarchy with the Galerkin elasticity operators, box
    factorisations, bordered coarsest LU, right-hand side) and the first
    `iters` FGMRES iterations with the chosen schedule's box order and
    sweeps; one thread.  Prints one JSON line."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import ibgen
    from oracle import krylov, mg, system
    w = ibgen.config_c3()
    dt = load_dt("c3")[0]["dt"]
    sch = c3_schedule()
    # box order per smoothed level: four colours below colours_from (0: every level), the checkerboard
    # from there on; two-colour schedules use the checkerboard throughout
    cf = sch.get("colours_from", 0) or sch["levels"]
    modes = ["colour" if sch["colours"] == 4 and l < cf else "colour2" for l in range(sch["levels"] - 1)]
    mode = "/".join(sorted(set(modes)))
    omega = sch.get("omega", 1.0)
    z = np.zeros((w.N, w.N))
    with threadpool_limits(1):
        t0 = time.perf_counter()
        lv = system.hierarchy(w.N, sch["levels"], w.rho, w.mu, dt, w.X, w.fiber_offsets, w.K)
        b = system.rhs(z, z, w.X, w.fiber_offsets, w.K, dt, w.rho)
        V = mg.VCycle(lv, sch["box"], sch["nu1"], sch["nu2"], modes, omega)
        t1 = time.perf_counter()
        krylov.fgmres(lv[0].A, b, V, rtol=w.rtol, maxit=iters)
        t2 = time.perf_counter()
    print(json.dumps({"setup_s": t1 - t0, "iter_s": (t2 - t1) / iters, "iters_run": iters,
                      "schedule": f"box {sch['box']}, V({sch['nu1']},{sch['nu2']}), {mode}, omega {omega:g}"}), flush=True)


def start_cpu_leg():
    """The oracle leg in a child process on one host core, started before
    the GPU timing so that the two overlap."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    cores = sorted(os.sched_getaffinity(0))
    p = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-leg"], stdout=subprocess.PIPE,
                         stderr=subprocess.PIPE, env=env, text=True,
                         preexec_fn=(lambda: os.sched_setaffinity(0, {cores[-1]})) if len(cores) > 1 else None)
    return p, cores


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def finish_cpu_leg(p, cores, iters_per_step, timeout_s=900):
    try:
        out, err = p.communicate(timeout=timeout_s)
    except Exception as e:   # noqa: BLE001
        p.kill()
        return {"error": f"cpu leg did not finish: {type(e).__name__}"}
    if p.returncode != 0:
        return {"error": f"cpu leg failed: {err.strip()[-300:]}"}
    d = json.loads(out.strip().splitlines()[-1])
    t_step = d["setup_s"] + iters_per_step * d["iter_s"]
    return {"value": 1.0 / t_step, "unit": "time-steps/s", "cores": 1, "kind": "oracle",
            "sample": (f"1024x1024 eight-ring workload, step 1: oracle setup ({d['setup_s']:.1f} s) and "
                       f"{d['iters_run']} FGMRES iterations ({d['iter_s']:.2f} s each, {d['schedule']}), "
                       f"extrapolated to one step at {iters_per_step:.1f} iterations (the GPU chosen form's "
                       f"mean); one thread (numpy/scipy, no BLAS threads)"),
            "host": {"nproc": len(cores), "cpu_model": cpu_model()}, "setup_s": d["setup_s"],
            "iter_s": d["iter_s"]}


def c3_roofline(s, cfg, w, dt, dev, iters_mean, reps=BOX_REPS, nvec=None):
    """HIP-event timing of the hot kernels of the chosen form on the state the
    timed runs left (setup at the current positions, the last solve's Krylov
    basis): the box relaxation and the residual pass of one colour phase on
    the finest level, and one Gram-Schmidt dot pass and update pass at the
    solve's mean basis size.  Each is `reps` launches replayed from a graph
    on the solver's stream.  The dominant kernel (the largest estimated time
    per step: launches per step times mean launch time) is the roofline
    entry; all four are listed."""
    import torch
    from paper_1311_5614_amd import ibmg
    X = torch.as_tensor(w.X, dtype=torch.float64, device=dev).contiguous()
    s.setup(dt, X)
    basis = cfg.restart or cfg.maxit
    if not nvec:   # the mean basis size of the timed solves (a counter run may fix it)
        nvec = max(1, min(int(round(iters_mean / 2)) + 1, basis - 1))
    phases = (cfg.nu1 + cfg.nu2) * cfg.colours                      # finest-level colour phases per V-cycle
    fused = cfg.colours == 4 and cfg.box in (2, 4)                   # one-launch phases (they form their residual)
    # finest-level residual passes per V-cycle: one per phase but the first (from zero) plus the one before
    # the restriction; with one-launch phases only the latter
    res_per_v = 1 if fused else phases
    cand = {
        "k_box": (ibmg.IBMG_KERNEL_BOX, 0, 0, phases * iters_mean, "box relaxation of one colour phase, finest level"),
        "k_res_ib": (ibmg.IBMG_KERNEL_RES, 0, 0, res_per_v * iters_mean, "residual pass, finest level"),
    }
    if cfg.orth == ibmg.IBMG_ORTH_DCGS2:     # one product pass and one update pass per iteration
        cand["k_multidot2"] = (ibmg.IBMG_KERNEL_DOT2, 0, nvec, iters_mean,
                               f"delayed Gram-Schmidt product pass over {nvec + 1} basis vectors, two vectors")
        cand["k_dcgs2_update"] = (ibmg.IBMG_KERNEL_UPDATE2, 0, nvec, iters_mean,
                                  f"delayed Gram-Schmidt update pass over {nvec} basis vectors")
    else:                                    # two of each
        cand["k_multidot"] = (ibmg.IBMG_KERNEL_MULTIDOT, 0, nvec, 2 * iters_mean,
                              f"Gram-Schmidt dot pass over {nvec} basis vectors")
        cand["k_update_acc"] = (ibmg.IBMG_KERNEL_UPDATE, 0, nvec, 2 * iters_mean,
                                f"Gram-Schmidt update pass over {nvec} basis vectors")
    out = {}
    for name, (k, level, arg, per_step, what) in cand.items():
        us, by = s.kernel_bench(k, level, arg, reps)
        gbs = by / (us * 1e-6) / 1e9
        out[name] = {"what": what, "avg_us": us, "bytes": by, "achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS,
                     "launches_per_step": per_step, "est_ms_per_step": per_step * us * 1e-3}
        print(f"[bench] {name}: {us:.2f} us, {by / 1e6:.2f} MB -> {gbs:.0f} GB/s ({100 * gbs / HBM_PEAK_GBS:.1f} %)",
              file=sys.stderr, flush=True)
    dom = max(out, key=lambda k: out[k]["est_ms_per_step"])
    d = out[dom]
    return {"kernel": f"{dom} ({d['what']})", "bound": "hbm", "achieved": d["achieved_GBs"], "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": d["frac"], "traffic": measured_traffic_c3(dom, d),
            "launch": {"avg_us": d["avg_us"], "bytes": d["bytes"], "reps": reps, "prec": "fp32" if
                       cfg.prec == ibmg.IBMG_FP32 else "fp64"},
            "kernels": out}


def measured_traffic_c3(name, d):
    """HBM bytes per launch of kernel `name` from the committed rocprofv3
    counter summary (profiles/<name>_1024x1024_traffic.txt: FETCH_SIZE and
    WRITE_SIZE scaled by a copy-kernel calibration), or None when there is no
    summary, it was taken for another launch size, or the kernel's sources
    changed since."""
    path = os.path.join(ROOT, "profiles", f"{name}_1024x1024_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.strip().split("=", 1)
                kv[k] = v
    if kv.get("kernel_source_sha1") != box_source_hash():
        return None
    if abs(float(kv.get("algorithmic_bytes", -1)) - d["bytes"]) > 1e-6 * d["bytes"]:
        return None
    return float(kv["traffic_bytes"])


def run_c3(args, dev):
    """The 1024x1024 eight-ring workload, plain and chosen forms."""
    import torch
    import ibgen
    from paper_1311_5614_amd import ibmg
    leg = None if args.no_cpu else start_cpu_leg()
    w = ibgen.config_c3()
    dt = load_dt("c3")[0]["dt"]
    forms = [f for f in args.forms.split(",") if f in C3_FORMS] or ["chosen", "plain"]
    res, solvers = {}, {}
    for form in forms:
        cfg = c3_config(form)
        start = c3_start(form)
        s = ibmg.Solver(cfg, w.fiber_offsets, dev)
        net = ibmg.Cnn(w.N, 1, dev) if start == "extrap" else None
        times, stats = timed_trajectory(s, w, dt, dev, args.steps, args.warmup, args.repeats, net)
        if net is not None:
            net.close()
        res[form] = form_summary(cfg, times, stats, args.steps, start)
        r = res[form]
        print(f"[bench] c3 {form}: {r['rate']:.3f} steps/s (runs {r['runs_s']} s), iters mean "
              f"{r['iters_mean']:.1f} max {r['iters_max']}, missed rtol {r['missed_rtol']}/{r['steps_timed']}",
              file=sys.stderr, flush=True)
        if form == "chosen" or len(forms) == 1:
            solvers[form] = (s, cfg)
        else:
            s.close()          # only the chosen form's state is timed further (its workspace is 30 GB)
            del s
            torch.cuda.empty_cache()
    chosen = "chosen" if "chosen" in res else forms[0]
    rc = res[chosen]
    s, cfg = solvers[chosen]
    roof = c3_roofline(s, cfg, w, dt, dev, rc["iters_mean"], nvec=args.roofline_nvec)
    for f, (sv, _) in solvers.items():
        sv.close()
    del solvers
    torch.cuda.empty_cache()
    out = {
        "metric": METRIC, "value": rc["rate"], "unit": "time-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": rc["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32" if cfg.prec == ibmg.IBMG_FP32 else "f64", "data": "synthetic",
        "config": {"workload": (f"1024x1024 periodic grid, 8 elastic rings x 2048 points (16384), K 1e6, "
                                f"dt 500 x explicit limit, {cfg.levels} levels, rtol 1e-8; chosen form: "
                                f"{describe(cfg, c3_start(chosen))}"),
                   "grid": w.N, "points": w.M, "rings": 8, "K": w.K, "dt_factor": w.dt_factor,
                   "repeats": args.repeats, "timing": "median of the repeats"},
        "forms": res,
        "iters_per_solve": {f: round(r["iters_mean"], 2) for f, r in res.items()},
        "roofline": roof,
    }
    if "plain" in res and chosen != "plain":
        out["speedup_vs_plain"] = rc["rate"] / res["plain"]["rate"]
    return out, leg


def run_efficiency(args, dev, steps=20, probe_steps=60, sample=100):
    """Implicit against explicit time stepping on the 256x256 single-ellipse
    geometry (Sec. 7's comparison, on the periodic workload): per stiffness,
    the wall time per unit of simulated time of the implicit method at
    100 x dt_exp (tuned schedule) and of the explicit method (Sec. 2.3.1: the
    force at X^n, a Stokes solve per step) at the largest multiple of dt_exp
    among 1, 2, 4 whose run of `probe_steps` steps stays bounded, timed over
    `sample` steps.  The ratio is the efficiency factor of Sec. 7 measured in
    wall time on this GPU."""
    import torch
    from paper_1311_5614_amd import ibmg
    cases, dts = workloads("c2")
    tcases, precs = tuned("c2", cases)
    out = {}
    for k in (2, 4):                        # K = 1e4 and 1e6 at 100 x dt_exp
        w, dt, prec = tcases[k], dts[k], precs[k]
        dte = dt / w.dt_factor
        t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev).contiguous()
        gu, gv = t(w.g_u), t(w.g_v)

        def fresh():
            z = torch.zeros(w.N, w.N, dtype=torch.float64, device=dev)
            return z.clone(), z.clone(), z.clone(), t(w.X)

        r = Run(w, dt, prec, dev)
        for _ in range(2):
            r.step()
        r.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its_i = [r.step()["iters"] for _ in range(steps)]
        torch.cuda.synchronize()
        t_imp = (time.perf_counter() - t0) / steps
        r.s.close()
        del r
        cfg = ibmg.Config(N=w.N, levels=w.levels, K=w.K, rho=w.rho, mu=w.mu, box=4, nu1=2, nu2=2, maxit=200,
                          rtol=w.rtol, prec=ibmg.IBMG_FP64, colours=2, scheme=ibmg.IBMG_EXPLICIT)
        se = ibmg.Solver(cfg, w.fiber_offsets, dev)
        f_ok = None
        for f in (1.0, 2.0, 4.0):
            u, v, p, X = fresh()
            X0 = X.clone()
            try:
                for _ in range(probe_steps):
                    se.step(f * dte, u, v, p, X, gu, gv)
                bounded = float((X - X0).abs().max()) * w.N < 0.25 * w.N
            except ibmg.IBMGError:
                bounded = False
            if not bounded:
                break
            f_ok = f
        if f_ok is None:
            out[f"K{w.K:.0e}"] = {"error": "explicit method unstable at dt_exp"}
            se.close()
            continue
        u, v, p, X = fresh()
        se.step(f_ok * dte, u, v, p, X, gu, gv)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its_e = [se.step(f_ok * dte, u, v, p, X, gu, gv)["iters"] for _ in range(sample)]
        torch.cuda.synchronize()
        t_exp = (time.perf_counter() - t0) / sample
        se.close()
        per_time_imp = t_imp / dt                 # wall seconds per unit simulated time
        per_time_exp = t_exp / (f_ok * dte)
        out[f"K{w.K:.0e}"] = {
            "implicit": {"dt_over_dt_exp": w.dt_factor, "ms_per_step": 1e3 * t_imp,
                         "iters_mean": sum(its_i) / len(its_i), "schedule": "tuned (schedules.json c2)"},
            "explicit": {"dt_over_dt_exp": f_ok, "ms_per_step": 1e3 * t_exp, "iters_mean": sum(its_e) / len(its_e),
                         "stability": f"bounded over {probe_steps} steps at {f_ok:g} x dt_exp, "
                                      f"{'not tried' if f_ok == 4.0 else 'unbounded'} above"},
            "efficiency_factor": per_time_exp / per_time_imp}
        print(f"[bench] efficiency K={w.K:.0e}: implicit {1e3 * t_imp:.2f} ms/step at {w.dt_factor:g} dt_exp, "
              f"explicit {1e3 * t_exp:.2f} ms/step at {f_ok:g} dt_exp -> factor "
              f"{out[f'K{w.K:.0e}']['efficiency_factor']:.1f}", file=sys.stderr, flush=True)
    torch.cuda.empty_cache()
    return out


def run_mg_solver(args, dev, factors=(1.0, 10.0, 100.0, 160.0, 1000.0), spectrum=True):
    """Multigrid alone against multigrid-preconditioned FGMRES (Sec. 5.1,
    Fig. 3's comparison) on the 32x32 single-ellipse geometry: single-cell
    boxes, V(1,1), four colours, relative residual 1e-6 (the paper's
    tolerance), at several multiples of the explicit limit; iteration counts
    of both solvers from a zero start, and (spectrum) the spectral radius of
    the V-cycle iteration matrix I - M A (Sec. 5.2), assembled column by
    column through the C ABI and diagonalised on the host."""
    import numpy as np
    import torch
    from paper_1311_5614_amd import ibmg
    import ibgen
    w = ibgen.config_c1()
    dte = load_dt("c1")[0]["dt"] / w.dt_factor
    N = w.N
    n = 3 * N * N
    out = []
    for f in factors:
        dt = f * dte
        row = {"dt_over_dt_exp": f}
        for name, solver in (("mg", ibmg.IBMG_SOLVER_MG), ("mg_fgmres", ibmg.IBMG_SOLVER_FGMRES)):
            cfg = ibmg.Config(N=N, levels=4, K=w.K, box=1, nu1=1, nu2=1, colours=4, rtol=1e-6, maxit=1000,
                              restart=200, solver=solver)
            s = ibmg.Solver(cfg, w.fiber_offsets, dev)
            s.setup(dt, torch.as_tensor(w.X, dtype=torch.float64, device=dev).contiguous())
            z = torch.zeros(N, N, dtype=torch.float64, device=dev)
            b = s.rhs(z, z)
            x = torch.zeros_like(b)
            st = s.solve(b, x)
            row[name] = {"iters": st["iters"], "converged": st["converged"],
                         "rel_resid": st["rel_resid_true"]}
            if spectrum and solver == ibmg.IBMG_SOLVER_MG:
                T = np.zeros((n, n))
                for k in range(n):
                    e = torch.zeros(n, dtype=torch.float64, device=dev)
                    e[k] = 1.0
                    T[:, k] = (e - s.vcycle(s.apply(0, e))).cpu().numpy()
                q = np.zeros(n)
                q[2 * N * N:] = 1.0 / N
                Pm = np.eye(n) - np.outer(q, q)
                ev = np.abs(np.linalg.eigvals(Pm @ T @ Pm))
                row["spectral_radius"] = float(ev.max())
                row["eig_fraction_above_0.5"] = float(np.mean(ev > 0.5))
            s.close()
        out.append(row)
        print(f"[bench] mg solver {f:g} x dt_exp: {row}", file=sys.stderr, flush=True)
    return {"workload": "32x32 single ellipse (128 points, K 1e4), single-cell boxes, V(1,1), 4 colours, "
                        "rtol 1e-6, zero start", "rows": out}


def run_cavity(args, dev, spectrum=True):
    """The paper's walled test problem on the GPU (Sec. 4-6): the thick
    annulus in the lid-driven cavity, steady Stokes (rho = 0), cosine delta,
    at relative stiffness alpha / alpha_exp (alpha_exp of the oracle, stored
    in tests/golden/workload_dt.json), the lid as right-hand side, zero
    start, residual reduced by 1e-6.  The GPU's box orders are coloured
    (Jacobi within a colour), not the paper's lexicographic one, so its
    counts are those of a different (valid) smoother.  Rows: Fig. 3's
    MG-FGMRES (cap 100) and multigrid-alone counts at h = 2^-5 with
    single-cell boxes; Table 2's box sizes and sweeps at h = 2^-6; the grid
    refinement of Fig. 7 (alpha = 6, 60, 600, 3000); and (spectrum) the
    spectral radius of the V-cycle iteration matrix I - M A (Sec. 5.2)
    assembled column by column through the C ABI."""
    import numpy as np
    import torch
    from paper_1311_5614_amd import ibmg
    import ibgen
    aexp = {e["N"]: e["alpha_exp"] for e in load_dt("cavity")}

    def solver(N, box, nu, colours, alpha, kind, maxit):
        X, offs, M1, M2 = ibgen.annulus(N)
        levels = int(np.log2(N // max(4, box))) + 1
        cfg = ibmg.Config(N=N, levels=levels, K=alpha, rho=0.0, box=box, nu1=nu[0], nu2=nu[1], maxit=maxit,
                          rtol=1e-6, colours=colours, tail_max=1, delta=ibmg.IBMG_DELTA_COS4,
                          domain=ibmg.IBMG_CAVITY, solver=kind, restart=0 if maxit <= 1000 else 1000)
        s = ibmg.Solver(cfg, offs, dev)
        s.setup(1.0, torch.as_tensor(X, dtype=torch.float64, device=dev).contiguous())
        return s

    lids = {}

    def lid(N):
        if N not in lids:
            cfg = ibmg.Config(N=N, levels=int(np.log2(N // 16)) + 1, K=0.0, rho=0.0, box=1, tail_max=1,
                              domain=ibmg.IBMG_CAVITY)
            s = ibmg.Solver(cfg, None, dev)
            s.setup(1.0, None)
            z = torch.zeros(N, N, dtype=torch.float64, device=dev)
            lids[N] = s.rhs(z, z).clone()
            s.close()
        return lids[N]

    def count(N, box, nu, colours, alpha, kind, maxit):
        s = solver(N, box, nu, colours, alpha, kind, maxit)
        b = lid(N)
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = s.solve(b, x)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        s.close()
        return {"iters": st["iters"], "converged": st["converged"], "ms": round(ms, 2)}

    out = {"workload": "thick annulus in the lid-driven cavity, steady Stokes, cosine delta, lid right-hand "
                       "side, zero start, rtol 1e-6; coloured box orders", "alpha_exp": aexp}
    fig3 = []
    for colours in (4, 2):
        for r in (1.0, 10.0, 100.0, 160.0, 500.0, 800.0):
            a = r * aexp[32]
            row = {"colours": colours, "ratio": r,
                   "mg_fgmres": count(32, 1, (1, 1), colours, a, ibmg.IBMG_SOLVER_FGMRES, 100),
                   "mg": count(32, 1, (1, 1), colours, a, ibmg.IBMG_SOLVER_MG, 300)}
            fig3.append(row)
            print(f"[bench] cavity fig3 {row}", file=sys.stderr, flush=True)
    out["fig3_h32"] = fig3
    tab2 = []
    for box in (1, 4, 8):
        for nu in ((1, 0), (1, 1), (2, 1), (2, 2)):
            row = {"box": box, "nu": list(nu), "iters": []}
            for r in (10.0, 100.0, 500.0):
                c = count(64, box, nu, 4, r * aexp[64], ibmg.IBMG_SOLVER_FGMRES, 100)
                row["iters"].append(c["iters"] if c["converged"] else ">=100")
            tab2.append(row)
            print(f"[bench] cavity table2 {row}", file=sys.stderr, flush=True)
    out["table2_h64_colours4"] = tab2
    refine = []
    for alpha in (6.0, 60.0, 600.0, 3000.0):
        for box in (1, 4, 8):
            row = {"alpha": alpha, "box": box, "iters": {}}
            for N in (32, 64, 128):
                c = count(N, box, (1, 1), 4, alpha, ibmg.IBMG_SOLVER_FGMRES, 100)
                row["iters"][str(N)] = c["iters"] if c["converged"] else ">=100"
            refine.append(row)
            print(f"[bench] cavity refinement {row}", file=sys.stderr, flush=True)
    out["fig7_refinement_colours4"] = refine
    out["efficiency_h32"] = cavity_efficiency(dev, aexp[32])
    if spectrum:
        N = 32
        n = 3 * N * N
        spec = []
        for colours in (4,):
            for r in (0.0, 1.0, 10.0, 100.0):
                s = solver(N, 1, (1, 1), colours, r * aexp[N], ibmg.IBMG_SOLVER_MG, 10)
                T = np.zeros((n, n))
                for k in range(n):
                    e = torch.zeros(n, dtype=torch.float64, device=dev)
                    e[k] = 1.0
                    T[:, k] = (e - s.vcycle(s.apply(0, e))).cpu().numpy()
                s.close()
                # the wall faces are decoupled identity rows (eigenvalue 0); the
                # constant pressure is the trivial eigenvalue 1: project it out
                q = np.zeros(n)
                q[2 * N * N:] = 1.0 / N
                Pm = np.eye(n) - np.outer(q, q)
                ev = np.abs(np.linalg.eigvals(Pm @ T @ Pm))
                row = {"colours": colours, "ratio": r, "spectral_radius": float(ev.max()),
                       "frac_above_0.25": float(np.mean(ev > 0.25)), "frac_above_0.5": float(np.mean(ev > 0.5))}
                spec.append(row)
                print(f"[bench] cavity spectrum {row}", file=sys.stderr, flush=True)
        out["spectrum_h32_single_cell"] = spec
    return out


def cavity_efficiency(dev, alpha_exp, N=32, dt=1.0 / 40, steps=40, probe=200):
    """Implicit against explicit time stepping on the walled test problem, in
    the manner of Sec. 7: steady Stokes with the structure's position lagged
    (rho = 0), h = 2^-5, the implicit method at dt = 1/40 with MG-FGMRES
    (nu1 = nu2 = 1, residual reduced by 1e-6), the explicit one just below its
    stability limit (0.95 dt_exp, dt_exp = alpha_exp / gamma with Table 1's
    alpha_exp of this grid), `steps` steps of each, extrapolated to t = 1.
    Sec. 7 drives the annulus with a shear flow in a 2 x 1 rectangle; here the
    square cavity's lid drives it (the domain this library has).  The
    efficiency factor is the explicit method's work to t = 1 over the
    implicit one's, counted in MG-FGMRES iterations (the paper's measure) and
    in wall time.  A stability probe at relative stiffness 10 runs the
    explicit method `probe` steps at 0.95 and 1.1 dt_exp."""
    import numpy as np
    import torch
    from paper_1311_5614_amd import ibmg
    import ibgen
    X0, offs, M1, M2 = ibgen.annulus(N)
    X0 = torch.as_tensor(X0, dtype=torch.float64, device=dev).contiguous()

    def solver(box, gamma, scheme):
        levels = int(np.log2(N // max(4, box))) + 1
        cfg = ibmg.Config(N=N, levels=levels, K=gamma, rho=0.0, box=box, nu1=1, nu2=1, maxit=1000, rtol=1e-6,
                          colours=4, tail_max=1, delta=ibmg.IBMG_DELTA_COS4, domain=ibmg.IBMG_CAVITY,
                          scheme=scheme, guess=ibmg.IBMG_GUESS_PREV)
        return ibmg.Solver(cfg, offs, dev)

    def run(box, gamma, scheme, step_dt, n):
        s = solver(box, gamma, scheme)
        z = torch.zeros(N, N, dtype=torch.float64, device=dev)
        u, v, p, X = z.clone(), z.clone(), z.clone(), X0.clone()
        its, conv, drift = [], True, []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            st = s.step(step_dt, u, v, p, X)
            its.append(st["iters"])
            conv = conv and bool(st["converged"])
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / n
        s.close()
        return {"iters_mean": sum(its) / n, "ms_per_step": round(ms, 3), "all_converged": conv,
                "max_displacement": float((X - X0).abs().max()) if bool(torch.isfinite(X).all()) else float("inf")}

    rows = []
    for box in (1, 4, 8):
        for rel in (1.0, 10.0, 100.0, 1000.0):
            gamma = rel * alpha_exp / dt
            dte = 0.95 * alpha_exp / gamma
            imp = run(box, gamma, ibmg.IBMG_IMPLICIT, dt, steps)
            exp = run(box, gamma, ibmg.IBMG_EXPLICIT, dte, steps)
            f_its = (exp["iters_mean"] / dte) / (imp["iters_mean"] / dt)
            f_time = (exp["ms_per_step"] / dte) / (imp["ms_per_step"] / dt)
            rows.append({"box": box, "relative_stiffness": rel, "gamma": gamma, "implicit": imp,
                         "explicit": dict(exp, dt=dte), "efficiency_iters": round(f_its, 2),
                         "efficiency_time": round(f_time, 2)})
            print(f"[bench] cavity efficiency box {box} rel {rel:g}: implicit {imp['iters_mean']:.1f} its "
                  f"{imp['ms_per_step']:.2f} ms, explicit {exp['iters_mean']:.1f} its {exp['ms_per_step']:.2f} ms "
                  f"-> factor {f_its:.1f} (iterations), {f_time:.1f} (time)", file=sys.stderr, flush=True)
    gamma = 10.0 * alpha_exp / dt
    stab = {f"{f:g}_dt_exp": run(4, gamma, ibmg.IBMG_EXPLICIT, f * alpha_exp / gamma, probe)["max_displacement"]
            for f in (0.95, 1.1)}
    print(f"[bench] explicit stability probe (max displacement after {probe} steps): {stab}",
          file=sys.stderr, flush=True)
    return {"workload": f"thick annulus in the lid-driven cavity, {N}x{N}, steady Stokes with lagged structure, "
                        f"{steps} steps of each method, work extrapolated to t = 1",
            "rows": rows, "explicit_stability_probe": stab}


def run_d3(args, dev, steps=5, only=None):
    """The three-dimensional form (include/ibmg3.h) on the periodic unit
    cube: closed latitude rings on a stretched sphere (ibgen.sphere_rings,
    about 0.6 k points at 32^3, 2.5 k at 64^3), rho = mu = 1, dt = 0.01,
    dt K = 10 and 100, MG-FGMRES with checkerboard boxes of 2^3 cells
    (44 unknowns) and 4^3 cells (304 unknowns, the paper's 750 KB block),
    in two forms: the paper's undamped boxes with V(1,1), and V(2,1) with
    box corrections weighted by 0.5 (this build's damping option),
    rtol 1e-8, FGMRES(500), implicit steps from rest.  Per row: the first
    step (from the stretched rings at rest, the hardest solve) on its own,
    then `steps` more: ms per step (setup with the box inverses,
    right-hand side, solve, point update), the setup alone, FGMRES
    iterations per step and the boxes with own inverses on level 0."""
    import numpy as np
    import torch
    from paper_1311_5614_amd import ibmg
    import ibgen
    rows = []
    for N in (32, 64):
        X, offs = ibgen.sphere_rings(N)
        for box in (2, 4):
            levels = int(np.log2(N // (2 if box == 2 else 4))) + 1
            for alpha, form in ((10.0, "paper"), (100.0, "paper"), (10.0, "damped"), (100.0, "damped")):
                if only is not None and (N, box, alpha) != only:
                    continue
                dt = 0.01
                nu, omega = ((1, 1), 1.0) if form == "paper" else ((2, 1), 0.5)
                cfg = ibmg.Config3(N=N, levels=levels, K=alpha / dt, box=box, nu1=nu[0], nu2=nu[1], maxit=500,
                                   rtol=1e-8, omega=omega)
                s = ibmg.Solver3(cfg, offs, dev)
                n3 = N ** 3
                uvw = torch.zeros(3 * n3, dtype=torch.float64, device=dev)
                p = torch.zeros(n3, dtype=torch.float64, device=dev)
                Xg = torch.as_tensor(X, dtype=torch.float64, device=dev).contiguous()
                # the first step starts from the stretched rings at rest (the hardest solve; it
                # also forms the shared plain-box inverses): timed and reported on its own
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st0 = s.step(dt, uvw, p, Xg)
                torch.cuda.synchronize()
                first = {"ms": 1e3 * (time.perf_counter() - t0), "iters": st0["iters"],
                         "converged": bool(st0["converged"])}
                its, conv, ms = [], 0, []
                for _ in range(steps):
                    t0 = time.perf_counter()
                    st = s.step(dt, uvw, p, Xg)
                    torch.cuda.synchronize()
                    ms.append(1e3 * (time.perf_counter() - t0))
                    its.append(st["iters"])
                    conv += int(st["converged"])
                t0 = time.perf_counter()
                s.setup(dt, Xg)
                torch.cuda.synchronize()
                setup_ms = 1e3 * (time.perf_counter() - t0)
                own, total = s.box_counts(0)
                row = {"N": N, "box": box, "form": form, "nu": list(nu), "omega": omega,
                       "unknowns_per_box": 3 * (box + 1) * box * box + box ** 3,
                       "levels": levels, "dt_K": alpha, "points": int(offs[-1]), "ms_per_step": float(np.median(ms)),
                       "setup_ms": setup_ms, "iters_mean": sum(its) / steps, "converged": f"{conv}/{steps}",
                       "own_boxes_level0": own, "boxes_level0": total, "first_step": first}
                rows.append(row)
                print(f"[bench] 3-D {N}^3 box {box} dtK {alpha:g} {form}: first step {first['ms']:.1f} ms, "
                      f"{first['iters']} its, converged {first['converged']}; then {row['ms_per_step']:.1f} ms/step "
                      f"(setup {setup_ms:.1f} ms), {row['iters_mean']:.1f} its, {conv}/{steps} converged, "
                      f"{own}/{total} own boxes", file=sys.stderr, flush=True)
                s.close()
                del s
                torch.cuda.empty_cache()
    return {"workload": "sphere rings in the periodic unit cube, implicit steps from rest, MG-FGMRES V(1,1), "
                        "checkerboard boxes, rtol 1e-8", "rows": rows}


PROBE_N = 4096   # bandwidth probe: plain V(2,2) with no structure on this grid


def vcycle_probe(dev, N=PROBE_N, reps=10, colours=2):
    """Plain FP64 V(2,2) with 4x4 boxes and no structure on an N x N grid
    (coarsest 16 x 16), large enough to be bandwidth-bound rather than
    latency-bound.  Times `reps` V-cycles (one captured graph each) between
    HIP events on the solver's stream, and the finest-level box launch.
    Algorithmic bytes of a V(nu1, nu2): (9 (nu1 + nu2) + 13.5) words per
    finest cell times 4/3 for the level hierarchy (one read of b and w and
    one write of w per sweep and level, plus residual, restriction and
    prolongation), 528 B per cell in FP64 at V(2,2)."""
    import math
    import torch
    from paper_1311_5614_amd import ibmg
    levels = int(math.log2(N // 16)) + 1
    cfg = ibmg.Config(N=N, levels=levels, K=0.0, box=4, nu1=2, nu2=2, maxit=4, prec=ibmg.IBMG_FP64, colours=colours)
    s = ibmg.Solver(cfg, None, dev)
    try:
        s.setup(1.0 / N, None)
        gen = torch.Generator(device=dev)
        gen.manual_seed(1311_4096)
        r = torch.randn(3 * N * N, dtype=torch.float64, device=dev, generator=gen)
        for _ in range(2):
            s.vcycle(r)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        for _ in range(reps):
            s.vcycle(r)
        e1.record(s.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        alg = (9 * (cfg.nu1 + cfg.nu2) + 13.5) * 8 * 4 / 3 * N * N
        us, by = s.box_bench(0, 0, BOX_REPS)
        gbs = alg / (ms * 1e-3) / 1e9
        kb = by / (us * 1e-6) / 1e9
        out = {"workload": f"{N}x{N}, {levels} levels, plain FP64 V(2,2), 4x4 boxes, {colours} colours, no structure",
               "vcycle_ms": ms, "vcycle_bytes": alg, "vcycle_GBs": gbs, "vcycle_frac": gbs / HBM_PEAK_GBS,
               "target_frac": 0.5, "target_met": gbs / HBM_PEAK_GBS >= 0.5,
               "k_box_us": us, "k_box_bytes": by, "k_box_GBs": kb, "k_box_frac": kb / HBM_PEAK_GBS}
        print(f"[bench] probe {N}x{N}: V-cycle {ms:.3f} ms -> {gbs:.0f} GB/s ({100 * gbs / HBM_PEAK_GBS:.1f} %), "
              f"k_box {us:.1f} us -> {kb:.0f} GB/s ({100 * kb / HBM_PEAK_GBS:.1f} %)", file=sys.stderr, flush=True)
        return out
    finally:
        s.close()
        del s
        torch.cuda.empty_cache()


def run_sweep(args, dev, workload, forms, steps, warmup):
    """The 256x256 stiffness sweep (c2) or the 64-problem batch (c4) in the
    given forms; returns the result line without probe and CPU leg."""
    import torch
    from paper_1311_5614_amd import ibmg
    cases, dts = workloads(workload)
    for c in cases:
        if args.levels:
            c.levels = args.levels
        if args.nu:
            c.nu1, c.nu2 = (int(x) for x in args.nu.split(","))
        c.colours = args.colours
        if args.box:
            c.box = args.box
        if args.tail_max:
            c.tail_max = args.tail_max
    forms = list(forms)
    res = {}
    for form in forms:
        # plain: FP64 V-cycle, default schedule.  fp32: FP32 V-cycle, default
        # schedule.  tuned: per-class autotuned schedule and precision.
        # batch / batch64: every trajectory in one batch handle (tuned
        # schedules, FP32 / FP64 V-cycle).
        if form.startswith("batch"):
            prec = ibmg.IBMG_FP64 if form == "batch64" else ibmg.IBMG_FP32
            bcases, _ = tuned(workload, cases)
            br = BatchRun(bcases, dts, prec, dev)
            t, its, conv, rounds = timed_batch(br, steps, warmup)
            n = steps * len(cases)
            res[form] = dict(time_s=t, timesteps=n, rate=n / t, iters_mean=sum(its) / len(its), iters_max=max(its),
                             converged=sum(conv), rounds=rounds, phase=None)
            print(f"[bench] {form}: {n} steps in {t:.3f} s -> {n / t:.2f} steps/s, iters mean "
                  f"{res[form]['iters_mean']:.2f} max {max(its)}, converged {sum(conv)}/{n}, {rounds} lockstep "
                  f"rounds", file=sys.stderr, flush=True)
            del br
            torch.cuda.empty_cache()
            continue
        if form in ("tuned", "concurrent"):
            fcases, precs = tuned(workload, cases)
        else:
            fcases = cases
            precs = [ibmg.IBMG_FP32 if form == "fp32" else ibmg.IBMG_FP64] * len(cases)
        if form == "concurrent":
            # concurrent: the tuned form with every trajectory on its own
            # stream and host thread.  Streams are spread over the device's
            # hardware queues in creation order, so they are created from the
            # most to the least expensive trajectory (the autotuner's time per
            # step of its class): the costliest trajectories get queues of
            # their own.  The form runs first in the default order, before
            # other forms' streams come and go.
            from paper_1311_5614_amd import autotune
            table = autotune.load().get(workload, {})
            cost = [table.get(schedule_key(workload, w), {}).get("ms_per_step", 0.0) for w in cases]
            streams = [None] * len(cases)
            for k in sorted(range(len(cases)), key=lambda k: -cost[k]):
                streams[k] = torch.cuda.Stream(dev)
            runs = [Run(w, dt, pr, dev, stream=st) for w, dt, pr, st in zip(fcases, dts, precs, streams)]
            torch.cuda.synchronize()
            t, its, conv, _ = timed_concurrent(runs, steps, warmup)
        else:
            runs = [Run(w, dt, pr, dev) for w, dt, pr in zip(fcases, dts, precs)]
            t, its, conv, _ = timed(runs, steps, warmup, timing=False)
        failed = dict(timed.failed)
        per_case = [round(sum(x) / max(1, len(x)), 1) for x in timed.per_case]
        # roofline of the box kernel: on the finest level of the first
        # trajectory in the form's V-cycle precision, BOX_REPS back-to-back
        # launches between two HIP events on the solver's stream
        ph = None
        main_prec = max(set(precs), key=precs.count)
        rb = next((k for k, pr in enumerate(precs) if k not in failed and pr == main_prec), None)
        if rb is not None:
            r = runs[rb]
            r.s.setup(r.dt, r.X)
            us, by = r.s.box_bench(0, 0, BOX_REPS)
            ph = dict(avg_us=us, bytes=by, level=0, grid=r.w.N, case=r.w.name,
                      prec="fp32" if precs[rb] == ibmg.IBMG_FP32 else "fp64", reps=BOX_REPS)
        n = sum(1 for _ in its) - (1 if failed else 0)   # completed implicit steps
        res[form] = dict(time_s=t, timesteps=n, rate=n / t, iters_mean=sum(its) / max(1, n), iters_max=max(its),
                         converged=sum(conv), phase=ph, failed=failed)
        print(f"[bench] {form}: {n} steps in {t:.3f} s -> {n / t:.2f} steps/s, iters mean "
              f"{res[form]['iters_mean']:.2f} max {max(its)}, converged {sum(conv)}/{n}; per case {per_case}",
              file=sys.stderr, flush=True)
        res[form]["iters_per_case"] = per_case
        if form == "concurrent":
            res[form]["seconds_per_case"] = [round(x, 3) for x in timed.case_s]
            print(f"[bench] concurrent: wall seconds per trajectory {res[form]['seconds_per_case']}",
                  file=sys.stderr, flush=True)
        del runs
        torch.cuda.empty_cache()
    chosen = next((f for f in ("batch", "concurrent", "tuned", "fp32") if f in res), forms[0])
    rc = res[chosen]
    ph = next((res[f]["phase"] for f in (chosen, "tuned", "fp32", "plain") if f in res and res[f]["phase"]), None)
    achieved = ph["bytes"] / (ph["avg_us"] * 1e-6) / 1e9 if ph else None
    w0 = cases[0]
    out = {
        "metric": METRIC,
        "value": rc["rate"],
        "unit": "time-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": 1e3 * rc["time_s"] / steps,
        "ms_per_timestep": 1e3 * rc["time_s"] / rc["timesteps"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if chosen in ("plain", "batch64") else "f64+f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{len(cases)} trajectories on {w0.N}x{w0.N}, {w0.M} Lagrangian points, "
                         f"{w0.levels} levels, V({w0.nu1},{w0.nu2}), box {w0.box}, rtol {w0.rtol:g}"),
            "grid": w0.N, "points": w0.M, "trajectories": len(cases), "levels": w0.levels,
            "K": sorted({c.K for c in cases}), "dt_factor": sorted({c.dt_factor for c in cases}),
            "chosen_form": {"fp32": "fp32 V-cycle inside fp64 FGMRES",
                            "tuned": "autotuned schedule and V-cycle precision per case inside fp64 FGMRES",
                            "concurrent": "autotuned schedule and V-cycle precision per case inside fp64 FGMRES, "
                                          "trajectories advanced concurrently (one stream and host thread each)",
                            "batch": "all trajectories in one batch, fp32 V-cycle, autotuned schedules"}.get(chosen,
                                                                                                      chosen),
        },
        "forms": {k: {kk: vv for kk, vv in v.items() if kk != "phase"} for k, v in res.items()},
        "roofline": {
            "kernel": "k_box (box relaxation, one colour phase)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": measured_traffic(ph),
            "launch": ph,
        },
    }
    out["_cases"] = (cases, dts)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 20; c5: half-trajectory 200)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--repeats", type=int, default=3, help="c3: timed runs per form (median reported)")
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--no-extras", action="store_true", help="c3: skip the 256x256 sweep and the batch")
    ap.add_argument("--cpu-leg", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--forms", default="", help="c3: chosen,plain; c2: concurrent,plain,fp32,tuned")
    ap.add_argument("--levels", type=int, default=0, help="override the workload's level count")
    ap.add_argument("--nu", default="", help="override smoothing sweeps, e.g. 1,1")
    ap.add_argument("--colours", type=int, default=2)
    ap.add_argument("--box", type=int, default=0, help="override the box edge (1, 2, 4 or 8 cells)")
    ap.add_argument("--tail-max", type=int, default=0, help="override the V-cycle tail size")
    ap.add_argument("--epochs", type=int, default=20, help="c5: training epochs of the warm-start network")
    ap.add_argument("--lr", type=float, default=1e-3, help="c5: Adam learning rate")
    ap.add_argument("--no-probe", action="store_true", help="skip the 4096x4096 bandwidth probe")
    ap.add_argument("--probe-only", action="store_true", help="run only the 4096x4096 bandwidth probe")
    ap.add_argument("--probe-n", type=int, default=PROBE_N, help="grid of the bandwidth probe")
    ap.add_argument("--roofline-nvec", type=int, default=0,
                    help="basis size of the Gram-Schmidt roofline launches (default: from the timed solves)")
    ap.add_argument("--d3-case", default="", help="d3: one row only, N,box,dtK (e.g. 64,4,100)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only copy a device buffer of this many MiB, 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.cpu_leg:
        return cpu_leg_c3()
    if not args.forms:
        args.forms = ",".join(C3_FORMS) if args.workload == "c3" else "concurrent,plain,fp32,tuned"
    if args.copy_probe:
        import torch
        a = torch.ones(args.copy_probe * (1 << 20) // 8, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_mib": args.copy_probe, "launches": 5}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (multi-GPU sharding is "
                                   "described in DESIGN.md, not implemented)"}))
        sys.exit(2)
    import torch
    from paper_1311_5614_amd import ibmg
    dev = "cuda:0"
    if args.probe_only:
        print(json.dumps({"probe": vcycle_probe(dev, args.probe_n, colours=args.colours)}))
        return
    if args.workload == "c5":
        return run_learned(args, dev)
    if args.workload == "mgsolver":
        print(json.dumps({"mg_solver": run_mg_solver(args, dev)}))
        return
    if args.workload == "efficiency":
        print(json.dumps({"efficiency": run_efficiency(args, dev)}))
        return
    if args.workload == "cavity":
        print(json.dumps({"cavity": run_cavity(args, dev)}))
        return
    if args.workload == "d3":
        only = None
        if args.d3_case:
            a, b, c = args.d3_case.split(",")
            only = (int(a), int(b), float(c))
        print(json.dumps({"d3": run_d3(args, dev, steps=args.steps or 5, only=only)}))
        return
    args.steps = args.steps or 20
    if args.workload == "c3":
        out, leg = run_c3(args, dev)
        if not args.no_extras:
            extra = {}
            for wl, forms, steps in (("c2", ("concurrent", "plain"), 20), ("c4", ("batch",), 10)):
                try:
                    r = run_sweep(args, dev, wl, forms, steps, 1)
                    r.pop("_cases", None)
                    extra[wl] = {k: r[k] for k in ("value", "unit", "ms_per_step", "config", "forms")}
                except Exception as e:   # noqa: BLE001  (extra figures; the headline stands without them)
                    extra[wl] = {"error": f"{type(e).__name__}: {e}"}
            try:
                extra["implicit_vs_explicit"] = run_efficiency(args, dev)
            except Exception as e:   # noqa: BLE001
                extra["implicit_vs_explicit"] = {"error": f"{type(e).__name__}: {e}"}
            out["extra_workloads"] = extra
        if not args.no_probe:
            try:
                out["probe"] = vcycle_probe(dev)
            except Exception as e:   # the probe is an extra figure; the workload's line stands without it
                out["probe"] = {"error": f"{type(e).__name__}: {e}"}
        if leg is not None:
            out["cpu_baseline"] = finish_cpu_leg(*leg, iters_per_step=out["forms"]["chosen"]["iters_mean"]
                                                 if "chosen" in out["forms"] else 100.0)
        print(json.dumps(out))
        return
    steps = args.steps or 20
    out = run_sweep(args, dev, args.workload, args.forms.split(","), steps, args.warmup)
    cases, dts = out.pop("_cases")
    if not args.no_probe:
        try:
            out["probe"] = vcycle_probe(dev)
        except Exception as e:   # the probe is an extra figure; the workload's line stands without it
            out["probe"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_cpu:
        k = 2 if len(cases) > 2 else 0
        out["cpu_baseline"] = cpu_baseline(cases[k], dts[k], "bounded sample of the same workload")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
