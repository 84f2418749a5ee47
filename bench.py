"""Benchmark: implicit IB time steps per second on one MI355X.

Workload (default): the 256x256 single-ellipse stiffness sweep -- one
perturbed ellipse of 1024 points, a smooth random body force (16 Fourier
modes per component), springs K in {1e2, 1e4, 1e6, 1e8} and dt in {100, 1000}
x the explicit stability limit: 8 independent trajectories.  One bench step
advances every trajectory by one implicit time step (FGMRES to relative
residual 1e-8, V(2,2), 4x4 boxes, 5 levels).  Timed twice from the same
initial state: the plain FP64 solver and the chosen form (FP32 V-cycle
inside FP64 FGMRES).  `value` is the chosen form's whole-job rate in
time steps per second; inputs are resident in HBM before timing starts.

Also reported: iterations per solve for both forms, the HIP-event
roofline of the dominant kernel (the box-relaxation phase kernel), and the
CPU oracle timed on a bounded sample on the host.

python bench.py [--gpus 1] [--steps 20] [--warmup 1] [--workload c2|c1|c5|c3]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "IB time-steps/sec and FGMRES iters/solve at rel resid 1e-8, plain vs chosen"


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
    if name == "c5":
        return [ibgen.config_c5()], [load_dt("c5")[0]["dt"]]
    if name == "c3":
        return [ibgen.config_c3()], [load_dt("c3")[0]["dt"]]
    if name == "c4":
        return ibgen.config_c4(), [d["dt"] for d in load_dt("c4")]
    raise SystemExit(f"unknown workload {name}")


class Run:
    """Device state of one trajectory plus its solver handle."""

    def __init__(self, w, dt, prec, dev):
        import torch
        from paper_1311_5614_amd import ibmg
        self.w, self.dt = w, dt
        cfg = ibmg.Config(N=w.N, levels=w.levels, K=w.K, rho=w.rho, mu=w.mu, box=w.box, nu1=w.nu1,
                          nu2=w.nu2, maxit=100, rtol=w.rtol, prec=prec, colours=getattr(w, "colours", 2),
                          tail_max=getattr(w, "tail_max", 0))
        self.s = ibmg.Solver(cfg, w.fiber_offsets, dev)
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
                            nu2=w.nu2, maxit=100, rtol=w.rtol, prec=prec, colours=getattr(w, "colours", 2),
                            tail_max=getattr(w, "tail_max", 0))
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


def timed(runs, steps, warmup, timing=False):
    """Warm up, reset every trajectory, then time `steps` steps of all of them.
    With timing set, the box kernels are event-timed (eager launches instead of
    the replayed V-cycle graph)."""
    import torch
    for r in runs:
        r.reset()
    for _ in range(warmup):
        for r in runs:
            r.step()
    for r in runs:
        r.reset()
        r.s.set_timing(timing)
    torch.cuda.synchronize()
    its, conv = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        for r in runs:
            st = r.step()
            its.append(st["iters"])
            conv.append(st["converged"])
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
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


def cpu_baseline(w, dt, budget_note):
    """Oracle (plain numpy/scipy, FP64) on one time step of one case."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import step as ostep
    N = w.N
    z = np.zeros((N, N))
    with threadpool_limits(1):
        t0 = time.perf_counter()
        o = ostep.step(z, z, z, w.X, w.fiber_offsets, w.K, dt, w.levels, w.rho, w.mu, w.box, w.nu1,
                       w.nu2, w.rtol, g_u=w.g_u, g_v=w.g_v)
        t = time.perf_counter() - t0
    return {"value": 1.0 / t, "unit": "time-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"1 implicit step of {w.name} ({o.iters} FGMRES iterations, {t:.1f} s); "
                      f"1 BLAS thread; {budget_note}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--forms", default="plain,fp32")
    ap.add_argument("--levels", type=int, default=0, help="override the workload's level count")
    ap.add_argument("--nu", default="", help="override smoothing sweeps, e.g. 1,1")
    ap.add_argument("--colours", type=int, default=2)
    ap.add_argument("--tail-max", type=int, default=0, help="override the V-cycle tail size")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only copy a device buffer of this many MiB, 5 times (HBM counter calibration)")
    args = ap.parse_args()
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
    cases, dts = workloads(args.workload)
    for c in cases:
        if args.levels:
            c.levels = args.levels
        if args.nu:
            c.nu1, c.nu2 = (int(x) for x in args.nu.split(","))
        c.colours = args.colours
        if args.tail_max:
            c.tail_max = args.tail_max
    forms = args.forms.split(",")
    res = {}
    for form in forms:
        if form.startswith("batch"):
            # all trajectories in one batch handle: "batch" = FP32 V-cycle, "batch64" = FP64
            prec = ibmg.IBMG_FP64 if form == "batch64" else ibmg.IBMG_FP32
            br = BatchRun(cases, dts, prec, dev)
            t, its, conv, rounds = timed_batch(br, args.steps, args.warmup)
            n = args.steps * len(cases)
            res[form] = dict(time_s=t, timesteps=n, rate=n / t, iters_mean=sum(its) / len(its), iters_max=max(its),
                             converged=sum(conv), rounds=rounds, phase=None)
            print(f"[bench] {form}: {n} steps in {t:.3f} s -> {n / t:.2f} steps/s, iters mean "
                  f"{res[form]['iters_mean']:.2f} max {max(its)}, converged {sum(conv)}/{n}, {rounds} lockstep "
                  f"rounds", file=sys.stderr, flush=True)
            del br
            torch.cuda.empty_cache()
            continue
        prec = ibmg.IBMG_FP32 if form == "fp32" else ibmg.IBMG_FP64
        runs = [Run(w, dt, prec, dev) for w, dt in zip(cases, dts)]
        t, its, conv, _ = timed(runs, args.steps, args.warmup, timing=False)
        # roofline of the box kernel: the same trajectories, one more (untimed)
        # step with every box launch bracketed by HIP events on its stream
        _, _, _, ph = timed(runs, 1, 0, timing=True)
        n = args.steps * len(runs)
        res[form] = dict(time_s=t, timesteps=n, rate=n / t, iters_mean=sum(its) / len(its), iters_max=max(its),
                         converged=sum(conv), phase=ph)
        print(f"[bench] {form}: {n} steps in {t:.3f} s -> {n / t:.2f} steps/s, iters mean "
              f"{res[form]['iters_mean']:.2f} max {max(its)}, converged {sum(conv)}/{n}; per case "
              f"{[round(sum(its[c::len(runs)]) / args.steps, 1) for c in range(len(runs))]}", file=sys.stderr,
              flush=True)
        del runs
        torch.cuda.empty_cache()
    chosen = next((f for f in ("batch", "fp32") if f in res), forms[0])
    rc = res[chosen]
    ph = next((res[f]["phase"] for f in (chosen, "fp32", "plain") if f in res and res[f]["phase"]), None)
    achieved = ph["bytes"] / (ph["total_ms"] * 1e-3) / 1e9 if ph and ph["total_ms"] > 0 else None
    w0 = cases[0]
    out = {
        "metric": METRIC,
        "value": rc["rate"],
        "unit": "time-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * rc["time_s"] / args.steps,
        "ms_per_timestep": 1e3 * rc["time_s"] / rc["timesteps"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if chosen == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{len(cases)} trajectories on {w0.N}x{w0.N}, {w0.M} Lagrangian points, "
                         f"{w0.levels} levels, V({w0.nu1},{w0.nu2}), box {w0.box}, rtol {w0.rtol:g}"),
            "grid": w0.N, "points": w0.M, "trajectories": len(cases), "levels": w0.levels,
            "K": sorted({c.K for c in cases}), "dt_factor": sorted({c.dt_factor for c in cases}),
            "chosen_form": "fp32 V-cycle inside fp64 FGMRES" if chosen == "fp32" else chosen,
        },
        "forms": {k: {kk: vv for kk, vv in v.items() if kk != "phase"} for k, v in res.items()},
        "roofline": {
            "kernel": "k_box (box relaxation, one colour phase)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": None,
            "launches": ph["launches"] if ph else 0,
            "avg_launch_us": 1e3 * ph["total_ms"] / ph["launches"] if ph and ph["launches"] else None,
        },
    }
    if not args.no_cpu:
        k = 2 if len(cases) > 2 else 0
        out["cpu_baseline"] = cpu_baseline(cases[k], dts[k], "bounded sample of the same workload")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
