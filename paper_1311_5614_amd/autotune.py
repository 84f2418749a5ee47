"""Schedule autotuner for the multigrid preconditioner.

For each problem class of a workload (the 256x256 stiffness sweep: one class
per (K, dt) case; the batch: one class per grid size; the 1024x1024
eight-ring trajectory: one class, timed over a dozen steps because its later
steps are the hard ones) it times candidate
V-cycle schedules on seeded calibration problems -- same class, geometry
drawn with other seeds than the benchmark's -- and keeps, per class, the
fastest schedule whose steps all reach the tolerance.  A schedule is

    box       box edge n (4 x 4 or 8 x 8 cells; the batch takes 4 x 4 only),
    levels    multigrid depth (coarsest 4^2, 8^2 or 16^2),
    tail_max  largest level run by the LDS-resident one-workgroup tail,
    nu1, nu2  smoothing sweeps (Algorithm 1),
    colours   box colour classes of a sweep (2 or 4), and colours_from, the
              level from which the checkerboard order takes over,
    prec      V-cycle precision (FP32, or FP64 where FP32 is slower or stalls),

inside FP64 FGMRES.  The result is written as JSON
(`schedules.json` next to this file) and read by the benchmark.  Time steps
use the dt values stored for the workload (tests/golden/workload_dt.json,
written by the oracle's explicit-limit estimate) for the class.

python -m paper_1311_5614_amd.autotune [--workload c2|c4|c3|all] [--steps 2]
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "schedules.json")
CAL_INSTANCE = 900   # seeds 1311000 + 100 * config + 900 + k are calibration-only
CAL_GEOMETRIES = 2   # calibration geometries per class (256x256 sweep, 1024x1024 rings)
MAXIT = 200          # FGMRES iteration cap (no restart), as in the benchmark
C3_BASIS, C3_CAP = 600, 1000   # the 1024x1024 trajectory: FGMRES(600), at most 1000 iterations


def _dt_table():
    with open(os.path.join(ROOT, "tests", "golden", "workload_dt.json")) as f:
        return json.load(f)


def classes(workload):
    """(key, [calibration Workloads], dt) per class of the workload."""
    import numpy as np
    sys.path.insert(0, ROOT)
    import ibgen
    dts = _dt_table()
    out = []
    if workload == "c2":
        geos = []
        for g in range(CAL_GEOMETRIES):
            rng = np.random.default_rng(ibgen.seed_for(2, CAL_INSTANCE + g))
            X, _ = ibgen.ellipse(rng, 1024)
            gu, gv = ibgen.fourier_force(rng, 256)
            geos.append((X, gu, gv, ibgen.seed_for(2, CAL_INSTANCE + g)))
        for case, d in zip(ibgen.config_c2_cases(), dts["c2"]):
            ws = [ibgen.Workload(f"cal-{case.name}", 256, case.levels, X.copy(), np.array([0, 1024], np.int32),
                                 case.K, case.dt_factor, rtol=case.rtol, g_u=gu, g_v=gv, seed=seed)
                  for X, gu, gv, seed in geos]
            out.append((f"{case.K:.0e}-{int(case.dt_factor)}", ws, d["dt"]))
    elif workload == "c4":
        cases = ibgen.config_c4()
        seen = set()
        for case, d in zip(cases, dts["c4"]):
            if case.N in seen:
                continue
            seen.add(case.N)
            rng = np.random.default_rng(ibgen.seed_for(4, CAL_INSTANCE + len(seen)))
            X, _ = ibgen.ellipse(rng, case.M)
            w = ibgen.Workload(f"cal-{case.N}", case.N, case.levels, X, np.array([0, case.M], np.int32),
                               1e5, case.dt_factor, rtol=case.rtol, seed=ibgen.seed_for(4, CAL_INSTANCE))
            # dt of the class: the stored dt of this grid size rescaled from its K to 1e5
            out.append((str(case.N), [w], d["dt"] * case.K / 1e5))
    elif workload == "c3":
        c3 = ibgen.config_c3()
        ws = []
        for g in range(CAL_GEOMETRIES):
            seed = ibgen.seed_for(3, CAL_INSTANCE + g)
            X, offs, _ = ibgen.rings(np.random.default_rng(seed), 8, 2048, c3.N)
            ws.append(ibgen.Workload(f"cal-1024-{g}", c3.N, c3.levels, X, offs, c3.K, c3.dt_factor,
                                     rtol=c3.rtol, seed=seed))
        out.append(("1024", ws, dts["c3"][0]["dt"]))
    else:
        raise SystemExit(f"unknown workload {workload}")
    return out


def candidates_c3(w):
    """The eight-ring trajectory: FP64 V-cycles of 4 x 4 boxes down to 16^2,
    the coarsest solve spread over the grid (tail 1), over box orders (four
    colours on every level, on the two or three finest only, or the
    checkerboard throughout) and sweeps.  FP32 V-cycles are tried on the best of these in
    the second stage.  FGMRES delays its second Gram-Schmidt projection
    (orth 1), as the benchmark's chosen form does.  (V(3,3) stalled on a
    calibration step in every order and weight, and V(2,2) with four colours
    on every level overflowed; neither is tried any more.)  Box weights 1,
    0.8 and 0.6."""
    for (col, cf), nu, om in itertools.product(((4, 2), (4, 3), (2, 0)), ((2, 2), (2, 1), (1, 1)), (1.0, 0.8, 0.6)):
        yield dict(box=4, levels=w.levels, tail_max=1, nu1=nu[0], nu2=nu[1], colours=col, colours_from=cf, prec=0,
                   maxit=C3_CAP, restart=C3_BASIS, omega=om, guess=1, orth=1)
    # 8 x 8 boxes (Sec. 6: bigger boxes flatten the growth with stiffness), checkerboard
    for nu, om in itertools.product(((2, 1), (1, 1)), (1.0, 0.8)):
        yield dict(box=8, levels=w.levels, tail_max=1, nu1=nu[0], nu2=nu[1], colours=2, colours_from=0, prec=0,
                   maxit=C3_CAP, restart=C3_BASIS, omega=om, guess=1, orth=1)


def candidates(w, boxes=(4,)):
    """Stage 1: the parameters that change convergence (box, depth, sweeps,
    colours), with the tail at 8.  A smoothed level holds at least two boxes
    per side, so 8 x 8 boxes stop at an 8^2 or 16^2 coarsest grid."""
    full = w.levels
    for box in boxes:
        lv = [full - d for d in (0, 1, 2)
              if (w.N >> (full - d - 1)) <= 16 and (w.N >> (full - d - 2)) >= 2 * box]
        for levels, nu, col in itertools.product(lv, ((1, 1), (2, 2), (3, 3), (2, 1)), (2, 4)):
            yield dict(box=box, levels=levels, tail_max=8, nu1=nu[0], nu2=nu[1], colours=col, prec=1)


def tails(w, sch):
    """Stage 2: launch schedules of one V-cycle (tail sizes), and the FP64
    V-cycle at the stage-1 tail.  (8 x 8 boxes run no LDS-resident tail.)"""
    for tail in (1, 8, 16, 32):
        if tail >= 8 and ((w.N >> (sch["levels"] - 1)) > tail or sch["box"] > 4):
            continue   # the tail would hold only the coarsest level: same as tail 1
        yield dict(sch, tail_max=tail)
    yield dict(sch, prec=0)


def time_schedule(w, dt, sch, steps, dev):
    import torch
    from . import ibmg
    cfg = ibmg.Config(N=w.N, levels=sch["levels"], K=w.K, box=sch["box"], nu1=sch["nu1"], nu2=sch["nu2"],
                      maxit=sch.get("maxit", MAXIT), restart=sch.get("restart", 0), rtol=w.rtol, prec=sch["prec"],
                      colours=sch["colours"], colours_from=sch.get("colours_from", 0), tail_max=sch["tail_max"],
                      omega=sch.get("omega", 1.0), guess=sch.get("guess", 0), orth=sch.get("orth", 0))
    s = ibmg.Solver(cfg, w.fiber_offsets, dev)
    t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev).contiguous()
    gu = t(w.g_u) if w.g_u is not None else None
    gv = t(w.g_v) if w.g_v is not None else None
    z = torch.zeros(w.N, w.N, dtype=torch.float64, device=dev)
    u, v, p, X = z.clone(), z.clone(), z.clone(), t(w.X)
    s.step(dt, u, v, p, X, gu, gv)          # warm-up (graph capture)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its, ok = [], True
    for _ in range(steps):
        st = s.step(dt, u, v, p, X, gu, gv)
        its.append(st["iters"])
        if st["converged"] != 1:   # a schedule that misses rtol is out: stop timing it
            ok = False
            break
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / len(its)
    s.close()
    return el, its, ok


def _try(ws, dt, sch, steps, dev, workload, key):
    """Mean time per step and the iterations over the class's calibration
    geometries."""
    from .ibmg import IBMGError
    el, its, ok = 0.0, [], True
    try:
        for w in ws:
            e1, i1, o1 = time_schedule(w, dt, sch, steps, dev)
            el += e1 / len(ws)
            its += i1
            ok = ok and o1
    except IBMGError as e:          # e.g. a diverged trajectory leaves the window
        print(f"[autotune] {workload} {key} {sch} -> error {e}", flush=True)
        return None
    print(f"[autotune] {workload} {key} {sch} -> {1e3 * el:.2f} ms/step, iters {its}"
          f"{'' if ok else ' NOT CONVERGED'}", flush=True)
    return el, its, ok


def tune(workload, steps, dev="cuda:0"):
    """Per class: the fastest converging schedule; if none converges, the one
    with the fewest iterations (recorded with converged = false)."""
    res = {}
    boxes = (4, 8) if workload == "c2" else (4,)   # the batched kernels take 4 x 4 boxes
    for key, ws, dt in classes(workload):
        w = ws[0]
        scored, failed = [], []
        for sch in (candidates_c3(w) if workload == "c3" else candidates(w, boxes)):
            r = _try(ws, dt, sch, steps, dev, workload, key)
            if r is None:
                continue
            (scored if r[2] else failed).append((r[0], sch, r[1]))
        if scored:
            scored.sort(key=lambda x: x[0])
            best, conv = scored[0], True
            top = scored[:3]
        else:
            failed.sort(key=lambda x: (sum(x[2]), x[0]))
            best, conv = failed[0], False
            top = failed[:1]
        for _, sch, _ in top:
            for cand in ([dict(sch, prec=1)] if workload == "c3" else tails(w, sch)):
                if cand == sch:
                    continue
                r = _try(ws, dt, cand, steps, dev, workload, key)
                if r is None:
                    continue
                el, its, ok = r
                if ok and (not conv or el < best[0]):
                    best, conv = (el, cand, its), True
                elif not conv and not ok and sum(its) < sum(best[2]):
                    best = (el, cand, its)
        res[key] = dict(best[1], ms_per_step=round(1e3 * best[0], 3), iters=best[2], converged=conv)
        print(f"[autotune] {workload} {key} best {res[key]}", flush=True)
    return res


def load(path=OUT):
    with open(path) as f:
        return json.load(f)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="all")
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args()
    data = load(args.out) if os.path.exists(args.out) else {}
    for wl in (("c2", "c4", "c3") if args.workload == "all" else (args.workload,)):
        old = data.get(wl, {})
        data[wl] = tune(wl, args.steps)
        for key, sch in data[wl].items():   # the start rule is chosen by hand, not tuned: keep it
            if isinstance(old.get(key), dict) and "start" in old[key]:
                sch["start"] = old[key]["start"]
    meta = data.get("meta", {})
    meta.update({"form": "V-cycle (prec 1 = fp32, 0 = fp64) in fp64 FGMRES", "c2_geometries": CAL_GEOMETRIES,
                 "c3_geometries": CAL_GEOMETRIES,
                 "calibration_instance": CAL_INSTANCE, "maxit": MAXIT})
    meta.pop("steps_timed", None)
    for wl in (("c2", "c4", "c3") if args.workload == "all" else (args.workload,)):
        meta[f"steps_timed_{wl}"] = args.steps
    data["meta"] = meta
    with open(args.out, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print(f"[autotune] wrote {args.out}")


if __name__ == "__main__":
    main()
