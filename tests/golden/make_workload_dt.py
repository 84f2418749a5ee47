"""Write tests/golden/workload_dt.json: the explicit stability limit of each
seeded workload, computed by the oracle only.

For each workload instance this stores lambda_max, the spectral radius of
S^* L_0^{-1} S (-L) at the initial configuration (steady periodic MAC Stokes,
mu = 1), from which dt_exp = 2 / (K lambda_max) (explicit-stability analysis,
Sec. 4.1 of the paper, read for nodal springs) and the workload's
dt = factor * dt_exp.  The time step is an input of the solve; the GPU path
reads it from this file and never computes it.

For the walled test problem ("cavity") it stores alpha_exp of the thick
annulus at N = 32, 64, 128 (Table 1's quantity, from the oracle).

Usage: python tests/golden/make_workload_dt.py [c1 c2 c3 c4 c5 cavity]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import ibgen  # noqa: E402
from oracle import dtexp  # noqa: E402

OUT = os.path.join(HERE, "workload_dt.json")


def entry(w):
    t = time.time()
    lam = dtexp.lambda_max(w.X, w.fiber_offsets, w.N, w.mu)
    dt_exp = 2.0 / (w.K * lam)
    return dict(name=w.name, N=w.N, M=w.M, K=w.K, factor=w.dt_factor, lambda_max=lam,
                dt_exp=dt_exp, dt=w.dt_factor * dt_exp, seed=w.seed,
                seconds=round(time.time() - t, 2))


def main(which):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    if "c1" in which:
        data["c1"] = [entry(ibgen.config_c1())]
    if "c2" in which:
        cases = ibgen.config_c2_cases()
        lam_entry = entry(cases[0])
        out = []
        for w in cases:   # shared geometry: lambda_max is K-independent
            e = dict(lam_entry)
            e.update(name=w.name, K=w.K, factor=w.dt_factor,
                     dt_exp=2.0 / (w.K * lam_entry["lambda_max"]))
            e["dt"] = w.dt_factor * e["dt_exp"]
            out.append(e)
        data["c2"] = out
    if "c3" in which:
        data["c3"] = [entry(ibgen.config_c3())]
    if "c4" in which:
        data["c4"] = [entry(w) for w in ibgen.config_c4()]
    if "c5" in which:
        data["c5"] = [entry(ibgen.config_c5())]
    if "cavity" in which:   # the walled test problem: alpha_exp of Table 1 (Sec. 4.1)
        from oracle import cavity
        data["cavity"] = [dict(N=N, alpha_exp=cavity.alpha_exp(N)) for N in (32, 64, 128)]
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print("wrote", OUT, sorted(data))


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2", "c5"])
