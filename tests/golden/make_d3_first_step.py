"""Writes d3_first_step_64.json: the oracle's FGMRES(40) on the first implicit
step from rest of the 3-D benchmark problem at 64^3 (closed latitude rings
on a stretched sphere, ibgen.sphere_rings(64); rho = mu = 1, dt = 0.01,
K = 1e3; 4^3 boxes, checkerboard, V(1,1), five levels).  Calls oracle/ and
ibgen/ only.  About three minutes on one core.

Usage: python tests/golden/make_d3_first_step.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import ibgen  # noqa: E402
from oracle import d3, krylov  # noqa: E402

N, LEVELS, DT, K, BOX, MAXIT = 64, 5, 0.01, 1e3, 4, 40


def main():
    X, offs = ibgen.sphere_rings(N)
    lv = d3.hierarchy(N, LEVELS, 1.0, 1.0, DT, X, offs, K)
    V = d3.VCycle(lv, BOX, 1, 1)
    z = np.zeros(N ** 3)
    b = d3.rhs(N, 1.0 / DT, [z] * 3, X, offs, K)
    res = krylov.fgmres(lv[0].A, b, V, rtol=1e-8, maxit=MAXIT)
    out = {"N": N, "levels": LEVELS, "dt": DT, "K": K, "box": BOX, "nu": [1, 1], "maxit": MAXIT,
           "iters": res.iters, "converged": bool(res.converged),
           "rel_resid_true": float(np.linalg.norm(b - lv[0].A @ res.x) / np.linalg.norm(b)),
           "history": [float(h) for h in res.history]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "d3_first_step_64.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["iters"], out["rel_resid_true"])


if __name__ == "__main__":
    main()
