"""Writes tests/golden/solve_hdiv_n256.json: the oracle's sparse-LU solution of the H(div)
problem (Sec. 3 remark on H(div)-elliptic problems, eq. (graddiv); BDM1, Gamma = the whole
boundary) at n = 256, K = 1, gamma = 1, b = workloads.normal_vector(N, 2560), sampled at 4096
seeded indices plus its norm.  The sparse LU alone leaves a relative residual of ~6e-9 at this size,
so its solution is improved by iterative refinement with the same factorization
(x += LU^{-1} (b - A x)) while a step at least halves the residual: it settles at ~1e-10, the
rounding floor of b - A x for this system (||x|| ~ ||b|| / h^2, so ||A|| ||x|| >> ||b||).  Calls only oracle/ (its assembled matrix) and the input generator.

    python tests/golden/make_hdiv_n256.py
"""
import json
import os
import sys
import time

import numpy as np
import scipy.sparse.linalg as spla

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import hdiv  # noqa: E402

N_CELLS, K, GAMMA, SEED, SAMPLES = 256, 1.0, 1.0, 2560, 4096


def main():
    t0 = time.time()
    P = hdiv.HdivProblem(N_CELLS, K, GAMMA)
    t1 = time.time()
    b = workloads.normal_vector(P.N, SEED)
    lu = spla.splu(P.A.tocsc())
    x = lu.solve(b)
    res0 = float(np.linalg.norm(P.apply(x) - b) / np.linalg.norm(b))
    steps, r = 0, np.linalg.norm(P.apply(x) - b)
    while steps < 40:
        y = x + lu.solve(b - P.apply(x))
        ry = np.linalg.norm(P.apply(y) - b)
        if ry > 0.5 * r:
            break
        x, r, steps = y, ry, steps + 1
    t2 = time.time()
    res = float(np.linalg.norm(P.apply(x) - b) / np.linalg.norm(b))
    idx = np.sort(np.random.default_rng(SEED).choice(len(x), SAMPLES, replace=False))
    out = {"problem": "H(div), eq. (graddiv), BDM1", "n": N_CELLS, "K": K, "gamma": GAMMA,
           "rhs": f"workloads.normal_vector(N, {SEED})", "solver": "oracle HdivProblem.solve_splu",
           "N": int(len(x)), "norm_x": float(np.linalg.norm(x)), "oracle_rel_residual": res,
           "indices": idx.tolist(), "values": [float(v) for v in x[idx]],
           "seconds": {"assembly": round(t1 - t0, 1), "solve": round(t2 - t1, 1)}}
    with open(os.path.join(ROOT, "tests", "golden", "solve_hdiv_n256.json"), "w") as f:
        json.dump(out, f)
    print(f"N {len(x)} residual {res0:.2e} -> {res:.2e} ({steps} refinement steps) assembly {t1 - t0:.1f} s solve {t2 - t1:.1f} s")


if __name__ == "__main__":
    main()
