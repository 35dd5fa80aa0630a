"""Writes tests/golden/solve_ds_n128.json: the oracle's sparse-LU solution of the coupled
Darcy-Stokes system (Sec. 4, eq. (darcy_stokes); Taylor-Hood P2-P1 Stokes on (0,1) x (1,2), P1
Darcy pressure on the unit square, n = 128, K = 1e-2, mu = 1e-4, alpha = 3,
b = workloads.normal_vector(N, 128)), sampled at 4096 seeded indices plus its norm.  Calls only
oracle/ and the input generator.

    python tests/golden/make_ds_n128.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import darcy_stokes  # noqa: E402

N_CELLS, K, MU, ALPHA, SEED, SAMPLES = 128, 1e-2, 1e-4, 3.0, 128, 4096


def main():
    t0 = time.time()
    P = darcy_stokes.DarcyStokes(N_CELLS, K, MU, ALPHA)
    t1 = time.time()
    b = workloads.normal_vector(P.N, SEED)
    x = P.solve_splu(b)
    t2 = time.time()
    res = float(np.linalg.norm(P.A @ x - b) / np.linalg.norm(b))
    idx = np.sort(np.random.default_rng(SEED).choice(len(x), SAMPLES, replace=False))
    out = {"problem": "coupled Darcy-Stokes, eq. (darcy_stokes)", "n": N_CELLS, "K": K, "mu": MU,
           "alpha": ALPHA, "rhs": f"workloads.normal_vector(N, {SEED})",
           "solver": "oracle DarcyStokes.solve_splu", "N": int(len(x)),
           "norm_x": float(np.linalg.norm(x)), "oracle_rel_residual": res,
           "indices": idx.tolist(), "values": [float(v) for v in x[idx]],
           "seconds": {"assembly": round(t1 - t0, 1), "solve": round(t2 - t1, 1)}}
    with open(os.path.join(ROOT, "tests", "golden", "solve_ds_n128.json"), "w") as f:
        json.dump(out, f)
    print(f"N {len(x)} residual {res:.2e} assembly {t1 - t0:.1f} s solve {t2 - t1:.1f} s")


if __name__ == "__main__":
    main()
