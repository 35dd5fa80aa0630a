"""Writes tests/golden/solve_3d_n64.json: the oracle's sparse-LU solution of the 3D Riesz-map
problem (eq. (riesz), Kuhn tetrahedra, n = 64, K = 1, mu = 1e-4, b = workloads.rhs(3, 64, 3064)),
sampled at 4096 seeded indices plus its norm.  Calls only oracle/ and the input generator.

    python tests/golden/make_3d_n64.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import system  # noqa: E402

N_CELLS, K, MU, SEED, SAMPLES = 64, 1.0, 1e-4, 3064, 4096


def main():
    t0 = time.time()
    R = system.Riesz(3, N_CELLS, K, MU)
    t1 = time.time()
    b = workloads.rhs(3, N_CELLS, SEED)
    x = R.solve_splu(b)
    t2 = time.time()
    res = float(np.linalg.norm(R.apply(x) - b) / np.linalg.norm(b))
    idx = np.sort(np.random.default_rng(SEED).choice(len(x), SAMPLES, replace=False))
    out = {"problem": "3D Riesz map, eq. (riesz), Gamma = the face z = 1", "n": N_CELLS, "K": K,
           "mu": MU, "rhs": f"workloads.rhs(3, {N_CELLS}, {SEED})", "solver": "oracle Riesz.solve_splu",
           "N": int(len(x)), "norm_x": float(np.linalg.norm(x)), "oracle_rel_residual": res,
           "indices": idx.tolist(), "values": [float(v) for v in x[idx]],
           "seconds": {"assembly": round(t1 - t0, 1), "solve": round(t2 - t1, 1)}}
    with open(os.path.join(ROOT, "tests", "golden", "solve_3d_n64.json"), "w") as f:
        json.dump(out, f)
    print(f"N {len(x)} residual {res:.2e} assembly {t1 - t0:.1f} s solve {t2 - t1:.1f} s")


if __name__ == "__main__":
    main()
