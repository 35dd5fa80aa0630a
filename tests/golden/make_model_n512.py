"""Writes tests/golden/solve_model_n512.json: the oracle's sparse-LU solution of the paper's own
model problem (Sec. 3, eq. (model_problem); 2D, Gamma = the whole boundary, exact L^t by eq.
(gevp)) at n = 512, K = 1, gamma = 1, t = -1/2, b = workloads.normal_vector(N, 5120), sampled at
4096 seeded indices plus its norm.  Calls only oracle/ and the input generator.

    python tests/golden/make_model_n512.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import model  # noqa: E402

N_CELLS, K, GAMMA, T, SEED, SAMPLES = 512, 1.0, 1.0, -0.5, 5120, 4096


def main():
    t0 = time.time()
    P = model.ModelProblem(N_CELLS, K, GAMMA, T)
    t1 = time.time()
    b = workloads.normal_vector(P.N, SEED)
    x = P.solve_splu(b)
    t2 = time.time()
    res = float(np.linalg.norm(P.apply(x) - b) / np.linalg.norm(b))
    idx = np.sort(np.random.default_rng(SEED).choice(len(x), SAMPLES, replace=False))
    out = {"problem": "model problem, eq. (model_problem), Gamma = the boundary", "n": N_CELLS,
           "K": K, "gamma": GAMMA, "t": T, "rhs": f"workloads.normal_vector(N, {SEED})",
           "solver": "oracle ModelProblem.solve_splu", "N": int(len(x)),
           "norm_x": float(np.linalg.norm(x)), "oracle_rel_residual": res,
           "indices": idx.tolist(), "values": [float(v) for v in x[idx]],
           "seconds": {"assembly_and_gevp": round(t1 - t0, 1), "solve": round(t2 - t1, 1)}}
    with open(os.path.join(ROOT, "tests", "golden", "solve_model_n512.json"), "w") as f:
        json.dump(out, f)
    print(f"N {len(x)} residual {res:.2e} set-up {t1 - t0:.1f} s solve {t2 - t1:.1f} s")


if __name__ == "__main__":
    main()
