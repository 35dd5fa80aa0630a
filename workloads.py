"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers and lays out parameter sweeps.  It holds none
of the solver's arithmetic, so both the GPU path and the CPU oracle may use it.

Workload shapes follow the paper's experiments: the unit square (or cube) with
Gamma a boundary facet, P1 elements, K and mu swept over orders of magnitude, and a
right-hand side b in V' drawn i.i.d. N(0, 1) over all free dofs.
"""
import numpy as np


def free_dof_count(dim, n):
    """Number of free dofs: interior plus the interface facet."""
    return n * (n - 1) if dim == 2 else n * (n - 1) ** 2


def rhs(dim, n, seed):
    """b ~ N(0, 1) in float64 over all free dofs (Gamma dofs last)."""
    return np.random.default_rng(seed).standard_normal(free_dof_count(dim, n))


def sweep_2d():
    """The 2D mesh/parameter sweep: n x K x mu, with a seed per case."""
    cases = []
    idx = 0
    for n in (128, 256, 512, 1024, 2048):
        for K in (1.0, 1e-2, 1e-4):
            for mu in (1e-6, 1e-3, 1.0, 1e3):
                cases.append(dict(n=n, K=K, mu=mu, seed=1000 + idx))
                idx += 1
    return cases


def sweep_3d():
    """The 3D sweep: n x mu at K = 1."""
    cases = []
    idx = 0
    for n in (32, 64, 128):
        for mu in (1e-4, 1.0, 1e2):
            cases.append(dict(n=n, K=1.0, mu=mu, seed=3000 + idx))
            idx += 1
    return cases


def batch_instances(count=256, seed=4, sizes=None):
    """Independent 2D instances: n uniform on {64, 96, ..., 512}, log-uniform K and mu.

    log10 K ~ U[-4, 0], log10 mu ~ U[-6, 2]; instance i uses rhs seed 4000 + i.
    """
    rng = np.random.default_rng(seed)
    grid = np.arange(64, 513, 32) if sizes is None else np.asarray(sizes)
    out = []
    for i in range(count):
        n = int(rng.choice(grid))
        K = float(10.0 ** rng.uniform(-4.0, 0.0))
        mu = float(10.0 ** rng.uniform(-6.0, 2.0))
        out.append(dict(n=n, K=K, mu=mu, seed=4000 + i))
    return out


def sine_series_traces(count, n, kmax=64, seed=5):
    """Interface traces sum_{k<=kmax} a_k sin(k pi x) at the n-1 free Gamma nodes.

    a_k ~ N(0, 1/k^2) (standard deviation 1/k).  Returns (coeffs (count, kmax),
    traces (count, n-1)).
    """
    rng = np.random.default_rng(seed)
    k = np.arange(1, kmax + 1)
    a = rng.standard_normal((count, kmax)) / k[None, :]
    x = np.arange(1, n) / n
    basis = np.sin(np.pi * k[:, None] * x[None, :])      # (kmax, n-1)
    return a, a @ basis


def cnn_init(widths=(5, 32, 32, 32, 32, 32, 1), seed=6):
    """Seeded He-normal weights (std sqrt(2 / fan_in), fan_in = 9 C_in) and zero biases.

    Returns [(W (3, 3, C_in, C_out), b (C_out,))] in float64.
    """
    rng = np.random.default_rng(seed)
    params = []
    for cin, cout in zip(widths[:-1], widths[1:]):
        W = rng.standard_normal((3, 3, cin, cout)) * np.sqrt(2.0 / (9 * cin))
        params.append((W, np.zeros(cout)))
    return params


def normal_vector(size, seed):
    """b ~ N(0, 1) of the given length in FP64 (the right-hand sides of the coupled Darcy-Stokes
    system, whose unknowns are not those of a facet problem)."""
    return np.random.default_rng(seed).standard_normal(size)
