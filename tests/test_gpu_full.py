"""GPU parity of the full-system PCG with the lazy block preconditioner (fdd_dd_precond_apply,
fdd_solve_full) against the oracle (system.lazy_precond / lazy_full_pcg with the plain V-cycle
of oracle/multigrid.py), and against the exact solution.

Both sides use the same rational tables, built by the oracle's AAA and handed to the library
with fdd_ratpc_from_table.  Tolerances:
  * one preconditioner application (FP64 V-cycles): 1e-12 relative, element by element up to
    rounding order (the V-cycles are the same operator);
  * FP32 V-cycles: 1e-5 relative (single-precision smoothing and coarse solve);
  * solves at outer rtol 1e-10: ||x - x_ref|| / ||x_ref|| <= 1e-8 against the oracle's lazy PCG
    and against the exact solution, PCG counts within one of the oracle's.
"""
import numpy as np
import pytest

import workloads
from oracle import aaa, multigrid, spectral, system

torch = pytest.importorskip("torch")
F = pytest.importorskip("paper_2211_15308_amd")

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_tables(n, K, mu, tol=1e-12):
    lo, hi = spectral.spectral_interval(2, n)
    lam = spectral.interface_eigs_1d(n)
    tp = aaa.ra_table(spectral.f_precond(K, 1.0 / mu), lo, hi, tol, extra=lam)
    th = aaa.ra_table(spectral.g_operator, lo, hi, tol, extra=lam)
    return tp, th


def setup(n, K, mu, tol=1e-12):
    P = F.setup_mesh(n, K, mu)
    P.bind_workspace()
    tp, th = oracle_tables(n, K, mu, tol)
    TP = P.ratpc_from_table(F.FDD_RA_PRECOND, tp[0], list(tp[1]), list(tp[2]))
    TH = P.ratpc_from_table(F.FDD_RA_OPERATOR, th[0], list(th[1]), list(th[2]))
    return P, TP, TH, tp, th


@pytest.mark.parametrize("n,K,mu,nu", [(8, 1.0, 1.0, 1), (16, 1e-2, 1e-3, 2), (64, 1.0, 1e-6, 2),
                                       (128, 1e-4, 1e3, 1), (256, 1.0, 1.0, 2)])
def test_dd_precond_apply_fp64_matches_oracle(n, K, mu, nu):
    print(f"[dd precond fp64] n={n} K={K} mu={mu} nu={nu}", flush=True)
    P, TP, _, tp, _ = setup(n, K, mu)
    r = workloads.rhs(2, n, 40 + n)
    z = torch.zeros(P.N, dtype=torch.float64, device="cuda")
    P.dd_precond_apply(TP, dev(r), z, F.opts_default(precision=F.FDD_FP64, mg_nu=nu))
    R = system.Riesz(2, n, K, mu)
    z_ref = system.lazy_precond(R, tp, multigrid.VCycle(n - 1, nu=nu))(r)
    err = rel(host(z), z_ref)
    print(f"[dd precond fp64] rel err {err:.2e}", flush=True)
    assert err <= 1e-12


@pytest.mark.parametrize("n,nu", [(64, 2), (256, 1), (512, 2)])
def test_dd_precond_apply_fp32_matches_oracle(n, nu):
    # FP32 V-cycles solve the first level with at most 63 x 63 points exactly (sine transforms)
    print(f"[dd precond fp32] n={n} nu={nu}", flush=True)
    K, mu = 1.0, 1e-3
    P, TP, _, tp, _ = setup(n, K, mu)
    r = workloads.rhs(2, n, 80 + n)
    z = torch.zeros(P.N, dtype=torch.float64, device="cuda")
    P.dd_precond_apply(TP, dev(r), z, F.opts_default(precision=F.FDD_MIXED, mg_nu=nu))
    R = system.Riesz(2, n, K, mu)
    z_ref = system.lazy_precond(R, tp, multigrid.VCycle(n - 1, nu=nu, exact_nf=63))(r)
    err = rel(host(z), z_ref)
    print(f"[dd precond fp32] rel err {err:.2e}", flush=True)
    assert err <= 1e-5


@pytest.mark.parametrize("n,K,mu,nu", [(32, 1.0, 1.0, 2), (64, 1e-2, 1e-3, 1), (128, 1e-4, 1e3, 2),
                                       (128, 1.0, 1e-6, 2)])
def test_solve_full_matches_oracle_lazy_pcg(n, K, mu, nu):
    print(f"[solve full] n={n} K={K} mu={mu} nu={nu}", flush=True)
    P, TP, TH, tp, th = setup(n, K, mu)
    b = workloads.rhs(2, n, 7 + n)
    x = torch.zeros(P.N, dtype=torch.float64, device="cuda")
    st = P.solve_full(TP, TH, dev(b), x, F.opts_default(precision=F.FDD_FP64, mg_nu=nu,
                                                         outer_rtol=1e-10, check_true_residual=1))
    R = system.Riesz(2, n, K, mu)
    x_ref, its_ref, _ = system.lazy_full_pcg(R, b, tp, th, nu=nu, rtol=1e-10)
    x_h = host(x)
    e_lazy = rel(x_h, x_ref)
    e_exact = rel(x_h, system.solve_dst_2d(n, K, mu, b))
    print(f"[solve full] its {st['outer_its']} (oracle {its_ref}) err vs lazy {e_lazy:.2e} "
          f"vs exact {e_exact:.2e} true res {st['true_rel_res']:.2e}", flush=True)
    assert abs(st["outer_its"] - its_ref) <= 1
    assert e_lazy <= 1e-8
    assert e_exact <= 1e-8
    assert st["true_rel_res"] <= 1e-8


@pytest.mark.parametrize("n,mu", [(256, 1e-3), (512, 1.0), (1024, 1e3), (1024, 1e-6)])
def test_solve_full_large_against_exact(n, mu):
    print(f"[solve full large] n={n} mu={mu}", flush=True)
    K = 1.0
    P, TP, TH, _, _ = setup(n, K, mu)
    # two right-hand sides on one problem: the second solve enqueues as many iterations ahead
    # of its first read-back as the first one took (those beyond its stop return at once)
    for seed in (300 + n, 301 + n):
        b = workloads.rhs(2, n, seed)
        x = torch.zeros(P.N, dtype=torch.float64, device="cuda")
        st = P.solve_full(TP, TH, dev(b), x, F.opts_default(precision=F.FDD_FP64, mg_nu=2,
                                                             outer_rtol=1e-10, outer_maxit=200))
        err = rel(host(x), system.solve_dst_2d(n, K, mu, b))
        print(f"[solve full large] seed {seed} its {st['outer_its']} err {err:.2e}", flush=True)
        assert err <= 1e-8
        assert st["outer_its"] <= 60


def test_solve_full_counts_bounded_in_h_and_gamma():
    # Fig. 4-left: with one V-cycle for the leading block the count stays bounded in h and gamma
    counts = {}
    for n in (64, 256, 1024):
        for mu in (1e-3, 1.0, 1e3):
            P, TP, TH, _, _ = setup(n, 1.0, mu)
            b = workloads.rhs(2, n, 500 + n)
            x = torch.zeros(P.N, dtype=torch.float64, device="cuda")
            st = P.solve_full(TP, TH, dev(b), x, F.opts_default(precision=F.FDD_FP64, mg_nu=2,
                                                                 outer_rtol=1e-10, outer_maxit=200))
            counts[(n, mu)] = st["outer_its"]
    print("[solve full counts]", counts, flush=True)
    for mu in (1e-3, 1.0, 1e3):
        assert counts[(1024, mu)] <= counts[(64, mu)] + 10
    assert max(counts.values()) <= 60


@pytest.mark.parametrize("n", [256, 1024])
def test_solve_full_fp32_vcycles(n):
    # FP32 V-cycles inside the FP64 PCG: the preconditioner is perturbed at single precision,
    # the recurrences and the operator stay FP64, and the solution meets the tolerance
    print(f"[solve full fp32] n={n}", flush=True)
    K, mu = 1.0, 1.0
    P, TP, TH, _, _ = setup(n, K, mu)
    b = workloads.rhs(2, n, 900 + n)
    x = torch.zeros(P.N, dtype=torch.float64, device="cuda")
    st = P.solve_full(TP, TH, dev(b), x, F.opts_default(precision=F.FDD_MIXED, mg_nu=2,
                                                         outer_rtol=1e-10, outer_maxit=200,
                                                         check_true_residual=1))
    err = rel(host(x), system.solve_dst_2d(n, K, mu, b))
    print(f"[solve full fp32] its {st['outer_its']} err {err:.2e} res {st['true_rel_res']:.2e}",
          flush=True)
    assert err <= 1e-8


def test_full_error_paths():
    P = F.setup_mesh(8, 1.0, 1.0, dim=3)
    P.bind_workspace()
    T = P.build_rational_pc(F.FDD_RA_PRECOND, 1e-8)
    v = torch.zeros(P.N, dtype=torch.float64, device="cuda")
    with pytest.raises(F.FddError) as e:
        P.dd_precond_apply(T, v, v)
    assert e.value.status == F.FDD_E_ARG
    Q, TP, TH, _, _ = setup(16, 1.0, 1.0)
    x = torch.zeros(Q.N, dtype=torch.float64, device="cuda")
    with pytest.raises(F.FddError) as e:
        Q.solve_full(TH, TP, x, x)      # tables swapped
    assert e.value.status == F.FDD_E_STATE
