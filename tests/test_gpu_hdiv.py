"""GPU parity of the H(div) problem (Sec. 3 remark on H(div)-elliptic problems, eq. (graddiv);
BDM1, Gamma = the whole boundary) against the oracle (oracle/hdiv.py).

Tolerances: products 1e-12 relative (FP64 sums in another order); the preconditioner against the
oracle's realization of the same table 1e-12; interior solves at inner rtol 1e-12 within 1e-9 of
the oracle's sparse LU; solves at outer rtol 1e-10 within 1e-8 of the oracle's sparse LU of the
whole system, outer counts within one of the oracle's Schur PCG with the same table.
"""
import numpy as np
import pytest

from oracle import aaa, hdiv

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


def setup(n, K, gamma, tol=1e-12):
    P = F.setup_hdiv(n, K, gamma)
    P.bind_workspace()
    M = hdiv.HdivProblem(n, K, gamma)
    lam = hdiv.loop_eigs(n)
    tab = aaa.ra_table(M.g_table_function(), lam[0], lam[-1], tol, extra=lam)
    TP = P.ratpc_from_table(F.FDD_RA_PRECOND, tab[0], list(tab[1]), list(tab[2]))
    return P, TP, M, tab


@pytest.mark.parametrize("n,K,gamma", [(4, 1.0, 1.0), (8, 1.3, 2.0), (32, 1e-2, 1e3)])
def test_operator_and_preconditioner_match_oracle(n, K, gamma):
    print(f"[hdiv products] n={n} K={K} gamma={gamma}", flush=True)
    P, TP, M, tab = setup(n, K, gamma)
    assert (P.N, P.NI, P.NG) == hdiv.sizes(n)
    assert abs(P.lam_lo - 1.0) < 1e-12 and abs(P.lam_hi / hdiv.loop_eigs(n)[-1] - 1) < 1e-12
    x = np.random.default_rng(n).standard_normal(M.N)
    y = torch.zeros(M.N, dtype=torch.float64, device="cuda")
    P.apply_operator(None, dev(x), y)
    e1 = rel(host(y), M.A @ x)
    r = np.random.default_rng(n + 1).standard_normal(M.NG)
    z = torch.zeros(M.NG, dtype=torch.float64, device="cuda")
    P.precond_apply(TP, dev(r), z)
    D = hdiv.ra_precond(M.L, M.M_Q, tab)
    e2 = rel(host(z), D @ r)
    print(f"[hdiv products] operator {e1:.2e} precond {e2:.2e}", flush=True)
    assert e1 <= 1e-12 and e2 <= 1e-12
    # the library's own table: within its error of the exact S_Gamma^{-1}
    TL = P.build_rational_pc(F.FDD_RA_PRECOND, 1e-12)
    z2 = torch.zeros(M.NG, dtype=torch.float64, device="cuda")
    P.precond_apply(TL, dev(r), z2)
    err = TL.query()["max_rel_err"]
    assert rel(host(z2), M.exact_precond() @ r) <= 2 * err + 1e-11


@pytest.mark.parametrize("n,K,gamma", [(256, 1.0, 1e-3), (1024, 1.0, 1.0), (1024, 1e-2, 1e3)])
def test_preconditioner_large_matches_fourier_oracle(n, K, gamma):
    # up to the largest loop (4n = 4096 segments: the cyclic reduction's LDS limit) against the
    # oracle's Fourier-mode application of the same table (pinned to the dense one)
    print(f"[hdiv precond large] n={n} K={K} gamma={gamma}", flush=True)
    P = F.setup_hdiv(n, K, gamma)
    P.bind_workspace()
    T = P.build_rational_pc(F.FDD_RA_PRECOND, 1e-12)
    q = T.query()
    tab = (q["c0"], np.array(q["c"]), np.array(q["p"]))
    r = np.random.default_rng(n + 5).standard_normal(P.NG)
    z = torch.zeros(P.NG, dtype=torch.float64, device="cuda")
    P.precond_apply(T, dev(r), z)
    err = rel(host(z), hdiv.ra_precond_apply_fft(n, tab, r))
    print(f"[hdiv precond large] {q['m']} poles, rel err {err:.2e}", flush=True)
    assert err <= 1e-11


@pytest.mark.parametrize("n,nu", [(4, 1), (8, 1), (32, 1), (32, 2), (128, 1)])
def test_interior_solve_matches_oracle(n, nu):
    print(f"[hdiv interior] n={n} nu={nu}", flush=True)
    P = F.setup_hdiv(n, 1.0, 1.0)
    P.bind_workspace()
    M = hdiv.HdivProblem(n, 1.0, 1.0)
    f = np.random.default_rng(7 + n).standard_normal(M.N0)
    u = torch.zeros(M.N0, dtype=torch.float64, device="cuda")
    its = P.interior_solve(dev(f), u, F.opts_default(inner_rtol=1e-12, mg_nu=nu))
    err = rel(host(u), M.interior_lu().solve(f))
    print(f"[hdiv interior] its {its} rel err {err:.2e}", flush=True)
    assert err <= 1e-9
    assert its <= (18 if nu == 1 else 12)


def test_interior_iterations_bounded_in_h():
    counts = []
    for n in (64, 256, 1024):
        P = F.setup_hdiv(n, 1.0, 1.0)
        P.bind_workspace()
        f = np.random.default_rng(n).standard_normal(P.NI)
        u = torch.zeros(P.NI, dtype=torch.float64, device="cuda")
        counts.append(P.interior_solve(dev(f), u, F.opts_default(inner_rtol=1e-10)))
    print(f"[hdiv interior counts] {counts}", flush=True)
    assert max(counts) - min(counts) <= 3


@pytest.mark.parametrize("n,K,gamma", [(4, 1.0, 1.0), (16, 1e-2, 10.0)])
def test_schur_apply_matches_oracle(n, K, gamma):
    P, TP, M, tab = setup(n, K, gamma)
    S = M.schur_dense()
    p = np.random.default_rng(3).standard_normal(M.NG)
    y = torch.zeros(M.NG, dtype=torch.float64, device="cuda")
    P.schur_apply(None, dev(p), y, F.opts_default(inner_rtol=1e-13))
    err = rel(host(y), S @ p)
    print(f"[hdiv schur] n={n} rel err {err:.2e}", flush=True)
    assert err <= 1e-9


@pytest.mark.parametrize("n,K,gamma", [(8, 1.0, 1.0), (16, 1.0, 1e-3), (16, 1e-2, 1e3), (32, 1.0, 10.0),
                                       (64, 1e-2, 1.0), (16, 1.0, 0.0)])
def test_solve_matches_oracle(n, K, gamma):
    print(f"[hdiv solve] n={n} K={K} gamma={gamma}", flush=True)
    P, TP, M, tab = setup(n, K, gamma)
    b = np.random.default_rng(100 + n).standard_normal(M.N)
    x = torch.zeros(M.N, dtype=torch.float64, device="cuda")
    st = P.solve(TP, None, dev(b), x, F.opts_default(outer_rtol=1e-10, inner_rtol=1e-12,
                                                     check_true_residual=1))
    x_ref = M.solve_splu(b)
    err = rel(host(x), x_ref)
    D = hdiv.ra_precond(M.L, M.M_Q, tab)
    _, its_ref = M.schur_pcg(b, precond=lambda r: D @ r, rtol=1e-10)
    res_ref = rel(M.A @ host(x), b)
    print(f"[hdiv solve] outer {st['outer_its']} (oracle {its_ref}) inner {st['inner_its_total']} "
          f"err {err:.2e} res {st['true_rel_res']:.2e} (oracle's residual of x {res_ref:.2e})", flush=True)
    assert err <= 1e-8
    assert abs(st["outer_its"] - its_ref) <= 1
    # the reported true residual is the oracle's ||b - A x|| / ||b|| of the returned x, up to the
    # rounding of forming b - A x in another order (at most ~(row length) eps |A| |x| per entry)
    xh = host(x)
    rounding = 16 * np.finfo(float).eps * np.linalg.norm(abs(M.A) @ abs(xh)) / np.linalg.norm(b)
    assert abs(st["true_rel_res"] - res_ref) <= 1e-3 * res_ref + rounding


@pytest.mark.parametrize("gamma", [1e-3, 1.0, 1e3])
def test_outer_counts_bounded_in_h_and_gamma(gamma):
    # the robustness of Fig. 4 (right): outer PCG counts bounded in the mesh size and gamma
    counts = []
    for n in (32, 128, 512):
        P = F.setup_hdiv(n, 1.0, gamma)
        P.bind_workspace()
        TP = P.build_rational_pc(F.FDD_RA_PRECOND, 1e-12)
        b = np.random.default_rng(n).standard_normal(P.N)
        x = torch.zeros(P.N, dtype=torch.float64, device="cuda")
        st = P.solve(TP, None, dev(b), x, F.opts_default(outer_rtol=1e-10, inner_rtol=1e-12,
                                                         check_true_residual=1))
        print(f"[hdiv robust] n={n} gamma={gamma} outer {st['outer_its']} inner {st['inner_its_total']} "
              f"res {st['true_rel_res']:.2e}", flush=True)
        assert st["true_rel_res"] <= 1e-8
        counts.append(st["outer_its"])
    assert max(counts) <= 30 and max(counts) - min(counts) <= 3


def test_solve_n256_against_golden():
    # n = 256 (394,240 dofs) against the oracle's sparse-LU solution (refined to the rounding floor
    # of its residual) written by tests/golden/make_hdiv_n256.py (4096 seeded entries and the norm)
    import json
    import os

    import workloads
    G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "solve_hdiv_n256.json")))
    n, K, gamma = G["n"], G["K"], G["gamma"]
    print(f"[hdiv n256] n={n} K={K} gamma={gamma} against the stored oracle solution", flush=True)
    P = F.setup_hdiv(n, K, gamma)
    P.bind_workspace()
    assert P.N == G["N"]
    TP = P.build_rational_pc(F.FDD_RA_PRECOND, 1e-12)
    b = workloads.normal_vector(P.N, 2560)
    x = torch.zeros(P.N, dtype=torch.float64, device="cuda")
    st = P.solve(TP, None, dev(b), x, F.opts_default(outer_rtol=1e-10, inner_rtol=1e-12,
                                                     check_true_residual=1))
    xh = host(x)
    idx = np.array(G["indices"])
    ref = np.array(G["values"])
    err = float(np.linalg.norm(xh[idx] - ref) / np.linalg.norm(ref))
    nerr = abs(np.linalg.norm(xh) - G["norm_x"]) / G["norm_x"]
    print(f"[hdiv n256] outer {st['outer_its']} sampled rel err {err:.2e} norm rel err {nerr:.2e} "
          f"res {st['true_rel_res']:.2e}", flush=True)
    assert err <= 1e-8 and nerr <= 1e-8


def test_hdiv_error_paths():
    for args in ((6, 1.0, 1.0), (2, 1.0, 1.0), (2048, 1.0, 1.0), (8, 0.0, 1.0), (8, 1.0, -1.0)):
        with pytest.raises(F.FddError) as e:
            F.setup_hdiv(*args)
        assert e.value.status == F.FDD_E_ARG
    P, TP, M, tab = setup(8, 1.0, 1.0)
    with pytest.raises(F.FddError) as e:
        P.build_rational_pc(F.FDD_RA_OPERATOR, 1e-10)
    assert e.value.status == F.FDD_E_ARG
    x = torch.zeros(P.N, dtype=torch.float64, device="cuda")
    with pytest.raises(F.FddError) as e:
        P.apply_operator(TP, x, x)                      # no operator table on this problem
    assert e.value.status == F.FDD_E_ARG
    r = torch.zeros(P.NG, dtype=torch.float64, device="cuda")
    with pytest.raises(F.FddError) as e:
        P.precond_apply_static(TP, r, r)
    assert e.value.status == F.FDD_E_ARG
    with pytest.raises(F.FddError) as e:
        F.Batch([P], [TP], [TP])                        # batches take facet problems only
    assert e.value.status in (F.FDD_E_ARG, F.FDD_E_STATE)
    Q = F.setup_mesh(16, 1.0, 1.0)
    Q.bind_workspace()
    TQ = Q.build_rational_pc(F.FDD_RA_PRECOND, 1e-8)
    with pytest.raises(F.FddError) as e:
        P.precond_apply(TQ, r, r)                       # a facet problem's table
    assert e.value.status == F.FDD_E_STATE
