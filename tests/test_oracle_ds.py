"""Pins of the Darcy-Stokes oracle (oracle/darcy_stokes.py; Sec. 4 eq. (darcy_stokes), eq.
(darcy_stokes_precond); Appendix), independent of its own assembly where possible:

* divergence, interface and Beavers-Joseph-Saffman blocks against closed-form integrals of fields
  the P2 / P1 spaces hold exactly;
* the Taylor-Hood inf-sup constant bounded below in h (a textbook property of P2-P1);
* second-order nodal convergence of all three fields to a manufactured solution that satisfies
  every interface and boundary condition (a dropped term or a wrong sign gives O(1) errors);
* FGMRES: its least-squares residual equals the true residual of its iterate, one step with the
  exact inverse as preconditioner, k steps for k distinct eigenvalues, agreement with a direct
  solve;
* the robustness the Appendix reports: iteration counts bounded in h, mu and K, and practically
  the same with the Darcy block by inexact PCG as with exact blocks.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import aaa, darcy_stokes as ds, fem, spectral


def velocity_interp(n, fx, fy):
    out = np.zeros(ds.sizes(n)[0])
    for B in range(2 * n + 1):
        for A in range(1, 2 * n):
            x, y = A / (2 * n), 1 + B / (2 * n)
            out[ds.vel_index(n, 0, A, B)] = fx(x, y)
            out[ds.vel_index(n, 1, A, B)] = fy(x, y)
    return out


def pressure_interp(n, f):
    return np.array([f(i / n, 1 + j / n) for j in range(n + 1) for i in range(n + 1)])


def test_sizes_and_symmetry():
    for n in (2, 4, 8):
        P = ds.DarcyStokes(n, 1.0, 1.0, 1.0)
        Nu, Np, ND, N = ds.sizes(n)
        assert (Nu, Np, ND) == (2 * (2 * n - 1) * (2 * n + 1), (n + 1) ** 2, n * (n - 1))
        assert P.A.shape == (N, N)
        assert abs(P.A - P.A.T).max() <= 1e-15 * abs(P.A).max()


@pytest.mark.parametrize("n", [2, 4, 8])
def test_divergence_block_exact(n):
    # u = (x(1 - x), 0): div u = 1 - 2x (P1), so B I(u) = -M_p I(1 - 2x); u = (0, x(1 - x)): div 0
    P = ds.DarcyStokes(n, 1.0, 1.0)
    u1 = velocity_interp(n, lambda x, y: x * (1 - x), lambda x, y: 0.0)
    u2 = velocity_interp(n, lambda x, y: 0.0, lambda x, y: x * (1 - x))
    d = pressure_interp(n, lambda x, y: 1 - 2 * x)
    assert np.abs(P.B @ u1 + P.M_p @ d).max() <= 1e-14
    assert np.abs(P.B @ u2).max() <= 1e-14
    # and the divergence of a linear-in-y field: u = (0, y x(1 - x)) is cubic, not in P2: the
    # identity must fail there (the check is sensitive)
    u3 = velocity_interp(n, lambda x, y: 0.0, lambda x, y: y * y * x * (1 - x))
    d3 = pressure_interp(n, lambda x, y: 2 * y * x * (1 - x))
    assert np.abs(P.B @ u3 + P.M_p @ d3).max() > 1e-6


@pytest.mark.parametrize("n,K,mu,alpha", [(4, 1.0, 1.0, 3.0), (8, 1e-2, 1e-3, 1.5)])
def test_interface_terms_exact(n, K, mu, alpha):
    # BJS: the difference of the velocity blocks with and without alpha is
    # alpha mu K^{-1/2} int_Gamma u_x v_x; for u_x = v_x = x(1 - x) the integral is 1/30
    A1 = ds.DarcyStokes(n, K, mu, alpha).A_u
    A0 = ds.DarcyStokes(n, K, mu, 0.0).A_u
    u = velocity_interp(n, lambda x, y: x * (1 - x), lambda x, y: 0.0)
    assert abs(u @ (A1 - A0) @ u - alpha * mu / np.sqrt(K) / 30.0) <= 1e-14
    # coupling: v_y = x(1 - x) against the Darcy hat of interface node i: -int hat_i x(1 - x)
    P = ds.DarcyStokes(n, K, mu, alpha)
    v = velocity_interp(n, lambda x, y: 0.0, lambda x, y: x * (1 - x))
    g, w = np.polynomial.legendre.leggauss(8)
    h = 1.0 / n
    for i in range(1, n):
        exact = 0.0
        for a, b, up in ((i - 1) * h, i * h, True), (i * h, (i + 1) * h, False):
            x = (a + b) / 2 + (b - a) / 2 * g
            hat = (x - a) / h if up else (b - x) / h
            exact += (b - a) / 2 * np.sum(w * hat * x * (1 - x))
        col = P.C[:, P.darcy_gamma_index(i)].toarray().ravel()
        assert abs(v @ col + exact) <= 1e-15
    # only the normal velocity on Gamma couples
    assert P.C[:P.NV].nnz == 0


def test_inf_sup_bounded_below():
    # Taylor-Hood: min over p of (B A_u^{-1} B^T p, p) / (M_p p, p) bounded below uniformly in h
    vals = []
    for n in (4, 8, 16):
        P = ds.DarcyStokes(n, 1.0, 1.0, 0.0)
        Ainv_Bt = spla.splu(P.A_u.tocsc()).solve(P.B.T.toarray())
        S = P.B @ Ainv_Bt
        lam = sla.eigh(S, P.M_p.toarray(), eigvals_only=True)
        vals.append(lam[0])
    assert min(vals) > 0.05
    assert max(vals) / min(vals) < 1.5


@pytest.mark.parametrize("K,mu,alpha", [(1.0, 1.0, 3.0), (1e-2, 1e-2, 0.0)])
def test_manufactured_second_order(K, mu, alpha):
    errs = []
    for n in (8, 16, 32):
        P = ds.DarcyStokes(n, K, mu, alpha)
        ex, data = P.manufactured()
        x = P.solve_splu(P.load(data))
        e = x - P.interpolate(ex)
        Nu, Np = P.Nu, P.Np
        errs.append([np.abs(e[:Nu]).max(), np.abs(e[Nu:Nu + Np]).max(), np.abs(e[Nu + Np:]).max()])
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    assert rates.min() >= 1.8, rates


def test_manufactured_sensitive_to_coupling_sign():
    # the same solve with the interface coupling's sign flipped misses the manufactured solution
    P = ds.DarcyStokes(16, 1.0, 1.0, 3.0)
    ex, data = P.manufactured()
    F = P.load(data)
    A_bad = sp.bmat([[P.A_u, P.B.T, -P.C], [P.B, None, None], [-P.C.T, None, -P.A_D]], format="csc")
    e_good = np.abs(P.solve_splu(F) - P.interpolate(ex)).max()
    e_bad = np.abs(spla.spsolve(A_bad, F) - P.interpolate(ex)).max()
    assert e_bad > 20 * e_good   # O(1) against the O(h^2) of the right sign


def test_fgmres_invariants():
    rng = np.random.default_rng(3)
    P = ds.DarcyStokes(8, 1.0, 1.0, 3.0)
    b = rng.standard_normal(P.N)
    B = P.precond_exact()
    A = lambda v: P.A @ v  # noqa: E731
    # least-squares residual = true residual of the iterate after k steps (no restart)
    for k in (1, 5, 20):
        x, its, hist = ds.fgmres(A, b, B, rtol=1e-14, maxit=k)
        assert its == k
        assert abs(hist[-1] - np.linalg.norm(b - P.A @ x)) <= 1e-9 * np.linalg.norm(b)
        assert all(hist[i + 1] <= hist[i] * (1 + 1e-12) for i in range(len(hist) - 1))
    # the exact inverse as preconditioner: one step
    lu = spla.splu(P.A.tocsc())
    x, its, _ = ds.fgmres(A, b, lu.solve, rtol=1e-12, maxit=10)
    assert its == 1 and np.linalg.norm(x - lu.solve(b)) <= 1e-12 * np.linalg.norm(x)
    # three distinct eigenvalues, no preconditioning: three steps
    d = np.repeat([1.0, 2.0, 5.0], 20)
    x, its, _ = ds.fgmres(lambda v: d * v, rng.standard_normal(60), lambda v: v, rtol=1e-12, maxit=10)
    assert its == 3
    # the coupled system to the direct solution
    x, its, _ = ds.fgmres(A, b, B, rtol=1e-12, maxit=300)
    assert np.linalg.norm(x - P.solve_splu(b)) <= 1e-9 * np.linalg.norm(x)


def tables(n, K, mu, tol=1e-12):
    lo, hi = spectral.spectral_interval(2, n)
    lam = spectral.interface_eigs_1d(n)
    tp = aaa.ra_table(spectral.f_precond(K, 1.0 / mu), lo, hi, tol, extra=lam)
    th = aaa.ra_table(spectral.g_operator, lo, hi, tol, extra=lam)
    return tp, th


def test_counts_bounded_in_h_mu_K():
    # Appendix (Fig. 6): FGMRES counts with the block-diagonal preconditioner bounded in mu, K, h
    rng = np.random.default_rng(5)
    rows = {}
    for K in (1e-2, 1.0):
        for mu in (1e-4, 1.0):
            c = []
            for n in (8, 16):
                P = ds.DarcyStokes(n, K, mu, 3.0)
                _, its, _ = ds.fgmres(lambda v: P.A @ v, rng.standard_normal(P.N), P.precond_exact(),
                                      rtol=1e-10, maxit=300)
                c.append(its)
            rows[(K, mu)] = c
    for c in rows.values():
        assert max(c) <= 90 and max(c) - min(c) <= 6, rows


def test_inexact_darcy_block_keeps_counts():
    # Appendix: the Darcy block by PCG (rtol 1e-5) with the lazy DD preconditioner and RA gives
    # practically the counts of exact blocks
    n, K, mu = 8, 1e-2, 1e-4
    P = ds.DarcyStokes(n, K, mu, 3.0)
    b = np.random.default_rng(7).standard_normal(P.N)
    tp, th = tables(n, K, mu)
    Bl, inner = P.precond_lazy(tp, th, darcy_rtol=1e-5)
    x1, its1, _ = ds.fgmres(lambda v: P.A @ v, b, Bl, rtol=1e-10, maxit=300)
    _, its0, _ = ds.fgmres(lambda v: P.A @ v, b, P.precond_exact(), rtol=1e-10, maxit=300)
    assert abs(its1 - its0) <= 2
    assert max(inner) <= 10
    assert np.linalg.norm(x1 - P.solve_splu(b)) <= 1e-8 * np.linalg.norm(x1)


def test_darcy_block_is_the_facet_problem():
    # the preconditioner's third block is the Riesz map of eq. (riesz) on the Darcy unknowns
    P = ds.DarcyStokes(8, 2.0, 0.5)
    R = P.riesz()
    r = np.random.default_rng(1).standard_normal(P.ND)
    y = R.solve_splu(r)
    Afacet = (R.K * R.P.A).toarray()
    Afacet[R.P.NI:, R.P.NI:] += R.gamma * R.H
    assert np.linalg.norm(Afacet @ y - r) <= 1e-12 * np.linalg.norm(r)
    assert abs(P.A_D - 2.0 * fem.Problem(2, 8).A).max() == 0.0
