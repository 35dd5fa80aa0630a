"""Pins of the oracle's fractional powers (eq. (gevp)) and RA evaluation (eq. (RA))."""
import numpy as np
import pytest

from oracle import aaa, fem, ra, spectral


@pytest.fixture(scope="module")
def iface():
    P = fem.Problem(2, 16)
    return P.A_G, P.M_G


def test_powers_zero_and_one(iface):
    L, M = iface
    assert np.allclose(spectral.frac_power(L, M, 1.0), L, atol=1e-10 * np.abs(L).max())
    assert np.allclose(spectral.frac_power(L, M, 0.0), M, atol=1e-13)


def test_half_powers_compose_through_mass_inverse(iface):
    L, M = iface
    Lh = spectral.frac_power(L, M, 0.5)
    assert np.allclose(Lh @ np.linalg.solve(M, Lh), L, atol=1e-9 * np.abs(L).max())
    Lm = spectral.frac_power(L, M, -0.5)
    # L^{1/2} M^{-1} L^{-1/2} = M
    assert np.allclose(Lh @ np.linalg.solve(M, Lm), M, atol=1e-12)
    assert np.allclose(Lh, Lh.T, atol=1e-12) and np.linalg.eigvalsh(Lm).min() > 0


def test_fractional_norm_of_sine_converges():
    # f_h . L_h^s f_h -> ||sin(k pi x)||_s^2 = (k pi)^{2 s} / 2 for the Dirichlet Laplacian
    k = 3
    for s in (0.5, -0.5):
        errs = []
        for n in (32, 64, 128):
            P = fem.Problem(2, n)
            x = np.arange(1, n) / n
            f = np.sin(k * np.pi * x)
            val = f @ spectral.frac_power(P.A_G, P.M_G, s) @ f
            exact = (k * np.pi) ** (2 * s) / 2
            errs.append(abs(val - exact) / exact)
        assert errs[-1] < 2e-3
        assert errs[0] / errs[-1] > 10  # second-order convergence


def test_precond_inverse(iface):
    L, M = iface
    for K, g in ((1.0, 1.0), (1e-4, 1e6), (1.0, 1e-3)):
        S = spectral.schur_precond(L, M, K, g)
        Si = spectral.schur_precond_inverse(L, M, K, g)
        assert np.allclose(S @ Si, np.eye(len(L)), atol=1e-9)


def test_ra_scalar_equals_dense_operator(iface):
    L, M = iface
    lam, U = spectral.gevp(L, M)
    c0, c, p = 0.3, np.array([1.0, -0.2, 2.5]), np.array([0.0, 3.0, 1e4])
    D = ra.dense_operator(L, M, c0, c, p)
    V = (U * ra.eval_scalar(c0, c, p, lam)) @ U.T
    assert np.allclose(D, V, atol=1e-12 * np.abs(V).max())


def test_oracle_aaa_pole_count_and_accuracy():
    n = 64
    lam = spectral.interface_eigs_1d(n)
    lo, hi = lam[0], lam[-1]
    f = spectral.f_precond(1.0, 1.0)
    c0, c, p = aaa.ra_table(f, lo, hi, tol=1e-12, extra=lam)
    assert ra.max_rel_error(f, c0, c, p, lam) < 1e-11
    assert np.all(p >= 0)
    assert 10 <= len(p) <= 26
    # lambda^{-1/2} is a Stieltjes function: every residue of its RA is positive
    d0, d, q = aaa.ra_table(spectral.g_operator, lo, hi, tol=1e-12, extra=lam)
    assert ra.max_rel_error(spectral.g_operator, d0, d, q, lam) < 1e-11
    assert np.all(d > 0) and np.all(q >= 0)


def test_paper_pole_count_statement():
    # Sec. 3: epsilon_RA = 1e-14 yields roughly m = 20 poles (3D, L = -Delta + I on the
    # boundary of the cube, so lambda >= 1; the finest mesh has n = 32).
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_statements.json")))
    m_paper = gold["ra_poles_at_eps_1e-14"]["value"]
    f = spectral.f_precond(1.0, 1.0)
    # relative-error AAA in FP64 stalls at its rounding floor just above 1e-14, so the
    # tolerance is taken at 1e-13 relative (the paper does not state its error norm)
    c0, c, p = aaa.ra_table(f, 1.0, 36.0 * 32 * 32, tol=1e-13)
    z = np.geomspace(1.0, 36.0 * 32 * 32, 5000)
    assert ra.max_rel_error(f, c0, c, p, z) < 1e-12
    assert abs(len(p) - m_paper) <= 6
    # the interface size statement: 6 n^2 + 2 nodes on the boundary of the cube at n = 32
    assert 6 * 32 * 32 + 2 < gold["interface_unknowns_3d_upper"]["value"]


@pytest.mark.parametrize("dim,n", [(2, 16), (2, 48), (3, 6)])
def test_operator_table_realizes_inverse_square_root(dim, n):
    # eq. (RA) applied to g(lambda) = lambda^{-1/2}: M (d0 M^{-1} + sum_k d_k (L + q_k M)^{-1}) M
    # must equal the exact L^{-1/2} = (M U) Lambda^{-1/2} (M U)^T of eq. (gevp) to the table's
    # error on the spectrum (relative, since both are SPD and share the eigenvectors U)
    P = fem.Problem(dim, n)
    L, M = P.A_G, P.M_G
    lam, _ = spectral.gevp(L, M)
    d0, d, q = aaa.ra_table(spectral.g_operator, lam[0], lam[-1], tol=1e-12, extra=lam)
    err = ra.max_rel_error(spectral.g_operator, d0, d, q, lam)
    H_ra = ra.dense_operator_H(L, M, d0, d, q)
    H = spectral.frac_power(L, M, -0.5)
    assert np.linalg.norm(H_ra - H, 2) <= 2 * err * np.linalg.norm(H, 2)
    # a dropped term is visible: without the d0 M part the operator is off by far more
    H_bad = ra.dense_operator_H(L, M, 0.0, d, q)
    assert np.linalg.norm(H_bad - H, 2) > 1e3 * err * np.linalg.norm(H, 2)


def test_tridiagonal_ra_apply_equals_dense_operator():
    P = fem.Problem(2, 40)
    L, M = P.A_G, P.M_G
    lam = spectral.interface_eigs_1d(40)
    c0, c, p = aaa.ra_table(spectral.f_precond(1e-2, 1e3), lam[0], lam[-1], tol=1e-10, extra=lam)
    r = np.random.default_rng(2).standard_normal(39)
    z = ra.apply_tridiagonal(L, M, c0, c, p, r)
    zd = ra.dense_operator(L, M, c0, c, p) @ r
    assert np.linalg.norm(z - zd) <= 1e-12 * np.linalg.norm(zd)
