"""Pins of the oracle's model problem (oracle/model.py; Sec. 3, eq. (model_problem), 2D)."""
import numpy as np
import pytest

from oracle import aaa, model, spectral


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n", [4, 8, 16])
def test_loop_spectrum_closed_form(n):
    A_G, M_G = model.loop_matrices(n)
    lam = spectral.gevp(A_G + M_G, M_G)[0]
    assert np.max(np.abs(lam - model.loop_eigs(n))) < 1e-10 * lam.max()
    # closed curve of length 4: constants are in the kernel of A_G, M_G integrates to the length
    one = np.ones(4 * n)
    assert np.max(np.abs(A_G @ one)) < 1e-12
    assert abs(one @ M_G @ one - 4.0) < 1e-12


def test_fractional_power_identities():
    n = 8
    P = model.ModelProblem(n, 1.0, 1.0, 0.0)
    assert np.max(np.abs(P.Lt - P.M_G)) < 1e-12            # L^0 = M
    L1 = spectral.frac_power(P.L, P.M_G, 1.0, P.eig)
    assert np.max(np.abs(L1 - P.L)) < 1e-10                 # L^1 = L
    Lm1 = spectral.frac_power(P.L, P.M_G, -1.0, P.eig)
    assert np.max(np.abs(Lm1 - P.M_G @ np.linalg.solve(P.L, P.M_G))) < 1e-12   # L^-1 = M L^-1 M
    Q = model.ModelProblem(n, 1.0, 1.0, 0.5)
    R = model.ModelProblem(n, 1.0, 1.0, -0.5)
    # L^{1/2} M^{-1} L^{-1/2} = M ... composition through the mass matrix
    assert np.max(np.abs(Q.Lt @ np.linalg.solve(P.M_G, R.Lt) - P.M_G)) < 1e-10


def test_dof_order_and_block_structure():
    n = 6
    P = model.ModelProblem(n, 1.0, 2.0, -0.5)
    assert P.N == (n + 1) ** 2 and P.NI == (n - 1) ** 2 and P.NG == 4 * n
    order = model.dof_order(n)
    assert len(set(order.tolist())) == P.N
    # the interior block is the 7-point stencil of stiffness (4, -1 x 4) plus mass
    # (h^2/2 centre, h^2/12 on the six neighbours of the diagonal-split mesh)
    h = 1.0 / n
    B_II = P.blocks()[0].toarray()
    c = (n - 1) * 2 + 2                                        # interior node (3, 3)
    assert abs(B_II[c, c] - (4 + h * h / 2)) < 1e-12
    for d in (1, -1, n - 1, -(n - 1)):
        assert abs(B_II[c, c + d] - (-1 + h * h / 12)) < 1e-12
    for d in (n, -n):                                          # (i+1, j+1) and (i-1, j-1)
        assert abs(B_II[c, c + d] - h * h / 12) < 1e-12
    assert abs(B_II[c, c + (n - 2)]) < 1e-14                   # (i-1, j+1): no edge


def test_dense_and_sparse_solves_agree():
    for t in (-0.5, 0.5, 0.0):
        P = model.ModelProblem(8, 1e-2, 3.0, t)
        b = np.random.default_rng(1).standard_normal(P.N)
        x = P.solve_dense(b)
        assert rel(P.solve_splu(b), x) < 1e-12
        assert rel(P.apply(x), b) < 1e-12


def test_manufactured_neumann_solution_second_order():
    # gamma = 0: K(-Delta + I) u = f with natural (Neumann) conditions; u = cos(pi x) cos(pi y)
    # has zero normal derivative and -Delta u + u = (2 pi^2 + 1) u.  Load b = M f_h.
    errs = []
    for n in (8, 16, 32):
        P = model.ModelProblem(n, 1.0, 0.0, -0.5)
        order = model.dof_order(n)
        ij = np.array([(g % (n + 1), g // (n + 1)) for g in order]) / n
        u = np.cos(np.pi * ij[:, 0]) * np.cos(np.pi * ij[:, 1])
        x = P.solve_splu(P.M @ ((2 * np.pi ** 2 + 1) * u))
        errs.append(np.max(np.abs(x - u)))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def test_schur_complement_identity_and_equivalence():
    counts = []
    for n in (8, 16, 32):
        P = model.ModelProblem(n, 1.0, 1.0, -0.5)
        Ad = P.matrix_sparse().toarray()
        NI = P.NI
        S_ref = Ad[NI:, NI:] - Ad[NI:, :NI] @ np.linalg.solve(Ad[:NI, :NI], Ad[:NI, NI:])
        S = P.schur_dense()
        assert np.max(np.abs(S - S_ref)) < 1e-10 * np.max(np.abs(S))
        assert np.max(np.abs(S - S.T)) < 1e-10 * np.max(np.abs(S))
        ev = np.linalg.eigvals(P.exact_precond() @ S).real
        counts.append(ev.max() / ev.min())
    # S_Gamma = K L^{1/2} + gamma L^t is spectrally equivalent to S: a condition number of about
    # 4 that grows by under 5% per halving of h (3.86, 4.03, 4.21 at n = 8, 16, 32)
    assert max(counts) < 5.0
    assert all(b < 1.1 * a for a, b in zip(counts, counts[1:]))


@pytest.mark.parametrize("t", [-0.5, 0.5, -0.9, 0.9])
def test_schur_pcg_with_exact_preconditioner(t):
    P = model.ModelProblem(16, 1.0, 10.0, t)
    b = np.random.default_rng(2).standard_normal(P.N)
    x, its = P.schur_pcg(b, rtol=1e-10)
    assert rel(x, P.solve_splu(b)) < 1e-9
    assert its <= 30


@pytest.mark.parametrize("t", [-0.5, 0.5])
def test_ra_operator_within_table_error(t):
    n = 16
    P = model.ModelProblem(n, 1.0, 1.0, t)
    lam = model.loop_eigs(n)
    lo, hi = lam[0], lam[-1]
    g = (lambda x: x ** t) if t < 0 else (lambda x: x ** (t - 1))
    tab = aaa.ra_table(g, lo, hi, 1e-12, extra=lam)
    Lt_ra = model.ra_operator(P.L, P.M_G, t, tab)
    assert rel(Lt_ra, P.Lt) < 1e-10
    # the preconditioner table: eq. (RA) as a matrix is U f_RA(Lambda) U^T, so its distance to
    # the exact S_Gamma^{-1} is the table's scalar error on the spectrum
    tp = aaa.ra_table(P.f_precond(), lo, hi, 1e-10, extra=lam)
    from oracle import ra
    D = ra.dense_operator(P.L, P.M_G, *tp)
    f_ra = lambda x: ra.eval_scalar(*tp, x)
    assert rel(D, spectral.spectral_function(P.L, P.M_G, f_ra, P.eig)) < 1e-12
    err = ra.max_rel_error(P.f_precond(), *tp, lam)
    assert err < 1e-7
    assert rel(D, P.exact_precond()) < 2 * err
