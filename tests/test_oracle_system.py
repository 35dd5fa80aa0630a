"""Pins of the oracle's full solve, Schur complement and reference PCG drivers."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads
from oracle import fem, spectral, system


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n,K,mu", [(8, 1.0, 1.0), (12, 1e-2, 1e-3), (16, 1e-4, 1e3), (10, 1.0, 1e-6)])
def test_three_solvers_agree_2d(n, K, mu):
    R = system.Riesz(2, n, K, mu)
    b = workloads.rhs(2, n, n)
    x_dense = R.solve_dense(b)
    assert rel(R.solve_splu(b), x_dense) < 1e-12
    assert rel(system.solve_dst_2d(n, K, mu, b), x_dense) < 1e-12
    assert rel(R.apply(x_dense), b) < 1e-12


def test_dense_and_splu_agree_3d():
    R = system.Riesz(3, 4, 1.0, 1e-2)
    b = workloads.rhs(3, 4, 7)
    x = R.solve_dense(b)
    assert rel(R.solve_splu(b), x) < 1e-12
    S = R.schur_dense()
    assert np.allclose(S, S.T, atol=1e-12) and np.linalg.eigvalsh(S).min() > 0


def test_manufactured_mixed_poisson_converges():
    # gamma -> 0 leaves -K Delta x = f with x = 0 on three sides and a natural condition on
    # Gamma.  u = sin(pi x) sin(pi y / 2) satisfies du/dy = 0 at y = 1 and
    # -Delta u = (5 pi^2 / 4) u.  The P1 solution converges at second order at the nodes.
    errs = []
    for n in (8, 16, 32):
        R = system.Riesz(2, n, 1.0, 1e30)
        nodes, tris = fem.mesh_2d(n)
        _, M = fem.assemble(nodes, tris)
        fd = fem.free_dofs(2, n)
        u = np.sin(np.pi * nodes[:, 0]) * np.sin(np.pi * nodes[:, 1] / 2)
        b = (M @ (1.25 * np.pi ** 2 * u))[fd]
        x = system.solve_dst_2d(n, 1.0, 1e30, b)
        errs.append(np.max(np.abs(x - u[fd])))
    assert errs[-1] < 2e-3
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


@pytest.mark.parametrize("n", [8, 13])
def test_schur_spectrum_closed_form(n):
    for K, mu in ((1.0, 1.0), (1e-2, 1e-6)):
        R = system.Riesz(2, n, K, mu)
        S = R.schur_dense()
        assert np.allclose(S, S.T, atol=1e-12 * np.abs(S).max())
        ev = np.sort(np.linalg.eigvalsh(S))
        cf = np.sort(system.schur_eigs_2d(n, K, mu))
        assert np.max(np.abs(ev - cf)) < 1e-12 * cf.max()


def test_harmonic_extension_closed_form():
    n = 32
    R = system.Riesz(2, n, 1.0, 1.0)
    for q in (1, 5, 31):
        s = np.sin(q * np.pi * np.arange(1, n) / n)
        assert np.max(np.abs(R.harmonic_extension(s) - system.harmonic_extension_sine_2d(n, q))) < 1e-13


def test_dst_solver_large_n_residual():
    # the separable solver is the oracle at every 2D sweep size; check its residual
    # matrix-free at a size too big for dense algebra
    n = 256
    K, mu = 1e-2, 1e-3
    b = workloads.rhs(2, n, 11)
    x = system.solve_dst_2d(n, K, mu, b)
    P = fem.Problem(2, n)
    lam, U = spectral.gevp(P.A_G, P.M_G)
    H = spectral.frac_power(P.A_G, P.M_G, -0.5, (lam, U))
    y = K * (P.A @ x)
    y[P.NI:] += (1.0 / mu) * (H @ x[P.NI:])
    assert rel(y, b) < 1e-12


def test_preconditioned_spectrum_bounds():
    # spec(S_Gamma^{-1} S) lies in [1, sqrt(6)] (2D closed forms) over the sweep's K, mu
    for n in (16, 64, 256):
        h = 1.0 / n
        th = np.arange(1, n) * np.pi / n
        lam = spectral.interface_eigs_1d(n)
        mq = (h / 6) * (4 + 2 * np.cos(th))
        for K in (1.0, 1e-2, 1e-4):
            for mu in (1e-6, 1e-3, 1.0, 1e3):
                s = system.schur_eigs_2d(n, K, mu)
                sg = mq * (K * np.sqrt(lam) + np.sqrt(lam) ** -1 / mu)
                ratio = s / sg
                assert ratio.min() >= 1 - 1e-12 and ratio.max() <= np.sqrt(6) + 1e-12


@pytest.mark.parametrize("K,mu", [(1.0, 1.0), (1e-2, 1e-3), (1e-4, 1e3), (1.0, 1e-6)])
def test_schur_pcg_converges_to_solution_with_bounded_iterations(K, mu):
    n = 16
    R = system.Riesz(2, n, K, mu)
    b = workloads.rhs(2, n, 3)
    x_ref = R.solve_dense(b)
    x, its, _ = R.schur_pcg(b, rtol=1e-12)
    assert rel(x, x_ref) < 1e-10
    assert its <= 20
    # the full-system PCG with the block preconditioner differs by about one iteration
    _, its_s = R.schur_pcg(b, rtol=1e-10)[:2]
    _, its_f = R.full_pcg(b, rtol=1e-10)
    assert abs(its_s - its_f) <= 2


def test_small_K_makes_preconditioner_exact():
    # K -> 0: S -> gamma H and S_Gamma -> gamma L^{-1/2} = gamma H, so PCG stops in 1-2 steps
    R = system.Riesz(2, 16, 1e-12, 1.0)
    _, its, _ = R.schur_pcg(workloads.rhs(2, 16, 1), rtol=1e-8)
    assert its <= 2


@pytest.mark.parametrize("n,K,mu", [(16, 1.0, 1.0), (32, 1e-2, 1e-3), (24, 1e-4, 1e3), (32, 1.0, 1e-6)])
def test_sine_basis_schur_pcg_equals_assembled_schur_pcg(n, K, mu):
    # the same PCG, once on assembled matrices (LU of A_II, dense S_Gamma^{-1} or a dense RA
    # operator) and once in the sine basis: same iteration count, same residual history, same x
    from oracle import aaa, ra, spectral
    R = system.Riesz(2, n, K, mu)
    b = workloads.rhs(2, n, 11)
    x1, its1, h1 = R.schur_pcg(b, rtol=1e-10)
    x2, its2, h2 = system.schur_pcg_dst_2d(n, K, mu, b, spectral.f_precond(K, 1.0 / mu), rtol=1e-10)
    assert its1 == its2
    assert np.allclose(h1, h2, rtol=1e-8, atol=1e-12 * h1[0])
    assert rel(x2, x1) < 1e-11
    assert rel(x2, R.solve_dense(b)) < 1e-9
    # with a coarse rational table as the preconditioner (many more iterations)
    lam = spectral.interface_eigs_1d(n)
    c0, c, p = aaa.ra_table(spectral.f_precond(K, 1.0 / mu), lam[0], lam[-1], tol=1e-3, extra=lam)
    D = ra.dense_operator(R.P.A_G, R.P.M_G, c0, c, p)
    x3, its3, h3 = R.schur_pcg(b, precond=lambda r: D @ r, rtol=1e-10)
    x4, its4, h4 = system.schur_pcg_dst_2d(n, K, mu, b, lambda l: ra.eval_scalar(c0, c, p, l), rtol=1e-10)
    assert its3 == its4
    assert np.allclose(h3, h4, rtol=1e-7, atol=1e-12 * h3[0])
    assert rel(x4, x3) < 1e-10


def test_sine_basis_schur_pcg_large_n_solves_the_system():
    n, K, mu = 512, 1e-2, 1e-3
    from oracle import spectral
    b = workloads.rhs(2, n, 12)
    x, its, _ = system.schur_pcg_dst_2d(n, K, mu, b, spectral.f_precond(K, 1.0 / mu), rtol=1e-11)
    assert rel(x, system.solve_dst_2d(n, K, mu, b)) < 1e-10
    assert 2 <= its <= 20
