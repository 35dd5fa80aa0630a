"""Pins of the oracle's V-cycle (oracle/multigrid.py) and of the full-system PCG with the lazy
block preconditioner (system.lazy_full_pcg; remark on evaluating the operator, Sec. 3)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads
from oracle import aaa, fem, multigrid, spectral, system


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def hat_prolongation(nc):
    """Coarse hat functions evaluated at the fine interior nodes by barycentric coordinates on
    the coarse mesh's own triangles (brute force: every triangle is tried)."""
    n_c = nc + 1
    nf = 2 * nc + 1
    nodes_c, tris_c = fem.mesh_2d(n_c)
    Pm = np.zeros((nf * nf, nc * nc))
    for jc in range(1, nc + 1):
        for ic in range(1, nc + 1):
            cn = jc * (n_c + 1) + ic
            for jf in range(1, nf + 1):
                for i_f in range(1, nf + 1):
                    xy = np.array([i_f, jf]) / (2.0 * n_c)
                    for t in tris_c:
                        v = nodes_c[t]
                        lam12 = np.linalg.solve(np.array([v[1] - v[0], v[2] - v[0]]).T, xy - v[0])
                        lam = np.array([1 - lam12.sum(), lam12[0], lam12[1]])
                        if np.all(lam >= -1e-12):
                            w = np.nonzero(t == cn)[0]
                            Pm[(jf - 1) * nf + i_f - 1, (jc - 1) * nc + ic - 1] = lam[w[0]] if len(w) else 0.0
                            break
    return Pm


def test_prolongation_is_p1_interpolation():
    for nc in (1, 3):
        P = multigrid.prolongation(nc).toarray()
        assert np.max(np.abs(P - hat_prolongation(nc))) < 1e-14


@pytest.mark.parametrize("nc", [3, 7])
def test_stiffness_and_galerkin_identity(nc):
    nf = 2 * nc + 1
    # the 5-point matrix is the assembled interior stiffness of the P1 problem
    Pf = fem.Problem(2, nf + 1)
    assert np.max(np.abs(multigrid.stiffness(nf).toarray() - Pf.A.toarray()[:Pf.NI, :Pf.NI])) < 1e-12
    P = multigrid.prolongation(nc)
    G = (P.T @ multigrid.stiffness(nf) @ P).toarray()
    assert np.max(np.abs(G - multigrid.stiffness(nc).toarray())) < 1e-12


def test_hierarchy_rule():
    assert multigrid.hierarchy(1023) == [1023, 511, 255, 127, 63, 31, 15, 7]
    assert multigrid.hierarchy(119) == [119, 59, 29, 14]
    assert multigrid.hierarchy(95) == [95, 47, 23, 11, 5]
    assert multigrid.hierarchy(7) == [7, 3]


def test_half_sweep_is_gauss_seidel_on_its_colour():
    rng = np.random.default_rng(0)
    nf = 9
    A = multigrid.stiffness(nf)
    f = rng.standard_normal((nf, nf))
    u = rng.standard_normal((nf, nf))
    for red in (True, False):
        v = multigrid.half_sweep(u, f, red)
        res = (f.ravel() - A @ v.ravel()).reshape(nf, nf)
        mask = multigrid.red_mask(nf) if red else ~multigrid.red_mask(nf)
        assert np.max(np.abs(res[mask])) < 1e-13           # own equations now hold
        assert np.array_equal(v[~mask], u[~mask])          # the other colour is untouched


def vcycle_matrix(V, nf):
    return np.column_stack([V.apply(e) for e in np.eye(nf * nf)])


@pytest.mark.parametrize("nf,nu", [(15, 1), (15, 2), (31, 2)])
def test_vcycle_is_symmetric_positive_definite(nf, nu):
    V = multigrid.VCycle(nf, nu=nu)
    M = vcycle_matrix(V, nf)
    assert np.max(np.abs(M - M.T)) < 1e-12 * np.max(np.abs(M))
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0


@pytest.mark.parametrize("nf,nu,bound", [(31, 1, 0.5), (63, 1, 0.5), (31, 2, 0.3), (63, 2, 0.3)])
def test_vcycle_contraction(nf, nu, bound):
    # a multigrid V(nu, nu) cycle contracts the error by a factor bounded away from 1 independently
    # of the grid; with P1 interpolation on the diagonal-split mesh and red-black Gauss-Seidel the
    # two-grid factor is about 0.38 (nu = 1) and 0.18 (nu = 2), the V-cycle's a little above.
    # A restriction off by a factor 4 gives about 0.9, a sweep that misses a colour diverges.
    V = multigrid.VCycle(nf, nu=nu)
    A = multigrid.stiffness(nf)
    E = spla.LinearOperator(A.shape, matvec=lambda e: e - V.apply(A @ e))
    rho = abs(spla.eigs(E, k=1, which="LM", return_eigenvectors=False, tol=1e-8)[0])
    assert rho < bound


def test_vcycle_with_exact_first_coarse_level():
    # exact_nf = 63 solves the 63 x 63 level exactly: a two-grid cycle on 127 x 127 points
    V = multigrid.VCycle(127, nu=2, exact_nf=63)
    assert V.sizes == [127, 63]
    f = np.random.default_rng(1).standard_normal(63 * 63)
    assert rel(V.apply(f, level=1), spla.spsolve(multigrid.stiffness(63).tocsc(), f)) < 1e-12


def tables(n, K, mu, tol=1e-12):
    lo, hi = spectral.spectral_interval(2, n)
    lam = spectral.interface_eigs_1d(n)
    tp = aaa.ra_table(spectral.f_precond(K, 1.0 / mu), lo, hi, tol, extra=lam)
    th = aaa.ra_table(spectral.g_operator, lo, hi, tol, extra=lam)
    return tp, th


class ExactInterior:
    """Stands in for a V-cycle: the exact A_II^{-1}."""

    def __init__(self, R):
        self.lu = R.interior_lu()

    def apply(self, f):
        return self.lu.solve(f)


def test_lazy_preconditioner_reduces_to_the_exact_block_preconditioner():
    # with the exact A_II^{-1} in place of the V-cycle and the exact S_Gamma^{-1} in place of the
    # table, B must be the exact preconditioner of eq. (dd_preconditioner) that full_pcg uses
    n, K, mu = 8, 1e-2, 1e-3
    R = system.Riesz(2, n, K, mu)
    P = R.P
    NI = P.NI
    A_II, A_IG, A_GI, _ = P.blocks()
    Sinv = R.exact_precond()
    # eq. (dd_preconditioner) assembled factor by factor
    A00 = K * A_II.toarray()
    A0i = K * A_IG.toarray()
    Ai0 = K * A_GI.toarray()
    I0, Ii = np.eye(NI), np.eye(P.NG)
    Z = np.zeros((NI, P.NG))
    U = np.block([[I0, -np.linalg.solve(A00, A0i)], [Z.T, Ii]])
    D = np.block([[np.linalg.inv(A00), Z], [Z.T, Sinv]])
    L = np.block([[I0, Z], [-Ai0 @ np.linalg.inv(A00), Ii]])
    B_exact = U @ D @ L
    tp, _ = tables(n, K, mu)
    Bl = system.lazy_precond(R, tp, ExactInterior(R))
    Bm = np.column_stack([Bl(e) for e in np.eye(P.N)])
    # the only difference left is the table's error in S_Gamma^{-1}
    assert rel(Bm, B_exact) < 1e-9
    assert np.max(np.abs(Bm - Bm.T)) < 1e-9 * np.max(np.abs(Bm))


def test_lazy_preconditioner_is_spd_with_a_vcycle():
    n = 16
    R = system.Riesz(2, n, 1.0, 1.0)
    tp, _ = tables(n, 1.0, 1.0)
    V = multigrid.VCycle(n - 1, nu=1)
    Bl = system.lazy_precond(R, tp, V)
    Bm = np.column_stack([Bl(e) for e in np.eye(R.P.N)])
    assert np.max(np.abs(Bm - Bm.T)) < 1e-10 * np.max(np.abs(Bm))
    assert np.linalg.eigvalsh(0.5 * (Bm + Bm.T)).min() > 0


def test_operator_ra_matches_exact_operator_to_table_error():
    n, K, mu = 16, 1.0, 1e-2
    R = system.Riesz(2, n, K, mu)
    _, th = tables(n, K, mu)
    A, HR = system.operator_ra(R, th)
    x = workloads.rhs(2, n, 3)
    assert rel(A(x), R.apply(x)) < 1e-10
    assert rel(HR, R.H) < 1e-10


@pytest.mark.parametrize("n,K,mu", [(16, 1.0, 1.0), (32, 1e-2, 1e-3), (32, 1e-4, 1e3), (64, 1.0, 1e-6)])
def test_lazy_full_pcg_solves_the_ra_system(n, K, mu):
    R = system.Riesz(2, n, K, mu)
    tp, th = tables(n, K, mu)
    b = workloads.rhs(2, n, 11)
    x, its, hist = system.lazy_full_pcg(R, b, tp, th, nu=2, rtol=1e-10)
    A, HR = system.operator_ra(R, th)
    # dense solve of the operator with H_RA
    M = (K * R.P.A).toarray()
    M[R.P.NI:, R.P.NI:] += R.gamma * HR
    x_ref = np.linalg.solve(M, b)
    assert rel(x, x_ref) < 1e-8
    assert hist[-1] <= 1e-10 * hist[0]
    assert its <= 40
    # and the exact system's solution differs only by the operator table's error
    assert rel(x, system.solve_dst_2d(n, K, mu, b)) < 1e-8


def test_lazy_full_pcg_counts_bounded_in_mesh_size():
    # Fig. 4-left: with one V-cycle for the leading block the PCG count stays bounded as h -> 0
    counts = []
    for n in (16, 32, 64, 128):
        R = system.Riesz(2, n, 1.0, 1.0)
        tp, th = tables(n, 1.0, 1.0)
        _, its, _ = system.lazy_full_pcg(R, workloads.rhs(2, n, 5), tp, th, nu=2, rtol=1e-10)
        counts.append(its)
    assert max(counts) <= 40
    assert counts[-1] <= counts[0] + 8
