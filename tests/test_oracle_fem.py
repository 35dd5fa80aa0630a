"""Pins of the oracle's P1 assembly (CPU only).

Each check is fixed by mathematics the assembly code does not encode: textbook
stencils of P1 on structured meshes, reproduction of linear functions, the measure
of the domain, and the closed-form eigenpairs of the 1D interface operators.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem, spectral


@pytest.mark.parametrize("n", [4, 8, 16])
def test_2d_stiffness_rows_are_five_point(n):
    P = fem.Problem(2, n)
    A = P.A.toarray()
    # an interior node away from every boundary: (i, j) = (n/2, n/2)
    i, j = n // 2, n // 2
    r = (j - 1) * (n - 1) + (i - 1)
    row = A[r]
    assert row[r] == pytest.approx(4.0)
    for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        c = (j + dj - 1) * (n - 1) + (i + di - 1)
        assert row[c] == pytest.approx(-1.0)
    assert np.count_nonzero(np.abs(row) > 1e-14) == 5
    # Gamma row: natural boundary -> (2, -1/2, -1/2, -1 below)
    r = P.NI + (i - 1)
    row = A[r]
    assert row[r] == pytest.approx(2.0)
    assert row[r - 1] == pytest.approx(-0.5) and row[r + 1] == pytest.approx(-0.5)
    assert row[(n - 2) * (n - 1) + (i - 1)] == pytest.approx(-1.0)
    assert np.count_nonzero(np.abs(row) > 1e-14) == 4


def test_3d_kuhn_stiffness_rows_are_seven_point():
    n = 6
    h = 1.0 / n
    P = fem.Problem(3, n)
    A = P.A.toarray()
    i = j = k = 3

    def idx(i, j, k):
        return ((k - 1) * (n - 1) + (j - 1)) * (n - 1) + (i - 1)

    row = A[idx(i, j, k)]
    assert row[idx(i, j, k)] == pytest.approx(6.0 * h)
    for d in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        assert row[idx(i + d[0], j + d[1], k + d[2])] == pytest.approx(-h)
    assert np.count_nonzero(np.abs(row) > 1e-14) == 7
    row = A[idx(i, j, n)]
    assert row[idx(i, j, n)] == pytest.approx(3.0 * h)
    assert row[idx(i, j, n - 1)] == pytest.approx(-h)
    assert np.count_nonzero(np.abs(row) > 1e-14) == 6


@pytest.mark.parametrize("dim,n", [(2, 5), (2, 8), (3, 3)])
def test_linear_functions_are_discretely_harmonic(dim, n):
    # a(x_1, v) = int d v / d x_1 = 0 for v vanishing on the boundary, so the full
    # (all-node) stiffness maps the coordinate function to zero at interior nodes.
    nodes, cells = fem.mesh_2d(n) if dim == 2 else fem.mesh_3d(n)
    A, M = fem.assemble(nodes, cells)
    interior = np.all((nodes > 1e-12) & (nodes < 1 - 1e-12), axis=1)
    for c in range(dim):
        y = A @ nodes[:, c]
        assert np.max(np.abs(y[interior])) < 1e-12
    # constants are in the kernel everywhere
    assert np.max(np.abs(A @ np.ones(len(nodes)))) < 1e-12
    # the mass integrates 1 to the measure of the unit square/cube
    assert np.ones(len(nodes)) @ (M @ np.ones(len(nodes))) == pytest.approx(1.0, rel=1e-13)


@pytest.mark.parametrize("dim,n", [(2, 6), (3, 3)])
def test_free_stiffness_is_spd(dim, n):
    P = fem.Problem(dim, n)
    A = P.A.toarray()
    assert np.allclose(A, A.T, atol=1e-14)
    assert np.linalg.eigvalsh(A).min() > 0


@pytest.mark.parametrize("n", [8, 16, 33])
def test_interface_gevp_matches_closed_form(n):
    P = fem.Problem(2, n)
    lam, U = spectral.gevp(P.A_G, P.M_G)
    exact = spectral.interface_eigs_1d(n)
    assert np.max(np.abs(lam - np.sort(exact)) / exact.max()) < 1e-13
    assert np.max(np.abs(U.T @ P.M_G @ U - np.eye(n - 1))) < 1e-12
    # eigenvectors are sin(q pi i / n)
    i = np.arange(1, n)
    for q in (1, 2, n - 1):
        s = np.sin(q * np.pi * i / n)
        u = U[:, q - 1]
        c = (u @ s) / (s @ s)
        assert np.max(np.abs(u - c * s)) < 1e-10


def test_interface_face_mesh_3d():
    n = 5
    nodes, cells = fem.interface_mesh(3, n)
    assert cells.shape == (2 * n * n, 3)
    P = fem.Problem(3, n)
    # face stiffness of 2D P1 on the diagonal-split mesh is the 5-point stencil (scale free)
    i = j = 2
    r = (j - 1) * (n - 1) + (i - 1)
    row = P.A_G[r]
    assert row[r] == pytest.approx(4.0)
    assert np.count_nonzero(np.abs(row) > 1e-14) == 5
    # consistent face mass: 6 neighbours (x, y and one diagonal) with weight h^2/12
    h = 1.0 / n
    mrow = P.M_G[r]
    assert mrow[r] == pytest.approx(6 * h * h / 12)
    assert np.count_nonzero(np.abs(mrow) > 1e-14) == 7


def test_rayleigh_ritz_bounds_on_interface_spectrum():
    # conforming P1 eigenvalues bound the continuous ones from above: lambda_1 >= pi^2 (1D)
    for n in (8, 64, 512):
        lam = spectral.interface_eigs_1d(n)
        assert lam[0] >= np.pi ** 2
        assert lam[-1] <= 12.0 * n * n
    lo, hi = spectral.spectral_interval(3, 6)
    assert lo >= 2 * np.pi ** 2
    assert hi <= 36.0 * 36


def test_galerkin_coarse_operator_is_rediscretized_stencil():
    # nested diagonal-split meshes: P^T A_h P = A_2h with P the P1 interpolation
    nc = 4
    nf = 2 * nc
    Pf = fem.Problem(2, nf)
    Pc = fem.Problem(2, nc)
    A_h = Pf.A.toarray()[:Pf.NI, :Pf.NI]
    A_2h = Pc.A.toarray()[:Pc.NI, :Pc.NI]
    nodes_c, tris_c = fem.mesh_2d(nc)
    # evaluate coarse interior basis functions at fine interior nodes
    Pmat = np.zeros((Pf.NI, Pc.NI))
    for jc in range(1, nc):
        for ic in range(1, nc):
            col = (jc - 1) * (nc - 1) + (ic - 1)
            for jf in range(1, nf):
                for i_f in range(1, nf):
                    x, y = i_f / nf, jf / nf
                    # barycentric value of the coarse hat at (x, y) on its support
                    val = 0.0
                    for t in tris_c:
                        v = nodes_c[t]
                        Bm = np.array([v[1] - v[0], v[2] - v[0]]).T
                        lam12 = np.linalg.solve(Bm, np.array([x, y]) - v[0])
                        lam = np.array([1 - lam12.sum(), lam12[0], lam12[1]])
                        if np.all(lam >= -1e-12):
                            cn = jc * (nc + 1) + ic
                            where = np.nonzero(t == cn)[0]
                            val = lam[where[0]] if len(where) else 0.0
                            break
                    Pmat[(jf - 1) * (nf - 1) + (i_f - 1), col] = val
    assert np.max(np.abs(Pmat.T @ A_h @ Pmat - A_2h)) < 1e-12
