"""Pins of the oracle's H(div) problem (oracle/hdiv.py; Sec. 3 remark, eq. (graddiv), BDM1)."""
import numpy as np
import pytest

from oracle import aaa, hdiv, ra, spectral


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def tri_rule(order=8):
    """Points and weights on the reference triangle {(s, t): s, t >= 0, s + t <= 1} from a
    Gauss-Legendre tensor rule on the square mapped by the collapsed (Duffy) transform."""
    g, w = np.polynomial.legendre.leggauss(order)
    g = (g + 1) / 2
    w = w / 2
    pts, wts = [], []
    for a, wa in zip(g, w):
        for b, wb in zip(g, w):
            pts.append((a, b * (1 - a)))
            wts.append(wa * wb * (1 - a))
    return np.array(pts), np.array(wts)


def field_at(n, coef, T, x):
    return coef[np.array(T.dofs)] @ T.eval(x)


def interpolate(n, u):
    """BDM1 coefficients of a vector field: u(endpoint) . n_e at every dof."""
    h = 1.0 / n
    c = np.zeros(hdiv.sizes(n)[0])
    for e, (p, q, nrm) in enumerate(hdiv.edges(n)):
        c[2 * e] = u(np.array(p) * h) @ np.array(nrm)
        c[2 * e + 1] = u(np.array(q) * h) @ np.array(nrm)
    return c


def test_dual_basis_and_normal_traces():
    n = 3
    h = 1.0 / n
    E = hdiv.edges(n)
    for T in hdiv.triangle_bases(n):
        c = T.coords.mean(axis=0)
        for a, dof in enumerate(T.dofs):
            e = dof // 2
            p, q, nrm = E[e]
            for pt, idx in ((p, 2 * e), (q, 2 * e + 1)):
                x = np.array(pt) * h
                x = x + 1e-9 * (c - x)                       # just inside T
                for b, other in enumerate(T.dofs):
                    if other // 2 == e:
                        v = T.eval(x)[b] @ np.array(nrm)
                        assert abs(v - (1.0 if other == idx else 0.0)) < 1e-7
            # no normal component on the triangle's other two edges
            for b, other in enumerate(T.dofs):
                eo = other // 2
                if eo == e:
                    continue
                po, qo, no = E[eo]
                mid = (np.array(po) + np.array(qo)) * h / 2
                assert abs(T.eval(mid)[a] @ np.array(no)) < 1e-12


def test_linear_fields_exact():
    # BDM1 contains the linear vector fields: their interpolant reproduces them pointwise, and the
    # assembled forms give the closed-form integrals over the unit square
    n = 4
    a = np.array([0.3, -1.2, 0.7])
    b = np.array([-0.5, 0.4, 1.9])
    u = lambda x: np.array([a[0] + a[1] * x[0] + a[2] * x[1], b[0] + b[1] * x[0] + b[2] * x[1]])
    c = interpolate(n, u)
    rng = np.random.default_rng(0)
    for T in hdiv.triangle_bases(n)[::3]:
        lam = rng.dirichlet(np.ones(3))
        x = lam @ T.coords
        assert np.max(np.abs(field_at(n, c, T, x) - u(x))) < 1e-12
    Mass, Div, Bd = hdiv.assemble(n)

    def sq_int(p):
        # int over the unit square of (p0 + p1 x + p2 y)^2
        p0, p1, p2 = p
        return p0 ** 2 + p0 * (p1 + p2) + p1 ** 2 / 3 + p2 ** 2 / 3 + p1 * p2 / 2
    assert abs(c @ Mass @ c - (sq_int(a) + sq_int(b))) < 1e-12
    assert abs(c @ Div @ c - (a[1] + b[2]) ** 2) < 1e-12

    def line_sq(c0, c1):
        # int_0^1 (c0 + c1 s)^2 ds
        return c0 ** 2 + c0 * c1 + c1 ** 2 / 3
    # u.nu on the four sides: bottom -u_y(x, 0), right u_x(1, y), top u_y(x, 1), left -u_x(0, y)
    bnd = (line_sq(b[0], b[1]) + line_sq(a[0] + a[1], a[2]) + line_sq(b[0] + b[2], b[1])
           + line_sq(a[0], a[2]))
    assert abs(c @ Bd @ c - bnd) < 1e-12


def test_divergence_theorem_per_triangle():
    n = 3
    E = hdiv.edges(n)
    for T in hdiv.triangle_bases(n):
        d = T.div()
        centroid = T.coords.mean(axis=0)
        for a in range(6):
            flux = 0.0
            for k in range(3):
                x0, x1 = T.coords[k], T.coords[(k + 1) % 3]
                tang = x1 - x0
                nout = np.array([tang[1], -tang[0]])
                if nout @ (centroid - x0) > 0:
                    nout = -nout                              # |nout| = edge length
                # the normal component is linear along the edge: trapezoid rule is exact
                flux += 0.5 * (T.eval(x0 + 1e-12 * (centroid - x0))[a] @ nout
                               + T.eval(x1 + 1e-12 * (centroid - x1))[a] @ nout)
            assert abs(d[a] * T.area - flux) < 1e-9


@pytest.mark.parametrize("nc", [2, 4])
def test_nested_spaces_galerkin(nc):
    # BDM1 on the refined mesh contains the coarse space: P^T A_f P = A_c for mass and div-div,
    # and the inclusion maps the interpolant of a linear field to the fine interpolant
    P = hdiv.prolongation(nc)
    Mf, Df, _ = hdiv.assemble(2 * nc)
    Mc, Dc, _ = hdiv.assemble(nc)
    assert abs(P.T @ Mf @ P - Mc).max() < 1e-14
    assert abs(P.T @ Df @ P - Dc).max() < 1e-12
    u = lambda x: np.array([0.2 - x[0] + 3 * x[1], 1.1 + 0.5 * x[0] - 2 * x[1]])
    assert np.max(np.abs(P @ interpolate(nc, u) - interpolate(2 * nc, u))) < 1e-12


def test_manufactured_solution_second_order():
    # K (u - grad div u) = f in Omega, K div u + gamma u.nu = g on the boundary (the natural
    # condition of eq. (graddiv)); u = (sin(pi x) cos(pi y / 2), x^2 e^y)
    K, gamma = 1.3, 2.0
    pi = np.pi

    def u(x):
        return np.array([np.sin(pi * x[0]) * np.cos(pi * x[1] / 2), x[0] ** 2 * np.exp(x[1])])

    def div(x):
        return pi * np.cos(pi * x[0]) * np.cos(pi * x[1] / 2) + x[0] ** 2 * np.exp(x[1])

    def grad_div(x):
        return np.array([-pi ** 2 * np.sin(pi * x[0]) * np.cos(pi * x[1] / 2) + 2 * x[0] * np.exp(x[1]),
                         -pi ** 2 / 2 * np.cos(pi * x[0]) * np.sin(pi * x[1] / 2) + x[0] ** 2 * np.exp(x[1])])

    qp, qw = tri_rule(6)
    gl, gw = np.polynomial.legendre.leggauss(6)
    errs = []
    for n in (4, 8, 16):
        P = hdiv.HdivProblem(n, K, gamma)
        bases = hdiv.triangle_bases(n)
        b = np.zeros(P.N)
        for T in bases:
            B = np.array([T.coords[1] - T.coords[0], T.coords[2] - T.coords[0]]).T
            for (s, t), w in zip(qp, qw):
                x = T.coords[0] + B @ np.array([s, t])
                f = K * (u(x) - grad_div(x))
                b[np.array(T.dofs)] += w * 2 * T.area * (T.eval(x) @ f)
        h = 1.0 / n
        for k, (p, q, nrm) in enumerate(hdiv.loop_edges(n)):
            x0, x1 = np.array(p) * h, np.array(q) * h
            nu = np.array(nrm)
            for s, w in zip((gl + 1) / 2, gw / 2):
                x = x0 + s * (x1 - x0)
                g = K * div(x) + gamma * (u(x) @ nu)
                b[P.N0 + 2 * k] += w * h * g * (1 - s)
                b[P.N0 + 2 * k + 1] += w * h * g * s
        c = P.solve_splu(b)
        e2 = 0.0
        for T in bases:
            B = np.array([T.coords[1] - T.coords[0], T.coords[2] - T.coords[0]]).T
            for (s, t), w in zip(qp, qw):
                x = T.coords[0] + B @ np.array([s, t])
                d = field_at(n, c, T, x) - u(x)
                e2 += w * 2 * T.area * (d @ d)
        errs.append(np.sqrt(e2))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


@pytest.mark.parametrize("n", [2, 4, 8])
def test_loop_spectrum_closed_form(n):
    L, M = hdiv.loop_sipg(n), hdiv.loop_mass(n)
    lam = spectral.gevp(L, M)[0]
    assert np.max(np.abs(lam - hdiv.loop_eigs(n))) < 1e-11 * lam.max()
    assert np.max(np.abs(L - L.T)) < 1e-12 and lam.min() > 0
    one = np.ones(8 * n)
    assert np.max(np.abs(L @ one - M @ one)) < 1e-12           # constants: lambda = 1
    assert abs(lam.min() - 1.0) < 1e-12


def test_loop_operator_consistent():
    # phi_h^T L phi_h -> int (phi'^2 + phi^2) ds over the loop (length 4) for a smooth periodic
    # phi sampled at the segment ends (continuous, so the jump terms vanish), second order
    errs = []
    for n in (4, 8, 16):
        m = 4 * n
        s = np.arange(m + 1) * (4.0 / m)
        phi = np.cos(np.pi * s / 2) + 0.5 * np.sin(np.pi * s)
        v = np.empty(2 * m)
        v[0::2], v[1::2] = phi[:-1], phi[1:]
        ss = np.linspace(0, 4, 200001)
        ph = np.cos(np.pi * ss / 2) + 0.5 * np.sin(np.pi * ss)
        dph = -np.pi / 2 * np.sin(np.pi * ss / 2) + 0.5 * np.pi * np.cos(np.pi * ss)
        exact = np.trapezoid(ph ** 2 + dph ** 2, ss)
        errs.append(abs(v @ hdiv.loop_sipg(n) @ v - exact))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def test_loop_operator_consistent_with_discontinuous_tests():
    # For smooth periodic phi, l(phi_h, v) = int (-phi'' + phi) v ds + O(h^2) for every DG test
    # function v (the symmetric interior-penalty form is consistent: the mean-derivative term
    # cancels the vertex terms of the integration by parts; dropping it or flipping its sign
    # leaves an O(1) error in the first derivative)
    errs = []
    gl, gw = np.polynomial.legendre.leggauss(5)
    for n in (4, 8, 16, 32):
        m = 4 * n
        h = 1.0 / n
        phi = lambda s: np.cos(np.pi * s / 2) + 0.5 * np.sin(np.pi * s)
        g = lambda s: (1 + np.pi ** 2 / 4) * np.cos(np.pi * s / 2) + 0.5 * (1 + np.pi ** 2) * np.sin(np.pi * s)
        sv = np.arange(m + 1) * h
        v = np.empty(2 * m)
        v[0::2], v[1::2] = phi(sv[:-1]), phi(sv[1:])
        lhs = hdiv.loop_sipg(n) @ v
        rhs = np.empty(2 * m)
        for k in range(m):
            t = (gl + 1) / 2
            x = sv[k] + t * h
            rhs[2 * k] = h * np.sum(gw / 2 * g(x) * (1 - t))
            rhs[2 * k + 1] = h * np.sum(gw / 2 * g(x) * t)
        errs.append(np.max(np.abs(lhs - rhs)))
    assert all(a / b > 3.5 for a, b in zip(errs, errs[1:]))


def test_schur_identity_and_robust_preconditioner():
    kappas = {}
    for n in (4, 8, 16):
        for K, gamma in ((1.0, 1e-3), (1.0, 1.0), (1e-2, 1e3)):
            P = hdiv.HdivProblem(n, K, gamma)
            A = P.A.toarray()
            S = P.schur_dense()
            # the Schur complement inverts to the trace block of the inverse
            Sinv_ref = np.linalg.inv(A)[P.N0:, P.N0:]
            assert rel(np.linalg.inv(S), Sinv_ref) < 1e-10
            assert np.max(np.abs(S - S.T)) < 1e-10 * np.max(np.abs(S))
            ev = np.linalg.eigvals(np.linalg.solve(P.schur_precond(), S)).real
            kappas[(n, K, gamma)] = ev.max() / ev.min()
            # exact_precond is the inverse of S_Gamma
            assert rel(P.exact_precond() @ P.schur_precond(), np.eye(P.NG)) < 1e-10
    # bounded in h and gamma (7.06, 7.25, ... at gamma/K = 1e-3; ~2.8 at 1; ~1 at 1e5)
    assert max(kappas.values()) < 8.0
    for K, gamma in ((1.0, 1e-3), (1.0, 1.0), (1e-2, 1e3)):
        ks = [kappas[(n, K, gamma)] for n in (4, 8, 16)]
        assert all(b < 1.05 * a for a, b in zip(ks, ks[1:]))


@pytest.mark.parametrize("K,gamma", [(1.0, 1.0), (1.0, 1e-3), (1e-2, 10.0)])
def test_ra_preconditioner_within_table_error(K, gamma):
    n = 8
    P = hdiv.HdivProblem(n, K, gamma)
    lam = hdiv.loop_eigs(n)
    tab = aaa.ra_table(P.g_table_function(), lam[0], lam[-1], 1e-12, extra=lam)
    D = hdiv.ra_precond(P.L, P.M_Q, tab)
    # the realization is U (lam g_RA(lam)) U^T; its distance to S_Gamma^{-1} is the table's error
    f_ra = lambda x: x * ra.eval_scalar(*tab, x)
    assert rel(D, spectral.spectral_function(P.L, P.M_Q, f_ra, P.eig)) < 1e-10
    err = ra.max_rel_error(P.g_table_function(), *tab, lam)
    assert err < 1e-9
    assert rel(D, P.exact_precond()) < 2 * err + 1e-11


@pytest.mark.parametrize("K,gamma", [(1.0, 1.0), (1.0, 1e-3), (1e-2, 1e3)])
def test_schur_pcg_matches_direct(K, gamma):
    P = hdiv.HdivProblem(8, K, gamma)
    b = np.random.default_rng(3).standard_normal(P.N)
    x, its = P.schur_pcg(b, rtol=1e-10)
    assert rel(x, P.solve_splu(b)) < 1e-9
    assert rel(P.solve_dense(b), P.solve_splu(b)) < 1e-12
    assert its <= 30


@pytest.mark.parametrize("n,K,gamma", [(4, 1.0, 1.0), (8, 1e-2, 1e3), (8, 1.0, 0.0)])
def test_fft_preconditioner_matches_dense(n, K, gamma):
    # the block-circulant (Fourier-mode) application used at sizes beyond the dense oracle
    P = hdiv.HdivProblem(n, K, gamma)
    lam = hdiv.loop_eigs(n)
    tab = aaa.ra_table(P.g_table_function(), lam[0], lam[-1], 1e-12, extra=lam)
    r = np.random.default_rng(n).standard_normal(P.NG)
    z = hdiv.ra_precond_apply_fft(n, tab, r)
    assert rel(z, hdiv.ra_precond(P.L, P.M_Q, tab) @ r) < 1e-12
    own, prev, Ms = hdiv.loop_symbols(n)
    assert np.max(np.abs(P.L[2:4, 2:4] - own)) < 1e-12 and np.max(np.abs(P.L[2:4, 0:2] - prev)) < 1e-12

