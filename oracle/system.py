"""The full discrete problem and reference solvers (oracle; test infrastructure only).

Definition reached by the method (plain definition, computed directly):

    x = A^{-1} b,   A = K A_Omega + gamma T^T H T,   H = L_h^{-1/2} = (M_G U) Lambda^{-1/2} (M_G U)^T

with gamma = 1/mu, A_Omega the free-dof P1 stiffness of -Delta, T the nodal injection
onto the interface dofs (the last N_Gamma free dofs), L_h = A_Gamma, M_h = M_Gamma.
This is eq. (riesz) written in the form of eq. (generic) with the P1 realization
gamma T_h^T L_h^t T_h of the perturbation (Sec. 3) at t = -1/2.

Solvers (three independent ways to the same x):
  * ``solve_dense``    dense Cholesky of A                      (tiny sizes)
  * ``solve_splu``     sparse LU of K A_Omega plus the dense Gamma block
  * ``solve_dst_2d``   separable sine-transform solver, 2D only, any size

Domain decomposition pieces (Sec. 2, eq. (block_op), eq. (dd_preconditioner)):
  * ``schur_dense``    S = K (A_GG - A_GI A_II^{-1} A_IG) + gamma H
  * ``harmonic_extension``  E = -A_II^{-1} A_IG
  * ``schur_pcg``      PCG on S x_G = g from x_0 = 0, stopping when the preconditioned
                       residual norm (r^T z)^{1/2} has fallen by the factor rtol (Sec. 3)
  * ``full_pcg``       PCG on the whole A with the symmetric block preconditioner B of
                       eq. (dd_preconditioner), exact leading block
  * ``lazy_full_pcg``  the same PCG with the operator's H by RA and B's leading block by one
                       multigrid V-cycle (remark on evaluating the operator, Sec. 3)

Parity: pinned by agreement of the three solvers, by the closed-form Schur and
harmonic-extension spectra in 2D, by the gamma = 0 reduction to the mixed
Dirichlet-Neumann Poisson problem, and by symmetry/positivity invariants
(tests/test_oracle_system.py).
"""
import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import spectral
from .fem import Problem


class Riesz:
    """One instance of the discrete problem: Problem + (K, mu) + the exact H."""

    def __init__(self, dim, n, K, mu, prob=None):
        if K <= 0 or mu <= 0:
            raise ValueError("K and mu must be positive")
        self.P = prob if prob is not None else Problem(dim, n)
        self.dim, self.n = dim, n
        self.K, self.mu = float(K), float(mu)
        self.gamma = 1.0 / self.mu
        self.eig = spectral.gevp(self.P.A_G, self.P.M_G)
        self.H = spectral.frac_power(self.P.A_G, self.P.M_G, -0.5, self.eig)

    # -- operators -------------------------------------------------------------
    def gamma_block(self):
        return self.gamma * self.H

    def matrix_sparse(self):
        """K A_Omega + gamma T^T H T as a sparse matrix (dense Gamma block included)."""
        P = self.P
        NI = P.NI
        Gblk = sp.coo_matrix(self.gamma_block())
        G = sp.coo_matrix((Gblk.data, (Gblk.row + NI, Gblk.col + NI)), shape=(P.N, P.N))
        return (self.K * P.A + G).tocsc()

    def matrix_dense(self):
        return self.matrix_sparse().toarray()

    def apply(self, x):
        """A x."""
        P = self.P
        y = self.K * (P.A @ x)
        y[P.NI:] += self.gamma_block() @ x[P.NI:]
        return y

    # -- solvers ---------------------------------------------------------------
    def solve_dense(self, b):
        A = self.matrix_dense()
        c = sla.cho_factor(A)
        return sla.cho_solve(c, b)

    def solve_splu(self, b):
        lu = spla.splu(self.matrix_sparse())
        return lu.solve(b)

    # -- Schur complement -------------------------------------------------------
    def interior_lu(self):
        if not hasattr(self, "_lu"):
            A_II, _, _, _ = self.P.blocks()
            self._lu = spla.splu(A_II.tocsc())
        return self._lu

    def schur_omega_dense(self):
        """S_Omega = A_GG - A_GI A_II^{-1} A_IG (K-free), dense."""
        A_II, A_IG, A_GI, A_GG = self.P.blocks()
        lu = self.interior_lu()
        X = lu.solve(A_IG.toarray())
        return A_GG - A_GI @ X

    def schur_dense(self):
        """S = K S_Omega + gamma H."""
        return self.K * self.schur_omega_dense() + self.gamma_block()

    def harmonic_extension(self, p):
        """E p = -A_II^{-1} A_IG p: interior values of the discrete harmonic extension."""
        A_II, A_IG, _, _ = self.P.blocks()
        return -self.interior_lu().solve(A_IG @ p)

    def schur_apply(self, p):
        A_II, A_IG, A_GI, A_GG = self.P.blocks()
        u = self.interior_lu().solve(A_IG @ p)
        return self.K * (A_GG @ p - A_GI @ u) + self.gamma_block() @ p

    def reduced_rhs(self, b):
        """g = b_G - A_GI A_II^{-1} b_I  (block elimination of eq. (block_op))."""
        NI = self.P.NI
        _, _, A_GI, _ = self.P.blocks()
        w = self.interior_lu().solve(b[:NI])
        return b[NI:] - A_GI @ w

    def back_substitute(self, b, xG):
        """x_I = A_II^{-1} (b_I / K - A_IG x_G)."""
        NI = self.P.NI
        _, A_IG, _, _ = self.P.blocks()
        return self.interior_lu().solve(b[:NI] / self.K - A_IG @ xG)

    def exact_precond(self):
        """Dense exact S_Gamma^{-1}."""
        return spectral.schur_precond_inverse(self.P.A_G, self.P.M_G, self.K, self.gamma, self.eig)

    def schur_pcg(self, b, precond=None, rtol=1e-10, maxit=500):
        """Schur-complement PCG (x_0 = 0, stop on the preconditioned residual norm).

        precond: callable r -> z, default the exact S_Gamma^{-1}.
        Returns (x, iterations, history of (r^T z)^{1/2}).
        """
        if precond is None:
            Pm = self.exact_precond()
            precond = lambda r: Pm @ r
        g = self.reduced_rhs(b)
        xG = np.zeros_like(g)
        r = g.copy()
        z = precond(r)
        rz = r @ z
        rz0 = rz
        hist = [np.sqrt(rz)]
        p = z.copy()
        its = 0
        while np.sqrt(rz) > rtol * np.sqrt(rz0) and its < maxit:
            q = self.schur_apply(p)
            alpha = rz / (p @ q)
            xG += alpha * p
            r -= alpha * q
            z = precond(r)
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
            its += 1
            hist.append(np.sqrt(abs(rz)))
        xI = self.back_substitute(b, xG)
        return np.concatenate([xI, xG]), its, hist

    def full_pcg(self, b, rtol=1e-10, maxit=500):
        """PCG on the whole A with the symmetric DD preconditioner of eq. (dd_preconditioner).

        Leading block A^00 = K A_II inverted exactly (LU, as in Sec. 3); S_Gamma exact.
        """
        P = self.P
        NI = P.NI
        A_II, A_IG, A_GI, _ = P.blocks()
        lu = self.interior_lu()
        K = self.K
        Sinv = self.exact_precond()

        def B(r):
            rI, rG = r[:NI], r[NI:]
            # lower factor: [I 0; -A^{i0} (A^{00})^{-1} I]
            w = lu.solve(rI) / K
            tG = rG - K * (A_GI @ w)
            # block diagonal inverse
            yI = w
            yG = Sinv @ tG
            # upper factor: [I -(A^{00})^{-1} A^{0i}; 0 I]
            yI = yI - lu.solve(A_IG @ yG)
            return np.concatenate([yI, yG])

        x = np.zeros_like(b)
        r = b.copy()
        z = B(r)
        rz = rz0 = r @ z
        p = z.copy()
        its = 0
        while np.sqrt(rz) > rtol * np.sqrt(rz0) and its < maxit:
            q = self.apply(p)
            alpha = rz / (p @ q)
            x += alpha * p
            r -= alpha * q
            z = B(r)
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
            its += 1
        return x, its


# ----------------------------------------------------------------------------
# Full-system PCG with the lazy block preconditioner (remark on evaluating the operator)
# ----------------------------------------------------------------------------

def operator_ra(R, tabH):
    """x -> A_RA x = K A_Omega x + gamma T^T H_RA T x, with H_RA the rational realization of
    L^{-1/2} by the table (d0, d_k, q_k): H_RA = M (d0 M^{-1} + sum_k d_k (L + q_k M)^{-1}) M
    (eq. (RA) for g(lambda) = lambda^{-1/2}; the remark on evaluating the operator, Sec. 3)."""
    from . import ra
    P = R.P
    d0, d, q = tabH
    HR = ra.dense_operator_H(P.A_G, P.M_G, d0, d, q)

    def apply(x):
        y = R.K * (P.A @ x)
        y[P.NI:] += R.gamma * (HR @ x[P.NI:])
        return y
    return apply, HR


def lazy_precond(R, tabP, vcycle):
    """r -> B r, the preconditioner of eq. (dd_preconditioner) with the leading block
    (A^00)^{-1} = (K A_II)^{-1} replaced by V / K (V one multigrid V-cycle for A_II, a
    ``multigrid.VCycle``) and S_Gamma^{-1} by the rational table (c0, c_k, p_k) of eq. (RA).

    With A^{i0} = K A_GI and A^{0i} = K A_IG the three factors give
      lower:     t_G = r_G - A^{i0} (V r_I / K) = r_G - A_GI V r_I
      diagonal:  y_I = V r_I / K,  z_G = S_Gamma^{-1} t_G
      upper:     z_I = y_I - (V / K) A^{0i} z_G = V (r_I - K A_IG z_G) / K.
    Every factor is applied as written (two V-cycles per application)."""
    from . import ra
    P = R.P
    NI = P.NI
    _, A_IG, A_GI, _ = P.blocks()
    c0, c, p = tabP

    def apply(r):
        rI, rG = r[:NI], r[NI:]
        tG = rG - A_GI @ vcycle.apply(rI)
        zG = ra.apply_tridiagonal(P.A_G, P.M_G, c0, c, p, tG)
        zI = vcycle.apply(rI - R.K * (A_IG @ zG)) / R.K
        return np.concatenate([zI, zG])
    return apply


def lazy_full_pcg(R, b, tabP, tabH, nu=2, exact_nf=0, rtol=1e-10, maxit=500):
    """PCG on the whole system A_RA x = b (operator with H by RA) preconditioned by the lazy B
    (one V-cycle for the leading block, RA for S_Gamma^{-1}); x_0 = 0, stop when (r^T z)^{1/2}
    has fallen by rtol (Sec. 3).  Returns (x, iterations, history of (r^T z)^{1/2})."""
    from .multigrid import VCycle
    V = VCycle(R.n - 1, nu=nu, exact_nf=exact_nf)
    A, _ = operator_ra(R, tabH)
    B = lazy_precond(R, tabP, V)
    x = np.zeros_like(b)
    r = np.array(b, dtype=np.float64)
    z = B(r)
    rz = rz0 = r @ z
    hist = [np.sqrt(rz)]
    p = z.copy()
    its = 0
    while np.sqrt(rz) > rtol * np.sqrt(rz0) and its < maxit:
        q = A(p)
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = B(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        its += 1
        hist.append(np.sqrt(abs(rz)))
    return x, its, hist


# ----------------------------------------------------------------------------
# 2D separable solver (no assembly; closed-form symbols)
# ----------------------------------------------------------------------------

def solve_dst_2d(n, K, mu, b):
    """Exact solve of A x = b in 2D by a sine transform along x and tridiagonal solves in y.

    Each row of free dofs (fixed j) is expanded in sin(theta_q i), theta_q = q pi / n.
    With sigma_q = 2 - 2 cos theta_q, the P1 stiffness acts on the coefficient y_j as
      rows j < n :  (2 + sigma_q) y_j - y_{j-1} - y_{j+1}        (y_0 = 0)
      row  j = n :  (1 + sigma_q / 2) y_n - y_{n-1}
    and H = L_h^{-1/2} acts on the Gamma row as mu_q lambda_q^{-1/2}, with
    mu_q = (h/6)(4 + 2 cos theta_q) the mass symbol and lambda_q the interface eigenvalue.
    """
    gamma = 1.0 / mu
    h = 1.0 / n
    B = np.asarray(b, dtype=np.float64).reshape(n, n - 1)      # rows j = 1..n
    Bh = sfft.dst(B, type=1, axis=1)
    th = np.arange(1, n) * np.pi / n
    sig = 2.0 - 2.0 * np.cos(th)
    mu_q = (h / 6.0) * (4.0 + 2.0 * np.cos(th))
    lam_q = spectral.interface_eigs_1d(n)
    Xh = np.empty_like(Bh)
    for q in range(n - 1):
        ab = np.zeros((3, n))
        ab[0, 1:] = -K                      # super-diagonal
        ab[2, :-1] = -K                     # sub-diagonal
        ab[1, :] = K * (2.0 + sig[q])
        ab[1, -1] = K * (1.0 + sig[q] / 2.0) + gamma * mu_q[q] / np.sqrt(lam_q[q])
        Xh[:, q] = sla.solve_banded((1, 1), ab, Bh[:, q])
    X = sfft.idst(Xh, type=1, axis=1)
    return X.ravel()


def schur_eigs_2d(n, K, mu):
    """Closed-form eigenvalues of S on sin(theta_q i), 2D.

    S_Omega has eigenvalue sinh(omega_q) coth(n omega_q) with cosh omega_q = 2 - cos theta_q;
    H has mu_q lambda_q^{-1/2}.
    """
    gamma = 1.0 / mu
    h = 1.0 / n
    th = np.arange(1, n) * np.pi / n
    om = np.arccosh(2.0 - np.cos(th))
    mu_q = (h / 6.0) * (4.0 + 2.0 * np.cos(th))
    lam = spectral.interface_eigs_1d(n)
    return K * np.sinh(om) / np.tanh(n * om) + gamma * mu_q / np.sqrt(lam)


def harmonic_extension_sine_2d(n, q):
    """Closed form of E sin(theta_q .): sin(theta_q i) sinh(omega_q j)/sinh(omega_q n), j < n."""
    th = q * np.pi / n
    om = np.arccosh(2.0 - np.cos(th))
    i = np.arange(1, n)
    j = np.arange(1, n)
    # sinh(om j)/sinh(om n) written without overflow for large n
    ratio = np.exp(om * (j - n)) * (-np.expm1(-2.0 * om * j)) / (-np.expm1(-2.0 * om * n))
    return (np.sin(th * i)[None, :] * ratio[:, None]).ravel()


def schur_pcg_dst_2d(n, K, mu, b, precond_symbol, rtol=1e-10, maxit=500):
    """The Schur-complement PCG of ``Riesz.schur_pcg`` computed in the interface sine basis (2D).

    Sec. 2, eq. (block_op) and the PCG of Sec. 3 (x_0 = 0, stop when (r^T z)^{1/2} has fallen by
    rtol).  In 2D every operator on Gamma is diagonal on s_q = sin(theta_q i): S has the
    closed-form eigenvalue of ``schur_eigs_2d``, and an interface preconditioner of the form
    U phi(Lambda) U^T (eq. (RA) or the exact S_Gamma^{-1}) has phi(lambda_q) / mu_q, with mu_q the
    mass symbol.  Writing every Gamma vector as v = sum_q v_q s_q turns the PCG into the same
    recurrences on coefficient vectors with the inner product (n/2) sum_q v_q w_q.  The reduced
    right-hand side and the back-substitution are the block elimination of eq. (block_op),
    done per mode by tridiagonal solves along y (interior rows j = 1..n-1, zero at j = 0 and
    j = n); A_{Gamma I} couples the interface node to the one below it with weight -1.

    precond_symbol: callable lambda -> phi(lambda) (e.g. ``ra.eval_scalar`` of a table, or
    ``spectral.f_precond``).  Returns (x, iterations, history of (r^T z)^{1/2}).
    """
    gamma = 1.0 / mu
    h = 1.0 / n
    B = np.asarray(b, dtype=np.float64).reshape(n, n - 1)
    # coefficients on s_q: v = sum_q vhat_q s_q, vhat_q = (2/n) sum_i v_i sin(theta_q i)
    Bh = sfft.dst(B, type=1, axis=1) / n
    th = np.arange(1, n) * np.pi / n
    sig = 2.0 - 2.0 * np.cos(th)
    mu_q = (h / 6.0) * (4.0 + 2.0 * np.cos(th))
    lam_q = spectral.interface_eigs_1d(n)

    def interior_solve(F):
        """A_II^{-1} per mode: F is (n-1 rows j, n-1 modes q) of sine coefficients."""
        W = np.empty_like(F)
        for q in range(n - 1):
            ab = np.zeros((3, n - 1))
            ab[0, 1:] = -1.0
            ab[2, :-1] = -1.0
            ab[1, :] = 2.0 + sig[q]
            W[:, q] = sla.solve_banded((1, 1), ab, F[:, q])
        return W

    W = interior_solve(Bh[: n - 1])
    g = Bh[n - 1] + W[n - 2]                          # g = b_G - A_GI A_II^{-1} b_I
    s_diag = schur_eigs_2d(n, K, mu)
    p_diag = np.asarray(precond_symbol(lam_q), dtype=np.float64) / mu_q
    dot = lambda u, v: 0.5 * n * float(u @ v)
    xg = np.zeros(n - 1)
    r = g.copy()
    z = p_diag * r
    rz = rz0 = dot(r, z)
    hist = [np.sqrt(rz)]
    p = z.copy()
    its = 0
    while np.sqrt(rz) > rtol * np.sqrt(rz0) and its < maxit:
        q = s_diag * p
        alpha = rz / dot(p, q)
        xg += alpha * p
        r -= alpha * q
        z = p_diag * r
        rz_new = dot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
        its += 1
        hist.append(np.sqrt(abs(rz)))
    # x_I = A_II^{-1} (b_I / K - A_IG x_G): -A_IG x_G adds x_G on the row below Gamma
    F = Bh[: n - 1] / K
    F[n - 2] += xg
    XI = interior_solve(F)
    Xh = np.vstack([XI, xg[None, :]])
    # back to nodal values: v_i = sum_q vhat_q sin(theta_q i)
    X = sfft.idst(Xh * n, type=1, axis=1)
    return X.ravel(), its, hist
