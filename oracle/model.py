"""The paper's own model problem (Sec. 3, eq. (model_problem)) in 2D (oracle; test infrastructure).

Find x in V = H^1(Omega), Omega = (0, 1)^2, with Gamma = the whole boundary, such that

    K (-Delta + I) x + gamma (-Delta_Gamma + I)^t x = b,      K > 0, gamma >= 0, -1 < t < 1.

P1 elements on the diagonal-split mesh of n cells per side; every node is a dof.  In the form of
eq. (generic): A = K (A_Omega + M_Omega) + gamma T^T L_h^t T, with A_Omega, M_Omega the P1
stiffness and mass on all (n+1)^2 nodes (natural boundary conditions), T the nodal trace onto
the 4n boundary nodes, and L_h^t = (M_G U) Lambda^t (M_G U)^T from L_h U = M_G U Lambda
(eq. (gevp)) with L_h = A_G + M_G the matrix of -Delta_Gamma + I on the closed boundary curve
(1D P1 on a loop of 4n segments of length h, corners included) and M_G its mass.

Dof order (the product's order too): the (n-1)^2 interior nodes, index (j-1)(n-1) + (i-1) for
j, i = 1..n-1, then the 4n boundary nodes counter-clockwise from the corner (0, 0):
  k = i            bottom, (i, 0),      i = 0..n-1
  k = n + j        right,  (n, j),      j = 0..n-1
  k = 2n + (n - i) top,    (i, n),      i = n..1
  k = 3n + (n - j) left,   (0, j),      j = n..1

Domain decomposition (Sec. 2-3): S = K S_Omega + gamma L_h^t with S_Omega the Schur complement
of A_Omega + M_Omega onto the boundary, preconditioned by S_Gamma = K L^{1/2} + gamma L^t
(the operators coincide with L = -Delta_Gamma + I, Sec. 3).

Parity: pinned by the closed-form spectrum of the loop operators (circulant), the identities
t = 0 (L^0 = M_G), t = 1 (L), t = -1 (M L^{-1} M), second-order convergence to a manufactured
Neumann solution, agreement of dense and sparse solves, the Schur complement identity and
spectral equivalence of S and S_Gamma (tests/test_oracle_model.py).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import spectral
from .fem import assemble, mesh_2d


def loop_nodes(n):
    """(i, j) grid coordinates of the boundary nodes in loop order."""
    out = [(i, 0) for i in range(n)]
    out += [(n, j) for j in range(n)]
    out += [(i, n) for i in range(n, 0, -1)]
    out += [(0, j) for j in range(n, 0, -1)]
    return out


def dof_order(n):
    """Global node numbers (j (n+1) + i) in dof order: interior, then the boundary loop."""
    inner = [j * (n + 1) + i for j in range(1, n) for i in range(1, n)]
    loop = [j * (n + 1) + i for (i, j) in loop_nodes(n)]
    return np.array(inner + loop, dtype=np.int64)


def loop_matrices(n):
    """A_G and M_G of the closed boundary curve, assembled segment by segment from the 1D P1
    element matrices of a segment of length l: (1/l)[[1, -1], [-1, 1]] and (l/6)[[2, 1], [1, 2]]
    (tangential derivative along the curve)."""
    h = 1.0 / n
    pts = np.array(loop_nodes(n), dtype=np.float64) * h
    m = 4 * n
    A = np.zeros((m, m))
    M = np.zeros((m, m))
    for k in range(m):
        a, b = k, (k + 1) % m
        ln = float(np.linalg.norm(pts[b] - pts[a]))
        idx = np.ix_([a, b], [a, b])
        A[idx] += np.array([[1.0, -1.0], [-1.0, 1.0]]) / ln
        M[idx] += np.array([[2.0, 1.0], [1.0, 2.0]]) * ln / 6.0
    return A, M


def loop_eigs(n):
    """Closed form of the spectrum of (A_G + M_G, M_G) on the loop (circulant operators):
    lambda_q = (2 - 2 cos th_q) / h / ((h / 6)(4 + 2 cos th_q)) + 1, th_q = 2 pi q / (4 n)."""
    h = 1.0 / n
    th = 2.0 * np.pi * np.arange(4 * n) / (4 * n)
    return np.sort((2.0 - 2.0 * np.cos(th)) / h / ((h / 6.0) * (4.0 + 2.0 * np.cos(th))) + 1.0)


class ModelProblem:
    """One instance (n, K, gamma, t) of eq. (model_problem) in 2D with exact L^t."""

    def __init__(self, n, K, gamma, t):
        if K <= 0 or gamma < 0 or not (-1.0 < t < 1.0):
            raise ValueError("need K > 0, gamma >= 0, -1 < t < 1")
        self.n, self.K, self.gamma, self.t = n, float(K), float(gamma), float(t)
        nodes, cells = mesh_2d(n)
        A, M = assemble(nodes, cells)
        order = dof_order(n)
        self.A = A[order][:, order].tocsr()       # stiffness, dof order
        self.M = M[order][:, order].tocsr()       # mass
        self.NI = (n - 1) ** 2
        self.NG = 4 * n
        self.N = self.NI + self.NG
        self.A_G, self.M_G = loop_matrices(n)
        self.L = self.A_G + self.M_G
        self.eig = spectral.gevp(self.L, self.M_G)
        self.Lt = spectral.frac_power(self.L, self.M_G, self.t, self.eig)

    # -- operators -------------------------------------------------------------
    def omega_block(self):
        """A_Omega + M_Omega (K-free), sparse."""
        return (self.A + self.M).tocsr()

    def matrix_sparse(self):
        NI = self.NI
        G = sp.coo_matrix(self.gamma * self.Lt)
        G = sp.coo_matrix((G.data, (G.row + NI, G.col + NI)), shape=(self.N, self.N))
        return (self.K * self.omega_block() + G).tocsc()

    def apply(self, x):
        y = self.K * (self.omega_block() @ x)
        y[self.NI:] += self.gamma * (self.Lt @ x[self.NI:])
        return y

    def solve_dense(self, b):
        return sla.cho_solve(sla.cho_factor(self.matrix_sparse().toarray()), b)

    def solve_splu(self, b):
        return spla.splu(self.matrix_sparse()).solve(b)

    # -- domain decomposition -----------------------------------------------------
    def blocks(self):
        B = self.omega_block()
        NI = self.NI
        return (B[:NI, :NI].tocsc(), B[:NI, NI:].tocsc(), B[NI:, :NI].tocsc(),
                B[NI:, NI:].toarray())

    def interior_lu(self):
        if not hasattr(self, "_lu"):
            self._lu = spla.splu(self.blocks()[0])
        return self._lu

    def schur_dense(self):
        """S = K (B_GG - B_GI B_II^{-1} B_IG) + gamma L^t, with B = A_Omega + M_Omega."""
        B_II, B_IG, B_GI, B_GG = self.blocks()
        X = self.interior_lu().solve(B_IG.toarray())
        return self.K * (B_GG - B_GI @ X) + self.gamma * self.Lt

    def schur_apply(self, p):
        _, B_IG, B_GI, B_GG = self.blocks()
        u = self.interior_lu().solve(B_IG @ p)
        return self.K * (B_GG @ p - B_GI @ u) + self.gamma * (self.Lt @ p)

    def f_precond(self):
        K, g, t = self.K, self.gamma, self.t
        return lambda lam: 1.0 / (K * np.sqrt(lam) + g * lam ** t)

    def exact_precond(self):
        """S_Gamma^{-1} = U (K Lambda^{1/2} + gamma Lambda^t)^{-1} U^T."""
        return spectral.spectral_function(self.L, self.M_G, self.f_precond(), self.eig)

    def reduced_rhs(self, b):
        _, _, B_GI, _ = self.blocks()
        w = self.interior_lu().solve(b[:self.NI])
        return b[self.NI:] - B_GI @ w

    def back_substitute(self, b, xG):
        _, B_IG, _, _ = self.blocks()
        return self.interior_lu().solve(b[:self.NI] / self.K - B_IG @ xG)

    def schur_pcg(self, b, precond=None, rtol=1e-10, maxit=500):
        """PCG on S x_G = g from 0, stopping when (r^T z)^{1/2} has fallen by rtol (Sec. 3)."""
        if precond is None:
            Pm = self.exact_precond()
            precond = lambda r: Pm @ r
        g = self.reduced_rhs(b)
        xG = np.zeros_like(g)
        r = g.copy()
        z = precond(r)
        rz = rz0 = r @ z
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
        return np.concatenate([self.back_substitute(b, xG), xG]), its


def ra_operator(L, M, t, table):
    """The rational realization of L^t (eq. (RA) form) for a table (d0, d_k, q_k):
      t < 0:  table approximates lambda^t:      L^t ~ M (d0 M^{-1} + sum d_k (L + q_k M)^{-1}) M
      t >= 0: table approximates lambda^(t-1):  lambda^t ~ d0 lambda + sum d_k lambda/(lambda+q_k)
              = d0 lambda + sum d_k - sum d_k q_k / (lambda + q_k), so
              L^t ~ d0 L + (sum d_k) M - sum d_k q_k M (L + q_k M)^{-1} M."""
    d0, d, q = table
    if t < 0:
        out = d0 * M
        for dk, qk in zip(d, q):
            out = out + dk * M @ np.linalg.solve(L + qk * M, M)
        return out
    out = d0 * L + float(np.sum(d)) * M
    for dk, qk in zip(d, q):
        out = out - dk * qk * M @ np.linalg.solve(L + qk * M, M)
    return out
