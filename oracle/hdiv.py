"""The H(div) variant of the interface-perturbed problem (Sec. 3, remark on H(div)-elliptic
problems, eq. (graddiv)), 2D (oracle; test infrastructure only).

Find u in V = H(div, Omega), Omega = (0, 1)^2, with

    K int_Omega (u.v + div u div v) + gamma int_{dOmega} (u.nu)(v.nu) = <b, v>   for all v in V,

discretized by lowest-order Brezzi-Douglas-Marini elements (BDM1: piecewise linear vector fields
with continuous normal components) on the diagonal-split mesh of n cells per side.  Gamma is the
whole boundary; V_0 = BDM1 with zero normal trace; the trace space Q_h is the discontinuous P1
space on the 4n boundary segments (the normal traces of BDM1).

Degrees of freedom: two per edge, the normal component u.n_e at the edge's first and at its second
endpoint.  Edge order (interior edges first, then the boundary loop):
  horizontal (i, j) -> (i+1, j), j = 1..n-1, i = 0..n-1,   n_e = (0, 1),  index (j-1) n + i
  vertical   (i, j) -> (i, j+1), i = 1..n-1, j = 0..n-1,   n_e = (1, 0),  n(n-1) + j(n-1) + i-1
  diagonal   (i, j) -> (i+1, j+1), i, j = 0..n-1,          n_e = (1, -1)/sqrt 2, 2n(n-1) + j n + i
  boundary segment k of the counter-clockwise loop from (0, 0) (bottom, right, top, left; first
  endpoint = the one met first), n_e = outward normal nu, index 3n^2 - 2n + k.
Edge e holds dofs 2e (first endpoint) and 2e + 1 (second).  So the last 8n dofs are the DG P1
trace values of u.nu, segment by segment along the loop.

Basis: on a triangle T with edge e = (p, q), psi_{e,p} = lambda_p w_q with the constant field
w_q = curl lambda_q / (curl lambda_q . n_e), curl phi = (d_y phi, -d_x phi); curl lambda_q is
parallel to the edge opposite q, so psi_{e,p} has no normal component on the other two edges,
and on e its normal component is lambda_p (1 at p, 0 at q).  Likewise psi_{e,q} = lambda_q w_p.
The element matrices follow: int psi_a . psi_b = (w_a . w_b) |T| (1 + delta) / 12 (delta: same
vertex), div psi_a = grad lambda_{v_a} . w_a.

Domain decomposition (eq. (dd_preconditioner)): A^00 = K(I - grad div) on V_0, S the Schur
complement of the assembled matrix onto the trace dofs, preconditioned by
S_Gamma = K L^{-1/2} + gamma I_Gamma (the remark), I_Gamma = M_Q the DG P1 mass on the loop and
L^{-1/2} from eq. (gevp) with L the matrix of -Delta_Gamma + I on Q_h.

Reading (the paper does not say how -Delta_Gamma acts on the discontinuous space): L is the
symmetric interior-penalty discretization of -u'' + u on the closed loop of 4n segments of length
h, penalty sigma / h on the jumps at the 4n loop vertices, sigma = 4:
  l(u, v) = sum_e int_e (u'v' + uv) - sum_vertices ({u'}[v] + {v'}[u]) + (sigma / h) sum [u][v],
with [u] = u(end of the segment before the vertex) - u(start of the one after) and {u'} the mean
of the two segments' derivatives along the loop.  Both L and M_Q are block circulant (2 x 2
blocks, one per segment), so their generalized spectrum has a closed form per Fourier mode.

Parity: pinned by the dual-basis property of the BDM1 fields (evaluated pointwise), exactness on
linear vector fields (mass, divergence and boundary terms against closed-form integrals), the
divergence theorem per triangle, nestedness (the Galerkin product of the inclusion reproduces the
coarse matrices, and linear fields are carried over exactly), second-order convergence to a manufactured solution, the closed
form of the loop spectrum, consistency of L on smooth periodic functions, the Schur complement
identity, bounded condition numbers of S_Gamma^{-1} S over h and gamma, and the agreement of the
dense and the Fourier-mode application of the preconditioner
(tests/test_oracle_hdiv.py).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import spectral
from .fem import mesh_2d

SIGMA = 4.0


def _curl_of_grad(g):
    """curl lambda = (d_y lambda, -d_x lambda) from grad lambda = (d_x, d_y)."""
    return np.array([g[1], -g[0]])


def edges(n):
    """(first endpoint, second endpoint, normal) of every edge, in edge order; endpoints as grid
    coordinates (i, j)."""
    out = []
    for j in range(1, n):
        for i in range(n):
            out.append(((i, j), (i + 1, j), (0.0, 1.0)))
    for j in range(n):
        for i in range(1, n):
            out.append(((i, j), (i, j + 1), (1.0, 0.0)))
    s = 1.0 / np.sqrt(2.0)
    for j in range(n):
        for i in range(n):
            out.append(((i, j), (i + 1, j + 1), (s, -s)))
    out.extend(loop_edges(n))
    return out


def loop_edges(n):
    """The boundary segments in loop order with their outward normals."""
    out = [((i, 0), (i + 1, 0), (0.0, -1.0)) for i in range(n)]
    out += [((n, j), (n, j + 1), (1.0, 0.0)) for j in range(n)]
    out += [((n - i, n), (n - i - 1, n), (0.0, 1.0)) for i in range(n)]
    out += [((0, n - j), (0, n - j - 1), (-1.0, 0.0)) for j in range(n)]
    return out


def sizes(n):
    """(N, N_0, N_Gamma)."""
    n0 = 2 * (3 * n * n - 2 * n)
    return n0 + 8 * n, n0, 8 * n


class Basis:
    """The BDM1 fields of one triangle: for each local dof (edge e, its vertex v) the vertex v and
    the constant field w, so that psi = lambda_v w."""

    def __init__(self, coords, local):
        # coords (3, 2); local: list of (global dof, vertex position 0..2, other vertex, normal)
        B = (coords[1:] - coords[0]).T
        Binv = np.linalg.inv(B)
        self.grads = np.vstack([-Binv.sum(axis=0), Binv])
        self.area = abs(np.linalg.det(B)) / 2.0
        self.coords = coords
        self.dofs, self.vert, self.w = [], [], []
        for dof, v, other, nrm in local:
            c = _curl_of_grad(self.grads[other])
            self.dofs.append(dof)
            self.vert.append(v)
            self.w.append(c / float(c @ np.asarray(nrm)))
        self.w = np.array(self.w)

    def bary(self, x):
        """Barycentric coordinates of the point x."""
        lam1 = np.linalg.solve((self.coords[1:] - self.coords[0]).T, np.asarray(x) - self.coords[0])
        return np.concatenate([[1.0 - lam1.sum()], lam1])

    def eval(self, x):
        """(6, 2): the value of every local field at the point x."""
        lam = self.bary(x)
        return np.array([lam[v] * w for v, w in zip(self.vert, self.w)])

    def div(self):
        return np.array([self.grads[v] @ w for v, w in zip(self.vert, self.w)])

    def mass(self):
        k = len(self.vert)
        out = np.empty((k, k))
        for a in range(k):
            for b in range(k):
                same = 1.0 if self.vert[a] == self.vert[b] else 0.0
                out[a, b] = (self.w[a] @ self.w[b]) * self.area * (1.0 + same) / 12.0
        return out


def triangle_bases(n):
    """The Basis of every triangle of the mesh (same triangles as fem.mesh_2d)."""
    nodes, tris = mesh_2d(n)
    where = {}
    for e, (p, q, nrm) in enumerate(edges(n)):
        where[(p, q)] = (e, nrm, p)
        where[(q, p)] = (e, nrm, p)
    out = []
    for t in tris:
        ij = [(int(round(nodes[v, 0] * n)), int(round(nodes[v, 1] * n))) for v in t]
        local = []
        for a in range(3):
            for b in range(3):
                if a == b:
                    continue
                e, nrm, p = where[(ij[a], ij[b])]
                # dof of vertex a on edge (a, b): 2e if a is the edge's first endpoint
                dof = 2 * e + (0 if ij[a] == p else 1)
                local.append((dof, a, b, nrm))
        out.append(Basis(nodes[t], local))
    return out


def assemble(n):
    """Mass and div-div matrices of BDM1 (all dofs) and the boundary matrix of
    int (u.nu)(v.nu) (nonzero on the trace dofs only), sparse CSR."""
    N = sizes(n)[0]
    rows, cols, mv, dv = [], [], [], []
    for T in triangle_bases(n):
        d = np.array(T.dofs)
        k = len(d)
        rows.append(np.repeat(d, k))
        cols.append(np.tile(d, k))
        mv.append(T.mass().ravel())
        dd = T.div()
        dv.append((T.area * np.outer(dd, dd)).ravel())
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    Mass = sp.coo_matrix((np.concatenate(mv), (r, c)), shape=(N, N)).tocsr()
    Div = sp.coo_matrix((np.concatenate(dv), (r, c)), shape=(N, N)).tocsr()
    Bd = sp.lil_matrix((N, N))
    n0 = sizes(n)[1]
    h = 1.0 / n
    for k in range(4 * n):
        a, b = n0 + 2 * k, n0 + 2 * k + 1
        Bd[a, a] += 2 * h / 6
        Bd[b, b] += 2 * h / 6
        Bd[a, b] += h / 6
        Bd[b, a] += h / 6
    return Mass, Div, Bd.tocsr()


def prolongation(nc):
    """The natural inclusion of BDM1 on n_c cells per side into BDM1 on 2 n_c (the meshes are
    nested): each fine dof "u.n_e at an endpoint" of a coarse field is its value there, taken in
    the coarse triangle that holds the fine edge, times the fine edge's normal.  All dofs."""
    nf = 2 * nc
    coarse = triangle_bases(nc)
    rows, cols, vals = [], [], []
    for e, (p, q, nrm) in enumerate(edges(nf)):
        mid = (np.array(p) + np.array(q)) / 2.0 / nf
        xc = mid * nc
        ci = min(int(np.floor(xc[0])), nc - 1)
        cj = min(int(np.floor(xc[1])), nc - 1)
        t = 2 * (cj * nc + ci) + (0 if xc[0] - ci >= xc[1] - cj else 1)
        T = coarse[t]
        for k, pt in enumerate((p, q)):
            v = T.eval(np.array(pt) / nf) @ np.array(nrm)
            for d, val in zip(T.dofs, v):
                if abs(val) > 1e-14:
                    rows.append(2 * e + k)
                    cols.append(d)
                    vals.append(val)
    return sp.coo_matrix((vals, (rows, cols)), shape=(sizes(nf)[0], sizes(nc)[0])).tocsr()


# ----------------------------------------------------------------------------
# the trace space Q_h (DG P1 on the loop)
# ----------------------------------------------------------------------------

def loop_mass(n):
    """M_Q: per segment (h/6)[[2, 1], [1, 2]]."""
    h = 1.0 / n
    m = 4 * n
    M = np.zeros((2 * m, 2 * m))
    for k in range(m):
        M[2 * k:2 * k + 2, 2 * k:2 * k + 2] = (h / 6) * np.array([[2.0, 1.0], [1.0, 2.0]])
    return M


def loop_sipg(n, sigma=SIGMA):
    """L: symmetric interior penalty form of -u'' + u on the closed loop of 4n segments.
    Segment k carries (u at its start, u at its end) = dofs (2k, 2k+1); its derivative along the
    loop is (u_end - u_start) / h."""
    h = 1.0 / n
    m = 4 * n
    L = loop_mass(n)
    for k in range(m):
        s = slice(2 * k, 2 * k + 2)
        L[s, s] += (1.0 / h) * np.array([[1.0, -1.0], [-1.0, 1.0]])
    for k in range(m):
        # the vertex between segment a = k - 1 (its end) and segment b = k (its start)
        a, b = (k - 1) % m, k
        jump = np.zeros(2 * m)
        jump[2 * a + 1] += 1.0
        jump[2 * b] -= 1.0
        dmean = np.zeros(2 * m)
        dmean[2 * a] -= 0.5 / h
        dmean[2 * a + 1] += 0.5 / h
        dmean[2 * b] -= 0.5 / h
        dmean[2 * b + 1] += 0.5 / h
        L -= np.outer(dmean, jump) + np.outer(jump, dmean)
        L += (sigma / h) * np.outer(jump, jump)
    return L


def loop_eigs(n, sigma=SIGMA):
    """Closed form of the spectrum of (L, M_Q): both are block circulant with 2 x 2 blocks, so
    for theta = 2 pi q / (4n) the eigenvalues are those of the 2 x 2 pencil of their symbols
    D + C_prev e^{-i theta} + C_next e^{i theta}."""
    h = 1.0 / n
    m = 4 * n
    Ms = (h / 6) * np.array([[2.0, 1.0], [1.0, 2.0]])
    # blocks of row segment k: own (D), coupling to segment k-1 (P) and to k+1 (Q = P^T)
    D = Ms + (1.0 / h) * np.array([[1.0, -1.0], [-1.0, 1.0]])
    # vertex at the start of k (segment a = k-1 end, b = k start) and at its end (k end, k+1 start)
    # jump j = u_a,end - u_b,start ; derivative mean d = (u_a,end - u_a,start + u_b,end - u_b,start)/(2h)
    # contributions -(d j + j d) + (sigma/h) j j, split into blocks
    ja = np.array([0.0, 1.0])    # segment a's coefficients in j
    jb = np.array([-1.0, 0.0])   # segment b's
    da = np.array([-0.5, 0.5]) / h
    db = np.array([-0.5, 0.5]) / h
    def vert(x, y):
        return -(np.outer(x[0], y[1]) + np.outer(x[1], y[0])) + (sigma / h) * np.outer(x[1], y[1])
    # x = (d coefficients, j coefficients) of the row segment, y of the column segment
    Daa = vert((da, ja), (da, ja))   # segment k as the "a" of its end vertex
    Dbb = vert((db, jb), (db, jb))   # segment k as the "b" of its start vertex
    Pba = vert((db, jb), (da, ja))   # row k (as b), column k-1 (as a)
    Dtot = D + Daa + Dbb
    out = []
    for q in range(m):
        th = 2 * np.pi * q / m
        S = Dtot + Pba * np.exp(-1j * th) + Pba.T * np.exp(1j * th)
        out.extend(sla.eigvalsh(S, Ms.astype(complex)))
    return np.sort(np.real(np.array(out)))


class HdivProblem:
    """One instance (n, K, gamma) of eq. (graddiv) in BDM1."""

    def __init__(self, n, K, gamma, sigma=SIGMA):
        if K <= 0 or gamma < 0:
            raise ValueError("need K > 0, gamma >= 0")
        self.n, self.K, self.gamma = n, float(K), float(gamma)
        self.N, self.N0, self.NG = sizes(n)
        self.Mass, self.Div, self.Bd = assemble(n)
        self.A = (self.K * (self.Mass + self.Div) + self.gamma * self.Bd).tocsr()
        self.L = loop_sipg(n, sigma)
        self.M_Q = loop_mass(n)
        self.eig = spectral.gevp(self.L, self.M_Q)

    # -- operator ----------------------------------------------------------------
    def apply(self, x):
        return self.A @ x

    def solve_splu(self, b):
        return spla.splu(self.A.tocsc()).solve(b)

    def solve_dense(self, b):
        return sla.cho_solve(sla.cho_factor(self.A.toarray()), b)

    # -- domain decomposition -----------------------------------------------------
    def blocks(self):
        n0 = self.N0
        A = self.A
        return (A[:n0, :n0].tocsc(), A[:n0, n0:].tocsc(), A[n0:, :n0].tocsc(), A[n0:, n0:].toarray())

    def interior_lu(self):
        if not hasattr(self, "_lu"):
            self._lu = spla.splu(self.blocks()[0])
        return self._lu

    def schur_dense(self):
        A00, A0G, AG0, AGG = self.blocks()
        return AGG - AG0 @ self.interior_lu().solve(A0G.toarray())

    def schur_apply(self, p):
        _, A0G, AG0, AGG = self.blocks()
        return AGG @ p - AG0 @ self.interior_lu().solve(A0G @ p)

    def f_precond(self):
        """f(lambda) = 1 / (K lambda^{-1/2} + gamma): the symbol of S_Gamma^{-1}."""
        K, g = self.K, self.gamma
        return lambda lam: 1.0 / (K / np.sqrt(lam) + g)

    def g_table_function(self):
        """f(lambda) / lambda = 1 / (K lambda^{1/2} + gamma lambda): decreasing, the function whose
        rational table realizes the preconditioner (f_RA = lambda g_RA)."""
        K, g = self.K, self.gamma
        return lambda lam: 1.0 / (K * np.sqrt(lam) + g * lam)

    def schur_precond(self):
        """S_Gamma = K L^{-1/2} + gamma M_Q."""
        return self.K * spectral.frac_power(self.L, self.M_Q, -0.5, self.eig) + self.gamma * self.M_Q

    def exact_precond(self):
        return spectral.spectral_function(self.L, self.M_Q, self.f_precond(), self.eig)

    def reduced_rhs(self, b):
        _, _, AG0, _ = self.blocks()
        return b[self.N0:] - AG0 @ self.interior_lu().solve(b[:self.N0])

    def back_substitute(self, b, xG):
        _, A0G, _, _ = self.blocks()
        return self.interior_lu().solve(b[:self.N0] - A0G @ xG)

    def schur_pcg(self, b, precond=None, rtol=1e-10, maxit=500):
        """PCG on S x_G = g from 0, stopping when (r^T z)^{1/2} has fallen by rtol."""
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


def ra_precond(L, M, table):
    """The preconditioner from a table (d0, d_k, q_k) of g(lambda) = f(lambda) / lambda:
    f_RA(lambda) = lambda g_RA(lambda) = d0 lambda + sum d_k - sum d_k q_k / (lambda + q_k), so
    S_Gamma^{-1} ~ d0 M^{-1} L M^{-1} + (sum d_k) M^{-1} - sum d_k q_k (L + q_k M)^{-1}."""
    d0, d, q = table
    Minv = np.linalg.inv(M)
    out = d0 * Minv @ L @ Minv + float(np.sum(d)) * Minv
    for dk, qk in zip(d, q):
        out = out - dk * qk * np.linalg.inv(L + qk * M)
    return out


def loop_symbols(n, sigma=SIGMA):
    """The 2 x 2 blocks of L on the loop (own segment, previous segment; the next one is the
    transpose) and of M_Q, as the closed-form spectrum uses them."""
    h = 1.0 / n
    Ms = (h / 6) * np.array([[2.0, 1.0], [1.0, 2.0]])
    own = Ms + (1.0 / h) * np.array([[1.0, -1.0], [-1.0, 1.0]])
    ja, jb = np.array([0.0, 1.0]), np.array([-1.0, 0.0])
    da = db = np.array([-0.5, 0.5]) / h

    def vert(dr, jr, dc, jc):
        return -(np.outer(dr, jc) + np.outer(jr, dc)) + (sigma / h) * np.outer(jr, jc)
    own = own + vert(db, jb, db, jb) + vert(da, ja, da, ja)
    prev = vert(db, jb, da, ja)
    return own, prev, Ms


def ra_precond_apply_fft(n, table, r, sigma=SIGMA):
    """The preconditioner of ra_precond applied to r by the discrete Fourier transform over the 4n
    loop segments (L and M_Q are block circulant): per mode theta the 2 x 2 symbol
    S = own + prev e^{-i theta} + prev^T e^{i theta}, and
    z_hat = (d0 Ms^-1 S Ms^-1 + (sum d) Ms^-1 - sum d_k q_k (S + q_k Ms)^-1) r_hat."""
    d0, d, q = table
    m = 4 * n
    own, prev, Ms = loop_symbols(n, sigma)
    th = 2.0 * np.pi * np.arange(m) / m
    S = (own[None] + prev[None] * np.exp(-1j * th)[:, None, None]
         + prev.T[None] * np.exp(1j * th)[:, None, None])
    Msi = np.linalg.inv(Ms)
    R = np.fft.fft(np.asarray(r, dtype=float).reshape(m, 2), axis=0)
    op = d0 * (Msi[None] @ S @ Msi[None]) + float(np.sum(d)) * Msi[None]
    for dk, qk in zip(d, q):
        op = op - dk * qk * np.linalg.inv(S + qk * Ms[None])
    Z = np.einsum("qab,qb->qa", op, R)
    return np.fft.ifft(Z, axis=0).real.reshape(-1)

