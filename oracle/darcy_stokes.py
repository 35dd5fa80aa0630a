"""The coupled Darcy-Stokes problem and its block-diagonal preconditioner (Sec. 4, eq.
(darcy_stokes), eq. (darcy_stokes_precond); Appendix), 2D (oracle; test infrastructure only).

Geometry (reading: the paper's domain is drawn only in a figure, with a curved interface; here
the interface is straight so the Darcy part is the facet problem of eq. (riesz)):
  Omega_D = (0, 1)^2 (Darcy),  Omega_S = (0, 1) x (1, 2) (Stokes),  Gamma = (0, 1) x {1},
  nu = (0, -1) the unit normal on Gamma pointing out of Omega_S.
Boundary conditions: no slip (u = 0) on the Stokes sides x = 0 and x = 1, zero traction on the
Stokes top y = 2, Darcy pressure zero on the rest of the Darcy boundary.

Equations (reading of sigma: sigma(u, p) = mu grad u - p I): find u (Stokes velocity), p_S
(Stokes pressure), p_D (Darcy pressure) with
  -div sigma = f_S, div u = g in Omega_S;   -div(K grad p_D) = f_D in Omega_D;
  on Gamma: u.nu + K grad p_D . nu = 0,  -nu.sigma nu - p_D = 0,
            -P_nu(sigma nu) - alpha mu K^{-1/2} P_nu u = 0   (Beavers-Joseph-Saffman).
Weak form (symmetric; the Darcy equation is multiplied by -1):
  a(u, v) + b(v, p_S) + c(v, p_D) = (f_S, v)
  b(u, q_S)                       = -(g, q_S)
  c(u, q_D) - d(p_D, q_D)         = -(f_D, q_D)
with a(u, v) = mu int grad u : grad v + alpha mu K^{-1/2} int_Gamma u_x v_x,
b(v, q) = -int q div v, c(v, q) = int_Gamma q v.nu = -int_Gamma q v_y, d(p, q) = K int grad p .
grad q.

Discretization (reading: the paper uses P2-P1-P2; the Darcy pressure here is P1 so that its
preconditioner block is the P1 facet problem of eq. (riesz) itself): Taylor-Hood P2-P1 on the
Stokes mesh, P1 for p_D on the Darcy mesh; both meshes are the diagonal-split mesh of n cells per
side (fem.mesh_2d, the Stokes one shifted up by one), so they match on Gamma.

Unknowns, in this order:
  u_x, u_y   P2 nodes (A h/2, 1 + B h/2), A = 1..2n-1 (x = 0 and 1 are no-slip), B = 0..2n,
             index c NV + B (2n - 1) + (A - 1), NV = (2n - 1)(2n + 1), c = 0 (x), 1 (y);
  p_S        P1 vertices (i h, 1 + j h), i, j = 0..n, index Nu + j (n + 1) + i;
  p_D        the facet problem's free dofs (fem.free_dofs, Gamma last), index Nu + Np + k.

Preconditioner (eq. (darcy_stokes_precond)):
  B = diag(A_u, mu^{-1} M_p, K A_D + mu^{-1} T^T H T)^{-1},
A_u the matrix of a(., .), M_p the P1 pressure mass, and the last block the Riesz map of eq.
(riesz) with gamma = 1/mu (system.Riesz).  Its blocks are applied exactly (sparse LU), as in the
Appendix, or the Darcy block by PCG with the preconditioner of eq. (dd_preconditioner) to a
relative tolerance (the Appendix: 1e-5; Sec. 4: 1e-4).

Outer solver: flexible GMRES (Saad), right preconditioned, x_0 = 0, no restart; the iteration
stops when the least-squares residual ||b - A x_k||_2 has fallen below rtol ||b||_2 (reading of
the paper's "relative tolerance on the residual norm": the norm that FGMRES minimizes).

Element matrices by quadrature (Stroud conical product rule from Gauss-Legendre points, exact for
the polynomial degrees assembled here), basis in barycentric coordinates: vertex functions
lambda_i (2 lambda_i - 1), edge functions 4 lambda_i lambda_j.

Parity: pinned by exactness of every block on polynomial fields (against tensor Gauss integrals
over the rectangle and the interface), the Stokes inf-sup constant bounded below in h, convergence
to a manufactured solution that satisfies all interface conditions, and the FGMRES invariants
(equality of its least-squares residual with the true residual, one step with the exact inverse
as preconditioner, termination in k steps for k distinct eigenvalues) (tests/test_oracle_ds.py).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem
from .system import Riesz, lazy_full_pcg


# ----------------------------------------------------------------------------
# quadrature and the P2 basis
# ----------------------------------------------------------------------------

def triangle_rule(k):
    """Stroud conical product rule with k x k points on the reference triangle: barycentric
    points (m, 3) and weights summing to 1 (fractions of the area); exact to degree 2k - 2."""
    g, w = np.polynomial.legendre.leggauss(k)
    t, wt = (g + 1) / 2, w / 2
    pts, wts = [], []
    for a, wa in zip(t, wt):
        for b, wb in zip(t, wt):
            x, y = a, b * (1 - a)           # Duffy map of the unit square
            pts.append((1 - x - y, x, y))
            wts.append(wa * wb * (1 - a) * 2)
    return np.array(pts), np.array(wts)


def segment_rule(k):
    """Gauss-Legendre on [0, 1]: points and weights (summing to 1)."""
    g, w = np.polynomial.legendre.leggauss(k)
    return (g + 1) / 2, w / 2


def p2_values(L):
    """The six P2 basis values at barycentric point L (vertices 0, 1, 2, then the midpoints of
    edges 01, 12, 02)."""
    l0, l1, l2 = L
    return np.array([l0 * (2 * l0 - 1), l1 * (2 * l1 - 1), l2 * (2 * l2 - 1),
                     4 * l0 * l1, 4 * l1 * l2, 4 * l0 * l2])


def p2_gradients(L, G):
    """Gradients (6, 2) of the P2 basis at L; G (3, 2) holds the barycentric gradients."""
    l0, l1, l2 = L
    return np.array([(4 * l0 - 1) * G[0], (4 * l1 - 1) * G[1], (4 * l2 - 1) * G[2],
                     4 * (l0 * G[1] + l1 * G[0]), 4 * (l1 * G[2] + l2 * G[1]),
                     4 * (l0 * G[2] + l2 * G[0])])


def barycentric_gradients(X):
    B = np.array([X[1] - X[0], X[2] - X[0]]).T
    Binv = np.linalg.inv(B)
    G = np.vstack([-Binv.sum(axis=0), Binv])
    return G, abs(np.linalg.det(B)) / 2


# ----------------------------------------------------------------------------
# meshes and numbering
# ----------------------------------------------------------------------------

def sizes(n):
    """(Nu, Np, ND, N): velocity, Stokes pressure, Darcy pressure, total."""
    nv = (2 * n - 1) * (2 * n + 1)
    nd = fem.sizes(2, n)[0]
    return 2 * nv, (n + 1) ** 2, nd, 2 * nv + (n + 1) ** 2 + nd


def stokes_mesh(n):
    """Vertices (i h, 1 + j h) numbered j (n + 1) + i and the triangles of fem.mesh_2d."""
    nodes, tris = fem.mesh_2d(n)
    return nodes + np.array([0.0, 1.0]), tris


def p2_node(n, vi):
    """Half-grid coordinates (A, B) of the six P2 nodes of a triangle with vertex numbers vi."""
    ij = [(v % (n + 1), v // (n + 1)) for v in vi]
    pts = [(2 * i, 2 * j) for i, j in ij]
    for a, b in ((0, 1), (1, 2), (0, 2)):
        pts.append((ij[a][0] + ij[b][0], ij[a][1] + ij[b][1]))
    return pts


def vel_index(n, c, A, B):
    """Velocity unknown of component c at half-grid node (A, B), or -1 on the no-slip sides."""
    if A <= 0 or A >= 2 * n:
        return -1
    return c * (2 * n - 1) * (2 * n + 1) + B * (2 * n - 1) + (A - 1)


# ----------------------------------------------------------------------------
# the problem
# ----------------------------------------------------------------------------

class DarcyStokes:
    """Assembled matrices of one (n, K, mu, alpha) instance (all sparse CSR)."""

    def __init__(self, n, K, mu, alpha=0.0, qk=4):
        if n < 2 or K <= 0 or mu <= 0 or alpha < 0:
            raise ValueError("need n >= 2, K > 0, mu > 0, alpha >= 0")
        self.n, self.K, self.mu, self.alpha = n, float(K), float(mu), float(alpha)
        self.Nu, self.Np, self.ND, self.N = sizes(n)
        self.NV = self.Nu // 2
        self._assemble(qk)

    def _assemble(self, qk):
        n, mu, K = self.n, self.mu, self.K
        nodes, tris = stokes_mesh(n)
        pts, wts = triangle_rule(qk)
        au_r, au_c, au_v = [], [], []
        mp_r, mp_c, mp_v = [], [], []
        b_r, b_c, b_v = [], [], []
        for tri in tris:
            X = nodes[tri]
            G, area = barycentric_gradients(X)
            loc = p2_node(n, tri)
            S = np.zeros((6, 6))
            M1 = np.zeros((3, 3))
            D = np.zeros((3, 6, 2))      # int lambda_k d_c phi_a
            for L, w in zip(pts, wts):
                dphi = p2_gradients(L, G)
                S += w * area * dphi @ dphi.T
                M1 += w * area * np.outer(L, L)
                D += w * area * L[:, None, None] * dphi[None, :, :]
            for c in range(2):
                gi = [vel_index(n, c, A, B) for A, B in loc]
                for a in range(6):
                    if gi[a] < 0:
                        continue
                    for b in range(6):
                        if gi[b] >= 0:
                            au_r.append(gi[a]); au_c.append(gi[b]); au_v.append(mu * S[a, b])
                    for k in range(3):
                        b_r.append(tri[k]); b_c.append(gi[a]); b_v.append(-D[k, a, c])
            for a in range(3):
                for b in range(3):
                    mp_r.append(tri[a]); mp_c.append(tri[b]); mp_v.append(M1[a, b])
        # interface terms, segment k from (k h, 1) to ((k + 1) h, 1): P2 nodes A = 2k, 2k+1, 2k+2
        h = 1.0 / n
        sp_, sw = segment_rule(4)
        bjs = self.alpha * mu / np.sqrt(K)
        c_r, c_c, c_v = [], [], []
        for k in range(n):
            for t, w in zip(sp_, sw):
                phi = np.array([(1 - t) * (1 - 2 * t), 4 * t * (1 - t), t * (2 * t - 1)])
                hat = np.array([1 - t, t])
                for a in range(3):
                    ia = vel_index(n, 0, 2 * k + a, 0)
                    if ia >= 0 and bjs > 0:
                        for b in range(3):
                            ib = vel_index(n, 0, 2 * k + b, 0)
                            if ib >= 0:
                                au_r.append(ia); au_c.append(ib)
                                au_v.append(w * h * bjs * phi[a] * phi[b])
                    iy = vel_index(n, 1, 2 * k + a, 0)
                    if iy < 0:
                        continue
                    for e in range(2):
                        i = k + e                      # Darcy interface node i (1..n-1 free)
                        if 1 <= i <= n - 1:
                            c_r.append(iy); c_c.append(self.darcy_gamma_index(i))
                            c_v.append(-w * h * hat[e] * phi[a])
        Nu, Np, ND = self.Nu, self.Np, self.ND
        self.A_u = sp.coo_matrix((au_v, (au_r, au_c)), shape=(Nu, Nu)).tocsr()
        self.B = sp.coo_matrix((b_v, (b_r, b_c)), shape=(Np, Nu)).tocsr()
        self.M_p = sp.coo_matrix((mp_v, (mp_r, mp_c)), shape=(Np, Np)).tocsr()
        self.C = sp.coo_matrix((c_v, (c_r, c_c)), shape=(Nu, ND)).tocsr()
        self.darcy = fem.Problem(2, n)
        self.A_D = (K * self.darcy.A).tocsr()
        for M in (self.A_u, self.B, self.M_p, self.C):
            M.sum_duplicates()
        self.A = sp.bmat([[self.A_u, self.B.T, self.C],
                          [self.B, None, None],
                          [self.C.T, None, -self.A_D]], format="csr")

    def darcy_gamma_index(self, i):
        """Darcy unknown (within p_D) of the interface node (i h, 1), i = 1..n-1."""
        return fem.sizes(2, self.n)[1] + (i - 1)

    # -- blocks of the preconditioner ------------------------------------------------------
    def riesz(self):
        if not hasattr(self, "_riesz"):
            self._riesz = Riesz(2, self.n, self.K, self.mu, prob=self.darcy)
        return self._riesz

    def precond_exact(self):
        """r -> B r with every block inverted exactly (sparse LU; the Darcy block by the sparse
        LU of K A_Omega plus the dense Gamma block, system.Riesz.solve_splu)."""
        lu_u = spla.splu(self.A_u.tocsc())
        lu_p = spla.splu(self.M_p.tocsc())
        R = self.riesz()
        Nu, Np = self.Nu, self.Np

        def apply(r):
            return np.concatenate([lu_u.solve(r[:Nu]), self.mu * lu_p.solve(r[Nu:Nu + Np]),
                                   R.solve_splu(r[Nu + Np:])])
        return apply

    def precond_lazy(self, tabP, tabH, darcy_rtol=1e-5, nu=2):
        """r -> B r with exact Stokes blocks and the Darcy block by PCG on the Riesz system with
        the lazy preconditioner of eq. (dd_preconditioner) (one multigrid V-cycle for the leading
        block, RA for S_Gamma, H by RA in the operator: system.lazy_full_pcg) to darcy_rtol.
        Returns (apply, the list of inner PCG counts it fills)."""
        lu_u = spla.splu(self.A_u.tocsc())
        lu_p = spla.splu(self.M_p.tocsc())
        R = self.riesz()
        Nu, Np = self.Nu, self.Np
        counts = []

        def apply(r):
            zD, its, _ = lazy_full_pcg(R, r[Nu + Np:], tabP, tabH, nu=nu, rtol=darcy_rtol)
            counts.append(its)
            return np.concatenate([lu_u.solve(r[:Nu]), self.mu * lu_p.solve(r[Nu:Nu + Np]), zD])
        return apply, counts

    def solve_splu(self, b):
        return spla.spsolve(self.A.tocsc(), b)

    # -- manufactured solution ---------------------------------------------------------------
    def manufactured(self, beta=1.0):
        """A smooth solution satisfying every interface and boundary condition, with its data:
        s = x(1 - x), u = (s a(y), s b(y)), p_S = s pi(y), p_D = s y, where
        a = 1 + c1 (y - 1) - (c1 / 2)(y - 1)^2, c1 = alpha K^{-1/2} (BJS at y = 1, zero shear at
        y = 2), b = -K + beta (y - 1)^2 (normal flux continuity), pi = 1 + (2 mu beta - 1)(y - 1)
        (normal stress balance at y = 1, zero normal traction at y = 2).
        Returns (exact functions, data functions) as dicts of callables (x, y)."""
        K, mu, al = self.K, self.mu, self.alpha
        c1 = al / np.sqrt(K)

        def s(x): return x * (1 - x)
        def a(y): return 1 + c1 * (y - 1) - 0.5 * c1 * (y - 1) ** 2
        def bfun(y): return -K + beta * (y - 1) ** 2
        def pi(y): return 1 + (2 * mu * beta - 1) * (y - 1)
        exact = {
            "ux": lambda x, y: s(x) * a(y),
            "uy": lambda x, y: s(x) * bfun(y),
            "pS": lambda x, y: s(x) * pi(y),
            "pD": lambda x, y: s(x) * y,
        }
        # -mu Lap u + grad p_S,  div u,  -K Lap p_D
        data = {
            "fx": lambda x, y: -mu * (-2 * a(y) + s(x) * (-c1)) + (1 - 2 * x) * pi(y),
            "fy": lambda x, y: -mu * (-2 * bfun(y) + s(x) * 2 * beta) + s(x) * (2 * mu * beta - 1),
            "g": lambda x, y: (1 - 2 * x) * a(y) + s(x) * 2 * beta * (y - 1),
            "fD": lambda x, y: 2 * K * y,
        }
        return exact, data

    def load(self, data, qk=6):
        """The right-hand side [(f_S, v); -(g, q_S); -(f_D, q_D)] by quadrature."""
        n = self.n
        F = np.zeros(self.N)
        pts, wts = triangle_rule(qk)
        nodes, tris = stokes_mesh(n)
        for tri in tris:
            X = nodes[tri]
            _, area = barycentric_gradients(X)
            loc = p2_node(n, tri)
            for L, w in zip(pts, wts):
                x, y = L @ X
                phi = p2_values(L)
                fx, fy, g = data["fx"](x, y), data["fy"](x, y), data["g"](x, y)
                for a in range(6):
                    for c, f in ((0, fx), (1, fy)):
                        gi = vel_index(n, c, *loc[a])
                        if gi >= 0:
                            F[gi] += w * area * f * phi[a]
                for k in range(3):
                    F[self.Nu + tri[k]] -= w * area * g * L[k]
        dn, dt = fem.mesh_2d(n)
        fd = fem.free_dofs(2, n)
        pos = -np.ones(dn.shape[0], dtype=np.int64)
        pos[fd] = np.arange(fd.size)
        off = self.Nu + self.Np
        for tri in dt:
            X = dn[tri]
            _, area = barycentric_gradients(X)
            for L, w in zip(pts, wts):
                x, y = L @ X
                f = data["fD"](x, y)
                for k in range(3):
                    if pos[tri[k]] >= 0:
                        F[off + pos[tri[k]]] -= w * area * f * L[k]
        return F

    def interpolate(self, exact):
        """The exact solution at the unknowns' nodes."""
        n, h = self.n, 1.0 / self.n
        out = np.zeros(self.N)
        for B in range(2 * n + 1):
            for A in range(1, 2 * n):
                x, y = A * h / 2, 1 + B * h / 2
                out[vel_index(n, 0, A, B)] = exact["ux"](x, y)
                out[vel_index(n, 1, A, B)] = exact["uy"](x, y)
        for j in range(n + 1):
            for i in range(n + 1):
                out[self.Nu + j * (n + 1) + i] = exact["pS"](i * h, 1 + j * h)
        fd = fem.free_dofs(2, n)
        for k, g in enumerate(fd):
            i, j = g % (n + 1), g // (n + 1)
            out[self.Nu + self.Np + k] = exact["pD"](i * h, j * h)
        return out


# ----------------------------------------------------------------------------
# flexible GMRES
# ----------------------------------------------------------------------------

def fgmres(apply_A, b, apply_B, rtol=1e-10, maxit=200):
    """Flexible GMRES (Saad 1993): right preconditioning by a possibly varying B, x_0 = 0, no
    restart, modified Gram-Schmidt Arnoldi, Givens rotations on the Hessenberg matrix.  Stops when
    the least-squares residual |g_{k+1}| (= ||b - A x_k||_2) is at most rtol ||b||_2.
    Returns (x, iterations, history of the least-squares residual)."""
    b = np.asarray(b, dtype=np.float64)
    beta = np.linalg.norm(b)
    if beta == 0:
        return np.zeros_like(b), 0, [0.0]
    V = [b / beta]
    Z = []
    H = np.zeros((maxit + 1, maxit))
    cs, sn = np.zeros(maxit), np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = beta
    hist = [beta]
    k = 0
    while k < maxit and abs(g[k]) > rtol * beta:
        z = apply_B(V[k])
        Z.append(z)
        w = apply_A(z)
        for i in range(k + 1):
            H[i, k] = w @ V[i]
            w = w - H[i, k] * V[i]
        H[k + 1, k] = np.linalg.norm(w)
        V.append(w / H[k + 1, k] if H[k + 1, k] > 0 else w)
        for i in range(k):
            t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
            H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
            H[i, k] = t
        r = np.hypot(H[k, k], H[k + 1, k])
        cs[k], sn[k] = H[k, k] / r, H[k + 1, k] / r
        H[k, k], H[k + 1, k] = r, 0.0
        g[k + 1] = -sn[k] * g[k]
        g[k] = cs[k] * g[k]
        k += 1
        hist.append(abs(g[k]))
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
    x = np.zeros_like(b)
    for i in range(k):
        x += y[i] * Z[i]
    return x, k, hist
