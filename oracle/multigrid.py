"""Geometric multigrid V-cycle for the interior Dirichlet block (oracle; test infrastructure only).

The paper's remark on evaluating the operator (Sec. 3, Fig. 4-left) replaces the exact leading
block (A^00)^{-1} of the preconditioner of eq. (dd_preconditioner) by a single multigrid V-cycle
(algebraic multigrid there).  This module writes out one geometric V-cycle for A_II, the P1
stiffness of -Delta on the (n-1) x (n-1) interior grid of the unit square (the 5-point stencil
4, -1, -1, -1, -1 on the diagonal-split mesh), as the plain definition of the textbook method:

  * grids: the interior grid of n cells per side has nf = n - 1 points per side; the next coarser
    grid is the nested mesh of n / 2 cells, nf_c = (nf - 1) / 2; coarsening continues while the
    point count is odd and ends at the first grid below the finest with <= 7 points per side or
    an even count;
  * prolongation P: P1 interpolation of the coarse finite-element function at the fine nodes
    (nested meshes, each cell split along the diagonal from (i, j) to (i+1, j+1));
  * restriction R = P^T, coarse operators P^T A P (equal to the rediscretized stencil);
  * smoother: red-black Gauss-Seidel, red = points with i + j even (1-based indices); before
    the coarse correction 2 nu half-sweeps from a zero iterate starting with red, after it 2 nu
    half-sweeps starting with black (the symmetric V(nu, nu) cycle);
  * the coarsest grid, or the first grid with at most `exact_nf` points per side, is solved
    exactly (dense LU).

Parity: pinned by the geometric evaluation of the coarse hat functions (P), the Galerkin
identity, symmetry and positivity of the V-cycle operator, its exactness when the finest grid
is the coarsest, the Gauss-Seidel property of each half-sweep, and the textbook contraction of
the V-cycle iteration (tests/test_oracle_multigrid.py).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def hierarchy(nf):
    """Point counts per side of every grid, finest first (the coarsening rule above)."""
    out = [nf]
    while True:
        if len(out) >= 2 and (out[-1] <= 7 or out[-1] % 2 == 0):
            return out
        if out[-1] < 3:
            return out
        out.append((out[-1] - 1) // 2)


def stiffness(nf):
    """5-point interior stiffness (unit diagonal scale 4) on an nf x nf grid, x fastest."""
    e = np.ones(nf)
    T = sp.diags([-e[:-1], 2 * e, -e[:-1]], [-1, 0, 1])
    I = sp.identity(nf)
    return (sp.kron(I, T) + sp.kron(T, I)).tocsr()


def prolongation(nc):
    """P1 interpolation from the coarse interior grid (nc points per side, nc + 1 cells) to the
    nested fine grid (2 nc + 1 points per side): column (J, I) holds the values of the coarse hat
    function of node (I, J) at the fine interior nodes."""
    nf = 2 * nc + 1
    Hc = 1.0 / (nc + 1)
    rows, cols, vals = [], [], []
    for jf in range(1, nf + 1):
        for i_f in range(1, nf + 1):
            x, y = i_f * Hc / 2, jf * Hc / 2
            # coarse cell containing (x, y) and its lower-left corner
            ci = min(int(np.floor(x / Hc + 1e-12)), nc)
            cj = min(int(np.floor(y / Hc + 1e-12)), nc)
            sx, sy = x / Hc - ci, y / Hc - cj        # local coordinates in [0, 1]
            # the cell is split along its diagonal: lower triangle (0,0),(1,0),(1,1) when
            # sx >= sy, upper triangle (0,0),(1,1),(0,1) otherwise; barycentric weights
            if sx >= sy:
                verts = [(ci, cj), (ci + 1, cj), (ci + 1, cj + 1)]
                lam = [1 - sx, sx - sy, sy]
            else:
                verts = [(ci, cj), (ci + 1, cj + 1), (ci, cj + 1)]
                lam = [1 - sy, sx, sy - sx]
            for (I, J), w in zip(verts, lam):
                if abs(w) < 1e-14 or not (1 <= I <= nc and 1 <= J <= nc):
                    continue  # Dirichlet nodes carry no coarse unknown
                rows.append((jf - 1) * nf + (i_f - 1))
                cols.append((J - 1) * nc + (I - 1))
                vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf * nf, nc * nc))


def red_mask(nf):
    """Boolean nf x nf mask of the red points (i + j even, 1-based indices)."""
    i = np.arange(1, nf + 1)
    return ((i[None, :] + i[:, None]) % 2) == 0


def half_sweep(u, f, red):
    """One Gauss-Seidel half-sweep over one colour of the 5-point system (u, f: nf x nf arrays,
    zero Dirichlet values outside): every point of the colour is set so that its own equation
    holds; points of one colour do not couple, so the order within the colour is immaterial."""
    nf = u.shape[0]
    up = np.zeros((nf + 2, nf + 2))
    up[1:-1, 1:-1] = u
    nb = up[:-2, 1:-1] + up[2:, 1:-1] + up[1:-1, :-2] + up[1:-1, 2:]
    mask = red_mask(nf) if red else ~red_mask(nf)
    out = u.copy()
    out[mask] = (f[mask] + nb[mask]) / 4.0
    return out


class VCycle:
    """The V(nu, nu) cycle for A_II on an nf x nf grid (see the module docstring)."""

    def __init__(self, nf, nu=2, exact_nf=0):
        self.nu = nu
        sizes = hierarchy(nf)
        # the first level (below the finest) with <= exact_nf points, else the coarsest
        last = len(sizes) - 1
        for l in range(1, len(sizes)):
            if sizes[l] <= exact_nf:
                last = l
                break
        self.sizes = sizes[:last + 1]
        self.A = [stiffness(m) for m in self.sizes]
        self.P = [prolongation(self.sizes[l + 1]) for l in range(len(self.sizes) - 1)]
        self.lu = sla.lu_factor(self.A[-1].toarray())

    def apply(self, f, level=0):
        """u = V f (f and u flat, x fastest)."""
        m = self.sizes[level]
        if level == len(self.sizes) - 1:
            return sla.lu_solve(self.lu, f)
        F = f.reshape(m, m)
        U = np.zeros((m, m))
        for s in range(2 * self.nu):          # red, black, red, ...
            U = half_sweep(U, F, red=(s % 2 == 0))
        r = f - self.A[level] @ U.ravel()
        ec = self.apply(self.P[level].T @ r, level + 1)
        U = U + (self.P[level] @ ec).reshape(m, m)
        for s in range(2 * self.nu):          # black, red, black, ...
            U = half_sweep(U, F, red=(s % 2 == 1))
        return U.ravel()
