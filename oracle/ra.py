"""Checks of rational-approximation tables (oracle; test infrastructure only).

Paper, Sec. 2, footnote with eq. (RA): the solution operator of alpha L^s + beta L^t
is approximated by  c_0 M_h^{-1} + sum_k c_k (L_h + p_k M_h)^{-1},  where the scalar
function f_RA(lambda) = c_0 + sum_k c_k / (lambda + p_k) approximates
f(lambda) = (alpha lambda^s + beta lambda^t)^{-1}.  Because U^T M U = I, the matrix
operator equals U f_RA(Lambda) U^T, so its error is governed by |f - f_RA| on the
discrete spectrum.

(The paper writes the residues with index i inside a sum over k; read c_k.  The
paper calls p_k >= 0 the poles; the poles of f_RA sit at -p_k.)

Parity: this module only evaluates given tables; it is pinned by comparing the
scalar evaluation with the dense matrix evaluation on the exact GEVP basis.
"""
import numpy as np


def eval_scalar(c0, c, p, lam):
    """f_RA(lambda) = c0 + sum_k c_k / (lambda + p_k), vectorised over lambda."""
    lam = np.asarray(lam, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    return c0 + (c[None, :] / (lam[:, None] + p[None, :])).sum(axis=1)


def max_rel_error(f, c0, c, p, lam):
    """max over lam of |f - f_RA| / |f|."""
    fv = f(np.asarray(lam, dtype=np.float64))
    return float(np.max(np.abs(fv - eval_scalar(c0, c, p, lam)) / np.abs(fv)))


def dense_operator(L, M, c0, c, p):
    """c0 M^{-1} + sum_k c_k (L + p_k M)^{-1}, as a dense matrix."""
    out = c0 * np.linalg.inv(M)
    for ck, pk in zip(c, p):
        out = out + ck * np.linalg.inv(L + pk * M)
    return out


def dense_operator_H(L, M, d0, d, q):
    """M (d0 M^{-1} + sum_k d_k (L + q_k M)^{-1}) M: the RA realization of L^{-1/2}."""
    return M @ dense_operator(L, M, d0, d, q) @ M


def apply_tridiagonal(L, M, c0, c, p, r):
    """c0 M^{-1} r + sum_k c_k (L + p_k M)^{-1} r for tridiagonal L, M (the 2D interface, eq. (RA)).

    Every shifted system is solved by a banded LU (scipy.linalg.solve_banded), the way a CPU
    code applies the rational preconditioner on a 1D interface.
    """
    import scipy.linalg as sla

    def banded(A):
        ab = np.zeros((3, A.shape[0]))
        ab[0, 1:] = np.diag(A, 1)
        ab[1, :] = np.diag(A)
        ab[2, :-1] = np.diag(A, -1)
        return ab

    out = c0 * sla.solve_banded((1, 1), banded(M), r)
    for ck, pk in zip(c, p):
        out = out + ck * sla.solve_banded((1, 1), banded(L + pk * M), r)
    return out
