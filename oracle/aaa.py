"""Plain AAA rational approximation (oracle; test infrastructure only).

The paper (Sec. 2, eq. (RA)) leaves the construction of the rational approximation to
the cited literature and fixes only the form c_0 + sum_k c_k / (lambda + p_k) and the
accuracy epsilon_RA.  This module is an independent textbook AAA (adaptive
Antoulas-Anderson; Nakatsukasa, Sete and Trefethen, SIAM J. Sci. Comput. 2018) with
relative weighting, written only to pin pole counts and the achievable accuracy
independently of the product's own builder.  It uses numpy's SVD and eigenvalue
routines as library steps.

Steps, in the order of the published algorithm:
  1. start with no support points; the approximant is the mean of f.
  2. add the sample with the largest (relative) error as a support point.
  3. the barycentric weights are the right singular vector of the smallest singular
     value of the (row-weighted) Loewner matrix on the remaining samples.
  4. repeat until the relative error on the samples is below tol.
Poles are the eigenvalues of the arrowhead pencil of the barycentric form; the
partial-fraction residues are then refit by least squares with relative weights.

Parity: pinned by tests that approximate sqrt and x^{-1/2} on a positive interval and
reach the requested accuracy, and that the poles of x^{-1/2} lie on the negative axis.
"""
import numpy as np
import scipy.linalg as sla


def aaa(F, Z, tol=1e-13, mmax=100):
    """Relative-error AAA.  Returns (support z, values f, weights w)."""
    Z = np.asarray(Z, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    scale = 1.0 / np.abs(F)
    mask = np.ones(len(Z), dtype=bool)
    R = np.full_like(F, F.mean())
    zs, fs = [], []
    w = None
    for _ in range(mmax):
        err = np.abs(F - R) * scale
        j = int(np.argmax(np.where(mask, err, -1.0)))
        zs.append(Z[j])
        fs.append(F[j])
        mask[j] = False
        zj = np.array(zs)
        fj = np.array(fs)
        C = 1.0 / (Z[mask][:, None] - zj[None, :])
        Loew = (F[mask][:, None] - fj[None, :]) * C * scale[mask][:, None]
        _, _, Vh = np.linalg.svd(Loew, full_matrices=False)
        w = Vh[-1, :]
        N = C @ (w * fj)
        D = C @ w
        R = F.copy()
        R[mask] = N / D
        if np.max(np.abs(F - R) * scale) <= tol:
            break
    return np.array(zs), np.array(fs), w


def poles(zj, wj):
    """Zeros of sum_j w_j / (z - z_j) from the (m+1) x (m+1) pencil."""
    m = len(zj)
    E = np.zeros((m + 1, m + 1))
    E[0, 1:] = wj
    E[1:, 0] = 1.0
    E[1:, 1:] = np.diag(zj)
    B = np.eye(m + 1)
    B[0, 0] = 0.0
    ev = sla.eigvals(E, B)
    return ev[np.isfinite(ev)]


def partial_fractions(F, Z, pole_list):
    """Least-squares residues (relative weights) for fixed real poles.

    Model: c0 + sum_k c_k / (z - pole_k).  Returns (c0, c).
    """
    Z = np.asarray(Z, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    cols = [np.ones_like(Z)] + [1.0 / (Z - pk) for pk in pole_list]
    A = np.stack(cols, axis=1) / np.abs(F)[:, None]
    coef, *_ = np.linalg.lstsq(A, F / np.abs(F), rcond=None)
    return coef[0], coef[1:]


def ra_table(f, lam_lo, lam_hi, tol=1e-12, nsamp=4000, extra=None):
    """Rational table (c0, c_k, p_k) with f(lam) ~ c0 + sum c_k/(lam + p_k) on [lam_lo, lam_hi].

    Samples: nsamp log-spaced points plus the given extra points; AAA runs on
    lam / lam_hi.  Complex poles and poles at positive lam are dropped and the residues
    refit (they would make a shifted operator L + p M indefinite or complex).
    """
    Z = np.geomspace(lam_lo, lam_hi, nsamp)
    if extra is not None:
        Z = np.unique(np.concatenate([Z, np.asarray(extra, dtype=np.float64)]))
    F = f(Z)
    zs = Z / lam_hi
    zj, fj, wj = aaa(F, zs, tol=tol)
    pl = poles(zj, wj)
    keep = [float(np.real(x)) for x in pl if abs(np.imag(x)) <= 1e-10 * max(1.0, abs(x))
            and np.real(x) < 0.0]
    c0, c = partial_fractions(F, zs, keep)
    p = -np.array(keep) * lam_hi
    c = np.asarray(c) * lam_hi
    return float(c0), c, p
