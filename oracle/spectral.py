"""Interface spectral calculus (oracle; test infrastructure only).

Paper, Sec. 2, footnote with eq. (gevp): for an SPD interface operator L with matrix
L_h and mass matrix M_h, the generalized eigenproblem L_h U = M_h U Lambda with
U^T M_h U = I defines the fractional power L_h^s = (M_h U) Lambda^s (M_h U)^T.
The cost is cubic; the oracle uses it only at the sizes where that is affordable.

Reading: L_h is the interface stiffness A_Gamma itself (no identity shift), with
homogeneous Dirichlet conditions at the boundary of Gamma.

For the Riesz map of eq. (riesz), the Schur-complement preconditioner of
eq. (schur_precond) is S_Gamma = K L^{1/2} + gamma L^{-1/2} (gamma = 1/mu, Sec. 4 with
s = 1/2, t = -1/2), and its exact inverse is U f(Lambda) U^T with
f(lambda) = 1 / (K lambda^{1/2} + gamma lambda^{-1/2}).

Parity: pinned by the closed-form 1D eigenpairs, the identities s = 0 -> M_h,
s = 1 -> L_h, L^{s} L^{-s} consistency through M^{-1}, and the Sobolev-norm limit
of sin(k pi x) (tests/test_oracle_spectral.py).
"""
import numpy as np
import scipy.linalg as sla


def gevp(L, M):
    """Lambda (ascending) and U with L U = M U diag(Lambda), U^T M U = I."""
    lam, U = sla.eigh(L, M)
    return lam, U


def frac_power(L, M, s, eig=None):
    """L_h^s = (M U) Lambda^s (M U)^T  (eq. (gevp))."""
    lam, U = eig if eig is not None else gevp(L, M)
    MU = M @ U
    return (MU * lam ** s) @ MU.T


def spectral_function(L, M, f, eig=None):
    """U f(Lambda) U^T: the operator with symbol f in the M-orthonormal eigenbasis.

    For f = 1/(alpha x^s + beta x^t) this is the exact inverse of alpha L^s + beta L^t.
    """
    lam, U = eig if eig is not None else gevp(L, M)
    return (U * f(lam)) @ U.T


def f_precond(K, gamma):
    """f(lambda) = (K lambda^{1/2} + gamma lambda^{-1/2})^{-1}."""
    return lambda lam: 1.0 / (K * np.sqrt(lam) + gamma / np.sqrt(lam))


def g_operator(lam):
    """g(lambda) = lambda^{-1/2}: symbol of the perturbation H = L^{-1/2} in U f U^T form."""
    return lam ** -0.5


def schur_precond(L, M, K, gamma, eig=None):
    """S_Gamma = K L^{1/2} + gamma L^{-1/2}  (eq. (schur_precond))."""
    eig = eig if eig is not None else gevp(L, M)
    return K * frac_power(L, M, 0.5, eig) + gamma * frac_power(L, M, -0.5, eig)


def schur_precond_inverse(L, M, K, gamma, eig=None):
    """Exact S_Gamma^{-1} = U (K Lambda^{1/2} + gamma Lambda^{-1/2})^{-1} U^T."""
    return spectral_function(L, M, f_precond(K, gamma), eig)


# ----------------------------------------------------------------------------
# closed forms for the 2D interface (1D P1 on n segments, Dirichlet ends)
# ----------------------------------------------------------------------------

def interface_eigs_1d(n):
    """Closed-form eigenvalues of (A_Gamma, M_Gamma) for the 1D P1 interface.

    A_Gamma = (1/h) tridiag(-1, 2, -1), M_Gamma = (h/6) tridiag(1, 4, 1); both are
    diagonalized by sin(theta_q i), theta_q = q pi / n, so
      lambda_q = 6 (1 - cos theta_q) / (h^2 (2 + cos theta_q)),  q = 1..n-1.
    """
    h = 1.0 / n
    th = np.arange(1, n) * np.pi / n
    return 6.0 * (1.0 - np.cos(th)) / (h * h * (2.0 + np.cos(th)))


def spectral_interval(dim, n):
    """[lambda_lo, lambda_hi] containing the discrete interface spectrum.

    2D: the exact extreme eigenvalues from the closed form.
    3D: computed from the dense GEVP (the oracle can afford it at its sizes).
    """
    if dim == 2:
        lam = interface_eigs_1d(n)
        return float(lam[0]), float(lam[-1])
    from .fem import Problem
    P = Problem(3, n)
    lam = sla.eigh(P.A_G, P.M_G, eigvals_only=True)
    return float(lam[0]), float(lam[-1])
