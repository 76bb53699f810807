"""Log-determinant by stochastic Lanczos quadrature from CG coefficients, Sec. 3.2.

TEST INFRASTRUCTURE ONLY.

* Eq. (tridiag): the U steps of Alg. 1 on A x = p with x_1 = 0 define the U x U symmetric
  tridiagonal Gamma-bar with
      Gamma_11 = 1/gamma_1,
      Gamma_uu = 1/gamma_u + xi_{u-1}/gamma_{u-1}             (1 < u <= U)
      Gamma_{u,u-1} = Gamma_{u-1,u} = sqrt(xi_{u-1})/gamma_{u-1}
  (the sign of the off-diagonal does not change eigenvalues or squared first components).
* Eq. (hutch-trace), truncated to U steps: p^T log(A) p ~= ||p||^2 sum_u S_{u,1}^2 log lambda_u,
  with (lambda_u, S_u) the eigenpairs of Gamma-bar and S_{u,1} the first component of the u-th
  unit eigenvector.  The paper writes the factor as D, which equals ||p||^2 for Rademacher probes;
  ||p||^2 is used so that other +-1 probe sets (Hadamard columns) are covered too.
* Eq. (logdet-est): nu-bar(Sigma) = -(1/K) sum_k tau_k with tau_k the quadrature of probe k;
  it estimates log det Sigma = -log det A = -tr log A.
"""

import numpy as np
from scipy.linalg import eigh_tridiagonal


def tridiagonal(gammas, xis):
    """Diagonal and off-diagonal of Gamma-bar (Eq. (tridiag)) from gamma_1..U and xi_1..U-1."""
    g = np.asarray(gammas, dtype=np.float64)
    x = np.asarray(xis, dtype=np.float64)[: max(len(g) - 1, 0)]
    U = len(g)
    diag = 1.0 / g
    if U > 1:
        diag[1:] += x / g[:-1]
    off = np.sqrt(x) / g[:-1]
    return diag, off


def quadrature_terms(gammas, xis):
    """Ritz values lambda_u and Gauss weights S_{u,1}^2 of Gamma-bar."""
    diag, off = tridiagonal(gammas, xis)
    if len(diag) == 1:
        return diag.copy(), np.ones(1)
    lam, S = eigh_tridiagonal(diag, off, lapack_driver="stev")   # implicit QL/QR (robust)
    return lam, S[0, :] ** 2


def quadrature_log(gammas, xis, pnorm2):
    """tau = ||p||^2 sum_u S_{u,1}^2 log(lambda_u): the estimate of p^T log(A) p (Eq. (hutch-trace))."""
    if len(gammas) == 0:
        return 0.0
    lam, w = quadrature_terms(gammas, xis)
    if not np.all(lam > 0):
        raise FloatingPointError("non-positive Ritz value: A is not numerically SPD")
    return float(pnorm2 * np.sum(w * np.log(lam)))


def logdet_estimate(taus):
    """nu-bar = -(1/K) sum_k tau_k, Eq. (logdet-est)."""
    return -float(np.mean(taus))
