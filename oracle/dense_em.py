"""Exact EM with explicit posterior covariances (Eqs. (estep), (mstep)).  TEST INFRASTRUCTURE ONLY.

This is the O(T C D^3) baseline that CoFEM replaces (Sec. 2).  It forms
Sigma_tc = (beta Phi_t^T Phi_t + diag(alpha_c))^-1 by a Cholesky factorisation, then
mu_tc = beta Sigma_tc Phi_t^T y_t, log det Sigma_tc = -2 sum log diag(chol), ell_tc, q_t, and the
M-step with the exact diagonal of Sigma_tc.  It is only used on tiny inputs, to pin the CoFEM
oracle (with Hadamard probes and converged CG the two must agree to rounding).
"""

import numpy as np
from scipy.linalg import cho_factor, cho_solve

from .cofem import responsibilities, log_likelihood, log_norm_const, rhs, update_log_pi


def estep(Phi, b, beta, alpha):
    alpha = np.asarray(alpha, np.float64)
    C, D = alpha.shape
    T = len(Phi)
    mu = np.zeros((T, C, D)); var = np.zeros((T, C, D))
    logdet = np.zeros((T, C)); ell = np.zeros((T, C))
    for t in range(T):
        P = np.asarray(Phi[t], np.float64)
        G = beta * (P.T @ P)
        for c in range(C):
            A = G + np.diag(alpha[c])
            cf = cho_factor(A, lower=True)
            mu[t, c] = cho_solve(cf, b[t])
            Sigma = cho_solve(cf, np.eye(D))
            var[t, c] = np.diag(Sigma)
            logdet[t, c] = -2.0 * np.sum(np.log(np.diag(cf[0])))
            ell[t, c] = logdet[t, c] + np.sum(np.log(alpha[c])) + b[t] @ mu[t, c]
    return dict(mu=mu, var=var, logdet=logdet, ell=ell)


def mstep(mu, var, q, alpha_old=None):
    """Eq. (mstep) with the exact diagonal (no guard needed: the denominator is positive)."""
    Nq = q.sum(axis=0)
    den = np.einsum("tc,tcd->cd", q, mu * mu + var)
    return Nq[:, None] / den


def fit(Phi, y, beta, alpha0, log_pi, n_em, learn_pi=False):
    """Exact EM; with ``learn_pi`` the M-step also updates the cluster weights."""
    b = rhs(Phi, y, beta)
    const = log_norm_const(Phi, y, beta)
    alpha = np.asarray(alpha0, np.float64).copy()
    log_pi = np.asarray(log_pi, np.float64).copy()
    hist = []
    for _ in range(n_em):
        e = estep(Phi, b, beta, alpha)
        q = responsibilities(e["ell"], log_pi)
        hist.append(dict(L=log_likelihood(e["ell"], log_pi, const), alpha=alpha.copy(), q=q,
                         ell=e["ell"].copy(), log_pi=log_pi.copy()))
        alpha = mstep(e["mu"], e["var"], q, alpha)
        if learn_pi:
            log_pi = update_log_pi(q)
    assign = np.argmax(q, axis=1)
    return dict(alpha=alpha, q=q, assign=assign, mu=e["mu"], var=e["var"], log_pi=log_pi,
                history=hist)
