"""Dense FP64 reference for the differentiation form.  TEST INFRASTRUCTURE ONLY.

For task t with cluster c_t the posterior mean is mu_t = A_t^-1 b_t with
A_t = beta Phi_t^T Phi_t + diag(alpha_{c_t}) and b_t = beta Phi_t^T y_t (Eqs. (estep), (lin-sys)).
For a scalar loss with upstream gradient g_t = dL/dmu_t, the adjoint system A_t lam_t = g_t
(A_t is symmetric) gives
    dL/db_t       = lam_t
    dL/dy_t       = beta Phi_t lam_t
    dL/dalpha_c   = -sum_{t : c_t = c} lam_t (.) mu_t
    dL/dPhi_t     = beta [ y_t lam_t^T - (Phi_t lam_t) mu_t^T - (Phi_t mu_t) lam_t^T ]
(the first term of dL/dPhi_t comes from b_t; the other two from A_t).  Everything here uses a
dense solve, so it is only for small D.
"""

import numpy as np


def operator(Phi_t, alpha_c, beta):
    P = np.asarray(Phi_t, np.float64)
    return beta * (P.T @ P) + np.diag(np.asarray(alpha_c, np.float64))


def forward(Phi, y, alpha, beta, cluster):
    """mu_t = A_t^-1 (beta Phi_t^T y_t) for every task, by dense solve."""
    mus = []
    for t, (P, v) in enumerate(zip(Phi, y)):
        A = operator(P, alpha[cluster[t]], beta)
        mus.append(np.linalg.solve(A, beta * (np.asarray(P, np.float64).T @ np.asarray(v, np.float64))))
    return np.stack(mus)


def backward(Phi, y, alpha, beta, cluster, grad_mu):
    """Gradients (dy, dalpha, dPhi, db) of L given grad_mu = dL/dmu (T x D)."""
    alpha = np.asarray(alpha, np.float64)
    mu = forward(Phi, y, alpha, beta, cluster)
    dalpha = np.zeros_like(alpha)
    dy, dPhi, db = [], [], []
    for t, (P, v) in enumerate(zip(Phi, y)):
        P = np.asarray(P, np.float64); v = np.asarray(v, np.float64)
        A = operator(P, alpha[cluster[t]], beta)
        lam = np.linalg.solve(A, np.asarray(grad_mu[t], np.float64))
        db.append(lam)
        dy.append(beta * (P @ lam))
        dalpha[cluster[t]] -= lam * mu[t]
        dPhi.append(beta * (np.outer(v, lam) - np.outer(P @ lam, mu[t]) - np.outer(P @ mu[t], lam)))
    return dict(mu=mu, dy=dy, dalpha=dalpha, dPhi=dPhi, db=np.stack(db))
