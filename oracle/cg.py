"""Conjugate gradient, Alg. 1 of the paper, in FP64.  TEST INFRASTRUCTURE ONLY.

Alg. 1 solves A x = b for symmetric positive definite A from x_1 = 0, r_1 = b, d_1 = r_1:
    gamma_u = (r_u . r_u) / (d_u . A d_u)
    x_{u+1} = x_u + gamma_u d_u
    r_{u+1} = r_u - gamma_u A d_u
    xi_u    = (r_{u+1} . r_{u+1}) / (r_u . r_u)
    d_{u+1} = r_{u+1} + xi_u d_u
The paper runs it "until convergence" (Alg. 1) or for U steps (Sec. 3.1, U = 50 in Sec. 4).  The
stopping policy below is this implementation's reading, applied per right-hand side:

* fixed mode (``fixed_iters = U > 0``): exactly U steps;
* tol mode: stop after step u once ||r_{u+1}||^2 <= tol^2 ||b||^2 (recursive residual), at most
  ``max_iters`` steps;
* either mode stops before a step whose d.Ad is not positive and finite (BREAKDOWN, no gamma
  recorded), and after a step whose new r.r is exactly zero (CONVERGED) or not finite (BREAKDOWN).

Several independent right-hand sides are iterated side by side (the paper solves all systems
simultaneously, Sec. 3.3); every column has its own scalars and its own stop, so each column's
arithmetic is that of Alg. 1 run alone.  A column that has stopped is no longer modified.
"""

import numpy as np

CONVERGED = 0   # tol met, fixed step count done, or exact zero residual
MAX_ITER = 1    # tol mode: max_iters reached without meeting tol
BREAKDOWN = 2   # d.Ad <= 0 or a non-finite scalar


class CGPolicy:
    """Stopping policy: fixed U steps (fixed_iters > 0) or tolerance with a step cap."""

    def __init__(self, fixed_iters=0, tol=1e-6, max_iters=200):
        self.fixed_iters = int(fixed_iters)
        self.tol = float(tol)
        self.max_iters = int(max_iters)

    @property
    def steps(self):
        return self.fixed_iters if self.fixed_iters > 0 else self.max_iters


def cg(apply_A, B, policy):
    """Run Alg. 1 on every column of B (D x R).

    Returns X (D x R), gammas and xis as lists of per-column arrays (length U_j = steps taken),
    iters (R,), status (R,).
    """
    B = np.asarray(B, dtype=np.float64)
    D, R = B.shape
    X = np.zeros((D, R))
    Rv = B.copy()
    Dv = B.copy()
    rr = np.einsum("dr,dr->r", Rv, Rv)
    thr = (policy.tol ** 2) * rr
    active = rr > 0                         # b = 0: x = 0 is exact, nothing to do
    status = np.full(R, CONVERGED, dtype=np.int32)
    iters = np.zeros(R, dtype=np.int32)
    gam = [[] for _ in range(R)]
    xis = [[] for _ in range(R)]
    for _u in range(policy.steps):
        if not active.any():
            break
        cols = np.flatnonzero(active)
        AD = apply_A(Dv[:, cols], cols)
        dAd = np.einsum("dr,dr->r", Dv[:, cols], AD)
        ok = np.isfinite(dAd) & (dAd > 0)
        for j in cols[~ok]:
            status[j] = BREAKDOWN
            active[j] = False
        cols, AD, dAd = cols[ok], AD[:, ok], dAd[ok]
        if cols.size == 0:
            break
        g = rr[cols] / dAd
        X[:, cols] += g * Dv[:, cols]
        Rv[:, cols] -= g * AD
        rr_new = np.einsum("dr,dr->r", Rv[:, cols], Rv[:, cols])
        xi = rr_new / rr[cols]
        Dv[:, cols] = Rv[:, cols] + xi * Dv[:, cols]
        for a, j in enumerate(cols):
            gam[j].append(g[a])
            xis[j].append(xi[a])
            iters[j] += 1
        rr[cols] = rr_new
        for a, j in enumerate(cols):
            if not np.isfinite(rr_new[a]):
                status[j] = BREAKDOWN
                active[j] = False
            elif rr_new[a] == 0.0 or (policy.fixed_iters <= 0 and rr_new[a] <= thr[j]):
                status[j] = CONVERGED
                active[j] = False
    if policy.fixed_iters <= 0:
        status[active] = MAX_ITER
    return X, [np.array(v) for v in gam], [np.array(v) for v in xis], iters, status


def pcg(apply_A, B, policy, m):
    """Alg. 1 with a diagonal preconditioner M = diag(m) (m: D x R, one column per right-hand
    side), the textbook preconditioned form: with z = M^-1 r,
        gamma_u = (r_u . z_u) / (d_u . A d_u),  x += gamma d,  r -= gamma A d,
        xi_u = (r_{u+1} . z_{u+1}) / (r_u . z_u),  d = z_{u+1} + xi_u d,
    from x_1 = 0, r_1 = b, d_1 = z_1.  It is CG on M^-1/2 A M^-1/2 with right-hand side
    M^-1/2 b (the iterates map through x = M^-1/2 x-hat), so gamma_u and xi_u are that run's and
    Eq. (tridiag) gives its Lanczos tridiagonal from the start vector M^-1/2 b.  The stopping
    policy is cg's, on the unpreconditioned residual ||r||.  m = 1 is cg exactly."""
    B = np.asarray(B, dtype=np.float64)
    m = np.broadcast_to(np.asarray(m, np.float64), B.shape)
    D, R = B.shape
    X = np.zeros((D, R))
    Rv = B.copy()
    Z = Rv / m
    Dv = Z.copy()
    rz = np.einsum("dr,dr->r", Rv, Z)
    rr0 = np.einsum("dr,dr->r", Rv, Rv)
    thr = (policy.tol ** 2) * rr0
    active = rr0 > 0
    status = np.full(R, CONVERGED, dtype=np.int32)
    iters = np.zeros(R, dtype=np.int32)
    gam = [[] for _ in range(R)]
    xis = [[] for _ in range(R)]
    for _u in range(policy.steps):
        if not active.any():
            break
        cols = np.flatnonzero(active)
        AD = apply_A(Dv[:, cols], cols)
        dAd = np.einsum("dr,dr->r", Dv[:, cols], AD)
        ok = np.isfinite(dAd) & (dAd > 0)
        for j in cols[~ok]:
            status[j] = BREAKDOWN
            active[j] = False
        cols, AD, dAd = cols[ok], AD[:, ok], dAd[ok]
        if cols.size == 0:
            break
        g = rz[cols] / dAd
        X[:, cols] += g * Dv[:, cols]
        Rv[:, cols] -= g * AD
        Z[:, cols] = Rv[:, cols] / m[:, cols]
        rz_new = np.einsum("dr,dr->r", Rv[:, cols], Z[:, cols])
        rr_new = np.einsum("dr,dr->r", Rv[:, cols], Rv[:, cols])
        xi = rz_new / rz[cols]
        Dv[:, cols] = Z[:, cols] + xi * Dv[:, cols]
        for a, j in enumerate(cols):
            gam[j].append(g[a])
            xis[j].append(xi[a])
            iters[j] += 1
        rz[cols] = rz_new
        for a, j in enumerate(cols):
            if not (np.isfinite(rr_new[a]) and np.isfinite(rz_new[a])):
                status[j] = BREAKDOWN
                active[j] = False
            elif rr_new[a] == 0.0 or (policy.fixed_iters <= 0 and rr_new[a] <= thr[j]):
                status[j] = CONVERGED
                active[j] = False
    if policy.fixed_iters <= 0:
        status[active] = MAX_ITER
    return X, [np.array(v) for v in gam], [np.array(v) for v in xis], iters, status
