"""CPU models of the reduced-precision arithmetic forms of the E-step, used by the tests to tell
what rounding alone does to the results.  TEST INFRASTRUCTURE ONLY (never imported by the
library).

The E-step is Alg. 2's inner loop (CG of Alg. 1 on A = beta Phi^T Phi + diag(alpha_c) over the
mean right-hand side and K probes, then Eq. (diag-est) and Eqs. (tridiag)-(logdet-est)), run here
with the operator products and the CG vectors rounded as a form rounds them:

* products "f64": exact products of the FP32 Phi (FP64 arithmetic);
* products "f32": W = Phi v and Phi^T W in FP32 with FP32 accumulation (numpy's float32 matmul);
* products "bf16" / "f16": Phi and v rounded to the 16-bit type, FP32 accumulation, W rounded to
  the 16-bit type before the second product; the true residual b - A x of a replacement step
  uses FP32 products;
* vectors "f64" or "f32": the storage and update arithmetic of x, r, d, A d.
The CG scalars are FP64 in every form, as in the library.  The probes are the oracle's.

The model follows the algorithm's arithmetic, not the library's order of operations, so its
results differ from the library's by rounding order: it predicts the size of a form's departure
from the FP64 oracle, not its digits.
"""

import numpy as np

from oracle import cofem, cg as ocg, probes as oprobes, slq


def round16(a, kind):
    """Round float32 values to bf16 or fp16 (nearest, ties to even), returned as float32."""
    a = np.asarray(a, np.float32)
    if kind == "f16":
        return a.astype(np.float16).astype(np.float32)
    u = a.copy().view(np.uint32)
    u += np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))
    u &= np.uint32(0xFFFF0000)
    return u.view(np.float32)


def operator(P, beta, alpha_col, prod):
    """(apply_A, apply_true): A V in the form's product arithmetic, and the true-residual
    operator of a replacement step (FP32 products for the 16-bit forms)."""
    P64 = np.asarray(P, np.float64)
    P32 = np.asarray(P, np.float32)

    def exact(V, cols):
        return beta * (P64.T @ (P64 @ V)) + alpha_col[:, cols] * V

    def f32(V, cols):
        W = P32 @ V.astype(np.float32)
        return beta * (P32.T @ W).astype(np.float64) + alpha_col[:, cols] * V

    if prod == "f64":
        return exact, exact
    if prod == "f32":
        return f32, f32
    P16 = round16(P32, prod)

    def p16(V, cols):
        W = round16(P16 @ round16(V, prod), prod)
        return beta * (P16.T @ W).astype(np.float64) + alpha_col[:, cols] * V

    return p16, f32


def cg(apply_A, apply_true, B, policy, vec="f64", refine=0):
    """Alg. 1 over the columns of B with the vectors stored in `vec` precision and FP64 scalars;
    refine = m > 0 replaces the recursive residual by b - A_true x every m steps.  Returns
    X (FP64 copy), the gamma and xi histories and the step counts."""
    vt = np.float64 if vec == "f64" else np.float32
    B = np.asarray(B, np.float64)
    D, R = B.shape
    X = np.zeros((D, R), vt)
    Rv = B.astype(vt)
    Dv = B.astype(vt)
    rr = np.einsum("dr,dr->r", Rv.astype(np.float64), Rv.astype(np.float64))
    thr = policy.tol ** 2 * rr
    active = rr > 0
    iters = np.zeros(R, np.int32)
    gam = [[] for _ in range(R)]
    xis = [[] for _ in range(R)]
    for u in range(policy.steps):
        if not active.any():
            break
        cols = np.flatnonzero(active)
        AD = apply_A(Dv[:, cols].astype(np.float64), cols).astype(vt)
        dAd = np.einsum("dr,dr->r", Dv[:, cols].astype(np.float64), AD.astype(np.float64))
        ok = np.isfinite(dAd) & (dAd > 0)
        active[cols[~ok]] = False
        cols, AD, dAd = cols[ok], AD[:, ok], dAd[ok]
        if cols.size == 0:
            break
        g = rr[cols] / dAd
        X[:, cols] = (X[:, cols] + g.astype(vt) * Dv[:, cols]).astype(vt)
        Rn = (Rv[:, cols] - g.astype(vt) * AD).astype(vt)
        if refine and (u + 1) % refine == 0:
            Rn = (B[:, cols] - apply_true(X[:, cols].astype(np.float64), cols)).astype(vt)
        rrn = np.einsum("dr,dr->r", Rn.astype(np.float64), Rn.astype(np.float64))
        xi = rrn / rr[cols]
        Rv[:, cols] = Rn
        Dv[:, cols] = (Rn + xi.astype(vt) * Dv[:, cols]).astype(vt)
        for a, j in enumerate(cols):
            gam[j].append(g[a])
            xis[j].append(xi[a])
            iters[j] += 1
        rr[cols] = rrn
        stop = (rrn == 0) | (~np.isfinite(rrn))
        if policy.fixed_iters <= 0:
            stop |= rrn <= thr[cols]
        active[cols[stop]] = False
    return X.astype(np.float64), [np.array(v) for v in gam], [np.array(v) for v in xis], iters


def estep(w, tasks, alpha, K, policy, prod="f64", vec="f64", refine=0, seed=1, it=0):
    """mu, s, nu (FP64 arrays [task][c](...)) and the extreme Ritz values of every probe's
    tridiagonal, for the workload `w` (synth.Workload) in the given arithmetic form."""
    alpha = np.asarray(alpha, np.float64)
    C, D = alpha.shape
    R = C * (K + 1)
    b = cofem.rhs(w.phi_list(), w.y_list(), w.beta)
    P_all = oprobes.rademacher(seed, it, w.T, C, K, D, t_sel=list(tasks))
    alpha_col = np.repeat(alpha, K + 1, axis=0).T
    mu = np.zeros((len(tasks), C, D)); s = np.zeros((len(tasks), C, D))
    nu = np.zeros((len(tasks), C)); kappa = np.zeros((len(tasks), C))
    for a, t in enumerate(tasks):
        B = np.zeros((D, R))
        for c in range(C):
            B[:, c * (K + 1)] = b[t]
            B[:, c * (K + 1) + 1:(c + 1) * (K + 1)] = P_all[a, c].T
        ap, ap_true = operator(w.phi(t), w.beta, alpha_col, prod)
        X, g, x, _ = cg(ap, ap_true, B, policy, vec, refine)
        for c in range(C):
            j0 = c * (K + 1)
            mu[a, c] = X[:, j0]
            s[a, c] = (P_all[a, c] * X[:, j0 + 1:j0 + K + 1].T).mean(axis=0)
            taus, lmin, lmax = [], np.inf, 0.0
            for k in range(K):
                j = j0 + 1 + k
                lam, _ = slq.quadrature_terms(g[j], x[j])
                lmin, lmax = min(lmin, lam.min()), max(lmax, lam.max())
                taus.append(slq.quadrature_log(g[j], x[j], float(D)) if lam.min() > 0 else np.nan)
            nu[a, c] = -np.mean(taus)
            kappa[a, c] = lmax / lmin
    return dict(mu=mu, s=s, nu=nu, kappa=kappa)


def errors(got, ref):
    """Largest relative errors over (t, c): vector norms for mu and s, values for nu."""
    def cols(a, r):
        return float(np.max(np.linalg.norm(a - r, axis=-1) / np.linalg.norm(r, axis=-1)))
    return dict(mu=cols(got["mu"], ref["mu"]), s=cols(got["s"], ref["s"]),
                nu=float(np.max(np.abs(got["nu"] - ref["nu"]) / np.abs(ref["nu"]))))


def policy_of(cfg):
    return ocg.CGPolicy(fixed_iters=cfg.fixed_iters, tol=cfg.tol, max_iters=cfg.max_iters)
