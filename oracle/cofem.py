"""CoFEM (covariance-free EM), Alg. 2, in FP64.  TEST INFRASTRUCTURE ONLY.

Model (Eq. (cmtcs)): a_t ~ Cat(pi), z_t | a_t = c ~ N(0, diag(alpha_c)^-1),
y_t | z_t ~ N(Phi_t z_t, beta^-1 I).

E-step of CoFEM for every task t and cluster c (Alg. 2 inner loop):
  * A = beta Phi_t^T Phi_t + diag(alpha_c), applied matrix-free (Sec. 3.3);
  * right-hand sides (Eq. (lin-sys)): b_t = beta Phi_t^T y_t for the posterior mean mu, and K
    Rademacher probes p_k for the diagonal estimate;
  * all solved with CG (Alg. 1); x_k = A^-1 p_k;
  * s = (1/K) sum_k p_k (.) x_k estimates diag Sigma (Eq. (diag-est));
  * nu-bar from the CG coefficients of the probe solves (Eqs. (tridiag), (hutch-trace),
    (logdet-est));
  * ell_tc = nu-bar + sum_d log alpha_cd + beta y_t^T Phi_t mu_tc   (Eq. (estep); the last term
    is b_t . mu_tc);
  * q_t = softmax_c(ell_tc / 2 + log pi_c)  (Eq. (estep)), evaluated with a max-shifted
    log-sum-exp.
M-step (Eq. (mstep)) with diag Sigma replaced by s:
  alpha_cd = sum_t q_tc / sum_t q_tc (mu_tcd^2 + s_tcd).
The paper does not discuss guards; since s is a Monte Carlo estimate the denominator can be
non-positive.  Reading used here: a cluster with sum_t q_tc < 1e-300 keeps its old alpha; otherwise
alpha_cd = Nq_c / den_cd when den_cd > Nq_c / alpha_max, else alpha_max.  Tasks whose q_tc is not
finite are left out of cluster c's sums, and an entry whose den_cd is not finite keeps its old
alpha_cd (a failed task must not overwrite the model).
Learned cluster weights (optional): the model of Sec. 2 takes pi as known but notes that it can
be learned as in finite-mixture EM.  That M-step maximises sum_tc q_tc log pi_c over the simplex,
whose maximiser is pi_c = (1/T) sum_t q_tc; ``update_log_pi`` returns log pi_c (-inf for a cluster
with no mass).
Final step (Alg. 2): a_t = argmax_c q_tc (lowest c on ties), return mu_{t, a_t} from the last
E-step.
"""

import numpy as np

from . import cg as _cg
from . import probes as _probes
from . import slq as _slq


def rhs(Phi, y, beta):
    """b_t = beta Phi_t^T y_t for every task (Eq. (lin-sys), right-hand side of the mean system)."""
    return [beta * (np.asarray(P, np.float64).T @ np.asarray(v, np.float64)) for P, v in zip(Phi, y)]


def log_norm_const(Phi, y, beta):
    """Per-task constant with ell/2 + const_t = log N(y_t; 0, beta^-1 I + Phi diag(alpha)^-1 Phi^T)."""
    out = []
    for P, v in zip(Phi, y):
        N = P.shape[0]
        v = np.asarray(v, np.float64)
        out.append(-0.5 * N * np.log(2 * np.pi) + 0.5 * N * np.log(beta) - 0.5 * beta * v @ v)
    return np.array(out)


def responsibilities(ell, log_pi):
    """q_t = softmax_c(ell_tc / 2 + log pi_c), max-shifted (Eq. (estep))."""
    z = 0.5 * np.asarray(ell, np.float64) + np.asarray(log_pi, np.float64)[None, :]
    m = z.max(axis=1, keepdims=True)
    lse = m + np.log(np.exp(z - m).sum(axis=1, keepdims=True))
    return np.exp(z - lse)


def estep(Phi, b, beta, alpha, log_pi, K, policy, seed=1, it=0, probes=None, t_sel=None,
          common_probes=False, precond=None):
    """One CoFEM E-step (Alg. 2, inner loop) for the tasks in ``t_sel`` (default: all).

    Phi: list of N_t x D arrays; b: list of D vectors (from ``rhs``); alpha: C x D; log_pi: C.
    probes: optional array [T][C][K][D] of +-1 overriding the SplitMix64 probes.
    common_probes: with generated probes, every cluster c of a task uses the probes drawn for
    c = 0 (common random numbers across clusters; a variance-reduction variant, not in the
    paper: each (t, c) estimator keeps its distribution, and the Monte Carlo errors of ell_tc
    and ell_tc' become correlated, so their difference, which decides q_t, varies less).
    precond="jacobi" (not in the paper): CG preconditioned by M = diag(A_tc) (cg.pcg), with the
    estimators adjusted so that one solve per probe still serves both: the probe right-hand side
    is M^1/2 p, so that the preconditioned run is CG on A-hat = M^-1/2 A M^-1/2 started at p and
    its Lanczos quadrature (Eqs. (tridiag), (hutch-trace)) estimates p^T log(A-hat) p; then
        log det Sigma = -(sum_d log M_dd + log det A-hat)  ->  nu-bar = -(sum log M + mean tau),
        s = M^-1/2 (.) (1/K) sum_k p_k (.) A^-1 M^1/2 p_k,
    unbiased for diag Sigma since E[p_d (A^-1 M^1/2 p)_d] = (A^-1)_dd M_dd^1/2.
    Returns a dict of FP64 arrays indexed [task-in-selection][c](...).
    """
    alpha = np.asarray(alpha, np.float64)
    C, D = alpha.shape
    T = len(Phi)
    tasks = list(range(T)) if t_sel is None else list(t_sel)
    if probes is None:
        P_all = _probes.rademacher(seed, it, T, C, K, D, t_sel=tasks)
        if common_probes:
            P_all = np.repeat(P_all[:, :1], C, axis=1)
    else:
        P_all = np.asarray(probes, np.float64)[tasks]
    R = C * (K + 1)
    n = len(tasks)
    mu = np.zeros((n, C, D)); s = np.zeros((n, C, D))
    nu = np.zeros((n, C)); ell = np.zeros((n, C))
    iters = np.zeros((n, C, K + 1), np.int32); status = np.zeros((n, C, K + 1), np.int32)
    taus = np.zeros((n, C, K))
    gam = [[None] * R for _ in range(n)]
    xis = [[None] * R for _ in range(n)]
    sum_log_alpha = np.log(alpha).sum(axis=1)
    # column j = c (K + 1) + k: k = 0 is the mean system, k = 1..K the probes
    alpha_col = np.repeat(alpha, K + 1, axis=0).T                     # D x R
    for a, t in enumerate(tasks):
        Pt = np.asarray(Phi[t], np.float64)
        if precond == "jacobi":
            mdiag = beta * (Pt * Pt).sum(axis=0)[:, None] + alpha.T     # D x C: diag(A_tc)
        elif precond is not None:
            raise ValueError("precond must be None or 'jacobi'")
        B = np.zeros((D, R))
        for c in range(C):
            B[:, c * (K + 1)] = b[t]
            pr = P_all[a, c].T
            if precond == "jacobi":
                pr = np.sqrt(mdiag[:, c:c + 1]) * pr
            B[:, c * (K + 1) + 1:(c + 1) * (K + 1)] = pr

        def apply_A(V, cols, Pt=Pt):
            return beta * (Pt.T @ (Pt @ V)) + alpha_col[:, cols] * V

        if precond == "jacobi":
            X, g, x, it_, st = _cg.pcg(apply_A, B, policy, np.repeat(mdiag, K + 1, axis=1))
        else:
            X, g, x, it_, st = _cg.cg(apply_A, B, policy)
        gam[a], xis[a] = g, x
        for c in range(C):
            j0 = c * (K + 1)
            mu[a, c] = X[:, j0]
            pk = P_all[a, c]                                          # K x D
            s[a, c] = (pk * X[:, j0 + 1:j0 + K + 1].T).mean(axis=0)
            for k in range(K):
                j = j0 + 1 + k
                taus[a, c, k] = _slq.quadrature_log(g[j], x[j], float(pk[k] @ pk[k]))
            nu[a, c] = _slq.logdet_estimate(taus[a, c])
            if precond == "jacobi":
                s[a, c] /= np.sqrt(mdiag[:, c])
                nu[a, c] -= np.log(mdiag[:, c]).sum()
            ell[a, c] = nu[a, c] + sum_log_alpha[c] + float(b[t] @ mu[a, c])
            iters[a, c] = it_[j0:j0 + K + 1]
            status[a, c] = st[j0:j0 + K + 1]
    q = responsibilities(ell, log_pi)
    return dict(mu=mu, s=s, nu=nu, ell=ell, q=q, taus=taus, iters=iters, status=status,
                gammas=gam, xis=xis, tasks=np.array(tasks))


def mstep(mu, s, q, alpha_old, alpha_max=1e10):
    """alpha update of Eq. (mstep) with the guards described in the module docstring."""
    mu = np.asarray(mu, np.float64); s = np.asarray(s, np.float64); q = np.asarray(q, np.float64)
    alpha_old = np.asarray(alpha_old, np.float64)
    new = alpha_old.copy()
    for c in range(alpha_old.shape[0]):
        use = np.isfinite(q[:, c])                                  # tasks entering the sums
        Nq = q[use, c].sum()
        den = q[use, c] @ (mu[use, c] ** 2 + s[use, c])             # D
        if Nq < 1e-300:
            continue
        floor = Nq / alpha_max
        with np.errstate(invalid="ignore"):
            upd = np.where(den > floor, Nq / np.where(den > floor, den, 1.0), alpha_max)
        new[c] = np.where(np.isfinite(den), upd, alpha_old[c])
    return new


def update_log_pi(q):
    """log pi_c = log((1/T) sum_t q_tc): the mixture-weight M-step when pi is learned (Sec. 2,
    model of Eq. (cmtcs)).  A cluster whose responsibilities are all zero gets -inf."""
    q = np.asarray(q, np.float64)
    with np.errstate(divide="ignore"):
        return np.log(q.sum(axis=0) / q.shape[0])


def log_likelihood(ell, log_pi, const):
    """L-hat(theta) = (1/T) sum_t log sum_c pi_c exp(ell_tc / 2 + const_t) (Sec. 2)."""
    z = 0.5 * np.asarray(ell) + np.asarray(log_pi)[None, :] + np.asarray(const)[:, None]
    m = z.max(axis=1, keepdims=True)
    return float(np.mean(m[:, 0] + np.log(np.exp(z - m).sum(axis=1))))


def fit(Phi, y, beta, alpha0, log_pi, K, policy, n_em, seed=1, probes_fn=None, alpha_max=1e10,
        learn_pi=False, common_probes=False, precond=None):
    """Alg. 2 end to end.  ``probes_fn(it)`` may supply explicit probes per EM iteration.  With
    ``learn_pi`` each M-step also replaces log_pi by ``update_log_pi(q)``."""
    b = rhs(Phi, y, beta)
    const = log_norm_const(Phi, y, beta)
    alpha = np.asarray(alpha0, np.float64).copy()
    log_pi = np.asarray(log_pi, np.float64).copy()
    hist = []
    out = None
    for it in range(n_em):
        pr = None if probes_fn is None else probes_fn(it)
        out = estep(Phi, b, beta, alpha, log_pi, K, policy, seed=seed, it=it, probes=pr,
                    common_probes=common_probes, precond=precond)
        hist.append(dict(L=log_likelihood(out["ell"], log_pi, const), alpha=alpha.copy(),
                         q=out["q"].copy(), ell=out["ell"].copy(), log_pi=log_pi.copy()))
        alpha = mstep(out["mu"], out["s"], out["q"], alpha, alpha_max)
        if learn_pi:
            log_pi = update_log_pi(out["q"])
    assign = np.argmax(out["q"], axis=1)
    recon = np.stack([out["mu"][t, assign[t]] for t in range(len(Phi))])
    return dict(alpha=alpha, q=out["q"], assign=assign, recon=recon, mu=out["mu"], s=out["s"],
                log_pi=log_pi, history=hist)
