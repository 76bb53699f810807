"""Pins of the dense EM and CoFEM oracles (Eqs. (estep), (mstep), (diag-est), Alg. 2)."""

import numpy as np
import pytest
from scipy.stats import multivariate_normal

import synth
from oracle import cg, cofem, dense_em


@pytest.fixture(scope="module")
def tiny():
    return synth.make("tiny")


def _Q(alpha, q, mu, var):
    """Q(theta | theta-hat) of Eq. (q-func) up to constants (the factor 1/(TC) is irrelevant)."""
    return np.sum(q[:, :, None] * (0.5 * np.log(alpha)[None] - 0.5 * alpha[None] * (mu ** 2 + var)))


def test_ell_is_gaussian_marginal_loglik(tiny):
    w = tiny
    Phi, y = w.phi_list(), w.y_list()
    b = cofem.rhs(Phi, y, w.beta)
    e = dense_em.estep(Phi, b, w.beta, w.alpha0)
    const = cofem.log_norm_const(Phi, y, w.beta)
    for t in range(w.T):
        P = Phi[t].astype(np.float64)
        for c in range(w.cfg.C):
            S = np.eye(P.shape[0]) / w.beta + P @ np.diag(1.0 / w.alpha0[c]) @ P.T
            ref = multivariate_normal.logpdf(y[t].astype(np.float64), np.zeros(P.shape[0]), S)
            assert np.isclose(0.5 * e["ell"][t, c] + const[t], ref, rtol=1e-9, atol=1e-7)


def test_dense_em_monotone_and_q_simplex(tiny):
    w = tiny
    r = dense_em.fit(w.phi_list(), w.y_list(), w.beta, w.alpha0, w.log_pi, n_em=20)
    L = [h["L"] for h in r["history"]]
    assert all(L[i + 1] >= L[i] - 1e-7 * abs(L[i]) for i in range(len(L) - 1))
    for h in r["history"]:
        assert np.allclose(h["q"].sum(axis=1), 1.0, atol=1e-14)
    # the true grouping {0,1},{2,3} is recovered
    a = r["assign"]
    assert a[0] == a[1] and a[2] == a[3] and a[0] != a[2]


def test_mstep_is_stationary_point_of_Q(tiny):
    w = tiny
    Phi, y = w.phi_list(), w.y_list()
    b = cofem.rhs(Phi, y, w.beta)
    e = dense_em.estep(Phi, b, w.beta, w.alpha0)
    q = cofem.responsibilities(e["ell"], w.log_pi)
    a_new = dense_em.mstep(e["mu"], e["var"], q)
    Q0 = _Q(a_new, q, e["mu"], e["var"])
    h = 1e-5
    for c, d in [(0, 0), (1, 5), (0, 63), (1, 31)]:
        ap = a_new.copy(); am = a_new.copy()
        ap[c, d] *= 1 + h; am[c, d] *= 1 - h
        grad = (_Q(ap, q, e["mu"], e["var"]) - _Q(am, q, e["mu"], e["var"])) / (2 * h * a_new[c, d])
        assert abs(grad) < 1e-6 * abs(Q0) / a_new[c, d] + 1e-8
        # and it is a maximum
        assert _Q(ap, q, e["mu"], e["var"]) < Q0 and _Q(am, q, e["mu"], e["var"]) < Q0


def test_identity_sensing_closed_forms():
    D, beta = 16, 3.0
    rng = np.random.default_rng(5)
    alpha = rng.uniform(0.2, 2.0, (1, D))
    y = rng.standard_normal(D)
    b = cofem.rhs([np.eye(D)], [y], beta)
    e = dense_em.estep([np.eye(D)], b, beta, alpha)
    assert np.allclose(e["mu"][0, 0], beta * y / (beta + alpha[0]), rtol=1e-13)
    assert np.allclose(e["var"][0, 0], 1.0 / (beta + alpha[0]), rtol=1e-13)
    assert np.isclose(e["logdet"][0, 0], -np.sum(np.log(beta + alpha[0])), rtol=1e-13)
    # single cluster, single task: the update is 1 / (mu_d^2 + Sigma_dd)
    a = dense_em.mstep(e["mu"], e["var"], np.ones((1, 1)))
    assert np.allclose(a[0], 1.0 / (e["mu"][0, 0] ** 2 + e["var"][0, 0]), rtol=1e-13)


def test_hadamard_probes_make_cofem_exact(tiny):
    """With K = D Hadamard probes and converged CG, s = diag Sigma and nu-bar = log det Sigma
    exactly, so one CoFEM E-step equals the dense E-step."""
    w = tiny
    Phi, y = w.phi_list(), w.y_list()
    b = cofem.rhs(Phi, y, w.beta)
    D, C = w.cfg.D, w.cfg.C
    H = synth.hadamard(6)                                   # 64 x 64
    pr = np.broadcast_to(H[None, None], (w.T, C, D, D))
    pol = cg.CGPolicy(tol=1e-13, max_iters=10 * D)
    o = cofem.estep(Phi, b, w.beta, w.alpha0, w.log_pi, D, pol, probes=pr)
    e = dense_em.estep(Phi, b, w.beta, w.alpha0)
    # kappa(A) is up to ~1e6 here, so a CG residual of 1e-13 bounds the mean's error by ~1e-7;
    # observed: mu 1.6e-9, s 1.7e-11, nu-bar 1.1e-12 relative; ell 1.7e-9 absolute
    assert np.max(np.abs(o["mu"] - e["mu"])) <= 1e-8 * np.max(np.abs(e["mu"]))
    assert np.max(np.abs(o["s"] - e["var"]) / e["var"]) < 1e-9
    assert np.max(np.abs(o["nu"] - e["logdet"]) / np.abs(e["logdet"])) < 1e-10
    assert np.max(np.abs(o["ell"] - e["ell"])) < 1e-7
    q = cofem.responsibilities(e["ell"], w.log_pi)
    assert np.max(np.abs(o["q"] - q)) < 1e-8


def test_hadamard_cofem_trajectory_equals_dense_em(tiny):
    w = tiny
    D, C = w.cfg.D, w.cfg.C
    H = synth.hadamard(6)
    pr = np.broadcast_to(H[None, None], (w.T, C, D, D))
    n_em = 20
    ref = dense_em.fit(w.phi_list(), w.y_list(), w.beta, w.alpha0, w.log_pi, n_em)
    got = cofem.fit(w.phi_list(), w.y_list(), w.beta, w.alpha0, w.log_pi, D,
                    cg.CGPolicy(tol=1e-13, max_iters=10 * D), n_em, probes_fn=lambda it: pr)
    for hr, hg in zip(ref["history"], got["history"]):
        assert np.isclose(hg["L"], hr["L"], rtol=1e-9)
        # prior variances 1/alpha are the well-conditioned quantity
        assert np.max(np.abs(1 / hg["alpha"] - 1 / hr["alpha"])) <= 1e-6 * np.max(1 / hr["alpha"])
    assert np.array_equal(got["assign"], ref["assign"])


def test_rademacher_estimators_unbiased(tiny):
    """E[s] = diag Sigma and E[nu] = log det Sigma (Hutchinson), checked by z-scores over
    independent probe draws, with full-length CG so only the Monte Carlo error remains."""
    w = tiny
    Phi, y = w.phi_list()[:1], w.y_list()[:1]
    b = cofem.rhs(Phi, y, w.beta)
    alpha = w.alpha0[:1]
    e = dense_em.estep(Phi, b, w.beta, alpha)
    pol = cg.CGPolicy(tol=1e-12, max_iters=640)
    s_list, nu_list = [], []
    for seed in range(40):
        o = cofem.estep(Phi, b, w.beta, alpha, np.zeros(1), 16, pol, seed=seed)
        s_list.append(o["s"][0, 0]); nu_list.append(o["nu"][0, 0])
    s = np.array(s_list); nu = np.array(nu_list)
    z_s = (s.mean(0) - e["var"][0, 0]) / (s.std(0, ddof=1) / np.sqrt(len(s)) + 1e-300)
    assert np.mean(np.abs(z_s) < 3.5) > 0.97
    z_nu = (nu.mean() - e["logdet"][0, 0]) / (nu.std(ddof=1) / np.sqrt(len(nu)))
    assert abs(z_nu) < 4.0


def test_estimator_error_decays_like_inverse_sqrt_K(tiny):
    w = tiny
    Phi, y = w.phi_list()[:1], w.y_list()[:1]
    b = cofem.rhs(Phi, y, w.beta)
    alpha = w.alpha0[:1]
    e = dense_em.estep(Phi, b, w.beta, alpha)
    pol = cg.CGPolicy(tol=1e-12, max_iters=640)
    Ks = [4, 16, 64]
    errs = []
    for K in Ks:
        err = []
        for seed in range(12):
            o = cofem.estep(Phi, b, w.beta, alpha, np.zeros(1), K, pol, seed=100 + seed)
            err.append(np.linalg.norm(o["s"][0, 0] - e["var"][0, 0]) / np.linalg.norm(e["var"][0, 0]))
        errs.append(np.sqrt(np.mean(np.square(err))))
    slope = np.polyfit(np.log(Ks), np.log(errs), 1)[0]
    assert -0.65 < slope < -0.35


def test_mstep_guards():
    mu = np.zeros((2, 2, 3)); s = np.ones((2, 2, 3))
    s[:, 0, 1] = -5.0                                # negative MC variance: denominator < 0
    q = np.array([[1.0, 0.0], [1.0, 0.0]])           # cluster 1 is empty
    old = np.full((2, 3), 7.0)
    a = cofem.mstep(mu, s, q, old, alpha_max=1e10)
    assert np.allclose(a[0], [1.0, 1e10, 1.0])
    assert np.array_equal(a[1], old[1])


def test_mstep_skips_failed_tasks():
    """A task whose q is NaN (all of its probes left out of nu-bar) drops out of the sums: the
    result equals the M-step over the other tasks; a non-finite mu entry keeps its old alpha."""
    rng = np.random.default_rng(3)
    mu = rng.standard_normal((4, 2, 5)); s = rng.random((4, 2, 5))
    q = rng.random((4, 2)); q /= q.sum(1, keepdims=True)
    old = np.full((2, 5), 3.0)
    bad = q.copy(); bad[2] = np.nan
    a = cofem.mstep(mu, s, bad, old)
    keep = [0, 1, 3]
    ref = cofem.mstep(mu[keep], s[keep], q[keep], old)
    assert np.array_equal(a, ref)
    # closed form of the kept tasks: alpha_cd = sum_t q / sum_t q (mu^2 + s)
    assert np.allclose(a, q[keep].sum(0)[:, None]
                       / np.einsum("tc,tcd->cd", q[keep], mu[keep] ** 2 + s[keep]), rtol=1e-14)
    mu2 = mu.copy(); mu2[1, 0, 3] = np.inf
    a2 = cofem.mstep(mu2, s, q, old)
    assert a2[0, 3] == 3.0 and np.array_equal(np.delete(a2[0], 3), np.delete(cofem.mstep(mu, s, q, old)[0], 3))


def test_responsibilities_are_bayes_posterior(tiny):
    """q_tc = pi_c N(y_t; 0, S_c) / sum_c' pi_c' N(y_t; 0, S_c') with S_c the marginal covariance,
    and L-hat = mean_t log sum_c pi_c N(y_t; 0, S_c), evaluated with scipy's Gaussian density."""
    w = tiny
    Phi, y = w.phi_list(), w.y_list()
    b = cofem.rhs(Phi, y, w.beta)
    alpha = w.alpha0 * np.array([[1.0], [3.0]])          # make the clusters differ
    log_pi = np.log([0.3, 0.7])
    e = dense_em.estep(Phi, b, w.beta, alpha)
    q = cofem.responsibilities(e["ell"], log_pi)
    L = cofem.log_likelihood(e["ell"], log_pi, cofem.log_norm_const(Phi, y, w.beta))
    Lref = 0.0
    for t in range(w.T):
        P = Phi[t].astype(np.float64)
        lp = np.array([multivariate_normal.logpdf(
            y[t].astype(np.float64), np.zeros(P.shape[0]),
            np.eye(P.shape[0]) / w.beta + P @ np.diag(1.0 / alpha[c]) @ P.T) for c in range(2)])
        z = lp + log_pi
        ref = np.exp(z - z.max()) / np.exp(z - z.max()).sum()
        assert np.allclose(q[t], ref, rtol=1e-8, atol=1e-12)
        Lref += (z.max() + np.log(np.exp(z - z.max()).sum())) / w.T
    assert np.isclose(L, Lref, rtol=1e-10)
