"""Pins of the learned cluster weights: the mixture-weight M-step that the model of Sec. 2
(Eq. (cmtcs)) allows in place of a known pi."""

import numpy as np
import pytest
from scipy.optimize import minimize

import synth
from oracle import cg, cofem, dense_em


@pytest.fixture(scope="module")
def tiny():
    return synth.make("tiny")


def _Qpi(log_pi, q):
    """The pi-dependent part of the expected complete-data log-likelihood: sum_tc q_tc log pi_c."""
    with np.errstate(invalid="ignore"):
        return float(np.sum(np.where(q > 0, q * log_pi[None, :], 0.0)))


def test_one_hot_responsibilities_give_cluster_fractions():
    q = np.zeros((5, 4))
    q[np.arange(5), [0, 0, 1, 2, 0]] = 1.0
    lp = cofem.update_log_pi(q)
    assert np.exp(lp[:3]).tolist() == [3 / 5, 1 / 5, 1 / 5]
    assert lp[3] == -np.inf


def test_update_maximises_expected_log_weights():
    """The simplex maximiser of sum_tc q_tc log pi_c, found two ways without the closed form:
    a numerical optimiser over softmax parameters, and 20000 random points of the simplex,
    none of which may do better."""
    rng = np.random.default_rng(7)
    q = rng.dirichlet(np.full(5, 0.6), size=7)
    lp = cofem.update_log_pi(q)
    assert np.isclose(np.exp(lp).sum(), 1.0, rtol=0, atol=1e-15)
    best = _Qpi(lp, q)

    def neg(theta):
        return -_Qpi(theta - np.log(np.exp(theta).sum()), q)

    r = minimize(neg, np.zeros(5), method="BFGS", options=dict(gtol=1e-12))
    pi_opt = np.exp(r.x) / np.exp(r.x).sum()
    assert np.max(np.abs(pi_opt - np.exp(lp))) < 1e-6
    cand = rng.dirichlet(np.ones(5), size=20000)
    vals = (q.sum(axis=0)[None, :] * np.log(cand)).sum(axis=1)
    assert vals.max() <= best + 1e-12


def test_exact_em_with_learned_pi_is_monotone(tiny):
    """Exact EM that updates both alpha and pi never lowers the marginal likelihood; from a
    wrong prior (0.9, 0.1) on two groups of two tasks the weights move to the group fractions."""
    w = tiny
    r = dense_em.fit(w.phi_list(), w.y_list(), w.beta, w.alpha0, np.log([0.9, 0.1]), n_em=25,
                     learn_pi=True)
    L = [h["L"] for h in r["history"]]
    assert all(L[i + 1] >= L[i] - 1e-9 * abs(L[i]) for i in range(len(L) - 1))
    assert L[-1] > L[0]
    a = r["assign"]
    assert a[0] == a[1] and a[2] == a[3] and a[0] != a[2]
    assert np.allclose(np.exp(r["log_pi"]), [0.5, 0.5], atol=1e-3)
    assert np.isclose(np.exp(r["log_pi"]).sum(), 1.0, rtol=0, atol=1e-14)


def test_learned_pi_cofem_trajectory_equals_exact_em(tiny):
    """With Hadamard probes (exact diagonal and log-determinant) and converged CG, CoFEM with
    learned weights follows exact EM with learned weights."""
    w = tiny
    D, C = w.cfg.D, w.cfg.C
    H = synth.hadamard(6)
    pr = np.broadcast_to(H[None, None], (w.T, C, D, D))
    lp0 = np.log([0.8, 0.2])
    ref = dense_em.fit(w.phi_list(), w.y_list(), w.beta, w.alpha0, lp0, 12, learn_pi=True)
    got = cofem.fit(w.phi_list(), w.y_list(), w.beta, w.alpha0, lp0, D,
                    cg.CGPolicy(tol=1e-13, max_iters=10 * D), 12, probes_fn=lambda it: pr,
                    learn_pi=True)
    for hr, hg in zip(ref["history"], got["history"]):
        assert np.isclose(hg["L"], hr["L"], rtol=1e-9)
        # log pi to 1e-8 absolute is pi to 1e-8 relative; the minor weight passes through 1e-4
        assert np.allclose(hg["log_pi"], hr["log_pi"], rtol=0, atol=1e-8)
    assert np.allclose(got["log_pi"], ref["log_pi"], rtol=0, atol=1e-8)
