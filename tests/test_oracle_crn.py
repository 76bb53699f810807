"""Pins of the common-random-number probes (one probe set per task, shared by its clusters): a
variance-reduction variant of the estimators of Sec. 3.1 and 3.2, not in the paper."""

import numpy as np
import pytest

import synth
from oracle import cg, cofem, dense_em


@pytest.fixture(scope="module")
def setup():
    w = synth.make("tiny")
    Phi, y = w.phi_list(), w.y_list()
    b = cofem.rhs(Phi, y, w.beta)
    alpha = np.stack([w.alpha0[0], w.alpha0[0] * 1.2])       # two similar clusters
    exact = dense_em.estep(Phi, b, w.beta, alpha)
    pol = cg.CGPolicy(fixed_iters=w.cfg.D)                   # full-length CG: MC error only
    draws = {}
    for crn in (False, True):
        draws[crn] = np.stack([cofem.estep(Phi, b, w.beta, alpha, w.log_pi, w.cfg.K, pol,
                                           seed=s, common_probes=crn)["ell"]
                               for s in range(1, 41)])       # [seed][t][c]
    return w, exact, draws


def test_each_estimator_keeps_its_distribution(setup):
    """Sharing probes across clusters leaves every ell_tc unbiased for the exact value (Hutchinson
    and stochastic Lanczos quadrature per (t, c) see the same probe law)."""
    w, exact, draws = setup
    ell = draws[True]
    z = (ell.mean(0) - exact["ell"]) / (ell.std(0, ddof=1) / np.sqrt(len(ell)))
    assert np.all(np.abs(z) < 4.5), z


def test_difference_of_clusters_varies_less(setup):
    """The difference ell_t0 - ell_t1, which decides q_t, has a much smaller Monte Carlo spread
    with common probes than with independent ones, and stays centred on the exact difference."""
    w, exact, draws = setup
    dif = {k: v[:, :, 0] - v[:, :, 1] for k, v in draws.items()}
    v_ind, v_crn = dif[False].var(0, ddof=1), dif[True].var(0, ddof=1)
    print("\nvar(ell_t0 - ell_t1): independent", v_ind, "common", v_crn)
    assert np.all(v_crn < 0.25 * v_ind)
    ex = exact["ell"][:, 0] - exact["ell"][:, 1]
    z = (dif[True].mean(0) - ex) / np.sqrt(v_crn / len(dif[True]))
    assert np.all(np.abs(z) < 4.5), z


def test_identical_clusters_give_identical_estimates():
    """With equal alphas, shared probes make the two clusters' systems and right-hand sides
    identical, so their estimates agree exactly; independent probes do not."""
    w = synth.make("tiny")
    Phi, y = w.phi_list(), w.y_list()
    b = cofem.rhs(Phi, y, w.beta)
    alpha = np.stack([w.alpha0[0], w.alpha0[0]])
    pol = cg.CGPolicy(fixed_iters=w.cfg.D)
    e1 = cofem.estep(Phi, b, w.beta, alpha, w.log_pi, w.cfg.K, pol, common_probes=True)
    e0 = cofem.estep(Phi, b, w.beta, alpha, w.log_pi, w.cfg.K, pol, common_probes=False)
    assert np.array_equal(e1["ell"][:, 0], e1["ell"][:, 1])
    assert np.array_equal(e1["s"][:, 0], e1["s"][:, 1])
    assert not np.allclose(e0["ell"][:, 0], e0["ell"][:, 1], rtol=1e-6, atol=0)
