"""Learned cluster weights on the device (cmtcs_mstep_pi): the mixture-weight M-step that the
model of Sec. 2 allows in place of a known pi, against the FP64 oracle."""

import numpy as np
import pytest
import torch

import synth
from gpu_common import DEV, device_model, alpha_dev, log_pi_dev, rel_cols
from oracle import cg as ocg, cofem
from paper_2310_00420_amd import fit

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("T,C", [(7, 4), (1, 1), (67, 3)])
def test_mstep_pi_parity(T, C):
    """log pi from identical FP64 q, including a cluster with no mass (-inf) where C > 1."""
    rng = np.random.default_rng(11 + T)
    q = rng.dirichlet(np.full(C, 0.7), size=T)
    if C > 1:
        q[:, -1] = 0.0
        q /= q.sum(1, keepdims=True)
    ref = cofem.update_log_pi(q)
    w = synth.make(synth.Config("pi", T=T, C=C, D=64, N=8, sparsity=3, groups=1, K=1))
    m = device_model(w)
    lp = log_pi_dev(np.zeros(C))
    m.mstep_pi(torch.tensor(q, device=DEV), lp)
    got = lp.cpu().numpy()
    fin = np.isfinite(ref)
    print("\nT=%d C=%d log pi %s max err %.2e" % (T, C, got, np.max(np.abs(got[fin] - ref[fin]))))
    assert np.array_equal(np.isfinite(got), fin)
    assert np.all(got[~fin] == -np.inf)
    assert np.max(np.abs(got[fin] - ref[fin])) <= 1e-14
    assert abs(np.exp(got[fin]).sum() - 1.0) <= 1e-14


def test_em_with_learned_pi_tracks_oracle():
    """Three EM iterations with learned weights from a wrong prior (0.8, 0.2), converged CG: the
    weights, alpha and the assignments follow the oracle's trajectory.  The device keeps alpha,
    mu and s in FP32, which moves log pi by about 4e-8 over these iterations."""
    w = synth.make(synth.Config("tiny-conv", T=4, C=2, D=64, N=32, sparsity=6, groups=2, K=16,
                                tol=1e-13, max_iters=640))
    lp0 = np.log([0.8, 0.2])
    m = device_model(w)
    out = fit(m, alpha_dev(w.alpha0), log_pi_dev(lp0), w.cfg.K, 3, tol=1e-13, max_iters=640,
              learn_pi=True)
    pol = ocg.CGPolicy(fixed_iters=w.cfg.fixed_iters, tol=w.cfg.tol, max_iters=w.cfg.max_iters)
    ref = cofem.fit(w.phi_list(), w.y_list(), w.beta, w.alpha0, lp0, w.cfg.K, pol, 3, seed=1,
                    learn_pi=True)
    e_pi = float(np.max(np.abs(out["log_pi"].cpu().numpy() - ref["log_pi"])))
    e_alpha = rel_cols(1.0 / out["alpha"].cpu().numpy().astype(np.float64), 1.0 / ref["alpha"])
    print("\nEM x3 learned pi: log pi %s err %.2e, 1/alpha rel %.2e"
          % (out["log_pi"].cpu().numpy(), e_pi, e_alpha))
    assert e_pi <= 1e-6
    assert e_alpha <= 1e-5
    assert np.array_equal(out["assign"], ref["assign"])


def test_fit_graph_with_learned_pi_matches_direct():
    """The recorded EM iteration reads log pi through its pointer, so updating the weights in
    place between replays gives the same trajectory as step-by-step launches, bit for bit."""
    w = synth.make("tiny")
    lp0 = log_pi_dev(np.log([0.7, 0.3]))
    out = []
    for graph in (False, True):
        m = device_model(w)
        out.append(fit(m, alpha_dev(w.alpha0), lp0, w.cfg.K, 4, fixed_iters=w.cfg.fixed_iters,
                       graph=graph, learn_pi=True))
    assert torch.equal(out[0]["log_pi"], out[1]["log_pi"])
    assert torch.equal(out[0]["alpha"], out[1]["alpha"])
    assert torch.equal(out[0]["q"], out[1]["q"])
    assert not torch.equal(out[0]["log_pi"], lp0)           # the caller's weights are not touched
    assert torch.equal(lp0, log_pi_dev(np.log([0.7, 0.3])))
