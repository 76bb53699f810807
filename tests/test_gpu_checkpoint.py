"""Checkpoint and resume of Alg. 2, and the device log-likelihood estimate.

* Probes are drawn from a counter-based generator keyed by (seed, EM iteration), so an EM run
  interrupted after k iterations and resumed from the saved alpha (and log pi) with
  start_iter = k continues it exactly: the final alpha, q, mu and ell equal those of an
  uninterrupted run bit for bit (step-by-step and graph-replayed iterations, learned pi).
* cmtcs_log_likelihood against the oracle's formula for Lhat (Sec. 2) on the same ell, and
  its per-task values against the dense EM oracle's exact marginal likelihood where ell is
  exact (Hadamard probes, converged CG)."""

import io

import numpy as np
import pytest
import torch

import synth
from oracle import cofem, dense_em
from paper_2310_00420_amd import fit
from gpu_common import DEV, alpha_dev, device_model, log_pi_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("graph,learn_pi", [(False, False), (True, False), (False, True)])
def test_resume_equals_uninterrupted(graph, learn_pi):
    w = synth.make("fp32", T=6)
    cfg = w.cfg
    kw = dict(tol=cfg.tol, max_iters=cfg.max_iters, seed=7, graph=graph, learn_pi=learn_pi)
    m = device_model(w)
    full = fit(m, alpha_dev(w.alpha0), log_pi_dev(w.log_pi), cfg.K, 5, **kw)
    torch.cuda.synchronize()
    m.close()
    # first 2 iterations, checkpoint through a byte buffer, then a fresh handle resumes
    m = device_model(w)
    part = fit(m, alpha_dev(w.alpha0), log_pi_dev(w.log_pi), cfg.K, 2, **kw)
    buf = io.BytesIO()
    torch.save({"alpha": part["alpha"].cpu(), "log_pi": part["log_pi"].cpu(), "next": 2}, buf)
    m.close()
    buf.seek(0)
    ck = torch.load(buf, weights_only=True)
    m = device_model(w)
    rest = fit(m, ck["alpha"].to(DEV), ck["log_pi"].to(DEV), cfg.K, 3, start_iter=ck["next"], **kw)
    torch.cuda.synchronize()
    m.close()
    for k in ("alpha", "q", "mu", "ell", "log_pi"):
        assert torch.equal(full[k], rest[k]), k
    assert np.array_equal(full["assign"], rest["assign"])


def test_log_likelihood_matches_oracle_formula():
    w = synth.make("fp32", T=8)
    cfg = w.cfg
    m = device_model(w)
    lp = log_pi_dev(np.log([0.1, 0.2, 0.3, 0.4]))
    g = m.estep(alpha_dev(w.alpha0), lp, cfg.K, tol=cfg.tol, max_iters=cfg.max_iters)
    Lt, L = m.log_likelihood(g["ell"], lp)
    torch.cuda.synchronize()
    ell = g["ell"].cpu().numpy()
    const = cofem.log_norm_const(w.phi_list(), w.y_list(), w.beta)
    ref = cofem.log_likelihood(ell, lp.cpu().numpy(), const)
    z = 0.5 * ell + lp.cpu().numpy()[None] + const[:, None]
    ref_t = z.max(1) + np.log(np.exp(z - z.max(1, keepdims=True)).sum(1))
    print("\nLhat device %.12e oracle %.12e" % (L.item(), ref))
    assert abs(L.item() - ref) <= 1e-12 * abs(ref)
    assert np.allclose(Lt.cpu().numpy(), ref_t, rtol=1e-12, atol=0)
    m.close()


def test_log_likelihood_exact_with_exact_ell():
    """Hadamard probes (K = D) and converged CG make ell exact, so L_t is the exact marginal
    log-likelihood log sum_c pi_c N(y_t; 0, beta^-1 I + Phi_t A_c^-1 Phi_t^T) that dense EM's
    ell gives; an empty task has L_t = 0 (no measurements)."""
    w = synth.make(synth.Config("ll", T=3, C=2, D=64, N=[32, 0, 50], sparsity=4, groups=2,
                                K=64, tol=1e-13, max_iters=640))
    m = device_model(w)
    H = synth.hadamard(6)
    pr = torch.tensor(np.ascontiguousarray(np.broadcast_to(H[None, None], (w.T, 2, 64, 64)),
                                           dtype=np.int8), device=DEV)
    lp = log_pi_dev(w.log_pi)
    g = m.estep(alpha_dev(w.alpha0), lp, 64, tol=1e-13, max_iters=640, probes=pr)
    Lt, _ = m.log_likelihood(g["ell"], lp)
    torch.cuda.synchronize()
    b = cofem.rhs(w.phi_list(), w.y_list(), w.beta)
    ref = dense_em.estep(w.phi_list(), b, w.beta, w.alpha0)
    const = cofem.log_norm_const(w.phi_list(), w.y_list(), w.beta)
    z = 0.5 * ref["ell"] + w.log_pi[None] + const[:, None]
    ref_t = z.max(1) + np.log(np.exp(z - z.max(1, keepdims=True)).sum(1))
    got = Lt.cpu().numpy()
    print("\nL_t device", got, "dense EM", ref_t)
    assert np.allclose(got, ref_t, rtol=1e-9, atol=1e-9)
    assert got[1] == pytest.approx(0.0, abs=1e-9)
    m.close()
