"""Partial-Fourier sensing (the experiments of Sec. 4: Phi_t = Omega_t F) on the device: the
FFT operator, the one-kernel CG solve and the E-step, against the FP64 oracle run on the dense
real-stacked sensing matrices written out from the DFT's definition (oracle/fourier.py, itself
pinned in tests/test_oracle_fourier.py)."""

import numpy as np
import pytest
import torch

import synth
from oracle import cofem, cg as ocg, fourier as ofourier
from paper_2310_00420_amd import Cmtcs
from gpu_common import DEV, alpha_dev, log_pi_dev, compare_estep, kappa_hat

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _model(w, K=None, max_iters=None, max_rhs=None):
    K = w.cfg.K if K is None else K
    return Cmtcs.partial_fourier(torch.tensor(w.freq, device=DEV), w.row_off,
                                 torch.tensor(w.yc, device=DEV), w.cfg.D, w.beta, w.cfg.C,
                                 max_iters=max_iters or w.cfg.max_iters, max_K=K,
                                 max_rhs=max_rhs)


def _dense(w, tasks):
    D = w.cfg.D
    Phi = [ofourier.sensing_matrix(w.freq_t(t), D) if t in tasks else None for t in range(w.T)]
    y = [ofourier.stack(w.yc_t(t)) if t in tasks else None for t in range(w.T)]
    return Phi, y


def _ragged(D, Ns, T=None, C=2, K=4, **kw):
    return synth.make_fourier(synth.Config("fourier-ragged", T=len(Ns), C=C, D=D, N=list(Ns),
                                           sparsity=max(1, D // 20), groups=min(C, len(Ns)),
                                           K=K, sigma=0.05, **kw))


@pytest.mark.parametrize("D", [64, 128, 512, 1024, 2048, 4096])
def test_operator_matches_oracle(D):
    """A V = beta Re(F^H Omega^T Omega F V) + alpha (.) V on ragged masks (empty, partial, every
    frequency, a quarter), odd and even log2 D, an odd column count (one column paired with
    padding), against the oracle's FFT operator (pinned to the dense matrix)."""
    Ns = [0, 5, D, D // 4]
    w = _ragged(D, Ns)
    R = 5
    rng = np.random.default_rng(D)
    V = rng.standard_normal((w.T, R, D))
    cc = rng.integers(0, w.cfg.C, (w.T, R)).astype(np.int32)
    m = _model(w, K=0, max_rhs=R, max_iters=1)
    AV = m.apply(alpha_dev(w.alpha0), torch.tensor(V, device=DEV), cc).cpu().numpy()
    worst = 0.0
    for t in range(w.T):
        ref = ofourier.apply(w.freq_t(t), D, w.beta, V[t].T).T + w.alpha0[cc[t]] * V[t]
        worst = max(worst, np.max(np.abs(AV[t] - ref)) / np.max(np.abs(ref)))
    print("\nD=%d operator: max entry error / max entry %.2e" % (D, worst))
    assert worst <= 1e-13
    m.close()


def test_solve_matches_oracle_cg():
    """cmtcs_solve on caller right-hand sides: solutions and the gamma/xi histories of Alg. 1
    against the oracle's CG with the same FFT operator, converged (alpha in (1, 2))."""
    D = 256
    w = _ragged(D, [64, 3, 256])
    R = 3
    rng = np.random.default_rng(7)
    B = rng.standard_normal((w.T, R, D))
    cc = np.array([0, 1, 1], np.int32)
    alpha = (w.alpha0 + 1.0).astype(np.float32).astype(np.float64)   # as the device sees it
    m = _model(w, K=0, max_rhs=R, max_iters=400)
    out = m.solve(alpha_dev(alpha), torch.tensor(B, device=DEV), cc, tol=1e-12, max_iters=400,
                  coefs=True, stats=True)
    X, g, xi, it = (out[k].cpu().numpy() for k in ("X", "gamma", "xi", "iters"))
    for t in range(w.T):
        f = w.freq_t(t)
        ac = alpha[cc].T

        def ap(V, cols, f=f, ac=ac):
            return ofourier.apply(f, D, w.beta, V) + ac[:, cols] * V

        Xr, gr, xr, itr, _ = ocg.cg(ap, B[t].T, ocg.CGPolicy(tol=1e-12, max_iters=400))
        # the step at which a column crosses tol 1e-12 may move by one with the rounding order
        assert np.max(np.abs(it[t] - itr)) <= 1, (it[t], itr)
        for j in range(R):
            assert np.linalg.norm(X[t, j] - Xr[:, j]) <= 1e-10 * np.linalg.norm(Xr[:, j])
            # the step sizes agree closely while the residual is well above rounding level (the
            # first half of the steps, residual reduced to ~1e-6); later gamma and xi are ratios
            # of residuals within a few digits of FP64 noise (relative rounding ~ u kappa ||b||
            # / ||r||), where FFT and dense products part
            n = min(it[t, j], itr[j]) // 2
            assert np.allclose(g[t, j, :n], gr[j][:n], rtol=1e-9, atol=0)
            assert np.allclose(xi[t, j, :n], xr[j][:n], rtol=1e-9, atol=0)
    m.close()


def _estep_parity(w, tasks, alpha=None):
    # the library takes alpha in float32: the oracle gets the same values
    alpha = np.asarray(w.alpha0 if alpha is None else alpha, np.float32).astype(np.float64)
    cfg = w.cfg
    m = _model(w)
    g = m.estep(alpha_dev(alpha), log_pi_dev(w.log_pi), cfg.K, tol=cfg.tol,
                max_iters=cfg.max_iters, stats=True)
    torch.cuda.synchronize()
    Phi, y = _dense(w, tasks)
    b = [None] * w.T
    for t in tasks:
        b[t] = cofem.rhs([Phi[t]], [y[t]], w.beta)[0]
    ref = cofem.estep(Phi, b, w.beta, alpha, w.log_pi, cfg.K,
                      ocg.CGPolicy(tol=cfg.tol, max_iters=cfg.max_iters), seed=1, it=0,
                      t_sel=tasks)
    err = compare_estep(g, ref, tasks)
    it_g = g["iters"].cpu().numpy()[np.asarray(tasks)]
    err["iters_maxdiff"] = int(np.max(np.abs(it_g - ref["iters"].reshape(len(tasks), -1))))
    err["kappa_hat"] = kappa_hat(g, tasks)
    print("\n%s (D=%d) tasks %s: %s" % (cfg.name, cfg.D, list(tasks),
                                        {k: v for k, v in err.items() if k != "per"}))
    assert (g["k_eff"].cpu().numpy() == cfg.K).all()
    for k in ("mu", "s", "mu_inf", "s_inf", "logdet", "ell"):
        assert err[k] <= TOL, (k, err[k])
    assert err["argmax_equal"]
    assert err["iters_maxdiff"] <= 1
    m.close()
    return err


def test_estep_fourier_small():
    """T=4, C=2, D=256, N=64 frequencies per task, K=16, beta = 400 (sigma = 0.05, Sec. 4),
    CG tol 1e-6 with at most 200 steps: every task against the oracle."""
    w = synth.make_fourier("fourier-small")
    _estep_parity(w, list(range(w.T)))


def test_estep_fourier_odd_log_length_ragged():
    """D=512 (a radix-2 stage), ragged N_t including an empty task, C*(K+1) odd, with CG run to
    convergence (alpha in (1, 2), tol 1e-12): the solutions are unique up to rounding.  (At the
    configuration's tol 1e-6 with alpha ~ U(0, 1) the step at which a column crosses the
    tolerance moves by a few steps with the order of the FP64 roundings, FFT against dense
    products, and mu with it.)"""
    w = _ragged(512, [128, 0, 300, 17], C=3, K=6, tol=1e-12, max_iters=400)
    _estep_parity(w, list(range(w.T)), alpha=w.alpha0 + 1.0)


def test_estep_fourier_metric_sizes():
    """The metric's task, cluster, probe and length sizes with the paper's sensing: T=64, C=4,
    D=4096, N=1024 frequencies, K=32, 5% sparse signals, sigma = 0.05, CG tol 1e-6 with at most
    200 steps; all 8448 right-hand sides on the device, the oracle on one task of each of two
    true clusters."""
    w = synth.make_fourier("fourier")
    _estep_parity(w, [0, 40])
