"""Jacobi-preconditioned CG (opts.precond; not in the paper) on the device against the oracle's
preconditioned E-step (oracle/cofem.py, precond="jacobi", pinned in tests/test_oracle_pcg.py):
M = diag(A_tc), probe right-hand sides M^1/2 p, the log-determinant corrected by sum log M and
the diagonal estimate rescaled by M^-1/2."""

import numpy as np
import pytest
import torch

import synth
from oracle import cofem, cg as ocg, dense_em
from gpu_common import DEV, device_model, alpha_dev, log_pi_dev
from test_gpu_estep import _run, _assert, _assert_fixed

pytestmark = pytest.mark.gpu


def _pruned(alpha, every=3, value=1e8):
    """alpha with every `every`-th coordinate pruned (set large), as EM leaves it after a few
    iterations (Eq. (mstep) drives alpha of coordinates outside the support to its cap)."""
    a = np.asarray(alpha, np.float64).copy()
    a[:, ::every] = value
    return a


def _tiny():
    return synth.make(synth.Config("tiny-conv", T=4, C=2, D=64, N=32, sparsity=6, groups=2, K=16,
                                   tol=1e-13, max_iters=640))


@pytest.mark.parametrize("math", ["f64", "f32"])
def test_estep_jacobi_tiny_converged(math):
    """Converged CG on the tiny problem with pruned coordinates: the preconditioned E-step
    against the oracle's at the fixed 1e-5 bar (FP32: beta = 1 and alpha + 1, where FP32 can
    meet it), and fewer CG steps than without the preconditioner."""
    w = _tiny() if math == "f64" else synth.make(synth.Config(
        "tiny-conv-wc", T=4, C=2, D=64, N=32, sparsity=6, groups=2, K=16, tol=1e-9,
        max_iters=640, sigma=1.0))
    alpha = _pruned(w.alpha0 + (0.0 if math == "f64" else 1.0))
    err, g, ref, sp = _run(w, range(w.T), math=math, alpha=alpha, spread=False, precond=True)
    _assert_fixed(err)
    plain = device_model(w, math=math).estep(alpha_dev(alpha), log_pi_dev(w.log_pi), w.cfg.K,
                                             tol=w.cfg.tol, max_iters=w.cfg.max_iters,
                                             stats=True)
    it_pc, it_plain = g["iters"].double().mean().item(), plain["iters"].double().mean().item()
    print("mean CG steps: Jacobi %.1f, plain %.1f" % (it_pc, it_plain))
    assert it_pc < it_plain


def test_estep_jacobi_fp32_config_f64():
    """The plain FP32 configuration's shape (T=32, C=4, D=1024, N=256, K=32) in FP64 with pruned
    coordinates, 100 fixed CG steps (the paper's U-step mode); bar as for the unpreconditioned
    E-step (1e-5, or 4x the oracle's own summation-order spread where that is larger).  In
    tolerance mode the preconditioned residual of some columns oscillates over three decades
    around tol 1e-6 for tens of steps (it is not monotone in CG), so the step at which such a
    column first crosses the tolerance -- and its mu -- moves with the rounding order."""
    w = synth.make("fp32", fixed_iters=100)
    err, g, ref, sp = _run(w, [0, 9, 18, 31], alpha=_pruned(w.alpha0), precond=True)
    _assert(err, sp)


def test_solve_jacobi_matches_oracle_pcg():
    """cmtcs_solve with the preconditioner on a problem whose preconditioned system is well
    conditioned (beta = 1, alpha in (1, 2) with every fourth coordinate at 1e6): the first step
    size against its closed form gamma_1 = b^T M^-1 b / z^T A z (z = M^-1 b, M = diag A), the
    whole gamma/xi histories and the step counts against the oracle's preconditioned CG, and
    the solutions against the dense solve."""
    w = synth.make(synth.Config("pcg-solve", T=3, C=2, D=96, N=[40, 0, 70], sparsity=4,
                                groups=1, K=0, sigma=1.0))
    R = 5
    rng = np.random.default_rng(9)
    B = rng.standard_normal((w.T, R, w.cfg.D))
    cc = rng.integers(0, 2, (w.T, R)).astype(np.int32)
    alpha = _pruned(w.alpha0 + 1.0, every=4, value=1e6).astype(np.float32).astype(np.float64)
    m = device_model(w, K=0, max_rhs=R, max_iters=400)
    out = m.solve(alpha_dev(alpha), torch.tensor(B, device=DEV), cc, tol=1e-10, max_iters=400,
                  coefs=True, stats=True, precond=True)
    X, g, xi, it = (out[k].cpu().numpy() for k in ("X", "gamma", "xi", "iters"))
    for t in range(w.T):
        P = w.phi(t).astype(np.float64)
        G = w.beta * P.T @ P
        mcol = np.stack([np.diag(G) + alpha[c] for c in cc[t]], axis=1)
        for j in range(R):
            A = G + np.diag(alpha[cc[t, j]])
            z = B[t, j] / mcol[:, j]
            g1 = (B[t, j] @ z) / (z @ A @ z)
            print("t=%d j=%d gamma_1 device %.15e closed form %.15e" % (t, j, g[t, j, 0], g1))
            assert abs(g[t, j, 0] - g1) <= 1e-12 * abs(g1)
        ap = lambda V, cols: G @ V + alpha[cc[t][cols]].T * V
        Xr, gr, xr, itr, _ = ocg.pcg(ap, B[t].T, ocg.CGPolicy(tol=1e-10, max_iters=400), mcol)
        print("t=%d steps device %s oracle %s" % (t, it[t], itr))
        assert np.max(np.abs(it[t] - itr)) <= 1, (t, it[t], itr)
        for j in range(R):
            x = np.linalg.solve(G + np.diag(alpha[cc[t, j]]), B[t, j])
            assert np.linalg.norm(X[t, j] - x) <= 1e-8 * np.linalg.norm(x)
            n = max(0, min(it[t, j], itr[j]) - 3)
            assert np.allclose(g[t, j, :n], gr[j][:n], rtol=1e-8, atol=0)
            assert np.allclose(xi[t, j, :n], xr[j][:n], rtol=1e-8, atol=0)


def test_jacobi_hadamard_trajectory_equals_dense_em():
    """20 EM iterations on the tiny problem with Hadamard probes (K = D) and converged
    preconditioned CG: the rescaled estimators are exact, so the trajectory is dense EM's (bar
    1e-6, as for the unpreconditioned trajectory: alpha is float32 in the library)."""
    from paper_2310_00420_amd import fit
    w = synth.make("tiny")
    D, C, n_em = w.cfg.D, w.cfg.C, 20
    H = synth.hadamard(6)
    pr = torch.tensor(np.ascontiguousarray(np.broadcast_to(H[None, None], (w.T, C, D, D)),
                                           dtype=np.int8), device=DEV)
    m = device_model(w, K=D, max_iters=10 * D)
    hist = []

    def keep(it, alpha, out):
        hist.append((alpha.cpu().numpy().astype(np.float64), out["ell"].cpu().numpy()))

    out = fit(m, alpha_dev(w.alpha0), log_pi_dev(w.log_pi), D, n_em, tol=1e-13,
              max_iters=10 * D, probes_fn=lambda it: pr, callback=keep, precond=True)
    ref = dense_em.fit(w.phi_list(), w.y_list(), w.beta, w.alpha0, w.log_pi, n_em)
    const = cofem.log_norm_const(w.phi_list(), w.y_list(), w.beta)
    worst_a = worst_L = 0.0
    for (a, ell), hr in zip(hist, ref["history"]):
        L = cofem.log_likelihood(ell, w.log_pi, const)
        worst_L = max(worst_L, abs(L - hr["L"]) / abs(hr["L"]))
        worst_a = max(worst_a, np.max(np.abs(1 / a - 1 / hr["alpha"])) / np.max(1 / hr["alpha"]))
    print("\nJacobi, 20 EM iterations vs dense EM: 1/alpha %.2e, L %.2e" % (worst_a, worst_L))
    assert worst_a <= 1e-6 and worst_L <= 1e-6
    assert np.array_equal(out["assign"], ref["assign"])


def test_em_iter_graph_jacobi_matches_step_by_step():
    """The recorded EM iteration with the preconditioner replays bit-identically to the
    step-by-step calls, over three iterations."""
    w = synth.make("fp32", T=8)
    kw = dict(tol=w.cfg.tol, max_iters=w.cfg.max_iters, seed=1, precond=True)
    res = []
    for graph in (False, True):
        m = device_model(w)
        a = alpha_dev(w.alpha0)
        lp = log_pi_dev(w.log_pi)
        out = None
        for it in range(3):
            out = m.em_iter(a, lp, w.cfg.K, out=out, em_iter=it, graph=graph, **kw)
        torch.cuda.synchronize()
        res.append((a.clone(), {k: v.clone() for k, v in out.items()}))
        m.close()
    assert torch.equal(res[0][0], res[1][0])
    for k in res[0][1]:
        assert torch.equal(res[0][1][k], res[1][1][k]), k
