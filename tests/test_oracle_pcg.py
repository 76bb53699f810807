"""Pins of the Jacobi-preconditioned variant of the oracle (cg.pcg and cofem.estep with
precond="jacobi"; not in the paper): the preconditioned recurrence, its Lanczos tridiagonal,
and the rescaled diagonal and log-determinant estimators."""

import numpy as np

import synth
from oracle import cg, cofem, dense_em, slq
from test_oracle_slq import _lanczos


def _spd_spread(D=40, N=20, seed=1, beta=50.0):
    """beta Phi^T Phi + diag(alpha) with alpha spread over eight decades (pruned coordinates)."""
    rng = np.random.default_rng(seed)
    Phi = rng.standard_normal((N, D)) / np.sqrt(N)
    alpha = 10.0 ** rng.uniform(-1, 7, D)
    return beta * Phi.T @ Phi + np.diag(alpha)


def test_unit_preconditioner_is_plain_cg():
    A = _spd_spread()
    B = np.random.default_rng(2).standard_normal((A.shape[0], 3))
    pol = cg.CGPolicy(tol=1e-12, max_iters=500)
    ap = lambda V, cols: A @ V
    X1, g1, x1, i1, s1 = cg.cg(ap, B, pol)
    X2, g2, x2, i2, s2 = cg.pcg(ap, B, pol, np.ones_like(B))
    assert np.array_equal(X1, X2) and np.array_equal(i1, i2) and np.array_equal(s1, s2)
    for a, b in zip(g1 + x1, g2 + x2):
        assert np.array_equal(a, b)


def test_converged_pcg_solves_and_needs_fewer_steps():
    A = _spd_spread()
    B = np.random.default_rng(3).standard_normal((A.shape[0], 4))
    pol = cg.CGPolicy(tol=1e-13, max_iters=2000)
    ap = lambda V, cols: A @ V
    m = np.repeat(np.diag(A)[:, None], B.shape[1], axis=1)
    X, g, x, it, st = cg.pcg(ap, B, pol, m)
    ref = np.linalg.solve(A, B)
    assert np.allclose(X, ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())
    assert (st == cg.CONVERGED).all()
    it_plain = cg.cg(ap, B, pol)[3]
    assert it.max() < it_plain.min()


def test_pcg_tridiagonal_is_lanczos_of_the_scaled_operator():
    """PCG's gamma, xi in Eq. (tridiag) give the Lanczos tridiagonal of M^-1/2 A M^-1/2 from
    the start vector M^-1/2 b (textbook Lanczos with full reorthogonalisation)."""
    A = _spd_spread()
    D = A.shape[0]
    b = np.random.default_rng(4).choice([-1.0, 1.0], size=D)
    m = np.diag(A).copy()
    U = 8
    X, g, x, it, st = cg.pcg(lambda V, cols: A @ V, b[:, None], cg.CGPolicy(fixed_iters=U),
                             m[:, None])
    diag, off = slq.tridiagonal(g[0], x[0])
    Ah = A / np.sqrt(np.outer(m, m))
    a, bb = _lanczos(Ah, b / np.sqrt(m), U)
    assert np.allclose(diag, a, rtol=1e-9)
    assert np.allclose(np.abs(off), bb, rtol=1e-9)


def test_hadamard_jacobi_estep_equals_dense_estep():
    """With Hadamard probes (K = D) and converged PCG the rescaled estimators are exact: mu, the
    Sigma diagonal and log det Sigma of dense EM, on the tiny problem with pruned coordinates
    (alpha up to 1e8) where the preconditioner matters."""
    w = synth.make("tiny")
    D, C = w.cfg.D, w.cfg.C
    alpha = w.alpha0.copy()
    alpha[:, ::3] = 1e8
    H = synth.hadamard(6)
    pr = np.broadcast_to(H[None, None], (w.T, C, D, D))
    b = cofem.rhs(w.phi_list(), w.y_list(), w.beta)
    pol = cg.CGPolicy(tol=1e-14, max_iters=20 * D)
    got = cofem.estep(w.phi_list(), b, w.beta, alpha, w.log_pi, D, pol, probes=pr,
                      precond="jacobi")
    ref = dense_em.estep(w.phi_list(), b, w.beta, alpha)
    assert np.allclose(got["mu"], ref["mu"], rtol=1e-8, atol=1e-10 * np.abs(ref["mu"]).max())
    assert np.allclose(got["s"], ref["var"], rtol=1e-8)
    assert np.allclose(got["nu"], ref["logdet"], rtol=1e-10)
    plain = cofem.estep(w.phi_list(), b, w.beta, alpha, w.log_pi, D, pol, probes=pr)
    assert got["iters"].mean() < plain["iters"].mean()


def test_jacobi_rademacher_estimators_unbiased():
    """Rademacher probes: over 200 seeds the mean of s and of nu-bar is within 4 standard
    errors of the exact diag Sigma and log det Sigma (tiny problem, converged PCG)."""
    w = synth.make("tiny", T=1)
    D = w.cfg.D
    b = cofem.rhs(w.phi_list(), w.y_list(), w.beta)
    alpha = w.alpha0[:1].copy()
    alpha[:, ::4] = 1e6
    ref = dense_em.estep(w.phi_list(), b, w.beta, alpha)
    pol = cg.CGPolicy(tol=1e-13, max_iters=20 * D)
    ss, nus = [], []
    for seed in range(200):
        o = cofem.estep(w.phi_list(), b, w.beta, alpha, np.zeros(1), 4, pol, seed=1000 + seed,
                        precond="jacobi")
        ss.append(o["s"][0, 0]); nus.append(o["nu"][0, 0])
    ss, nus = np.array(ss), np.array(nus)
    z_s = (ss.mean(0) - ref["var"][0, 0]) / (ss.std(0, ddof=1) / np.sqrt(len(ss)) + 1e-300)
    z_nu = (nus.mean() - ref["logdet"][0, 0]) / (nus.std(ddof=1) / np.sqrt(len(nus)))
    assert np.max(np.abs(z_s)) < 4.5 and abs(z_nu) < 4.0
