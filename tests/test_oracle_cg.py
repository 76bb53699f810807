"""Pins of the oracle's conjugate gradient (Alg. 1) against dense linear algebra."""

import numpy as np

import synth
from oracle import cg


def _system(D=64, N=32, seed=0, beta=1e2):
    rng = np.random.default_rng(seed)
    Phi = rng.standard_normal((N, D)) / np.sqrt(N)
    alpha = rng.uniform(0.5, 1.5, D)
    A = beta * Phi.T @ Phi + np.diag(alpha)
    return A, rng


def test_converged_matches_dense_solve():
    A, rng = _system()
    B = rng.standard_normal((64, 5))
    X, g, x, iters, st = cg.cg(lambda V, cols: A @ V, B, cg.CGPolicy(tol=1e-13, max_iters=2000))
    assert np.all(st == cg.CONVERGED)
    ref = np.linalg.solve(A, B)
    assert np.max(np.abs(X - ref)) / np.max(np.abs(ref)) < 1e-10


def test_recursive_residual_tracks_true_residual():
    A, rng = _system(seed=1)
    b = rng.standard_normal((64, 1))
    for U in (1, 5, 20):
        X, g, x, iters, st = cg.cg(lambda V, cols: A @ V, b, cg.CGPolicy(fixed_iters=U))
        assert iters[0] == U and len(g[0]) == U and len(x[0]) == U
        # replay the recurrence: r_{U+1}.r_{U+1} = prod xi * r_1.r_1
        rr = float(b[:, 0] @ b[:, 0]) * np.prod(x[0])
        r_true = b[:, 0] - A @ X[:, 0]
        assert abs(r_true @ r_true - rr) <= 1e-8 * (b[:, 0] @ b[:, 0])


def test_first_step_closed_form():
    A, rng = _system(seed=2)
    b = rng.standard_normal((64, 1))
    X, g, x, _, _ = cg.cg(lambda V, cols: A @ V, b, cg.CGPolicy(fixed_iters=1))
    bb, bAb = b[:, 0] @ b[:, 0], b[:, 0] @ A @ b[:, 0]
    assert np.isclose(g[0][0], bb / bAb, rtol=1e-14)
    assert np.allclose(X[:, 0], bb / bAb * b[:, 0], rtol=1e-13)
    r = b[:, 0] - bb / bAb * (A @ b[:, 0])
    assert np.isclose(x[0][0], (r @ r) / bb, rtol=1e-12)


def test_tol_mode_and_max_iter_status():
    A, rng = _system(seed=3)
    b = rng.standard_normal((64, 1))
    X, g, x, iters, st = cg.cg(lambda V, cols: A @ V, b, cg.CGPolicy(tol=1e-6, max_iters=500))
    r = b[:, 0] - A @ X[:, 0]
    assert st[0] == cg.CONVERGED and np.linalg.norm(r) <= 1.01e-6 * np.linalg.norm(b)
    # the step before the last did not meet the tolerance
    rr_prev = (b[:, 0] @ b[:, 0]) * np.prod(x[0][:-1])
    assert rr_prev > 1e-12 * (b[:, 0] @ b[:, 0])
    X, g, x, iters, st = cg.cg(lambda V, cols: A @ V, b, cg.CGPolicy(tol=1e-30, max_iters=3))
    assert st[0] == cg.MAX_ITER and iters[0] == 3


def test_zero_rhs_and_breakdown():
    A = np.diag([1.0, -1.0, 2.0])
    B = np.zeros((3, 3))
    B[1, 1] = 1.0                     # d.Ad = -1 < 0 at the first step
    B[:, 2] = [1.0, 0.0, 1.0]
    X, g, x, iters, st = cg.cg(lambda V, cols: A @ V, B, cg.CGPolicy(tol=1e-12, max_iters=10))
    assert st[0] == cg.CONVERGED and iters[0] == 0 and np.all(X[:, 0] == 0)
    assert st[1] == cg.BREAKDOWN and iters[1] == 0 and len(g[1]) == 0
    assert st[2] == cg.CONVERGED and np.allclose(X[:, 2], [1.0, 0.0, 0.5])


def test_columns_are_independent():
    # batching columns side by side must not change any column's result (well-conditioned
    # operator, so rounding-order differences of the dot products stay at rounding level)
    rng = np.random.default_rng(4)
    M = rng.standard_normal((64, 64)) / 8.0
    A = M @ M.T + 2.0 * np.eye(64)
    B = rng.standard_normal((64, 4))
    B[:, 2] *= 1e-3
    pol = cg.CGPolicy(tol=1e-8, max_iters=300)
    X, g, x, it, st = cg.cg(lambda V, cols: A @ V, B, pol)
    assert it.max() < 40
    for j in range(4):
        Xj, gj, xj, itj, stj = cg.cg(lambda V, cols: A @ V, B[:, j:j + 1], pol)
        assert itj[0] == it[j] and stj[0] == st[j]
        assert np.allclose(Xj[:, 0], X[:, j], rtol=1e-12, atol=1e-14 * np.abs(X[:, j]).max())
        assert np.allclose(gj[0], g[j], rtol=1e-11) and np.allclose(xj[0], x[j], rtol=1e-10)


def test_workload_operator_is_spd():
    w = synth.make("tiny")
    P = w.phi(0).astype(np.float64)
    A = w.beta * P.T @ P + np.diag(w.alpha0[0])
    assert np.all(np.linalg.eigvalsh(A) > 0)
