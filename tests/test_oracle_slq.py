"""Pins of the oracle's Lanczos quadrature (Eqs. (tridiag), (hutch-trace), (logdet-est))."""

import numpy as np

from oracle import cg, slq


def _spd(D=48, N=24, seed=0, beta=50.0):
    rng = np.random.default_rng(seed)
    Phi = rng.standard_normal((N, D)) / np.sqrt(N)
    A = beta * Phi.T @ Phi + np.diag(rng.uniform(0.5, 2.0, D))
    p = rng.choice([-1.0, 1.0], size=D)
    return A, p


def _cg_coeffs(A, p, **pol):
    X, g, x, it, st = cg.cg(lambda V, cols: A @ V, p[:, None], cg.CGPolicy(**pol))
    return g[0], x[0]


def _lanczos(A, p, U):
    """Textbook Lanczos with full reorthogonalisation from v1 = p/||p||."""
    D = len(p)
    V = np.zeros((D, U))
    a = np.zeros(U); b = np.zeros(max(U - 1, 0))
    V[:, 0] = p / np.linalg.norm(p)
    for j in range(U):
        w = A @ V[:, j]
        a[j] = V[:, j] @ w
        w -= V[:, :j + 1] @ (V[:, :j + 1].T @ w)
        w -= V[:, :j + 1] @ (V[:, :j + 1].T @ w)
        if j + 1 < U:
            b[j] = np.linalg.norm(w)
            V[:, j + 1] = w / b[j]
    return a, b


def test_cg_tridiagonal_equals_lanczos():
    A, p = _spd()
    U = 10
    g, x = _cg_coeffs(A, p, fixed_iters=U)
    diag, off = slq.tridiagonal(g, x)
    a, b = _lanczos(A, p, U)
    assert np.allclose(diag, a, rtol=1e-9)
    assert np.allclose(np.abs(off), b, rtol=1e-9)


def test_gauss_quadrature_moments():
    # ||p||^2 sum_u w_u lambda_u^j = p^T A^j p exactly for j <= 2U - 1
    A, p = _spd(seed=1)
    U = 6
    g, x = _cg_coeffs(A, p, fixed_iters=U)
    lam, w = slq.quadrature_terms(g, x)
    assert np.isclose(w.sum(), 1.0, rtol=1e-13)
    scale = np.linalg.norm(A, 2)
    v = p.copy()
    for j in range(2 * U):
        exact = p @ v / scale ** j
        quad = (p @ p) * np.sum(w * (lam / scale) ** j)
        assert np.isclose(quad, exact, rtol=1e-9), j
        v = A @ v


def test_full_length_equals_matrix_log():
    A, p = _spd(D=40, N=20, seed=2, beta=5.0)
    g, x = _cg_coeffs(A, p, tol=1e-14, max_iters=400)
    tau = slq.quadrature_log(g, x, p @ p)
    ev, Q = np.linalg.eigh(A)
    exact = p @ (Q @ (np.log(ev) * (Q.T @ p)))
    assert np.isclose(tau, exact, rtol=1e-9)


def test_one_step_closed_form():
    A, p = _spd(seed=3)
    g, x = _cg_coeffs(A, p, fixed_iters=1)
    tau = slq.quadrature_log(g, x, p @ p)
    assert np.isclose(tau, (p @ p) * np.log((p @ A @ p) / (p @ p)), rtol=1e-13)


def test_ritz_values_inside_spectrum_and_estimator_sign():
    A, p = _spd(seed=4)
    g, x = _cg_coeffs(A, p, fixed_iters=12)
    lam, w = slq.quadrature_terms(g, x)
    ev = np.linalg.eigvalsh(A)
    assert lam.min() >= ev.min() * (1 - 1e-12) and lam.max() <= ev.max() * (1 + 1e-12)
    # nu-bar is minus the mean of the quadratures (estimate of log det Sigma = -log det A)
    assert slq.logdet_estimate([1.0, 3.0]) == -2.0
