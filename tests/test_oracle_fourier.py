"""Pins of the partial-Fourier sensing oracle (Sec. 4 sensing; oracle/fourier.py)."""

import numpy as np
import pytest

import synth
from oracle import fourier, cofem, cg as ocg


def test_dft_matrix_is_unitary_and_transforms_a_cosine():
    D = 64
    F = fourier.dft_matrix(D)
    assert np.allclose(F.conj().T @ F, np.eye(D), atol=1e-13)
    # a cosine of frequency k0 has exactly two non-zero coefficients sqrt(D)/2 at k0 and D - k0
    k0 = 5
    v = np.cos(2 * np.pi * k0 * np.arange(D) / D)
    Fv = F @ v
    ref = np.zeros(D, complex)
    ref[k0] = ref[D - k0] = np.sqrt(D) / 2
    assert np.allclose(Fv, ref, atol=1e-12)
    # and the matrix agrees with numpy's FFT (a separate implementation of the same map)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(D)
    assert np.allclose(F @ x, np.fft.fft(x, norm="ortho"), atol=1e-12)


def test_fft_operator_and_rhs_equal_the_dense_real_stacked_matrix():
    w = synth.make_fourier("fourier-small")
    D, beta = w.cfg.D, w.beta
    rng = np.random.default_rng(1)
    V = rng.standard_normal((D, 7))
    for t in range(w.T):
        f = w.freq_t(t)
        P = fourier.sensing_matrix(f, D)
        assert P.shape == (2 * len(f), D)
        dense = beta * (P.T @ (P @ V))
        assert np.allclose(fourier.apply(f, D, beta, V), dense, rtol=0, atol=1e-11 * beta)
        b = beta * P.T @ fourier.stack(w.yc_t(t))
        assert np.allclose(fourier.rhs(f, w.yc_t(t), D, beta), b, atol=1e-11 * np.abs(b).max())


def test_spectrum_is_the_symmetrised_mask():
    """Phi^T Phi = Re(F^H Omega^T Omega F) is diagonalised by F with eigenvalue
    (m_k + m_{-k}) / 2 on frequency k, m the 0/1 mask: for a real signal the real part averages
    a frequency with its mirror image."""
    D = 64
    rng = np.random.default_rng(2)
    f = np.sort(rng.choice(D, 16, replace=False))
    P = fourier.sensing_matrix(f, D)
    m = np.zeros(D); m[f] = 1
    h = 0.5 * (m + m[(-np.arange(D)) % D])
    lam = np.linalg.eigvalsh(P.T @ P)
    assert np.allclose(np.sort(lam), np.sort(h), atol=1e-12)


def test_full_mask_reduces_to_closed_forms():
    """Omega = I: Phi^T Phi = I, so A = (beta + alpha) I: with converged CG and Hadamard probes
    (K = D) the E-step gives mu = b / (beta + alpha), s = 1 / (beta + alpha) exactly and
    nu-bar = -sum_d log(beta + alpha_d)."""
    D, C = 64, 2
    rng = np.random.default_rng(3)
    f = np.arange(D)
    yc = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    beta = 400.0
    alpha = synth.draw_alpha0(C, D)
    P = fourier.sensing_matrix(f, D)
    y = fourier.stack(yc)
    b = cofem.rhs([P], [y], beta)
    H = synth.hadamard(6)
    pr = np.broadcast_to(H[None, None], (1, C, D, D))
    out = cofem.estep([P], b, beta, alpha, np.log([0.5, 0.5]), D,
                      ocg.CGPolicy(tol=1e-14, max_iters=100), probes=pr)
    for c in range(C):
        assert np.allclose(out["mu"][0, c], b[0] / (beta + alpha[c]), rtol=1e-12)
        assert np.allclose(out["s"][0, c], 1.0 / (beta + alpha[c]), rtol=1e-10)
        assert np.isclose(out["nu"][0, c], -np.log(beta + alpha[c]).sum(), rtol=1e-12)
