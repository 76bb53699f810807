"""Partial-Fourier sensing (Sec. 4) in FP64.  TEST INFRASTRUCTURE ONLY.

The experiments of Sec. 4 use Phi_t = Omega_t F with F the D x D discrete Fourier transform and
Omega_t a row subset of the identity (N_t = D/4 rows chosen at random): a complex sensing matrix
in a model whose signals are real.  Readings used here:

* F is the unitary DFT, F[k, d] = exp(-2 pi i k d / D) / sqrt(D);
* the complex measurements y_t = Omega_t F z_t + noise enter the real model through the stacking
  of real and imaginary parts: Phi_t := [Re(Omega_t F); Im(Omega_t F)] (2 N_t x D real) and
  y_t := [Re y; Im y], with independent N(0, sigma^2) noise on each part, so beta = 1/sigma^2
  as for real measurements.  Then Phi^T Phi = Re((Omega F)^H (Omega F)) and
  Phi^T y = Re((Omega F)^H y): the operator of Eq. (lin-sys) is
      A v = beta Re(F^H Omega^T Omega F v) + alpha (.) v,
  which FFTs apply in O(D log D) (Sec. 3.3).

``sensing_matrix`` writes Phi_t out from the definition of F; the CoFEM oracle (cofem.estep)
runs on it unchanged.  ``apply`` and ``rhs`` are the same maps through numpy's FFT (a library
primitive), pinned against the dense matrix in tests/test_oracle_fourier.py.
"""

import numpy as np


def dft_matrix(D):
    """Unitary DFT matrix F[k, d] = exp(-2 pi i k d / D) / sqrt(D), from its definition (the
    product k d is reduced mod D exactly in integers before the exponential)."""
    k = np.arange(D)
    m = np.outer(k, k) % D
    return np.exp(-2j * np.pi * m / D) / np.sqrt(D)


def sensing_matrix(freq, D):
    """Real-stacked sensing matrix [Re(Omega F); Im(Omega F)] (2N x D) for the selected
    frequencies `freq` (the rows Omega keeps)."""
    F = dft_matrix(D)[np.asarray(freq)]
    return np.concatenate([F.real, F.imag], axis=0)


def stack(yc):
    """Real measurement vector [Re y; Im y] of complex measurements y (N,)."""
    yc = np.asarray(yc)
    return np.concatenate([yc.real, yc.imag]).astype(np.float64)


def apply(freq, D, beta, V):
    """beta Re(F^H Omega^T Omega F V) for the columns of V (D x R), through the FFT."""
    Y = np.fft.fft(np.asarray(V, np.float64), axis=0, norm="ortho")
    keep = np.zeros(D, bool)
    keep[np.asarray(freq)] = True
    Y[~keep] = 0.0
    return beta * np.fft.ifft(Y, axis=0, norm="ortho").real


def rhs(freq, yc, D, beta):
    """b = beta Phi^T y = beta Re(F^H Omega^T y) through the FFT."""
    Y = np.zeros(D, complex)
    Y[np.asarray(freq)] = np.asarray(yc)
    return beta * np.fft.ifft(Y, norm="ortho").real
