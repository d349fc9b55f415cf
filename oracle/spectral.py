"""Fourier pseudo-spectral operators on equispaced periodic samples (oracle; test-only).

The paper performs differentiation, integration and the Hilbert transform of periodic
interface quantities in Fourier space (Sec. 5.3, closing remark).  Conventions fixed
here (readings, not stated by the paper): the sampled function is the trigonometric
interpolant with modes |k| < M/2; the Nyquist mode k = M/2 is set to zero for every
derivative, antiderivative and Hilbert transform.

Pinned by: exact derivatives / antiderivatives / Hilbert transforms of trigonometric
polynomials (tests/test_oracle_spectral.py), H[H f] = -f for mean-free f; upsample2
reproduces a trigonometric polynomial at the doubled samples exactly
(tests/test_oracle_refine.py).
"""
from __future__ import annotations

import numpy as np


def wavenumbers(M: int) -> np.ndarray:
    """Integer wavenumbers in numpy FFT order with the Nyquist entry set to 0."""
    k = np.fft.fftfreq(M, d=1.0 / M)
    if M % 2 == 0:
        k[M // 2] = 0.0
    return k


def _nyq_mask(M: int) -> np.ndarray:
    m = np.ones(M)
    if M % 2 == 0:
        m[M // 2] = 0.0
    return m


def diff(f: np.ndarray, p: int = 1) -> np.ndarray:
    """p-th derivative in the periodic parameter alpha (multiplier (ik)^p)."""
    M = f.shape[-1]
    k = wavenumbers(M)
    fh = np.fft.fft(f, axis=-1) * ((1j * k) ** p) * _nyq_mask(M)
    return np.real(np.fft.ifft(fh, axis=-1))


def antiderivative_meanfree(f: np.ndarray) -> np.ndarray:
    """sum_{k != 0} f_k e^{ik a}/(ik): the periodic antiderivative with zero mean
    (the k = 0 part of f is dropped)."""
    M = f.shape[-1]
    k = wavenumbers(M)
    fh = np.fft.fft(f, axis=-1)
    mult = np.zeros(M, dtype=complex)
    nz = k != 0
    mult[nz] = 1.0 / (1j * k[nz])
    return np.real(np.fft.ifft(fh * mult, axis=-1))


def cumulative_meanfree(f: np.ndarray) -> np.ndarray:
    """Values at the samples a_j of sum_{k != 0} f_k (e^{ik a} - 1)/(ik), i.e. the
    integral from 0 to a_j of (f - mean f)."""
    A = antiderivative_meanfree(f)
    return A - A[..., :1]


def hilbert(f: np.ndarray) -> np.ndarray:
    """Periodic Hilbert transform, multiplier -i sgn(k) (Sec. 5.2.1)."""
    M = f.shape[-1]
    k = wavenumbers(M)
    fh = np.fft.fft(f, axis=-1) * (-1j * np.sign(k))
    return np.real(np.fft.ifft(fh, axis=-1))


def upsample2(f: np.ndarray) -> np.ndarray:
    """Values of the trigonometric interpolant (Nyquist mode dropped) at 2M equispaced
    samples a'_j = pi j / M; the even samples reproduce f when f has no Nyquist part."""
    M = f.shape[-1]
    fh = np.fft.fft(f, axis=-1) * _nyq_mask(M)
    g = np.zeros(f.shape[:-1] + (2 * M,), dtype=complex)
    h = M // 2
    g[..., :h] = fh[..., :h]
    g[..., 2 * M - h + 1:] = fh[..., h + 1:]
    return np.real(np.fft.ifft(g, axis=-1)) * 2.0
