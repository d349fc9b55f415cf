"""Pins for oracle.spectral: exact on trigonometric polynomials (Sec. 5.3 remark)."""
import numpy as np

from oracle import spectral


def _a(M):
    return 2 * np.pi * np.arange(M) / M


def test_derivatives_of_trig_polynomial_are_exact():
    M = 64
    a = _a(M)
    f = 0.3 + np.cos(3 * a) - 2.0 * np.sin(7 * a) + 0.5 * np.cos(31 * a)
    f1 = -3 * np.sin(3 * a) - 14.0 * np.cos(7 * a) - 15.5 * np.sin(31 * a)
    f2 = -9 * np.cos(3 * a) + 98.0 * np.sin(7 * a) - 480.5 * np.cos(31 * a)
    f3 = 27 * np.sin(3 * a) + 686.0 * np.cos(7 * a) + 14895.5 * np.sin(31 * a)
    assert np.allclose(spectral.diff(f, 1), f1, atol=1e-11)
    assert np.allclose(spectral.diff(f, 2), f2, atol=1e-9)
    assert np.allclose(spectral.diff(f, 3), f3, atol=1e-7)


def test_nyquist_mode_is_dropped():
    M = 16
    a = _a(M)
    f = np.cos(8 * a)           # pure Nyquist: every derivative is zero by convention
    for p in (1, 2, 3):
        assert np.allclose(spectral.diff(f, p), 0.0, atol=1e-12)
    assert np.allclose(spectral.hilbert(f), 0.0, atol=1e-12)


def test_antiderivatives():
    M = 128
    a = _a(M)
    f = 2.0 + np.cos(2 * a) + 3 * np.sin(5 * a)
    F = np.sin(2 * a) / 2 - 3 * np.cos(5 * a) / 5          # mean-free antiderivative of f - 2
    assert np.allclose(spectral.antiderivative_meanfree(f), F, atol=1e-13)
    C = F - F[0]                                            # int_0^a (f - 2)
    assert np.allclose(spectral.cumulative_meanfree(f), C, atol=1e-13)


def test_hilbert_transform():
    M = 64
    a = _a(M)
    # H[cos ka] = sin ka, H[sin ka] = -cos ka for k > 0 (multiplier -i sgn k)
    assert np.allclose(spectral.hilbert(np.cos(4 * a)), np.sin(4 * a), atol=1e-13)
    assert np.allclose(spectral.hilbert(np.sin(9 * a)), -np.cos(9 * a), atol=1e-13)
    rng = np.random.default_rng(0)
    f = rng.standard_normal(M)
    f -= f.mean()
    fh = np.fft.fft(f)
    fh[M // 2] = 0
    f = np.real(np.fft.ifft(fh))
    assert np.allclose(spectral.hilbert(spectral.hilbert(f)), -f, atol=1e-13)
