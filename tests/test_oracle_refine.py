"""Pins for the adaptive marker refinement of the theta-L state (oracle.thetal.refine)."""
import numpy as np

from oracle import spectral
from oracle import thetal as T
from paper_2309_01068_amd import workloads as W


def test_upsample2_is_exact_for_trigonometric_polynomials():
    M = 32
    a = 2 * np.pi * np.arange(M) / M
    a2 = np.pi * np.arange(2 * M) / M
    f = lambda x: 0.3 + np.cos(3 * x) - 0.2 * np.sin(7 * x) + 0.05 * np.cos(15 * x)
    assert np.max(np.abs(spectral.upsample2(f(a)) - f(a2))) < 1e-14
    # the Nyquist mode of the coarse grid is dropped, as in every spectral operation
    g = spectral.upsample2(np.cos(16 * a))
    assert np.max(np.abs(g)) < 1e-14


def test_refined_state_describes_the_same_curve():
    # 256 markers resolve cos(theta), sin(theta) of this curve to rounding, so the coarse
    # and the refined reconstructions agree at the old markers to rounding
    X = W.polar_curve(lambda a: 1 + 0.1 * np.cos(3 * a) + 0.05 * np.sin(5 * a), 256)
    eta, L, Xb = T.equal_arclength_init(X, 256)
    st = T.HSState(eta, L, Xb)
    r = T.refine(st)
    assert r.eta.size == 512 and r.L == L and np.array_equal(r.Xbar, Xb)
    X1, *_ = T.reconstruct(st.eta, st.L, st.Xbar)
    X2, *_ = T.reconstruct(r.eta, r.L, r.Xbar)
    assert np.max(np.abs(X2[:, ::2] - X1)) < 1e-12          # old markers kept
    # the new markers lie on the curve: equal arclength, and the enclosed area is kept
    sa = np.hypot(spectral.diff(X2[0]), spectral.diff(X2[1]))
    assert np.max(np.abs(sa - L / (2 * np.pi))) < 1e-9
    assert abs(T.area(X2) - T.area(X1)) < 1e-10 * T.area(X1)


def test_refinement_carries_the_explicit_history():
    """The history of the explicit term is the DFT of a function of alpha: after
    refinement it is the DFT of the same function sampled on the doubled grid."""
    M = 64
    a = 2 * np.pi * np.arange(M) / M
    f = lambda x: np.sin(2 * x) + 0.1 * np.cos(9 * x)
    st = T.HSState(np.zeros(M), 2 * np.pi, np.zeros(2), n=3, Nhat_prev=np.fft.fft(f(a)),
                   phi_prev=f(a) + 1.0)
    r = T.refine(st)
    a2 = np.pi * np.arange(2 * M) / M
    assert np.max(np.abs(r.Nhat_prev - np.fft.fft(f(a2)))) < 1e-12
    assert np.max(np.abs(r.phi_prev - (f(a2) + 1.0))) < 1e-13
    assert r.n == 3


def test_refinement_criterion():
    st = T.HSState(np.zeros(64), 2 * np.pi, np.zeros(2))
    h = 2 * np.pi / 64 / 1.5
    assert not T.refine_due(st, h * 1.001, 1.5, 4096)
    assert T.refine_due(st, h * 0.999, 1.5, 4096)
    assert not T.refine_due(st, h * 0.999, 1.5, 64)         # no room to double
    assert not T.refine_due(st, h * 0.999, 0.0, 4096)       # off
