"""Pins for oracle.warmstart: the reference network is checked against finite
differences, delta kernels, FFT correlation, the closed-form first Adam step and exact
bfloat16 rounding cases."""
import numpy as np
import pytest

from oracle import warmstart as WS


def rand_theta(seed, scale=0.3):
    return np.random.default_rng(seed).normal(0.0, scale, WS.N_PARAMS)


def test_parameter_count():
    assert WS.N_PARAMS == 64 * 5 * 5 + 64 + 2 * (64 * 5 * 64 + 64) + 5 * 64 + 1 == 43073


def test_delta_kernel_is_a_circular_shift():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 16, 5))
    W = np.zeros((64, 5, 5))
    for t0, ci0, co in ((0, 1, 3), (4, 2, 7), (2, 0, 0)):
        W[co, t0, ci0] = 1.0
    z = WS.conv(x, W, np.zeros(64))
    for t0, ci0, co in ((0, 1, 3), (4, 2, 7), (2, 0, 0)):
        for p in range(16):
            assert z[1, p, co] == x[1, (p + t0 - 2) % 16, ci0]
    assert np.all(z[..., 1] == 0.0)


def test_conv_matches_fft_correlation():
    rng = np.random.default_rng(2)
    M = 32
    x = rng.normal(size=(1, M, 1))
    w = rng.normal(size=(1, 5, 1))
    z = WS.conv(x, w, np.array([0.25]))[0, :, 0]
    kpad = np.zeros(M)
    for t in range(5):
        kpad[(t - 2) % M] = w[0, t, 0]
    ref = np.real(np.fft.ifft(np.fft.fft(x[0, :, 0]) * np.conj(np.fft.fft(kpad)))) + 0.25
    assert np.max(np.abs(z - ref)) < 1e-12


def test_silu_derivative():
    z = np.linspace(-6, 6, 101)
    fd = (WS.silu(z + 1e-6) - WS.silu(z - 1e-6)) / 2e-6
    assert np.max(np.abs(fd - WS.dsilu(z))) < 1e-8


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    theta = rand_theta(4, scale=0.06)  # activations of order one, so the loss is too
    X = rng.normal(size=(2, 16, 5))
    Y = rng.normal(size=(2, 16))
    _, g = WS.backward(theta, X, Y)
    idx = np.concatenate([rng.choice(np.arange(o, o + n), 6, replace=False)
                          for o, n in ((0, 1664), (1664, 20544), (22208, 20544), (42752, 321))])
    eps = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (WS.loss(tp, X, Y) - WS.loss(tm, X, Y)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(g[i]), (i, fd, g[i])


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(5)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    new, m, v = WS.adam_step(th, g, np.zeros(50), np.zeros(50), 1, lr=1e-3, eps=1e-8)
    # first step: bias-corrected moments are g and g^2, so the update is -lr g/(|g| + eps)
    assert np.allclose(new, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_bfloat16_rounding_cases():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.0 - 2 ** -7 - 2 ** -9, 3.0e38])
    r = WS.bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # tie to even
    assert r[2] == 1.0 + 2 ** -6            # tie to even (upwards)
    assert r[3] == -2.0 - 2 ** -6           # above the tie: away
    assert np.isfinite(r[4])


def test_features_and_guess():
    M = 16
    rng = np.random.default_rng(6)
    eta = rng.normal(size=M)
    tha = 1 + rng.normal(size=M) * 0.1
    phi1 = 2.0 + rng.normal(size=M)
    phi2 = phi1 - 0.01 * (1 + rng.normal(size=M))
    F, (s2, s1) = WS.features(eta, 7.0, 2 * np.pi, tha, phi1, phi2)
    assert abs(s1 - np.sqrt(np.mean(phi1 ** 2))) < 1e-15
    assert abs(np.sqrt(np.mean(F[:, 4] ** 2)) - 1.0) < 1e-12      # unit-RMS difference channel
    assert np.allclose(F[:, 1], 7.0 / (2 * np.pi))
    # an untrained network with a zero output layer returns the linear extrapolation
    theta = rand_theta(7)
    theta[42752:] = 0.0
    x0 = WS.initial_guess(theta, F, s2, 0.3, phi1, phi2)
    assert np.allclose(x0, 2 * phi1 - phi2, rtol=0, atol=1e-15)
    assert np.array_equal(WS.initial_guess(theta, F, 0.0, 0.3, phi1, phi2), phi1)
