"""Learned GMRES warm start: FP64 reference of the convolutional network (oracle; test-only).

The network maps per-marker features of the theta-L state to a correction of the
linear extrapolation of the pressure density between time steps (Sec. 5 supplies the
state; the network itself is an addition to the method and never changes the GMRES
answer, which is always converged to the same FP64 residual):

  features (M x 5): eta, L / L_ref, theta_a (= kappa L / 2pi), phi1 / s1,
                    (phi1 - phi2) / s2 with phi1, phi2 the densities of the two previous
                    steps, s1 = RMS(phi1) and s2 = RMS(phi1 - phi2)
  network:          four circular 1-D convolutions, kernel 5 (taps t = 0..4 act on the
                    sample p + t - 2 mod M), widths 5 -> 64 -> 64 -> 64 -> 1, SiLU after
                    the first three
  initial guess:    x0 = 2 phi1 - phi2 + s2 sigma net(features), sigma a fixed target
                    scale (the RMS of the training targets)
  training target:  (phi_n - 2 phi1 + phi2) / (s2 sigma), mean squared error, Adam.

Parameter vector (FP32 master copy on the GPU, float64 here), concatenated in this
order, weights indexed [co][t][ci]:
  W1 (64,5,5)  b1 (64)  W2 (64,5,64)  b2 (64)  W3 (64,5,64)  b3 (64)  W4 (1,5,64)  b4 (1)

``bf16=True`` rounds the inputs, the weights and every activation to bfloat16 (round to
nearest even) at the points where the GPU kernels store bfloat16, and keeps everything
else in float64, so that it matches kernels that accumulate in FP32 up to their
accumulation error.

Pinned by: central finite differences of the loss (backward), delta kernels (pure
circular shifts), circular correlation by FFT (forward), the closed-form first Adam step,
and the SiLU derivative (tests/test_oracle_warmstart.py).
"""
from __future__ import annotations

import numpy as np

CIN, WIDTH, TAPS, PAD = 5, 64, 5, 2
SHAPES = [((WIDTH, TAPS, CIN), (WIDTH,)), ((WIDTH, TAPS, WIDTH), (WIDTH,)),
          ((WIDTH, TAPS, WIDTH), (WIDTH,)), ((1, TAPS, WIDTH), (1,))]
N_PARAMS = sum(int(np.prod(w)) + int(np.prod(b)) for w, b in SHAPES)


def unflatten(theta: np.ndarray):
    """Flat parameter vector -> list of (W, b) per layer (views)."""
    out, o = [], 0
    for ws, bs in SHAPES:
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        out.append((theta[o:o + nw].reshape(ws), theta[o + nw:o + nw + nb]))
        o += nw + nb
    return out


def bf16(x: np.ndarray) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def features(eta, L, L_ref, theta_a, phi1, phi2):
    """Per-marker features (M, 5) and the scales (s2, s1)."""
    s1 = float(np.sqrt(np.mean(phi1 * phi1)))
    s2 = float(np.sqrt(np.mean((phi1 - phi2) ** 2)))
    i1 = 1.0 / s1 if s1 > 0 else 0.0
    i2 = 1.0 / s2 if s2 > 0 else 0.0
    M = eta.size
    F = np.stack([eta, np.full(M, L / L_ref), theta_a, phi1 * i1, (phi1 - phi2) * i2], axis=1)
    return F, (s2, s1)


def conv(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Circular convolution layer: x (B, M, Ci), W (Co, T, Ci) -> (B, M, Co),
    out[b, p, co] = b[co] + sum_t sum_ci W[co, t, ci] x[b, (p + t - PAD) mod M, ci]."""
    out = np.broadcast_to(b, x.shape[:2] + (W.shape[0],)).astype(np.float64).copy()
    for t in range(W.shape[1]):
        xs = np.roll(x, -(t - PAD), axis=1)  # xs[:, p] = x[:, p + t - PAD]
        out += xs @ W[:, t, :].T
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    sg = 1.0 / (1.0 + np.exp(-z))
    return sg * (1.0 + z * (1.0 - sg))


def forward(theta, X, bf=False):
    """X (B, M, 5) -> (output (B, M), cache)."""
    layers = unflatten(theta)
    r = bf16 if bf else (lambda v: v)
    a = r(X)
    cache = []
    for li, (W, b) in enumerate(layers):
        z = conv(a, r(W), b)
        cache.append((a, z))
        if li < len(layers) - 1:
            a = r(silu(z))
    return z[..., 0], cache


def loss(theta, X, Y, bf=False):
    y, _ = forward(theta, X, bf)
    return float(np.mean((y - Y) ** 2))


def backward(theta, X, Y, bf=False):
    """(loss, gradient of the loss with respect to theta) by the chain rule."""
    layers = unflatten(theta)
    r = bf16 if bf else (lambda v: v)
    y, cache = forward(theta, X, bf)
    n = y.size
    g = np.zeros_like(theta)
    gl = unflatten(g)
    dz = (2.0 / n) * (y - Y)[..., None]  # (B, M, 1)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        a, z = cache[li]
        gW, gb = gl[li]
        gb[:] = dz.sum(axis=(0, 1))
        for t in range(W.shape[1]):
            xs = np.roll(a, -(t - PAD), axis=1)
            gW[:, t, :] = np.einsum("bpo,bpi->oi", dz, xs)
        if li == 0:
            break
        # gradient with respect to this layer's input a = silu(z_prev)
        da = np.zeros_like(a)
        Wr = r(W)
        for t in range(W.shape[1]):
            da += np.roll(dz @ Wr[:, t, :], t - PAD, axis=1)  # da[p] += dz[p - t + PAD] W
        dz = da * dsilu(cache[li - 1][1])
        if bf:
            dz = bf16(dz)
    return float(np.mean((y - Y) ** 2)), g


def adam_step(theta, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def initial_guess(theta, F, s2, sigma, phi1, phi2, bf=True):
    """x0 = 2 phi1 - phi2 + s2 sigma net(F) (F: (M, 5)); phi1 if s2 = 0."""
    if s2 == 0.0:
        return phi1.copy()
    y, _ = forward(theta, F[None], bf)
    return 2.0 * phi1 - phi2 + s2 * sigma * y[0]
