"""Seeded synthetic inputs shared by the HIP path's tests/bench and by the CPU oracle.

This module only *samples* curves, densities and grid descriptions; it holds none of
the method's arithmetic (no derivatives, jumps, solves or reparametrisations), so the
oracle and the GPU library can both consume its arrays without sharing method code.

Workloads (all analytic, as in the paper's numerical section; no dataset is involved):

* ``ellipse``:  x = 0.6 cos a, y = 0.4 sin a in the box [-1,1]^2 (interior Dirichlet test).
* ``star``:     r(a) = 0.5 (1 + 0.2 cos 5a) in [-1,1]^2 (single-apply throughput workload).
* ``hs3``:      r(a) = 1 + 0.1 cos 3a + 0.05 sin 5a in [-2,2]^2 (Hele-Shaw evolution).
* ``perturbed``: r(a) = 1 + sum_{m=2..8} a_m cos(m a + phi_m), a_m ~ U(0,0.1) (warm-start data).
* densities: phi(a) = sum_{k=1..32} (z_k cos ka + z'_k sin ka)/k^2, z ~ N(0,1), numpy PCG64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Box:
    """Square box [x0, x0+side] x [y0, y0+side] split into N intervals per side."""
    x0: float
    y0: float
    side: float
    N: int

    @property
    def h(self) -> float:
        return self.side / self.N


def params(M: int) -> np.ndarray:
    """Equispaced parameter values a_k = 2 pi k / M, k = 0..M-1."""
    return 2.0 * math.pi * np.arange(M, dtype=np.float64) / M


def polar_curve(radius, M: int, center=(0.0, 0.0)) -> np.ndarray:
    """Sample (x, y) = c + r(a)(cos a, sin a) at a_k; returns shape (2, M), counter-clockwise."""
    a = params(M)
    r = radius(a)
    return np.stack([center[0] + r * np.cos(a), center[1] + r * np.sin(a)])


def ellipse(M: int = 256, ax: float = 0.6, ay: float = 0.4) -> np.ndarray:
    a = params(M)
    return np.stack([ax * np.cos(a), ay * np.sin(a)])


def star(M: int = 2048) -> np.ndarray:
    return polar_curve(lambda a: 0.5 * (1.0 + 0.2 * np.cos(5.0 * a)), M)


def circle(M: int, R: float, center=(0.0, 0.0)) -> np.ndarray:
    return polar_curve(lambda a: R + 0.0 * a, M, center)


def hs3(M: int = 1024) -> np.ndarray:
    return polar_curve(lambda a: 1.0 + 0.1 * np.cos(3.0 * a) + 0.05 * np.sin(5.0 * a), M)


def perturbed(M: int, seed: int, modes=range(2, 9), amp: float = 0.1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    ms = list(modes)
    am = rng.uniform(0.0, amp, size=len(ms))
    ph = rng.uniform(0.0, 2.0 * math.pi, size=len(ms))

    def r(a):
        out = np.ones_like(a)
        for m, c, p in zip(ms, am, ph):
            out = out + c * np.cos(m * a + p)
        return out
    return polar_curve(r, M)


def fourier_density(M: int, seed: int, kmax: int = 32) -> np.ndarray:
    """phi(a_k) = sum_{k=1..kmax} (z_k cos ka + z'_k sin ka) / k^2 with z ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(2 * kmax)
    a = params(M)
    out = np.zeros(M)
    for k in range(1, kmax + 1):
        out += (z[k - 1] * np.cos(k * a) + z[kmax + k - 1] * np.sin(k * a)) / (k * k)
    return out


def random_ring(N: int, seed: int) -> np.ndarray:
    """Arbitrary Dirichlet data on the box ring, layout (4, N+1): bottom, top, left, right."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((4, N + 1))


BOX_UNIT2 = Box(-1.0, -1.0, 2.0, 1024)


def box(lo: float, hi: float, N: int) -> Box:
    return Box(lo, lo, hi - lo, N)
