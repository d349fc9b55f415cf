"""Pins for the theta-L time integration of the oracle (oracle.thetal.advance, Sec. 5.1-5.3).

The interface update is driven here by prescribed normal-velocity laws instead of the
boundary integral solve, so that its result can be compared with an evolution known in
closed form:

* U = c0 + c1 X.n moves a curve X0 to X(t) = e^{c1 t} X0 + (c0/c1)(e^{c1 t} - 1) n0 at
  corresponding points (normals are kept).  The theta-L variables of X(t) follow from the
  equal-arclength resampling, started at the point that has moved along the normal from
  the initial marker 0 (the equal-arclength tangential velocity V of Sec. 5.1 vanishes at
  alpha = 0).  This fixes M = int theta_a U, V, the sign of U_a in eq. the-evo, Q of
  eq. ave-evo and the AB2 updates of L and Xbar.
* The same law plus the small-scale term the decomposition removes (Sec. 5.2:
  -lam (2pi/L)^2 H[theta_aa] for the third-order form, -lam (2pi/L) theta_a for the
  second-order one) has no closed form, but its time error must fall as tau^2 (the
  integrating-factor AB2 of eq. Fourier-theta1/2 is second order).
* Through the whole Hele-Shaw step, a small mode-m perturbation of a circle grows at the
  linear rate (m-1) J / R^2 - sigma m (m^2 - 1) / R^3 with R(t) = sqrt(R0^2 + 2 J t), the
  classical result for a Hele-Shaw bubble with injection (derived from eq. bie-HS with
  r = R + delta cos m phi: the pressure gains a decaying harmonic A r^-m cos m phi fixed by
  the Laplace-Young condition).

Each pin is shown to fail for a planted mistake: the tangential velocity dropped, and the
integrating factor of the previous explicit term replaced by the one of the current step
with the current term left unpropagated.
"""
import inspect
import math
import textwrap

import numpy as np
import pytest
from scipy.integrate import quad, solve_ivp

from oracle import spectral
from oracle import thetal as T
from paper_2309_01068_amd import workloads as W

TWO_PI = 2.0 * math.pi
# a convex curve without central symmetry, off the origin
A2, A3, R0, CX, CY = 0.06, 0.02, 0.5, 0.1, -0.05
C0, C1 = 1.0, 0.5
T_END = 0.4


def _base(beta):
    """Initial curve r = R0 (1 + A2 cos 2b + A3 sin 3b) about (CX, CY) with its unit
    tangent, speed |X_b| and curvature at parameter b."""
    r = R0 * (1 + A2 * np.cos(2 * beta) + A3 * np.sin(3 * beta))
    r1 = R0 * (-2 * A2 * np.sin(2 * beta) + 3 * A3 * np.cos(3 * beta))
    r2 = R0 * (-4 * A2 * np.cos(2 * beta) - 9 * A3 * np.sin(3 * beta))
    c, s = np.cos(beta), np.sin(beta)
    x, y = CX + r * c, CY + r * s
    x1, y1 = r1 * c - r * s, r1 * s + r * c
    x2, y2 = r2 * c - 2 * r1 * s - r * c, r2 * s + 2 * r1 * c - r * s
    sp = np.hypot(x1, y1)
    kap = (x1 * y2 - y1 * x2) / sp ** 3
    return x, y, x1 / sp, y1 / sp, sp, kap


def _scale_shift(t):
    s = math.exp(C1 * t)
    return s, C0 / C1 * (s - 1.0)


def _foot(t):
    """Parameter b(t) of the point that moved along the normal from b = 0: the
    tangential part of d/dt X(t, b(t)) vanishes, b' = -s'(X0.t0) / ((s + q kappa)|X0'|)."""
    if t == 0.0:
        return 0.0

    def f(tt, b):
        s, q = _scale_shift(tt)
        x, y, tx, ty, sp, kap = _base(b)
        return -C1 * s * (x * tx + y * ty) / ((s + q * kap) * sp)
    r = solve_ivp(f, (0.0, t), [0.0], method="DOP853", rtol=1e-13, atol=1e-15)
    return float(r.y[0, -1])


def exact_state(M, t, samples=2048):
    b = _foot(t) + TWO_PI * np.arange(samples) / samples
    x, y, tx, ty, sp, kap = _base(b)
    s, q = _scale_shift(t)
    X = np.stack([s * x + q * ty, s * y - q * tx])        # outward normal (t_y, -t_x)
    return T.equal_arclength_init(X, M)


def evolve(M, tau, lam, pw, stiff, advance=None):
    advance = advance or T.advance
    eta, L, Xb = exact_state(M, 0.0)
    st = T.HSState(eta, L, Xb)
    for _ in range(int(round(T_END / tau))):
        X, theta, n, s = T.reconstruct(st.eta, st.L, st.Xbar)
        U = C0 + C1 * (X[0] * n[0] + X[1] * n[1])
        if stiff and pw == 3:
            U = U - lam * (TWO_PI / st.L) ** 2 * spectral.hilbert(spectral.diff(st.eta, 2))
        elif stiff:
            U = U - lam * (TWO_PI / st.L) * spectral.diff(st.eta, 1)
        eta, L, Xb, Nhat, Mdot, Q = advance(st, U, lam, pw, tau)
        st = T.HSState(eta, L, Xb, st.n + 1, st.t + tau, Nhat, Mdot, Q, st.L)
    return st


def state_diff(a, b):
    return max(np.max(np.abs(a.eta - b.eta)), abs(a.L - b.L), np.max(np.abs(a.Xbar - b.Xbar)))


def exact_errors(advance=None, taus=(0.02, 0.01)):
    ee, Le, Xe = exact_state(128, T_END)
    ex = T.HSState(ee, Le, Xe)
    return [state_diff(evolve(128, tau, 0.0, 3, False, advance), ex) for tau in taus]


def stiff_orders(pw, lam, advance=None):
    ref = evolve(128, T_END / 1280, lam, pw, True, advance)
    e = [state_diff(evolve(128, tau, lam, pw, True, advance), ref) for tau in (0.02, 0.01, 0.005)]
    return [math.log2(e[0] / e[1]), math.log2(e[1] / e[2])]


def planted(old, new):
    """A copy of oracle.thetal.advance with one source fragment replaced."""
    src = textwrap.dedent(inspect.getsource(T.advance))
    assert old in src
    ns = dict(vars(T))
    exec(src.replace(old, new), ns)
    return ns["advance"]


NO_V = ("V = -spectral.cumulative_meanfree(gfun)", "V = 0.0 * gfun")
WRONG_IF = ("0.5 * tau * (3.0 * e1 * Nhat - e2 * st.Nhat_prev)",
            "0.5 * tau * (3.0 * Nhat - e1 * st.Nhat_prev)")


def test_scaling_plus_offset_law_matches_its_closed_form_at_second_order():
    e = exact_errors()
    assert e[0] < 2e-3 and e[1] < 5e-4, e
    assert 3.6 < e[0] / e[1] < 4.4, e


def test_scaling_plus_offset_law_fails_without_the_tangential_velocity():
    e = exact_errors(planted(*NO_V), taus=(0.01,))
    assert e[0] > 5e-2, e


@pytest.mark.parametrize("pw,lam", [(3, 0.05), (2, 0.2)])
def test_integrating_factor_ab2_is_second_order(pw, lam):
    p = stiff_orders(pw, lam)
    assert all(1.85 < q < 2.2 for q in p), p


@pytest.mark.parametrize("pw,lam", [(3, 0.05), (2, 0.2)])
def test_wrong_integrating_factor_is_caught(pw, lam):
    p = stiff_orders(pw, lam, planted(*WRONG_IF))
    assert min(p) < 1.8, p


def _polar_mode(st, m):
    X, *_ = T.reconstruct(st.eta, st.L, st.Xbar)
    x, y = X[0] - st.Xbar[0], X[1] - st.Xbar[1]
    r, ph = np.hypot(x, y), np.arctan2(y, x)
    A = np.stack([np.ones_like(ph), np.cos(m * ph), np.sin(m * ph)], 1)
    c = np.linalg.lstsq(A, r, rcond=None)[0]
    return math.hypot(c[1], c[2])


def linear_growth(m, J, sigma, steps=40, tau=2.5e-3, R=0.5, d0=1e-3):
    """(measured, predicted) amplification of the mode-m amplitude of r(phi)."""
    X = W.polar_curve(lambda a: R + d0 * np.cos(m * a), 256)
    eta, L, Xb = T.equal_arclength_init(X, 64)
    prm = T.HSParams(sigma=sigma, J=J, tau=tau, box=W.box(-1.5, 1.5, 128))
    st = T.HSState(eta, L, Xb)
    a0 = _polar_mode(st, m)
    for _ in range(steps):
        st, _info = T.hs_step(st, prm)

    def rate(s):
        Rs = math.sqrt(R * R + 2.0 * J * s)
        return (m - 1) * J / Rs ** 2 - sigma * m * (m * m - 1) / Rs ** 3
    return _polar_mode(st, m) / a0, math.exp(quad(rate, 0.0, st.t, epsabs=1e-13)[0])


GROWTH_CASES = [(3, 1.0, 0.02), (5, 0.0, 0.002)]


@pytest.mark.parametrize("m,J,sigma", GROWTH_CASES)
def test_perturbed_circle_grows_at_the_linear_rate(m, J, sigma):
    got, want = linear_growth(m, J, sigma)
    assert abs(got / want - 1.0) < 5e-4, (got, want)


@pytest.mark.parametrize("fault", ["no_V", "wrong_IF"])
def test_growth_rate_pin_catches_planted_mistakes(fault, monkeypatch):
    monkeypatch.setattr(T, "advance", planted(*(NO_V if fault == "no_V" else WRONG_IF)))
    got, want = linear_growth(*GROWTH_CASES[0])
    assert abs(got / want - 1.0) > 1e-3, (got, want)


@pytest.mark.parametrize("ssd", [1, 2])
def test_stefan_step_moves_the_interface_with_the_shared_update(ssd, monkeypatch):
    """The Stefan step hands U = psi, its lambda and the order of its small-scale term
    (second order for case 1, third order for case 2 of Sec. 5.2.2) to the pinned update."""
    from oracle import stefan as S
    seen = {}
    real = S.advance

    def spy(st, U, lam, pw, tau):
        seen.update(U=U.copy(), lam=lam, pw=pw, tau=tau)
        return real(st, U, lam, pw, tau)
    monkeypatch.setattr(S, "advance", spy)
    box = W.box(-1, 1, 32)
    prm = S.StefanParams(box=box, tau=1e-3, eC=(1e-3, 0.0, 0.0, 4, 0.0),
                         eV=(2e-3, 0.0, 0.0, 4, 0.0), bdf2=False, ssd=ssd)
    eta, L, Xb = T.equal_arclength_init(W.circle(16, 0.3), 16)
    _, info = S.stefan_step(S.StefanState(eta, L, Xb, np.full((33, 33), -0.5)), prm)
    assert seen["pw"] == 1 + ssd and seen["lam"] == prm.lam and seen["tau"] == prm.tau
    assert np.array_equal(seen["U"], info.psi)
