"""theta-L / small-scale-decomposition Hele-Shaw step (oracle; test-only).

Model (Sec. 2.1, 3.1): pressure p = v + w, v = -J ln|x|, w = D phi + int phi ds solving
    -phi/2 + D phi + int phi ds = -sigma kappa - v   on Gamma   (eq. bie-HS),
normal velocity U = -d_n p = J (x.n)/|x|^2 - d_n(D phi) (from the oil side).
Evolution (Sec. 5.1-5.3): equal-arclength theta-L variables, eta = theta - alpha,
    L_t = int theta_a U da,  theta_t = (2pi/L)(theta_a V - U_a)  (eq. L-evo, the-evo),
    V = (a/2pi) int_0^2pi theta_a U - int_0^a theta_a U,  Xbar_t = (1/2pi) int (U n + V s),
small-scale decomposition with L_2 = lambda_2 (2pi/L)^3 H[theta_aaa], lambda_2 = sigma,
explicit AB2 for L, Xbar and integrating-factor AB2 for eta_hat (eq. Fourier-theta2).

Readings where the paper is inconsistent or silent:
* theta_t sign: the form of eq. (the-evo) is used (the rewritten form in Sec. 5.3 has
  the opposite sign and an undefined T); it is the one that makes L_2 damping.
* AB2 for L and Xbar: L^{n+1} = L^n + (tau/2)(3 M^n - M^{n-1}) with M = +int theta_a U
  (the printed scheme lacks the 1/2 and negates M, contradicting eq. L-evo).
* start-up step: integrating-factor forward Euler.
* U uses the average of the two one-sided normal derivatives of D phi.
* reconstruction X = Xbar + (L/2pi) * antiderivative of (cos theta, sin theta) with the
  k = 0 mode dropped (closure), Nyquist modes zeroed everywhere.
* initialisation: equal-arclength resampling of a sampled curve by Newton on the
  trigonometric interpolant of the arclength function.

Adaptive marker refinement (Sec. 6.1, long-time computation): when the marker spacing
L/M exceeds ratio * h after a step, M is doubled; eta, the last density and the history of
the explicit term are carried to the doubled parameter grid by trigonometric
interpolation (zero padding in Fourier space; the unnormalised DFT doubles).  The paper
gives only the criterion; the interpolation is this reading.

Pinned by: a circle grows as R(t) = sqrt(R0^2 + 2 J t); J = 0 conserves area and
shortens the curve; equal-arclength resampling of a circle/ellipse
(tests/test_oracle_thetal.py); refinement keeps the curve, L, Xbar and the explicit-term
history (tests/test_oracle_refine.py).  The time update `advance` (M, V, Q, the
integrating-factor AB2) is pinned by the closed-form evolution of a non-circular curve
under the velocity law U = c0 + c1 X.n, by second-order time convergence with the
small-scale terms present, and, through hs_step, by the linear growth rate of a perturbed
circle; each of these fails for a dropped V or a wrong integrating factor
(tests/test_oracle_thetal_time.py).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import spectral
from . import geometry as geom
from . import kfbi
from .gmres import gmres

TWO_PI = 2.0 * math.pi


def _trig_coeffs(f: np.ndarray) -> np.ndarray:
    M = f.shape[-1]
    c = np.fft.fft(f) / M
    c[M // 2] = 0.0
    return c


def _trig_eval(c: np.ndarray, beta: np.ndarray, deriv: int = 0) -> np.ndarray:
    """Evaluate the trigonometric interpolant (Nyquist zeroed) or its derivative."""
    M = c.size
    k = spectral.wavenumbers(M)
    e = np.exp(1j * np.outer(np.atleast_1d(beta), k))
    return np.real(e @ (c * (1j * k) ** deriv))


def equal_arclength_init(X: np.ndarray, M: int | None = None):
    """Resample a closed ccw curve given at equispaced parameter samples to M points
    equispaced in arclength.  Returns (eta, L, Xbar)."""
    Mi = X.shape[1]
    M = Mi if M is None else M
    cx, cy = _trig_coeffs(X[0]), _trig_coeffs(X[1])
    b = TWO_PI * np.arange(Mi) / Mi
    sb = np.hypot(spectral.diff(X[0]), spectral.diff(X[1]))
    L = TWO_PI * np.mean(sb)
    cs = _trig_coeffs(sb)
    csm = cs.copy()
    csm[0] = 0.0
    k = spectral.wavenumbers(Mi)
    anti = np.zeros(Mi, dtype=complex)
    nz = k != 0
    anti[nz] = csm[nz] / (1j * k[nz])
    a0 = _trig_eval(anti, np.array([0.0]))[0]

    def s_of(beta):
        return (L / TWO_PI) * beta + _trig_eval(anti, beta) - a0

    target = L * np.arange(M) / M
    beta = TWO_PI * np.arange(M) / M
    for _ in range(50):
        f = s_of(beta) - target
        d = _trig_eval(cs, beta)
        step = f / d
        beta = beta - step
        if np.max(np.abs(step)) < 1e-14:
            break
    xb, yb = _trig_eval(cx, beta), _trig_eval(cy, beta)
    xd, yd = _trig_eval(cx, beta, 1), _trig_eval(cy, beta, 1)
    theta = np.unwrap(np.arctan2(yd, xd))
    alpha = TWO_PI * np.arange(M) / M
    eta = theta - alpha
    Xbar = np.array([np.mean(xb), np.mean(yb)])
    return eta, L, Xbar


def reconstruct(eta: np.ndarray, L: float, Xbar: np.ndarray):
    """X(alpha) from (eta, L, Xbar); returns X (2, M), theta, normal n, tangent s."""
    M = eta.size
    alpha = TWO_PI * np.arange(M) / M
    theta = alpha + eta
    cx = spectral.antiderivative_meanfree(np.cos(theta))
    cy = spectral.antiderivative_meanfree(np.sin(theta))
    X = np.stack([Xbar[0] + (L / TWO_PI) * cx, Xbar[1] + (L / TWO_PI) * cy])
    s = np.stack([np.cos(theta), np.sin(theta)])
    n = np.stack([np.sin(theta), -np.cos(theta)])
    return X, theta, n, s


def area(X: np.ndarray) -> float:
    """A = (1/2) int x.n ds = (1/2) sum (x y_a - y x_a) da."""
    xa, ya = spectral.diff(X[0]), spectral.diff(X[1])
    return 0.5 * np.sum(X[0] * ya - X[1] * xa) * TWO_PI / X.shape[1]


@dataclass
class HSParams:
    sigma: float
    J: float
    tau: float
    box: object
    lam2: float | None = None
    tol: float = 1e-10
    restart: int = 50
    maxit: int = 1000

    @property
    def lambda2(self) -> float:
        return self.sigma if self.lam2 is None else self.lam2


@dataclass
class HSState:
    eta: np.ndarray
    L: float
    Xbar: np.ndarray
    n: int = 0
    t: float = 0.0
    Nhat_prev: np.ndarray | None = None
    Mdot_prev: float = 0.0
    Q_prev: np.ndarray = field(default_factory=lambda: np.zeros(2))
    L_prev: float = 0.0
    phi_prev: np.ndarray | None = None


@dataclass
class StepInfo:
    iters: int
    relres: float
    area: float
    length: float
    phi: np.ndarray
    U: np.ndarray


def advance(st, U: np.ndarray, lam: float, pw: int, tau: float):
    """One theta-L time step given the normal velocity U at the markers (Sec. 5.1, 5.3).

    st carries eta, L, Xbar, the step index n and the previous step's history
    (Nhat_prev, Mdot_prev, Q_prev, L_prev).  With theta = alpha + eta and g = theta_a U:
      M = int g da (eq. L-evo), V = (a/2pi) int g - int_0^a g (equal arclength, Sec. 5.1),
      Q = (1/2pi) int (U n + V s) da (eq. ave-evo),
      N = (2pi/L)(theta_a V - U_a) - lam (2pi/L)^pw P[eta]     (the explicit part),
    with the stiff part P = H[d^3/da^3] (pw = 3, symbol -|k|^3) or d^2/da^2 (pw = 2,
    symbol -k^2) moved into the integrating factor.  L and Xbar take explicit AB2; eta_hat
    takes the integrating-factor AB2 of eq. Fourier-theta1/2 whose factors e_k integrate
    the symbol over [t_n, t_n+1] and [t_n-1, t_n+1] by the trapezoidal rule in time with
    L at the three levels.  The first step is the integrating-factor forward Euler.
    Returns (eta_new, L_new, Xbar_new, Nhat, Mdot, Q), the last three being the history
    of the next step."""
    M = st.eta.size
    L = st.L
    alpha = TWO_PI * np.arange(M) / M
    theta = alpha + st.eta
    s = np.stack([np.cos(theta), np.sin(theta)])
    n = np.stack([np.sin(theta), -np.cos(theta)])
    theta_a = 1.0 + spectral.diff(st.eta, 1)
    gfun = theta_a * U
    Mdot = TWO_PI * np.mean(gfun)
    V = -spectral.cumulative_meanfree(gfun)
    Q = np.array([np.mean(U * n[0] + V * s[0]), np.mean(U * n[1] + V * s[1])])
    if pw == 3:
        Lterm = lam * (TWO_PI / L) ** 3 * spectral.hilbert(spectral.diff(st.eta, 3))
    else:
        Lterm = lam * (TWO_PI / L) ** 2 * spectral.diff(st.eta, 2)
    Nfun = (TWO_PI / L) * (theta_a * V - spectral.diff(U, 1)) - Lterm
    Nhat = np.fft.fft(Nfun)
    k = np.abs(spectral.wavenumbers(M))
    ehat = np.fft.fft(st.eta)
    sym = (TWO_PI * k) ** pw
    if st.n == 0:
        Lnew = L + tau * Mdot
        Xnew = st.Xbar + tau * Q
        e1 = np.exp(-0.5 * lam * tau * sym * (1.0 / L ** pw + 1.0 / Lnew ** pw))
        ehat_new = e1 * (ehat + tau * Nhat)
    else:
        Lnew = L + 0.5 * tau * (3.0 * Mdot - st.Mdot_prev)
        Xnew = st.Xbar + 0.5 * tau * (3.0 * Q - st.Q_prev)
        e1 = np.exp(-0.5 * lam * tau * sym * (1.0 / L ** pw + 1.0 / Lnew ** pw))
        e2 = np.exp(-lam * tau * sym * (0.5 / st.L_prev ** pw + 1.0 / L ** pw + 0.5 / Lnew ** pw))
        ehat_new = e1 * ehat + 0.5 * tau * (3.0 * e1 * Nhat - e2 * st.Nhat_prev)
    ehat_new[M // 2] = 0.0
    eta_new = np.real(np.fft.ifft(ehat_new))
    return eta_new, Lnew, Xnew, Nhat, Mdot, Q


def hs_step(st: HSState, prm: HSParams) -> tuple[HSState, StepInfo]:
    M = st.eta.size
    L = st.L
    X, theta, n, s = reconstruct(st.eta, L, st.Xbar)
    eta_a = spectral.diff(st.eta, 1)
    theta_a = 1.0 + eta_a
    kappa = (TWO_PI / L) * theta_a
    r2 = X[0] ** 2 + X[1] ** 2
    rhs = -prm.sigma * kappa + prm.J * 0.5 * np.log(r2)

    g = geom.build_geometry(X, prm.box)

    def A(x):
        return kfbi.operator(g, x, kfbi.DOUBLE, kfbi.MINUS, 0.0, 1.0, 1.0, 0.0, kfbi.BOX_FREESPACE)

    x0 = np.zeros(M) if st.phi_prev is None else st.phi_prev
    phi, gs = gmres(A, rhs, x0, prm.tol, prm.restart, prm.maxit)
    res = kfbi.apply(g, kfbi.DOUBLE, phi, 0.0, kfbi.BOX_FREESPACE)
    dn = 0.5 * (res.dn_plus + res.dn_minus)
    U = prm.J * (X[0] * n[0] + X[1] * n[1]) / r2 - dn

    eta_new, Lnew, Xnew, Nhat, Mdot, Q = advance(st, U, prm.lambda2, 3, prm.tau)
    tau = prm.tau
    new = HSState(eta_new, Lnew, Xnew, st.n + 1, st.t + tau, Nhat, Mdot, Q, L, phi)
    info = StepInfo(gs.iters, gs.relres, area(X), L, phi, U)
    return new, info


def refine(st: HSState) -> HSState:
    """Double the markers of the state by trigonometric interpolation in alpha."""
    M = st.eta.size
    eta2 = spectral.upsample2(st.eta)
    nh = None
    if st.Nhat_prev is not None:
        nh = np.zeros(2 * M, dtype=complex)
        h = M // 2
        nh[:h] = 2.0 * st.Nhat_prev[:h]
        nh[2 * M - h + 1:] = 2.0 * st.Nhat_prev[h + 1:]
    phi = None if st.phi_prev is None else spectral.upsample2(st.phi_prev)
    return HSState(eta2, st.L, st.Xbar.copy(), st.n, st.t, nh, st.Mdot_prev, st.Q_prev.copy(),
                   st.L_prev, phi)


def refine_due(st: HSState, h: float, ratio: float, max_M: int) -> bool:
    """The refinement criterion: marker spacing L/M above ratio * h, room to double."""
    M = st.eta.size
    return ratio > 0.0 and st.L / M > ratio * h and 2 * M <= max_M
