"""Stefan problem step: Gibbs-Thomson boundary integral equation, temperature update and
theta-L / small-scale-decomposition interface motion (oracle; test-only).

Model (Sec. 2.2, 3.2): solid Omega+ inside Gamma, liquid Omega- outside, heat equation
in both phases, zero normal derivative of T on the box.  Time discretisation of the
heat equation (no flow, so the departure points are the grid nodes):
    backward Euler  (Delta - 1/tau) T^{n+1} = -T^n / tau,
    BDF2            (Delta - 3/(2 tau)) T^{n+1} = (T^{n-1} - 4 T^n) / (2 tau),
c^2 the constant on the left.  T^{n+1} = T1 + T2 with
    (Delta_h - c^2) T1 = right-hand side on the box (five-point scheme, mirrored ghosts),
    T2 = -S psi, the single layer of the box Green's function, psi = [d_n T2] = U,
and the Gibbs-Thomson relation T = -eps_C kappa - eps_V U on Gamma gives
    eps_V psi - S psi = -eps_C kappa - T1    on Gamma     (eq. bie-GT),
solved by GMRES with the KFBI operator {S, average trace, a = eps_V, b = -1}.
The interface moves with normal velocity U = psi by the theta-L equations of the
Hele-Shaw oracle (Sec. 5.1), with the small-scale decomposition of Sec. 5.2.2:
    case 1 (eps_V = O(1)): L_1 = lambda_1 (2pi/L)^2 theta_aa,  lambda_1 = max |eps_C/eps_V|
    case 2 (eps_V << 1):   L_2 = lambda_2 (2pi/L)^3 H[theta_aaa], lambda_2 = max |2 eps_C|
and the integrating-factor AB2 of eq. Fourier-theta1/2 (forward-Euler start).

Readings where the paper is silent:
* the boundary integral equation of step n is posed on the interface Gamma^n (the
  interface moves explicitly; the temperature is implicit);
* T1 at the markers is the six-point interpolation of Sec. 4.3 with zero jumps;
* BDF2 starts with T^{-1} = T^0 (a first-order first step with the same c^2);
* anisotropy eps(n) = e0 (1 + e1 cos(m (phi - phi0)) + e2 cos(2 m (phi - phi0))) of the
  angle phi of the outward normal with the x axis; lambda_1, lambda_2 are the maxima of
  the frozen-coefficient formulas over phi sampled at 4096 equispaced angles;
* the temperature is kept on the grid nodes (N+1)^2; the area of Omega+ for the energy
  balance is the curve's enclosed area.

Marker refinement as for the Hele-Shaw state (oracle.thetal.refine): eta, the last density
and the explicit-term history go to the doubled parameter grid by trigonometric
interpolation; the temperature is untouched.

The interface update is oracle.thetal.advance with U = psi, lambda of the chosen case
and the second- or third-order small-scale term.

Pinned by: the first-step density for a circle in a uniform field against the closed
form of the free-space single layer, the energy balance sum(T) h^2 - area(Omega+) kept
to discretisation error, the symmetry of a growing circle, and the two SSD propagators'
Fourier symbols (tests/test_oracle_stefan.py); the shared update's pins of both orders
and the hand-over of U, lambda and the order (tests/test_oracle_thetal_time.py).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import geometry as geom
from . import kfbi
from . import spectral
from .gmres import gmres
from .thetal import reconstruct, area, advance

TWO_PI = 2.0 * math.pi
N_LAMBDA = 4096


def eps_model(c, phi):
    """e0 (1 + e1 cos(m (phi - phi0)) + e2 cos(2 m (phi - phi0))), c = (e0, e1, e2, m, phi0)."""
    e0, e1, e2, m, p0 = c
    return e0 * (1.0 + e1 * np.cos(m * (phi - p0)) + e2 * np.cos(2 * m * (phi - p0)))


@dataclass
class StefanParams:
    box: object
    tau: float
    eC: tuple           # (e0, e1, e2, m, phi0)
    eV: tuple
    bdf2: bool = True
    ssd: int = 2        # 1: L_1 (second order), 2: L_2 (third order)
    tol: float = 1e-10
    restart: int = 50
    maxit: int = 1000

    @property
    def c2(self) -> float:
        return 1.5 / self.tau if self.bdf2 else 1.0 / self.tau

    @property
    def lam(self) -> float:
        phi = TWO_PI * np.arange(N_LAMBDA) / N_LAMBDA
        eC, eV = eps_model(self.eC, phi), eps_model(self.eV, phi)
        if self.ssd == 1:
            return float(np.max(np.abs(eC / eV)))
        return float(np.max(np.abs(2.0 * eC)))


@dataclass
class StefanState:
    eta: np.ndarray
    L: float
    Xbar: np.ndarray
    T: np.ndarray                      # (N+1, N+1) grid temperature [j, i]
    T_prev: np.ndarray | None = None
    n: int = 0
    t: float = 0.0
    Nhat_prev: np.ndarray | None = None
    Mdot_prev: float = 0.0
    Q_prev: np.ndarray | None = None
    L_prev: float = 0.0
    psi_prev: np.ndarray | None = None


@dataclass
class StefanInfo:
    iters: int
    relres: float
    area: float
    length: float
    psi: np.ndarray
    T1_at: np.ndarray
    rhs: np.ndarray


def t1_rhs(st: StefanState, prm: StefanParams) -> np.ndarray:
    """Right-hand side of the T1 problem on the grid."""
    if not prm.bdf2:
        return -st.T / prm.tau
    Tp = st.T if st.T_prev is None else st.T_prev
    return (Tp - 4.0 * st.T) / (2.0 * prm.tau)


def interp_smooth(g, grid):
    """Six-point interpolation of Sec. 4.3 at the markers with zero jumps."""
    z = np.zeros(g.mk.M)
    vp, *_ = kfbi.extract(g, grid, (z, z, z, z, z, z))
    return vp


def stefan_step(st: StefanState, prm: StefanParams) -> tuple[StefanState, StefanInfo]:
    M = st.eta.size
    L = st.L
    box = prm.box
    h = box.side / box.N
    c2 = prm.c2
    X, theta, n, s = reconstruct(st.eta, L, st.Xbar)
    g = geom.build_geometry(X, box)
    theta_a = 1.0 + spectral.diff(st.eta, 1)
    kappa = (TWO_PI / L) * theta_a
    nphi = theta - 0.5 * math.pi           # angle of n = (sin theta, -cos theta)
    epsC, epsV = eps_model(prm.eC, nphi), eps_model(prm.eV, nphi)

    T1 = kfbi.solve_neumann(t1_rhs(st, prm), h, c2)
    T1_at = interp_smooth(g, T1)
    rhs = -epsC * kappa - T1_at

    def A(x):
        return kfbi.operator(g, x, kfbi.SINGLE, kfbi.AVG, epsV, -1.0, 0.0, c2, kfbi.BOX_NEUMANN)

    x0 = np.zeros(M) if st.psi_prev is None else st.psi_prev
    psi, gs = gmres(A, rhs, x0, prm.tol, prm.restart, prm.maxit)
    T2 = kfbi.apply(g, kfbi.SINGLE, -psi, c2, kfbi.BOX_NEUMANN).grid
    Tnew = T1 + T2

    U = psi
    eta_new, Lnew, Xnew, Nhat, Mdot, Q = advance(st, U, prm.lam, 1 + prm.ssd, prm.tau)
    tau = prm.tau
    new = StefanState(eta_new, Lnew, Xnew, Tnew, st.T, st.n + 1, st.t + tau, Nhat, Mdot, Q, L,
                      psi)
    info = StefanInfo(gs.iters, gs.relres, area(X), L, psi, T1_at, rhs)
    return new, info


def seed_temperature(box, X, St: float) -> np.ndarray:
    """Initial field of a seed crystal: 0 (melting temperature) inside the curve X, St in
    the undercooled liquid; labels from the geometry of the grid crossings."""
    g = geom.build_geometry(X, box)
    return np.where(g.inside, 0.0, St).astype(np.float64)


def energy(st: StefanState, box) -> float:
    """sum of T over the box with trapezoid weights times h^2, minus the solid area
    (constant in time for the continuous problem with unit latent heat)."""
    h = box.side / box.N
    w = np.ones(box.N + 1)
    w[0] = w[-1] = 0.5
    X, *_ = reconstruct(st.eta, st.L, st.Xbar)
    return float(np.sum(w[:, None] * w[None, :] * st.T) * h * h - area(X))


def refine(st: StefanState) -> StefanState:
    """Double the markers (trigonometric interpolation of eta, psi and the DFT history)."""
    from .thetal import HSState, refine as hs_refine
    r = hs_refine(HSState(st.eta, st.L, st.Xbar, st.n, st.t, st.Nhat_prev, st.Mdot_prev,
                          np.zeros(2) if st.Q_prev is None else st.Q_prev, st.L_prev,
                          st.psi_prev))
    return StefanState(r.eta, st.L, st.Xbar.copy(), st.T, st.T_prev, st.n, st.t, r.Nhat_prev,
                       st.Mdot_prev, None if st.Q_prev is None else st.Q_prev.copy(), st.L_prev,
                       r.phi_prev)
