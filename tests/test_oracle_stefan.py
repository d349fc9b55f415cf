"""Pins for the Stefan oracle (oracle.stefan, Sec. 2.2, 3.2, 5.2.2)."""
import numpy as np
import pytest
from scipy.special import iv, kv

from oracle import spectral
from oracle import stefan as S
from oracle import thetal as T
from paper_2309_01068_amd import workloads as W

ISO_C = (1e-3, 0.0, 0.0, 4, 0.0)
ISO_V = (2e-3, 0.0, 0.0, 4, 0.0)


def first_step_psi(N, M, tau=1e-2, R=0.3, St=-0.5):
    box = W.box(-2, 2, N)
    prm = S.StefanParams(box=box, tau=tau, eC=ISO_C, eV=ISO_V, bdf2=False, ssd=2)
    eta, L, Xb = T.equal_arclength_init(W.circle(M, R), M)
    st = S.StefanState(eta, L, Xb, np.full((N + 1, N + 1), St))
    _, info = S.stefan_step(st, prm)
    c = np.sqrt(prm.c2)
    exact = (-ISO_C[0] / R - St) / (ISO_V[0] + R * iv(0, c * R) * kv(0, c * R))
    return info, exact


def test_first_step_density_of_a_circle_matches_the_closed_form():
    """Uniform T^0 = St: T1 = St exactly, and eq. bie-GT on a circle with constant psi
    reads (eps_V + R I0(cR) K0(cR)) psi = -eps_C/R - St (free-space single layer; the box
    is 17 decay lengths away).  Second-order convergence of the density."""
    e = []
    for N, M in ((256, 64), (512, 128)):
        info, exact = first_step_psi(N, M)
        assert np.max(np.abs(info.T1_at + 0.5)) < 1e-13
        e.append(np.max(np.abs(info.psi - exact)) / exact)
    assert e[1] < 1e-3 and e[0] / e[1] > 3.0, e


@pytest.mark.parametrize("bdf2", [False, True])
def test_energy_balance(bdf2):
    """sum T h^2 - area(Omega+) is constant for the continuous problem; here it drifts by
    a few per cent of the area change over ten steps from a seed with a staircase
    initial field (discretisation error)."""
    box = W.box(-1, 1, 64)
    prm = S.StefanParams(box=box, tau=1e-3, eC=ISO_C, eV=ISO_V, bdf2=bdf2, ssd=2)
    X = W.circle(32, 0.26)
    eta, L, Xb = T.equal_arclength_init(X, 32)
    st = S.StefanState(eta, L, Xb, S.seed_temperature(box, X, -0.5))
    E0 = S.energy(st, box)
    A0 = T.area(T.reconstruct(eta, L, Xb)[0])
    for _ in range(10):
        st, info = S.stefan_step(st, prm)
        assert info.relres <= 1e-10
    dA = T.area(T.reconstruct(st.eta, st.L, st.Xbar)[0]) - A0
    assert dA > 0.1                                  # the undercooled seed grows
    assert abs(S.energy(st, box) - E0) < 0.05 * dA
    assert np.max(np.abs(st.Xbar)) < 1e-14           # the grid's symmetry is kept


def test_lambda_from_the_frozen_coefficient_formulas():
    box = W.box(-1, 1, 64)
    eC = (2e-3, -0.75, 0.0, 4, 0.0)
    eV = (1e-2, 0.5, 0.0, 4, 0.0)
    p2 = S.StefanParams(box=box, tau=1e-3, eC=eC, eV=eV, ssd=2)
    p1 = S.StefanParams(box=box, tau=1e-3, eC=eC, eV=eV, ssd=1)
    assert abs(p2.lam - 2 * 2e-3 * 1.75) < 1e-15
    phi = 2 * np.pi * np.arange(4096) / 4096
    r = 2e-3 * (1 - 0.75 * np.cos(4 * phi)) / (1e-2 * (1 + 0.5 * np.cos(4 * phi)))
    assert p1.lam == np.max(np.abs(r))
    assert abs(p1.lam - 2e-3 * 1.75 / (1e-2 * 0.5)) < 1e-12   # at cos 4 phi = -1
    # the sampled anisotropy model: the paper's four-fold form 8/3 sin^4(2 phi)
    e = S.eps_model((1.0, -4.0 / 3.0, 1.0 / 3.0, 4, 0.0), phi)
    assert np.max(np.abs(e - 8.0 / 3.0 * np.sin(2 * phi) ** 4)) < 1e-14
    assert p1.c2 == 1.5e3 and S.StefanParams(box=box, tau=1e-3, eC=eC, eV=eV, bdf2=False).c2 == 1e3


def test_ssd_second_order_term_is_damping():
    """L_1 = lambda (2pi/L)^2 theta_aa has Fourier symbol -k^2 (eq. Fourier-theta1)."""
    M = 64
    a = 2 * np.pi * np.arange(M) / M
    for k in (1, 5, 20):
        assert np.allclose(spectral.diff(np.cos(k * a), 2), -k * k * np.cos(k * a), atol=1e-9)


def test_refinement_keeps_the_temperature_and_interpolates_the_state():
    box = W.box(-1, 1, 64)
    X = W.circle(16, 0.2)
    eta, L, Xb = T.equal_arclength_init(X, 16)
    st = S.StefanState(eta, L, Xb, np.full((65, 65), -0.5), psi_prev=np.cos(2 * np.linspace(0, 2 * np.pi, 16, endpoint=False)))
    r = S.refine(st)
    assert r.eta.size == 32 and r.T is st.T and r.L == L
    a2 = np.pi * np.arange(32) / 16
    assert np.max(np.abs(r.psi_prev - np.cos(2 * a2))) < 1e-14
