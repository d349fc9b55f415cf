"""Pins for oracle.stokes (App. A.2 jumps, the MAC scheme of Sec. 4.2.2, the corrected
scheme and the velocity traces) against flows known in closed form.

The flows are sums of plane waves A sin(a x + b y + g): a stream function psi gives the
divergence-free velocity u = psi_y, v = -psi_x, every derivative of a wave is a wave, and
the forcing f = (Delta - c^2) u - grad p, the traction T(u, p) = -p n + (grad u + grad u^T) n
and the jumps across a curve are evaluated exactly from the two flows.
"""
import math

import numpy as np
import pytest

from oracle import geometry as G
from oracle import stokes as S


class Flow:
    """psi = sum A sin(a x + b y + g) and p = sum B sin(a x + b y + g)."""

    def __init__(self, psi, p):
        self.psi = [tuple(map(float, w)) for w in psi]
        self.p = [tuple(map(float, w)) for w in p]

    @staticmethod
    def _d(waves, m, n, x, y):
        out = 0.0
        for A, a, b, g in waves:
            out = out + A * a ** m * b ** n * np.sin(a * x + b * y + g + 0.5 * math.pi * (m + n))
        return out

    def u(self, m, n, x, y):      # d^m/dx^m d^n/dy^n of u = psi_y
        return self._d(self.psi, m, n + 1, x, y)

    def v(self, m, n, x, y):      # of v = -psi_x
        return -self._d(self.psi, m + 1, n, x, y)

    def pr(self, m, n, x, y):
        return self._d(self.p, m, n, x, y)

    def f(self, c2, x, y):
        f1 = self.u(2, 0, x, y) + self.u(0, 2, x, y) - c2 * self.u(0, 0, x, y) - self.pr(1, 0, x, y)
        f2 = self.v(2, 0, x, y) + self.v(0, 2, x, y) - c2 * self.v(0, 0, x, y) - self.pr(0, 1, x, y)
        return f1, f2

    def traction(self, x, y, nx, ny):
        p, ux, uy = self.pr(0, 0, x, y), self.u(1, 0, x, y), self.u(0, 1, x, y)
        vx, vy = self.v(1, 0, x, y), self.v(0, 1, x, y)
        return (-p * nx + 2 * ux * nx + (uy + vx) * ny, -p * ny + (uy + vx) * nx + 2 * vy * ny)


INSIDE = Flow([(0.7, 1.3, -0.4, 0.2), (0.3, 0.5, 2.1, 1.0)], [(0.9, 1.1, 0.7, 0.3), (0.2, -2.0, 0.5, 0.0)])
OUTSIDE = Flow([(0.5, -0.8, 1.7, 0.6), (0.4, 2.2, 0.3, -0.7)], [(0.6, 0.4, -1.5, 1.2)])


def ellipse(M, ax=0.6, ay=0.4, cx=0.05, cy=-0.03):
    a = 2 * np.pi * np.arange(M) / M
    return np.stack([cx + ax * np.cos(a), cy + ay * np.sin(a)])


def interface_jumps(X, fin, fout, c2):
    """Phi = [u], Psi = [T] at the markers X (outward normal of the counter-clockwise
    curve), the jump of the forcing, and the marker geometry."""
    mk = G.marker_geometry(X)
    x, y = mk.X
    nx, ny = mk.normal
    Phi = np.stack([fin.u(0, 0, x, y) - fout.u(0, 0, x, y), fin.v(0, 0, x, y) - fout.v(0, 0, x, y)])
    ti, to = fin.traction(x, y, nx, ny), fout.traction(x, y, nx, ny)
    Psi = np.stack([ti[0] - to[0], ti[1] - to[1]])
    return mk, Phi, Psi


def fjump_of(fin, fout, c2):
    def fj(x, y):
        a, b = fin.f(c2, x, y), fout.f(c2, x, y)
        return a[0] - b[0], a[1] - b[1]
    return fj


# ----------------------------------------------------------------------------- jumps
@pytest.mark.parametrize("c2", [0.0, 40.0])
def test_jump_systems_give_the_exact_jumps(c2):
    """App. A.2: from [u], [T] and their alpha-derivatives (spectral, 256 markers) and
    [f], the 5x5 and 8x8 systems return every first and second velocity jump and the
    pressure jumps of the two flows."""
    X = ellipse(256)
    mk, Phi, Psi = interface_jumps(X, INSIDE, OUTSIDE, c2)
    q = S.interface_data(Phi, Psi)
    x, y = mk.X
    J = S.jumps(mk.xa, mk.ya, mk.xaa, mk.yaa, q.P1, q.P1a, q.P1aa, q.P2, q.P2a, q.P2aa,
                q.S1, q.S1a, q.S2, q.S2a, c2, *fjump_of(INSIDE, OUTSIDE, c2)(x, y))
    ords = {"": (0, 0), "x": (1, 0), "y": (0, 1), "xx": (2, 0), "yy": (0, 2), "xy": (1, 1)}
    for key in S.JUMP_KEYS:
        comp, d = key[0], key[1:]
        fn = {"u": Flow.u, "v": Flow.v, "p": Flow.pr}[comp]
        exact = fn(INSIDE, *ords[d], x, y) - fn(OUTSIDE, *ords[d], x, y)
        err = np.max(np.abs(J[key] - exact))
        assert err < 1e-9 * max(1.0, np.max(np.abs(exact))), (key, err)


def test_jump_systems_catch_a_wrong_traction_normal():
    """The inward normal in the traction jump must not pass (planted mistake)."""
    X = ellipse(128)
    mk, Phi, Psi = interface_jumps(X, INSIDE, OUTSIDE, 0.0)
    q = S.interface_data(Phi, -Psi)
    x, y = mk.X
    J = S.jumps(mk.xa, mk.ya, mk.xaa, mk.yaa, q.P1, q.P1a, q.P1aa, q.P2, q.P2a, q.P2aa,
                q.S1, q.S1a, q.S2, q.S2a, 0.0, *fjump_of(INSIDE, OUTSIDE, 0.0)(x, y))
    exact = INSIDE.pr(0, 0, x, y) - OUTSIDE.pr(0, 0, x, y)
    assert np.max(np.abs(J["p"] - exact)) > 1e-2


# -------------------------------------------------------------- MAC scheme, no interface
NOSLIP = Flow([(0.25, 0, 0, 0.5 * math.pi), (-0.25, 2 * math.pi, 0, 0.5 * math.pi),
               (-0.25, 0, 2 * math.pi, 0.5 * math.pi),
               (0.125, 2 * math.pi, 2 * math.pi, 0.5 * math.pi),
               (0.125, 2 * math.pi, -2 * math.pi, 0.5 * math.pi)],
              [(1.0, math.pi, 2 * math.pi, 0.3)])   # psi = sin^2(pi x) sin^2(pi y) on [0,1]^2


@pytest.mark.parametrize("c2", [0.0, 100.0])
def test_mac_scheme_converges_at_second_order_for_a_no_slip_flow(c2):
    """Eq. (mac-fds) on [0, 1]^2 with zero box velocity for psi = sin^2(pi x) sin^2(pi y):
    the velocity and the mean-free pressure converge at second order."""
    errs = []
    for N in (16, 32, 64):
        h = 1.0 / N
        I, J = np.meshgrid(np.arange(1, N), np.arange(1, N + 1))
        ru = NOSLIP.f(c2, I * h, (J - 0.5) * h)[0]
        I, J = np.meshgrid(np.arange(1, N + 1), np.arange(1, N))
        rv = NOSLIP.f(c2, (I - 0.5) * h, J * h)[1]
        u, v, p = S.solve_mac(N, h, c2, ru, rv, np.zeros((N, N)))
        I, J = np.meshgrid(np.arange(0, N + 1), np.arange(1, N + 1))
        eu = np.max(np.abs(u - NOSLIP.u(0, 0, I * h, (J - 0.5) * h)))
        I, J = np.meshgrid(np.arange(1, N + 1), np.arange(0, N + 1))
        ev = np.max(np.abs(v - NOSLIP.v(0, 0, (I - 0.5) * h, J * h)))
        I, J = np.meshgrid(np.arange(1, N + 1), np.arange(1, N + 1))
        pe = NOSLIP.pr(0, 0, (I - 0.5) * h, (J - 0.5) * h)
        ep = np.max(np.abs(p - (pe - pe.mean())))
        errs.append((eu, ev, ep))
    errs = np.array(errs)
    order = np.log2(errs[:-1] / errs[1:])
    # measured: velocity 1.98-2.00; pressure 1.79 then 1.90 (c^2 = 100), 2.0 (c^2 = 0)
    assert np.all(order[:, :2] > 1.9) and np.all(order[:, 2] > 1.7), (errs, order)


# ------------------------------------------------------ interface problem, corrected MAC
def run_interface(N, c2, M=None):
    box = G_box(N)
    M = M or 4 * N
    X = ellipse(M)
    mg = S.build_geometry(X, box)
    mk, Phi, Psi = interface_jumps(mg.mk.X, INSIDE, OUTSIDE, c2)

    def f1(x, y, ins):
        return np.where(ins, INSIDE.f(c2, x, y)[0], OUTSIDE.f(c2, x, y)[0])

    def f2(x, y, ins):
        return np.where(ins, INSIDE.f(c2, x, y)[1], OUTSIDE.f(c2, x, y)[1])

    res = S.solve_interface(mg, Phi, Psi, c2, f=(f1, f2), fjump=fjump_of(INSIDE, OUTSIDE, c2),
                            box_u=lambda x, y: OUTSIDE.u(0, 0, x, y),
                            box_v=lambda x, y: OUTSIDE.v(0, 0, x, y))
    h = box.side / N
    x0, y0 = box.x0, box.y0
    I, J = np.meshgrid(np.arange(0, N + 1), np.arange(1, N + 1))
    xu, yu = x0 + I * h, y0 + (J - 0.5) * h
    ins = mg.inside(2 * I, 2 * J - 1)
    eu = np.max(np.abs(res.u - np.where(ins, INSIDE.u(0, 0, xu, yu), OUTSIDE.u(0, 0, xu, yu))))
    I, J = np.meshgrid(np.arange(1, N + 1), np.arange(0, N + 1))
    xv, yv = x0 + (I - 0.5) * h, y0 + J * h
    ins = mg.inside(2 * I - 1, 2 * J)
    ev = np.max(np.abs(res.v - np.where(ins, INSIDE.v(0, 0, xv, yv), OUTSIDE.v(0, 0, xv, yv))))
    I, J = np.meshgrid(np.arange(1, N + 1), np.arange(1, N + 1))
    xp, yp = x0 + (I - 0.5) * h, y0 + (J - 0.5) * h
    ins = mg.inside(2 * I - 1, 2 * J - 1)
    pe = np.where(ins, INSIDE.pr(0, 0, xp, yp), OUTSIDE.pr(0, 0, xp, yp))
    ep = np.max(np.abs(res.p - (pe - pe.mean())))
    x, y = mg.mk.X
    et = max(np.max(np.abs(res.u_plus - np.stack([INSIDE.u(0, 0, x, y), INSIDE.v(0, 0, x, y)]))),
             np.max(np.abs(res.u_minus - np.stack([OUTSIDE.u(0, 0, x, y), OUTSIDE.v(0, 0, x, y)]))))
    return eu, ev, ep, et


class G_box_t:
    def __init__(self, N):
        self.x0, self.y0, self.side, self.N = -1.0, -1.0, 2.0, N


def G_box(N):
    return G_box_t(N)


@pytest.mark.parametrize("c2", [0.0, 50.0])
def test_corrected_mac_scheme_converges_at_second_order(c2):
    """Eq. (crc-mac-fds) for two flows glued along an ellipse with the jumps [u] and [T]
    they define, their forcing on each side and the outside flow on the box: the velocity
    at every MAC point and the traces from both sides at the markers converge at second
    order; the pressure converges at first order."""
    errs = np.array([run_interface(N, c2) for N in (32, 64, 128)])
    order = np.log2(errs[:-1] / errs[1:])
    print("errors (u, v, p, traces)", errs, "orders", order)
    # measured (c^2 = 0 / 50): velocity 1.6-1.95 rising to second order, traces 1.9-2.2,
    # pressure 0.98-1.01 (its jump enters with a first-order Taylor polynomial)
    assert np.all(order[:, [0, 1, 3]] > 1.5) and np.all(order[-1, [0, 1, 3]] > 1.75), (errs, order)
    assert np.all(order[:, 2] > 0.9), (errs, order)


@pytest.mark.parametrize("plant", ["no_pressure_correction", "wrong_side_sign",
                                   "first_order_velocity_taylor"])
def test_corrected_mac_scheme_catches_planted_mistakes(plant, monkeypatch):
    """Each planted mistake in the corrections breaks the second-order pin."""
    good = np.array([run_interface(N, 0.0) for N in (32, 64)])
    real_jumps = S.jumps

    if plant == "no_pressure_correction":
        def jumps(*a, **k):
            J = real_jumps(*a, **k)
            J["p"] = np.zeros_like(J["p"])
            J["px"] = np.zeros_like(J["px"])
            J["py"] = np.zeros_like(J["py"])
            return J
        monkeypatch.setattr(S, "jumps_at", lambda mg, q, c2, k, t, fj=None: jumps(
            *[G.interpolate_at(v, k, t) for v in (mg.mk.xa, mg.mk.ya, mg.mk.xaa, mg.mk.yaa)],
            *[G.interpolate_at(v, k, t) for v in (q.P1, q.P1a, q.P1aa, q.P2, q.P2a, q.P2aa,
                                                   q.S1, q.S1a, q.S2, q.S2a)], c2,
            *((0.0, 0.0) if fj is None else fj)))
    elif plant == "wrong_side_sign":
        monkeypatch.setattr(S, "side_sign", lambda q_inside: -1.0 if q_inside else 1.0)
    else:
        real_jumps_at = S.jumps_at

        def jumps_at(mg, q, c2, k, t, fj=None):
            J = real_jumps_at(mg, q, c2, k, t, fj)
            for key in ("uxx", "uyy", "vxx", "vyy"):
                J[key] = np.zeros_like(J[key])
            return J
        monkeypatch.setattr(S, "jumps_at", jumps_at)
    bad = np.array([run_interface(N, 0.0) for N in (32, 64)])
    print(plant, "good", good, "planted", bad)
    order_bad = np.log2(bad[0, [0, 1, 3]] / bad[1, [0, 1, 3]])
    assert np.max(bad[1, [0, 1, 3]] / good[1, [0, 1, 3]]) > 5.0 or np.min(order_bad) < 1.5
