"""Pins for oracle.kfbi: the DST-I solve, App. A jumps, the corrected scheme, the
corrected interpolation and whole applies against closed forms (Sec. 4.1-4.3, App. A.1)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.special import iv, kv, ivp, kvp

from oracle import geometry as G
from oracle import kfbi as K
from paper_2309_01068_amd import workloads as W


# ------------------------------------------------------------------ DST-I and solve
def test_dst1_matches_brute_force_sum():
    rng = np.random.default_rng(0)
    for n in (1, 2, 7, 15):
        a = rng.standard_normal(n)
        i = np.arange(1, n + 1)
        S = np.sin(np.pi * np.outer(i, i) / (n + 1))
        assert np.allclose(K.dst1(a, 0), S @ a, atol=1e-13)


@pytest.mark.parametrize("c2", [0.0, 50.0])
def test_solve_matches_sparse_direct(c2):
    N, h = 16, 0.13
    n = N - 1
    rng = np.random.default_rng(1)
    rhs = rng.standard_normal((n, n))
    T = sp.diags([np.ones(n - 1), -2 * np.ones(n), np.ones(n - 1)], [-1, 0, 1])
    I = sp.identity(n)
    A = (sp.kron(I, T) + sp.kron(T, I)) / h ** 2 - c2 * sp.identity(n * n)
    v_direct = spla.spsolve(A.tocsc(), rhs.ravel()).reshape(n, n)
    v = K.solve_fivepoint(rhs, h, c2)
    assert np.max(np.abs(v - v_direct)) < 1e-12 * np.max(np.abs(v_direct))


@pytest.mark.parametrize("c2", [0.0, 1000.0])
def test_solve_recovers_manufactured_grid_function(c2):
    N, h = 256, 2.0 / 256
    rng = np.random.default_rng(2)
    v = rng.standard_normal((N - 1, N - 1))
    rhs = K.fivepoint_apply(v, h, c2)
    assert np.max(np.abs(K.solve_fivepoint(rhs, h, c2) - v)) < 1e-11


# ----------------------------------------------------------------------------- jumps
def _ellipse_geom(M, ax=0.6, ay=0.4, x0=0.05, y0=-0.03):
    a = 2 * np.pi * np.arange(M) / M
    X = np.stack([x0 + ax * np.cos(a), y0 + ay * np.sin(a)])
    return G.marker_geometry(X)


@pytest.mark.parametrize("c", [0.0, 3.0])
def test_appendix_jumps_match_exact_jumps(c):
    """u+- with (Delta - c^2) u = 0 on both sides; jumps of u and derivatives from
    (Phi, Psi) along the curve must equal the exact differences (App. A.1)."""
    mk = _ellipse_geom(256)
    x, y = mk.X
    if c == 0.0:
        up = lambda x, y: (x * x - y * y + 0.3 * x * y, 2 * x + 0.3 * y, -2 * y + 0.3 * x, 2.0, -2.0, 0.3)
        um = lambda x, y: (np.exp(x) * np.sin(y), np.exp(x) * np.sin(y), np.exp(x) * np.cos(y),
                           np.exp(x) * np.sin(y), -np.exp(x) * np.sin(y), np.exp(x) * np.cos(y))
    else:
        def mk_exp(th):
            cx, cy = c * np.cos(th), c * np.sin(th)
            def f(x, y):
                e = np.exp(cx * x + cy * y)
                return e, cx * e, cy * e, cx * cx * e, cy * cy * e, cx * cy * e
            return f
        up, um = mk_exp(0.3), mk_exp(2.1)
    P, Mi = up(x, y), um(x, y)
    jump = [p - m for p, m in zip(P, Mi)]            # [u],[ux],[uy],[uxx],[uyy],[uxy]
    nx, ny = mk.normal
    Phi = jump[0]
    Psi = nx * jump[1] + ny * jump[2]
    q = K.marker_quantities(Phi, Psi)
    J = K.jumps(mk.xa, mk.ya, mk.xaa, mk.yaa, *q, c * c)
    for got, want in zip(J, jump):
        assert np.max(np.abs(got - want)) < 1e-9 * max(1.0, np.max(np.abs(want)))


# --------------------------------------------------------------- corrected scheme
def _piecewise_quadratic():
    up = lambda x, y: x * x - y * y + x * y + 0.2
    um = lambda x, y: 2 * x * y - x + 0.1 * y
    gup = lambda x, y: (2 * x + y, -2 * y + x)
    gum = lambda x, y: (2 * y - 1.0, 2 * x + 0.1)
    return up, um, gup, gum


@pytest.mark.parametrize("curve,N", [("ellipse", 64), ("star", 128)])
def test_corrected_scheme_exact_for_piecewise_harmonic_quadratics(curve, N):
    """Harmonic quadratics have zero truncation error in the five-point scheme and the
    second-order correction is exact for them, so the grid solution equals u+- at every
    node up to the interpolation of interface data between markers.  The star passes
    through the grid node (0, 0.5) up to rounding (column-crossing snapping)."""
    box = W.box(-1, 1, N)
    X = W.ellipse(512) if curve == "ellipse" else W.star(256)
    g = G.build_geometry(X, box)
    up, um, gup, gum = _piecewise_quadratic()
    x, y = g.mk.X
    nx, ny = g.mk.normal
    Phi = up(x, y) - um(x, y)
    gp, gm = gup(x, y), gum(x, y)
    Psi = nx * (gp[0] - gm[0]) + ny * (gp[1] - gm[1])
    zx, zy = K.ring_nodes(box)
    res = K.solve_interface(g, Phi, Psi, 0.0, um(zx, zy))
    h = box.side / N
    X, Y = np.meshgrid(box.x0 + np.arange(N + 1) * h, box.y0 + np.arange(N + 1) * h)
    exact = np.where(g.inside, up(X, Y), um(X, Y))
    # tolerance = 6-point Lagrange error of the interface data (the 5-fold star has
    # large high derivatives); a mis-assigned crossing would give errors ~h
    tol = 1e-8 if curve == "ellipse" else 2e-6
    assert np.max(np.abs(res.grid - exact)) < tol
    # and the extracted one-sided traces are exact too
    assert np.max(np.abs(res.v_plus - up(x, y))) < tol
    assert np.max(np.abs(res.v_minus - um(x, y))) < tol
    assert np.max(np.abs(res.dn_plus - (nx * gp[0] + ny * gp[1]))) < 10 * tol
    assert np.max(np.abs(res.dn_minus - (nx * gm[0] + ny * gm[1]))) < 10 * tol


def test_extraction_exact_on_quadratics():
    N = 48
    box = W.box(-1, 1, N)
    g = G.build_geometry(W.star(300), box)
    h = box.side / N
    up = lambda x, y: 1.0 + 2 * x - y + 0.5 * x * x + 3 * x * y - y * y
    um = lambda x, y: -0.5 + x + 4 * y - 2 * x * x + x * y + 0.7 * y * y
    X, Y = np.meshgrid(box.x0 + np.arange(N + 1) * h, box.y0 + np.arange(N + 1) * h)
    grid = np.where(g.inside, up(X, Y), um(X, Y))
    x, y = g.mk.X
    Jm = (up(x, y) - um(x, y), (2 + x + 3 * y) - (1 - 4 * x + y), (-1 + 3 * x - 2 * y) - (4 + x + 1.4 * y),
          (1.0 - (-4.0)) * np.ones_like(x), (-2.0 - 1.4) * np.ones_like(x), (3.0 - 1.0) * np.ones_like(x))
    vp, vxp, vyp, vm, vxm, vym = K.extract(g, grid, Jm)
    assert np.max(np.abs(vp - up(x, y))) < 1e-11
    assert np.max(np.abs(vxp - (2 + x + 3 * y))) < 1e-9
    assert np.max(np.abs(vyp - (-1 + 3 * x - 2 * y))) < 1e-9
    assert np.max(np.abs(vm - um(x, y))) < 1e-11


# ------------------------------------------------------- layer potentials on circles
R_C, M_C = 0.6, 3


def circle_exact(layer, c, zx, zy):
    """Closed forms of S/D with density cos(m theta) on the circle r = R (free space)."""
    R, m = R_C, M_C
    r = np.hypot(zx, zy)
    th = np.arctan2(zy, zx)
    rl, rg = np.minimum(r, R), np.maximum(r, R)
    if c == 0.0:
        if layer == K.DOUBLE:
            return np.where(r < R, 0.5 * (r / R) ** m, -0.5 * (R / r) ** m) * np.cos(m * th)
        return -(R / (2 * m)) * (rl / rg) ** m * np.cos(m * th)
    if layer == K.SINGLE:
        return -R * iv(m, c * rl) * kv(m, c * rg) * np.cos(m * th)
    return np.where(r < R, -c * R * kvp(m, c * R) * iv(m, c * r),
                    -c * R * ivp(m, c * R) * kv(m, c * r)) * np.cos(m * th)


def circle_trace_factors(layer, c):
    """(v+, v-, d_n v+, d_n v-) on r = R divided by cos(m theta)."""
    R, m = R_C, M_C
    if c == 0.0:
        if layer == K.DOUBLE:
            return 0.5, -0.5, 0.5 * m / R, 0.5 * m / R
        return -R / (2 * m), -R / (2 * m), -0.5, 0.5
    if layer == K.SINGLE:
        v = -R * iv(m, c * R) * kv(m, c * R)
        return v, v, -R * c * ivp(m, c * R) * kv(m, c * R), -R * c * iv(m, c * R) * kvp(m, c * R)
    return (-c * R * kvp(m, c * R) * iv(m, c * R), -c * R * ivp(m, c * R) * kv(m, c * R),
            -c * c * R * kvp(m, c * R) * ivp(m, c * R), -c * c * R * ivp(m, c * R) * kvp(m, c * R))


def circle_errors(layer, c, Ns=(64, 128, 256)):
    errs = []
    for N in Ns:
        box = W.box(-1, 1, N)
        X = W.circle(4 * N, R_C)
        g = G.build_geometry(X, box)
        dens = np.cos(M_C * np.arctan2(X[1], X[0]))
        zx, zy = K.ring_nodes(box)
        res = K.apply(g, layer, dens, c * c, K.BOX_USER, circle_exact(layer, c, zx, zy))
        fp, fm, dp, dm = circle_trace_factors(layer, c)
        errs.append(max(np.max(np.abs(res.v_plus - fp * dens)), np.max(np.abs(res.v_minus - fm * dens)),
                        np.max(np.abs(res.dn_plus - dp * dens)) * (2.0 / N),
                        np.max(np.abs(res.dn_minus - dm * dens)) * (2.0 / N)))
    return np.array(errs)


@pytest.mark.parametrize("layer", [K.SINGLE, K.DOUBLE])
@pytest.mark.parametrize("c", [0.0, 5.0])
def test_layer_potentials_on_circle_converge(layer, c):
    e = circle_errors(layer, c)
    order = np.log2(e[0] / e[-1]) / (len(e) - 1)
    assert e[-1] < 5e-5
    assert order > 1.6, (e, order)


def test_planted_sign_error_is_caught(monkeypatch):
    """A plausible mistake (wrong sign of the tangential-derivative jump) must fail the
    circle pin: the pin is not vacuous."""
    real = K.jumps

    def wrong(*args, **kw):
        out = list(real(*args, **kw))
        out[1] = -out[1]
        return tuple(out)
    monkeypatch.setattr(K, "jumps", wrong)
    e = circle_errors(K.DOUBLE, 0.0, Ns=(64, 128))
    assert e[-1] > 1e-2


def test_planted_ring_sign_error_is_caught(monkeypatch):
    real = K.corrected_rhs

    def wrong(g, q, c2, ring):
        return real(g, q, c2, None if ring is None else -ring)
    monkeypatch.setattr(K, "corrected_rhs", wrong)
    e = circle_errors(K.SINGLE, 0.0, Ns=(64, 128))
    assert e[-1] > 1e-2


@pytest.mark.parametrize("layer", [K.SINGLE, K.DOUBLE])
def test_freespace_box_data_matches_closed_form(layer):
    box = W.box(-1, 1, 64)
    X = W.circle(256, R_C)
    g = G.build_geometry(X, box)
    dens = np.cos(M_C * np.arctan2(X[1], X[0]))
    ring = K.freespace_ring(g, layer, dens)
    zx, zy = K.ring_nodes(box)
    assert np.max(np.abs(ring - circle_exact(layer, 0.0, zx, zy))) < 1e-12
