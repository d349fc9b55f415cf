"""Pins for oracle.geometry (Sec. 4.2 grid / irregular nodes, Sec. 4.3 stencil)."""
import numpy as np
import pytest

from oracle import geometry as G
from paper_2309_01068_amd import workloads as W


def test_lagrange6_reproduces_quintics():
    rng = np.random.default_rng(1)
    c = rng.standard_normal(6)
    P = np.polynomial.Polynomial(c)
    t = rng.uniform(0, 1, 50)
    w, dw = G.lagrange6(t)
    vals = P(G.T_NODES)
    assert np.allclose(w @ vals, P(t), atol=1e-12)
    assert np.allclose(dw @ vals, P.deriv()(t), atol=1e-11)
    assert np.allclose(w.sum(axis=1), 1.0, atol=1e-14)


@pytest.mark.parametrize("N", [32, 64])
def test_circle_crossings_and_labels(N):
    R = 0.61
    box = W.box(-1, 1, N)
    g = G.build_geometry(W.circle(512, R, (0.013, -0.021)), box)
    h = box.side / N
    cx, cy = 0.013, -0.021
    # crossings lie on the circle to Lagrange accuracy
    yj = box.y0 + g.hx.line * h
    r = np.hypot(g.hx.pos - cx, yj - cy)
    assert np.max(np.abs(r - R)) < 1e-9
    xi = box.x0 + g.vx.line * h
    r = np.hypot(xi - cx, g.vx.pos - cy)
    assert np.max(np.abs(r - R)) < 1e-9
    # labels agree with the polar in/out test
    x = box.x0 + np.arange(N + 1) * h
    X, Y = np.meshgrid(x, x)
    assert np.array_equal(g.inside, np.hypot(X - cx, Y - cy) < R)
    # every row crossed by the circle has exactly two crossings
    rows = np.abs(box.y0 + np.arange(1, N) * h - cy) < R
    counts = np.bincount(g.hx.line, minlength=N)[1:N]
    assert np.all(counts[rows] == 2) and np.all(counts[~rows] == 0)
    # irregular arms = label changes between interior node and neighbour
    lab = g.inside
    nar = 0
    for j in range(1, N):
        for i in range(1, N):
            for (di, dj) in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                nar += lab[j, i] != lab[j + dj, i + di]
    assert len(g.arms) == nar


def test_margin_is_enforced():
    with pytest.raises(G.GeometryError):
        G.build_geometry(W.circle(256, 0.95), W.box(-1, 1, 64))


def test_segment_cut_twice_is_not_cut():
    # a sliver far narrower than h: each row segment it spans is cut twice, the grid does
    # not resolve it, so both crossings are dropped and every node stays outside
    N = 32
    M = 256
    a = 2 * np.pi * np.arange(M) / M
    X = np.stack([0.003 * np.cos(a) + 0.0101, 0.5 * np.sin(a)])
    g = G.build_geometry(X, W.box(-1, 1, N))
    assert g.hx.line.size > 0 and not g.hx.keep.any()
    assert not g.inside.any() and g.arms.shape[0] == 0


def test_three_crossings_in_one_segment_rejected():
    cr = G.Crossings(np.array([5, 5, 5, 6]), np.zeros(4, int), np.zeros(4), np.zeros(4),
                     np.array([3, 3, 3, 3]))
    with pytest.raises(G.GeometryError):
        G._pair_out(cr, 32)
    cr = G.Crossings(np.array([5, 5, 6]), np.zeros(3, int), np.zeros(3), np.zeros(3),
                     np.array([3, 3, 3]))
    G._pair_out(cr, 32)
    assert cr.keep.tolist() == [False, False, True]


def test_double_crossing_between_two_markers_is_found():
    # a coarse circle (few markers per h) nearly tangent to the column x = x_i just
    # inside it: the markers next to the tangent point lie left of x_i while the
    # interpolant crosses it twice; both crossings are found and the labels agree
    N = 64
    h = 2.0 / N
    R = 0.75
    xi = -1 + 56 * h                       # column i = 56
    cx = xi - R + 0.004 * h                # the circle pokes 0.004 h past x_i
    M = 96
    a = 2 * np.pi * (np.arange(M) + 0.5) / M   # no marker at the tangent point
    X = np.stack([cx + R * np.cos(a), 0.01 + R * np.sin(a)])
    assert np.all(X[0] < xi)
    g = G.build_geometry(X, W.box(-1, 1, N))
    on = (g.vx.line == 56) & g.vx.keep
    assert on.sum() == 2 or (g.vx.line == 56).sum() == 2


def test_newton_root_accuracy():
    # the Newton root satisfies y_P(t) = y_j to rounding
    M = 128
    a = 2 * np.pi * np.arange(M) / M
    X = np.stack([0.5123 * np.cos(a), 0.5123 * np.sin(a)])
    g = G.build_geometry(X, W.box(-1, 1, 40))
    w, _ = G.lagrange6(g.hx.t)
    idx = G.stencil_markers(g.hx.k, M)
    yP = np.sum(w * X[1][idx], axis=1)
    assert np.max(np.abs(yP - (-1 + g.hx.line * (2 / 40)))) < 1e-14


def test_tangency_is_rejected():
    # a circle touching the line y = 0.5 at a marker gives two crossings at one point
    M = 128
    a = 2 * np.pi * np.arange(M) / M
    X = np.stack([0.5 * np.cos(a), 0.5 * np.sin(a)])
    with pytest.raises(G.GeometryError):
        G.build_geometry(X, W.box(-1, 1, 40))
