"""Interface geometry on the Cartesian grid (oracle; test-only).

Follows Sec. 4.2 (grid, irregular nodes, grid-line/interface intersection points) and
Sec. 4.3 (interpolation stencil).  The paper does not say how the interface is
evaluated between markers, how intersections are located, or how nodes are labelled
inside/outside; the readings used (identical on the GPU side, written independently):

* grid: x_i = x0 + i h, y_j = y0 + j h, i, j = 0..N, h = side/N (Sec. 4.2: N intervals);
* markers X_k at a_k = 2 pi k/M, counter-clockwise, outward normal (y_a, -x_a)/s_a (App. A);
* between markers, every marker quantity is interpolated by the 6-point Lagrange
  polynomial through markers k-2..k+3 in the local variable t = (a - a_k)/da in [0, 1];
* crossings are searched on the interpolant sampled at t = s/8, s = 0..8, of each marker
  interval (marker values at the ends): sub-interval s crosses y = y_j iff
  (y(t_s) >= y_j) != (y(t_{s+1}) >= y_j), so a curve nearly tangent to a line between
  two markers shows both of its crossings; the crossing parameter solves y_P(t) = y_j on
  the sub-interval by safeguarded Newton (bisection fallback);
* a grid segment cut exactly twice is treated as not cut (the grid does not resolve the
  bump between the two crossings; both are dropped); three or more crossings in one
  segment are a geometry error;
* node (i, j) lies in Omega+ iff the number of kept row-j crossings with xi < x_i is odd;
* every marker must stay 3h away from the box boundary; a label change without a
  crossing is a geometry error;
* a column crossing within 1e-9 h of a grid node may move to the adjacent column
  segment so that it sits where the row-based labels change (the interface passes
  through that node up to rounding).

Pinned by: exact crossings of straight/circular curves, label parity vs. a polar
in/out test on a circle, arm counts (tests/test_oracle_geometry.py).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import spectral

T_NODES = np.arange(-2.0, 4.0)       # Lagrange nodes t_m = m - 2, markers k-2..k+3


class GeometryError(RuntimeError):
    pass


def lagrange6(t: np.ndarray):
    """Weights l_m(t) and derivatives l_m'(t) of the 6-point Lagrange basis on t_m = m-2.

    Returns arrays of shape t.shape + (6,)."""
    t = np.asarray(t, dtype=np.float64)[..., None]
    tm = T_NODES
    w = np.ones(t.shape[:-1] + (6,))
    dw = np.zeros(t.shape[:-1] + (6,))
    for m in range(6):
        denom = 1.0
        for q in range(6):
            if q != m:
                denom *= (tm[m] - tm[q])
        # l_m(t) = prod_{q != m} (t - t_q) / denom
        prod = np.ones(t.shape[:-1])
        for q in range(6):
            if q != m:
                prod = prod * (t[..., 0] - tm[q])
        w[..., m] = prod / denom
        # derivative: sum_r prod_{q != m, r} (t - t_q) / denom
        d = np.zeros(t.shape[:-1])
        for r in range(6):
            if r == m:
                continue
            pr = np.ones(t.shape[:-1])
            for q in range(6):
                if q != m and q != r:
                    pr = pr * (t[..., 0] - tm[q])
            d = d + pr
        dw[..., m] = d / denom
    return w, dw


def stencil_markers(k: np.ndarray, M: int) -> np.ndarray:
    """Marker indices k-2..k+3 (periodic) for intervals k; shape k.shape + (6,)."""
    return (np.asarray(k)[..., None] + np.arange(-2, 4)) % M


@dataclass
class Markers:
    X: np.ndarray          # (2, M)
    xa: np.ndarray
    ya: np.ndarray
    xaa: np.ndarray
    yaa: np.ndarray
    sa: np.ndarray
    saa: np.ndarray

    @property
    def M(self) -> int:
        return self.X.shape[1]

    @property
    def normal(self) -> np.ndarray:
        return np.stack([self.ya, -self.xa]) / self.sa


def marker_geometry(X: np.ndarray) -> Markers:
    """Spectral derivatives of the marker positions (App. A: n = (y_a, -x_a)/s_a,
    s_a = |X_a|; s_aa = (x_a x_aa + y_a y_aa)/s_a)."""
    x, y = X
    xa, ya = spectral.diff(x, 1), spectral.diff(y, 1)
    xaa, yaa = spectral.diff(x, 2), spectral.diff(y, 2)
    sa = np.hypot(xa, ya)
    saa = (xa * xaa + ya * yaa) / sa
    return Markers(X.copy(), xa, ya, xaa, yaa, sa, saa)


def grid_coord(lo: float, h: float, i):
    return lo + np.asarray(i, dtype=np.float64) * h


def _newton_root(c: np.ndarray, target: np.ndarray, a: np.ndarray, b: np.ndarray,
                 ta: np.ndarray | None = None, tb: np.ndarray | None = None):
    """Solve P(t) = target on [ta, tb] (default [0, 1]) where P is the Lagrange
    polynomial with nodal values c (shape (K, 6)); a = P(ta) - target, b = P(tb) - target
    have opposite signs under the rule sign(v) = (v >= 0).  Safeguarded Newton: start
    from the secant point, keep a bracket, bisect whenever Newton leaves it; stop when the
    update is below 1e-12 (in t) or after 60 iterations."""
    K = c.shape[0]
    lo = np.zeros(K) if ta is None else np.array(ta, dtype=np.float64)
    hi = np.ones(K) if tb is None else np.array(tb, dtype=np.float64)
    t = lo + (hi - lo) * (a / (a - b))
    sa = a >= 0.0
    done = np.zeros(K, dtype=bool)
    for _ in range(60):
        w, dw = lagrange6(t)
        f = np.sum(w * c, axis=1) - target
        fp = np.sum(dw * c, axis=1)
        same = (f >= 0.0) == sa
        lo = np.where(same & ~done, t, lo)
        hi = np.where(~same & ~done, t, hi)
        with np.errstate(divide="ignore", invalid="ignore"):
            tn = t - f / fp
        bad = ~np.isfinite(tn) | (tn <= lo) | (tn >= hi)
        tn = np.where(bad, 0.5 * (lo + hi), tn)
        tn = np.where(f == 0.0, t, tn)
        step = np.abs(tn - t)
        t = np.where(done, t, tn)
        done = done | (step <= 1e-12)
        if done.all():
            break
    return t


# Sub-intervals per marker interval in the crossing search: the interpolant is sampled at
# t = s / SUB so that a line crossed twice between two markers (the curve nearly tangent
# to it) is found.
SUB = 8


@dataclass
class Crossings:
    """Intersections of the interface with grid lines."""
    line: np.ndarray       # j (horizontal lines y = y_j) or i (vertical lines x = x_i)
    k: np.ndarray          # marker interval
    t: np.ndarray          # local parameter in [0, 1]
    pos: np.ndarray        # x-coordinate (horizontal lines) or y-coordinate (vertical)
    seg: np.ndarray        # grid segment index: node index m with g_m <= pos < g_{m+1}
    keep: np.ndarray | None = None  # False for the two crossings of a segment cut twice


def find_crossings(mk: Markers, lo: float, h: float, N: int, axis: int) -> Crossings:
    """Crossings with lines y = y_j (axis=1: the varying coordinate is y) or x = x_i
    (axis=0), lines 1..N-1 (Sec. 4.2: intersection point (xi, y_j)).  Within marker
    interval k the coordinate follows the 6-point Lagrange polynomial through markers
    k-2..k+3; it is sampled at t = s/SUB (the marker values themselves at t = 0, 1) and a
    line g is crossed in sub-interval s iff (v(t_s) >= g) != (v(t_{s+1}) >= g)."""
    M = mk.M
    v = mk.X[axis]                 # coordinate compared with the line
    other = mk.X[1 - axis]
    kk_all = np.arange(M)
    cv = v[stencil_markers(kk_all, M)]                   # (M, 6)
    ts = np.arange(SUB + 1, dtype=np.float64) / SUB
    Wt, _ = lagrange6(ts)                                # (SUB+1, 6)
    vals = np.zeros((M, SUB + 1))
    for m in range(6):
        vals = vals + cv[:, m:m + 1] * Wt[None, :, m]
    vals[:, 0] = v
    vals[:, SUB] = np.roll(v, -1)
    jl = np.floor((vals.min(axis=1) - lo) / h).astype(np.int64) - 1
    jh = np.floor((vals.max(axis=1) - lo) / h).astype(np.int64) + 1
    ks, js, ss = [], [], []
    for kk in range(M):
        for j in range(max(jl[kk], 1), min(jh[kk], N - 1) + 1):
            above = vals[kk] >= lo + j * h
            for sidx in np.nonzero(above[:-1] != above[1:])[0]:
                ks.append(kk)
                js.append(j)
                ss.append(int(sidx))
    ks = np.array(ks, dtype=np.int64)
    js = np.array(js, dtype=np.int64)
    ss = np.array(ss, dtype=np.int64)
    if ks.size == 0:
        z = np.zeros(0)
        return Crossings(js, ks, z, z.copy(), js.copy(), np.ones(0, dtype=bool))
    g = lo + js * h
    idx = stencil_markers(ks, M)
    c = v[idx]
    t = _newton_root(c, g, vals[ks, ss] - g, vals[ks, ss + 1] - g, ts[ss], ts[ss + 1])
    w, _ = lagrange6(t)
    pos = np.sum(w * other[idx], axis=1)
    seg = np.floor((pos - lo) / h).astype(np.int64)
    # exact placement: lo + seg*h <= pos < lo + (seg+1)*h
    for _ in range(2):
        seg = np.where(lo + (seg + 1) * h <= pos, seg + 1, seg)
        seg = np.where(lo + seg * h > pos, seg - 1, seg)
    return Crossings(js, ks, t, pos, seg, np.ones(ks.size, dtype=bool))


def _pair_out(cr: Crossings, N: int):
    """A grid segment cut twice is treated as not cut (the grid does not resolve the
    bump between the two crossings): both crossings are dropped.  Three or more
    crossings in one segment are a geometry error."""
    if cr.line.size == 0:
        return
    key = cr.line * (N + 1) + cr.seg
    _, inv, cnt = np.unique(key, return_inverse=True, return_counts=True)
    c = cnt[inv]
    if np.any(c > 2):
        raise GeometryError("a grid segment holds more than two interface crossings")
    cr.keep = c == 1


@dataclass
class Geometry:
    box: object            # workloads.Box-like (x0, y0, side, N)
    mk: Markers
    hx: Crossings          # horizontal-line crossings (pos = xi)
    vx: Crossings          # vertical-line crossings (pos = eta)
    inside: np.ndarray     # (N+1, N+1) bool, indexed [j, i]; True = Omega+
    arms: dict = field(default_factory=dict)


def build_geometry(X: np.ndarray, box) -> Geometry:
    N, h = box.N, box.side / box.N
    x0, y0 = box.x0, box.y0
    mk = marker_geometry(np.asarray(X, dtype=np.float64))
    margin = 3.0 * h
    if (mk.X[0].min() < x0 + margin or mk.X[0].max() > x0 + box.side - margin or
            mk.X[1].min() < y0 + margin or mk.X[1].max() > y0 + box.side - margin):
        raise GeometryError("interface closer than 3h to the box boundary")
    hx = find_crossings(mk, y0, h, N, axis=1)
    vx = find_crossings(mk, x0, h, N, axis=0)
    if np.any((hx.seg < 0) | (hx.seg >= N)) or np.any((vx.seg < 0) | (vx.seg >= N)):
        raise GeometryError("crossing outside the grid")
    _pair_out(hx, N)
    _pair_out(vx, N)
    xi = grid_coord(x0, h, np.arange(N + 1))
    inside = np.zeros((N + 1, N + 1), dtype=bool)
    for j in range(1, N):
        sel = (hx.line == j) & hx.keep
        xs = np.sort(hx.pos[sel])
        cnt = np.searchsorted(xs, xi, side="left")     # #{xi_c < x_i}
        inside[j] = (cnt % 2) == 1
    g = Geometry(box, mk, hx, vx, inside)
    _check_and_build_arms(g)
    return g


def _snap_vertical(g: Geometry):
    """Assign each column crossing to the column segment whose end labels differ.

    Labels come from row crossings, column crossings from a separate root solve, so when
    the interface passes within rounding of a grid node the two can disagree by one
    segment.  Reading: a column crossing lying within 1e-9 h of a segment end moves to
    the neighbouring segment if only that one changes label; otherwise the geometry is
    rejected."""
    N, h = g.box.N, g.box.side / g.box.N
    y0 = g.box.y0
    lab = g.inside
    tol = 1e-9 * h
    seg = g.vx.seg.copy()
    for c in range(seg.size):
        i, s, eta = int(g.vx.line[c]), int(seg[c]), g.vx.pos[c]

        def flips(t):
            return 0 <= t <= N - 1 and lab[t, i] != lab[t + 1, i]
        if not g.vx.keep[c]:          # one of a pair: the segment must not change label
            if flips(s):
                raise GeometryError("vertical labels and crossings disagree")
            continue
        if flips(s):
            continue
        if eta - (y0 + s * h) <= tol and flips(s - 1):
            seg[c] = s - 1
        elif (y0 + (s + 1) * h) - eta <= tol and flips(s + 1):
            seg[c] = s + 1
        else:
            raise GeometryError("vertical labels and crossings disagree")
    g.vx.seg = seg


def _check_and_build_arms(g: Geometry):
    N = g.box.N
    lab = g.inside
    _snap_vertical(g)
    hk, vk = g.hx.keep, g.vx.keep
    # horizontal segments: (i, j)-(i+1, j); kept crossings keyed by (j, seg)
    hkey = g.hx.line[hk] * (N + 1) + g.hx.seg[hk]
    vkey = g.vx.line[vk] * (N + 1) + g.vx.seg[vk]
    if np.unique(hkey).size != hkey.size or np.unique(vkey).size != vkey.size:
        raise GeometryError("a grid segment holds two interface crossings")
    # label changes along rows <-> horizontal crossings
    dh = lab[:, 1:] != lab[:, :-1]          # [j, i] segment (i, i+1)
    dv = lab[1:, :] != lab[:-1, :]          # [j, i] segment (j, j+1) on column i
    hset = np.zeros_like(dh)
    hset[g.hx.line[hk], g.hx.seg[hk]] = True
    vset = np.zeros_like(dv)
    vset[g.vx.seg[vk], g.vx.line[vk]] = True
    if not np.array_equal(dh, hset):
        raise GeometryError("horizontal labels and crossings disagree")
    if not np.array_equal(dv, vset):
        raise GeometryError("vertical labels and crossings disagree")
    # irregular arms P -> Q, P interior: list of (iP, jP, iQ, jQ, crossing id, horizontal?)
    arms = []
    for c in np.nonzero(hk)[0]:
        j, s = int(g.hx.line[c]), int(g.hx.seg[c])
        for (ip, iq) in ((s, s + 1), (s + 1, s)):
            if 1 <= ip <= N - 1:
                arms.append((ip, j, iq, j, c, 1))
    for c in np.nonzero(vk)[0]:
        i, s = int(g.vx.line[c]), int(g.vx.seg[c])
        for (jp, jq) in ((s, s + 1), (s + 1, s)):
            if 1 <= jp <= N - 1:
                arms.append((i, jp, i, jq, c, 0))
    g.arms = np.array(arms, dtype=np.int64).reshape(-1, 6)


def interpolate_at(values: np.ndarray, k: np.ndarray, t: np.ndarray) -> np.ndarray:
    """6-point Lagrange interpolation of marker values (..., M) at (interval k, t)."""
    M = values.shape[-1]
    idx = stencil_markers(k, M)
    w, _ = lagrange6(t)
    return np.sum(w * values[..., idx], axis=-1)
