"""Modified Stokes interface problem and its double-layer boundary operator (oracle;
test-only).

Sec. 3.3 (eq. ms-bie): the flow part (u2, p2) is the double-layer potential D phi of a
vector density phi on Gamma for the modified Stokes operator (Delta - c^2) u - grad p with
the Green's function that vanishes on the box; on Gamma it satisfies
    -phi/2 + D_u phi = -u1.
As for the scalar layers (Sec. 4.1), D phi is the solution of the equivalent interface
problem of App. A.2,
    (Delta - c^2) u - grad p = f,  div u = 0  off Gamma,
    [u] = Phi,  [T(u, p)] = Psi  on Gamma,  u = u_b on the box,
with T(u, p) = -p n + (grad u + grad u^T) n, n the outward normal, [w] = w(Omega+) -
w(Omega-), Omega+ the inside of Gamma; the double layer has Phi = phi, Psi = 0, f = 0,
u_b = 0, and the left-hand side of eq. ms-bie is its trace from Omega- (the outside),
u- = (u+ + u-)/2 - phi/2.

Sec. 4.2.2 (eqs. mac-fds, crc-mac-fds): MAC grid, u at (x_i, y_j - h/2), i = 0..N,
j = 1..N; v at (x_i - h/2, y_j), i = 1..N, j = 0..N; p at (x_i - h/2, y_j - h/2),
i, j = 1..N; five-point Laplacian, forward-difference pressure gradient at the velocity
points, backward-difference divergence at the cells; on the box u = u_b at the points on
it and the tangential velocity by the symmetric ghost u_{i,0} = 2 u_b - u_{i,1} (and the
same on the other three sides).  The corrected scheme adds C_ij and D_ij built from jump
values.  The system is solved here by a sparse direct solver with the pressure fixed by
a zero mean (the paper uses multigrid; only the solution of the linear system matters).

App. A.2: [u], [v] = Phi; the 5x5 system for [u_x], [u_y], [v_x], [v_y], [p]; the 8x8
system for [u_xx], [u_yy], [u_xy], [v_xx], [v_yy], [v_xy], [p_x], [p_y], solved as
printed (numpy.linalg.solve).

Readings (the paper gives no formulas for C_ij, D_ij or for extracting velocity traces):
* labels and interface crossings of every MAC point and every half-spacing segment come
  from the scalar geometry of geometry.py on the grid of spacing h/2 (the doubled grid,
  on which u, v and p points are the nodes (2i, 2j-1), (2i-1, 2j) and (2i-1, 2j-1));
* correction of a difference equation at P, sum_Q a_Q w_Q = f(P): every stencil point Q
  on the other side of Gamma adds a_Q s_Q [w]_Q to the right-hand side, s_Q = +1 for Q in
  Omega+ and -1 for Q in Omega-; [w]_Q is the jump extended from the crossing point xi
  of the segment P-Q by its Taylor polynomial in d = (coordinate of Q) - (coordinate of
  xi) along the segment: [w] + d [w_s] + d^2/2 [w_ss] for velocity components, [p] + d
  [p_s] for the pressure (App. A.2 gives first derivatives of p only).  This is the
  scalar rule of eq. (modified-fdm) applied to every stencil of eq. (mac-fds);
* a pair of stencil points with the same label is not corrected (an even number of
  crossings between them, the rule for segments cut twice of geometry.py);
* traces at the markers (Sec. 4.3 applied to each velocity component on its own grid):
  closest point floor(t + 1/2) of the component's grid, the six-point stencil and the
  6x6 Taylor system of kfbi.py with the marker jumps; u- = u+ - [u];
* markers at least 3h from the box boundary.

Pinned by: the App. A.2 jumps against exact jumps of piecewise trigonometric flows; the
MAC solve against a smooth no-slip flow (second order); the corrected scheme and the
trace extraction against a piecewise flow with prescribed jumps and box data (second
order at the MAC points and at the markers), with planted mistakes in the corrections
failing that pin (tests/test_oracle_stokes.py).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import geometry as G
from . import spectral
from .geometry import GeometryError, interpolate_at

JUMP_KEYS = ("u", "ux", "uy", "uxx", "uyy", "uxy", "v", "vx", "vy", "vxx", "vyy", "vxy",
             "p", "px", "py")


# ----------------------------------------------------------------------------- jumps
def jumps(xa, ya, xaa, yaa, P1, P1a, P1aa, P2, P2a, P2aa, S1, S1a, S2, S2a, c2,
          f1j=0.0, f2j=0.0):
    """App. A.2: jump values at interface points with tangent (x_a, y_a) and second
    derivatives (x_aa, y_aa), from [u] = (P1, P2), its first two alpha-derivatives, the
    traction jump (S1, S2) and its alpha-derivative, and the jump of the forcing.
    Returns a dict over JUMP_KEYS."""
    xa, ya, xaa, yaa = (np.atleast_1d(np.asarray(a, dtype=np.float64)) for a in
                        (xa, ya, xaa, yaa))
    K = xa.size
    bc = lambda a: np.broadcast_to(np.asarray(a, dtype=np.float64), (K,))
    P1, P1a, P1aa, P2, P2a, P2aa, S1, S1a, S2, S2a, f1j, f2j = map(
        bc, (P1, P1a, P1aa, P2, P2a, P2aa, S1, S1a, S2, S2a, f1j, f2j))
    sa = np.hypot(xa, ya)
    saa = (xa * xaa + ya * yaa) / sa
    # 5x5: unknowns ([u_x], [u_y], [v_x], [v_y], [p])
    A5 = np.zeros((K, 5, 5))
    A5[:, 0, 0], A5[:, 0, 1] = xa, ya
    A5[:, 1, 2], A5[:, 1, 3] = xa, ya
    A5[:, 2, 0], A5[:, 2, 1], A5[:, 2, 2], A5[:, 2, 4] = 2 * ya, -xa, -xa, -ya
    A5[:, 3, 1], A5[:, 3, 2], A5[:, 3, 3], A5[:, 3, 4] = ya, ya, -2 * xa, xa
    A5[:, 4, 0], A5[:, 4, 3] = 1.0, 1.0
    b5 = np.stack([P1a, P2a, sa * S1, sa * S2, np.zeros(K)], axis=-1)
    ux, uy, vx, vy, p = np.linalg.solve(A5, b5[..., None])[..., 0].T
    # 8x8: unknowns ([u_xx], [u_yy], [u_xy], [v_xx], [v_yy], [v_xy], [p_x], [p_y])
    A8 = np.zeros((K, 8, 8))
    A8[:, 0, 0], A8[:, 0, 1], A8[:, 0, 2] = xa * xa, ya * ya, 2 * xa * ya
    A8[:, 1, 3], A8[:, 1, 4], A8[:, 1, 5] = xa * xa, ya * ya, 2 * xa * ya
    A8[:, 2, 0], A8[:, 2, 1], A8[:, 2, 2] = 2 * xa * ya, -xa * ya, 2 * ya * ya - xa * xa
    A8[:, 2, 3], A8[:, 2, 5], A8[:, 2, 6], A8[:, 2, 7] = -xa * xa, -xa * ya, -xa * ya, -ya * ya
    A8[:, 3, 1], A8[:, 3, 2], A8[:, 3, 3], A8[:, 3, 4] = ya * ya, xa * ya, xa * ya, -2 * xa * ya
    A8[:, 3, 5], A8[:, 3, 6], A8[:, 3, 7] = ya * ya - 2 * xa * xa, xa * xa, xa * ya
    A8[:, 4, 0], A8[:, 4, 1], A8[:, 4, 6] = 1.0, 1.0, -1.0
    A8[:, 5, 3], A8[:, 5, 4], A8[:, 5, 7] = 1.0, 1.0, -1.0
    A8[:, 6, 0], A8[:, 6, 5] = 1.0, 1.0
    A8[:, 7, 2], A8[:, 7, 4] = 1.0, 1.0
    r1 = P1aa - xaa * ux - yaa * uy
    r2 = P2aa - xaa * vx - yaa * vy
    r3 = saa * S1 + sa * S1a - 2 * yaa * ux + xaa * uy + xaa * vx + yaa * p
    r4 = saa * S2 + sa * S2a - yaa * uy - yaa * vx + 2 * xaa * vy - xaa * p
    b8 = np.stack([r1, r2, r3, r4, c2 * P1 + f1j, c2 * P2 + f2j, np.zeros(K), np.zeros(K)],
                  axis=-1)
    uxx, uyy, uxy, vxx, vyy, vxy, px, py = np.linalg.solve(A8, b8[..., None])[..., 0].T
    return dict(u=P1.copy(), ux=ux, uy=uy, uxx=uxx, uyy=uyy, uxy=uxy, v=P2.copy(), vx=vx,
                vy=vy, vxx=vxx, vyy=vyy, vxy=vxy, p=p, px=px, py=py)


# -------------------------------------------------------------------------- MAC grid
@dataclass
class MacGeometry:
    box: object
    g2: G.Geometry           # scalar geometry on the doubled grid (spacing h/2)
    hmap: dict               # (row jj, segment ii) -> kept horizontal crossing id
    vmap: dict               # (column ii, segment jj) -> kept vertical crossing id

    @property
    def N(self):
        return self.box.N

    @property
    def h(self):
        return self.box.side / self.box.N

    @property
    def mk(self):
        return self.g2.mk

    def inside(self, ii, jj):
        """Omega+ label of doubled-grid node(s) (ii, jj)."""
        return self.g2.inside[jj, ii]


@dataclass
class _Box:
    x0: float
    y0: float
    side: float
    N: int


def build_geometry(X: np.ndarray, box) -> MacGeometry:
    """Markers, labels and crossings for the MAC grid of `box` (N intervals)."""
    X = np.asarray(X, dtype=np.float64)
    h = box.side / box.N
    m = 3.0 * h
    if (X[0].min() < box.x0 + m or X[0].max() > box.x0 + box.side - m or
            X[1].min() < box.y0 + m or X[1].max() > box.y0 + box.side - m):
        raise GeometryError("interface closer than 3h to the box boundary")
    g2 = G.build_geometry(X, _Box(box.x0, box.y0, box.side, 2 * box.N))
    hmap = {(int(g2.hx.line[c]), int(g2.hx.seg[c])): int(c)
            for c in np.nonzero(g2.hx.keep)[0]}
    vmap = {(int(g2.vx.line[c]), int(g2.vx.seg[c])): int(c)
            for c in np.nonzero(g2.vx.keep)[0]}
    return MacGeometry(box, g2, hmap, vmap)


def _pair_crossing(mg: MacGeometry, A, B):
    """Crossing between doubled-grid nodes A and B (same row or column, 1 or 2 half-steps
    apart) when their labels differ: (horizontal?, crossing id); None otherwise."""
    (ia, ja), (ib, jb) = A, B
    if mg.inside(ia, ja) == mg.inside(ib, jb):
        return None
    if ja == jb:
        ids = [mg.hmap[(ja, s)] for s in range(min(ia, ib), max(ia, ib)) if (ja, s) in mg.hmap]
        horiz = True
    else:
        ids = [mg.vmap[(ia, s)] for s in range(min(ja, jb), max(ja, jb)) if (ia, s) in mg.vmap]
        horiz = False
    if len(ids) != 1:
        raise GeometryError("MAC stencil pair and crossings disagree")
    return horiz, ids[0]


# ------------------------------------------------------------------- interface data
@dataclass
class InterfaceData:
    """Marker values of the jump data and their alpha-derivatives."""
    P1: np.ndarray
    P1a: np.ndarray
    P1aa: np.ndarray
    P2: np.ndarray
    P2a: np.ndarray
    P2aa: np.ndarray
    S1: np.ndarray
    S1a: np.ndarray
    S2: np.ndarray
    S2a: np.ndarray


def interface_data(Phi, Psi) -> InterfaceData:
    """Fourier derivatives of Phi = [u] (2, M) and Psi = [T] (2, M) at the markers."""
    Phi = np.asarray(Phi, dtype=np.float64)
    Psi = np.asarray(Psi, dtype=np.float64)
    d = spectral.diff
    return InterfaceData(Phi[0], d(Phi[0], 1), d(Phi[0], 2), Phi[1], d(Phi[1], 1),
                         d(Phi[1], 2), Psi[0], d(Psi[0], 1), Psi[1], d(Psi[1], 1))


def jumps_at(mg: MacGeometry, q: InterfaceData, c2, k, t, fjump=None):
    """App. A.2 jumps at interface points given by marker interval k and parameter t."""
    mk = mg.mk
    geo = [interpolate_at(v, k, t) for v in (mk.xa, mk.ya, mk.xaa, mk.yaa)]
    dat = [interpolate_at(v, k, t) for v in (q.P1, q.P1a, q.P1aa, q.P2, q.P2a, q.P2aa, q.S1,
                                               q.S1a, q.S2, q.S2a)]
    f1j, f2j = (0.0, 0.0) if fjump is None else fjump
    return jumps(*geo, *dat, c2, f1j, f2j)


# ------------------------------------------------------------------------- unknowns
class MacIndex:
    """Unknown numbering: u (i = 1..N-1, j = 1..N), v (i = 1..N, j = 1..N-1), p (i, j =
    1..N), then one multiplier for the pressure mean."""

    def __init__(self, N):
        self.N = N
        self.nu = (N - 1) * N
        self.nv = N * (N - 1)
        self.np_ = N * N
        self.n = self.nu + self.nv + self.np_ + 1

    def u(self, i, j):
        return (j - 1) * (self.N - 1) + (i - 1)

    def v(self, i, j):
        return self.nu + (j - 1) * self.N + (i - 1)

    def p(self, i, j):
        return self.nu + self.nv + (j - 1) * self.N + (i - 1)

    @property
    def lam(self):
        return self.n - 1


def mac_matrix(N: int, h: float, c2: float):
    """Eq. (mac-fds) with zero box data (box values enter the right-hand side) and the
    bordered mean-zero pressure condition: rows u-momentum, v-momentum, continuity (with
    the multiplier, which absorbs the mean of the continuity right-hand side), mean."""
    ix = MacIndex(N)
    rows, cols, vals = [], [], []

    def add(r, c, a):
        rows.append(r)
        cols.append(c)
        vals.append(a)

    ih2, ih = 1.0 / (h * h), 1.0 / h
    for j in range(1, N + 1):
        for i in range(1, N):
            r = ix.u(i, j)
            diag = -4.0 * ih2 - c2
            for (a, b) in ((i - 1, j), (i + 1, j)):
                if 1 <= a <= N - 1:
                    add(r, ix.u(a, b), ih2)
            for b in (j - 1, j + 1):
                if 1 <= b <= N:
                    add(r, ix.u(i, b), ih2)
                else:
                    diag -= ih2        # ghost u_{i,0} = -u_{i,1} (zero box data)
            add(r, r, diag)
            add(r, ix.p(i + 1, j), -ih)
            add(r, ix.p(i, j), ih)
    for j in range(1, N):
        for i in range(1, N + 1):
            r = ix.v(i, j)
            diag = -4.0 * ih2 - c2
            for b in (j - 1, j + 1):
                if 1 <= b <= N - 1:
                    add(r, ix.v(i, b), ih2)
            for a in (i - 1, i + 1):
                if 1 <= a <= N:
                    add(r, ix.v(a, j), ih2)
                else:
                    diag -= ih2
            add(r, r, diag)
            add(r, ix.p(i, j + 1), -ih)
            add(r, ix.p(i, j), ih)
    for j in range(1, N + 1):
        for i in range(1, N + 1):
            r = ix.p(i, j)
            if i <= N - 1:
                add(r, ix.u(i, j), ih)
            if i - 1 >= 1:
                add(r, ix.u(i - 1, j), -ih)
            if j <= N - 1:
                add(r, ix.v(i, j), ih)
            if j - 1 >= 1:
                add(r, ix.v(i, j - 1), -ih)
            add(r, ix.lam, 1.0)
            add(ix.lam, r, 1.0)
    return sp.csc_matrix((vals, (rows, cols)), shape=(ix.n, ix.n)), ix


def side_sign(q_inside) -> float:
    """s_Q of the correction rule: w(Q) = w_P-side(Q) + s_Q [w](Q)."""
    return 1.0 if q_inside else -1.0


def corrected_rhs(mg: MacGeometry, q: InterfaceData, c2: float, f=None, fjump=None):
    """Right-hand side of eq. (crc-mac-fds): forcing at each point from its own side
    (f = (f1, f2) callables of (x, y, inside) or None for zero) plus the corrections.
    Returns (ru (N, N-1), rv (N-1, N), rp (N, N)) indexed [j-1, i-1]."""
    N, h = mg.N, mg.h
    x0, y0 = mg.box.x0, mg.box.y0
    ru = np.zeros((N, N - 1))
    rv = np.zeros((N - 1, N))
    rp = np.zeros((N, N))
    if f is not None:
        f1, f2 = f
        I, J = np.meshgrid(np.arange(1, N), np.arange(1, N + 1))
        ins = mg.inside(2 * I, 2 * J - 1)
        ru += f1(x0 + I * h, y0 + (J - 0.5) * h, ins)
        I, J = np.meshgrid(np.arange(1, N + 1), np.arange(1, N))
        ins = mg.inside(2 * I - 1, 2 * J)
        rv += f2(x0 + (I - 0.5) * h, y0 + J * h, ins)
    # every stencil pair (P, Q) with different labels: P's row gains a_Q s_Q [w]_Q.
    # Families: (target array, P's doubled-grid node and array index as functions of the
    # point indices, Q's offset in doubled-grid steps, coefficient, jump quantity)
    ih2, ih = 1.0 / (h * h), 1.0 / h
    lab = mg.g2.inside
    fam = []
    Iu, Ju = np.meshgrid(np.arange(1, N), np.arange(1, N + 1))          # u points
    Iv, Jv = np.meshgrid(np.arange(1, N + 1), np.arange(1, N))          # v points
    Ip, Jp = np.meshgrid(np.arange(1, N + 1), np.arange(1, N + 1))      # cells
    uP = (2 * Iu, 2 * Ju - 1, (Ju - 1, Iu - 1))
    vP = (2 * Iv - 1, 2 * Jv, (Jv - 1, Iv - 1))
    pP = (2 * Ip - 1, 2 * Jp - 1, (Jp - 1, Ip - 1))
    for (di, dj) in ((-2, 0), (2, 0), (0, -2), (0, 2)):
        fam.append((ru, uP, (di, dj), ih2, "u", Ju + dj // 2 >= 1, Ju + dj // 2 <= N))
        fam.append((rv, vP, (di, dj), ih2, "v", Iv + di // 2 >= 1, Iv + di // 2 <= N))
    fam.append((ru, uP, (1, 0), -ih, "p", None, None))
    fam.append((ru, uP, (-1, 0), ih, "p", None, None))
    fam.append((rv, vP, (0, 1), -ih, "p", None, None))
    fam.append((rv, vP, (0, -1), ih, "p", None, None))
    fam.append((rp, pP, (1, 0), ih, "u", None, None))
    fam.append((rp, pP, (-1, 0), -ih, "u", None, None))
    fam.append((rp, pP, (0, 1), ih, "v", None, None))
    fam.append((rp, pP, (0, -1), -ih, "v", None, None))
    pairs = []
    for (arr, (Pi, Pj, idx), (di, dj), a, qty, ok1, ok2) in fam:
        Qi, Qj = Pi + di, Pj + dj
        sel = lab[Pj, Pi] != lab[np.clip(Qj, 0, 2 * N), np.clip(Qi, 0, 2 * N)]
        if ok1 is not None:
            sel &= ok1 & ok2
        for r in zip(*np.nonzero(sel)):
            pairs.append((arr, (idx[0][r], idx[1][r]), a, (int(Pi[r]), int(Pj[r])),
                          (int(Qi[r]), int(Qj[r])), qty))
    found = []
    for (arr, idx, a, P, Q, qty) in pairs:
        c = _pair_crossing(mg, P, Q)
        if c is not None:
            found.append((arr, idx, a, P, Q, qty, c[0], c[1]))
    if not found:
        return ru, rv, rp
    hx, vx = mg.g2.hx, mg.g2.vx
    k = np.array([(hx if fd[6] else vx).k[fd[7]] for fd in found])
    t = np.array([(hx if fd[6] else vx).t[fd[7]] for fd in found])
    pos = np.array([(hx if fd[6] else vx).pos[fd[7]] for fd in found])
    fj = None
    if fjump is not None:
        xs = np.array([pos[n] if fd[6] else x0 + fd[4][0] * h / 2 for n, fd in enumerate(found)])
        ys = np.array([y0 + fd[4][1] * h / 2 if fd[6] else pos[n] for n, fd in enumerate(found)])
        fj = fjump(xs, ys)
    J = jumps_at(mg, q, c2, k, t, fj)
    for n, (arr, idx, a, P, Q, qty, horiz, cid) in enumerate(found):
        if horiz:
            d = (x0 + Q[0] * h / 2) - pos[n]
            s1, s2 = "x", "xx"
        else:
            d = (y0 + Q[1] * h / 2) - pos[n]
            s1, s2 = "y", "yy"
        if qty == "p":
            w = J["p"][n] + d * J["p" + s1][n]
        else:
            w = J[qty][n] + d * J[qty + s1][n] + 0.5 * d * d * J[qty + s2][n]
        arr[idx] += a * side_sign(mg.inside(*Q)) * w
    return ru, rv, rp


def solve_mac(N, h, c2, ru, rv, rp, box_u=None, box_v=None, x0=0.0, y0=0.0):
    """Solve eq. (crc-mac-fds) with right-hand sides ru, rv, rp and box velocity data
    (callables or None for zero; enter the right-hand side).  Returns the velocity
    components on their full grids, u (N, N+1) [j-1, i] with i = 0..N, v (N+1, N)
    [j, i-1] with j = 0..N, and the mean-zero pressure p (N, N) [j-1, i-1]."""
    A, ix = mac_matrix(N, h, c2)
    ru, rv, rp = ru.copy(), rv.copy(), rp.copy()
    ub_lr = np.zeros((2, N))       # u on the left/right box sides at y_{j-1/2}
    vb_bt = np.zeros((2, N))       # v on the bottom/top box sides at x_{i-1/2}
    ih2, ih = 1.0 / (h * h), 1.0 / h
    if box_u is not None or box_v is not None:
        bu = box_u or (lambda x, y: np.zeros_like(x))
        bv = box_v or (lambda x, y: np.zeros_like(x))
        yc = y0 + (np.arange(1, N + 1) - 0.5) * h
        xc = x0 + (np.arange(1, N + 1) - 0.5) * h
        xi = x0 + np.arange(1, N) * h
        yj = y0 + np.arange(1, N) * h
        ub_lr[0], ub_lr[1] = bu(np.full(N, x0), yc), bu(np.full(N, x0 + N * h), yc)
        vb_bt[0], vb_bt[1] = bv(xc, np.full(N, y0)), bv(xc, np.full(N, y0 + N * h))
        # u momentum: neighbours on the left/right sides, ghosts 2 u_b - u at bottom/top
        ru[:, 0] -= ih2 * ub_lr[0]
        ru[:, -1] -= ih2 * ub_lr[1]
        ru[0, :] -= ih2 * 2.0 * bu(xi, np.full(N - 1, y0))
        ru[-1, :] -= ih2 * 2.0 * bu(xi, np.full(N - 1, y0 + N * h))
        rv[0, :] -= ih2 * vb_bt[0]
        rv[-1, :] -= ih2 * vb_bt[1]
        rv[:, 0] -= ih2 * 2.0 * bv(np.full(N - 1, x0), yj)
        rv[:, -1] -= ih2 * 2.0 * bv(np.full(N - 1, x0 + N * h), yj)
        # continuity: boundary faces
        rp[:, 0] += ih * ub_lr[0]
        rp[:, -1] -= ih * ub_lr[1]
        rp[0, :] += ih * vb_bt[0]
        rp[-1, :] -= ih * vb_bt[1]
    b = np.concatenate([ru.ravel(), rv.ravel(), rp.ravel(), [0.0]])
    sol = spla.spsolve(A, b)
    u = np.zeros((N, N + 1))
    u[:, 1:N] = sol[:ix.nu].reshape(N, N - 1)
    u[:, 0], u[:, N] = ub_lr[0], ub_lr[1]
    v = np.zeros((N + 1, N))
    v[1:N, :] = sol[ix.nu:ix.nu + ix.nv].reshape(N - 1, N)
    v[0, :], v[N, :] = vb_bt[0], vb_bt[1]
    p = sol[ix.nu + ix.nv:ix.nu + ix.nv + ix.np_].reshape(N, N)
    return u, v, p - p.mean()


# ------------------------------------------------------------------------- traces
def _extract_component(mg: MacGeometry, vals, ox, oy, lab, Jm, comp):
    """Sec. 4.3 on one velocity component: grid points (ox + i h, oy + j h), values
    vals(i, j) and labels lab(i, j) (arrays of indices); Jm the marker jumps."""
    h = mg.h
    px, py = mg.mk.X
    i0 = np.floor((px - ox) / h + 0.5).astype(np.int64)
    j0 = np.floor((py - oy) / h + 0.5).astype(np.int64)
    d1 = np.where(px > ox + i0 * h, 1, -1)
    d2 = np.where(py > oy + j0 * h, 1, -1)
    r = np.array([0, 1, 0, 0, -1])
    s = np.array([0, 0, 1, -1, 0])
    I = np.concatenate([i0[:, None] + r, (i0 + d1)[:, None]], axis=1)
    J = np.concatenate([j0[:, None] + s, (j0 + d2)[:, None]], axis=1)
    dx = (ox + I * h - px[:, None]) / h
    dy = (oy + J * h - py[:, None]) / h
    A = np.stack([np.ones_like(dx), dx, dy, 0.5 * dx * dx, dx * dy, 0.5 * dy * dy], axis=-1)
    jv = Jm[comp][:, None]
    jx, jy = Jm[comp + "x"][:, None], Jm[comp + "y"][:, None]
    jxx, jyy, jxy = Jm[comp + "xx"][:, None], Jm[comp + "yy"][:, None], Jm[comp + "xy"][:, None]
    Dx, Dy = dx * h, dy * h
    C = jv + Dx * jx + Dy * jy + 0.5 * (Dx * Dx * jxx + 2.0 * Dx * Dy * jxy + Dy * Dy * jyy)
    b = vals(I, J) + np.where(lab(I, J), 0.0, C)
    sol = np.linalg.solve(A, b[..., None])[..., 0]
    plus = sol[:, 0]
    return plus, plus - Jm[comp]


@dataclass
class StokesResult:
    u_plus: np.ndarray       # (2, M) velocity traces from inside
    u_minus: np.ndarray      # (2, M) from outside
    u: np.ndarray            # full MAC fields as returned by solve_mac
    v: np.ndarray
    p: np.ndarray


def solve_interface(mg: MacGeometry, Phi, Psi, c2: float, f=None, fjump=None, box_u=None,
                    box_v=None) -> StokesResult:
    """The interface problem of App. A.2 on the MAC grid: corrected scheme, solve, and
    the velocity traces at the markers from both sides."""
    N, h = mg.N, mg.h
    x0, y0 = mg.box.x0, mg.box.y0
    q = interface_data(Phi, Psi)
    ru, rv, rp = corrected_rhs(mg, q, c2, f, fjump)
    u, v, p = solve_mac(N, h, c2, ru, rv, rp, box_u, box_v, x0, y0)
    mk = mg.mk
    fjm = None if fjump is None else fjump(mk.X[0], mk.X[1])
    Jm = jumps(mk.xa, mk.ya, mk.xaa, mk.yaa, q.P1, q.P1a, q.P1aa, q.P2, q.P2a, q.P2aa, q.S1,
               q.S1a, q.S2, q.S2a, c2, *(fjm if fjm is not None else (0.0, 0.0)))
    up, um = _extract_component(mg, lambda I, J: u[J - 1, I], x0, y0 - 0.5 * h,
                                lambda I, J: mg.inside(2 * I, 2 * J - 1), Jm, "u")
    vp, vm = _extract_component(mg, lambda I, J: v[J, I - 1], x0 - 0.5 * h, y0,
                                lambda I, J: mg.inside(2 * I - 1, 2 * J), Jm, "v")
    return StokesResult(np.stack([up, vp]), np.stack([um, vm]), u, v, p)


def apply_double_layer(mg: MacGeometry, phi, c2: float) -> StokesResult:
    """D phi through its interface problem: [u] = phi, [T] = 0, f = 0, zero box data."""
    phi = np.asarray(phi, dtype=np.float64).reshape(2, -1)
    return solve_interface(mg, phi, np.zeros_like(phi), c2)


def operator(mg: MacGeometry, x, c2: float) -> np.ndarray:
    """Left-hand side of eq. (ms-bie), -phi/2 + D_u phi = trace of D phi from outside;
    x and the result are flattened (phi_1 at the M markers, then phi_2)."""
    return apply_double_layer(mg, x, c2).u_minus.ravel()
