"""One KFBI operator apply, written out plainly (oracle; test-only).

Sec. 4.1: a layer potential v = S psi or D phi solves the equivalent interface problem
    (Delta - c^2) v = 0 off Gamma,  [v] = Phi,  [d_n v] = Psi,  v = g on the box,
with (Phi, Psi) = (0, -psi) for S and (phi, 0) for D (Table 2).
Sec. 4.2.1: five-point scheme with the correction C_ij (eq. modified-fdm) at irregular
    nodes; the system matrix is the plain five-point matrix, solved here exactly by
    the 2-D DST-I (the box carries Dirichlet data).
App. A.1: [u], [u_x], [u_y] from the 2x2 system, [u_xx], [u_yy], [u_xy] from the 3x3
    system (solved by Gaussian elimination, numpy.linalg.solve).
Sec. 4.3: one-sided limits v+, grad v+ from the 6x6 corrected Taylor system on the
    stencil {(0,0),(1,0),(0,1),(0,-1),(-1,0),(d1,d2)}; v- = v+ - [v] etc.; boundary
    operator = average of the one-sided limits.
Sec. 4.1 (Hele-Shaw): box data for the free-space problem by the composite trapezoidal
    rule of the layer potential on the box nodes.
Sec. 3.2 (Stefan): the box Green's function with zero normal derivative on the box.
    Reading: the five-point scheme then holds at every node (i, j = 0..N) with the
    ghost values mirrored across the box (v_{-1,j} = v_{1,j}, ...), which the 2-D DCT-I
    diagonalises (eigenvalues as for the DST with p, q = 0..N); the right-hand side off
    the irregular nodes is zero, also on the box.

Readings (see geometry.py for the geometric ones): the correction of eq. (modified-fdm)
is generalised to all four arm directions and both sides: for an arm P -> Q cut at the
crossing point with signed offset d = (coordinate of Q) - (crossing coordinate),
    T = [u] + d [u_s] + d^2/2 [u_ss]   (s = x for row arms, y for column arms),
    RHS_P += -T/h^2 if P in Omega+,  +T/h^2 if P in Omega-,
and the 6x6 system is solved in h-scaled unknowns (v, h v_x, h v_y, h^2 v_xx, ...).

Pinned by: DST solve vs direct sparse solve / brute-force sums, exactness on piecewise
harmonic quadratics, closed-form layer potentials on circles (second-order
convergence), App. A formulas vs exact jumps (tests/test_oracle_kfbi.py); the DCT-I
solve vs a direct sparse solve of the mirrored-ghost system and brute-force sums, and
layer potentials with the zero-normal-derivative box vs the free-space closed forms
when the box is many decay lengths 1/c away (tests/test_oracle_neumann.py).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.fft as sfft

from . import spectral
from .geometry import Geometry, interpolate_at

SINGLE, DOUBLE = 0, 1
PLUS, MINUS, AVG = 0, 1, 2
BOX_ZERO, BOX_USER, BOX_FREESPACE, BOX_NEUMANN = 0, 1, 2, 3


# ----------------------------------------------------------------------------- jumps
def jumps(xa, ya, xaa, yaa, Phi, Phia, Phiaa, Psi, Psia, c2, f_jump=0.0):
    """App. A.1: jump values ([u], [u_x], [u_y], [u_xx], [u_yy], [u_xy]) at interface
    points with tangent (x_a, y_a), second derivatives (x_aa, y_aa).  Solves the 2x2
    and 3x3 linear systems of App. A.1 literally."""
    xa, ya, xaa, yaa = map(np.asarray, (xa, ya, xaa, yaa))
    sa = np.hypot(xa, ya)
    saa = (xa * xaa + ya * yaa) / sa
    K = xa.size
    # 2x2:  x_a [u_x] + y_a [u_y] = Phi_a ;  y_a [u_x] - x_a [u_y] = s_a Psi
    A2 = np.empty((K, 2, 2))
    A2[:, 0, 0], A2[:, 0, 1] = xa, ya
    A2[:, 1, 0], A2[:, 1, 1] = ya, -xa
    b2 = np.stack([Phia, sa * Psi], axis=-1)
    ux, uy = np.linalg.solve(A2, b2[..., None])[..., 0].T
    # 3x3 for ([u_xx], [u_yy], [u_xy])
    A3 = np.zeros((K, 3, 3))
    A3[:, 0, 0], A3[:, 0, 1], A3[:, 0, 2] = xa * xa, ya * ya, 2.0 * xa * ya
    A3[:, 1, 0], A3[:, 1, 1], A3[:, 1, 2] = xa * ya, -xa * ya, ya * ya - xa * xa
    A3[:, 2, 0], A3[:, 2, 1] = 1.0, 1.0
    r1 = Phiaa - xaa * ux - yaa * uy
    r2 = saa * Psi + sa * Psia - yaa * ux + xaa * uy
    r3 = c2 * Phi + f_jump
    b3 = np.stack([r1, r2, r3 * np.ones_like(r1)], axis=-1)
    uxx, uyy, uxy = np.linalg.solve(A3, b3[..., None])[..., 0].T
    return np.asarray(Phi) * np.ones_like(ux), ux, uy, uxx, uyy, uxy


def layer_data(layer: int, density: np.ndarray):
    """Table 2: (Phi, Psi) for v = S psi (0, -psi) or v = D phi (phi, 0)."""
    z = np.zeros_like(density)
    if layer == DOUBLE:
        return density, z
    if layer == SINGLE:
        return z, -density
    raise ValueError("layer must be SINGLE or DOUBLE")


def marker_quantities(Phi, Psi):
    """(Phi, Phi_a, Phi_aa, Psi, Psi_a) at the markers by Fourier differentiation."""
    return (Phi, spectral.diff(Phi, 1), spectral.diff(Phi, 2), Psi, spectral.diff(Psi, 1))


# --------------------------------------------------------------------------- box data
def ring_nodes(box):
    """Box nodes in the ring layout (4, N+1): bottom (j=0), top (j=N), left (i=0),
    right (i=N), each ordered by the running index 0..N.  Returns (zx, zy)."""
    N, h = box.N, box.side / box.N
    r = box.x0 + np.arange(N + 1) * h
    c = box.y0 + np.arange(N + 1) * h
    zx = np.stack([r, r, np.full(N + 1, box.x0), np.full(N + 1, box.x0 + N * h)])
    zy = np.stack([np.full(N + 1, box.y0), np.full(N + 1, box.y0 + N * h), c, c])
    return zx, zy


def freespace_ring(g: Geometry, layer: int, density: np.ndarray) -> np.ndarray:
    """Sec. 4.1: free-space layer potential at the box nodes by the composite
    trapezoidal rule (G0 = ln|x|/2pi, ds = s_a da, da = 2pi/M)."""
    mk = g.mk
    M = mk.M
    zx, zy = ring_nodes(g.box)
    dx = mk.X[0][None, None, :] - zx[..., None]
    dy = mk.X[1][None, None, :] - zy[..., None]
    r2 = dx * dx + dy * dy
    if layer == DOUBLE:
        # dG0(y - z)/dn_y ds_y = (1/2pi) (y - z).n_y / |y - z|^2 s_a da
        ker = (dx * mk.ya + dy * (-mk.xa)) / r2
        return np.sum(ker * density, axis=-1) / M
    ker = 0.5 * np.log(r2) * mk.sa
    return np.sum(ker * density, axis=-1) / M


# -------------------------------------------------------------------------- RHS build
@dataclass
class InterfaceData:
    Phi: np.ndarray
    Phia: np.ndarray
    Phiaa: np.ndarray
    Psi: np.ndarray
    Psia: np.ndarray


def corrected_rhs(g: Geometry, q: InterfaceData, c2: float, ring: np.ndarray | None):
    """Right-hand side of the corrected five-point scheme on the interior nodes,
    array (N-1, N-1) indexed [j-1, i-1] (Sec. 4.2.1, eq. modified-fdm)."""
    N, h = g.box.N, g.box.side / g.box.N
    mk = g.mk
    rhs = np.zeros((N - 1, N - 1))
    if g.arms.size:
        arms = g.arms
        for horizontal, cr in ((1, g.hx), (0, g.vx)):
            sel = arms[:, 5] == horizontal
            if not np.any(sel):
                continue
            a = arms[sel]
            cid = a[:, 4]
            k, t = cr.k[cid], cr.t[cid]
            geo = [interpolate_at(v, k, t) for v in (mk.xa, mk.ya, mk.xaa, mk.yaa)]
            dens = [interpolate_at(v, k, t) for v in (q.Phi, q.Phia, q.Phiaa, q.Psi, q.Psia)]
            J = jumps(*geo, *dens, c2)
            if horizontal:
                d = (g.box.x0 + a[:, 2] * h) - cr.pos[cid]
                T = J[0] + d * J[1] + 0.5 * d * d * J[3]
            else:
                d = (g.box.y0 + a[:, 3] * h) - cr.pos[cid]
                T = J[0] + d * J[2] + 0.5 * d * d * J[4]
            ip, jp = a[:, 0], a[:, 1]
            sgn = np.where(g.inside[jp, ip], -1.0, 1.0)
            np.add.at(rhs, (jp - 1, ip - 1), sgn * T / (h * h))
    if ring is not None:
        bottom, top, left, right = ring
        rhs[0, :] -= bottom[1:N] / (h * h)
        rhs[-1, :] -= top[1:N] / (h * h)
        rhs[:, 0] -= left[1:N] / (h * h)
        rhs[:, -1] -= right[1:N] / (h * h)
    return rhs


# ------------------------------------------------------------------------------ solve
def dst1(a: np.ndarray, axis: int) -> np.ndarray:
    """X_p = sum_{i=1}^{n} a_i sin(pi p i / (n+1)) along `axis` (scipy's DST-I is twice this)."""
    return 0.5 * sfft.dst(a, type=1, axis=axis)


def solve_fivepoint(rhs: np.ndarray, h: float, c2: float) -> np.ndarray:
    """Unique solution of (Delta_h - c^2) v = rhs on the (N-1)^2 interior nodes with
    zero Dirichlet data, by diagonalisation with the 2-D DST-I (eigenvalues
    lambda_pq = -(4/h^2)(sin^2(p pi/2N) + sin^2(q pi/2N)) - c^2)."""
    n = rhs.shape[0]
    N = n + 1
    p = np.arange(1, N)
    s2 = np.sin(0.5 * np.pi * p / N) ** 2
    lam = -(4.0 / (h * h)) * (s2[:, None] + s2[None, :]) - c2
    F = dst1(dst1(rhs, 0), 1)
    V = dst1(dst1(F / lam, 0), 1) * (2.0 / N) ** 2
    return V


def dct1w(a: np.ndarray, axis: int) -> np.ndarray:
    """X_p = sum_{i=0}^{N} w_i a_i cos(pi p i / N), w_0 = w_N = 1/2, else 1 (scipy's DCT-I
    is twice this); applied twice it gives (N/2) a."""
    return 0.5 * sfft.dct(a, type=1, axis=axis)


def solve_neumann(rhs: np.ndarray, h: float, c2: float) -> np.ndarray:
    """Unique solution (c2 > 0) of (Delta_h - c^2) v = rhs on all (N+1)^2 nodes with the
    mirrored ghost values of the zero-normal-derivative box, by the 2-D DCT-I."""
    N = rhs.shape[0] - 1
    p = np.arange(N + 1)
    s2 = np.sin(0.5 * np.pi * p / N) ** 2
    lam = -(4.0 / (h * h)) * (s2[:, None] + s2[None, :]) - c2
    F = dct1w(dct1w(rhs, 0), 1)
    return dct1w(dct1w(F / lam, 0), 1) * (2.0 / N) ** 2


def fivepoint_apply_neumann(v: np.ndarray, h: float, c2: float) -> np.ndarray:
    """(Delta_h - c^2) v on all nodes with mirrored ghost values (for pins)."""
    p = np.pad(v, 1, mode="reflect")
    return ((p[1:-1, 2:] + p[1:-1, :-2] + p[2:, 1:-1] + p[:-2, 1:-1] - 4.0 * v) / (h * h)
            - c2 * v)


def fivepoint_apply(v: np.ndarray, h: float, c2: float) -> np.ndarray:
    """(Delta_h - c^2) v on interior nodes with zero boundary values (for pins)."""
    p = np.pad(v, 1)
    return ((p[1:-1, 2:] + p[1:-1, :-2] + p[2:, 1:-1] + p[:-2, 1:-1] - 4.0 * v) / (h * h)
            - c2 * v)


# ------------------------------------------------------------------------- extraction
def stencil(g: Geometry):
    """Sec. 4.3: closest node (i0, j0) (rounding floor(t + 1/2)), d1, d2 (ties -> -1),
    six points {(0,0),(1,0),(0,1),(0,-1),(-1,0),(d1,d2)}.  Returns (I, J) of shape (M, 6)."""
    box, mk = g.box, g.mk
    h = box.side / box.N
    px, py = mk.X
    i0 = np.floor((px - box.x0) / h + 0.5).astype(np.int64)
    j0 = np.floor((py - box.y0) / h + 0.5).astype(np.int64)
    d1 = np.where(px > box.x0 + i0 * h, 1, -1)
    d2 = np.where(py > box.y0 + j0 * h, 1, -1)
    r = np.array([0, 1, 0, 0, -1])
    s = np.array([0, 0, 1, -1, 0])
    I = np.concatenate([i0[:, None] + r, (i0 + d1)[:, None]], axis=1)
    J = np.concatenate([j0[:, None] + s, (j0 + d2)[:, None]], axis=1)
    return I, J


def extract(g: Geometry, grid: np.ndarray, Jm):
    """One-sided limits at the markers from grid values (N+1, N+1) [j, i] and the
    marker jumps Jm = ([v], [v_x], [v_y], [v_xx], [v_yy], [v_xy]) (Sec. 4.3)."""
    box, mk = g.box, g.mk
    h = box.side / box.N
    I, J = stencil(g)
    dx = (box.x0 + I * h - mk.X[0][:, None]) / h
    dy = (box.y0 + J * h - mk.X[1][:, None]) / h
    A = np.stack([np.ones_like(dx), dx, dy, 0.5 * dx * dx, dx * dy, 0.5 * dy * dy], axis=-1)
    jv, jx, jy, jxx, jyy, jxy = [np.asarray(a)[:, None] for a in Jm]
    Dx, Dy = dx * h, dy * h
    C = jv + Dx * jx + Dy * jy + 0.5 * (Dx * Dx * jxx + 2.0 * Dx * Dy * jxy + Dy * Dy * jyy)
    minus = ~g.inside[J, I]
    b = grid[J, I] + np.where(minus, C, 0.0)
    sol = np.linalg.solve(A, b[..., None])[..., 0]
    vp, vxp, vyp = sol[:, 0], sol[:, 1] / h, sol[:, 2] / h
    vm, vxm, vym = vp - Jm[0], vxp - Jm[1], vyp - Jm[2]
    return vp, vxp, vyp, vm, vxm, vym


# ------------------------------------------------------------------------------ apply
@dataclass
class ApplyResult:
    v_plus: np.ndarray
    v_minus: np.ndarray
    dn_plus: np.ndarray
    dn_minus: np.ndarray
    grid: np.ndarray        # (N+1, N+1) indexed [j, i]
    rhs: np.ndarray


def solve_interface(g: Geometry, Phi, Psi, c2: float, ring: np.ndarray | None,
                    neumann: bool = False) -> ApplyResult:
    """Solve the equivalent interface problem for given jumps (Phi, Psi) and box data
    (Dirichlet values `ring`, or the zero-normal-derivative box when `neumann`)."""
    N, h = g.box.N, g.box.side / g.box.N
    mk = g.mk
    q = InterfaceData(*marker_quantities(np.asarray(Phi, float), np.asarray(Psi, float)))
    rhs = corrected_rhs(g, q, c2, None if neumann else ring)
    if neumann:
        full = np.zeros((N + 1, N + 1))
        full[1:N, 1:N] = rhs
        grid = solve_neumann(full, h, c2)
        rhs = full
    else:
        v = solve_fivepoint(rhs, h, c2)
        grid = np.zeros((N + 1, N + 1))
        grid[1:N, 1:N] = v
    if ring is not None and not neumann:
        bottom, top, left, right = ring
        grid[0, :], grid[N, :] = bottom, top
        grid[:, 0], grid[:, N] = left, right
    Jm = jumps(mk.xa, mk.ya, mk.xaa, mk.yaa, q.Phi, q.Phia, q.Phiaa, q.Psi, q.Psia, c2)
    vp, vxp, vyp, vm, vxm, vym = extract(g, grid, Jm)
    nx, ny = mk.normal
    return ApplyResult(vp, vm, nx * vxp + ny * vyp, nx * vxm + ny * vym, grid, rhs)


def apply(g: Geometry, layer: int, density: np.ndarray, c2: float, box_bc: int = BOX_ZERO,
          ring: np.ndarray | None = None) -> ApplyResult:
    """Layer potential S psi / D phi evaluated through its equivalent interface problem."""
    Phi, Psi = layer_data(layer, np.asarray(density, dtype=np.float64))
    if box_bc == BOX_ZERO:
        ringv = None
    elif box_bc == BOX_USER:
        ringv = np.asarray(ring, dtype=np.float64)
    elif box_bc == BOX_FREESPACE:
        if c2 != 0.0:
            raise ValueError("free-space box data is defined for the Laplacian only")
        ringv = freespace_ring(g, layer, np.asarray(density, dtype=np.float64))
    elif box_bc == BOX_NEUMANN:
        if not c2 > 0.0:
            raise ValueError("the zero-normal-derivative box needs c2 > 0")
        return solve_interface(g, Phi, Psi, c2, None, neumann=True)
    else:
        raise ValueError("unknown box condition")
    return solve_interface(g, Phi, Psi, c2, ringv)


def trace(res: ApplyResult, side: int) -> np.ndarray:
    if side == PLUS:
        return res.v_plus
    if side == MINUS:
        return res.v_minus
    return 0.5 * (res.v_plus + res.v_minus)


def operator(g: Geometry, x: np.ndarray, layer: int, side: int, a, b: float, q: float,
             c2: float, box_bc: int = BOX_ZERO) -> np.ndarray:
    """Discrete boundary operator A x = a x + b trace_side(layer[x]) + q sum_k x_k s_a,k 2pi/M
    (a a scalar or one value per marker).
    Hele-Shaw (Sec. 3.1, eq. bie-HS): layer D, side -, a=0, b=1, q=1 gives
    -phi/2 + D phi + int phi ds.  Interior Dirichlet: D, side +, a=0, b=1, q=0.
    Gibbs-Thomson (Sec. 3.2, eq. bie-GT): layer S, average, a = eps_V, b = -1, q = 0 with
    the zero-normal-derivative box."""
    res = apply(g, layer, x, c2, box_bc)
    out = a * x + b * trace(res, side)
    if q != 0.0:
        M = g.mk.M
        out = out + q * np.sum(x * g.mk.sa) * (2.0 * np.pi / M)
    return out
