"""Pins for oracle.gmres and the interior Dirichlet problem of the ellipse workload."""
import numpy as np

from oracle import geometry as G
from oracle import kfbi as K
from oracle.gmres import gmres
from paper_2309_01068_amd import workloads as W


def _dense(A, M):
    cols = []
    for k in range(M):
        e = np.zeros(M)
        e[k] = 1.0
        cols.append(A(e))
    return np.array(cols).T


def test_gmres_matches_dense_solve():
    M, N = 96, 32
    g = G.build_geometry(W.ellipse(M), W.box(-1, 1, N))

    def A(x):
        return K.operator(g, x, K.DOUBLE, K.PLUS, 0.0, 1.0, 0.0, 0.0)
    b = np.exp(g.mk.X[0]) * np.sin(g.mk.X[1])
    x, st = gmres(A, b, tol=1e-13, restart=30)
    Ad = _dense(A, M)
    xd = np.linalg.solve(Ad, b)
    assert st.converged
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    # restarted GMRES with a short restart reaches the same answer
    x2, st2 = gmres(A, b, tol=1e-13, restart=12)
    assert st2.converged and st2.restarts > 1 and np.linalg.norm(x2 - xd) <= 1e-10 * np.linalg.norm(xd)


def test_hele_shaw_operator_is_second_kind_on_constants():
    """-phi/2 + D phi + int phi ds on a circle maps a constant c to 2 pi R c (eq. bie-HS)."""
    R = 0.7
    g = G.build_geometry(W.circle(128, R), W.box(-1.5, 1.5, 96))
    y = K.operator(g, np.ones(128), K.DOUBLE, K.MINUS, 0.0, 1.0, 1.0, 0.0, K.BOX_FREESPACE)
    assert np.max(np.abs(y - 2 * np.pi * R)) < 1e-3


def test_interior_dirichlet_second_order():
    """Interior Dirichlet Laplace problem on the 0.6 x 0.4 ellipse with data exp(x) sin(y):
    u = D phi, (1/2 + D) phi = g; the grid error at inside nodes falls ~4x per refinement.
    Markers are spaced about 1.6h apart, the regime the paper keeps by refinement (Sec. 6.1.4);
    with spacing below h the highest density modes alias on the grid."""
    errs = []
    for N in (32, 64, 128):
        box = W.box(-1, 1, N)
        g = G.build_geometry(W.ellipse(N), box)

        def A(x):
            return K.operator(g, x, K.DOUBLE, K.PLUS, 0.0, 1.0, 0.0, 0.0)
        b = np.exp(g.mk.X[0]) * np.sin(g.mk.X[1])
        phi, st = gmres(A, b, tol=1e-12)
        assert st.converged
        res = K.apply(g, K.DOUBLE, phi, 0.0)
        h = box.side / N
        X, Y = np.meshgrid(box.x0 + np.arange(N + 1) * h, box.y0 + np.arange(N + 1) * h)
        err = np.abs(res.grid - np.exp(X) * np.sin(Y))[g.inside]
        errs.append(err.max())
    errs = np.array(errs)
    orders = np.log2(errs[:-1] / errs[1:])
    assert np.all(orders > 1.6), (errs, orders)
    assert errs[-1] < 1e-4
