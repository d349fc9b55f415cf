"""GPU apply with the zero-normal-derivative box (KFBI_BOX_NEUMANN, the Stefan problem's
box Green's function) against the CPU oracle, element by element.

Bars as for the Dirichlet box: FP64 relative l2 <= 1e-10 per trace (and on the full
grid), FP32 grid stages <= 5e-5.
"""
import numpy as np
import pytest
import torch

from oracle import geometry as G
from oracle import gmres as OG
from oracle import kfbi as K
from paper_2309_01068_amd import workloads as W

from parity import TOL32, check, rel

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
KEYS = ("v_plus", "v_minus", "dn_plus", "dn_minus")


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def ctx_for(box, c2, M, **kw):
    from paper_2309_01068_amd import kfbi
    return kfbi.Context(box.x0, box.y0, box.side, box.N, c2, kfbi.BOX_NEUMANN,
                        max_markers=max(M, 64), **kw)


CASES = [
    ("star512_256", W.star(512), W.box(-1, 1, 256), 1000.0),
    ("ellipse256_128", W.ellipse(256), W.box(-1, 1, 128), 40.0),
    ("hs3_1024_512", W.hs3(1024), W.box(-2, 2, 512), 2000.0),
    ("circle_64", W.circle(96, 0.45), W.box(-1, 1, 64), 9.0),
    # one-marker chunks on a 512^2 grid: mode-split node sums, band column solve
    ("circle_m128_512", W.circle(128, 0.3), W.box(-1, 1, 512), 500.0),
    # near the top of the box: the band ends a few rows below the mirrored box row
    ("circle_top_512", W.circle(128, 0.05, (0.1, 0.9)), W.box(-1, 1, 512), 500.0),
]


@pytest.mark.parametrize("name,X,box,c2", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("layer", [K.SINGLE, K.DOUBLE])
def test_neumann_apply_parity_fp64(name, X, box, c2, layer):
    print(f"[case] neumann {name} layer={layer}", flush=True)
    M = X.shape[1]
    dens = W.fourier_density(M, seed=4)
    g = G.build_geometry(X, box)
    ref = K.apply(g, layer, dens, c2, K.BOX_NEUMANN)
    ctx = ctx_for(box, c2, M)
    ctx.set_interface(dev(X))
    out = ctx.apply(layer, dev(dens), grid=True)
    torch.cuda.synchronize()
    for k in KEYS:
        check(out[k].cpu().numpy(), getattr(ref, k), TOL64, k)
    check(out["grid"].cpu().numpy(), ref.grid, TOL64, "grid")
    # trace-only apply (band rows) after the full-grid one
    out2 = ctx.apply(layer, dev(dens))
    for k in KEYS:
        check(out2[k].cpu().numpy(), getattr(ref, k), TOL64, k)


@pytest.mark.parametrize("name,X,box,c2", CASES[:2], ids=[c[0] for c in CASES[:2]])
def test_neumann_apply_parity_fp32(name, X, box, c2):
    M = X.shape[1]
    dens = W.fourier_density(M, seed=5)
    g = G.build_geometry(X, box)
    ctx = ctx_for(box, c2, M)
    ctx.set_interface(dev(X))
    for layer in (K.SINGLE, K.DOUBLE):
        ref = K.apply(g, layer, dens, c2, K.BOX_NEUMANN)
        out = ctx.apply(layer, dev(dens), precision=1)
        for k in KEYS:
            check(out[k].cpu().numpy(), getattr(ref, k), TOL32[k], f"fp32 {name} layer={layer} {k}")


def test_neumann_full_size_star():
    """The star workload (2048 markers, 1024^2) with the mirrored-ghost box, c^2 = 2000."""
    box = W.box(-1, 1, 1024)
    X = W.star(2048)
    dens = W.fourier_density(2048, seed=0)
    g = G.build_geometry(X, box)
    ctx = ctx_for(box, 2000.0, 2048)
    ctx.set_interface(dev(X))
    for layer in (K.SINGLE, K.DOUBLE):
        print(f"[case] neumann full size layer={layer}", flush=True)
        ref = K.apply(g, layer, dens, 2000.0, K.BOX_NEUMANN)
        out = ctx.apply(layer, dev(dens))
        for k in KEYS:
            check(out[k].cpu().numpy(), getattr(ref, k), TOL64, k)


def test_gibbs_thomson_gmres_with_per_marker_coefficient():
    """eq. bie-GT: eps_V(x) psi - S psi = g with an anisotropic eps_V per marker."""
    box = W.box(-1, 1, 128)
    X = W.ellipse(128, 0.4, 0.3)
    M = 128
    c2 = 1000.0
    g = G.build_geometry(X, box)
    ang = np.arctan2(X[1], X[0])
    epsV = 2e-3 * (1 + 0.5 * np.cos(4 * ang))
    rhs = 0.5 + 0.1 * np.cos(2 * ang)
    A = lambda x: K.operator(g, x, K.SINGLE, K.AVG, epsV, -1.0, 0.0, c2, K.BOX_NEUMANN)
    ref, st = OG.gmres(A, rhs, np.zeros(M), 1e-12, 50, 500)
    ctx = ctx_for(box, c2, M)
    ctx.set_interface(dev(X))
    a = dev(epsV)
    y = ctx.operator(dev(ref), K.SINGLE, K.AVG, a, -1.0, 0.0)
    assert rel(y.cpu().numpy(), A(ref)) <= TOL64
    x = torch.zeros(M, dtype=torch.float64, device="cuda")
    x, gs = ctx.gmres(dev(rhs), x, K.SINGLE, K.AVG, a, -1.0, 0.0, tol=1e-12)
    assert gs["relres"] <= 1e-12
    assert rel(x.cpu().numpy(), ref) <= 1e-8


def test_neumann_batch_matches_single_applies():
    box = W.box(-1, 1, 128)
    X = W.star(256)
    ctx = ctx_for(box, 500.0, 256, max_batch=4)
    ctx.set_interface(dev(X))
    D = np.stack([W.fourier_density(256, seed=s) for s in range(3)])
    out = ctx.apply_batch(K.DOUBLE, dev(D))
    for b in range(3):
        one = ctx.apply(K.DOUBLE, dev(D[b]))
        for k in KEYS:
            assert torch.equal(out[k][b], one[k]), (b, k)


def test_neumann_needs_positive_c2():
    from paper_2309_01068_amd import kfbi
    with pytest.raises(kfbi.KfbiError) as e:
        kfbi.Context(-1, -1, 2, 128, 0.0, kfbi.BOX_NEUMANN)
    assert e.value.code == kfbi.E_INVALID


@pytest.mark.parametrize("precision", [0, 1])
def test_neumann_batch_fp32_and_fp64_match_single(precision):
    """Batched applies with the cosine basis, both precisions, small grid (E = 2)."""
    box = W.box(-1, 1, 64)
    X = W.circle(96, 0.45)
    ctx = ctx_for(box, 30.0, 96, max_batch=3)
    ctx.set_interface(dev(X))
    D = np.stack([W.fourier_density(96, seed=s) for s in range(3)])
    out = ctx.apply_batch(K.SINGLE, dev(D), precision)
    for b in range(3):
        one = ctx.apply(K.SINGLE, dev(D[b]), precision)
        for k in KEYS:
            assert torch.equal(out[k][b], one[k]), (b, k)


def test_neumann_profile_kernel_replay():
    """Replaying the cosine-basis kernels leaves the next apply's results unchanged."""
    box = W.box(-1, 1, 128)
    X = W.star(256)
    g = G.build_geometry(X, box)
    d = W.fourier_density(256, seed=3)
    ref = K.apply(g, K.DOUBLE, d, 500.0, K.BOX_NEUMANN)
    ctx = ctx_for(box, 500.0, 256)
    ctx.set_interface(dev(X))
    ctx.apply(K.DOUBLE, dev(d))
    for q in range(4):
        assert ctx.profile_kernel(q, reps=5) > 0.0
    out = ctx.apply(K.DOUBLE, dev(d))
    check(out["v_plus"].cpu().numpy(), ref.v_plus, TOL64, "v_plus")
