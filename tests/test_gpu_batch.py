"""GPU batched apply (kfbi_apply_batch): B densities on one installed interface.

Each batched trace must equal, bit for bit, the single apply of the same density (the
batch runs the same kernels on per-density slices of the workspaces), and the first and
last densities are also compared with the CPU oracle at the FP64 bar of the single apply
(relative l2 <= 1e-10).
"""
import numpy as np
import pytest
import torch

from oracle import geometry as G
from oracle import kfbi as K
from paper_2309_01068_amd import workloads as W

from parity import check, rel

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
KEYS = ("v_plus", "v_minus", "dn_plus", "dn_minus")


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def densities(M, B, seed):
    return np.stack([W.fourier_density(M, seed=seed + b) for b in range(B)])


def check_batch(ctx, layer, D, precision, rings=None, oracle=None):
    B = D.shape[0]
    out = ctx.apply_batch(layer, dev(D), precision, None if rings is None else dev(rings))
    torch.cuda.synchronize()
    for b in range(B):
        one = ctx.apply(layer, dev(D[b]), precision, None if rings is None else dev(rings[b]))
        torch.cuda.synchronize()
        for k in KEYS:
            assert torch.equal(out[k][b], one[k]), (b, k)
    if oracle is not None:
        g, c2, bc = oracle
        for b in (0, B - 1):
            ref = K.apply(g, layer, D[b], c2, bc, None if rings is None else rings[b])
            for k in KEYS:
                check(out[k][b].cpu().numpy(), getattr(ref, k), TOL64, f"density {b} {k}")
    return out


CASES = [
    # (name, curve, box, c2, box_bc); 384 markers leave a ragged last marker chunk
    ("star_mh", W.star(384), W.box(-1, 1, 256), 1000.0, K.BOX_ZERO),
    ("circle_user", W.circle(256, 0.6, (0.01, -0.02)), W.box(-1, 1, 128), 25.0, K.BOX_USER),
    ("hs3_free", W.hs3(256), W.box(-2, 2, 256), 0.0, K.BOX_FREESPACE),
]


@pytest.mark.parametrize("name,X,box,c2,bc", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("layer", [K.SINGLE, K.DOUBLE])
@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_single_applies(name, X, box, c2, bc, layer, precision):
    from paper_2309_01068_amd import kfbi
    M, B = X.shape[1], 5
    print(f"[case] batch {name} layer={layer} prec={precision} B={B}", flush=True)
    ctx = kfbi.Context(box.x0, box.y0, box.side, box.N, c2, bc, max_markers=M, max_batch=8)
    ctx.set_interface(dev(X))
    D = densities(M, B, 10)
    rings = (np.stack([W.random_ring(box.N, seed=20 + b) for b in range(B)])
             if bc == K.BOX_USER else None)
    oracle = (G.build_geometry(X, box), c2, bc) if precision == 0 else None
    check_batch(ctx, layer, D, precision, rings, oracle)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_full_size(precision):
    """The star workload at full size (2048 markers, 1024^2, c^2 = 1000) with 16 densities."""
    from paper_2309_01068_amd import kfbi
    box = W.box(-1, 1, 1024)
    X = W.star(2048)
    print(f"[case] batch full size prec={precision} B=16", flush=True)
    ctx = kfbi.Context(box.x0, box.y0, box.side, box.N, 1000.0, K.BOX_ZERO, max_markers=2048,
                       max_batch=16)
    ctx.set_interface(dev(X))
    D = densities(2048, 16, 100)
    oracle = (G.build_geometry(X, box), 1000.0, K.BOX_ZERO) if precision == 0 else None
    check_batch(ctx, K.DOUBLE, D, precision, None, oracle)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_split_into_launches(precision):
    """64 densities of the full-size star: more than one launch holds (kfbi_info.sub_batch),
    so the batch runs as several launches of nearly equal size; every result still equals
    the single apply bit for bit (and the oracle, FP64, for the first and last)."""
    from paper_2309_01068_amd import kfbi
    box = W.box(-1, 1, 1024)
    X = W.star(2048)
    ctx = kfbi.Context(box.x0, box.y0, box.side, box.N, 1000.0, K.BOX_ZERO, max_markers=2048,
                       max_batch=64)
    ctx.set_interface(dev(X))
    sb = ctx.info()["sub_batch"]
    print(f"[case] batch of 64 prec={precision}, sub_batch {sb}", flush=True)
    assert 1 <= sb < 64
    D = densities(2048, 64, 200)
    oracle = (G.build_geometry(X, box), 1000.0, K.BOX_ZERO) if precision == 0 else None
    check_batch(ctx, K.SINGLE, D, precision, None, oracle)


def test_batch_after_reinstalling_a_larger_interface():
    """The per-density workspaces follow the geometry when a new interface needs more."""
    from paper_2309_01068_amd import kfbi
    box = W.box(-1, 1, 256)
    ctx = kfbi.Context(box.x0, box.y0, box.side, box.N, 1000.0, K.BOX_ZERO, max_markers=1024,
                       max_batch=4)
    for M, X in ((128, W.circle(128, 0.3)), (1024, W.star(1024))):
        print(f"[case] batch reinstall M={M}", flush=True)
        ctx.set_interface(dev(X))
        check_batch(ctx, K.SINGLE, densities(M, 4, M), 0, None,
                    (G.build_geometry(X, box), 1000.0, K.BOX_ZERO))


def test_batch_of_one_and_errors():
    from paper_2309_01068_amd import kfbi
    box = W.box(-1, 1, 128)
    X = W.ellipse(256)
    ctx = kfbi.Context(box.x0, box.y0, box.side, box.N, 0.0, K.BOX_ZERO, max_markers=256,
                       max_batch=3)
    ctx.set_interface(dev(X))
    check_batch(ctx, K.DOUBLE, densities(256, 1, 7), 0)
    with pytest.raises(kfbi.KfbiError) as e:
        ctx.apply_batch(K.DOUBLE, dev(densities(256, 4, 0)))        # B > max_batch
    assert e.value.code == kfbi.E_INVALID
    with pytest.raises(kfbi.KfbiError) as e:
        ctx.apply_batch(K.DOUBLE, dev(np.zeros((0, 256))))           # empty batch
    assert e.value.code == kfbi.E_INVALID
    with pytest.raises(kfbi.KfbiError) as e:
        kfbi.Context(-1, -1, 2, 128, max_batch=65)
    assert e.value.code == kfbi.E_INVALID
    # a context created without a batch size holds one density
    one = kfbi.Context(box.x0, box.y0, box.side, box.N, 0.0, K.BOX_ZERO, max_markers=256)
    one.set_interface(dev(X))
    with pytest.raises(kfbi.KfbiError) as e:
        one.apply_batch(K.DOUBLE, dev(densities(256, 2, 0)))
    assert e.value.code == kfbi.E_INVALID
