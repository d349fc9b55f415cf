"""kfbi_gmres_solve_static (the GMRES solve for callers that cannot allocate) against
kfbi_gmres_solve: the same solutions and statistics on two calls in a row, the second on a
smaller interface, with no change of the device memory the context holds.  Both run the
same kernels in the same order, so the answers agree to the last bit; the bar is the
FP64 solve tolerance of the parity tests (1e-12 relative)."""
import numpy as np
import pytest
import torch

from paper_2309_01068_amd import workloads as W

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("precision", [0, 1])
def test_static_workspace_solve_matches_the_context_workspace_solve(precision):
    from paper_2309_01068_amd import kfbi
    box = W.box(-2, 2, 512)
    ctx = kfbi.Context(box.x0, box.y0, box.side, box.N, 0.0, kfbi.BOX_FREESPACE, 1024)
    for M in (512, 256):   # the second call on a smaller interface
        print(f"[case] static workspace M={M} precision={precision}", flush=True)
        X = W.hs3(M)
        ctx.set_interface(dev(X))
        rhs = dev(0.5 * np.log(X[0] ** 2 + X[1] ** 2) - 1e-3)
        bytes0 = ctx.info()["workspace_bytes"]
        xa = torch.zeros(M, dtype=torch.float64, device="cuda")
        xb = torch.zeros(M, dtype=torch.float64, device="cuda")
        _, sa = ctx.gmres(rhs, xa, kfbi.DOUBLE, kfbi.MINUS, 0.0, 1.0, 1.0, tol=1e-10,
                          precision=precision)
        _, sb = ctx.gmres(rhs, xb, kfbi.DOUBLE, kfbi.MINUS, 0.0, 1.0, 1.0, tol=1e-10,
                          precision=precision, static_workspace=True)
        assert sb["converged"] and sb["relres"] <= 1e-10
        assert (sa["iters"], sa["applies64"], sa["applies32"]) == \
            (sb["iters"], sb["applies64"], sb["applies32"])
        a, b = xa.cpu().numpy(), xb.cpu().numpy()
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a)
        assert ctx.info()["workspace_bytes"] == bytes0


def test_static_workspace_rejects_a_restart_beyond_the_limit():
    from paper_2309_01068_amd import kfbi
    box = W.box(-2, 2, 256)
    ctx = kfbi.Context(box.x0, box.y0, box.side, box.N, 0.0, kfbi.BOX_FREESPACE, 256)
    ctx.set_interface(dev(W.hs3(128)))
    x = torch.zeros(128, dtype=torch.float64, device="cuda")
    with pytest.raises(kfbi.KfbiError) as e:
        ctx.gmres(x, x, kfbi.DOUBLE, kfbi.MINUS, 0.0, 1.0, 1.0, restart=65,
                  static_workspace=True)
    assert e.value.code == kfbi.E_INVALID
