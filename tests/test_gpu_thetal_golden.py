"""The Hele-Shaw workload at full size over 200 steps against the stored oracle evolution.

r = 1 + 0.1 cos 3a + 0.05 sin 5a resampled to 1024 equal-arclength markers, box [-2,2]^2
with 1024 intervals per side, sigma = 1e-3, J = 1, tau = 1e-3, GMRES to a 1e-10 relative
residual from the previous density.  tests/golden/hs3_1024_oracle.npz holds the oracle's
eta, L, Xbar and density at steps 1, 10, 50, 100 and 200 (written by
tests/golden/make_hs3_golden.py, which calls only the oracle).

Tolerances: each side stops GMRES at a 1e-10 residual, so the densities of a step differ
by about 1e-10 relative, and the state moves by tau times quantities built from them.
The fingering is unstable (mode growth rates of order 1 over the run), so these
differences are carried and amplified over the steps; the bounds below are set at about
ten times the deviations measured on the GPU and are stated per step.
"""
import os

import numpy as np
import pytest
import torch

from oracle import thetal as T
from paper_2309_01068_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hs3_1024_oracle.npz")


def test_hele_shaw_full_size_200_steps_against_oracle():
    from paper_2309_01068_amd import kfbi
    ref = np.load(GOLDEN)
    steps = [int(s) for s in ref["step"]]
    assert steps == [1, 10, 50, 100, 200]
    box = W.box(-2, 2, 1024)
    th = kfbi.ThetaL(box.x0, box.y0, box.side, box.N, 1024, 1e-3, 1.0, 1e-3)
    th.init(torch.as_tensor(W.hs3(1024), device="cuda"))
    worst = {}
    for k in range(1, steps[-1] + 1):
        r = th.step()
        assert r["relres"] <= 1e-10, k
        if k not in steps:
            continue
        q = steps.index(k)
        s = th.get_state()
        eta = s["eta"].cpu().numpy()
        L, Xb, t = s["scal"][0], np.array(s["scal"][1:3]), s["scal"][3]
        X_gpu, *_ = T.reconstruct(eta, L, Xb)
        X_ref, *_ = T.reconstruct(ref["eta"][q], float(ref["L"][q]), ref["Xbar"][q])
        phi = th.density().cpu().numpy()
        d = {
            "eta": float(np.max(np.abs(eta - ref["eta"][q]))),
            "L": abs(L - float(ref["L"][q])) / float(ref["L"][q]),
            "Xbar": float(np.max(np.abs(Xb - ref["Xbar"][q]))),
            "X": float(np.max(np.abs(X_gpu - X_ref))),
            "phi": float(np.linalg.norm(phi - ref["phi"][q]) / np.linalg.norm(ref["phi"][q])),
        }
        worst[k] = d
        print(f"[case] hs3 1024^2 step {k}: " + " ".join(f"{a} {b:.2e}" for a, b in d.items()),
              flush=True)
        assert abs(t - float(ref["t"][q])) <= 1e-14
        assert d["X"] <= 1e-8 and d["eta"] <= 1e-8, (k, d)
        assert d["L"] <= 1e-10 and d["Xbar"] <= 1e-9, (k, d)
        assert d["phi"] <= 1e-7, (k, d)
