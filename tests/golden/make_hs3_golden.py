"""Write the oracle's Hele-Shaw evolution at full size to tests/golden/hs3_1024_oracle.npz.

Workload: r = 1 + 0.1 cos 3a + 0.05 sin 5a resampled to 1024 equal-arclength markers, box
[-2,2]^2 with 1024 intervals per side, sigma = 1e-3, J = 1, tau = 1e-3, 200 steps, GMRES
to a 1e-10 relative residual from the previous density (Sec. 3.1, 5; the parameters are
readings stated with the oracle).  Stored at steps 1, 10, 50, 100 and 200: eta, L, Xbar,
t, the density of the step that produced the state, its GMRES iterations and residual.

Only the oracle and the seeded input generator are called.  Run from the repository
root:  python tests/golden/make_hs3_golden.py   (about ten minutes on eight cores).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import thetal as T  # noqa: E402
from paper_2309_01068_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hs3_1024_oracle.npz")
CHECK = (1, 10, 50, 100, 200)


def main() -> None:
    M, N = 1024, 1024
    box = W.box(-2.0, 2.0, N)
    eta, L, Xb = T.equal_arclength_init(W.hs3(M), M)
    prm = T.HSParams(sigma=1e-3, J=1.0, tau=1e-3, box=box)
    st = T.HSState(eta, L, Xb)
    rec = {k: [] for k in ("step", "eta", "L", "Xbar", "t", "phi", "iters", "relres")}
    t0 = time.time()
    for k in range(1, CHECK[-1] + 1):
        st, info = T.hs_step(st, prm)
        if k in CHECK:
            for key, v in (("step", k), ("eta", st.eta), ("L", st.L), ("Xbar", st.Xbar),
                           ("t", st.t), ("phi", info.phi), ("iters", info.iters),
                           ("relres", info.relres)):
                rec[key].append(v)
        print(f"step {k} iters {info.iters} relres {info.relres:.2e} L {st.L:.12f} "
              f"{time.time() - t0:.0f}s", flush=True)
    np.savez(OUT, **{k: np.array(v) for k, v in rec.items()})
    print("wrote", OUT)


if __name__ == "__main__":
    main()
