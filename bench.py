"""Benchmark: KFBI operator applies per second on one MI355X.

Workload (one "step" = one KFBI apply, the operator evaluation that GMRES repeats):
star interface r(a) = 0.5 (1 + 0.2 cos 5a) with 2048 markers in [-1,1]^2, grid 1024^2,
modified Helmholtz Delta - c^2 with c^2 = 1/dt = 1000, single-layer potential, FP64
grid arithmetic, densities = seeded random Fourier series (modes 1..32, amplitudes
N(0,1)/k^2), eight densities cycled.  Inputs are resident in HBM before timing.

Prints one JSON line with the headline value plus:
  roofline      dominant kernel (k_colsolve) measured with HIP events around each launch
  cpu_baseline  the CPU oracle timed on a bounded sample of the same workload
  extra         2048^2 and FP32 rates, GMRES time to 1e-10 for plain FP64, FP32-inner
                refinement (same true FP64 residual)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--N", type=int, default=1024)
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    return ap.parse_args()


def algorithmic_bytes_colsolve(info, N, wbytes):
    """k_colsolve moves: the band of G it writes (rows row_lo..row_hi, N-1 modes) plus
    one read of the arm list (column index int32 + correction value) and the row
    offsets.  Per launch."""
    n = N - 1
    band = info["row_hi"] - info["row_lo"] + 1
    return band * n * wbytes + info["n_arms"] * (4 + wbytes) + (N + 1) * 4


def time_applies(ctx, kf, dens, outs, steps, warmup, layer, precision):
    import torch
    for i in range(warmup):
        ctx.apply(layer, dens[i % len(dens)], precision, out=outs)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for i in range(steps):
        ctx.apply(layer, dens[i % len(dens)], precision, out=outs)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3, wall


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2309_01068_amd import kfbi as kf
    from paper_2309_01068_amd import workloads as W

    dev = "cuda:0"
    torch.cuda.set_device(0)
    M = 2048
    c2 = 1000.0
    layer = kf.SINGLE
    box = W.box(-1.0, 1.0, a.N)
    X = W.star(M)
    dens_np = [W.fourier_density(M, seed=s) for s in range(8)]
    ctx = kf.Context(box.x0, box.y0, box.side, box.N, c2, kf.BOX_ZERO, M)
    ctx.set_interface(torch.tensor(X, device=dev))
    info = ctx.info()
    dens = [torch.tensor(d, device=dev) for d in dens_np]
    outs = {k: torch.empty(M, dtype=torch.float64, device=dev)
            for k in ("v_plus", "v_minus", "dn_plus", "dn_minus")}
    secs, wall = time_applies(ctx, kf, dens, outs, a.steps, a.warmup, layer, a.precision)
    value = a.steps / secs
    ms_per_step = 1e3 * secs / a.steps

    # dominant kernel: HIP events around each stage of the same applies
    ctx.profile(True)
    for i in range(min(a.steps, 1024)):
        ctx.apply(layer, dens[i % 8], a.precision, out=outs)
    ms, napp = ctx.profile_read()
    ctx.profile(False)
    stage_us = [1e3 * m / max(napp, 1) for m in ms]
    wb = 8 if a.precision == 0 else 4
    bytes_k2 = algorithmic_bytes_colsolve(info, a.N, wb)
    k2_s = stage_us[1] * 1e-6
    achieved = bytes_k2 / k2_s / 1e9
    roof = {"kernel": "k_colsolve", "bound": "hbm", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None, "algorithmic_bytes": bytes_k2, "avg_us": round(stage_us[1], 3),
            "stage_us": {"prep": round(stage_us[0], 3), "colsolve": round(stage_us[1], 3),
                         "nodes": round(stage_us[2], 3), "extract": round(stage_us[3], 3)}}
    result = {
        "metric": "KFBI applies/s at 1024^2 (single layer, modified Helmholtz, star, 2048 markers)"
        if a.N == 1024 else f"KFBI applies/s at {a.N}^2",
        "value": round(value, 1), "unit": "applies/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if a.precision == 0 else "f32",
        "data": "synthetic (seeded Fourier-series densities on an analytic star curve)",
        "config": {"workload": f"kfbi_apply star M={M} grid {a.N}^2 c2={c2} S-layer",
                   "grid": a.N, "markers": M, "c2": c2, "layer": "single",
                   "arms": info["n_arms"], "stencil_nodes": info["n_nodes"],
                   "band_rows": info["row_hi"] - info["row_lo"] + 1},
        "wall_s": round(wall, 4),
        "roofline": roof,
    }

    if not a.no_cpu:
        result["cpu_baseline"] = cpu_baseline(X, box, dens_np, c2, a.cpu_seconds)
        if result["cpu_baseline"]:
            result["cpu_baseline"]["gpu_over_cpu"] = round(value / result["cpu_baseline"]["value"], 1)

    if not a.no_extra:
        result["extra"] = extras(kf, W, torch, np, dev, dens, layer)
    print(json.dumps(result), flush=True)


def cpu_baseline(X, box, dens_np, c2, budget):
    """The FP64 numpy/scipy oracle (as it stands) on the same workload: geometry once,
    then applies until about `budget` seconds have passed."""
    try:
        from oracle import geometry as G
        from oracle import kfbi as K
    except Exception as e:  # pragma: no cover
        return {"error": repr(e)}
    g = G.build_geometry(X, box)
    n = 0
    t0 = time.perf_counter()
    while True:
        K.apply(g, K.SINGLE, dens_np[n % len(dens_np)], c2)
        n += 1
        el = time.perf_counter() - t0
        if el > budget or n >= 2000:
            break
    try:
        import threadpoolctl
        pools = threadpoolctl.threadpool_info()
        cores = max([p.get("num_threads", 1) for p in pools] + [1])
    except Exception:
        cores = 1
    return {"value": round(n / el, 3), "unit": "applies/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} applies of the same {box.N}^2 workload (geometry excluded), {el:.1f} s",
            "nproc": os.cpu_count()}


def extras(kf, W, torch, np, dev, dens, layer):
    out = {}
    M = 2048
    X = W.star(M)
    # 2048^2 and FP32 apply rates
    for N, prec in ((1024, 1), (2048, 0), (2048, 1)):
        box = W.box(-1.0, 1.0, N)
        ctx = kf.Context(box.x0, box.y0, box.side, N, 1000.0, kf.BOX_ZERO, M)
        ctx.set_interface(torch.tensor(X, device=dev))
        outs = {k: torch.empty(M, dtype=torch.float64, device=dev)
                for k in ("v_plus", "v_minus", "dn_plus", "dn_minus")}
        secs, _ = time_applies(ctx, kf, dens, outs, 500, 50, layer, prec)
        out[f"applies_per_s_{N}_{'f64' if prec == 0 else 'f32'}"] = round(500 / secs, 1)
        ctx.close()
    # GMRES: Hele-Shaw boundary integral equation on the initial curve, 1024^2, 1024 markers
    box = W.box(-2.0, 2.0, 1024)
    Xh = W.hs3(1024)
    ctx = kf.Context(box.x0, box.y0, box.side, 1024, 0.0, kf.BOX_FREESPACE, 1024)
    ctx.set_interface(torch.tensor(Xh, device=dev))
    r2 = Xh[0] ** 2 + Xh[1] ** 2
    b = torch.tensor(-1e-3 + 0.5 * np.log(r2), device=dev)
    for prec in (0, 1):
        x = torch.zeros(1024, dtype=torch.float64, device=dev)
        ctx.gmres(b, x, kf.DOUBLE, kf.MINUS, 0.0, 1.0, 1.0, tol=1e-10, precision=prec)
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = ctx.gmres(b, x, kf.DOUBLE, kf.MINUS, 0.0, 1.0, 1.0, tol=1e-10, precision=prec)
        el = time.perf_counter() - t0
        out[f"gmres_hs_{'f64' if prec == 0 else 'f32ir'}"] = {
            "seconds": round(el, 5), "iters": st["iters"], "relres": st["relres"],
            "applies64": st["applies64"], "applies32": st["applies32"]}
    return out


if __name__ == "__main__":
    main()
