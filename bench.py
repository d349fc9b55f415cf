"""Benchmark: KFBI operator applies per second on one MI355X.

Workload (one "step" = one KFBI apply, the operator evaluation that GMRES repeats):
star interface r(a) = 0.5 (1 + 0.2 cos 5a) with 2048 markers in [-1,1]^2, grid 1024^2,
modified Helmholtz Delta - c^2 with c^2 = 1/dt = 1000, single-layer potential, FP64
grid arithmetic, densities = seeded random Fourier series (modes 1..32, amplitudes
N(0,1)/k^2), eight densities cycled.  Inputs are resident in HBM before timing.

Prints one JSON line with the headline value plus:
  roofline      the dominant kernel of an apply (the one the committed rocprofv3 summary
                names): algorithmic bytes over its average duration (back-to-back replays
                between two HIP events on the context stream); the whole apply's
                algorithmic bytes over its timed duration; the per-kernel table
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
    ap.add_argument("--reps", type=int, default=400,
                    help="back-to-back replays per kernel for the per-kernel durations")
    ap.add_argument("--hs-steps", type=int, default=200,
                    help="Hele-Shaw steps timed per evolution (the workload runs 200)")
    ap.add_argument("--ws-train-runs", type=int, default=56,
                    help="training evolutions for the learned warm start (seeds 0..)")
    ap.add_argument("--ws-test-runs", type=int, default=8,
                    help="held-out evolutions for the learned warm start (seeds 56..)")
    ap.add_argument("--ws-epochs", type=int, default=30)
    ap.add_argument("--stefan-steps", type=int, default=60,
                    help="Stefan steps timed (the dendrite workload runs 500)")
    ap.add_argument("--st-train-runs", type=int, default=16,
                    help="training evolutions for the Stefan warm start")
    ap.add_argument("--st-test-runs", type=int, default=4,
                    help="held-out evolutions for the Stefan warm start")
    ap.add_argument("--only", default="",
                    help="comma list of extra sections to run (extra, batched, interior_dirichlet, "
                         "hele_shaw, warm_start, stefan, stefan_warm_start, stokes); empty = all")
    ap.add_argument("--stokes-n", default="128,256,512",
                    help="grid sizes of the modified Stokes section")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy 10 times (the reference "
                         "kernel for scaling hardware byte counters) and exit")
    return ap.parse_args()


def algorithmic_bytes(info, N, M, wbytes, batch=1):
    """Bytes each kernel of one apply must move at least (per launch), from its inputs and
    outputs: n = N-1 sine modes, A arms, P row parts, nb = row_hi-row_lo+1 rows of G written
    by the column solve, R = rows holding interpolation nodes, w = 8 (FP64) or 4 (FP32).
      k_prep           density, two differentiation vectors, trapezoid weights (8 B each per
                       marker) in; five marker quantities and the weighted sum out; per arm
                       11 coefficients, its marker and its list entry (8 + 4 + 4 B) in and
                       its correction (8 B) out
      k_rowdst         per arm the correction and its column (8 + 4 B), per part its
                       descriptor (16 B) in; per part one row of n transformed values out
      k_colsolve       the P n w part rows in, the nb n w rows of G out, per-mode constants
                       and the row-to-part offsets; the zero box runs the band solve
                       (k_colsolve_band: 2 + 6 doubles per mode and 2 per lane of its 64)
      k_nodes_extract  each of the R node rows of G once (R n w), per marker the 51
                       extraction values and 5 marker quantities (8 B), 6 stencil slots (4 B),
                       four traces out (8 B each)
    For a batch of B densities the per-density terms count B times and the geometry terms
    (differentiation vectors, weights, arm coefficients and columns, part descriptors,
    per-mode constants, extraction values, stencil slots) once.
    """
    n = N - 1
    P = info["n_parts"]
    nb = info["row_hi"] - info["row_lo"] + 1
    R = info["n_rows"]
    A = info["n_arms"]
    B = batch
    return {
        "k_prep": B * (M * 8 * (1 + 5) + 8 * (M // 8 + 1) + A * 8)
        + M * 8 * (2 + 1) + A * (11 * 8 + 4 + 4),
        "k_rowdst": B * (A * 8 + P * n * wbytes) + A * 4 + P * 16,
        "k_colsolve": B * (P * n * wbytes + nb * n * wbytes) + n * 8 * (2 + 6 + 128) + (N + 2) * 4,
        "k_nodes_extract": B * (R * n * wbytes + M * (5 * 8 + 4 * 8)) + M * (51 * 8 + 6 * 4),
    }


# (stage index of kfbi_profile / kfbi_profile_kernel, kernel) of the launches of an apply
KERNELS = [(0, "k_prep"), (1, "k_rowdst"), (2, "k_colsolve"), (3, "k_nodes_extract")]
STAGES = [k for _, k in KERNELS]
# GMRES precision modes: FP64; FP32 operator inside FP64 iterative refinement; FP64 GMRES
# whose applies are FP32 once the residual estimate is below MIXED_THRESH ||b||
PREC_NAMES = {0: "f64", 1: "f32ir", 2: "mixed"}
MIXED_THRESH = 1e-4


def measured_traffic(kname, N, precision):
    """HBM bytes per launch of `kname` (fetched + written) from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary of this workload, scaled by the copy calibration; None
    when there is no summary for it or the kernel source changed after it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"kfbi_apply_star2048_{N}_{'f64' if precision == 0 else 'f32'}_traffic.json")
    src = os.path.join(ROOT, "paper_2309_01068_amd", "csrc", "apply.hip")
    try:
        rec = json.load(open(path))
        cur = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
        if rec["source_sha256_16"] != cur or kname not in rec["per_launch"]:
            return None
        t = rec["per_launch"][kname]
        return int(t["fetch_bytes"] + t["write_bytes"])
    except (OSError, ValueError, KeyError):
        return None


def profiled_dominant(N, precision):
    """(kernel with the largest in-apply total time, its mean replayed and in-apply
    durations in us) from the committed rocprofv3 kernel-trace summary of this workload,
    or (None, None, None)."""
    path = os.path.join(ROOT, "profiles", f"kfbi_apply_star2048_{N}_{'f64' if precision == 0 else 'f32'}_kernel_stats.json")
    try:
        rec = json.load(open(path))
        k = rec["dominant"]
        return k, rec["replay_avg_us"][k], rec["in_apply_avg_us"][k]
    except (OSError, ValueError, KeyError):
        return None, None, None


def replay_kernels(ctx, reps, rounds=5):
    """Average duration (us) of each kernel of the last apply, replayed back to back (reps
    per kernel in all), the kernels taking turns over `rounds` rounds."""
    per = max(2, reps // rounds)
    tot = {k: 0.0 for k in STAGES}
    for _ in range(rounds):
        for q, k in KERNELS:
            tot[k] += ctx.profile_kernel(q, reps=per)
    return {k: t / rounds for k, t in tot.items()}


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


def time_graph_applies(kf, torch, X, box, c2, dens, layer, precision, steps, per_graph=8):
    """Applies replayed from a HIP graph: per_graph consecutive kfbi_apply calls (the same
    kernels and buffers as eager calls) captured once on a side stream, then replayed
    steps / per_graph times between two events on that stream.  Returns (seconds, steps)."""
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx = kf.Context(box.x0, box.y0, box.side, box.N, c2, kf.BOX_ZERO, X.shape[1], stream=s)
        ctx.set_interface(torch.tensor(X, device="cuda"))
        outs = {k: torch.empty(X.shape[1], dtype=torch.float64, device="cuda")
                for k in ("v_plus", "v_minus", "dn_plus", "dn_minus")}
        for i in range(16):
            ctx.apply(layer, dens[i % len(dens)], precision, out=outs)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for i in range(per_graph):
            ctx.apply(layer, dens[i % len(dens)], precision, out=outs)
    torch.cuda.synchronize()
    reps = max(1, steps // per_graph)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(s):
        for _ in range(4):
            g.replay()
        e0.record(s)
        for _ in range(reps):
            g.replay()
        e1.record(s)
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / 1e3
    ctx.close()
    return secs, reps * per_graph


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if a.copy_calibration:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": src.numel() * 8,
                          "copy_calibration_bytes_written": dst.numel() * 8, "launches": 10}))
        return

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
    gsecs, gsteps = time_graph_applies(kf, torch, X, box, c2, dens, layer, a.precision, a.steps)

    # per-kernel durations inside applies: HIP events on the context stream around every
    # kernel of the same applies (a second timed pass; the events add to each kernel)
    ctx.profile(True)
    for i in range(min(a.steps, 2048)):
        ctx.apply(layer, dens[i % 8], a.precision, out=outs)
    ms, napp = ctx.profile_read()
    ctx.profile(False)
    live_us = {k: 1e3 * ms[q] / max(napp, 1) for q, k in KERNELS}
    # and replayed back to back (no events between the launches): the durations used
    replay_us = replay_kernels(ctx, a.reps)
    # host cost of issuing one apply (Python binding + launches), no synchronisation
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(200):
        ctx.apply(layer, dens[i % 8], a.precision, out=outs)
    issue_us = 1e6 * (time.perf_counter() - t0) / 200
    torch.cuda.synchronize()
    wb = 8 if a.precision == 0 else 4
    byts = algorithmic_bytes(info, a.N, M, wb)
    prof_dom, prof_rep, prof_in = profiled_dominant(a.N, a.precision)
    kname = prof_dom if prof_dom in replay_us else max(replay_us, key=replay_us.get)
    achieved = byts[kname] / (replay_us[kname] * 1e-6) / 1e9
    whole = sum(byts.values())
    whole_ach = whole / (ms_per_step * 1e-3) / 1e9
    roof = {"kernel": kname, "bound": "hbm", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(kname, a.N, a.precision),
            "algorithmic_bytes": byts[kname], "avg_us": round(replay_us[kname], 3),
            "avg_us_from": "the kernel replayed back to back between two HIP events on the "
                           "context stream (kfbi_profile_kernel)",
            "dominant_from": "committed rocprofv3 summary" if prof_dom == kname else "replay timing",
            "profile_replay_avg_us": prof_rep if prof_dom == kname else None,
            "profile_in_apply_avg_us": prof_in if prof_dom == kname else None,
            "whole_apply": {"algorithmic_bytes": whole, "us": round(ms_per_step * 1e3, 3),
                            "achieved": round(whole_ach, 1),
                            "frac": round(whole_ach / HBM_PEAK_GBS, 4)},
            "kernels": {k: {"avg_us": round(replay_us[k], 3),
                            "in_apply_us": round(live_us[k], 3),
                            "bytes": byts[k], "GB_s": round(byts[k] / replay_us[k] / 1e3, 1),
                            "frac": round(byts[k] / replay_us[k] / 1e3 / HBM_PEAK_GBS, 4)}
                        for k in STAGES},
            "host_issue_us_per_apply": round(issue_us, 2)}
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
                   "row_parts": info["n_parts"], "node_rows": info["n_rows"],
                   "band_rows": info["row_hi"] - info["row_lo"] + 1},
        "wall_s": round(wall, 4),
        "graph": {"applies_per_s": round(gsteps / gsecs, 1),
                  "us_per_apply": round(1e6 * gsecs / gsteps, 3), "steps": gsteps,
                  "note": "the same applies replayed from a captured HIP graph (8 per graph)"},
        "roofline": roof,
    }

    if not a.no_cpu:
        result["cpu_baseline"] = cpu_baseline(X, box, dens_np, c2, a.cpu_seconds)
        if result["cpu_baseline"]:
            result["cpu_baseline"]["gpu_over_cpu"] = round(value / result["cpu_baseline"]["value"], 1)

    if not a.no_extra:
        want = set(a.only.split(",")) if a.only else None
        sections = [("extra", lambda: extras(kf, W, torch, np, dev, dens, layer)),
                    ("batched", lambda: batched(kf, W, torch, np, dev, a)),
                    ("interior_dirichlet", lambda: interior_dirichlet(kf, W, torch, np, dev)),
                    ("hele_shaw", lambda: hele_shaw(kf, W, torch, np, dev, a)),
                    ("warm_start", lambda: warm_start(kf, W, torch, np, dev, a)),
                    ("stefan", lambda: stefan(kf, W, torch, np, dev, a)),
                    ("stefan_warm_start", lambda: stefan_warm_start(kf, W, torch, np, dev, a)),
                    ("stokes", lambda: stokes(kf, W, torch, np, dev, a))]
        for name, fn in sections:
            if want is None or name in want:
                result[name] = fn()
    print(json.dumps(result), flush=True)


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(X, box, dens_np, c2, budget):
    """The FP64 numpy/scipy oracle (as it stands) on the same workload: geometry once,
    then applies until about `budget` seconds have passed, first with one thread (BLAS
    pools limited to one thread; scipy.fft at its default of one worker), then with every
    host core given to scipy.fft and BLAS (numpy's elementwise work stays on one thread)."""
    try:
        from oracle import geometry as G
        from oracle import kfbi as K
        import scipy.fft as sfft
        import threadpoolctl
    except Exception as e:  # pragma: no cover
        return {"error": repr(e)}
    g = G.build_geometry(X, box)
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()

    def rate(seconds):
        n = 0
        t0 = time.perf_counter()
        while True:
            K.apply(g, K.SINGLE, dens_np[n % len(dens_np)], c2)
            n += 1
            el = time.perf_counter() - t0
            if el > seconds or n >= 2000:
                return n, el
    with threadpoolctl.threadpool_limits(limits=1), sfft.set_workers(1):
        n1, el1 = rate(0.6 * budget)
    with threadpoolctl.threadpool_limits(limits=ncpu), sfft.set_workers(ncpu):
        nn, eln = rate(0.4 * budget)
    return {"value": round(n1 / el1, 3), "unit": "applies/s", "cores": 1, "kind": "oracle",
            "sample": f"{n1} applies of the same {box.N}^2 workload (geometry excluded), "
                      f"{el1:.1f} s, one thread",
            "all_cores": {"value": round(nn / eln, 3), "threads": ncpu,
                          "sample": f"{nn} applies, {eln:.1f} s, scipy.fft and BLAS on "
                                    f"{ncpu} threads"},
            "cpu_model": cpu_model(), "nproc": ncpu}


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
    # the double layer (two density derivatives per marker instead of one), FP64
    for N in (1024, 2048):
        box = W.box(-1.0, 1.0, N)
        ctx = kf.Context(box.x0, box.y0, box.side, N, 1000.0, kf.BOX_ZERO, M)
        ctx.set_interface(torch.tensor(X, device=dev))
        outs = {k: torch.empty(M, dtype=torch.float64, device=dev)
                for k in ("v_plus", "v_minus", "dn_plus", "dn_minus")}
        secs, _ = time_applies(ctx, kf, dens, outs, 500, 50, kf.DOUBLE, 0)
        out[f"applies_per_s_{N}_f64_double_layer"] = round(500 / secs, 1)
        ctx.close()
    # GMRES: Hele-Shaw boundary integral equation on the initial curve, 1024^2, 1024 markers
    box = W.box(-2.0, 2.0, 1024)
    Xh = W.hs3(1024)
    ctx = kf.Context(box.x0, box.y0, box.side, 1024, 0.0, kf.BOX_FREESPACE, 1024)
    ctx.set_interface(torch.tensor(Xh, device=dev))
    r2 = Xh[0] ** 2 + Xh[1] ** 2
    b = torch.tensor(-1e-3 + 0.5 * np.log(r2), device=dev)
    for prec in (0, 1, 2):
        itol = MIXED_THRESH if prec == 2 else 1e-5
        x = torch.zeros(1024, dtype=torch.float64, device=dev)
        ctx.gmres(b, x, kf.DOUBLE, kf.MINUS, 0.0, 1.0, 1.0, tol=1e-10, precision=prec,
                  inner_tol=itol)
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = ctx.gmres(b, x, kf.DOUBLE, kf.MINUS, 0.0, 1.0, 1.0, tol=1e-10, precision=prec,
                          inner_tol=itol)
        el = time.perf_counter() - t0
        out[f"gmres_hs_{PREC_NAMES[prec]}"] = {
            "seconds": round(el, 5), "iters": st["iters"], "relres": st["relres"],
            "applies64": st["applies64"], "applies32": st["applies32"]}
    return out


def batched(kf, W, torch, np, dev, a):
    """Batched apply on the headline workload: densities/s for several B, and per-kernel
    replay durations of one launch with the algorithmic bytes of its densities (the
    geometry-only terms counted once)."""
    M, N, c2 = 2048, a.N, 1000.0
    box = W.box(-1.0, 1.0, N)
    ctx = kf.Context(box.x0, box.y0, box.side, N, c2, kf.BOX_ZERO, M, max_batch=64)
    ctx.set_interface(torch.tensor(W.star(M), device=dev))
    info = ctx.info()
    D = torch.tensor(np.stack([W.fourier_density(M, seed=s) for s in range(64)]), device=dev)
    out = {}
    for B in (1, 4, 16, 64):
        d = D[:B].contiguous()
        res = ctx.apply_batch(kf.SINGLE, d, a.precision)
        reps = max(20, 2000 // B)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            ctx.apply_batch(kf.SINGLE, d, a.precision, out=res)
        e1.record()
        torch.cuda.synchronize()
        secs = e0.elapsed_time(e1) / 1e3
        # the library runs B as nl launches of nearly equal size (sub_batch at most); the
        # replay repeats the last launch, of B // nl densities
        nl = -(-B // info["sub_batch"])
        lb = B // nl
        kern = replay_kernels(ctx, max(10, a.reps // lb))
        byts = algorithmic_bytes(info, N, M, 8 if a.precision == 0 else 4, batch=lb)
        out[f"B{B}"] = {
            "densities_per_s": round(B * reps / secs, 1), "us_per_batch": round(1e6 * secs / reps, 2),
            "launches": nl, "launch_batch": lb,
            "kernels": {k: {"replay_us": round(kern[k], 3), "bytes": byts[k],
                            "GB_s": round(byts[k] / kern[k] / 1e3, 1)} for k in STAGES}}
    ctx.close()
    return out


def interior_dirichlet(kf, W, torch, np, dev):
    """Ellipse 0.6 x 0.4 (256 markers) in [-1,1]^2, N = 128, Laplace: interior Dirichlet
    BIE v+ = g for u = e^x sin y by FP64 GMRES to 1e-10 from x0 = 0; iterations, solve
    time and the error of the grid solution at the inside nodes."""
    box = W.box(-1.0, 1.0, 128)
    X = W.ellipse(256)
    ctx = kf.Context(box.x0, box.y0, box.side, 128, 0.0, kf.BOX_ZERO, 256)
    ctx.set_interface(torch.tensor(X, device=dev))
    g = torch.tensor(np.exp(X[0]) * np.sin(X[1]), device=dev)
    x = torch.zeros(256, dtype=torch.float64, device=dev)
    ctx.gmres(g, x, kf.DOUBLE, kf.PLUS, 0.0, 1.0, 0.0, tol=1e-10)   # warm-up
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, st = ctx.gmres(g, x, kf.DOUBLE, kf.PLUS, 0.0, 1.0, 0.0, tol=1e-10)
    el = time.perf_counter() - t0
    grid = ctx.apply(kf.DOUBLE, x, grid=True)["grid"].cpu().numpy()
    xs = box.x0 + box.h * np.arange(129)
    XX, YY = np.meshgrid(xs, xs)                     # [j, i]
    inside = (XX / 0.6) ** 2 + (YY / 0.4) ** 2 < 1.0
    err = np.abs(grid - np.exp(XX) * np.sin(YY))[inside]
    ctx.close()
    # grid refinement: N = 64 .. 512 with M = N markers (about 1.6 h apart), tol 1e-12
    refine = {}
    for N in (64, 128, 256, 512):
        bx = W.box(-1.0, 1.0, N)
        Xr = W.ellipse(N)
        c = kf.Context(bx.x0, bx.y0, bx.side, N, 0.0, kf.BOX_ZERO, N)
        c.set_interface(torch.tensor(Xr, device=dev))
        xr = torch.zeros(N, dtype=torch.float64, device=dev)
        xr, sr = c.gmres(torch.tensor(np.exp(Xr[0]) * np.sin(Xr[1]), device=dev), xr, kf.DOUBLE,
                         kf.PLUS, 0.0, 1.0, 0.0, tol=1e-12)
        gr = c.apply(kf.DOUBLE, xr, grid=True)["grid"].cpu().numpy()
        xs = bx.x0 + bx.h * np.arange(N + 1)
        XX, YY = np.meshgrid(xs, xs)
        ins = (XX / 0.6) ** 2 + (YY / 0.4) ** 2 < 1.0
        refine[f"N{N}"] = {"iters": sr["iters"],
                           "max_err_inside": float(np.abs(gr - np.exp(XX) * np.sin(YY))[ins].max())}
        c.close()
    return {"iters": st["iters"], "relres": st["relres"], "solve_ms": round(1e3 * el, 4),
            "max_err_inside": float(err.max()), "l2_err_inside": float(np.sqrt(np.mean(err ** 2))),
            "refinement": refine}


def stokes(kf, W, torch, np, dev, a):
    """Modified Stokes double layer (eq. ms-bie) on the MAC grid: the flower
    r = 0.55 (1 + 0.12 cos 3a + 0.05 sin 5a) in [-1,1]^2, c^2 = 1/tau with tau = 1e-3 (the
    flow step's 3/(2 tau) is of this size), markers about 1.6 h apart; per N the time of one
    apply (fields and traces), its Schur-complement CG iterations, the dense-transform
    product rate, and the GMRES solve of eq. ms-bie to 1e-10 for a smooth seeded
    right-hand side from x0 = 0."""
    out = {}
    c2 = 1000.0
    for N in (int(v) for v in a.stokes_n.split(",") if v):
        box = W.box(-1.0, 1.0, N)
        M = int(round(3.6 / (1.6 * box.h) / 2)) * 2
        X = W.polar_curve(lambda t: 0.55 * (1 + 0.12 * np.cos(3 * t) + 0.05 * np.sin(5 * t)), M)
        st = kf.Stokes(box.x0, box.y0, box.side, N, c2, max_markers=M, tol=1e-13)
        st.set_interface(torch.tensor(X, device=dev))
        phi = torch.tensor(np.stack([W.fourier_density(M, 1, kmax=8),
                                     W.fourier_density(M, 2, kmax=8)]), device=dev)
        st.apply(phi)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            st.apply(phi)
        torch.cuda.synchronize()
        us = 1e6 * (time.perf_counter() - t0) / reps
        info = st.info()
        # dense transform products of one CG iteration: 12 products of about N^3
        # multiply-adds (two velocity solves and the preconditioner, four each)
        flops_it = 12 * 2.0 * N ** 3
        g = np.stack([W.fourier_density(M, 9, kmax=8), W.fourier_density(M, 10, kmax=8)])
        x = torch.zeros(2 * M, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, gst = st.gmres(torch.tensor(g.ravel(), device=dev), x, tol=1e-10)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[f"N{N}"] = {"markers": M, "apply_ms": round(us / 1e3, 3),
                        "cg_iters": info["cg_iters"], "cg_relres": info["cg_relres"],
                        "transform_tflops": round(flops_it * info["cg_iters"] / (us * 1e-6) / 1e12, 3),
                        "gmres_iters": gst["iters"], "gmres_relres": gst["relres"],
                        "gmres_ms": round(1e3 * el, 2)}
        st.close()
    return out


def hele_shaw(kf, W, torch, np, dev, a):
    """Hele-Shaw evolution: r = 1 + 0.1 cos 3a + 0.05 sin 5a resampled to 1024 markers of
    equal arclength, [-2,2]^2 with 1024^2 intervals, sigma = 1e-3, J = 1, tau = 1e-3,
    previous-density initial guess, FP64 GMRES to 1e-10: wall time per step and its
    split, iterations, area and length."""
    box = W.box(-2.0, 2.0, 1024)
    out = {}
    for prec in (0, 1, 2):
        th = kf.ThetaL(box.x0, box.y0, box.side, 1024, 1024, 1e-3, 1.0, 1e-3, precision=prec,
                       inner_tol=MIXED_THRESH if prec == 2 else 1e-5)
        th.init(torch.tensor(W.hs3(1024), device=dev))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        recs = th.run(a.hs_steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        n = len(recs)
        key = PREC_NAMES[prec]
        out[key] = {
            "steps": n, "ms_per_step": round(1e3 * el / n, 4),
            "ms_split": {k: round(sum(r[k] for r in recs) / n, 4)
                         for k in ("ms_geometry", "ms_gmres", "ms_apply", "ms_update")},
            "mean_iters": round(sum(r["iters"] for r in recs) / n, 3),
            "applies64": round(sum(r["applies64"] for r in recs) / n, 3),
            "applies32": round(sum(r["applies32"] for r in recs) / n, 3),
            "max_relres": max(r["relres"] for r in recs),
            "area_first_last": [recs[0]["area"], recs[-1]["area"]],
            "length_first_last": [recs[0]["length"], recs[-1]["length"]],
            "t_end": recs[-1]["t"]}
        th.close()
    return out


def stefan(kf, W, torch, np, dev, a):
    """Stefan dendrite: seed circle of radius 0.1 in [-4,4]^2 with 2048^2 intervals, 128
    markers (spacing 1.3 h), undercooling St = -0.5, backward Euler with tau = 5e-4
    (c^2 = 1/tau), four-fold surface tension eps_C = 2e-3 (1 - 0.75 cos 4 phi) (anisotropy
    strength 0.05 in the stiffness form 1 - 15 eps cos 4 phi), eps_V = 2e-3, third-order SSD;
    GMRES to 1e-10 from the previous density, FP64 and FP32-inner.  Wall time per step and
    its split, iterations, and the energy balance sum(T) h^2 - area over the run."""
    N, M, tau, St = 2048, 128, 5e-4, -0.5
    box = W.box(-4.0, 4.0, N)
    eC = (2e-3, -0.75, 0.0, 4, 0.0)
    eV = (2e-3, 0.0, 0.0, 4, 0.0)
    w = np.ones(N + 1)
    w[0] = w[-1] = 0.5
    out = {"workload": f"stefan seed r=0.1 box [-4,4]^2 grid {N}^2 M={M} tau={tau} St={St} BE"}
    for prec in (0, 1, 2):
        sf = kf.Stefan(box.x0, box.y0, box.side, N, M, tau, eC, eV, bdf2=False, ssd=2,
                       precision=prec, inner_tol=MIXED_THRESH if prec == 2 else 1e-5)
        sf.init(torch.tensor(W.circle(M, 0.1), device=dev), None, St)

        def energy():
            Tg = sf.temperature()
            xy = sf.markers().cpu().numpy()
            e = float((torch.tensor(w[:, None] * w[None, :], device=dev) * Tg).sum()) * box.h ** 2
            ar = 0.5 * float(np.sum(xy[0] * np.roll(xy[1], -1) - np.roll(xy[0], -1) * xy[1]))
            return e - ar, ar
        E0, A0 = energy()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        recs = sf.run(a.stefan_steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        E1, A1 = energy()
        n = len(recs)
        out[PREC_NAMES[prec]] = {
            "steps": n, "ms_per_step": round(1e3 * el / n, 4),
            "ms_split": {k: round(sum(r[k] for r in recs) / n, 4)
                         for k in ("ms_geometry", "ms_temperature", "ms_gmres", "ms_update")},
            "mean_iters": round(sum(r["iters"] for r in recs) / n, 3),
            "applies64": round(sum(r["applies64"] for r in recs) / n, 3),
            "applies32": round(sum(r["applies32"] for r in recs) / n, 3),
            "max_relres": max(r["relres"] for r in recs),
            "area_first_last": [recs[0]["area"], recs[-1]["area"]],
            "energy_drift_over_area_change": round((E1 - E0) / (A1 - A0), 5),
            "t_end": recs[-1]["t"]}
        sf.close()
    return out


def stefan_warm_start(kf, W, torch, np, dev, a):
    """Learned initial guess of psi on the dendrite workload (as `stefan`, seeds scaled to
    radius 0.1 from the perturbed curves r = 1 + sum_{m=2..8} a_m cos(m a + p_m)): data
    from training evolutions, GPU training, then per-step GMRES iterations and wall time on
    held-out evolutions for x0 = 0, the previous density and the learned guess, FP64 and
    FP32-inner, all to the same 1e-10 FP64 residual."""
    N, M, tau, St, nst = 2048, 128, 5e-4, -0.5, a.stefan_steps
    box = W.box(-4.0, 4.0, N)
    eC = (2e-3, -0.75, 0.0, 4, 0.0)
    eV = (2e-3, 0.0, 0.0, 4, 0.0)

    def seedc(sd):
        return torch.tensor(0.1 * W.perturbed(M, sd), device=dev)

    def make(prec=0):
        return kf.Stefan(box.x0, box.y0, box.side, N, M, tau, eC, eV, bdf2=False, ssd=2,
                         precision=prec, inner_tol=MIXED_THRESH if prec == 2 else 1e-5)
    ws = kf.WarmStart(M, max_batch=64, capacity=max(a.st_train_runs * nst, 64), seed=0)
    extrap = kf.WarmStart(M, max_batch=1, capacity=1, seed=0)
    t0 = time.perf_counter()
    used, sd = 0, 0
    while used < a.st_train_runs and sd < 4 * a.st_train_runs:
        sf = make()
        try:  # a seed whose curve the grid stops resolving is replaced by the next one
            sf.init(seedc(sd), None, St)
            th = sf.thetal
            for _ in range(nst):
                ws.predict(th)
                sf.step()
                ws.record(th)
            used += 1
        except kf.KfbiError:
            pass
        sf.close()
        sd += 1
    gen_s = time.perf_counter() - t0
    n = ws.n_samples()
    t0 = time.perf_counter()
    losses = ws.train(n, a.ws_epochs, 64)
    torch.cuda.synchronize()
    res = {"train_runs": used, "seeds_tried": sd, "samples": n, "data_gen_s": round(gen_s, 2),
           "train_s": round(time.perf_counter() - t0, 2), "epochs": a.ws_epochs,
           "loss_first_last": [losses[0], losses[-1]] if losses else None}
    x0 = torch.empty(M, dtype=torch.float64, device=dev)
    for prec in (0, 1, 2):
        for mode in ("zero", "previous", "extrapolation", "learned"):
            its, tsum, nsteps = [], 0.0, 0
            for k in range(a.st_test_runs):
                sf = make(prec)
                try:
                    sf.init(seedc(1000 + k), None, St)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(nst):
                        if mode == "zero":
                            x0.zero_()
                            r = sf.step(x0)
                        elif mode == "previous":
                            r = sf.step()
                        else:
                            (ws if mode == "learned" else extrap).predict(sf.thetal, x0)
                            r = sf.step(x0)
                        its.append(r["iters"])
                    torch.cuda.synchronize()
                    tsum += time.perf_counter() - t0
                    nsteps += nst
                except kf.KfbiError:
                    pass
                sf.close()
            res[f"{PREC_NAMES[prec]}_{mode}"] = {
                "mean_iters": round(float(np.mean(its)), 3) if its else None,
                "ms_per_step": round(1e3 * tsum / max(nsteps, 1), 4), "steps": nsteps}
    return res


def warm_start(kf, W, torch, np, dev, a):
    """Learned initial guess on the Hele-Shaw setup with perturbed curves
    r = 1 + sum_{m=2..8} a_m cos(m a + p_m), a_m ~ U(0, 0.1): data from training
    evolutions (seeds 0..), training on the GPU, then per-step GMRES iterations and wall
    time on held-out evolutions (seeds 56..) for x0 = 0, the previous density, the linear
    extrapolation 2 phi1 - phi2 (the untrained network, whose output layer is zero) and the
    learned guess, for each GMRES precision mode, all to the same 1e-10 FP64 residual."""
    box = W.box(-2.0, 2.0, 1024)
    M, nst = 1024, a.hs_steps
    args = (box.x0, box.y0, box.side, 1024, M, 1e-3, 1.0, 1e-3)
    cap = a.ws_train_runs * nst
    ws = kf.WarmStart(M, max_batch=64, capacity=max(cap, 64), seed=0)
    extrap = kf.WarmStart(M, max_batch=1, capacity=1, seed=0)
    t0 = time.perf_counter()
    used, skipped = [], []
    sd = 0
    while len(used) < a.ws_train_runs:
        th = kf.ThetaL(*args)
        th.init(torch.tensor(W.perturbed(M, sd), device=dev))
        try:
            for _ in range(nst):
                ws.predict(th)
                th.step()
                ws.record(th)
            used.append(sd)
        except kf.KfbiError:  # a curve the grid stops resolving: replaced by the next seed
            skipped.append(sd)
        th.close()
        sd += 1
    gen_s = time.perf_counter() - t0
    n = ws.n_samples()
    t0 = time.perf_counter()
    losses = ws.train(n, a.ws_epochs, 64)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    res = {"train_runs": len(used), "skipped_seeds": skipped, "samples": n,
           "data_gen_s": round(gen_s, 2), "train_s": round(train_s, 2), "epochs": a.ws_epochs,
           "loss_first_last": [losses[0], losses[-1]] if losses else None,
           "target_scale": ws.target_scale()}
    x0 = torch.empty(M, dtype=torch.float64, device=dev)
    for prec in (0, 1, 2):
        for mode in ("zero", "previous", "extrapolation", "learned"):
            its, tsum, nsteps = [], 0.0, 0
            for k in range(a.ws_test_runs):
                th = kf.ThetaL(*args, precision=prec,
                               inner_tol=MIXED_THRESH if prec == 2 else 1e-5)
                th.init(torch.tensor(W.perturbed(M, 56 + k), device=dev))
                try:
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(nst):
                        if mode == "zero":
                            x0.zero_()
                            r = th.step(x0)
                        elif mode == "previous":
                            r = th.step()
                        else:
                            (ws if mode == "learned" else extrap).predict(th, x0)
                            r = th.step(x0)
                        its.append(r["iters"])
                    torch.cuda.synchronize()
                    tsum += time.perf_counter() - t0
                    nsteps += nst
                except kf.KfbiError:
                    pass
                th.close()
            res[f"{PREC_NAMES[prec]}_{mode}"] = {
                "mean_iters": round(float(np.mean(its)), 3) if its else None,
                "ms_per_step": round(1e3 * tsum / max(nsteps, 1), 4), "steps": nsteps}
    return res


if __name__ == "__main__":
    main()
