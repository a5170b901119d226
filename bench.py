#!/usr/bin/env python3
"""Exchange builds per second of the rPS occ-RI exchange on one MI355X.

One step = one exchange build (K_occ and E_x, Eq. 16 of the paper): U = Phi C,
U_g, the fused V-streaming kernel, the fit-fit kernel on W, the ordered
reductions and the final combine.  The ISDF set-up (points, V, W) runs once
before the timed region and is reported separately.  Inputs (C) are resident
in device memory when the timed region starts.

Default workload: the 8-atom diamond-like cell (L = 6.74 bohr, 48^3 grid,
N = 104, n_occ = 16) with N_aux = 6N = 624, FP64 path.  --c selects another
N_aux/N of the convergence sweep (4, 6, 8, 10).

Prints one JSON line.  The roofline block refers to the fused V-streaming
kernel, timed with HIP events recorded by the library on its own stream; its
algorithmic work per launch is 6 n N_aux N_g flops (P = U_g U^T, M1 = A^T U_g,
M2 = A U, each 2 n N_aux N_g) on 8 N_aux N_g bytes of V.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 (matrix = vector)
PEAK_HBM_GBS = 8000.0


def cpu_baseline(w, nrep: int = 3):
    """The FP64 oracle's rPS build (oracle.rps.build_occ) timed on the host
    cores on arrays of the full workload shape (Phi N_g x N, V N_aux x N_g,
    W N_aux x N_aux, C N x n; seeded uniform values: the cost of the build does
    not depend on the values).  Returns builds/s and the BLAS thread count."""
    import numpy as np
    from oracle import rps as orps
    try:
        from threadpoolctl import threadpool_info
        cores = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [os.cpu_count() or 1])
    except Exception:
        cores = os.cpu_count() or 1
    rng = np.random.default_rng(7)
    Phi = rng.random((w.ngrid, w.nbas))
    V = rng.random((w.naux, w.ngrid))
    W = rng.random((w.naux, w.naux))
    W = 0.5 * (W + W.T)
    C = rng.random((w.nbas, w.nocc))
    pts = np.sort(rng.choice(w.ngrid, w.naux, replace=False))
    dV = w.volume / w.ngrid
    orps.build_occ(Phi, pts, V, W, C, dV)     # warm
    t0 = time.perf_counter()
    for _ in range(nrep):
        orps.build_occ(Phi, pts, V, W, C, dV)
    dt = (time.perf_counter() - t0) / nrep
    return {"value": round(1.0 / dt, 4), "unit": "builds/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{nrep} full FP64 oracle builds (numpy/BLAS) of the same N_g x N, N_aux x N_g shapes "
                      f"on seeded arrays, after one warm-up; {dt:.3f} s per build"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--c", type=float, default=6.0, help="N_aux / N (4, 6, 8 or 10)")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64",
                    help="fp64: FP64 V and products; fp32: V stored FP32, FP32 in-tile products, FP64 across tiles")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the exchange build of one cell "
              f"is not sharded here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2207_04636_amd as P
    import rps_inputs as ri

    w = ri.diamond_cell(args.c)
    t0 = time.perf_counter()
    prec = P.PREC_FP64 if args.precision == "fp64" else P.PREC_FP32
    ctx = P.Context.from_workload(w, seed=w.sketch_seed(), precision=prec)
    setup_s = time.perf_counter() - t0
    info = ctx.info()
    S = ctx.overlap()
    C = ri.lowdin(ri.random_coefficients(w), S)
    dev = torch.device("cuda:0")
    Cd = torch.from_numpy(C).to(dev)
    K = torch.empty((w.nbas, w.nocc), dtype=torch.float64, device=dev)
    ex = torch.zeros(1, dtype=torch.float64, device=dev)

    for _ in range(args.warmup):
        ctx.build(Cd, K, ex)
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.build(Cd, K, ex)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = ctx.profile()
    ctx.set_profiling(False)
    Ex = float(ex.item())

    n, naux, ng, N = w.nocc, w.naux, w.ngrid, w.nbas
    fused_s = prof["fused_ms"] / max(prof["builds"], 1) * 1e-3
    line3_s = prof["line3_ms"] / max(prof["builds"], 1) * 1e-3
    flops = 6.0 * n * naux * ng
    vbytes = 8.0 * naux * ng
    achieved = flops / fused_s / 1e12
    out = {
        "metric": "exchange builds/s (K_occ + E_x)",
        "value": round(args.steps / dt, 2),
        "unit": "builds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded diamond-like cell, random S-orthonormal occupied coefficients)",
        "config": {"workload": f"diamond 1x1x1 L=6.74 bohr, 48^3 grid, N={N}, n_occ={n}, "
                               f"N_aux={naux} (c={args.c:g}), FP64 rPS occ-RI", "global_batch": 1,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": None,
                     "kernel": "fused V-streaming kernel (Eq. 16 lines 1-2)",
                     "kernel_avg_us": round(fused_s * 1e6, 3),
                     "hbm_view_GBs": round(vbytes / fused_s / 1e9, 1),
                     "hbm_view_frac": round(vbytes / fused_s / 1e9 / PEAK_HBM_GBS, 4)},
        "line3_avg_us": round(line3_s * 1e6, 3),
        "build_avg_us_events": round(prof["build_ms"] / max(prof["builds"], 1) * 1e3, 3),
        "setup_s": round(setup_s, 3),
        "setup_s_library": round(float(info["setup_seconds"]), 3),
        "E_x": Ex,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
