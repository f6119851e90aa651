#!/usr/bin/env python3
"""Throughput of the matrix-free finite-strain tangent apply on one MI355X.

A step is one application v = K(u) w of the tangent on the 48^3 Q2 box
(2,738,019 DoF), with the linearisation point and the per-point caches set up
before the timed region (they are built once per linearisation point; their
build time is reported separately).  Every strategy is timed; the headline
`value` is the fastest one.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload box48_q2]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tangent apply GDoF/s (FP64 vs mixed) + Newton-CG time-to-1e-8 residual"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
STRATEGIES = ["otf", "otf_geom", "t2", "t4", "otf_ad"]
KERNEL_SOURCES = ["paper_2505_15535_amd/csrc/mfe_kernels.hip", "paper_2505_15535_amd/csrc/mfe_device.hpp"]


# --------------------------------------------------------------------------- work model
def sweep_flops_per_q(n: int) -> float:
    """Forward or backward sum factorization of a 3-vector field per
    quadrature point, even-odd 1D kernels, FMA = 2 flops."""
    c = 2 * (((n + 1) // 2) ** 2 + (n // 2) ** 2) + 4 * (n // 2)
    return 18.0 * c / n


def work_model(strategy: str, degree: int, n_dofs: int, n_q: int, n_vertices: int) -> dict:
    """Algorithmic flops and bytes of one apply (each vector read or written
    once, per-point data streamed once)."""
    sf = sweep_flops_per_q(degree + 1)
    transform, jxw, geom, kin = 54.0, 9.0, 150.0, 50.0
    pointwise = {"otf": 153.0, "otf_ad": 153.0, "otf_geom": 153.0, "t2": 80.0, "t4": 123.0}[strategy]
    if strategy in ("otf", "otf_ad"):
        fq = 3 * sf + 3 * transform + jxw + geom + kin + pointwise
        bq, bvec = 0.0, 3 * 8.0 * n_dofs + 24.0 * n_vertices
    elif strategy == "otf_geom":
        fq = 3 * sf + 3 * transform + jxw + kin + pointwise
        bq, bvec = 80.0, 3 * 8.0 * n_dofs
    elif strategy == "t2":
        fq = 2 * sf + 2 * transform + pointwise
        bq, bvec = 17 * 8.0, 2 * 8.0 * n_dofs
    else:
        fq = 2 * sf + 2 * transform + pointwise
        bq, bvec = 36 * 8.0, 2 * 8.0 * n_dofs
    flops = fq * n_q
    nbytes = bq * n_q + bvec
    ai = flops / nbytes
    bound = "alu" if ai > FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9) else "hbm"
    return {"flops_per_q": fq, "bytes_per_q": bq, "vector_bytes": bvec, "flops": flops, "bytes": nbytes,
            "intensity": ai, "bound": bound}


def roofline(model: dict, kernel_ms: float, traffic) -> dict:
    t = kernel_ms * 1e-3
    if model["bound"] == "alu":
        achieved, peak, unit = model["flops"] / t / 1e12, FP64_PEAK_TFLOPS, "TFLOP/s"
    else:
        achieved, peak, unit = model["bytes"] / t / 1e9, HBM_PEAK_GBS, "GB/s"
    return {"bound": model["bound"], "achieved": round(achieved, 3), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 4), "traffic": traffic}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, strategy: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    rec = data.get(f"{workload}/{strategy}")
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


# --------------------------------------------------------------------------- CPU baseline
def cpu_baseline(cfg, target_s: float = 12.0) -> dict:
    """The FP64 oracle's naive cell loop (as it stands) on a bounded sample of
    the workload's cells, scaled to DoF/s of a whole apply."""
    import numpy as np
    from oracle.fem import Problem
    from oracle.mesh import BoxMesh

    mesh = BoxMesh(cfg.nx, cfg.ny, cfg.nz, cfg.degree, cfg.vertices())
    P = Problem(mesh, cfg.mu, cfg.lam, chunk=512)
    u, w = cfg.displacement(), cfg.test_vector(0)
    n_cells = 512
    t_wall = 0.0
    while True:
        cells = np.arange(min(n_cells, mesh.n_elems))
        c0, t0 = time.process_time(), time.perf_counter()
        P.apply_naive(u, w, elems=cells)
        t_wall, t_cpu = time.perf_counter() - t0, time.process_time() - c0
        if t_wall >= target_s or n_cells >= mesh.n_elems:
            break
        n_cells = min(mesh.n_elems, int(n_cells * max(2.0, min(8.0, 1.2 * target_s / max(t_wall, 1e-3)))))
    frac = len(cells) / mesh.n_elems
    rate = cfg.n_dofs * frac / t_wall / 1e9
    return {"value": rate, "unit": "GDoF/s", "cores": max(1, int(round(t_cpu / t_wall))), "kind": "oracle",
            "sample": f"naive FP64 cell loop (explicit 81-entry tangent, numpy) over {len(cells)} of "
                      f"{mesh.n_elems} cells of {cfg.name} in {t_wall:.1f} s, scaled by the cell fraction",
            "host_threads": os.cpu_count()}


# --------------------------------------------------------------------------- main
def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="box48_q2")
    ap.add_argument("--strategies", default=",".join(STRATEGIES))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--out", default=None, help="also write the JSON line to this file")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run 3 plain device copies of this many MiB (reference for HBM counters)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the multi-GPU path is a design, not a build)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2505_15535_amd as mfe
    import synthetic

    cfg = synthetic.get_config(args.workload)
    strategies = [s for s in args.strategies.split(",") if s]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    verts, u_h, w_h = cfg.vertices(), cfg.displacement(), cfg.test_vector(0)
    op = mfe.Operator(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts, cfg.mu, cfg.lam, device=0)
    u = torch.from_numpy(u_h).to(dev)
    w = torch.from_numpy(w_h).to(dev)
    v = torch.empty_like(w)
    print(f"[bench] {cfg.name}: {op.n_dofs} dofs, {op.n_cells} cells, {op.n_qpoints} points", file=sys.stderr,
          flush=True)

    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copies: 3 x {args.calibrate_copy_mib} MiB", file=sys.stderr, flush=True)
        del src, dst

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op.set_state(u)
    torch.cuda.synchronize()
    state_ms = (time.perf_counter() - t0) * 1e3

    results = {}
    for s in strategies:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op.build_cache(s)
        torch.cuda.synchronize()
        build_ms = (time.perf_counter() - t0) * 1e3
        for _ in range(args.warmup):
            op.apply(w, out=v, strategy=s)
        op.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            op.apply(w, out=v, strategy=s)
        torch.cuda.synchronize()
        step_ms = (time.perf_counter() - t0) * 1e3 / args.steps
        kern_ms, n_ev = op.apply_kernel_ms()
        op.set_timing(False)
        if not np.isfinite(float(v.abs().max())):
            raise RuntimeError(f"non-finite result for strategy {s}")
        model = work_model(s, cfg.degree, op.n_dofs, op.n_qpoints, (cfg.nx + 1) * (cfg.ny + 1) * (cfg.nz + 1))
        results[s] = {
            "ms_per_step": round(step_ms, 5),
            "gdofs": op.n_dofs / (step_ms * 1e-3) / 1e9,
            "kernel_ms": round(kern_ms, 5),
            "kernel_launches_timed": n_ev,
            "cache_build_ms": round(build_ms, 3),
            "cache_mb": round(op.cache_bytes(s) / 1e6, 1),
            "roofline": roofline(model, kern_ms, measured_traffic(cfg.name, s)),
            "work_model": {k: (round(x, 3) if isinstance(x, float) else x) for k, x in model.items()},
        }
        print(f"[bench] {s}: {step_ms * 1e3:.1f} us/step, kernel {kern_ms * 1e3:.1f} us, "
              f"{results[s]['gdofs']:.2f} GDoF/s, {results[s]['roofline']['frac'] * 100:.1f}% of "
              f"{results[s]['roofline']['bound']} roof", file=sys.stderr, flush=True)

    best = max(results, key=lambda k: results[k]["gdofs"])
    r = results[best]
    line = {
        "metric": METRIC,
        "value": round(r["gdofs"], 4),
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg.description, "name": cfg.name, "strategy": best, "n_dofs": op.n_dofs,
                   "degree": cfg.degree, "cells": op.n_cells, "qpoints": op.n_qpoints,
                   "mu": cfg.mu, "lambda": cfg.lam, "u_amplitude": cfg.amplitude},
        "roofline": dict(r["roofline"], kernel=f"cell_kernel apply {best}", kernel_ms=r["kernel_ms"]),
        "set_state_ms": round(state_ms, 3),
        "strategies": results,
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(cfg)
    op.close()
    text = json.dumps(line)
    print(text, flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
