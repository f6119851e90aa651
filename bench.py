#!/usr/bin/env python3
"""Throughput of the matrix-free finite-strain tangent apply on one MI355X,
the mixed-precision apply, and Newton-CG time to a 1e-8 residual.

A step is one application v = K(u) w of the tangent on the 48^3 Q2 box
(2,738,019 DoF), with the linearisation point and the per-point caches set up
before the timed region (they are built once per linearisation point; their
build time is reported separately).  Every strategy is timed; the headline
`value` is the fastest one; kernel durations (roofline) come from every
10th launch of the timed steps.  Beside it, under "mixed": FP64 applies and
applies with FP32 vectors and caches whose sweeps run in FP32 on the vector
ALUs (with --mfma also on the matrix cores: bf16x3, bf16), on the Q4 24^3 and Q6 12^3 boxes
(and the headline box), with the error of each against the FP64 result; per
strategy, "cold" times the apply with the caches flushed between applies;
"cpu_csr" is the assembled-matrix product on the host cores; under "hex": the apply on
general hexahedral meshes (the headline box given as one, and an unstructured
mesh of the same size); under "newton": the twisted beam (64x16x16 Q2,
lambda/mu = 100, 90 degrees in 10 load steps) solved to ||R|| <= 1e-8 with
GMG-preconditioned CG, FP64 V-cycle and FP32 V-cycle.
Before every timed region the GPU is kept under untimed load for --settle
seconds (default 0.3), so that the timed steps run at its steady clocks.
Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload box48_q2]
                  [--mixed box24_q4,box12_q6] [--mfma] [--no-newton] [--settle 0.3]
                  [--legs apply,mixed,split,hex,newton,learned] [--out FILE]
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
KERNEL_SOURCES = ["paper_2505_15535_amd/csrc/mfe_kernels.hip", "paper_2505_15535_amd/csrc/mfe_kernels_hex.hip",
                  "paper_2505_15535_amd/csrc/mfe_cell.hpp", "paper_2505_15535_amd/csrc/mfe_device.hpp",
                  "paper_2505_15535_amd/csrc/mfe_kernels_wave.hip", "paper_2505_15535_amd/csrc/mfe_wave.hpp"]


def apply_kernel_name(strategy: str, degree: int, precision: str = "fp64") -> str:
    """The kernel that runs an apply on a structured box (default summation
    order): the wavefront-per-two-cells kernel for the cached strategies at Q2
    and for the geometry-cached one with FP32 vectors, else the brick kernel."""
    wave = degree == 2 and (strategy in ("t2", "t4") or (strategy == "otf_geom" and precision == "fp32"))
    return ("wave_kernel" if wave else "cell_kernel") + f" apply {strategy} {precision}"


# --------------------------------------------------------------------------- work model
def sweep_flops_per_q(n: int) -> float:
    """Forward or backward sum factorization of a 3-vector field per
    quadrature point, even-odd 1D kernels, FMA = 2 flops."""
    c = 2 * (((n + 1) // 2) ** 2 + (n // 2) ** 2) + 4 * (n // 2)
    return 18.0 * c / n


def work_model(strategy: str, degree: int, n_dofs: int, n_q: int, n_vertices: int, elem: int = 8) -> dict:
    """Algorithmic flops and bytes of one apply (each vector read or written
    once, per-point data streamed once); elem = bytes of a vector and cache
    entry (8 for FP64, 4 for the FP32-sweep apply, whose on-the-fly
    strategies still read the FP64 state, vertices and geometry)."""
    sf = sweep_flops_per_q(degree + 1)
    transform, jxw, geom, kin = 54.0, 9.0, 150.0, 50.0
    pointwise = {"otf": 153.0, "otf_ad": 153.0, "otf_geom": 153.0, "t2": 80.0, "t4": 123.0}[strategy]
    if strategy in ("otf", "otf_ad"):
        fq = 3 * sf + 3 * transform + jxw + geom + kin + pointwise
        bq, bvec = 0.0, (8.0 + 2 * elem) * n_dofs + 24.0 * n_vertices
    elif strategy == "otf_geom":
        fq = 3 * sf + 3 * transform + jxw + kin + pointwise
        bq, bvec = 80.0, (8.0 + 2 * elem) * n_dofs
    elif strategy == "t2":
        fq = 2 * sf + 2 * transform + pointwise
        bq, bvec = 17.0 * elem, 2.0 * elem * n_dofs
    else:
        fq = 2 * sf + 2 * transform + pointwise
        bq, bvec = 36.0 * elem, 2.0 * elem * n_dofs
    flops = fq * n_q
    nbytes = bq * n_q + bvec
    ai = flops / nbytes
    bound = "alu" if ai > FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9) else "hbm"
    return {"flops_per_q": fq, "bytes_per_q": bq, "vector_bytes": bvec, "flops": flops, "bytes": nbytes,
            "intensity": ai, "bound": bound}


FP32_PEAK_TFLOPS = 157.3      # vector FP32
# Kernel durations come from every TIMING_EVERY-th launch of the timed steps:
# a timestamped dispatch costs a few microseconds of stream time, which would
# otherwise be added to every step.
TIMING_EVERY = 10
# Untimed settling before each timed region: the GPU raises its clocks only
# after some time under load, and an apply timed right after host-side set-up
# (a new operator, a cache build) runs up to 25% slower than the same apply
# in steady state (T2 on the 48^3 box: 88-111 us against 84-87 us after
# 0.3 s of load).  The timed steps and the warm-up steps are as requested.
SETTLE_S = 0.3


def settle(fn, seconds=None):
    """Call fn (which queues GPU work) until `seconds` of wall time have passed."""
    import torch
    seconds = SETTLE_S if seconds is None else seconds
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(8):
            fn()
        torch.cuda.synchronize()


def roofline(model: dict, kernel_ms: float, traffic, alu_peak: float = FP64_PEAK_TFLOPS) -> dict:
    t = kernel_ms * 1e-3
    if model["bound"] == "alu":
        achieved, peak, unit = model["flops"] / t / 1e12, alu_peak, "TFLOP/s"
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
def cpu_baseline(cfg, target_s: float = 12.0, product=None) -> dict:
    """The FP64 oracle's naive cell loop (as it stands) on a bounded sample of
    the workload's cells, scaled to DoF/s of a whole apply.  When the sample
    is every cell, product["naive_loop"] receives the oracle's v = K(u) w."""
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
        v_or = P.apply_naive(u, w, elems=cells)
        t_wall, t_cpu = time.perf_counter() - t0, time.process_time() - c0
        if t_wall >= target_s or n_cells >= mesh.n_elems:
            break
        n_cells = min(mesh.n_elems, int(n_cells * max(2.0, min(8.0, 1.2 * target_s / max(t_wall, 1e-3)))))
    frac = len(cells) / mesh.n_elems
    rate = cfg.n_dofs * frac / t_wall / 1e9
    if product is not None and len(cells) == mesh.n_elems:
        product["naive_loop"] = v_or
    return {"value": rate, "unit": "GDoF/s", "cores": max(1, int(round(t_cpu / t_wall))), "kind": "oracle",
            "sample": f"naive FP64 cell loop (explicit 81-entry tangent, numpy) over {len(cells)} of "
                      f"{mesh.n_elems} cells of {cfg.name} in {t_wall:.1f} s, scaled by the cell fraction",
            "host_threads": os.cpu_count(), "host": host_cpu()}


def oracle_check(v_gpu: dict, products: dict) -> dict:
    """Relative 2-norm error of every strategy's timed GPU result against the
    oracle's full-size products (the naive cell loop and the assembled CSR
    product, each when it ran over the whole workload), every dof compared."""
    import numpy as np
    out = {}
    for kind, ref in products.items():
        nr = float(np.linalg.norm(ref))
        out[kind] = {s: float(np.linalg.norm(v - ref) / nr) for s, v in v_gpu.items()}
    return out


def host_cpu() -> dict:
    """Model name and logical CPU count of the host (from /proc/cpuinfo)."""
    model, n = "unknown", 0
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name") and model == "unknown":
                    model = line.split(":", 1)[1].strip()
                if line.startswith("processor"):
                    n += 1
    except OSError:
        pass
    return {"model": model, "logical_cpus": n}


def cpu_csr_baseline(cfg, product=None) -> dict:
    """The assembled-matrix alternative the paper compares against (Sec.
    3.2.2) at the headline workload's full size: the oracle's tangent of the
    same box, state and material assembled into CSR by the oracle's C/OpenMP
    assembly (same definition as the numpy assembly, pinned against it entry
    by entry), then y = K w with the oracle's OpenMP CSR kernel on all host
    cores, median of 10 products, reported as DoF/s."""
    import ctypes

    import numpy as np
    from oracle.assemble_c import assemble_tangent_box
    from oracle.mesh import BoxMesh

    mesh = BoxMesh(cfg.nx, cfg.ny, cfg.nz, cfg.degree, cfg.vertices())
    t0 = time.perf_counter()
    indptr, indices, data, asm_threads = assemble_tangent_box(mesh, cfg.mu, cfg.lam, cfg.displacement())
    t_asm = time.perf_counter() - t0
    lib_path = os.path.join(ROOT, "oracle", "libcsr_spmv.so")
    if not os.path.exists(lib_path):
        raise RuntimeError("oracle/libcsr_spmv.so is not built (run the build step)")
    lib = ctypes.CDLL(lib_path)
    lib.csr_spmv.restype = ctypes.c_int
    lib.csr_spmv.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 5
    n = indptr.size - 1
    x = cfg.test_vector(0)
    y = np.empty_like(x)
    times, threads = [], 1
    for _ in range(11):
        t0 = time.perf_counter()
        threads = lib.csr_spmv(n, indptr.ctypes.data, indices.ctypes.data, data.ctypes.data, x.ctypes.data,
                               y.ctypes.data)
        times.append(time.perf_counter() - t0)
    t = float(np.median(times[1:]))
    if product is not None:
        product["assembled_csr"] = y
    nnz = int(indptr[-1])
    mb = (data.nbytes + indices.nbytes + indptr.nbytes) / 1e6
    del indptr, indices, data
    return {"value": n / t / 1e9, "unit": "GDoF/s", "cores": int(threads), "kind": "oracle assembled CSR",
            "sample": f"{cfg.description}: {n} DoF, {nnz} stored entries ({nnz / n:.1f} per row, {mb:.0f} MB CSR); "
                      f"median of 10 OpenMP products",
            "assembly_s": round(t_asm, 2), "assembly_threads": int(asm_threads), "spmv_ms": round(t * 1e3, 3),
            "host": host_cpu()}


# --------------------------------------------------------------------------- mixed precision
def time_applies(op, w, v, strategy, precision, steps, warmup):
    import torch
    settle(lambda: op.apply(w, out=v, strategy=strategy, precision=precision))
    for _ in range(warmup):
        op.apply(w, out=v, strategy=strategy, precision=precision)
    op.set_timing(TIMING_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        op.apply(w, out=v, strategy=strategy, precision=precision)
    torch.cuda.synchronize()
    step_ms = (time.perf_counter() - t0) * 1e3 / steps
    kern_ms, _ = op.apply_kernel_ms()
    op.set_timing(False)
    return step_ms, kern_ms


def mixed_leg(name, steps, warmup, strategies=("otf", "t2", "t4"), precisions=("fp64", "fp32")) -> dict:
    """FP64 applies and applies with FP32 vectors and caches whose sweeps run in
    FP32 on the vector ALUs (and, with --mfma, on the matrix cores as bf16x3,
    the three-piece split that is FP32-accurate, or bf16, one product); error
    of each result against the FP64 one (the FP64 path itself matches the
    oracle to 1e-12)."""
    import numpy as np
    import torch

    import paper_2505_15535_amd as mfe
    import synthetic

    cfg = synthetic.get_config(name)
    dev = torch.device("cuda", 0)
    op = mfe.Operator(cfg.nx, cfg.ny, cfg.nz, cfg.degree, cfg.vertices(), cfg.mu, cfg.lam, device=0)
    op.set_state(torch.from_numpy(cfg.displacement()).to(dev))
    w64 = torch.from_numpy(cfg.test_vector(0).astype(np.float32).astype(np.float64)).to(dev)
    w32 = w64.float()
    v64 = torch.empty_like(w64)
    nv = (cfg.nx + 1) * (cfg.ny + 1) * (cfg.nz + 1)
    out = {"n_dofs": op.n_dofs, "degree": cfg.degree, "description": cfg.description}
    for s in strategies:
        rec = {}
        for prec in precisions:
            w, elem = (w64, 8) if prec == "fp64" else (w32, 4)
            v = v64 if prec == "fp64" else torch.empty_like(w32)
            op.build_cache(s, precision=prec)
            step_ms, kern_ms = time_applies(op, w, v, s, prec, steps, warmup)
            model = work_model(s, cfg.degree, op.n_dofs, op.n_qpoints, nv, elem)
            rl = roofline(model, kern_ms, measured_traffic(name, s if prec == "fp64" else f"{s}/{prec}"),
                          FP64_PEAK_TFLOPS if prec == "fp64" else FP32_PEAK_TFLOPS)
            rec[prec] = {"ms_per_step": round(step_ms, 5), "kernel_ms": round(kern_ms, 5),
                         "gdofs": round(op.n_dofs / (step_ms * 1e-3) / 1e9, 4), "roofline": rl}
            if prec != "fp64":
                err = float(torch.linalg.norm(v.double() - v64) / torch.linalg.norm(v64))
                rec[prec]["rel_err_vs_fp64"] = err
                rec[prec]["speedup_vs_fp64"] = round(rec["fp64"]["ms_per_step"] / step_ms, 3)
        out[s] = rec
        print(f"[bench] mixed {name} {s}: " + ", ".join(
            f"{p} {rec[p]['gdofs']:.2f} GDoF/s" + (f" (err {rec[p]['rel_err_vs_fp64']:.1e})" if p != "fp64" else "")
            for p in precisions), file=sys.stderr, flush=True)
    op.close()
    return out


# --------------------------------------------------------------------------- split law
def split_leg(name, steps, warmup) -> dict:
    """The split neo-Hookean law (mu, kappa = the workload's lambda) through
    the model-independent strategies, FP64: dual-number on-the-fly and the
    fourth-order cache (filled from dual-number derivatives)."""
    import torch

    import paper_2505_15535_amd as mfe
    import synthetic

    cfg = synthetic.get_config(name)
    dev = torch.device("cuda", 0)
    op = mfe.Operator(cfg.nx, cfg.ny, cfg.nz, cfg.degree, cfg.vertices(), cfg.mu, cfg.lam, device=0)
    op.set_model("split")
    op.set_state(torch.from_numpy(cfg.displacement()).to(dev))
    w = torch.from_numpy(cfg.test_vector(0)).to(dev)
    v = torch.empty_like(w)
    out = {"workload": cfg.description, "law": "split neo-Hookean, mu=1, kappa=lambda"}
    for s in ("otf_ad", "t4"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op.build_cache(s)
        torch.cuda.synchronize()
        build_ms = (time.perf_counter() - t0) * 1e3
        step_ms, kern_ms = time_applies(op, w, v, s, "fp64", steps, warmup)
        out[s] = {"ms_per_step": round(step_ms, 5), "kernel_ms": round(kern_ms, 5),
                  "gdofs": round(op.n_dofs / (step_ms * 1e-3) / 1e9, 4), "cache_build_ms": round(build_ms, 3)}
        print(f"[bench] split law {s}: {out[s]['gdofs']:.2f} GDoF/s (build {build_ms:.2f} ms)", file=sys.stderr,
              flush=True)
    op.close()
    return out


# --------------------------------------------------------------------------- general meshes
def hex_model(strategy, degree, n_dofs, n_q, n_vertices, n_cells) -> dict:
    """work_model plus the index tables a general mesh reads: the int32
    cell-node table (every apply) and the cell-vertex table (geometry on the
    fly)."""
    m = work_model(strategy, degree, n_dofs, n_q, n_vertices)
    m["index_bytes"] = 4.0 * n_cells * (degree + 1) ** 3 + (32.0 * n_cells if strategy in ("otf", "otf_ad") else 0.0)
    m["bytes"] += m["index_bytes"]
    m["intensity"] = m["flops"] / m["bytes"]
    m["bound"] = "alu" if m["intensity"] > FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9) else "hbm"
    return m


def hex_leg(name, steps, warmup, strategies=("otf", "t2", "t4")) -> dict:
    """The tangent apply on general hexahedral meshes (cells gathered through
    the cell-node table, every node scattered with atomics): the headline box
    given as a general mesh (same state and input, permuted to the canonical
    numbering) and an unstructured cube-in-cube mesh of about the same size."""
    import numpy as np
    import torch
    from scipy.spatial import cKDTree

    import paper_2505_15535_amd as mfe
    import synthetic

    dev = torch.device("cuda", 0)
    cfg = synthetic.get_config(name)
    verts = cfg.vertices()
    box = mfe.Operator(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts, cfg.mu, cfg.lam, device=0)
    box_xyz = box.node_coordinates()
    box.close()
    meshes = [("box_as_hex", f"{cfg.description}, given as a general mesh (cells in box order)", verts,
               synthetic.box_cells(cfg.nx, cfg.ny, cfg.nz), "box")]
    v2, c2 = synthetic.cube_in_cube(25, jitter=0.1, rng=np.random.default_rng(3))
    meshes.append(("cube_in_cube25_q2", "unit cube as a central cube and six shells, 7 x 25^3 = 109,375 "
                   "jittered Q2 cells, 3^3 Gauss", v2, c2, "sine"))
    out = {}
    for key, desc, vv, cc, state in meshes:
        op = mfe.Operator.from_hex(vv, cc, cfg.degree, cfg.mu, cfg.lam, device=0)
        xyz = op.node_coordinates()
        if state == "box":   # the headline state and input, in the canonical numbering
            d, perm = cKDTree(box_xyz).query(xyz)
            assert d.max() < 1e-12
            dm = (3 * perm[:, None] + np.arange(3)).reshape(-1)
            u_h, w_h = cfg.displacement()[dm], cfg.test_vector(0)[dm]
        else:
            u_h = synthetic.sine_field(xyz, 0.03, np.random.default_rng(5))
            w_h = np.random.default_rng(6).standard_normal(op.n_dofs)
        op.set_state(torch.from_numpy(np.ascontiguousarray(u_h)).to(dev))
        w = torch.from_numpy(np.ascontiguousarray(w_h)).to(dev)
        v = torch.empty_like(w)
        rec = {"workload": desc, "n_dofs": op.n_dofs, "cells": op.n_cells}
        for s in strategies:
            op.build_cache(s)
            step_ms, kern_ms = time_applies(op, w, v, s, "fp64", steps, warmup)
            model = hex_model(s, cfg.degree, op.n_dofs, op.n_qpoints, len(vv), op.n_cells)
            rec[s] = {"ms_per_step": round(step_ms, 5), "kernel_ms": round(kern_ms, 5),
                      "gdofs": round(op.n_dofs / (step_ms * 1e-3) / 1e9, 4),
                      "roofline": roofline(model, kern_ms, measured_traffic(key, s))}
            print(f"[bench] general mesh {key} {s}: {rec[s]['gdofs']:.2f} GDoF/s, kernel {kern_ms * 1e3:.1f} us, "
                  f"{rec[s]['roofline']['frac'] * 100:.1f}% of {model['bound']} roof", file=sys.stderr, flush=True)
        out[key] = rec
        op.close()
    return out


# --------------------------------------------------------------------------- Newton-CG
# V-cycle kernels launched one by one (mg_graph=0): replaying them from a HIP
# graph is no faster at the beam's sizes (0.56 ms per cycle either way), and
# re-capturing the graph after every Newton step's set-up costs ~0.4 ms.
# Lagged set-up (mg_lag=4): after a full set-up, up to four CG solves of the
# same Newton solve keep its spectrum estimates and coarse inverse (the level
# operators are always current): 7-9% less time, the same iteration counts
NEWTON_OPTS = dict(strategy="t2", preconditioner="gmg", max_newton=30, max_cg=2000, newton_atol=1e-8,
                   cg_rtol=1e-3, cheb_degree=4, cheb_range=15.0, coarse_degree=15, coarse_range=200.0,
                   coarse_direct=1, forcing=0.5, mg_graph=0, mg_lag=4)


def settle_beam(op, u):
    """The untimed settling before a solve: T2 applies at the starting state u."""
    import torch
    op.set_state(u)
    op.build_cache("t2")
    w = torch.ones_like(u)
    v = torch.empty_like(u)
    settle(lambda: op.apply(w, out=v, strategy="t2"))


def newton_leg(nx=64, ny=16, nz=16, lam=100.0, degrees=90.0, steps=10) -> dict:
    """Twisted beam: left face clamped, right face rotated by `degrees` about
    the beam axis in `steps` equal load steps, each started from the last
    converged state; inexact Newton (Eisenstat-Walker forcing, at most 0.5)
    with GMG-preconditioned CG; time to ||R|| <= 1e-8 at the end of the path
    with the FP64 V-cycle and with the FP32 V-cycle."""
    import numpy as np
    import torch

    import paper_2505_15535_amd as mfe
    import synthetic

    L = (nx / ny, 1.0, 1.0)
    dev = torch.device("cuda", 0)
    verts = synthetic.box_vertices(nx, ny, nz, L)
    cdofs, _ = synthetic.clamp_and_twist(nx, ny, nz, 2, L, 0.0)
    out = {"workload": f"beam {nx}x{ny}x{nz} Q2, mu=1, lambda={lam}, {degrees:g} deg twist in {steps} load steps",
           "tolerance": 1e-8, "opts": dict(NEWTON_OPTS)}
    for prec in ("fp64", "fp32"):
        op = mfe.Operator(nx, ny, nz, 2, verts, 1.0, lam, device=0)
        op.set_constraints(cdofs)
        u = torch.zeros(op.n_dofs, dtype=torch.float64, device=dev)
        settle_beam(op, u)
        t0 = time.perf_counter()
        reps = op.solve_load_path(u, lambda t: synthetic.clamp_and_twist(nx, ny, nz, 2, L, np.deg2rad(degrees) * t),
                                  steps, mg_precision=prec, extrapolate=False, **NEWTON_OPTS)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        res = float(np.linalg.norm(op.residual(u).cpu().numpy()))
        out[prec] = {"seconds": round(secs, 3), "final_residual": res,
                     "load_steps_accepted": sum(1 for r in reps if not r.get("failed")),
                     "load_steps_rejected": sum(1 for r in reps if r.get("failed")),
                     "newton_iterations": sum(r["newton_iterations"] for r in reps),
                     "cg_iterations": sum(r["cg_iterations"] for r in reps),
                     "pc_fallbacks": sum(r.get("pc_fallbacks", 0) for r in reps),
                     "per_step": [{"t": round(r["t"], 4), "newton": r["newton_iterations"], "cg": r["cg_iterations"],
                                   "backtracks": r.get("backtracks", 0), "failed": bool(r.get("failed"))}
                                  for r in reps]}
        out["n_dofs"] = op.n_dofs
        print(f"[bench] newton {prec} V-cycle: {secs:.2f} s, ||R|| {res:.2e}, {out[prec]['newton_iterations']} "
              f"Newton / {out[prec]['cg_iterations']} CG iterations", file=sys.stderr, flush=True)
        op.close()
    out["speedup_fp32"] = round(out["fp64"]["seconds"] / out["fp32"]["seconds"], 3)
    return out


# --------------------------------------------------------------------------- learned correction
def learned_leg(nx=64, ny=16, nz=16, epochs=20, variant="relu", n_paths=8, seed=1) -> dict:
    """Train the learned smoother step on residuals from load paths with
    seeded random twist angles (uniform in 30-120 deg) and lambda/mu
    (log-uniform in 10-1000), two states per path, one random load, CG
    residuals after 0-8 iterations (about 2e4 patch pairs), then solve the
    held-out twisted beam (90 deg, lambda = 100, 10 steps) with GMG and with
    the learned step in the finest post-smoother; CG iterations and time."""
    import numpy as np
    import torch

    from paper_2505_15535_amd import learned

    t0 = time.perf_counter()
    paths = learned.random_paths(n_paths, seed)
    data = learned.generate(paths, nx=nx, ny=ny, nz=nz, states_per_path=2, n_loads=1, seed=seed)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    netw, hist = learned.train(data, nx=nx, ny=ny, nz=nz, epochs=epochs, lr=1e-3, seed=0, variant=variant)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    n_res = sum(len(s.residuals) for _, ss in data for s in ss)
    P = (nx // 4) * (ny // 4) * (nz // 4)
    out = {"workload": f"held-out beam {nx}x{ny}x{nz} Q2, lambda=100, 90 deg in 10 steps",
           "training": {"paths": [[round(a, 2), round(b, 2)] for a, b in paths], "variant": variant,
                        "residuals": n_res, "patches_per_residual": P, "pairs": n_res * P, "epochs": epochs,
                        "generate_s": round(t_gen, 2), "train_s": round(t_train, 2),
                        "mean_energy_first_last": [hist[0], hist[-1]]}}
    op, bv, cd = learned.beam(nx, ny, nz, 100.0)
    op.set_network(netw.params(), variant)
    for pc in ("gmg", "gmg_net"):
        u = torch.zeros(op.n_dofs, dtype=torch.float64, device=op.device)
        op.set_network(netw.params(), variant)  # clears a fallback of an earlier solve
        settle_beam(op, u)
        t0 = time.perf_counter()
        reps = op.solve_load_path(u, bv(90.0), 10, extrapolate=False, **dict(NEWTON_OPTS, preconditioner=pc))
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        out[pc] = {"seconds": round(secs, 3),
                   "final_residual": float(np.linalg.norm(op.residual(u).cpu().numpy())),
                   "newton_iterations": sum(r["newton_iterations"] for r in reps),
                   "cg_iterations": sum(r["cg_iterations"] for r in reps),
                   "net_fallbacks": sum(r.get("net_fallbacks", 0) for r in reps)}
        print(f"[bench] learned {pc}: {secs:.2f} s, {out[pc]['cg_iterations']} CG iterations, "
              f"{out[pc]['net_fallbacks']} fallbacks", file=sys.stderr, flush=True)
    op.close()
    out["cg_iteration_ratio"] = round(out["gmg_net"]["cg_iterations"] / max(out["gmg"]["cg_iterations"], 1), 3)
    out["time_ratio"] = round(out["gmg_net"]["seconds"] / out["gmg"]["seconds"], 3)
    return out


# --------------------------------------------------------------------------- main
def main(argv=None):
    global SETTLE_S
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="box48_q2")
    ap.add_argument("--strategies", default=",".join(STRATEGIES))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mixed", default="box24_q4,box12_q6",
                    help="workloads of the FP64-vs-FP32 apply comparison (the headline one is added)")
    ap.add_argument("--no-newton", action="store_true")
    ap.add_argument("--mfma", action="store_true",
                    help="also time the matrix-core (bf16x3, bf16) sweeps in the mixed leg (slower than FP32 on "
                         "the vector ALUs at these degrees; not part of the default run)")
    ap.add_argument("--legs", default="apply,mixed,split,hex,newton,learned",
                    help="subset of apply,mixed,split,hex,newton,learned to run (profiling runs; the default runs "
                         "all)")
    ap.add_argument("--out", default=None, help="also write the JSON line to this file")
    ap.add_argument("--settle", type=float, default=SETTLE_S,
                    help="seconds of untimed load before each timed region, so the GPU runs at its steady clocks")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run 3 plain device copies of this many MiB (reference for HBM counters)")
    args = ap.parse_args(argv)
    SETTLE_S = max(0.0, args.settle)

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the multi-GPU path is a design, not a build)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2505_15535_amd as mfe
    import synthetic

    cfg = synthetic.get_config(args.workload)
    legs = set(x for x in args.legs.split(",") if x)
    mixed_precs = ("fp64", "fp32", "bf16x3", "bf16") if args.mfma else ("fp64", "fp32")
    strategies = [s for s in args.strategies.split(",") if s] if "apply" in legs else []
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
    v_host = {}   # each strategy's v = K(u) w, for the whole-vector check against the oracle
    if strategies:
        flush_src = torch.ones(1 << 26, dtype=torch.float64, device=dev)   # 512 MiB each
        flush_dst = torch.empty_like(flush_src)
    for s in strategies:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op.build_cache(s)
        torch.cuda.synchronize()
        build_ms = (time.perf_counter() - t0) * 1e3
        settle(lambda: op.apply(w, out=v, strategy=s))
        for _ in range(args.warmup):
            op.apply(w, out=v, strategy=s)
        op.set_timing(TIMING_EVERY)
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
        v_host[s] = v.cpu().numpy()
        # cold: a 1 GiB copy between applies evicts the L2s and the 256 MB
        # Infinity Cache, so the vectors come from HBM as well (kernel time only)
        op.set_timing(True)
        for _ in range(10):
            flush_dst.copy_(flush_src)
            op.apply(w, out=v, strategy=s)
        torch.cuda.synchronize()
        cold_ms, _ = op.apply_kernel_ms()
        op.set_timing(False)
        model = work_model(s, cfg.degree, op.n_dofs, op.n_qpoints, (cfg.nx + 1) * (cfg.ny + 1) * (cfg.nz + 1))
        results[s] = {
            "ms_per_step": round(step_ms, 5),
            "gdofs": op.n_dofs / (step_ms * 1e-3) / 1e9,
            "kernel_ms": round(kern_ms, 5),
            "kernel_launches_timed": n_ev,
            "cache_build_ms": round(build_ms, 3),
            "cache_mb": round(op.cache_bytes(s) / 1e6, 1),
            "cold": {"kernel_ms": round(cold_ms, 5), "gdofs_kernel": round(op.n_dofs / (cold_ms * 1e-3) / 1e9, 4)},
            "roofline": roofline(model, kern_ms, measured_traffic(cfg.name, s)),
            "work_model": {k: (round(x, 3) if isinstance(x, float) else x) for k, x in model.items()},
        }
        print(f"[bench] {s}: {step_ms * 1e3:.1f} us/step, kernel {kern_ms * 1e3:.1f} us, "
              f"{results[s]['gdofs']:.2f} GDoF/s, {results[s]['roofline']['frac'] * 100:.1f}% of "
              f"{results[s]['roofline']['bound']} roof", file=sys.stderr, flush=True)

    if not results:  # a profiling run of the other legs only
        op.close()
        line = {"metric": METRIC, "legs": sorted(legs)}
        if "mixed" in legs:
            line["mixed"] = {m: mixed_leg(m, args.steps, args.warmup, precisions=mixed_precs)
                             for m in [cfg.name] + [m for m in args.mixed.split(",") if m and m != cfg.name]}
        if "split" in legs:
            line["split"] = split_leg(cfg.name, args.steps, args.warmup)
        if "hex" in legs:
            line["hex"] = hex_leg(cfg.name, args.steps, args.warmup)
        if "newton" in legs and not args.no_newton:
            line["newton"] = newton_leg()
        if "learned" in legs:
            line["learned"] = learned_leg()
        text = json.dumps(line)
        print(text, flush=True)
        if args.out:
            with open(args.out, "w") as fh:
                fh.write(text + "\n")
        return 0
    best = max(results, key=lambda k: results[k]["gdofs"])
    r = results[best]
    line = {
        "metric": METRIC,
        "value": round(r["gdofs"], 4),
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle_s": SETTLE_S,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg.description, "name": cfg.name, "strategy": best, "n_dofs": op.n_dofs,
                   "degree": cfg.degree, "cells": op.n_cells, "qpoints": op.n_qpoints,
                   "mu": cfg.mu, "lambda": cfg.lam, "u_amplitude": cfg.amplitude},
        "roofline": dict(r["roofline"], kernel=apply_kernel_name(best, cfg.degree), kernel_ms=r["kernel_ms"]),
        "set_state_ms": round(state_ms, 3),
        "strategies": results,
    }
    op.close()
    if "mixed" in legs:
        line["mixed"] = {m: mixed_leg(m, args.steps, args.warmup, precisions=mixed_precs)
                         for m in [cfg.name] + [m for m in args.mixed.split(",") if m and m != cfg.name]}
    if "split" in legs:
        line["split"] = split_leg(cfg.name, args.steps, args.warmup)
    if "hex" in legs:
        line["hex"] = hex_leg(cfg.name, args.steps, args.warmup)
    if "newton" in legs and not args.no_newton:
        line["newton"] = newton_leg()
    if "learned" in legs:
        line["learned"] = learned_leg()
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        products = {}
        line["cpu_baseline"] = cpu_baseline(cfg, product=products)
        print("[bench] timing the assembled-CSR product on the host cores", file=sys.stderr, flush=True)
        try:
            line["cpu_csr"] = cpu_csr_baseline(cfg, product=products)
        except (OSError, RuntimeError) as e:   # a host without the built oracle library or OpenMP
            line["cpu_csr"] = {"value": None, "error": str(e)}
        if v_host and products:
            line["oracle_check"] = oracle_check(v_host, products)
            print(f"[bench] whole-vector error against the oracle: {line['oracle_check']}", file=sys.stderr,
                  flush=True)
    text = json.dumps(line)
    print(text, flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
