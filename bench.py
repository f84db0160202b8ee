"""Benchmark of the DoGIP hot path on one MI355X.

Workload: 3D unit cube, 64^3 cubes x 6 Kuhn tetrahedra (1,572,864 cells), P3 scalar
elliptic problem (W = D_{N,4}, 35 double-grid nodes per cell), per-cell lognormal
coefficient exp(g) with g a Gaussian field (std 1, correlation length 0.1), zero
Dirichlet boundary.  A step is one FP64 operator apply y = A u (Algorithm 1) with u and
D resident in HBM; value = dofs / (seconds per apply) in GDoF/s.

The same line carries: the FP32 apply, FP64 and mixed-precision PCG time-to-1e-8,
the roofline of the tile kernel (algorithmic bytes / measured kernel time, HBM peak
8 TB/s) and the CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 64] [--k 3] [--no-solve] [--no-cpu]
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
METRIC = "DoGIP apply GDoF/s + PCG time-to-1e-8 (3D P3), mixed vs FP64, % HBM roofline"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_problem(n, k, seed):
    import numpy as np
    import torch

    from paper_1710_09913_amd import Mesh, Operator, Space
    from workloads import coef_lognormal, unit_mesh

    t0 = time.time()
    coords, cells = unit_mesh(3, n)
    coef = coef_lognormal(coords, cells, seed)
    log(f"[setup] coefficient field {time.time() - t0:.1f}s")
    t0 = time.time()
    mesh = Mesh.unit(3, n)
    space = Space(mesh, k, "se", "dirichlet")
    log(f"[setup] space ndofs={space.ndofs} {time.time() - t0:.1f}s")
    t0 = time.time()
    op = Operator(space, torch.from_numpy(coef), "scalar", fp32=True)
    torch.cuda.synchronize()
    log(f"[setup] operator (D build + diagonal) {time.time() - t0:.1f}s, info {op.info}")
    # right-hand side f = 1: b_i = int phi_i = (mass matrix) 1, from the projection operator with m = 1
    wp = Operator(Space(mesh, k, "wp", "none"), torch.ones(space.ncells, dtype=torch.float64), "scalar", fp32=False)
    ones = torch.ones(space.ndofs, dtype=torch.float64, device="cuda")
    b = wp.apply(ones)
    b[torch.from_numpy(space.boundary().astype(np.int64)).cuda()] = 0.0
    del wp
    return space, op, b


def time_apply(op, u, y, prec, steps, warmup):
    import torch

    for _ in range(warmup):
        op.apply(u, y, prec=prec)
    torch.cuda.synchronize()
    op.timer_enable(True)
    op.timer_read()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        op.apply(u, y, prec=prec)
    e1.record(s)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    kern_ms, cnt = op.timer_read()
    op.timer_enable(False)
    return total_ms / steps, kern_ms / max(cnt, 1)


def cpu_baseline(k, n_sample=20):
    """The oracle's vectorised Algorithm 1 (numpy, float64) on a bounded sample of the same
    workload family: a 20^3 Kuhn mesh at the same order."""
    import numpy as np

    from oracle import dogip as odg
    from oracle import fem
    from workloads import coef_lognormal, random_vector, unit_mesh

    coords, cells = unit_mesh(3, n_sample)
    coef = coef_lognormal(coords, cells, 0)
    osp = fem.make_space(coords, cells, k)
    D = odg.build_d(osp, coef, "se")
    u = random_vector(osp.ndofs, 0)
    odg.apply_dirichlet(osp, D, u, "se")  # warm-up
    reps, t0 = 0, time.time()
    while reps < 3 or time.time() - t0 < 10.0:
        odg.apply_dirichlet(osp, D, u, "se")
        reps += 1
        if time.time() - t0 > 30.0:
            break
    dt = (time.time() - t0) / reps
    return {
        "value": round(osp.ndofs / dt / 1e9, 6),
        "unit": "GDoF/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"3D {n_sample}^3 Kuhn mesh ({len(cells)} cells, {osp.ndofs} dofs), P{k} elliptic, "
                  f"FP64 numpy apply x{reps}, {dt * 1e3:.1f} ms each; host has {os.cpu_count()} logical CPUs",
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--k", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    a = ap.parse_args(argv)
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the multi-GPU path (element partition with an interface-dof "
              "exchange) is not built, so --gpus must be 1", file=sys.stderr)
        return 2

    import torch

    torch.cuda.set_device(0)
    space, op, b = build_problem(a.n, a.k, a.seed)
    from workloads import random_vector

    u = torch.from_numpy(random_vector(space.ndofs, a.seed)).cuda()
    y = torch.empty_like(u)
    ms64, kms64 = time_apply(op, u, y, "f64", a.steps, a.warmup)
    log(f"[apply f64] {ms64:.4f} ms/apply (tile kernel {kms64:.4f} ms)")
    ms32, kms32 = time_apply(op, u, y, "f32", a.steps, a.warmup)
    log(f"[apply f32] {ms32:.4f} ms/apply (tile kernel {kms32:.4f} ms)")
    info = op.info
    gdofs = space.ndofs / (ms64 * 1e-3) / 1e9
    achieved = info["alg_bytes_f64"] / (kms64 * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(gdofs, 4),
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms64, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"3D unit cube {a.n}^3 x 6 Kuhn tets, P{a.k} scalar elliptic (W = D_(N,{2 * a.k - 2})), "
                        "lognormal per-cell coefficient (std 1, corr. length 0.1), zero Dirichlet",
            "ncells": space.ncells,
            "ndofs": space.ndofs,
            "tile_cells": info["tile_cells"],
            "variant": "unrolled" if info["variant"] == 1 else "looped",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "kernel": "k_apply (tile kernel), FP64",
            "alg_bytes_per_launch": info["alg_bytes_f64"],
            "kernel_ms": round(kms64, 5),
        },
        "apply_f32": {
            "GDoF_s": round(space.ndofs / (ms32 * 1e-3) / 1e9, 4),
            "ms": round(ms32, 5),
            "kernel_ms": round(kms32, 5),
            "achieved_GB_s": round(info["alg_bytes_f32"] / (kms32 * 1e-3) / 1e9, 1),
            "frac": round(info["alg_bytes_f32"] / (kms32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        },
    }
    if not a.no_solve:
        res = {}
        for mode in ("f64", "mixed", "mixed_restart"):
            x = torch.zeros_like(b)
            op.pcg(b, x, tol=1e-8, maxit=20000, mode=mode)  # warm-up (allocates the workspace)
            torch.cuda.synchronize()
            t0 = time.time()
            x, st = op.pcg(b, None, tol=1e-8, maxit=20000, mode=mode, inner_tol=1e-4 if mode == "mixed_restart" else 0.0)
            torch.cuda.synchronize()
            dt = time.time() - t0
            res[mode] = {"seconds": round(dt, 4), "iters": st["iters"], "outer": st["outer"],
                         "relres_true": st["relres_true"]}
            log(f"[pcg {mode}] {dt:.3f}s {st}")
        res["speedup_mixed_vs_f64"] = round(res["f64"]["seconds"] / res["mixed"]["seconds"], 3)
        res["mixed"]["method"] = "FP32 apply, FP64 vectors, FP64 residual replacement (reliable updates)"
        res["mixed_restart"]["method"] = "FP64 iterative refinement around restarted FP32-apply PCG (inner 1e-4)"
        out["pcg_time_to_1e-8"] = res
    if not a.no_cpu:
        t0 = time.time()
        out["cpu_baseline"] = cpu_baseline(a.k)
        log(f"[cpu baseline] {time.time() - t0:.1f}s {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
