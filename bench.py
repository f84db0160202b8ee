"""Benchmark of the DoGIP hot path on one MI355X.

Workload: 3D unit cube, 64^3 cubes x 6 Kuhn tetrahedra (1,572,864 cells), P3 scalar
elliptic problem (W = D_{N,4}, 35 double-grid nodes per cell), per-cell lognormal
coefficient exp(g) with g a Gaussian field (std 1, correlation length 0.1), zero
Dirichlet boundary.  A step is one FP64 operator apply y = A u (Algorithm 1) with u and
D resident in HBM; value = dofs / (seconds per apply) in GDoF/s.

The same line carries:
  * roofline: the apply's two kernels (tile kernel + shared-dof finish), algorithmic
    bytes / their measured time against 8 TB/s; traffic = HBM bytes from the committed
    counter summary of these kernels (null once their sources changed);
  * apply_f32: the FP32 apply (FP32 copy of D) with its fraction;
  * pcg_time_to_1e-8: time to a true FP64 relative residual of 1e-8 per solve mode
    (Jacobi FP64; mixed with FP32-stored residual; mixed_v64 with every vector FP64 and
    only the apply FP32; restarted refinement; multigrid with FP32 and FP64 V-cycles,
    the first multigrid call timed with its hierarchy build), each with its speedup and
    its difference from the FP64 solution;
  * p2: the same operator at P2 (apply fractions, Jacobi and multigrid solves);
  * secondary: the batch of 256 uneven 2D problems (batched apply, batched FP64 vs mixed
    PCG), the 2D 512^2 P5 anisotropic operator (apply fractions, PCG modes) and the 2D
    256^2 P3 inverse problem (seconds per adjoint gradient, central-difference check);
  * cpu_baseline: the CPU oracle on a bounded sample at 1 thread and all cores (CSR SpMV
    of the quadrature-assembled matrix, Algorithm 1, Jacobi-PCG), every solve mode's
    error against the oracle's direct solve on that sample, and the oracle's rows of
    b - A x at sampled dofs of each full-size solve.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 64] [--k 3] [--no-solve]
                    [--no-cpu] [--no-p2] [--no-secondary] [--workload c3|c2|c4|c5|qp|incl]
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
    tile_ms, fin_ms, cnt = op.timer_read()
    op.timer_enable(False)
    cnt = max(cnt, 1)
    return total_ms / steps, tile_ms / cnt, fin_ms / cnt


def time_apply_cold(op, u, y, prec, steps, scrub_mib=512):
    """Kernel durations of applies that each start with cold caches: before every apply a
    read-only pass over scrub_mib MiB (a sum) evicts the memory-side cache (256 MB on MI355X)
    and L2 without leaving dirty lines behind; only the apply's two launches are timed
    (the operator's HIP-event timer).  Repeated applies of one operator keep its index
    arrays and vectors (about 0.28 GB at 3D 64^3 P3) partly cache-resident, so they read
    less than all their bytes from HBM; this loop reads them all from HBM."""
    import torch

    scrub = torch.ones(scrub_mib * 1024 * 1024 // 8, dtype=torch.float64, device="cuda")
    acc = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(2):
        acc += scrub.sum()
        op.apply(u, y, prec=prec)
    torch.cuda.synchronize()
    op.timer_enable(True)
    op.timer_read()
    for _ in range(steps):
        acc += scrub.sum()
        op.apply(u, y, prec=prec)
    tile_ms, fin_ms, cnt = op.timer_read()
    op.timer_enable(False)
    del scrub
    cnt = max(cnt, 1)
    return tile_ms / cnt, fin_ms / cnt


def measured_traffic(n, k):
    """HBM bytes per apply from the committed rocprofv3 counter summary of this workload
    (FETCH_SIZE and WRITE_SIZE, calibrated by a copy of known size), per precision; empty
    when the summary is missing or was measured on other apply kernels (their sources,
    tile planning, launch code or compiler flags changed since)."""
    from paper_1710_09913_amd.build import apply_hash

    path = os.path.join(ROOT, "profiles", f"traffic_k_apply_3d{n}_p{k}_se.json")
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        doc = json.load(fh)
    if doc.get("apply_hash") != apply_hash():
        return {}
    return {p: round(v["bytes_per_apply"]) for p, v in doc.get("traffic", {}).items()}


def _host_threads():
    """Threads for the all-cores legs: the CPUs this process may run on, at most 16 (a
    one-GPU share of the host)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(16, n))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _match(product_xyz, oracle_xyz):
    """Oracle dof of each product dof, matched by coordinates."""
    from scipy.spatial import cKDTree

    dist, idx = cKDTree(oracle_xyz).query(product_xyz)
    assert dist.max() < 1e-9 and len(set(idx.tolist())) == len(idx), "dof matching failed"
    return idx


def _timed(fn, min_s=1.5, max_reps=50):
    fn()  # warm-up
    reps, t0 = 0, time.time()
    while reps < 3 or (time.time() - t0 < min_s and reps < max_reps):
        fn()
        reps += 1
    return (time.time() - t0) / reps, reps


def cpu_baseline(k, sample_solves=None, full_check=None, n_sample=10):
    """The CPU FP64 oracle on the host, on a bounded sample of the same workload (3D
    n_sample^3 Kuhn mesh, same order, lognormal coefficient), each leg at one thread and
    at all cores (threads = host CPUs available, at most 16):
      (i)   CSR SpMV of the quadrature-assembled matrix (scipy; all cores: row blocks on
            threads);
      (ii)  the oracle's Algorithm 1 (numpy; all cores: cell blocks on threads, outputs
            summed), the leg quoted as value;
      (iii) the oracle's Jacobi-PCG to 1e-8 with the Algorithm-1 apply.
    With sample_solves (GPU solutions of the same sample problem per solve mode), each
    is compared with the oracle's direct solve; with full_check (GPU solutions at full
    size), the oracle's rows of b - A x at sampled dofs are reported per mode."""
    import concurrent.futures as cf

    import numpy as np
    import scipy.sparse.linalg as spla
    from threadpoolctl import threadpool_limits

    from oracle import dogip as odg
    from oracle import fem
    from oracle import solve as osolve
    from workloads import coef_lognormal, random_vector, unit_mesh

    nthr = _host_threads()
    coords, cells = unit_mesh(3, n_sample)
    coef = coef_lognormal(coords, cells, 0)
    osp = fem.make_space(coords, cells, k)
    D = odg.build_d(osp, coef, "se")
    u = random_vector(osp.ndofs, 0)
    # 2k + 1 - 3 >= 2k - 2: the collapsed rule with k + 1 points per direction is exact for
    # the integrand of a per-cell constant coefficient
    A = fem.assemble(osp, fem.element_matrices(osp, coef, "se", nquad=k + 1))
    parts = np.array_split(np.arange(len(cells)), nthr)
    subs = [(fem.Space(coords, cells[p], k, osp.cell_dofs[p], osp.dof_coords, osp.boundary), D[p]) for p in parts]
    rows = np.array_split(np.arange(osp.ndofs), nthr)
    blocks = [A[r] for r in rows]
    legs = {}
    with threadpool_limits(limits=1), cf.ThreadPoolExecutor(nthr) as ex:
        t1, r1 = _timed(lambda: A @ u)
        tn, rn = _timed(lambda: np.concatenate(list(ex.map(lambda b: b @ u, blocks))))
        legs["csr_spmv"] = {"GDoF_s_1_thread": round(osp.ndofs / t1 / 1e9, 6),
                            "GDoF_s_all_cores": round(osp.ndofs / tn / 1e9, 6), "nnz": int(A.nnz),
                            "ms_1_thread": round(t1 * 1e3, 3), "ms_all_cores": round(tn * 1e3, 3)}
        t1, r1 = _timed(lambda: odg.apply(osp, D, u, "se"))
        tn, rn = _timed(lambda: sum(ex.map(lambda sd: odg.apply(sd[0], sd[1], u, "se"), subs)))
        legs["dogip_apply"] = {"GDoF_s_1_thread": round(osp.ndofs / t1 / 1e9, 6),
                               "GDoF_s_all_cores": round(osp.ndofs / tn / 1e9, 6),
                               "ms_1_thread": round(t1 * 1e3, 3), "ms_all_cores": round(tn * 1e3, 3)}
        value = osp.ndofs / tn / 1e9
        # (iii) Jacobi-PCG to 1e-8, f = 1, zero Dirichlet (identity rows)
        b = fem.load_vector(osp, 1.0)
        b[osp.boundary] = 0.0
        dg = odg.diagonal(osp, D, "se", True)
        mv1 = lambda v: odg.apply_dirichlet(osp, D, v, "se")  # noqa: E731

        def mvn(v):
            vt = v.copy()
            vt[osp.boundary] = 0.0
            y = sum(ex.map(lambda sd: odg.apply(sd[0], sd[1], vt, "se"), subs))
            y[osp.boundary] = v[osp.boundary]
            return y

        t0 = time.time()
        _, it1, rr1 = osolve.pcg(mv1, b, dg, 1e-8)
        s1 = time.time() - t0
        t0 = time.time()
        _, itn, rrn = osolve.pcg(mvn, b, dg, 1e-8)
        sn = time.time() - t0
        legs["jacobi_pcg_1e-8"] = {"seconds_1_thread": round(s1, 3), "seconds_all_cores": round(sn, 3),
                                   "iters": it1, "iters_all_cores": itn, "relres": max(rr1, rrn)}
    out = {
        "value": round(value, 6),
        "unit": "GDoF/s",
        "cores": nthr,
        "kind": "oracle",
        "sample": f"3D {n_sample}^3 Kuhn mesh ({len(cells)} cells, {osp.ndofs} dofs), P{k} elliptic, lognormal "
                  f"coefficient; value: the oracle's numpy Algorithm-1 apply on {nthr} threads (cell blocks); "
                  f"legs at 1 thread and at {nthr}",
        "cpu_model": _cpu_model(),
        "logical_cpus": os.cpu_count(),
        "legs": legs,
    }
    if sample_solves is not None:
        # the same problem solved by the oracle's sparse LU (interior block, x_B = 0)
        mask = np.ones(osp.ndofs, bool)
        mask[osp.boundary] = False
        I = np.nonzero(mask)[0]
        xo = np.zeros(osp.ndofs)
        xo[I] = spla.splu(A[I][:, I].tocsc()).solve(b[I])
        perm = _match(sample_solves["dof_coords"], osp.dof_coords)
        chk = {}
        for mode, x in sample_solves["x"].items():
            xg = np.zeros(osp.ndofs)
            xg[perm] = x
            r = b[I] - A[I][:, I] @ xg[I]
            chk[mode] = {"rel_err_vs_oracle_direct": float(np.linalg.norm(xg - xo) / np.linalg.norm(xo)),
                         "oracle_relres": float(np.linalg.norm(r) / np.linalg.norm(b[I]))}
        out["sample_solves_vs_oracle"] = chk
    if full_check is not None:
        out["full_size_solves_oracle_rows"] = _full_rows(full_check, k)
    return out


def _full_rows(fc, k, nsample=200, seed=77):
    """Oracle rows of b - A x at a seeded sample of interior dofs of the full-size problem,
    for each mode's x: rows of A from the oracle's Algorithm 1 on the sub-mesh of every cell
    that touches a sampled dof, rows of b = int phi_i from the oracle's load vector there.
    Reports ||(b - A x)_S|| / ||b_S|| per mode."""
    import numpy as np

    from oracle import dogip as odg
    from oracle import fem

    cd, bnd = fc["cell_dofs"], fc["boundary"]
    rng = np.random.default_rng(seed)
    interior = np.setdiff1d(np.arange(fc["ndofs"]), bnd)
    samples = np.sort(rng.choice(interior, nsample, replace=False))
    touch = np.isin(cd, samples).any(axis=1)
    sub = np.nonzero(touch)[0]
    verts, local = np.unique(fc["cells"][sub], return_inverse=True)
    cells_sub = local.reshape(len(sub), -1).astype(fc["cells"].dtype)
    osp = fem.make_space(fc["coords"][verts], cells_sub, k)
    D = odg.build_d(osp, fc["coef"][sub], "se")
    bo = fem.load_vector(osp, 1.0)
    pid = np.unique(cd[sub])
    perm = _match(fc["dof_coords"][pid], osp.dof_coords)
    at = perm[np.searchsorted(pid, samples)]
    out = {}
    for mode, x in fc["x"].items():
        xo = np.zeros(osp.ndofs)
        xo[perm] = x[pid]
        xo[perm[np.isin(pid, bnd)]] = 0.0
        r = bo[at] - odg.apply(osp, D, xo, "se")[at]
        out[mode] = float(np.linalg.norm(r) / np.linalg.norm(bo[at]))
    return {"sampled_dofs": nsample, "relres_sampled": out}


def _base(metric, unit, value, ms, a, config, dtype="f64", hib=True):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
            "ms_per_step": ms, "higher_is_better": hib, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config}


def _rhs_f1(space, mesh, k):
    """b_i = int phi_i (f = 1) from the projection operator with m = 1; zero on Dirichlet dofs."""
    import numpy as np
    import torch

    from paper_1710_09913_amd import Operator, Space

    wp = Operator(Space(mesh, k, "wp", "none"), torch.ones(space.ncells, dtype=torch.float64), "scalar", fp32=False)
    b = wp.apply(torch.ones(space.ndofs, dtype=torch.float64, device="cuda"))
    if space.info["bc"]:
        b[torch.from_numpy(space.boundary().astype(np.int64)).cuda()] = 0.0
    return b


def run_c2(a):
    """2D unit square 512^2 x 2 triangles, P1..P5, projection (m ~ U[1,100]) and elliptic
    (anisotropic SPD per cell): FP64 and FP32 apply, and for the elliptic problem PCG to
    1e-8 (FP64, mixed, and multigrid-preconditioned with the FP32 V-cycle).  The projection rows also time the global form (Theorem 1: one D
    value per dof of C_{N,2k}) beside the element-wise one (Theorem 2)."""
    import torch

    from paper_1710_09913_amd import Mesh, Operator, Space
    from workloads import coef_aniso_2d, coef_uniform, random_vector

    n = 512
    mesh = Mesh.unit(2, n)
    rows = []
    for kind in ("wp", "se"):
        for k in (1, 2, 3, 4, 5):
            sp = Space(mesh, k, kind, "dirichlet" if kind == "se" else "none")
            if kind == "wp":
                op = Operator(sp, torch.from_numpy(coef_uniform(sp.ncells, 1, 100, a.seed)), "scalar", fp32=True)
            else:
                op = Operator(sp, torch.from_numpy(coef_aniso_2d(sp.ncells, a.seed)), "sym", fp32=True)
            u = torch.from_numpy(random_vector(sp.ndofs, a.seed)).cuda()
            y = torch.empty_like(u)
            row = {"kind": kind, "k": k, "ndofs": sp.ndofs, "d_bytes_f64": op.info["bytes_d64"]}

            def timed(o, tag):
                for prec in ("f64", "f32"):
                    ms, kms, fms = time_apply(o, u, y, prec, a.steps, a.warmup)
                    kms += fms
                    ab = o.info["alg_bytes_" + prec]
                    row[tag + prec] = {"GDoF_s": round(sp.ndofs / (ms * 1e-3) / 1e9, 3), "ms": round(ms, 5),
                                       "frac": round(ab / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

            timed(op, "")
            if kind == "wp":
                og = Operator(sp, torch.from_numpy(coef_uniform(sp.ncells, 1, 100, a.seed)), "scalar", fp32=True,
                              global_w=True)
                timed(og, "global_")
                row["global_d_bytes_f64"] = og.info["bytes_d64"]
                del og
            if kind == "se" and not a.no_solve:
                b = _rhs_f1(sp, mesh, k)
                for mode in ("f64", "mixed", "pmg_mixed"):
                    torch.cuda.synchronize()
                    t0 = time.time()
                    op.pcg(b, tol=1e-8, maxit=200000, mode=mode, raise_on_error=False)  # warm-up / hierarchy
                    torch.cuda.synchronize()
                    first = time.time() - t0
                    t0 = time.time()
                    _, st = op.pcg(b, tol=1e-8, maxit=200000, mode=mode, raise_on_error=False)
                    dt = time.time() - t0
                    row["pcg_" + mode] = {"seconds": round(dt, 4), "iters": st["iters"], "status": st["status"],
                                          "relres_true": st["relres_true"]}
                    if mode.startswith("pmg"):
                        row["pcg_" + mode]["first_call_seconds"] = round(first, 4)
            log(f"[c2] {row}")
            rows.append(row)
            del op
    head = next(r for r in rows if r["kind"] == "se" and r["k"] == 5)
    out = _base("DoGIP apply GDoF/s, 2D 512^2 P1..P5 (projection and elliptic)", "GDoF/s", head["f64"]["GDoF_s"],
                head["f64"]["ms"], a, {"workload": "2D unit square 512^2 x 2 triangles, P1..P5, projection "
                                                   "(m ~ U[1,100]) and elliptic (anisotropic SPD, eigenvalues ~ U[1,100])",
                                       "value_row": "elliptic P5 FP64 apply"})
    out["rows"] = rows
    return out


def run_c4(a):
    """2D 256^2 P3 inverse problem: time of one gradient (forward PCG + adjoint PCG +
    contraction) with Jacobi or multigrid preconditioning, FP64 or mixed, and a
    finite-difference spot check."""
    import numpy as np
    import torch

    from paper_1710_09913_amd import Mesh, Operator, Space
    from paper_1710_09913_amd.autograd import solve
    from workloads import theta_normal

    n, k = 256, 3
    mesh = Mesh.unit(2, n)
    sp = Space(mesh, k, "se", "dirichlet")
    op = Operator(sp, torch.zeros(sp.ncells, dtype=torch.float64), "logscalar", fp32=True)
    b = _rhs_f1(sp, mesh, k)
    bnd = torch.from_numpy(sp.boundary().astype(np.int64)).cuda()
    with torch.no_grad():
        u_star = solve(torch.from_numpy(theta_normal(sp.ncells, 99)).cuda(), b, op, tol=1e-12)
        rms = torch.sqrt(torch.mean(u_star ** 2))
        u_obs = u_star + 0.01 * rms * torch.from_numpy(np.random.default_rng(5).standard_normal(sp.ndofs)).cuda()
        u_obs[bnd] = 0.0
    theta0 = torch.from_numpy(theta_normal(sp.ncells, 1)).cuda()
    times, grads = {}, {}
    for mode, tol in (("f64", 1e-10), ("mixed", 1e-10), ("pmg", 1e-10), ("pmg_mixed", 1e-10)):
        for rep in range(2):
            th = theta0.clone().requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.time()
            u = solve(th, b, op, tol=tol, mode=mode)
            J = 0.5 * ((u - u_obs) ** 2).sum()
            J.backward()
            torch.cuda.synchronize()
            times[mode] = time.time() - t0
        grads[mode] = th.grad.detach()
        log(f"[c4] gradient ({mode}) {times[mode]:.3f}s J={J.item():.6e}")
    g = grads["mixed"]
    gdiff = {m: float(torch.linalg.norm(grads[m] - grads["f64"]) / torch.linalg.norm(grads["f64"])) for m in grads}
    rng = np.random.default_rng(7)
    errs = []
    with torch.no_grad():
        for _ in range(4):
            v = torch.from_numpy(rng.standard_normal(sp.ncells)).cuda()
            jp = 0.5 * ((solve(theta0 + 1e-6 * v, b, op, tol=1e-14) - u_obs) ** 2).sum()
            jm = 0.5 * ((solve(theta0 - 1e-6 * v, b, op, tol=1e-14) - u_obs) ** 2).sum()
            gv = torch.dot(g, v).item()
            errs.append(abs((jp - jm).item() / 2e-6 - gv) / abs(gv))
    out = _base("Adjoint gradient dJ/dtheta, 2D 256^2 P3 inverse problem: seconds per gradient", "s",
                round(times["mixed"], 4), round(times["mixed"] * 1e3, 3), a,
                {"workload": "2D 256^2 x 2 triangles, P3 elliptic, theta ~ N(0, 0.5^2), u_obs from hidden theta* + 1% noise",
                 "ndofs": sp.ndofs, "ncells": sp.ncells}, hib=False)
    out["gradient_seconds"] = {m: round(t, 4) for m, t in times.items()}
    out["gradient_rel_diff_vs_f64"] = gdiff
    out["fd_rel_err_max_4dirs"] = max(errs)
    return out


def c5_problems(seed):
    """The batch workload: 256 2D elliptic problems (N ~ logU[32,256], k ~ U{1..4},
    a ~ U[1,10], zero Dirichlet) with tuned tiles, as operators, their Batch, and the
    coefficients (mesh cell order)."""
    import torch

    from paper_1710_09913_amd import Batch, Mesh, Operator, Space, tune
    from workloads import batch_spec, coef_uniform

    unrolled = 1  # batched launches take the unrolled kernels with at most 256-cell tiles
    for k in (1, 2, 3, 4):
        if tune.tuned(2, k, "se", "f32", tag="batch") == (0, 0):
            tune.tune(2, k, "se", "f32", max_tile_cells=256, variants=(unrolled,), tag="batch")
    spec = batch_spec(256, seed)
    ops, coefs, meshes = [], [], {}
    for n, k, sub in spec:
        if n not in meshes:
            meshes[n] = Mesh.unit(2, n)
        sp = Space(meshes[n], k, "se", "dirichlet")
        tw, var = tune.tuned(2, k, "se", "f32", tag="batch")
        coefs.append(coef_uniform(sp.ncells, 1, 10, seed, sub))
        ops.append(Operator(sp, torch.from_numpy(coefs[-1]), "scalar", fp32=True, tile_waves=tw, variant=var))
    return ops, Batch(ops), coefs


def run_c5(a):
    """256 independent 2D elliptic problems (N ~ logU[32,256], k ~ U{1..4}, a ~ U[1,10]):
    tuned tiles, one persistent launch per apply, batched FP64 vs mixed PCG to 1e-8,
    against solving the problems one after another."""
    import numpy as np
    import torch

    t0 = time.time()
    ops, bt, _ = c5_problems(a.seed)
    log(f"[c5] {len(ops)} problems, {bt.ndofs} dofs, setup {time.time() - t0:.1f}s")
    rhs = torch.ones(bt.ndofs, dtype=torch.float64, device="cuda")
    for i, op in enumerate(ops):
        rhs[torch.from_numpy(op.space.boundary().astype(np.int64) + int(bt.offsets[i])).cuda()] = 0.0
    u = torch.ones(bt.ndofs, dtype=torch.float64, device="cuda")
    y = torch.empty_like(u)
    apply_ms = {}
    for prec in ("f64", "f32"):
        for _ in range(a.warmup):
            bt.apply(u, y, prec=prec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.steps):
            bt.apply(u, y, prec=prec)
        e1.record()
        torch.cuda.synchronize()
        apply_ms[prec] = e0.elapsed_time(e1) / a.steps
    solve_s = {}
    for mode in ("f64", "mixed"):
        bt.pcg(rhs, tol=1e-8, maxit=50000, mode=mode)
        torch.cuda.synchronize()
        t0 = time.time()
        _, stats = bt.pcg(rhs, tol=1e-8, maxit=50000, mode=mode)
        torch.cuda.synchronize()
        solve_s[mode] = time.time() - t0
        bad = [s for s in stats if s["status"] != 0]
        dof_it = sum(s["iters"] * (int(bt.offsets[i + 1]) - int(bt.offsets[i])) for i, s in enumerate(stats))
        log(f"[c5] batched pcg {mode}: {solve_s[mode]:.3f}s, max iters {max(s['iters'] for s in stats)}, "
            f"failures {len(bad)}, {dof_it / solve_s[mode] / 1e9:.2f} G dof-iterations/s")
    t0 = time.time()
    for i, op in enumerate(ops):
        lo, hi = int(bt.offsets[i]), int(bt.offsets[i + 1])
        op.pcg(rhs[lo:hi].contiguous(), tol=1e-8, maxit=50000, mode="mixed")
    torch.cuda.synchronize()
    seq = time.time() - t0
    log(f"[c5] one problem after another (mixed): {seq:.3f}s")
    # one after another with the multigrid preconditioner: a first pass builds each
    # problem's hierarchy, the second is timed
    pmg = {}
    for rep in ("first_pass", "timed"):
        t0 = time.time()
        worst = 0.0
        for i, op in enumerate(ops):
            lo, hi = int(bt.offsets[i]), int(bt.offsets[i + 1])
            _, st = op.pcg(rhs[lo:hi].contiguous(), tol=1e-8, maxit=5000, mode="pmg_mixed")
            worst = max(worst, st["relres_true"])
        torch.cuda.synchronize()
        pmg[rep] = time.time() - t0
    log(f"[c5] one problem after another (multigrid, FP32 V-cycle): {pmg['timed']:.3f}s "
        f"(first pass with the hierarchies {pmg['first_pass']:.3f}s), worst relres {worst:.2e}")
    # the same solves from several host threads, each on its own stream (every operator owns its
    # work buffers and hierarchy, so the small, latency-bound solves overlap on the GPU)
    import concurrent.futures

    nthreads = max(1, a.threads)
    streams = [torch.cuda.Stream() for _ in range(nthreads)]
    torch.cuda.synchronize()

    def solve_share(t):
        w = 0.0
        with torch.cuda.stream(streams[t]):
            for i in range(t, len(ops), nthreads):
                lo, hi = int(bt.offsets[i]), int(bt.offsets[i + 1])
                _, st = ops[i].pcg(rhs[lo:hi].contiguous(), tol=1e-8, maxit=5000, mode="pmg_mixed",
                                   stream=streams[t])
                w = max(w, st["relres_true"] if st["status"] == 0 else float("inf"))
        return w

    t0 = time.time()
    with concurrent.futures.ThreadPoolExecutor(nthreads) as ex:
        worst_mt = max(ex.map(solve_share, range(nthreads)))
    torch.cuda.synchronize()
    pmg["threads"] = time.time() - t0
    log(f"[c5] multigrid solves from {nthreads} threads / streams: {pmg['threads']:.3f}s, worst relres {worst_mt:.2e}")
    out = _base("Batch of 256 uneven 2D elliptic problems: batched mixed PCG time-to-1e-8", "s",
                round(solve_s["mixed"], 4), round(apply_ms["f32"], 5), a,
                {"workload": "256 2D elliptic problems, N ~ round(logU[32,256]), k ~ U{1..4}, a ~ U[1,10]",
                 "ndofs_total": bt.ndofs}, hib=False)
    out["batch_apply_GDoF_s"] = {p: round(bt.ndofs / (ms * 1e-3) / 1e9, 3) for p, ms in apply_ms.items()}
    out["batched_pcg_seconds"] = {m: round(t, 4) for m, t in solve_s.items()}
    out["sequential_mixed_pcg_seconds"] = round(seq, 4)
    out["sequential_pmg_mixed_seconds"] = round(pmg["timed"], 4)
    out["sequential_pmg_mixed_first_pass_seconds"] = round(pmg["first_pass"], 4)
    out["threaded_pmg_mixed_seconds"] = {"threads": nthreads, "seconds": round(pmg["threads"], 4),
                                         "worst_relres_true": worst_mt}
    return out


def run_qp(a):
    """DoGIP against the conventional quadrature-point apply (the comparison of Section 3.3)
    on the 3D 64^3 P3 elliptic operator: the quadrature-point operator with the collapsed
    Gauss rule of n = 2..6 points per direction (n = 4 is the lowest exact for a per-cell
    constant coefficient, degree 2k-2 = 4; n = 6 integrates degree 3k = 9), beside the
    DoGIP apply (W_T = 35 nodes).  The per-point samples repeat the cell's lognormal
    value (the timing does not depend on the values)."""
    import torch

    from paper_1710_09913_amd import Mesh, Operator, Space
    from workloads import random_vector

    coef = torch.from_numpy(_lognormal(a.n, a.seed))
    space = Space(Mesh.unit(3, a.n), a.k, "se", "dirichlet")
    op = Operator(space, coef, "scalar", fp32=True)
    coef = coef.cuda()
    u = torch.from_numpy(random_vector(space.ndofs, a.seed)).cuda()
    y = torch.empty_like(u)
    rows = []

    def timed(o, label, extra):
        row = {"method": label, **extra}
        for prec in ("f64", "f32"):
            ms, tms, fms = time_apply(o, u, y, prec, a.steps, a.warmup)
            kms = tms + fms
            ab, fl = o.info["alg_bytes_" + prec], o.info["alg_flops"]
            row[prec] = {"ms": round(ms, 5), "GDoF_s": round(space.ndofs / (ms * 1e-3) / 1e9, 3),
                         "alg_GB": round(ab / 1e9, 4), "hbm_frac": round(ab / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "TFLOP_s": round(fl / (kms * 1e-3) / 1e12, 2)}
        log(f"[qp] {row}")
        rows.append(row)

    timed(op, "dogip", {"points": space.info["wt"]})
    d = 3
    for n in (2, 3, 4, 5, 6):
        nq = n ** d
        samples = coef[:, None].expand(space.ncells, nq).contiguous()
        q = Operator.quadrature(space, n, samples)
        del samples
        timed(q, "quadrature", {"points": nq, "per_dir": n, "exact_degree": 2 * n - d})
        del q
        torch.cuda.empty_cache()
    dog = rows[0]["f64"]["ms"]
    cross = [r for r in rows[1:] if r["f64"]["ms"] > dog]
    out = _base("DoGIP vs quadrature-point apply, 3D 64^3 P3 elliptic: ms per FP64 apply", "ms", dog, dog, a,
                {"workload": f"3D unit cube {a.n}^3 x 6 Kuhn tets, P{a.k} elliptic, collapsed Gauss n = 2..6"},
                hib=False)
    out["rows"] = rows
    out["quadrature_slower_than_dogip_from_points"] = cross[0]["points"] if cross else None
    return out


def run_inclusions(a):
    """A coefficient with jumps inside the cells (the case Sections 2 and 3.3 argue DoGIP
    suits): 3D 64^3 P3 elliptic with a = 100 inside 64 random balls (radius 0.04..0.1) and
    1 outside.  D comes from sub-cell quadrature (red refinement of cut sub-simplices, depth
    3, collapsed Gauss 3^3 per leaf); reports its build time and quadrature points per
    cell, the apply (unchanged), PCG to 1e-8 (FP64, mixed, p-multigrid), and a quadrature-point apply
    that would evaluate about as many points at every apply."""
    import numpy as np
    import torch

    from paper_1710_09913_amd import Mesh, Operator, Space

    rng = np.random.default_rng(a.seed + 11)
    balls = np.hstack([rng.uniform(0.05, 0.95, size=(64, 3)), rng.uniform(0.04, 0.1, size=(64, 1))])
    mesh = Mesh.unit(3, a.n)
    space = Space(mesh, a.k, "se", "dirichlet")
    op = Operator(space, torch.ones(space.ncells, dtype=torch.float64), "scalar", fp32=True)
    op.set_inclusions(balls, 100.0, 1.0, depth=1, ng=2)  # warm-up (module load)
    torch.cuda.synchronize()
    t0 = time.time()
    mean_pts = op.set_inclusions(balls, 100.0, 1.0, depth=3, ng=3)
    torch.cuda.synchronize()
    t_build = time.time() - t0
    log(f"[incl] D by sub-cell quadrature {t_build:.3f}s, {mean_pts:.1f} points per cell")
    from workloads import random_vector

    u = torch.from_numpy(random_vector(space.ndofs, a.seed)).cuda()
    y = torch.empty_like(u)
    res = {"d_build_seconds": round(t_build, 4), "points_per_cell": round(mean_pts, 2)}
    for prec in ("f64", "f32"):
        ms, tms, fms = time_apply(op, u, y, prec, a.steps, a.warmup)
        res["apply_" + prec] = {"ms": round(ms, 5), "GDoF_s": round(space.ndofs / (ms * 1e-3) / 1e9, 3)}
    b = _rhs_f1(space, mesh, a.k)
    for mode in ("f64", "mixed", "pmg", "pmg_mixed"):
        torch.cuda.synchronize()
        t0 = time.time()
        # warm-up: workspace (and, for the multigrid modes, the hierarchy: each level's D by
        # the same sub-cell quadrature)
        op.pcg(b, tol=1e-8, maxit=100000, mode=mode, raise_on_error=False)
        torch.cuda.synchronize()
        first = time.time() - t0
        t0 = time.time()
        _, st = op.pcg(b, tol=1e-8, maxit=100000, mode=mode, raise_on_error=False)
        res["pcg_" + mode] = {"seconds": round(time.time() - t0, 4), "iters": st["iters"], "status": st["status"],
                              "relres_true": st["relres_true"]}
        if mode.startswith("pmg"):
            res["pcg_" + mode]["first_call_seconds"] = round(first, 4)
        log(f"[incl] pcg {mode} {res['pcg_' + mode]}")
    n_eq = max(2, int(round(mean_pts ** (1.0 / 3.0))))
    q = Operator.quadrature(space, n_eq, torch.ones(space.ncells * n_eq ** 3, dtype=torch.float64))
    ms, _, _ = time_apply(q, u, y, "f64", a.steps, a.warmup)
    res["quadrature_apply_f64"] = {"points": n_eq ** 3, "ms": round(ms, 5)}
    del q
    log(f"[incl] {res}")
    out = _base("DoGIP with sub-cell quadrature D, 3D 64^3 P3 elliptic with inclusions: FP64 apply GDoF/s",
                "GDoF/s", res["apply_f64"]["GDoF_s"], res["apply_f64"]["ms"], a,
                {"workload": f"3D unit cube {a.n}^3 x 6 Kuhn tets, P{a.k} elliptic, a = 100 in 64 balls, 1 outside, "
                             "sub-cell quadrature depth 3, 3^3 points per leaf"})
    out["inclusions"] = res
    return out


def _lognormal(n, seed):
    from workloads import coef_lognormal, unit_mesh

    coords, cells = unit_mesh(3, n)
    return coef_lognormal(coords, cells, seed)


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
    ap.add_argument("--no-p2", action="store_true", help="skip the 3D P2 block")
    ap.add_argument("--no-secondary", action="store_true", help="skip the batch and 2D P5 rows")
    ap.add_argument("--threads", type=int, default=16, help="host threads for the batch's concurrent solves")
    ap.add_argument("--workload", default="c3", choices=["c3", "c2", "c4", "c5", "qp", "incl"],
                    help="c3: 3D 64^3 P3 (default, the headline); c2: 2D 512^2 P1..P5 sweep; "
                         "c4: 2D 256^2 P3 adjoint gradient; c5: batch of 256 uneven 2D problems; "
                         "qp: DoGIP vs the quadrature-point apply on the 3D operator; "
                         "incl: inclusions (jumps inside cells) with sub-cell quadrature D")
    a = ap.parse_args(argv)
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the multi-GPU path (element partition with an interface-dof "
              "exchange) is not built, so --gpus must be 1", file=sys.stderr)
        return 2

    import torch

    torch.cuda.set_device(0)
    if a.workload != "c3":
        out = {"c2": run_c2, "c4": run_c4, "c5": run_c5, "qp": run_qp, "incl": run_inclusions}[a.workload](a)
        print(json.dumps(out), flush=True)
        return 0
    space, op, b = build_problem(a.n, a.k, a.seed)
    from workloads import random_vector

    u = torch.from_numpy(random_vector(space.ndofs, a.seed)).cuda()
    y = torch.empty_like(u)
    ms64, tms64, fms64 = time_apply(op, u, y, "f64", a.steps, a.warmup)
    log(f"[apply f64] {ms64:.4f} ms/apply (tile kernel {tms64:.4f} ms, finish {fms64:.4f} ms)")
    ms32, tms32, fms32 = time_apply(op, u, y, "f32", a.steps, a.warmup)
    log(f"[apply f32] {ms32:.4f} ms/apply (tile kernel {tms32:.4f} ms, finish {fms32:.4f} ms)")
    kms64, kms32 = tms64 + fms64, tms32 + fms32
    info = op.info
    cold = {}
    for prec in ("f64", "f32"):
        t, f = time_apply_cold(op, u, y, prec, a.steps)
        ab = info["alg_bytes_" + prec]
        cold[prec] = {"kernel_ms": round(t + f, 5), "tile_ms": round(t, 5), "finish_ms": round(f, 5),
                      "achieved_GB_s": round(ab / ((t + f) * 1e-3) / 1e9, 1),
                      "frac": round(ab / ((t + f) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"[apply {prec} cold caches] tile {t:.4f} ms, finish {f:.4f} ms, frac {cold[prec]['frac']}")
    gdofs = space.ndofs / (ms64 * 1e-3) / 1e9
    achieved = info["alg_bytes_f64"] / (kms64 * 1e-3) / 1e9
    traffic = measured_traffic(a.n, a.k)
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
            "traffic": traffic.get("f64"),
            "kernel": "FP64 apply: k_apply tile kernel + k_apply_finish (shared dofs, Dirichlet rows)",
            "alg_bytes_per_launch": info["alg_bytes_f64"],
            "kernel_ms": round(kms64, 5),
            "tile_ms": round(tms64, 5),
            "finish_ms": round(fms64, 5),
        },
        "apply_f32": {
            "GDoF_s": round(space.ndofs / (ms32 * 1e-3) / 1e9, 4),
            "ms": round(ms32, 5),
            "kernel_ms": round(kms32, 5),
            "tile_ms": round(tms32, 5),
            "traffic": traffic.get("f32"),
            "achieved_GB_s": round(info["alg_bytes_f32"] / (kms32 * 1e-3) / 1e9, 1),
            "frac": round(info["alg_bytes_f32"] / (kms32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        },
        "apply_cold_caches": dict(cold, note="each apply after a read-only 512 MiB pass that evicts the "
                                  "memory-side cache and L2: every byte from HBM (the loops above repeat one "
                                  "apply, whose index arrays and vectors stay partly cache-resident)"),
    }
    full_check = sample_solves = None
    if not a.no_solve:
        res, xs = solve_modes(op, b, SOLVE_MODES, keep_x=not a.no_cpu)
        out["pcg_time_to_1e-8"] = res
        if not a.no_cpu:
            coords, cells = unit_mesh_np(a.n)
            full_check = {"x": xs, "cell_dofs": space.cell_dofs(), "boundary": space.boundary(),
                          "dof_coords": space.dof_coords(), "ndofs": space.ndofs, "coords": coords,
                          "cells": cells, "coef": _lognormal(a.n, a.seed)}
    del op
    torch.cuda.empty_cache()
    if not a.no_p2 and a.k == 3:
        out["p2"] = run_p2_block(a)
    if not a.no_secondary:
        out["secondary"] = run_secondary(a)
    if not a.no_cpu:
        if not a.no_solve:
            sample_solves = solve_sample(a.k, 10)
        t0 = time.time()
        out["cpu_baseline"] = cpu_baseline(a.k, sample_solves, full_check)
        log(f"[cpu baseline] {time.time() - t0:.1f}s {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)
    return 0


# solve modes of the headline line, in this order: the multigrid's FP32-cycle mode first so
# that its first call includes the hierarchy build
SOLVE_MODES = ("f64", "mixed", "mixed_v64", "mixed_restart", "pmg_mixed", "pmg")
MODE_METHOD = {
    "f64": "Jacobi-PCG, FP64 throughout",
    "mixed": "FP32 apply with r, p and A p STORED IN FP32 (x and inner products FP64), FP64 residual replacement "
             "(reliable updates): the residual is kept in reduced precision between replacements",
    "mixed_v64": "FP32 apply only (D copy and element arithmetic); x, r, p, A p, every inner product and the D "
                 "construction FP64, FP64 residual replacement: the stated precision contract",
    "mixed_restart": "FP64 iterative refinement around restarted FP32-apply Jacobi-PCG (inner 1e-4); residual "
                     "and inner products FP64",
    "pmg": "flexible CG, multigrid V-cycle preconditioner: orders k..1 on the mesh (Chebyshev degree 3 on "
           "[lmax/8, 1.1 lmax]), then P1 on nested meshes halved down to at most 400 interior dofs (degree 4 on "
           "[lmax/20, 1.1 lmax]), the coarsest solved with its dense inverse; FP64 cycle",
    "pmg_mixed": "the same multigrid with the V-cycle's applies in FP32 and the finest smoother's residual and "
                 "direction stored in FP32; outer CG residual and inner products FP64",
}


def solve_modes(op, b, modes, keep_x=False, tol=1e-8, maxit=20000):
    """Time-to-tolerance per mode: a first call (workspace; for the multigrid modes, the
    first of them also builds the hierarchy: its first_call_seconds is the set-up-inclusive
    time), then a timed second call from x0 = 0."""
    import torch

    res, xs = {}, {}
    for mode in modes:
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.time()
        op.pcg(b, x, tol=tol, maxit=maxit, mode=mode, inner_tol=1e-4 if mode == "mixed_restart" else 0.0)
        torch.cuda.synchronize()
        first = time.time() - t0
        t0 = time.time()
        x, st = op.pcg(b, None, tol=tol, maxit=maxit, mode=mode, inner_tol=1e-4 if mode == "mixed_restart" else 0.0)
        torch.cuda.synchronize()
        dt = time.time() - t0
        res[mode] = {"seconds": round(dt, 4), "first_call_seconds": round(first, 4), "iters": st["iters"],
                     "outer": st["outer"], "relres_true": st["relres_true"], "method": MODE_METHOD[mode]}
        if mode == "f64":
            x64 = x.clone()
        # against the FP64 Jacobi-PCG solution (both to tol: they differ by up to about cond(A) tol)
        res[mode]["rel_diff_vs_f64"] = float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64))
        if keep_x:
            xs[mode] = x.cpu().numpy()
        log(f"[pcg {mode}] {dt:.3f}s (first call {first:.3f}s) {st}")
    f64 = res["f64"]["seconds"]
    for m in modes:
        if m != "f64":
            res[m]["speedup_vs_f64"] = round(f64 / res[m]["seconds"], 3)
    pm = [m for m in modes if m.startswith("pmg")]
    if pm:
        res[pm[0]]["setup_inclusive_seconds"] = res[pm[0]]["first_call_seconds"]
        res[pm[0]]["speedup_vs_f64_setup_inclusive"] = round(f64 / res[pm[0]]["first_call_seconds"], 3)
        res[pm[0]]["note"] = "first_call_seconds builds the multigrid hierarchy (set-up inclusive)"
        for m in pm[1:]:
            res[m]["note"] = "first_call_seconds reuses the hierarchy built by " + pm[0]
    return res, xs


def unit_mesh_np(n):
    from workloads import unit_mesh

    return unit_mesh(3, n)


def solve_sample(k, n):
    """The sample problem of the CPU leg (3D n^3, order k, lognormal, f = 1) solved on the
    GPU in every mode, for the comparison with the oracle's direct solve."""
    import torch

    from paper_1710_09913_amd import Mesh, Operator, Space

    mesh = Mesh.unit(3, n)
    space = Space(mesh, k, "se", "dirichlet")
    op = Operator(space, torch.from_numpy(_lognormal(n, 0)), "scalar", fp32=True)
    b = _rhs_f1(space, mesh, k)
    xs = {}
    for mode in SOLVE_MODES:
        x, st = op.pcg(b, None, tol=1e-8, maxit=20000, mode=mode, inner_tol=1e-4 if mode == "mixed_restart" else 0.0)
        xs[mode] = x.cpu().numpy()
    return {"x": xs, "dof_coords": space.dof_coords()}


def run_p2_block(a):
    """3D 64^3 P2 elliptic (the P2 operator of the same workload): FP64 and FP32 apply with
    their roofline fractions, and PCG to 1e-8 in the Jacobi and multigrid modes."""
    import torch

    space, op, b = build_problem(a.n, 2, a.seed)
    from workloads import random_vector

    u = torch.from_numpy(random_vector(space.ndofs, a.seed)).cuda()
    y = torch.empty_like(u)
    blk = {"ndofs": space.ndofs, "tile_cells": op.info["tile_cells"]}
    for prec in ("f64", "f32"):
        ms, tms, fms = time_apply(op, u, y, prec, a.steps, a.warmup)
        kms = tms + fms
        ab = op.info["alg_bytes_" + prec]
        blk["apply_" + prec] = {"GDoF_s": round(space.ndofs / (ms * 1e-3) / 1e9, 4), "ms": round(ms, 5),
                                "kernel_ms": round(kms, 5), "alg_bytes": ab,
                                "frac": round(ab / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if not a.no_solve:
        res, _ = solve_modes(op, b, ("f64", "mixed", "mixed_v64", "pmg_mixed"))
        blk["pcg_time_to_1e-8"] = res
    log(f"[p2] {blk}")
    del op
    torch.cuda.empty_cache()
    return blk


def run_secondary(a):
    """Compact rows of three more workloads: the batch of 256 uneven 2D problems (batched
    apply, batched FP64 vs mixed PCG to 1e-8), the 2D 512^2 P5 anisotropic elliptic
    operator (apply fractions, also through the factored B^; FP64 vs mixed vs multigrid PCG
    to 1e-8) and the 2D 256^2 P3 inverse problem (gradient_row)."""
    import numpy as np
    import torch

    from paper_1710_09913_amd import Mesh, Operator, Space, capi
    from workloads import coef_aniso_2d, random_vector

    out = {}
    t0 = time.time()
    ops, bt, _ = c5_problems(a.seed)
    rhs = torch.ones(bt.ndofs, dtype=torch.float64, device="cuda")
    for i, op in enumerate(ops):
        rhs[torch.from_numpy(op.space.boundary().astype(np.int64) + int(bt.offsets[i])).cuda()] = 0.0
    setup = time.time() - t0
    u = torch.ones(bt.ndofs, dtype=torch.float64, device="cuda")
    y = torch.empty_like(u)
    c5 = {"problems": len(ops), "ndofs_total": bt.ndofs, "setup_seconds": round(setup, 2)}
    for prec in ("f64", "f32"):
        for _ in range(a.warmup):
            bt.apply(u, y, prec=prec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.steps):
            bt.apply(u, y, prec=prec)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / a.steps
        c5["batch_apply_" + prec] = {"ms": round(ms, 5), "GDoF_s": round(bt.ndofs / (ms * 1e-3) / 1e9, 3)}
    for mode in ("f64", "mixed"):
        bt.pcg(rhs, tol=1e-8, maxit=8, mode=mode, raise_on_error=False)  # workspace
        torch.cuda.synchronize()
        t0 = time.time()
        _, stats = bt.pcg(rhs, tol=1e-8, maxit=50000, mode=mode)
        torch.cuda.synchronize()
        c5["batched_pcg_" + mode] = {"seconds": round(time.time() - t0, 4),
                                     "max_iters": max(s["iters"] for s in stats),
                                     "failures": sum(1 for s in stats if s["status"] != 0),
                                     "worst_relres_true": max(s["relres_true"] for s in stats)}
    c5["speedup_mixed_vs_f64"] = round(c5["batched_pcg_f64"]["seconds"] / c5["batched_pcg_mixed"]["seconds"], 3)
    log(f"[secondary c5] {c5}")
    out["batch_256_uneven_2d"] = c5
    del ops, bt
    torch.cuda.empty_cache()

    mesh = Mesh.unit(2, 512)
    sp = Space(mesh, 5, "se", "dirichlet")
    op = Operator(sp, torch.from_numpy(coef_aniso_2d(sp.ncells, a.seed)), "sym", fp32=True)
    uu = torch.from_numpy(random_vector(sp.ndofs, a.seed)).cuda()
    yy = torch.empty_like(uu)
    c2 = {"ndofs": sp.ndofs}
    for prec in ("f64", "f32"):
        ms, tms, fms = time_apply(op, uu, yy, prec, a.steps, a.warmup)
        ab = op.info["alg_bytes_" + prec]
        c2["apply_" + prec] = {"GDoF_s": round(sp.ndofs / (ms * 1e-3) / 1e9, 3), "ms": round(ms, 5),
                               "frac": round(ab / ((tms + fms) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    # the same operator through the factored B^ (B1: gradient at the P4 nodes, B2: P4
    # interpolation to the W nodes; 946 instead of 1516 multiply-adds per product)
    opf = Operator(sp, torch.from_numpy(coef_aniso_2d(sp.ncells, a.seed)), "sym", fp32=True,
                   variant=capi.DOGIP_VARIANT_FACTORED)
    for prec in ("f64", "f32"):
        ms, tms, fms = time_apply(opf, uu, yy, prec, a.steps, a.warmup)
        ab = opf.info["alg_bytes_" + prec]
        c2["apply_" + prec + "_factored"] = {"GDoF_s": round(sp.ndofs / (ms * 1e-3) / 1e9, 3), "ms": round(ms, 5),
                                             "frac": round(ab / ((tms + fms) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    del opf
    b = _rhs_f1(sp, mesh, 5)
    for mode in ("pmg_mixed", "f64", "mixed"):
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.time()
        # first call: workspace (multigrid: the hierarchy, so this is its set-up-inclusive time)
        op.pcg(b, x, tol=1e-8, maxit=200000 if mode == "pmg_mixed" else 8, mode=mode, raise_on_error=False)
        torch.cuda.synchronize()
        first = time.time() - t0
        t0 = time.time()
        _, st = op.pcg(b, None, tol=1e-8, maxit=200000, mode=mode, raise_on_error=False)
        torch.cuda.synchronize()
        c2["pcg_" + mode] = {"seconds": round(time.time() - t0, 4), "iters": st["iters"], "status": st["status"],
                             "relres_true": st["relres_true"]}
        if mode == "pmg_mixed":
            c2["pcg_" + mode]["setup_inclusive_seconds"] = round(first, 4)
    log(f"[secondary c2 p5] {c2}")
    out["2d512_p5_aniso_se"] = c2
    del op
    torch.cuda.empty_cache()
    out["inverse_2d256_p3_gradient"] = gradient_row(a)
    return out


def gradient_row(a):
    """The inverse problem (2D 256^2 P3, theta ~ N(0, 0.5^2), u_obs from a hidden theta* plus
    1% noise): seconds per gradient dJ/dtheta (forward PCG to 1e-10, adjoint PCG, contraction
    -lambda_T^T A_T u_T) with Jacobi (FP64, mixed) and multigrid preconditioning, the
    gradients' difference from the FP64 one, and central differences (h = 1e-6) on two
    random directions."""
    import numpy as np
    import torch

    from paper_1710_09913_amd import Mesh, Operator, Space
    from paper_1710_09913_amd.autograd import solve
    from workloads import theta_normal

    mesh = Mesh.unit(2, 256)
    sp = Space(mesh, 3, "se", "dirichlet")
    op = Operator(sp, torch.zeros(sp.ncells, dtype=torch.float64), "logscalar", fp32=True)
    b = _rhs_f1(sp, mesh, 3)
    bnd = torch.from_numpy(sp.boundary().astype(np.int64)).cuda()
    with torch.no_grad():
        u_star = solve(torch.from_numpy(theta_normal(sp.ncells, 99)).cuda(), b, op, tol=1e-12)
        rms = torch.sqrt(torch.mean(u_star ** 2))
        u_obs = u_star + 0.01 * rms * torch.from_numpy(np.random.default_rng(5).standard_normal(sp.ndofs)).cuda()
        u_obs[bnd] = 0.0
    theta0 = torch.from_numpy(theta_normal(sp.ncells, 1)).cuda()
    row, grads = {"ndofs": sp.ndofs, "ncells": sp.ncells}, {}
    for mode in ("f64", "mixed", "pmg_mixed"):
        for rep in range(2):  # the first call allocates (multigrid: builds the hierarchy)
            th = theta0.clone().requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.time()
            u = solve(th, b, op, tol=1e-10, mode=mode)
            J = 0.5 * ((u - u_obs) ** 2).sum()
            J.backward()
            torch.cuda.synchronize()
            dt = time.time() - t0
        grads[mode] = th.grad.detach()
        row["gradient_seconds_" + mode] = round(dt, 4)
    g64 = grads["f64"]
    row["gradient_rel_diff_vs_f64"] = {m: float(torch.linalg.norm(g - g64) / torch.linalg.norm(g64))
                                      for m, g in grads.items() if m != "f64"}
    rng = np.random.default_rng(7)
    errs = []
    with torch.no_grad():
        for _ in range(2):
            v = torch.from_numpy(rng.standard_normal(sp.ncells)).cuda()
            jp = 0.5 * ((solve(theta0 + 1e-6 * v, b, op, tol=1e-14) - u_obs) ** 2).sum()
            jm = 0.5 * ((solve(theta0 - 1e-6 * v, b, op, tol=1e-14) - u_obs) ** 2).sum()
            gv = torch.dot(g64, v).item()
            errs.append(abs((jp - jm).item() / 2e-6 - gv) / abs(gv))
    row["central_difference_rel_err_max"] = max(errs)
    log(f"[secondary c4] {row}")
    return row


if __name__ == "__main__":
    sys.exit(main())
