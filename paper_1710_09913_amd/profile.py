"""Driver and summarizer for rocprofv3 runs of the apply kernels.

Run (each a process of its own; counters in separate passes):

    rocprofv3 --kernel-trace --stats --output-format csv -d T -o run -- python3 -m paper_1710_09913_amd.profile > T.log
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d F -o run -- python3 -m paper_1710_09913_amd.profile > F.log
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d W -o run -- python3 -m paper_1710_09913_amd.profile > W.log

The run applies the operator --reps times in FP64, then --reps times in FP32 (--variant 3:
the FP32 applies on the matrix cores; default:
3D 64^3 x 6 Kuhn tets, P3 elliptic, uniform coefficient: neither traffic nor time
depends on its values), then makes --copies device-to-device copies of a 1 GiB
buffer.  The copies' known byte counts calibrate the counters: FETCH_SIZE and
WRITE_SIZE (KiB per dispatch) are scaled by bytes moved / bytes counted.

    python3 -m paper_1710_09913_amd.profile summarize --trace T --fetch F --write W \
        --log F.log --name k_apply_3d64_p3_se --out profiles

writes <out>/<name>.md (durations and calibrated traffic per kernel) and
<out>/traffic_<name>.json (bytes per apply, with the source hash of the build
that was measured; a benchmark reports the traffic only while the hash matches).
"""

from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def run(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--dim", type=int, default=3)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--k", type=int, default=3)
    ap.add_argument("--kind", default="se")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--copies", type=int, default=3)
    ap.add_argument("--variant", type=int, default=0, help="element-kernel variant (3: matrix-core FP32 apply)")
    a = ap.parse_args(argv)

    import torch

    from paper_1710_09913_amd import Mesh, Operator, Space
    from paper_1710_09913_amd.build import apply_hash, source_hash
    from workloads import random_vector

    torch.cuda.set_device(0)
    sp = Space(Mesh.unit(a.dim, a.n), a.k, a.kind, "dirichlet" if a.kind == "se" else "none")
    op = Operator(sp, torch.ones(sp.ncells, dtype=torch.float64), "scalar", fp32=True, variant=a.variant)
    u = torch.from_numpy(random_vector(sp.ndofs, 0)).cuda()
    y = torch.empty_like(u)
    for prec in ("f64", "f32"):
        for _ in range(a.reps):
            op.apply(u, y, prec=prec)
    x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
    z = torch.empty_like(x)
    for _ in range(a.copies):
        z.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"ndofs": sp.ndofs, "ncells": sp.ncells, "alg_bytes_f64": op.info["alg_bytes_f64"],
                      "alg_bytes_f32": op.info["alg_bytes_f32"], "copy_bytes_each": 2 * x.numel() * 8,
                      "source_hash": source_hash(), "apply_hash": apply_hash()}), flush=True)


def _csv(path):
    import csv

    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _find(d, suffix):
    import glob

    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def _short(name):
    """Kernel name without the argument list."""
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i].replace("void ", "")
    return name.replace("void ", "")


def _run_info(log):
    with open(log) as fh:
        for line in fh:
            if line.startswith("{") and "source_hash" in line:
                return json.loads(line)
    raise ValueError(f"no run line in {log}")


def _durations(stats):
    lines = ["| kernel | calls | avg us | min us | max us | total ms |", "|---|---|---|---|---|---|"]
    for r in stats:
        lines.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.1f} |")
    return lines


def _trace_only(a, stats):
    lines = [f"# {a.name}: rocprofv3 kernel durations", ""]
    if a.command:
        lines += ["Command (from the repository root):", "", "```", a.command, "```", ""]
    lines += ["## Kernel trace (--kernel-trace --stats)", ""] + _durations(stats)
    os.makedirs(a.out, exist_ok=True)
    with open(os.path.join(a.out, f"{a.name}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def summarize(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", help="FETCH_SIZE run (omit with --write for a trace-only summary)")
    ap.add_argument("--write", help="WRITE_SIZE run")
    ap.add_argument("--log", help="stdout of one of the profiled runs (its JSON line)")
    ap.add_argument("--name", required=True)
    ap.add_argument("--out", default="profiles")
    ap.add_argument("--command", default="", help="command line recorded in the summary")
    a = ap.parse_args(argv)
    stats = _csv(_find(a.trace, "kernel_stats.csv"))
    if not (a.fetch and a.write and a.log):
        return _trace_only(a, stats)
    info = _run_info(a.log)
    fetch = _csv(_find(a.fetch, "counter_collection.csv"))
    write = _csv(_find(a.write, "counter_collection.csv"))

    def per_dispatch(rows, counter):
        out = []  # (dispatch id, kernel, KiB)
        for r in rows:
            if r["Counter_Name"] == counter:
                out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
        return sorted(out)

    fd, wd = per_dispatch(fetch, "FETCH_SIZE"), per_dispatch(write, "WRITE_SIZE")
    copy_read = info["copy_bytes_each"] // 2
    copies_f = [v for _, n, v in fd if "copyBuffer" in n and v * 1024 > copy_read / 8]
    copies_w = [v for _, n, v in wd if "copyBuffer" in n and v * 1024 > copy_read / 8]
    if not copies_f or not copies_w:
        raise ValueError("calibration copies not found in the counter runs")
    fscale = copy_read / (sum(copies_f) / len(copies_f) * 1024)
    wscale = copy_read / (sum(copies_w) / len(copies_w) * 1024)

    # apply dispatches in order: reps x (tile, finish) in FP64, then the same in FP32; a
    # finish with no tile kernel before it (the one after the Jacobi diagonal) is skipped
    def apply_pairs(disp):
        seq = [(n, v) for _, n, v in disp if "k_apply" in n]
        pairs = []
        i = 0
        while i < len(seq):
            n0, v0 = seq[i]
            if "k_apply_finish" in n0:
                i += 1
                continue
            if i + 1 >= len(seq) or "k_apply_finish" not in seq[i + 1][0]:
                raise ValueError("unexpected dispatch order")
            is32 = "k_apply_mfma" in n0 or ("float" in n0.split(",")[3] if n0.count(",") >= 3 else False)
            pairs.append((is32, v0, seq[i + 1][1]))
            i += 2
        return pairs

    res = {}
    for prec, want32 in (("f64", False), ("f32", True)):
        pf = [(t, f) for is32, t, f in apply_pairs(fd) if is32 == want32]
        pw = [(t, f) for is32, t, f in apply_pairs(wd) if is32 == want32]
        if not pf or not pw:
            continue
        mean = lambda xs: sum(xs) / len(xs)  # noqa: E731
        tile_r = mean([t for t, _ in pf]) * 1024 * fscale
        fin_r = mean([f for _, f in pf]) * 1024 * fscale
        tile_w = mean([t for t, _ in pw]) * 1024 * wscale
        fin_w = mean([f for _, f in pw]) * 1024 * wscale
        res[prec] = {"tile_read": tile_r, "tile_write": tile_w, "finish_read": fin_r, "finish_write": fin_w,
                     "bytes_per_apply": tile_r + tile_w + fin_r + fin_w,
                     "alg_bytes_per_apply": info["alg_bytes_" + prec]}
    os.makedirs(a.out, exist_ok=True)
    doc = {"name": a.name, "source_hash": info["source_hash"], "apply_hash": info.get("apply_hash"), "ndofs": info["ndofs"], "ncells": info["ncells"],
           "fetch_scale": fscale, "write_scale": wscale, "traffic": res}
    with open(os.path.join(a.out, f"traffic_{a.name}.json"), "w") as fh:
        json.dump(doc, fh, indent=1)
    lines = [f"# {a.name}: rocprofv3 kernel durations and HBM traffic", ""]
    if a.command:
        lines += ["Commands (from the repository root):", "", "```", a.command, "```", ""]
    lines += [f"Build source hash `{info['source_hash']}`, apply sources hash `{info.get('apply_hash')}`; "
              f"{info['ncells']} cells, {info['ndofs']} dofs.", "",
              "## Kernel trace (--kernel-trace --stats)", ""] + _durations(stats)
    lines += ["", "## Traffic (--pmc FETCH_SIZE, then --pmc WRITE_SIZE)", "",
              f"Calibration: a 1 GiB device copy reads {copy_read} B and the counters report "
              f"FETCH {sum(copies_f) / len(copies_f):.0f} KiB, WRITE {sum(copies_w) / len(copies_w):.0f} KiB: "
              f"scale FETCH x{fscale:.4f}, WRITE x{wscale:.4f}.", "",
              "| apply | tile read MB | tile write MB | finish read MB | finish write MB | total MB | algorithmic MB | ratio |",
              "|---|---|---|---|---|---|---|---|"]
    for prec, r in res.items():
        lines.append(f"| {prec} | {r['tile_read'] / 1e6:.1f} | {r['tile_write'] / 1e6:.1f} | "
                     f"{r['finish_read'] / 1e6:.1f} | {r['finish_write'] / 1e6:.1f} | "
                     f"{r['bytes_per_apply'] / 1e6:.1f} | {r['alg_bytes_per_apply'] / 1e6:.1f} | "
                     f"{r['bytes_per_apply'] / r['alg_bytes_per_apply']:.3f} |")
    with open(os.path.join(a.out, f"{a.name}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(json.dumps(doc))


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    if argv and argv[0] == "summarize":
        return summarize(argv[1:])
    return run(argv)


if __name__ == "__main__":
    main()
