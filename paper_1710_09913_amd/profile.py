"""Driver and summarizer for rocprofv3 runs of the apply kernels.

Run (each a process of its own; counters in separate passes):

    rocprofv3 --kernel-trace --stats --output-format csv -d T -o run -- python3 -m paper_1710_09913_amd.profile > T.log
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d F -o run -- python3 -m paper_1710_09913_amd.profile > F.log
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d W -o run -- python3 -m paper_1710_09913_amd.profile > W.log
    rocprofv3 --pmc TCC_EA0_RDREQ_32B_sum TCC_EA0_RDREQ_64B_sum TCC_EA0_RDREQ_128B_sum TCC_EA0_RDREQ_sum \
        --output-format csv -d R -o run -- python3 -m paper_1710_09913_amd.profile > R.log
    rocprofv3 --pmc TCC_EA0_WRREQ_sum TCC_EA0_WRREQ_64B_sum --output-format csv -d Q -o run \
        -- python3 -m paper_1710_09913_amd.profile > Q.log

The run applies the operator --reps times in FP64, then --reps times in FP32 (--variant 3:
the FP32 applies on the matrix cores; default:
3D 64^3 x 6 Kuhn tets, P3 elliptic, uniform coefficient: neither traffic nor time
depends on its values), then makes --copies device-to-device copies of a 1 GiB
buffer.  The copies' known byte counts calibrate the counters: FETCH_SIZE and
WRITE_SIZE (KiB per dispatch) are scaled by bytes moved / bytes counted.

    python3 -m paper_1710_09913_amd.profile summarize --trace T --fetch F --write W \
        --log F.log --name k_apply_3d64_p3_se --out profiles [--rdreq R --wrreq Q]

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
    ap.add_argument("--variant", type=int, default=0,
                    help="element-kernel variant (3: matrix-core FP32 apply, 4: factored B^)")
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
    ap.add_argument("--rdreq", help="run with TCC_EA0_RDREQ_32B/_64B/_128B/RDREQ (_sum): read bytes by request size")
    ap.add_argument("--wrreq", help="run with TCC_EA0_WRREQ/_64B (_sum): write bytes by request size")
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
    # cross-check of the single copy-calibrated factor: HBM bytes counted request by request
    # (32, 64 and 128-byte reads; 32 and 64-byte writes), for the copy and for each apply kernel
    reqsize = {}
    if a.rdreq and a.wrreq:
        rrows = _csv(_find(a.rdreq, "counter_collection.csv"))
        wrows = _csv(_find(a.wrreq, "counter_collection.csv"))

        def by_dispatch(rows):
            d = {}
            for r in rows:
                k = (int(r["Dispatch_Id"]), r["Kernel_Name"])
                d.setdefault(k, {})[r["Counter_Name"]] = float(r["Counter_Value"])
            return [(i, n, c) for (i, n), c in sorted(d.items())]

        def rbytes(c):
            n32, n64, n128 = (c.get(f"TCC_EA0_RDREQ_{w}B_sum", 0.0) for w in (32, 64, 128))
            return 32 * n32 + 64 * n64 + 128 * n128, c.get("TCC_EA0_RDREQ_sum", 0.0) - (n32 + n64 + n128)

        def wbytes(c):
            n, n64 = c.get("TCC_EA0_WRREQ_sum", 0.0), c.get("TCC_EA0_WRREQ_64B_sum", 0.0)
            return 32 * (n - n64) + 64 * n64

        rd, wr = by_dispatch(rrows), by_dispatch(wrows)
        cr = [rbytes(c)[0] for _, n, c in rd if "copyBuffer" in n and rbytes(c)[0] > copy_read / 8]
        cw = [wbytes(c) for _, n, c in wr if "copyBuffer" in n and wbytes(c) > copy_read / 8]
        seq_r = [(n, rbytes(c)) for _, n, c in rd if "k_apply" in n]
        seq_w = [(n, wbytes(c)) for _, n, c in wr if "k_apply" in n]

        def pairs_of(seq):
            out, i = [], 0
            while i < len(seq):
                n0 = seq[i][0]
                if "k_apply_finish" in n0 or i + 1 >= len(seq):
                    i += 1
                    continue
                is32 = "k_apply_mfma" in n0 or ("float" in n0.split(",")[3] if n0.count(",") >= 3 else False)
                out.append((is32, seq[i][1], seq[i + 1][1]))
                i += 2
            return out

        pr, pw = pairs_of(seq_r), pairs_of(seq_w)
        for prec, want32 in (("f64", False), ("f32", True)):
            r_ = [(t, f) for is32, t, f in pr if is32 == want32]
            w_ = [(t, f) for is32, t, f in pw if is32 == want32]
            if not r_ or not w_:
                continue
            mean = lambda xs: sum(xs) / len(xs)  # noqa: E731
            reqsize[prec] = {"tile_read": mean([t[0] for t, _ in r_]), "finish_read": mean([f[0] for _, f in r_]),
                             "tile_write": mean([t for t, _ in w_]), "finish_write": mean([f for _, f in w_]),
                             "unsized_read_requests": mean([t[1] + f[1] for t, f in r_])}
            reqsize[prec]["bytes_per_apply"] = sum(reqsize[prec][k] for k in
                                                   ("tile_read", "finish_read", "tile_write", "finish_write"))
        reqsize["copy_read_ratio"] = (sum(cr) / len(cr)) / copy_read if cr else None
        reqsize["copy_write_ratio"] = (sum(cw) / len(cw)) / copy_read if cw else None
    os.makedirs(a.out, exist_ok=True)
    doc = {"name": a.name, "source_hash": info["source_hash"], "apply_hash": info.get("apply_hash"), "ndofs": info["ndofs"], "ncells": info["ncells"],
           "fetch_scale": fscale, "write_scale": wscale, "traffic": res, "by_request_size": reqsize}
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
    if reqsize:
        lines += ["", "## Cross-check: bytes by request size (--pmc TCC_EA0_RDREQ_32B/64B/128B/RDREQ, then "
                  "TCC_EA0_WRREQ/WRREQ_64B)", "",
                  f"The same 1 GiB copy counts {reqsize['copy_read_ratio']:.4f} of its read bytes and "
                  f"{reqsize['copy_write_ratio']:.4f} of its written bytes this way (no factor applied).", "",
                  "| apply | tile read MB | tile write MB | finish read MB | finish write MB | total MB | "
                  "vs FETCH/WRITE scaled | unsized read requests |", "|---|---|---|---|---|---|---|---|"]
        for prec, r in reqsize.items():
            if not isinstance(r, dict):
                continue
            lines.append(f"| {prec} | {r['tile_read'] / 1e6:.1f} | {r['tile_write'] / 1e6:.1f} | "
                         f"{r['finish_read'] / 1e6:.1f} | {r['finish_write'] / 1e6:.1f} | "
                         f"{r['bytes_per_apply'] / 1e6:.1f} | "
                         f"{r['bytes_per_apply'] / res[prec]['bytes_per_apply']:.3f} | "
                         f"{r['unsized_read_requests']:.0f} |")
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
