"""Autotuner for the apply kernels: picks the tile size (cells per tile, taken by one
workgroup in passes when larger than its lanes) and the element-kernel variant per
(dim, k, kind, precision) by timing candidates on a representative structured mesh, and
caches the choice as JSON.

    python -m paper_1710_09913_amd.tune --dim 2 --kind se --k 1 2 3 4 --prec f64 f32

Cache: $DOGIP_TUNE_CACHE, else ~/.cache/dogip/tune.json.  ``tuned`` returns the cached
choice to pass to ``Operator(..., tile_waves=, variant=)``; with 0 the library's built-in
defaults apply.
"""

from __future__ import annotations

import argparse
import json
import os

from . import capi

TILE_WAVES = (1, 2, 4, 8, 12, 16, 24, 48)  # cells per tile / 64; tiles above 8 waves run in passes


def cache_path() -> str:
    return os.environ.get("DOGIP_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "dogip", "tune.json")


def _key(dim, k, kind, prec, tag=""):
    return f"d{dim}-k{k}-{kind}-{prec}" + (f"-{tag}" if tag else "")


def load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(c: dict) -> None:
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def tuned(dim, k, kind, prec="f64", tag=""):
    """(tile_waves, variant) from the cache, or (0, 0) for the library defaults.  tag names
    a restricted search (for instance "batch": unrolled kernels and at most 256-cell tiles,
    what batched launches accept)."""
    e = load_cache().get(_key(dim, k, kind, prec, tag))
    return (e["tile_waves"], e["variant"]) if e else (0, 0)


BATCH_COPIES = 4  # operators in the batch that times a candidate for batched launches


def _op_ms(op, u, y, prec, reps):
    """Mean time of one apply (tile kernel + second pass, the operator's HIP-event timer)."""
    import torch

    for _ in range(3):
        op.apply(u, y, prec=prec)
    torch.cuda.synchronize()
    op.timer_enable(True)
    op.timer_read()
    for _ in range(reps):
        op.apply(u, y, prec=prec)
    t, fin, cnt = op.timer_read()
    op.timer_enable(False)
    return (t + fin) / cnt


def _batch_ms(bt, u, y, prec, reps):
    """Mean time of one batched apply (HIP events on the current stream around reps applies)."""
    import torch

    for _ in range(3):
        bt.apply(u, y, prec=prec)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        bt.apply(u, y, prec=prec)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _mesh_size(dim, k, cells_target):
    per = 2 if dim == 2 else 6
    return max(2, int(round((cells_target / per) ** (1.0 / dim))))


def tune(dim, k, kind, prec="f64", cells_target=400_000, reps=20, tile_waves=TILE_WAVES, variants=None,
         max_tile_cells=3072, verbose=False, tag="") -> dict:
    """Time every candidate on a unit mesh of about cells_target cells; store and return the
    best under the key of (dim, k, kind, prec, tag).  With tag "batch" a candidate is timed
    as the batched kernel runs it: BATCH_COPIES operators of the mesh in one batch, one
    persistent launch per apply (the batched kernel weighs a tile's fixed costs differently
    from the single-operator kernel, so the single-operator timing would mislead it)."""
    import torch

    from .dogip import Batch, Mesh, Operator, Space

    n = _mesh_size(dim, k, cells_target // BATCH_COPIES if tag == "batch" else cells_target)
    space = Space(Mesh.unit(dim, n), k, kind, "dirichlet" if kind == "se" else "none")
    coef = torch.ones(space.ncells, dtype=torch.float64)
    u = torch.ones(space.ndofs * (BATCH_COPIES if tag == "batch" else 1), dtype=torch.float64, device="cuda")
    y = torch.empty_like(u)
    has_unrolled = (dim == 2 and k <= 5) or (dim == 3 and (k <= 3 if kind == "se" else k <= 2))
    if variants is None:
        variants = (capi.DOGIP_VARIANT_UNROLLED, capi.DOGIP_VARIANT_LOOPED) if has_unrolled else (capi.DOGIP_VARIANT_LOOPED,)
        if dim == 3 and k == 3 and kind == "se" and prec == "f32":  # the matrix-core FP32 apply
            variants = variants + (capi.DOGIP_VARIANT_MFMA,)
        if kind == "se" and 2 <= k <= (5 if dim == 2 else 3):  # the factored B^
            variants = variants + (capi.DOGIP_VARIANT_FACTORED,)
    rows = []
    for var in variants:
        for tw in tile_waves:
            if 64 * tw > max_tile_cells or (var == capi.DOGIP_VARIANT_MFMA and tw > 8):
                continue
            op = Operator(space, coef, "scalar", fp32=(prec == "f32"), tile_waves=tw, variant=var)
            if op.info["tile_cells"] != 64 * tw:  # shrunk to fit the LDS budget: duplicate candidate
                del op
                continue
            if tag == "batch":
                ops = [op] + [Operator(space, coef, "scalar", fp32=(prec == "f32"), tile_waves=tw, variant=var)
                              for _ in range(BATCH_COPIES - 1)]
                ms = _batch_ms(Batch(ops), u, y, prec, reps)
                del ops
            else:
                ms = _op_ms(op, u, y, prec, reps)
            rows.append({"tile_waves": tw, "variant": var, "ms": ms})
            if verbose:
                print(f"  {_key(dim, k, kind, prec, tag)} tw={tw} var={var}: {ms:.4f} ms", flush=True)
            del op
    best = min(rows, key=lambda r: r["ms"])
    entry = {"tile_waves": best["tile_waves"], "variant": best["variant"], "ms": best["ms"],
             "mesh_n": n, "ndofs": space.ndofs, "candidates": rows}
    c = load_cache()
    c[_key(dim, k, kind, prec, tag)] = entry
    save_cache(c)
    return entry


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--dim", type=int, default=2)
    ap.add_argument("--kind", default="se")
    ap.add_argument("--k", type=int, nargs="+", default=[1, 2, 3, 4])
    ap.add_argument("--prec", nargs="+", default=["f64", "f32"])
    ap.add_argument("--cells", type=int, default=400_000)
    ap.add_argument("--max-tile-cells", type=int, default=3072)
    a = ap.parse_args(argv)
    for k in a.k:
        for prec in a.prec:
            e = tune(a.dim, k, a.kind, prec, cells_target=a.cells, max_tile_cells=a.max_tile_cells, verbose=True)
            print(json.dumps({_key(a.dim, k, a.kind, prec): {x: e[x] for x in ("tile_waves", "variant", "ms")}}),
                  flush=True)


if __name__ == "__main__":
    main()
