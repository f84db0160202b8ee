"""The autotuner's choice against the library default on the tuning mesh: the tuned
(tile_waves, variant) is never slower than the default configuration (to timing noise),
and the default is among the candidates it timed.  For batched launches both are timed
as the tuner times them, in batches of copies of the operator."""

import statistics

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _mean_ms(op, u, y, prec, reps):
    op.timer_read()
    for _ in range(reps):
        op.apply(u, y, prec=prec)
    t, f, n = op.timer_read()
    return (t + f) / n


def _ms_pair(a, b, u, y, prec, reps=20, rounds=7):
    """Medians over rounds of the mean apply time (tile kernel + finish, HIP events) of two
    operators, timed in alternating rounds so that clock and thermal drift hit both."""
    for op in (a, b):
        for _ in range(3):
            op.apply(u, y, prec=prec)
        op.timer_enable(True)
    torch.cuda.synchronize()
    ta, tb = [], []
    for _ in range(rounds):
        ta.append(_mean_ms(a, u, y, prec, reps))
        tb.append(_mean_ms(b, u, y, prec, reps))
    for op in (a, b):
        op.timer_enable(False)
    return statistics.median(ta), statistics.median(tb)


def _batch_ms_pair(a, b, u, y, prec, reps=20, rounds=7):
    """The same for two batches (one persistent launch per apply, HIP events around reps)."""
    from paper_1710_09913_amd import tune

    ta, tb = [], []
    for _ in range(rounds):
        ta.append(tune._batch_ms(a, u, y, prec, reps))
        tb.append(tune._batch_ms(b, u, y, prec, reps))
    return statistics.median(ta), statistics.median(tb)


@pytest.mark.parametrize("dim,k,prec,tag,max_cells,variants", [
    (2, 3, "f32", "", 512, None),
    (2, 2, "f32", "batch", 256, (1,)),
    (3, 2, "f64", "", 512, None),
])
def test_tuned_not_slower_than_default(tmp_path, monkeypatch, dim, k, prec, tag, max_cells, variants):
    from paper_1710_09913_amd import Mesh, Operator, Space, tune

    monkeypatch.setenv("DOGIP_TUNE_CACHE", str(tmp_path / "tune.json"))
    print(f"[tune] d={dim} k={k} {prec} tag={tag!r}", flush=True)
    e = tune.tune(dim, k, "se", prec, cells_target=1_000_000, reps=10, max_tile_cells=max_cells, variants=variants,
                  tag=tag)
    assert tune.tuned(dim, k, "se", prec, tag=tag) == (e["tile_waves"], e["variant"])
    space = Space(Mesh.unit(dim, e["mesh_n"]), k, "se", "dirichlet")
    coef = torch.ones(space.ncells, dtype=torch.float64)
    default = Operator(space, coef, "scalar", fp32=prec == "f32")
    dflt = (default.info["tile_cells"] // 64, default.info["variant"])
    if default.info["tile_cells"] <= max_cells and (variants is None or dflt[1] in variants):
        assert any((c["tile_waves"], c["variant"]) == dflt for c in e["candidates"]), "default not timed"
    if (e["tile_waves"], e["variant"]) == dflt:
        return  # the tuner chose the default configuration: nothing to compare
    tuned = Operator(space, coef, "scalar", fp32=prec == "f32", tile_waves=e["tile_waves"], variant=e["variant"])
    if tag == "batch":  # compared as the tuner timed them: in batches of copies of the operator
        from paper_1710_09913_amd import Batch

        def copies(tw, var):
            return [Operator(space, coef, "scalar", fp32=prec == "f32", tile_waves=tw, variant=var)
                    for _ in range(tune.BATCH_COPIES)]

        bd, bt = Batch(copies(*dflt)), Batch(copies(e["tile_waves"], e["variant"]))
        u = torch.ones(bd.ndofs, dtype=torch.float64, device="cuda")
        y = torch.empty_like(u)
        t_def, t_tun = _batch_ms_pair(bd, bt, u, y, prec)
    else:
        u = torch.ones(space.ndofs, dtype=torch.float64, device="cuda")
        y = torch.empty_like(u)
        t_def, t_tun = _ms_pair(default, tuned, u, y, prec)
    print(f"[tune] default {dflt}: {t_def:.4f} ms, tuned {(e['tile_waves'], e['variant'])}: {t_tun:.4f} ms",
          flush=True)
    if default.info["tile_cells"] <= max_cells and (variants is None or dflt[1] in variants):
        assert t_tun <= 1.10 * t_def
