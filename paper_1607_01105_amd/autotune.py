"""Tile-shape autotuner of the stage kernels.

The library offers a few work-group tile shapes per dimensionality
(``ppml_tile_count`` / ``ppml_tile_shape``): a work group owns a tx x ty
column of cells (3-D kernels march it along z).  Every shape runs the same
per-cell arithmetic, so the results are bit-identical; what changes is the
halo overhead per cell, the LDS footprint (hence resident work groups per
CU), and how well the tiles cover the grid.  The best shape depends on the
grid size, the precision and, for batches, on the mix of grids, so the tuner
times each shape on the caller's own workload -- HIP events on the solver's
stream around a few steps -- and returns the fastest.  Results are memoised
per workload key within the process.

The timing runs advance the given state; callers re-set it afterwards.
"""
from __future__ import annotations

import collections

from .ppml import Batch, Grid, load, ppml_tile_count, ppml_tile_shape

_cache: dict = {}


def pick(times: dict) -> int:
    """The fastest shape; a tie goes to the lower index (the default first)."""
    return min(sorted(times), key=lambda v: (times[v], v))


def tune_grid(prob, prec="fp32", steps=8, warmup=2, log=None) -> dict:
    """Best tile shape for stepping this problem alone (solo launches).

    Returns {"tile": index, "shape": (tx, ty), "ms_per_step": {index: ms}}."""
    # the workload's name as well: its force terms select other kernel
    # instantiations than a plain grid of the same size
    key = ("grid", prob.name, prob.ndim, tuple(prob.n[:prob.ndim]), prec)
    if key in _cache:
        return _cache[key]
    lib = load()
    times = {}
    for v in range(ppml_tile_count(prob.ndim, lib)):
        g = Grid.from_problem(prob, prec=prec, tile=v)
        g.step(warmup)
        g.sync()
        g.set_timing(steps)
        g.step(steps)
        me, ml, n = g.get_timing()
        times[v] = (me + ml) / max(n, 1)
        if log:
            log(f"[autotune] {prob.ndim}-D {prec} tile {ppml_tile_shape(prob.ndim, v, lib)}: {times[v]:.4f} ms/step")
        del g
    best = pick(times)
    res = {"tile": best, "shape": ppml_tile_shape(prob.ndim, best, lib), "ms_per_step": times}
    _cache[key] = res
    return res


def tune_batch(probs, prec="fp32", steps=10, warmup=2, log=None) -> dict:
    """Best tile shape per dimensionality for a batch of these problems.

    The grids of each dimensionality are stepped together, alone in a batch,
    once per shape (eager launches timed with HIP events on the batch
    stream).  Returns {ndim: {"tile": index, "shape": (tx, ty),
    "ms_per_step": {index: ms}}}."""
    import torch

    key = ("batch", prec, tuple(sorted((p.ndim, tuple(p.n[:p.ndim])) for p in probs)))
    if key in _cache:
        return _cache[key]
    lib = load()
    by_nd = collections.defaultdict(list)
    for p in probs:
        by_nd[p.ndim].append(p)
    stream = torch.cuda.Stream()
    out = {}
    for nd in sorted(by_nd):
        ps = by_nd[nd]
        grids = [Grid.from_problem(p, prec=prec, stream=stream) for p in ps]
        times = {}
        for v in range(ppml_tile_count(nd, lib)):
            b = Batch(len(ps), stream=stream)
            b.set_tile(nd, v)
            slots = [b.admit(g) for g in grids]
            b.step(warmup, graph=False)
            b.sync()
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record(stream)
            b.step(steps, graph=False)
            t1.record(stream)
            b.sync()
            times[v] = t0.elapsed_time(t1) / steps
            for s in slots:
                b.retire(s)
            del b
            if log:
                log(f"[autotune] batch of {len(ps)} {nd}-D grids, {prec}, tile {ppml_tile_shape(nd, v, lib)}: "
                    f"{times[v]:.4f} ms/step")
        best = pick(times)
        out[nd] = {"tile": best, "shape": ppml_tile_shape(nd, best, lib), "ms_per_step": times}
        del grids
    _cache[key] = out
    return out
