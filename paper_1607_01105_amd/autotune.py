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
per workload key within the process and persisted in a JSON file keyed by
the device (name, architecture, compute units), the library build (SHA-256
of the shared object) and the workload, so a later process on the same
device and build skips the search.

The timing runs advance the given state; callers re-set it afterwards.
"""
from __future__ import annotations

import collections
import hashlib
import json
import os

from .ppml import LIB_PATH, Batch, Grid, load, ppml_tile_count, ppml_tile_shape

_cache: dict = {}
_lib_sha: dict = {}


def cache_path() -> str | None:
    """The persisted results: $PPML_AUTOTUNE_CACHE, else
    $XDG_CACHE_HOME/ppml/autotune.json ($HOME/.cache when XDG_CACHE_HOME is
    unset).  An empty PPML_AUTOTUNE_CACHE turns persistence off."""
    p = os.environ.get("PPML_AUTOTUNE_CACHE")
    if p is not None:
        return p or None
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "ppml", "autotune.json")


def device_id() -> str:
    import torch

    pr = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{pr.name}|{getattr(pr, 'gcnArchName', '')}|{pr.multi_processor_count}"


def library_id(path: str = LIB_PATH) -> str:
    if path not in _lib_sha:
        h = hashlib.sha256()
        with open(path, "rb") as f:
            for chunk in iter(lambda: f.read(1 << 20), b""):
                h.update(chunk)
        _lib_sha[path] = h.hexdigest()
    return _lib_sha[path]


def _pkey(device: str, lib: str, key) -> str:
    return json.dumps([device, lib, list(key)], separators=(",", ":"))


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _decode(res):
    """JSON turns the integer tile indices of ms_per_step into strings."""
    def one(r):
        return {"tile": int(r["tile"]), "shape": tuple(r["shape"]),
                "ms_per_step": {int(k): float(v) for k, v in r["ms_per_step"].items()}}
    if "tile" in res:
        return one(res)
    return {int(nd): one(r) for nd, r in res.items()}


def persisted_get(key, device: str, lib: str, path: str | None):
    if not path:
        return None
    r = _load(path).get(_pkey(device, lib, key))
    try:
        return None if r is None else _decode(r)
    except (KeyError, TypeError, ValueError):
        return None


def persisted_put(key, res, device: str, lib: str, path: str | None) -> None:
    """Add one result to the file (read, update, write a temporary file and
    rename it over the old one, so a reader never sees a partial file)."""
    if not path:
        return
    d = _load(path)
    d[_pkey(device, lib, key)] = res
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(d, f)
    os.replace(tmp, path)


def _lookup(key):
    if key in _cache:
        return _cache[key]
    try:
        r = persisted_get(key, device_id(), library_id(), cache_path())
    except OSError:
        r = None
    if r is not None:
        _cache[key] = r
    return r


def _remember(key, res) -> None:
    _cache[key] = res
    try:
        persisted_put(key, res, device_id(), library_id(), cache_path())
    except OSError:
        pass  # a read-only cache location only costs the search next time


def pick(times: dict) -> int:
    """The fastest shape; a tie goes to the lower index (the default first)."""
    return min(sorted(times), key=lambda v: (times[v], v))


def tune_grid(prob, prec="fp32", steps=8, warmup=2, log=None) -> dict:
    """Best tile shape for stepping this problem alone (solo launches).

    Returns {"tile": index, "shape": (tx, ty), "ms_per_step": {index: ms}}."""
    # the workload's name as well: its force terms select other kernel
    # instantiations than a plain grid of the same size
    key = ("grid", prob.name, prob.ndim, tuple(prob.n[:prob.ndim]), prec)
    hit = _lookup(key)
    if hit is not None:
        return hit
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
    _remember(key, res)
    return res


def tune_batch(probs, prec="fp32", steps=10, warmup=2, log=None) -> dict:
    """Best tile shape per dimensionality for a batch of these problems.

    The grids of each dimensionality are stepped together, alone in a batch,
    once per shape (eager launches timed with HIP events on the batch
    stream).  Returns {ndim: {"tile": index, "shape": (tx, ty),
    "ms_per_step": {index: ms}}}."""
    import torch

    key = ("batch", prec, tuple(sorted((p.ndim, tuple(p.n[:p.ndim])) for p in probs)))
    hit = _lookup(key)
    if hit is not None:
        return hit
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
    _remember(key, out)
    return out
