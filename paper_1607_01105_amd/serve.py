"""Serving loop: continuous batching of simulation requests on one GPU.

Requests of a served trace arrive on a Poisson clock.  Each scheduler round

1. admits the grids prepared during the previous round into the batch;
2. enqueues the advance of every admitted grid by min(its remaining steps,
   round_steps) in one batched launch sequence, replayed as a captured HIP
   graph (captured again when the batch's grids change; every grid keeps its
   own CFL time step);
3. while the GPU runs that round, prepares arrived requests, oldest first,
   while the memory budget (state + scratch of the admitted and prepared
   grids) and the batch capacity allow: the request's initial state is
   copied to new device buffers on a second stream, so the copies and the
   state conversion overlap the batch's kernels; a request whose initial
   data are still being generated joins a later round unless nothing else
   could run, so the GPU starts on what is ready;
4. waits for the round and retires grids whose steps are done; their final
   states are copied to the host while the next round runs (before that
   round's admissions are prepared), the completion latency (arrival -> final
   state on the host) is recorded and their memory is released.

Requests that arrive while others are on the GPU join at the next round
boundary, so new work overlaps the running work on the device.  The
per-grid results do not depend on the mix (each grid's arithmetic and time
step use only its own data), which the tests check bit for bit.

The initial data of a request are produced by a small host thread pool ahead
of the request's arrival (a client would send them with the request); time a
request waits for its data after its arrival is counted in its latency and
reported separately.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import time

import numpy as np


@dataclasses.dataclass
class Completed:
    rid: int
    ndim: int
    n: int
    steps: int
    arrival: float
    admitted: float
    done: float
    data_wait: float
    rho_checksum: float

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Server:
    """Continuous-batching server over the batch API of the HIP library."""

    def __init__(self, budget_bytes: int = 4 << 30, capacity: int = 256, prec: str = "fp32", round_steps: int = 50,
                 graph: bool = True, device: str = "cuda", prep_workers: int = 8, lookahead: int = 16,
                 keep_results: bool = False, batch=None, tiles: dict | None = None):
        from .ppml import Batch

        self.prec = prec
        self.round_steps = int(round_steps)
        self.graph = graph
        self.budget = int(budget_bytes)
        self.batch = batch if batch is not None else Batch(capacity, budget_bytes, device)
        for nd, v in (tiles or {}).items():  # tile shape per dimensionality (autotune.tune_batch)
            self.batch.set_tile(nd, v)
        self.capacity = capacity
        self.prep_workers = prep_workers
        self.lookahead = lookahead
        self.keep_results = keep_results
        self.results: dict[int, np.ndarray] = {}

    def _grid_bytes(self, req) -> int:
        from .ppml import make_desc, ppml_scratch_bytes, ppml_state_bytes

        d = make_desc(req.ndim, (req.n,) * req.ndim, (0.0,) * req.ndim, (1.0,) * req.ndim, 5.0 / 3.0, 0.3,
                      prec=self.prec)
        return ppml_state_bytes(d, self.batch.lib) + ppml_scratch_bytes(d, self.batch.lib)

    def run(self, trace, time_scale: float = 1.0, log=None) -> dict:
        """Serve the requests of `trace` (workloads.served_trace) in real time;
        arrival times are multiplied by time_scale."""
        side = self.batch.side_stream()  # admissions are prepared here
        reqs = sorted(trace, key=lambda r: r.arrival)
        for r in reqs:
            if self._grid_bytes(r) > self.budget:
                raise ValueError(f"request {r.rid} needs more memory than the whole budget")
        pool = cf.ThreadPoolExecutor(max_workers=self.prep_workers)
        futures: dict[int, cf.Future] = {}
        nxt = 0  # next request whose data are not yet submitted
        pending = collections.deque(reqs)
        waiting: collections.deque = collections.deque()
        prepared: collections.deque = collections.deque()  # (request, grid, bytes, data wait)
        active: dict[int, list] = {}
        done: list[Completed] = []
        in_use = 0
        zu_done = 0
        rounds = 0
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0  # noqa: E731

        def prefetch():
            nonlocal nxt
            while nxt < len(reqs) and nxt < (len(done) + len(active) + self.lookahead):
                r = reqs[nxt]
                futures[r.rid] = pool.submit(r.problem)
                nxt += 1

        def arrivals():
            now = clock()
            while pending and pending[0].arrival * time_scale <= now:
                waiting.append(pending.popleft())

        def prepare():
            # FIFO while budget and capacity allow: state set on the side
            # stream (the call returns once the state is on the device).  A
            # request whose fields are still being generated waits for a later
            # round unless nothing else could run, so the GPU starts on what
            # is ready instead of idling until the budget is filled.
            nonlocal in_use
            while waiting and len(active) + len(prepared) < self.capacity:
                r = waiting[0]
                need = self._grid_bytes(r)
                if in_use + need > self.budget:
                    break
                fut = futures.get(r.rid)
                if fut is not None and not fut.done() and (prepared or active):
                    break
                t_req = clock()
                futures.pop(r.rid, None)
                prob = fut.result() if fut is not None else r.problem()
                data_wait = max(0.0, clock() - max(t_req, r.arrival * time_scale))
                g = self.batch.new_grid(prob, prec=self.prec, stream=side)
                in_use += need
                prepared.append((r, g, need, data_wait))
                waiting.popleft()
                prefetch()

        finished: list = []  # retired grids whose final state is still on the device

        def read_back():
            # final states of the retired grids (on their own streams, so the
            # copies overlap a round that is already running); their memory
            # returns to the budget afterwards
            nonlocal in_use, zu_done
            for a in finished:
                r, g = a[0], a[1]
                rho = g.get("rho")
                t_done = clock()
                if self.keep_results:
                    self.results[r.rid] = rho
                done.append(Completed(r.rid, r.ndim, r.n, r.steps, r.arrival * time_scale, a[3], t_done, a[4],
                                      float(np.sum(rho))))
                zu_done += r.cells * r.steps
                in_use -= a[5]
                if log:
                    log(f"[serve] done rid={r.rid} {r.ndim}d n={r.n} steps={r.steps} "
                        f"latency={t_done - r.arrival * time_scale:.3f}s active={len(active)}")
            finished.clear()

        try:
            while pending or waiting or prepared or active or finished:
                prefetch()
                arrivals()
                while prepared:
                    r, g, need, data_wait = prepared.popleft()
                    slot = self.batch.admit(g)
                    active[slot] = [r, g, r.steps, clock(), data_wait, need]
                if not active:
                    read_back()
                    prepare()
                    if not prepared and pending:
                        time.sleep(max(0.0, min(pending[0].arrival * time_scale - clock(), 0.05)))
                    continue
                steps = {s: min(a[2], self.round_steps) for s, a in active.items()}
                self.batch.step(max(steps.values()), steps, graph=self.graph)
                # the round runs on the GPU meanwhile: results of the previous
                # round, then the next admissions
                read_back()
                arrivals()
                prepare()
                self.batch.sync()
                rounds += 1
                for s in list(active):
                    a = active[s]
                    a[2] -= steps[s]
                    if a[2] > 0:
                        continue
                    self.batch.retire(s)
                    finished.append(a)
                    del active[s]
        finally:
            pool.shutdown(wait=True)
        t_end = clock()
        lat = np.array([c.latency for c in done])
        first = min(c.arrival for c in done)
        return {
            "requests": len(done),
            "rounds": rounds,
            "wall_s": t_end - first,
            "zone_updates": zu_done,
            "zone_updates_per_s": zu_done / (t_end - first),
            "latency_p50_s": float(np.percentile(lat, 50)),
            "latency_p99_s": float(np.percentile(lat, 99)),
            "latency_mean_s": float(lat.mean()),
            "data_wait_mean_s": float(np.mean([c.data_wait for c in done])),
            "completed": done,
        }


def measure_capacity(n_requests=300, seed=1000, budget_bytes=4 << 30, round_steps=50, tiles=None, log=None) -> float:
    """Saturated throughput of the server (zone-updates/s): every request of
    a trace is present at time zero, so the batch is always full."""
    from . import workloads as W

    trace = W.served_trace(seed, n_requests, 1.0)
    srv = Server(budget_bytes=budget_bytes, capacity=256, round_steps=round_steps, tiles=tiles,
                 prep_workers=16, lookahead=64)
    st = srv.run(trace, time_scale=0.0, log=log)
    return st["zone_updates_per_s"]


def main(argv=None):
    """Served runs at several loads: python -m paper_1607_01105_amd.serve."""
    import argparse
    import json
    import sys

    import torch

    from . import autotune
    from . import workloads as W

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--loads", default="0.25,0.5,0.8", help="arrival rates as fractions of the saturated capacity")
    ap.add_argument("--budget-gib", type=float, default=4.0)
    ap.add_argument("--round-steps", type=int, default=50)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--capacity-requests", type=int, default=300)
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    budget = int(a.budget_gib * (1 << 30))
    sample = [r.problem() for r in W.served_trace(a.seed + 1, 6, 1.0, n2_range=(64, 256), n3_range=(64, 96))]
    tiles = {nd: r["tile"] for nd, r in autotune.tune_batch(sample, prec="fp32", steps=4, log=log).items()}
    cap = measure_capacity(a.capacity_requests, seed=a.seed + 1000, budget_bytes=budget, round_steps=a.round_steps,
                           tiles=tiles, log=log)
    probe = W.served_trace(a.seed, 4000, 1.0)
    mean_zu = sum(r.cells * r.steps for r in probe) / len(probe)
    log(f"[serve] saturated capacity {cap:.3e} zone-updates/s; mean work {mean_zu:.3e} zone-updates per request")
    for load in [float(x) for x in a.loads.split(",")]:
        rate = load * cap / mean_zu
        trace = W.served_trace(a.seed, a.requests, rate)
        log(f"[serve] load {load:.2f}: {a.requests} requests at {rate:.2f}/s")
        srv = Server(budget_bytes=budget, capacity=256, round_steps=a.round_steps, tiles=tiles, prep_workers=16,
                     lookahead=64)
        st = srv.run(trace, log=log)  # one line per completed request
        out = {"load_vs_capacity": load, "rate_per_s": rate, "requests": st["requests"],
               "capacity_zone_updates_per_s": cap, "zone_updates_per_s": st["zone_updates_per_s"],
               "latency_p50_s": st["latency_p50_s"], "latency_p99_s": st["latency_p99_s"],
               "latency_mean_s": st["latency_mean_s"], "data_wait_mean_s": st["data_wait_mean_s"],
               "rounds": st["rounds"], "wall_s": st["wall_s"], "budget_GiB": a.budget_gib,
               "round_steps": a.round_steps, "tiles": {str(k): v for k, v in tiles.items()}}
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
