"""Serving loop: scheduler logic on the CPU with a fake batch that steps the
oracle, and on the GPU the alone-vs-mix equality of every served result."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1607_01105_amd import workloads as W


class _FakeGrid:
    def __init__(self, prob):
        self.prob = prob
        self.o = oracle.Oracle(prob.ndim, prob.n, prob.lo, prob.hi, prob.gamma, prob.cfl, bc=prob.bc)
        self.o.set_primitive(prob.rho, prob.vx, prob.vy, prob.vz, prob.p)
        self.taken = 0

    def get(self, f):
        return self.o.get(f)


class _FakeBatch:
    """Stands in for the GPU batch: same calls, steps the CPU oracle; records
    the admission order and the memory in use."""

    def __init__(self, capacity, budget, lib):
        self.capacity, self.budget, self.lib = capacity, budget, lib
        self.grids, self.order, self.max_in_use, self.in_use = {}, [], 0, 0

    def new_grid(self, prob, prec="fp32", stream=None):
        return _FakeGrid(prob)

    def side_stream(self):
        return None

    def _bytes(self, g):
        from paper_1607_01105_amd.ppml import make_desc, ppml_scratch_bytes, ppml_state_bytes

        p = g.prob
        d = make_desc(p.ndim, p.n[:p.ndim], (0.0,) * p.ndim, (1.0,) * p.ndim, 5.0 / 3.0, 0.3, prec="fp32")
        return ppml_state_bytes(d, self.lib) + ppml_scratch_bytes(d, self.lib)

    def admit(self, g):
        assert len(self.grids) < self.capacity
        s = min(set(range(self.capacity)) - set(self.grids))
        self.grids[s] = g
        self.order.append(g.prob.name)
        self.in_use += self._bytes(g)
        self.max_in_use = max(self.max_in_use, self.in_use)
        assert self.in_use <= self.budget
        return s

    def retire(self, s):
        g = self.grids.pop(s)
        self.in_use -= self._bytes(g)
        return g

    def step(self, nsteps, steps, graph=False):
        for s, k in steps.items():
            g = self.grids[s]
            g.o.run(k)
            g.taken += k

    def sync(self):
        pass


def _small_trace(n=14, seed=5, rate=400.0):
    return W.served_trace(seed, n, rate, n2_range=(12, 40), n3_range=(6, 12), steps_range=(3, 25))


def test_scheduler_logic_cpu():
    """Every request completes with exactly its steps, admission is FIFO and
    never exceeds the budget, and each result equals the request run alone."""
    from paper_1607_01105_amd import ppml
    from paper_1607_01105_amd.serve import Server

    lib = ppml.load()
    trace = _small_trace()
    budget = 6 * 12 ** 3 * 4 * 2 + 200000  # a few of the largest grids at once
    fake = _FakeBatch(capacity=5, budget=budget, lib=lib)
    srv = Server(budget_bytes=budget, capacity=5, round_steps=7, keep_results=True, batch=fake, prep_workers=2)
    st = srv.run(trace, time_scale=0.0)
    assert st["requests"] == len(trace)
    assert fake.order == [r.problem().name for r in sorted(trace, key=lambda r: r.arrival)]
    assert fake.max_in_use <= budget
    assert st["latency_p99_s"] >= st["latency_p50_s"] > 0.0
    for r in trace[:6]:
        o = oracle.Oracle(r.ndim, (r.n,) * r.ndim, (0.0,) * r.ndim, (1.0,) * r.ndim, 5.0 / 3.0, 0.3, bc="periodic")
        p = r.problem()
        o.set_primitive(p.rho, p.vx, p.vy, p.vz, p.p)
        o.run(r.steps)
        assert np.array_equal(srv.results[r.rid], o.get("rho")), r.rid


def test_round_does_not_wait_for_data_still_being_generated_cpu():
    """A request whose initial data are still being generated joins a later
    round: the requests that are ready are stepped meanwhile, and admission
    stays first come, first served."""
    import dataclasses
    import threading

    from paper_1607_01105_amd import ppml
    from paper_1607_01105_amd.serve import Server

    release = threading.Event()

    @dataclasses.dataclass
    class SlowRequest(W.Request):
        def problem(self):
            release.wait(timeout=60)
            return super().problem()

    fast, second = _small_trace(n=2, seed=7)
    slow = SlowRequest(**dataclasses.asdict(second))
    lib = ppml.load()
    fake = _FakeBatch(capacity=4, budget=1 << 30, lib=lib)
    resident = []
    step = fake.step

    def step_and_release(nsteps, steps, graph=False):
        resident.append(len(fake.grids))
        step(nsteps, steps, graph)
        release.set()  # the slow request's data arrive once a round has run

    fake.step = step_and_release
    srv = Server(budget_bytes=1 << 30, capacity=4, round_steps=2, keep_results=True, batch=fake, prep_workers=2)
    st = srv.run([fast, slow], time_scale=0.0)
    assert st["requests"] == 2
    assert resident[0] == 1  # the first round ran the ready request alone
    assert fake.order == [fast.problem().name, slow.problem().name]
    for r in (fast, slow):
        o = oracle.Oracle(r.ndim, (r.n,) * r.ndim, (0.0,) * r.ndim, (1.0,) * r.ndim, 5.0 / 3.0, 0.3, bc="periodic")
        p = r.problem()
        o.set_primitive(p.rho, p.vx, p.vy, p.vz, p.p)
        o.run(r.steps)
        assert np.array_equal(srv.results[r.rid], o.get("rho")), r.rid


@pytest.mark.gpu
def test_served_results_equal_alone_gpu():
    """GPU: requests served in a changing mix (budget forces queueing, rounds
    of 7 steps split runs) give the same bits as each request run alone."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_01105_amd.ppml import Grid
    from paper_1607_01105_amd.serve import Server

    trace = _small_trace(n=20, seed=9)
    srv = Server(budget_bytes=8 << 20, capacity=6, round_steps=7, keep_results=True)
    print("[case] served trace of 20 requests", flush=True)
    st = srv.run(trace, time_scale=0.0)
    assert st["requests"] == len(trace)
    for r in trace:
        g = Grid.from_problem(r.problem(), prec="fp32")
        g.step(r.steps)
        assert np.array_equal(srv.results[r.rid], g.get("rho")), r.rid
