"""Batched launches on the GPU (through the C ABI): many grids of uneven
sizes and dimensionalities stepped by the same kernels give, grid by grid,
the same bits as each grid stepped alone; the exact build equals the FP64
oracle; admission honours the memory budget and the capacity."""
from __future__ import annotations

import numpy as np
import pytest

from helpers import make_oracle
from paper_1607_01105_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _fields(ndim):
    return [0] + [1 + a for a in range(ndim)] + [4, 5]


def _mixed_problems():
    probs = W.batch_mix(seed=3, n1d=5, n2d=4, n1_range=(64, 700), n2_range=(20, 70))
    probs += [W.blocks(3, (19, 13, 21), seed=31), W.random_smooth(3, (40, 9, 17), seed=32, bc="outflow"),
              W.blocks(2, (33, 17), seed=33, bc="reflect")]
    return probs


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("graph", [True, False])
def test_batch_equals_solo_bitwise(prec, graph):
    from paper_1607_01105_amd.ppml import Batch, Grid

    probs = _mixed_problems()
    steps = [7 + (3 * i) % 9 for i in range(len(probs))]  # uneven per-grid step counts
    nmax = max(steps)
    print(f"[case] batch of {len(probs)} grids prec={prec} graph={graph}", flush=True)
    b = Batch(capacity=32)
    slots = []
    for p in probs:
        slots.append(b.admit(b.new_grid(p, prec=prec)))
    b.step(nmax, {s: k for s, k in zip(slots, steps)}, graph=graph)
    b.sync()
    for p, s, k in zip(probs, slots, steps):
        g = b.grids[s]
        solo = Grid.from_problem(p, prec=prec)
        solo.step(k)
        tb, db, nb = g.time()
        ts, ds, ns = solo.time()
        assert nb == ns == k and tb == ts and db == ds, (p.name, nb, ns, tb, ts)
        for f in _fields(p.ndim):
            assert np.array_equal(g.get(f), solo.get(f)), (p.name, f)


def test_batch_graph_replay_and_resume():
    """Graph replays in consecutive calls continue the run exactly like one
    eager call of the summed steps."""
    from paper_1607_01105_amd.ppml import Batch

    probs = _mixed_problems()[:6]
    a, b = Batch(capacity=8), Batch(capacity=8)
    for p in probs:
        a.admit(a.new_grid(p))
        b.admit(b.new_grid(p))
    for _ in range(3):
        a.step(5, graph=True)
    b.step(15, graph=False)
    a.sync()
    b.sync()
    for s in a.grids:
        ga, gb = a.grids[s], b.grids[s]
        assert ga.time() == gb.time()
        for f in _fields(ga.ndim):
            assert np.array_equal(ga.get(f), gb.get(f))


def test_exact_batch_equals_oracle():
    from paper_1607_01105_amd.ppml import Batch

    probs = _mixed_problems()[:7]
    b = Batch(capacity=8, exact=True)
    slots = [b.admit(b.new_grid(p, prec="fp64")) for p in probs]
    b.step(10, graph=True)
    b.sync()
    for p, s in zip(probs, slots):
        o = make_oracle(p)
        o.run(10)
        g = b.grids[s]
        assert g.time()[0] == o.t
        for f in _fields(p.ndim):
            assert np.array_equal(g.get(f), o.get(f)), (p.name, f)


def test_admission_budget_capacity_and_states():
    from paper_1607_01105_amd import ppml
    from paper_1607_01105_amd.ppml import Batch

    probs = [W.blocks(2, (40, 40), seed=40 + i) for i in range(4)]
    one = ppml.ppml_state_bytes(ppml.make_desc(2, (40, 40), (0, 0), (1, 1), 1.4, 0.4, prec="fp32")) + \
        ppml.ppml_scratch_bytes(ppml.make_desc(2, (40, 40), (0, 0), (1, 1), 1.4, 0.4, prec="fp32"))
    b = Batch(capacity=3, budget_bytes=2 * one)
    g0, g1, g2 = (b.new_grid(p) for p in probs[:3])
    s0 = b.admit(g0)
    b.admit(g1)
    with pytest.raises(ppml.PPMLError) as e:
        b.admit(g2)
    assert e.value.status == ppml.PPML_EBUDGET
    assert b.info() == (2, 2 * one)
    with pytest.raises(ppml.PPMLError) as e:
        g0.step(1)  # stepped only by its batch
    assert e.value.status == ppml.PPML_ESTATE
    r = b.retire(s0)
    assert r is g0
    b.admit(g2)  # the freed budget admits the next grid
    r.step(2)    # a retired grid steps on its own again
    r.sync()
    with pytest.raises(ppml.PPMLError) as e:
        b.admit(b.new_grid(W.blocks(2, (40, 40), seed=50), prec="fp64"))
    assert e.value.status in (ppml.PPML_EINVAL, ppml.PPML_EBUDGET)
    c = Batch(capacity=1)
    c.admit(c.new_grid(probs[3]))
    with pytest.raises(ppml.PPMLError) as e:
        c.admit(c.new_grid(probs[0]))
    assert e.value.status == ppml.PPML_EBUDGET
    with pytest.raises(ppml.PPMLError) as e:
        c.step(3, {0: 5})
    assert e.value.status == ppml.PPML_EINVAL


def test_reads_of_batched_grid_on_its_own_stream_wait_for_the_batch():
    """A grid created on a stream of its own and stepped by a batch on
    another stream: its read-back calls, issued right after the batch's
    launches with no explicit synchronisation, wait for the batch's work and
    return the stepped state (the bits of the same grid stepped alone)."""
    import torch

    from paper_1607_01105_amd.ppml import Batch, Grid

    prob = W.blocks(3, (64, 48, 40), seed=71)
    own = torch.cuda.Stream()
    g = Grid.from_problem(prob, prec="fp32", stream=own)
    b = Batch(capacity=2, stream=torch.cuda.Stream())
    b.admit(g)
    b.step(30, graph=False)
    got = [g.get(f) for f in _fields(3)]       # no b.sync() before the reads
    t = g.time()
    solo = Grid.from_problem(prob, prec="fp32")
    solo.step(30)
    for f, a in zip(_fields(3), got):
        assert np.array_equal(a, solo.get(f)), f
    assert t[2] == 30
