"""Long ppml_step calls of a solo grid replay a captured chunk of steps (a HIP
graph, launched on the grid's own stream, the null stream included).  The
replayed steps run the same kernels as single steps, so the results are the
same bits: checked against one-step calls and against the oracle (exact
build), over several replays with eager work and synchronisation between
them, with run limits (t_stop, dt_fixed), on the null stream and on a
stream of its own."""
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


def _state(g, ndim):
    return [g.get(f) for f in _fields(ndim)] + [np.array(g.time())]


def _same(a, b, tag):
    for i, (x, y) in enumerate(zip(a, b)):
        assert np.array_equal(x, y), (tag, i, int(np.sum(x != y)))


def _single_steps(prob, prec, exact, n, **kw):
    from paper_1607_01105_amd.ppml import Grid

    g = Grid.from_problem(prob, prec=prec, exact=exact)
    for _ in range(n):
        g.step(1, **kw)
    return g


@pytest.mark.parametrize("prec,exact", [("fp64", True), ("fp32", False)], ids=["exact_fp64", "fp32"])
@pytest.mark.parametrize("name,prob", [("riemann_1d", W.riemann_1d(3)),
                                       ("blocks_2d", W.blocks(2, (45, 37), seed=8, bc="reflect")),
                                       ("modes_3d", W.periodic_modes(24, seed=2))],
                         ids=["1d", "2d", "3d"])
def test_replayed_chunks_equal_single_steps(name, prob, prec, exact):
    from paper_1607_01105_amd.ppml import Grid

    print(f"[case] {name} {prec} exact={exact}: 2 x 45 steps in calls vs 90 single steps", flush=True)
    g = Grid.from_problem(prob, prec=prec, exact=exact)
    g.step(45)                    # one replay of the chunk + 13 single launches
    mid = _state(g, prob.ndim)    # eager read-back and synchronisation between replays
    g.step(45)
    ref = _single_steps(prob, prec, exact, 90)
    _same(_state(g, prob.ndim), _state(ref, prob.ndim), name)
    ref45 = _single_steps(prob, prec, exact, 45)
    _same(mid, _state(ref45, prob.ndim), name + " after the first call")


def test_replayed_chunks_equal_the_oracle():
    """Exact build, 1-D Riemann problem run to t_stop in calls of 64 steps
    (the steps after t_stop are no-ops): the oracle's bits and step count."""
    from paper_1607_01105_amd.ppml import Grid

    prob = W.riemann_1d(5)
    print("[case] riemann_1d seed 5 to t_stop, exact fp64, calls of 64", flush=True)
    g = Grid.from_problem(prob, prec="fp64", exact=True)
    t, _, steps = g.run_to(prob.t_stop, chunk=64)
    o = make_oracle(prob)
    taus = o.run(10 ** 6, t_stop=prob.t_stop)
    assert t == o.t and steps == len(taus), (t, o.t, steps, len(taus))
    for f in _fields(1):
        assert np.array_equal(g.get(f), o.get(f)), f


def test_fixed_dt_and_own_stream():
    """dt_fixed steps on a grid of its own stream: replays equal single steps,
    and a second grid's eager work on the null stream between the replays
    does not disturb them."""
    import torch

    from paper_1607_01105_amd.ppml import Grid

    prob = W.periodic_modes(20, seed=4)
    s = torch.cuda.Stream()
    print("[case] 20^3 fp64 exact, dt_fixed 1e-4, own stream, 3 x 40 steps", flush=True)
    g = Grid.from_problem(prob, prec="fp64", exact=True, stream=s)
    other = Grid.from_problem(W.riemann_1d(1), prec="fp64")
    for _ in range(3):
        g.step(40, dt_fixed=1e-4)
        other.step(3)
        other.get("rho")
    ref = _single_steps(prob, "fp64", True, 120, dt_fixed=1e-4)
    _same(_state(g, 3), _state(ref, 3), "own stream")
    t, dt, n = g.time()
    assert n == 120 and abs(t - 120 * 1e-4) < 1e-15 and dt == 1e-4
