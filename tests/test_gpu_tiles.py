"""Work-group tile shapes and the autotuner on the GPU (through the C ABI):
every tile shape of the stage kernels gives the same bits, alone and in a
batch, in the FP64 operation-exact build and in the FP32 product build; the
tuner returns one of the offered shapes."""
from __future__ import annotations

import numpy as np
import pytest

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


def _problems():
    p3 = W.random_smooth(3, (70, 20, 26), seed=41)
    p3.bc = [("reflect", "outflow"), ("periodic", "periodic"), ("outflow", "reflect")]
    p2 = W.blocks(2, (75, 37), seed=42, bc="reflect")
    p1 = W.riemann_1d(7)
    p4 = W.blocks(3, (37, 21, 19), seed=44)
    p4.bc = [("inflow", "outflow"), ("reflect", "inflow"), ("inflow", "reflect")]
    p4.inflow = {0: (1.4, 2.5, 0.3, -0.2, 1.0), 3: (0.8, 0.1, -1.5, 0.4, 0.6), 4: (1.1, -0.3, 0.2, 1.8, 0.9)}
    return [("1d", p1), ("2d", p2), ("3d", p3), ("3d_inflow", p4)]


@pytest.mark.parametrize("exact,prec", [(True, "fp64"), (False, "fp32")], ids=["exact_fp64", "fp32"])
@pytest.mark.parametrize("name,prob", _problems(), ids=[n for n, _ in _problems()])
def test_every_tile_shape_gives_the_same_bits(name, prob, exact, prec):
    from paper_1607_01105_amd.ppml import Grid, ppml_tile_count

    ref = None
    for v in range(ppml_tile_count(prob.ndim)):
        print(f"[case] {name} {prec} exact={exact} tile={v}", flush=True)
        g = Grid.from_problem(prob, prec=prec, exact=exact, tile=v)
        g.step(9)
        out = [g.get(f) for f in _fields(prob.ndim)] + [np.array(g.time()[:2])]
        if ref is None:
            ref = out
        else:
            for a, b in zip(out, ref):
                assert np.array_equal(a, b), (name, v)


@pytest.mark.parametrize("exact", [True, False], ids=["exact", "product"])
def test_fp64_two_pass_tiles_bitwise_64cube(exact):
    """FP64 Lagrangian kernels take the fields in two LDS passes; every shape
    (including 2-wave work groups) and z chunks of several planes give the
    default shape's bits on the 64^3 box with its pressure sphere."""
    from paper_1607_01105_amd.ppml import Grid, ppml_tile_count

    prob = W.periodic_modes(64, seed=0)
    ref = None
    for v in range(ppml_tile_count(3)):
        print(f"[case] 64^3 fp64 exact={exact} tile={v}", flush=True)
        g = Grid.from_problem(prob, prec="fp64", exact=exact, tile=v)
        g.step(3)
        out = [g.get(f) for f in _fields(3)]
        if ref is None:
            ref = out
        for a, b in zip(out, ref):
            assert np.array_equal(a, b), v


def test_batch_with_tuned_shapes_equals_solo():
    """Batch launches with a non-default shape per dimensionality give the
    bits of the default solo launches."""
    from paper_1607_01105_amd.ppml import Batch, Grid, ppml_tile_count

    probs = [p for _, p in _problems()] + [W.blocks(3, (19, 13, 21), seed=43)]
    b = Batch(capacity=8)
    for nd in (1, 2, 3):
        b.set_tile(nd, ppml_tile_count(nd) - 1)
    slots = [b.admit(b.new_grid(p, prec="fp32")) for p in probs]
    print("[case] batch with the last tile shape of each dimensionality", flush=True)
    b.step(6, graph=True)
    b.sync()
    for p, s in zip(probs, slots):
        solo = Grid.from_problem(p, prec="fp32")
        solo.step(6)
        for f in _fields(p.ndim):
            assert np.array_equal(b.grids[s].get(f), solo.get(f)), (p.name, f)
    # the shape cannot change while grids of that dimensionality are admitted
    from paper_1607_01105_amd.ppml import PPMLError

    with pytest.raises(PPMLError):
        b.set_tile(3, 0)


def test_autotuner_returns_an_offered_shape():
    from paper_1607_01105_amd import autotune
    from paper_1607_01105_amd.ppml import ppml_tile_count, ppml_tile_shape

    prob = W.periodic_modes(40, seed=1)
    print("[case] tune_grid 40^3 fp32", flush=True)
    r = autotune.tune_grid(prob, prec="fp32", steps=3, warmup=1)
    assert 0 <= r["tile"] < ppml_tile_count(3)
    assert r["shape"] == ppml_tile_shape(3, r["tile"])
    assert set(r["ms_per_step"]) == set(range(ppml_tile_count(3)))
    assert all(t > 0 for t in r["ms_per_step"].values())
    probs = W.batch_mix(seed=5, n1d=3, n2d=3, n1_range=(64, 300), n2_range=(20, 60))
    print("[case] tune_batch 3 1-D + 3 2-D", flush=True)
    rb = autotune.tune_batch(probs, prec="fp32", steps=3, warmup=1)
    assert set(rb) == {1, 2}
    for nd, r in rb.items():
        assert 0 <= r["tile"] < ppml_tile_count(nd)
