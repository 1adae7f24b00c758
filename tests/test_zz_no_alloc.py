"""The allocation-free entry point (ppml_step_noalloc) against the regular
one (ppml_create + ppml_step) through the C ABI: same kernels, so the same
bits, on two calls in a row that share the library's fixed work area, the
second on a smaller grid; and its rejection of grids whose work area does
not fit."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _pair(prob, prec, nsteps):
    """Step a grid with ppml_step; return it and a copy of its initial state."""
    import torch

    from paper_1607_01105_amd.ppml import Grid

    g = Grid.from_problem(prob, prec=prec)
    start = g.state.clone()
    g.step(nsteps)
    g.sync()
    torch.cuda.synchronize()
    return g, start


def _noalloc(g, state, nsteps):
    import torch

    from paper_1607_01105_amd import ppml

    stream = torch.cuda.current_stream().cuda_stream
    t, n = ppml.ppml_step_noalloc(g.desc, state.data_ptr(), nsteps, stream=stream, lib=g.lib)
    torch.cuda.synchronize()
    return t, n


def test_noalloc_equals_ppml_step_two_calls():
    import torch

    from paper_1607_01105_amd import workloads as W

    cases = [
        (W.blocks(3, (40, 36, 33), seed=3), "fp32", 7),   # 3-D, ragged tiles, several z chunks
        (W.blocks(2, (40, 24), seed=1), "fp64", 5),       # smaller, other precision and dimensionality
    ]
    for prob, prec, nsteps in cases:
        print(f"noalloc vs ppml_step: {prob.name} {prec} {nsteps} steps", flush=True)
        g, state = _pair(prob, prec, nsteps)
        t_ref, _, n_ref = g.time()
        t, n = _noalloc(g, state, nsteps)
        assert n == n_ref == nsteps
        assert t == t_ref
        assert torch.equal(state, g.state), f"{prob.name}: states differ"


def test_noalloc_fixed_step_and_t_stop():
    import torch

    from paper_1607_01105_amd import workloads as W

    prob = W.riemann_1d(4)
    from paper_1607_01105_amd.ppml import Grid

    g = Grid.from_problem(prob, prec="fp64")
    state = g.state.clone()
    g.step(40, 0.0, 0.05)
    g.sync()
    t_ref, _, n_ref = g.time()
    from paper_1607_01105_amd import ppml

    t, n = ppml.ppml_step_noalloc(g.desc, state.data_ptr(), 40, t_stop=0.05,
                                  stream=torch.cuda.current_stream().cuda_stream, lib=g.lib)
    torch.cuda.synchronize()
    assert (t, n) == (t_ref, n_ref)
    assert torch.equal(state, g.state)


def test_noalloc_rejects_oversized_grid():
    import torch

    from paper_1607_01105_amd import ppml

    lib = ppml.load()
    d = ppml.make_desc(3, (256, 256, 256), (0, 0, 0), (1, 1, 1), 5.0 / 3.0, 0.3, prec="fp32")
    buf = torch.empty(256, dtype=torch.uint8, device="cuda")
    with pytest.raises(ppml.PPMLError) as ei:
        ppml.ppml_step_noalloc(d, buf.data_ptr(), 1, lib=lib)
    assert ei.value.status == ppml.PPML_EINVAL
    assert b"work area" in lib.ppml_last_error()
