#!/usr/bin/env python3
"""Benchmark of the PPML hot path on one MI355X.

Workload (the headline configuration): 3-D 256^3 periodic unit cube,
gamma = 5/3, density = 1 + 0.1 * (sum of 8 seeded random-phase Fourier modes
with integer |k| <= 4), p = 1 with a p = 100 sphere of radius 0.1 at the
centre, u = 0, CFL 0.3, 100 steps.  FP32 state (FP64 totals and energy
recovery) is the headline value; the FP64 run is reported beside it with the
L1 distance of the two densities after the run.

A step is one full pass of the method: Eulerian kernel + Lagrangian kernel
(energy correction and CFL maxima fused).  The state is resident in HBM
when the timed region starts; the K timed steps start from the initial state
(the warm-up steps are discarded by re-setting it) and are bracketed by
device synchronisation and HIP events on the solver's stream.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
FP64_VECTOR_PEAK_TFLOPS = 78.6

WORKLOAD_STEPS = 100
WORKLOAD = ("3D 256^3 periodic unit cube, gamma 5/3, rho = 1 + 0.1 * 8 random modes (|k| <= 4), "
            f"p = 1 with p = 100 sphere r = 0.1 at centre, u = 0, CFL 0.3; a {WORKLOAD_STEPS}-step run "
            "(its first `steps` steps timed; accuracy after all of it)")


# Algorithmic floating-point operations per zone of each 3-D stage kernel,
# counted from the method (each add, sub, mul, div and sqrt of the formulas is
# one operation; interface quantities shared by two cells counted once;
# compares, min/max and selects not counted).  Eulerian: cell prep 7 +
# 3 axes x (2 parabolas 58 + Riemann 48 + differences 7) + update 16 = 362.
# Lagrangian: 3 axes x (velocity 1 + 9-point template 11 + interface velocity
# 5 + Courant number 2 + 6 fields x (parabola 29 + average 5 + flux 3) +
# shared average terms 4) + sqrt(rho) 1 + update 24 + energy correction 8 +
# CFL speeds 13 = 781.  Parabola 29 = limited slope 7 + interface value 5 +
# monotonisation 17.
ALGO_FLOP_PER_ZONE_3D = {"euler": 362, "lagr": 781}
# VALU peak of the kernels as built (packed FP32 instructions are disabled):
# 256 CU x 64 lanes x 2 FLOP (FMA) x 2.4 GHz = 78.6 TFLOP/s for FP32 and for
# FP64; the published FP32 figure (157.3) assumes packed FP32.
VALU_PEAK_TFLOPS = {"f32": 78.6, "f64": 78.6}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_box256.json")
KERNEL_SOURCES = ("paper_1607_01105_amd/csrc/ppml_kernels.hpp", "paper_1607_01105_amd/csrc/ppml_euler_plane.inc",
                  "paper_1607_01105_amd/csrc/ppml_lagr_plane.inc", "paper_1607_01105_amd/csrc/ppml_device.hpp",
                  "paper_1607_01105_amd/build.py")


def measured_counters(kernel_key: str):
    """The committed rocprofv3 counter summary of one kernel: HBM bytes per
    launch (FETCH_SIZE and WRITE_SIZE scaled by the calibration kernel) and
    VALU lane-instructions per zone (SQ_INSTS_VALU x 64 / zones), or None
    when the kernel sources changed since the counters were taken."""
    import hashlib

    try:
        tr = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, s), "rb").read())
    if tr.get("source_sha256") != h.hexdigest() or kernel_key not in tr:
        return None
    return tr[kernel_key]


def measured_traffic(kernel_key: str):
    c = measured_counters(kernel_key)
    return None if c is None else c["bytes"]


# VALU issue roof: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 3.93e13 lane-instructions/s
VALU_ISSUE_PEAK = 256 * 64 * 2.4e9


def algorithmic_bytes_per_zone(kernel: str, ndim: int, width: int) -> int:
    """Compulsory HBM bytes of one kernel per zone: the Eulerian kernel reads
    the F = 3 + ndim conserved fields and writes the F - 1 it changes (rho is
    unchanged); the Lagrangian kernel reads F fields and writes F."""
    F = 3 + ndim
    return (2 * F - 1) * width if kernel == "euler" else 2 * F * width


def run_precision(prob, prec, steps, warmup, tile=0):
    import torch

    from paper_1607_01105_amd.ppml import Grid

    g = Grid.from_problem(prob, prec=prec, device="cuda:0", tile=tile)
    if warmup > 0:
        g.step(warmup)
        g.sync()
        g.set_primitive(prob.rho, prob.vx, prob.vy, prob.vz, prob.p)
    g.set_timing(steps)
    stream = g.stream
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    g.step(steps)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    me, ml, nt = g.get_timing()
    g.sync()
    t, dt, taken = g.time()
    rho = g.get("rho")
    tot = g.totals()
    del g
    torch.cuda.empty_cache()
    return dict(ms=ms, ms_euler=me / max(nt, 1), ms_lagr=ml / max(nt, 1), timed_steps=nt, t=t, steps_taken=taken,
                rho=rho, totals=tot)


def run_batched(seed=0, steps=200, tune=True):
    """Batched configuration: 128 1-D Riemann problems (64-4096 cells) and
    128 2-D periodic boxes (sides 32-256), FP32, 200 steps each.  Plain
    per-grid launches against one batched launch sequence replayed from a HIP
    graph; the two give the same bits for every grid.  Both use the tile
    shape per dimensionality that the autotuner picks for the batch."""
    import numpy as np
    import torch

    from paper_1607_01105_amd import autotune
    from paper_1607_01105_amd import workloads as W
    from paper_1607_01105_amd.ppml import Batch, Grid

    probs = W.batch_mix(seed, steps=steps)
    cells = sum(p.cells for p in probs)
    tuned = autotune.tune_batch(probs, prec="fp32", log=_log) if tune else {}
    tiles = {nd: r["tile"] for nd, r in tuned.items()}
    stream = torch.cuda.Stream()
    plain = [Grid.from_problem(p, prec="fp32", stream=stream, tile=tiles.get(p.ndim, 0)) for p in probs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in plain:
        g.step(steps)
    for g in plain:
        g.sync()
    t_plain = time.perf_counter() - t0
    b = Batch(len(probs))
    for nd, v in tiles.items():
        b.set_tile(nd, v)
    slots = [b.admit(b.new_grid(p, prec="fp32")) for p in probs]
    t0 = time.perf_counter()
    b.step(steps, graph=True)  # records the graph, then replays it
    b.sync()
    t_first = time.perf_counter() - t0
    for p, s in zip(probs, slots):
        b.grids[s].set_primitive(p.rho, p.vx, p.vy, p.vz, p.p)
    b.sync()
    t0 = time.perf_counter()
    b.step(steps, graph=True)
    b.sync()
    t_batch = time.perf_counter() - t0
    same = all(np.array_equal(b.grids[s].get("rho"), g.get("rho")) for s, g in zip(slots, plain))
    return {"workload": "128 1-D Riemann (64-4096 cells) + 128 2-D periodic (sides 32-256), FP32, 200 steps each",
            "grids": len(probs), "cells": cells, "steps": steps,
            "plain_zone_updates_per_s": cells * steps / t_plain, "plain_s": t_plain,
            "batched_graph_zone_updates_per_s": cells * steps / t_batch, "batched_s": t_batch,
            "batched_first_call_s": t_first, "speedup": t_plain / t_batch, "bitwise_equal_to_plain": bool(same),
            "tile_shapes": {str(nd): list(r["shape"]) for nd, r in tuned.items()}}


def run_served(n_requests=400, loads=(0.5, 0.8), seed=0, budget_gib=4.0, round_steps=50, capacity_requests=150):
    """Served configuration: Poisson arrivals of 2-D (64^2-512^2) and 3-D
    (64^3-192^3) periodic boxes with a high-pressure sphere, 50-500 steps,
    FP32, admitted by an HBM budget.  The server's saturated throughput is
    measured first (every request of a trace of another seed present at time
    zero); then n_requests arrive at each load x that capacity (divided by
    the mean work per request) and p50/p99 completion latency is reported."""
    import numpy as np

    from paper_1607_01105_amd import autotune
    from paper_1607_01105_amd import workloads as W
    from paper_1607_01105_amd.serve import Server, measure_capacity

    budget = int(budget_gib * (1 << 30))
    # tile shapes for the mix, tuned on a few requests of another seed
    sample = [r.problem() for r in W.served_trace(seed + 1, 6, 1.0, n2_range=(64, 256), n3_range=(64, 96))]
    tiles = {nd: r["tile"] for nd, r in autotune.tune_batch(sample, prec="fp32", steps=4, log=_log).items()}
    cap = measure_capacity(capacity_requests, seed=seed + 1000, budget_bytes=budget, round_steps=round_steps,
                           tiles=tiles)
    _log(f"[bench] served saturation: {cap:.3e} zone-updates/s over {capacity_requests} requests")
    probe = W.served_trace(seed, 4000, 1.0)
    mean_zu = float(np.mean([r.cells * r.steps for r in probe]))
    out = {"workload": "Poisson arrivals, 50% 2-D 64^2-512^2 / 50% 3-D 64^3-192^3 periodic boxes with one "
                       "p=100 sphere, 50-500 steps, FP32",
           "budget_GiB": budget_gib, "round_steps": round_steps, "tiles": {str(a): v for a, v in tiles.items()},
           "saturated_zone_updates_per_s": cap, "saturation_requests": capacity_requests,
           "mean_zone_updates_per_request": mean_zu, "loads": {}}
    for load in loads:
        rate = load * cap / mean_zu
        trace = W.served_trace(seed, n_requests, rate)
        srv = Server(budget_bytes=budget, capacity=256, prec="fp32", round_steps=round_steps, tiles=tiles,
                     prep_workers=16, lookahead=64)
        st = srv.run(trace)
        _log(f"[bench] served load {load:.2f}: {st['requests']} requests at {rate:.2f}/s, p50 "
             f"{st['latency_p50_s']:.3f} s, p99 {st['latency_p99_s']:.3f} s")
        out["loads"][f"{load:.2f}"] = {
            "requests": st["requests"], "rate_per_s": rate, "latency_p50_s": st["latency_p50_s"],
            "latency_p99_s": st["latency_p99_s"], "latency_mean_s": st["latency_mean_s"],
            "zone_updates_per_s": st["zone_updates_per_s"], "rounds": st["rounds"],
            "data_wait_mean_s": st["data_wait_mean_s"]}
    return out


def run_disk(steps=500, isothermal=False):
    """Rotating-disk configuration: 512 x 512 x 64, logarithmic potential,
    outflow, CFL 0.2, 500 steps.  FP32 (the configuration's state) and FP64,
    each with its own CFL steps, with the L1 distance of the two densities.
    isothermal=True: the same disk in the isothermal variant (p = cs^2 rho,
    the paper's approximation for its disks)."""
    import numpy as np
    import torch

    from paper_1607_01105_amd import workloads as W
    from paper_1607_01105_amd.ppml import Grid

    prob = W.disk(nsteps=steps, isothermal=isothermal)
    kind = "isothermal (p = cs^2 rho, cs = 0.05)" if isothermal else "adiabatic (gamma = 5/3)"
    out = {"workload": f"rotating gas disk 512x512x64, {kind}, in a logarithmic potential, outflow, CFL 0.2, "
                       f"{steps} steps", "cells": prob.cells, "steps": steps}
    for prec in ("fp32", "fp64"):
        g = Grid.from_problem(prob, prec=prec)
        g.sync()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(g.stream)
        g.step(steps)
        t1.record(g.stream)
        g.sync()
        ms = t0.elapsed_time(t1)
        t, _, n = g.time()
        out[prec] = {"zone_updates_per_s": prob.cells * steps / (ms * 1e-3), "ms_per_step": ms / steps, "t": t}
        del g
        torch.cuda.empty_cache()
    # accuracy at equal times (untimed): FP64 with its CFL steps, one at a
    # time to record them, and FP32 driven by the same steps.  Beside it, the
    # floor of any FP32 state on this flow: an FP64 run whose density alone is
    # rounded to FP32 after every step (all arithmetic FP64), compared with
    # the plain FP64 run.
    n = prob.cells
    g64 = Grid.from_problem(prob, prec="fp64")
    g32 = Grid.from_problem(prob, prec="fp32")
    gr = Grid.from_problem(prob, prec="fp64")

    def rho_of(g):
        return g.state.view(torch.float64 if g.desc.prec == 1 else torch.float32)[:n].double()

    def l1(a, b):
        return float((a - b).abs().sum() / a.abs().sum())

    marks = {}
    for s in range(1, steps + 1):
        g64.step(1)
        tau = g64.time()[1]
        g32.step(1, dt_fixed=float(tau))
        gr.step(1, dt_fixed=float(tau))
        gr.sync()
        v = gr.state.view(torch.float64)
        v[:n] = v[:n].float().double()
        if s in (100, steps):
            g32.sync()
            marks[s] = (l1(rho_of(g64), rho_of(g32)), l1(rho_of(g64), rho_of(gr)))
    del g64, g32, gr
    torch.cuda.empty_cache()
    out["l1_rho_fp32_vs_fp64_same_steps"] = marks[steps][0]
    out["l1_rho_fp64_with_rho_rounded_to_fp32_each_step"] = marks[steps][1]
    if 100 in marks and steps != 100:
        out["l1_rho_fp32_vs_fp64_after_100_steps"] = marks[100][0]
        out["l1_rho_fp64_with_rho_rounded_after_100_steps"] = marks[100][1]
    return out


def run_riemann_1d(seeds=range(16)):
    """1-D Riemann configuration: 512 cells, FP64, 16 seeds, each run to
    t = 0.15 with its own CFL steps (latency-bound: two small launches per
    step)."""
    import torch

    from paper_1607_01105_amd import workloads as W
    from paper_1607_01105_amd.ppml import Grid

    import numpy as np

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import exact_riemann as er  # the exact solution, written from the mathematics

    zu, sec = 0, 0.0
    l1, l1x = [], []
    for s in seeds:
        prob = W.riemann_1d(s)
        g = Grid.from_problem(prob, prec="fp64")
        g.sync()
        t0 = time.perf_counter()
        _, _, n = g.run_to(prob.t_stop)
        sec += time.perf_counter() - t0
        zu += prob.cells * n
        left, right = W.riemann_states(s)
        ex = er.cell_averages(left, right, prob.gamma, 0.5, prob.t_stop, np.linspace(0.0, 1.0, 513), sub=8)
        l1.append(float(np.mean(np.abs(g.get("rho").ravel() - ex[0]))))
        del g
        # waves can reach x = 0 or 1 by t = 0.15: the same problem on [-1, 2]
        # (1536 cells), compared on [0, 1], leaves the outflow faces out
        big = W.riemann_1d(s, n=1536, lo=-1.0, hi=2.0)
        gb = Grid.from_problem(big, prec="fp64")
        gb.run_to(big.t_stop)
        l1x.append(float(np.mean(np.abs(gb.get("rho").ravel()[512:1024] - ex[0]))))
        del gb
    torch.cuda.empty_cache()
    return {"workload": "1-D Riemann, 512 cells, FP64, seeds 0-15, t = 0.15 (host-driven chunks of 64 steps)",
            "zone_updates_per_s": zu / sec, "zone_updates": zu, "seconds": sec,
            "l1_rho_vs_exact": {"mean": float(np.mean(l1)), "max": float(np.max(l1))},
            "l1_rho_vs_exact_extended_domain": {"mean": float(np.mean(l1x)), "max": float(np.max(l1x))}}


def run_suite():
    """The paper's test-suite workloads at their full sizes, each run to its
    stop time with CFL steps (host-driven chunks of 64 steps): two blast
    waves (1-D, 2400 cells, FP64, t = 0.038), Sedov (100^3, t = 0.05) and
    Kelvin-Helmholtz (256^2, t = 1) in FP32 and FP64; tile shapes from the
    autotuner; and Rayleigh-Taylor (100 x 600, t = 6) with the growth rate
    of its seeded mode."""
    import torch

    from paper_1607_01105_amd import autotune
    from paper_1607_01105_amd import workloads as W
    from paper_1607_01105_amd.ppml import Grid, ppml_tile_shape

    out = {}
    for name, prob, precs in (("blast_waves_2400", W.blast_waves(), ("fp64",)),
                              ("sedov_100", W.sedov(100), ("fp32", "fp64")),
                              ("kelvin_helmholtz_256", W.kelvin_helmholtz(256), ("fp32", "fp64")),
                              ("rayleigh_taylor_100x600", W.rayleigh_taylor(t_stop=6.0), ("fp32", "fp64"))):
        out[name] = {}
        for prec in precs:
            tile = autotune.tune_grid(prob, prec, steps=8, warmup=2)["tile"]
            g = Grid.from_problem(prob, prec=prec, tile=tile)
            g.sync()
            t0 = time.perf_counter()
            t, _, n = g.run_to(prob.t_stop)
            sec = time.perf_counter() - t0
            out[name][prec] = {"steps": n, "t": t, "zone_updates_per_s": prob.cells * n / sec, "seconds": sec,
                               "tile": list(ppml_tile_shape(prob.ndim, tile))}
            if name.startswith("rayleigh_taylor"):
                # growth of the seeded mode at the unstable interface over
                # t = 3 .. 6 (untimed rerun), against linear theory sqrt(A g k)
                import numpy as np

                k = 4.0 * math.pi
                x, y = prob.centres(0), prob.centres(1)
                sel = np.abs(y + 0.75) <= 0.25
                g2 = Grid.from_problem(prob, prec=prec, tile=tile)
                ts = np.arange(3.0, 6.01, 0.5)
                amp = []
                for tt in ts:
                    g2.run_to(float(tt))
                    vy = (g2.get("my") / g2.get("rho"))[0]
                    amp.append(2.0 * float(abs(np.mean(vy[sel] * np.cos(k * x)[None, :]))))
                out[name][prec]["growth_rate"] = float(np.polyfit(ts, np.log(amp), 1)[0])
                out[name][prec]["growth_rate_linear_theory"] = math.sqrt((1.0 / 3.0) * 0.1 * k)
                del g2
            del g
        torch.cuda.empty_cache()
    return out


# the relative errors of the Poisson solver that the paper prints (Sec. 2.5
# table, its own machine and code), quoted beside ours as context
PAPER_POISSON_ERR = {16: 4.799777e-05, 32: 2.978253e-06, 64: 1.862059e-07, 128: 1.164110e-08, 256: 7.278760e-10}


def run_gravity(n=256, steps=50):
    """Self-gravity (Sec. 2.5): the verification sphere's density as a
    collapsing gas ball, n^3 on [-2, 2]^3, outflow, CFL 0.3; FP32 and FP64,
    each with its own CFL steps: zone-updates/s of the whole step (potential
    solve + both stage kernels), the split per part, the transforms'
    algorithmic GEMM rate against the matrix-core peak, FP32 against FP64 in
    L1 after the run; and the Poisson verification table (the analytic
    potential's relative error on 16^3 ... 256^3, FP64)."""
    import math

    import numpy as np
    import torch

    from paper_1607_01105_amd import autotune
    from paper_1607_01105_amd import workloads as W
    from paper_1607_01105_amd.ppml import Grid, ppml_tile_shape

    prob = W.gravity_sphere(n, noise=0.01, seed=0)
    cells = prob.cells
    # sine transforms: 3 axes forward + 3 back, each 2 n_a FLOP per cell
    gemm_flop = 4.0 * cells * sum(prob.n)
    out = {"workload": f"self-gravitating ball {n}^3 on [-2,2]^3 (density 2r^3-3r^2+1 + 1e-3 floor, 1% noise), "
                       f"p = 0.05, outflow, CFL 0.3, {steps} steps", "cells": cells, "steps": steps}
    rho = {}
    for prec in ("fp32", "fp64"):
        # trials long enough to tell tile shapes within 10% of each other apart
        tile = autotune.tune_grid(prob, prec, steps=8, warmup=2)["tile"]
        g = Grid.from_problem(prob, prec=prec, tile=tile)
        g.step(2)
        g.sync()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(g.stream)
        g.step(steps)
        t1.record(g.stream)
        g.sync()
        ms = t0.elapsed_time(t1)
        rho[prec] = g.get("rho")
        g.set_timing(10)
        g.step(10)
        mg, me, ml, k = g.get_timing_split()
        peak = 157.3 if prec == "fp32" else 78.6
        out[prec] = {"zone_updates_per_s": cells * steps / (ms * 1e-3), "ms_per_step": ms / steps,
                     "tile": list(ppml_tile_shape(3, tile)),
                     "split_ms": {"gravity": mg / k, "euler": me / k, "lagr": ml / k},
                     "transforms": {"algorithmic_gemm_flop": gemm_flop, "achieved_TFLOPs_over_gravity_solve":
                                    gemm_flop / (mg / k * 1e-3) / 1e12, "mfma_peak_TFLOPs": peak}}
        _log(f"[bench] gravity {n}^3 {prec}: {out[prec]['ms_per_step']:.3f} ms/step, solve {mg / k:.3f} ms")
        del g
        torch.cuda.empty_cache()
    out["l1_rho_fp32_vs_fp64_own_steps"] = float(np.sum(np.abs(rho["fp32"] - rho["fp64"])) / np.sum(rho["fp64"]))
    table = {}
    for m in (16, 32, 64, 128, 256):
        sp = W.gravity_sphere(m, rho_floor=1e-12)
        g = Grid.from_problem(sp, prec="fp64")
        phi = g.potential()[1:-1, 1:-1, 1:-1]
        del g
        X, Y, Z = (sp.centres(a) for a in range(3))
        Zm, Ym, Xm = np.meshgrid(Z, Y, X, indexing="ij")
        r = np.sqrt(Xm ** 2 + Ym ** 2 + Zm ** 2)
        pi = math.pi
        ex = np.where(r <= 1.0, 4 * pi / 15 * r ** 5 - 3 * pi / 5 * r ** 4 + 2 * pi / 3 * r ** 2 - 3 * pi / 5,
                      -4 * pi / (15 * r))
        table[str(m)] = {"rel_err": float(np.max(np.abs(phi - ex)) / np.max(np.abs(ex))),
                         "paper_printed": PAPER_POISSON_ERR[m]}
    torch.cuda.empty_cache()
    out["poisson_sphere_table_fp64"] = table
    return out


def run_galaxy(steps=20, sizes=((256, ("fp32", "fp64")), (512, ("fp32",)))):
    """The paper's galactic-disk configuration with synthetic data (Sec. 4:
    isothermal gas, self-gravity, fixed halo potential, CFL 0.2), on 256^3
    (FP32 and FP64) and on the paper's 512^3 mesh (FP32): zone-updates/s of
    whole steps (potential solve + both stage kernels) and the split."""
    import torch

    from paper_1607_01105_amd import autotune
    from paper_1607_01105_amd import workloads as W
    from paper_1607_01105_amd.ppml import Grid, ppml_tile_shape

    out = {"workload": "isothermal self-gravitating disk (cs = 0.05, G = 1) in the paper's dark-matter halo "
                       "(density rho0 / (1 + (r/r0)^2) out to rh = 49.1 r0, r0 = 0.05), "
                       f"box [-1/2,1/2]^3, outflow, CFL 0.2, {steps} steps"}
    for n, precs in sizes:
        prob = W.galaxy_disk(n)
        out[str(n)] = {}
        for prec in precs:
            tile = autotune.tune_grid(prob, prec, steps=3, warmup=1)["tile"]
            g = Grid.from_problem(prob, prec=prec, tile=tile)
            g.step(2)
            g.sync()
            g.set_timing(steps)
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record(g.stream)
            g.step(steps)
            t1.record(g.stream)
            g.sync()
            ms = t0.elapsed_time(t1)
            mg, me, ml, k = g.get_timing_split()
            out[str(n)][prec] = {"zone_updates_per_s": prob.cells * steps / (ms * 1e-3), "ms_per_step": ms / steps,
                                 "tile": list(ppml_tile_shape(3, tile)),
                                 "split_ms": {"gravity": mg / k, "euler": me / k, "lagr": ml / k}}
            _log(f"[bench] galaxy {n}^3 {prec}: {ms / steps:.3f} ms/step (gravity {mg / k:.3f} ms)")
            del g
            torch.cuda.empty_cache()
        del prob
    return out


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(prob, steps=100):
    """The FP64 oracle, untuned, on this host's cores: the full workload
    (steps of the 256^3 box), timed around the step loop, then one step on a
    single core.  Returns the baseline and the oracle's time steps and final
    fields, against which the GPU runs are checked after the run."""
    import oracle

    o = oracle.Oracle(prob.ndim, prob.n, prob.lo, prob.hi, prob.gamma, prob.cfl, bc=prob.bc)
    o.set_primitive(prob.rho, prob.vx, prob.vy, prob.vz, prob.p)
    cores = oracle.max_threads()
    t0 = time.perf_counter()
    taus = [float(t) for t in o.run(steps)]
    sec = time.perf_counter() - t0
    final = [o.get(f) for f in range(6)]
    # one more step on one core (results are independent of the threads)
    oracle.set_threads(1)
    tau = o.dt()
    t0 = time.perf_counter()
    o.step(tau)
    sec1 = time.perf_counter() - t0
    oracle.set_threads(cores)
    del o
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    base = {"value": prob.cells * steps / sec, "unit": "zone-updates/s", "cores": cores, "kind": "oracle",
            "cpu_model": model, "nproc": os.cpu_count(),
            "sample": f"the full workload: {steps} steps of the 256^3 box ({prob.cells * steps} zone-updates), "
                      f"FP64, {sec:.1f} s of stepping on {cores} threads; then 1 step on 1 thread",
            "one_core_value": prob.cells / sec1}
    return base, taus, final


def parity_after_run(prob, taus, final):
    """GPU FP64 and FP32 runs of the whole workload driven by the oracle's
    time steps, compared with the oracle's final state: per field the
    normwise relative error max|a - b| / max|b| (FP64) and the L1 relative
    error of the density (FP32)."""
    import numpy as np
    import torch

    from paper_1607_01105_amd.ppml import Grid

    out = {"steps": len(taus), "against": "FP64 oracle, same time steps"}
    for prec in ("fp64", "fp32"):
        g = Grid.from_problem(prob, prec=prec)
        for tau in taus:
            g.step(1, dt_fixed=tau)
        g.sync()
        if prec == "fp64":
            out["fp64_normwise_rel_err_per_field"] = {
                name: float(np.max(np.abs(g.get(f) - final[f])) / max(np.max(np.abs(final[f])), 1e-300))
                for f, name in enumerate(("rho", "mx", "my", "mz", "Et", "e"))}
        else:
            r = g.get("rho")
            out["fp32_l1_rho"] = float(np.sum(np.abs(r - final[0])) / np.sum(np.abs(final[0])))
        del g
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only", choices=["fp32", "fp64"], default=None)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched and served runs")
    ap.add_argument("--serve-requests", type=int, default=400, help="requests per served load")
    ap.add_argument("--no-tune", action="store_true", help="use the default tile shape instead of the autotuner's")
    ap.add_argument("--leg", choices=["gravity", "galaxy", "disk", "disk_isothermal", "suite", "batched", "riemann_1d"],
                    default=None,
                    help="run only this configuration (its JSON object, no headline line); for profiling")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run one plain 256 MiB streaming kernel (torch.mul out-of-place: reads 256 MiB, "
                         "writes 256 MiB), the reference kernel for scaling the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU design is "
              "described in DESIGN.md and not run", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1607_01105_amd import workloads as W

    torch.cuda.set_device(0)
    if args.calib_copy:
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()
        del a, b
        print("[bench] calibration copy: 268435456 bytes read, 268435456 bytes written", file=sys.stderr, flush=True)
    if args.leg is not None:
        legs = {"gravity": lambda: run_gravity(steps=args.steps), "disk": lambda: run_disk(steps=args.steps),
                "disk_isothermal": lambda: run_disk(steps=args.steps, isothermal=True), "suite": run_suite,
                "batched": lambda: run_batched(steps=args.steps), "galaxy": lambda: run_galaxy(steps=args.steps),
                "riemann_1d": run_riemann_1d}
        print(json.dumps({args.leg: legs[args.leg]()}))
        return
    prob = W.periodic_modes(args.n, seed=0)
    cells = prob.cells
    res = {}
    for prec in ("fp32", "fp64"):
        if args.only and prec != args.only:
            continue
        tile, tuned = 0, None
        if not args.no_tune:
            from paper_1607_01105_amd import autotune

            tuned = autotune.tune_grid(prob, prec, steps=5, warmup=1, log=_log)
            tile = tuned["tile"]
        print(f"[bench] {prec} {args.n}^3 steps={args.steps} warmup={args.warmup} tile={tile}", file=sys.stderr,
              flush=True)
        res[prec] = run_precision(prob, prec, args.steps, args.warmup, tile)
        res[prec]["tuned"] = tuned
        r = res[prec]
        print(f"[bench] {prec}: {r['ms'] / args.steps:.3f} ms/step, euler {r['ms_euler']:.3f} ms, "
              f"lagr {r['ms_lagr']:.3f} ms, {cells * args.steps / (r['ms'] * 1e-3):.3e} zu/s",
              file=sys.stderr, flush=True)

    head = "fp32" if "fp32" in res else "fp64"
    r = res[head]
    value = cells * args.steps / (r["ms"] * 1e-3)
    width = 4 if head == "fp32" else 8
    # dominant kernel; the path is bound by the vector ALUs (see the design
    # notes): algorithmic FLOPs per launch / measured launch duration
    kern = "lagr" if r["ms_lagr"] >= r["ms_euler"] else "euler"
    ms_k = r["ms_" + kern]
    dt = "f32" if head == "fp32" else "f64"
    flops_launch = ALGO_FLOP_PER_ZONE_3D[kern] * cells
    achieved_tflops = flops_launch / (ms_k * 1e-3) / 1e12
    bytes_launch = algorithmic_bytes_per_zone(kern, 3, width) * cells
    achieved_gbs = bytes_launch / (ms_k * 1e-3) / 1e9
    from paper_1607_01105_amd.ppml import ppml_tile_shape

    tx, ty = ppml_tile_shape(3, r["tuned"]["tile"] if r["tuned"] else 0)
    key = f"k_{kern}<{'float' if width == 4 else 'double'},3,{tx},{ty}" + (
        f",{6 if width == 4 else 3}>" if kern == "lagr" else ">")
    traffic = measured_traffic(key)
    cnt = measured_counters(key)
    valu_issue = None
    if cnt and "valu_lane_instr_per_zone" in cnt:
        # every lane-instruction the kernel issues (address arithmetic,
        # selects and moves included) against the VALU issue rate
        ach = cnt["valu_lane_instr_per_zone"] * cells / (ms_k * 1e-3)
        valu_issue = {"lane_instr_per_zone": cnt["valu_lane_instr_per_zone"], "achieved": ach,
                      "peak": VALU_ISSUE_PEAK, "unit": "lane-instr/s", "frac": ach / VALU_ISSUE_PEAK,
                      "valu_busy_pct": cnt.get("valu_busy_pct")}
    out = {
        "metric": "zone-updates/sec FP32 vs FP64 at stated L1 error; p50/p99 latency when served",
        "value": value,
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "grid": [args.n] * 3, "gamma": 5.0 / 3.0, "cfl": 0.3, "seed": 0,
                   "state": head, "tile": [tx, ty]},
        "autotune": {p: {"ms_per_step_by_tile": {"x".join(map(str, ppml_tile_shape(3, v))): t
                                                  for v, t in res[p]["tuned"]["ms_per_step"].items()}}
                     for p in res if res[p]["tuned"]},
        "kernels_ms": {"euler": r["ms_euler"], "lagr": r["ms_lagr"]},
        # the dominant kernel against the published vector peak of its type
        # (FP32 157.3 TFLOP/s counts packed FP32 instructions, which this build
        # does not use; the rate of the unpacked FMA it does use, 78.6, is
        # beside it), with the VALU issue fraction that shows the bound and the
        # whole step's compulsory HBM bytes against 8 TB/s
        "roofline": {"bound": "alu", "kernel": "k_" + kern, "achieved": achieved_tflops,
                     "peak": FP32_VECTOR_PEAK_TFLOPS if dt == "f32" else FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tflops / (FP32_VECTOR_PEAK_TFLOPS if dt == "f32" else FP64_VECTOR_PEAK_TFLOPS),
                     "traffic": traffic, "algorithmic_flop_per_zone": ALGO_FLOP_PER_ZONE_3D[kern],
                     "unpacked_fma_peak": VALU_PEAK_TFLOPS[dt],
                     "frac_of_unpacked_fma_peak": achieved_tflops / VALU_PEAK_TFLOPS[dt],
                     "valu_issue": valu_issue,
                     "launch_ms": ms_k,
                     "hbm": {"achieved_GBs": achieved_gbs, "peak_GBs": HBM_PEAK_GBS,
                             "frac": achieved_gbs / HBM_PEAK_GBS,
                             "algorithmic_bytes_per_zone": algorithmic_bytes_per_zone(kern, 3, width),
                             "measured_GBs": (traffic / (ms_k * 1e-3) / 1e9) if traffic else None},
                     "step_hbm": {"compulsory_bytes_per_zone": 2 * 6 * width,
                                  "achieved_GBs": 2 * 6 * width * cells / (r["ms"] / args.steps * 1e-3) / 1e9,
                                  "peak_GBs": HBM_PEAK_GBS,
                                  "frac": 2 * 6 * width * cells / (r["ms"] / args.steps * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                  "target_frac": 0.6}},
    }
    if "fp64" in res and "fp32" in res:
        r64 = res["fp64"]
        out["fp64"] = {"value": cells * args.steps / (r64["ms"] * 1e-3), "ms_per_step": r64["ms"] / args.steps,
                       "kernels_ms": {"euler": r64["ms_euler"], "lagr": r64["ms_lagr"]},
                       "tile": list(ppml_tile_shape(3, r64["tuned"]["tile"] if r64["tuned"] else 0))}
    if not args.no_batch and "fp32" in res:
        print("[bench] batched configuration", file=sys.stderr, flush=True)
        out["batched"] = run_batched()
        print(f"[bench] batched: {out['batched']['speedup']:.1f}x over plain launches", file=sys.stderr, flush=True)
        print("[bench] served configuration", file=sys.stderr, flush=True)
        out["served"] = run_served(n_requests=args.serve_requests)
    if not args.no_batch:
        print("[bench] disk configuration", file=sys.stderr, flush=True)
        out["disk"] = run_disk()
        print(f"[bench] disk: fp32 {out['disk']['fp32']['zone_updates_per_s']:.3e} zu/s, "
              f"fp64 {out['disk']['fp64']['zone_updates_per_s']:.3e} zu/s", file=sys.stderr, flush=True)
        out["disk_isothermal"] = run_disk(isothermal=True)
        print(f"[bench] isothermal disk: fp32 {out['disk_isothermal']['fp32']['zone_updates_per_s']:.3e} zu/s",
              file=sys.stderr, flush=True)
        print("[bench] 1-D Riemann configuration", file=sys.stderr, flush=True)
        out["riemann_1d"] = run_riemann_1d()
        print("[bench] test-suite workloads", file=sys.stderr, flush=True)
        out["suite"] = run_suite()
        print("[bench] self-gravity workload", file=sys.stderr, flush=True)
        out["gravity"] = run_gravity()
    if not args.no_cpu:
        print("[bench] cpu baseline: the oracle runs the full workload", file=sys.stderr, flush=True)
        out["cpu_baseline"], taus, final = cpu_baseline(prob, steps=WORKLOAD_STEPS)
        print(f"[bench] oracle: {out['cpu_baseline']['value']:.3e} zone-updates/s on "
              f"{out['cpu_baseline']['cores']} threads", file=sys.stderr, flush=True)
        out["parity_after_run"] = parity_after_run(prob, taus, final)
        pr = out["parity_after_run"]
        print(f"[bench] after {pr['steps']} steps vs oracle: fp64 max normwise "
              f"{max(pr['fp64_normwise_rel_err_per_field'].values()):.2e}, fp32 L1(rho) {pr['fp32_l1_rho']:.2e}",
              file=sys.stderr, flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
