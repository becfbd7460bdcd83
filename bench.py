"""Benchmark of the HOSC hot path on one MI355X.

Workload: the paper's power-law cavity at 129^3 (n = 0.75 shear-thinning, Ra = 1e5,
Pr = 1, dt = 5e-5, FP64, implicit-system tolerance 1e-10, seeded noise of 1e-3 on the
linear conduction profile, seed 2).  One step = the whole hot path: viscosity and
sources, HOSC assembly, the four implicit solves, update, pressure correction, and
the Nusselt / entropy / Bejan reductions.

Under the stated scheme this march is stable only for its first ~15 steps from the
impulsive start (the FP64 oracle diverges at step 16 exactly like the GPU path), so
the timed steps are taken in segments of SEGMENT steps from the seeded initial
state; the clock is stopped while the state is re-initialised between segments.

`--workload piter` is the benchmark workload with pressure iterations: up to three
momentum solves per step, the pressure corrected after each (div_tol = 0, so all
three run).  After the timed run it also marches a Newtonian 41^3 cavity (Ra = 1e4,
Pr = 1, dt = 0.4 h^2) to a per-step residual of 2.5e-12 with one and with four
pressure iterations and reports steps and seconds of each.

`--workload serve` replays the seeded Poisson trace in real time against the
server (completed solves/s, p50/p99 latency, a mix-vs-alone check) and then
compares, on a saturated queue of its first 40 requests, the server (FP32 refined
and FP64) with the plain path of one FP64 single-cavity solver after another.
`--workload batch12` advances the 12-cavity batch with fused launches and compares
it with the same steps cavity by cavity.

`--workload fp32r` is the precision form (n = 1.25, Ra = 1e4, FP32 rows and inner
sweeps with FP64 residuals and refinement).  Shear-thickening flow cannot start
from rest under the stated scheme (the second step's rows lose their centre), so
it starts from a flowing state: the seeded rest state advanced by 20 Newtonian
FP64 steps at the same Ra and dt.  After the timed run the same segment is run in
FP64 from the same start and the relative L2 difference of every field and of the
Nu/Be/entropy scalars is reported.

`--workload sizes` reports the half-sweep bandwidth for grids from 129^3 to 385^3:
at 129^3 part of each launch's working set stays in the 256 MB Infinity Cache
between launches, from 257^3 on it streams from HBM.

Prints one JSON line: cell-updates/s (interior nodes x steps / second), the
roofline of the dominant kernel (the red-black sweep, HIP events around every
launch, algorithmic bytes per launch), with the whole step's algorithmic bytes
against the HBM peak (`roofline.step`) and the half-sweep on a 257^3 grid whose
working set streams from HBM (`roofline.hbm_streaming`), each beside the library's
streaming probe with the half-sweep's access mix on arrays of that grid's size
(`mix_probe_GBs`, `frac_of_mix_probe`), the same segment with its state handed
over from and back to host memory through the C ABI (`pcie_inclusive`; `value`
itself starts and ends with the state in HBM), and the FP64 CPU oracle
timed on the host cores on a bounded sample of the same workload.  The default
run also carries the metric's second half: `serving` (24 small requests of the
seeded trace marched to res 1e-8 through the server, FP32 refined, against the
plain FP64 path one cavity after another: solves/s, p50/p99 time to steady
state, a mix-vs-alone check) and `batch` (the 12-cavity batch against the same
steps cavity by cavity, and the small requests as one batch marched to steady
state with hosc_batch_run_to_steady).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM traffic of one k_sweep launch on this workload from FETCH_SIZE / WRITE_SIZE
# (two rocprofv3 --pmc passes, calibrated against the copy probe), valid for the
# kernel source with this sha256 prefix; any other source reports null.
SWEEP_TRAFFIC = {"kernels_sha256_16": "7830199ce6df33a9", "bytes_per_launch": 1.4950e+08}
METRIC = "cell-updates/s + HBM roofline % at 129^3; served solves/s, p50/p99 latency"
WORKLOADS = {
    # the benchmark workload: FP64, shear-thinning, Ra = 1e5
    "fp64": dict(N=129, Ra=1e5, n_pl=0.75, Pr=1.0, dt=5e-5, seed=2, noise=1e-3, solve_rtol=1e-10, precision=0,
                 label="HOSC cavity 129^3, n=0.75, Ra=1e5, Pr=1, dt=5e-5, FP64, rtol 1e-10, seed 2"),
    # precision form: shear-thickening, Ra = 1e4, FP32 rows and sweeps with FP64 refinement
    # batched form: dt = max(5e-5, 0.2 h^2) per cavity.  At 5e-5 the 33^3 shear-
    # thickening cavities lose their implicit rows within a few steps (on the oracle as
    # on the GPU), and 0.2 h^2 everywhere does the same to the 97^3 ones at Ra = 1e5.
    "batch12": dict(kind="batch", Pr=1.0, dt=5e-5, dt_over_h2=0.2, noise=1e-3, solve_rtol=1e-10, precision=1, segment=30,
                    label="12 HOSC cavities, (Ra, n) in {1e2,1e3,1e4,1e5} x {0.75,1,1.25}, sizes 33^3/65^3/97^3 "
                          "(4 each, seeded shuffle, seed 4), Pr=1, dt=max(5e-5, 0.2 h^2), FP32 rows/sweeps + FP64 refinement, "
                          "rtol 1e-10, cavity seeds 100+i, seeded rest start"),
    # serving form: the seeded Poisson trace (rate 2/s); each request runs to res 1e-8 or
    # max_steps steps with dt = 0.4 h^2; a 4 GiB HBM budget forces queueing
    "serve": dict(kind="serve", requests=120, rate=2.0, trace_seed=5, dt_over_h2=0.4, res_tol=1e-8, max_steps=200,
                  budget=4 << 30, max_resident=64, precision=1, solve_rtol=1e-10, noise=1e-3, sample=20,
                  label="serving trace: Poisson arrivals at 2/s (seed 5), N uniform over {33,49,65,97,129}, "
                        "Ra log-uniform in [1e2,1e5], n uniform in [0.7,1.3], Pr=1, dt=0.4 h^2, FP32 rows/sweeps + "
                        "FP64 refinement, rtol 1e-10, each request to res < 1e-8 or 200 steps, HBM budget 4 GiB"),
    # pressure iterations: the benchmark workload with three momentum solves per step
    "piter": dict(N=129, Ra=1e5, n_pl=0.75, Pr=1.0, dt=5e-5, seed=2, noise=1e-3, solve_rtol=1e-10, precision=0,
                  p_iters=3,
                  label="HOSC cavity 129^3, n=0.75, Ra=1e5, Pr=1, dt=5e-5, FP64, rtol 1e-10, seed 2, "
                        "3 pressure iterations per step (momentum re-solved after each correction)"),
    # half-sweep bandwidth against grid size: from a working set that partly stays in
    # the 256 MB Infinity Cache (129^3) to ones that stream from HBM; the benchmark
    # physics with dt = 0.82 h^2 (the benchmark's dt/h^2), FP64, SOR
    "sizes": dict(kind="sizes", grids=(129, 161, 193, 257, 385), Ra=1e5, n_pl=0.75, Pr=1.0, dt_over_h2=0.82, seed=2,
                  noise=1e-3, solve_rtol=1e-10,
                  label="HOSC half-sweep bandwidth against grid size (129^3 to 385^3), n=0.75, Ra=1e5, Pr=1, "
                        "dt=0.82 h^2, FP64, rtol 1e-10, seed 2; 3 untimed and 6 timed steps per grid"),
    "fp32r": dict(N=129, Ra=1e4, n_pl=1.25, Pr=1.0, dt=5e-5, seed=3, noise=1e-3, solve_rtol=1e-10, precision=1,
                  newtonian_start=20, segment=60,
                  label="HOSC cavity 129^3, n=1.25, Ra=1e4, Pr=1, dt=5e-5, FP32 rows/sweeps + FP64 refinement, "
                        "rtol 1e-10, seed 3, flowing start (20 Newtonian FP64 steps)"),
}
WORKLOAD = WORKLOADS["fp64"]
SEGMENT = 12


def sweep_traffic():
    path = os.path.join(ROOT, "paper_2411_06563_amd", "csrc", "hosc_kernels.hpp")
    with open(path, "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()[:16]
    return SWEEP_TRAFFIC["bytes_per_launch"] if h == SWEEP_TRAFFIC["kernels_sha256_16"] else None


def cpu_baseline(budget_s: float = 20.0) -> dict:
    """The oracle as it stands, on the same 129^3 workload from the same initial
    state, for as many steps as fit in about budget_s seconds (at least one)."""
    from oracle import oracle as orc
    from paper_2411_06563_amd.inputs import initial_state
    W = WORKLOAD
    o = orc.Oracle(orc.Params(N=W["N"], Ra=W["Ra"], n_pl=W["n_pl"], Pr=W["Pr"], dt=W["dt"], solve_tol=1e-13))
    o.set_state(**initial_state(W["N"], W["seed"], W["noise"]))
    t0 = time.perf_counter()
    steps = 0
    while True:
        o.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 10:
            break
    M3 = (W["N"] - 2) ** 3
    cores = orc.num_threads()
    return {"value": M3 * steps / el, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"first {steps} step(s) of the 129^3 workload from its initial state "
                      f"({el:.1f} s, FP64, BiCGSTAB tol 1e-13, {cores} OpenMP threads)"}


def steady_comparison(hosc, torch, N=41, tol=2.5e-12):
    """Steps and seconds to a steady residual `tol` per step for a Newtonian cavity
    (Ra = 1e4, Pr = 1, dt = 0.4 h^2) with one and with four pressure iterations,
    and the largest field difference of the two steady states."""
    import numpy as np
    h = 1.0 / (N - 1)
    out, states = {"grid": N, "res_tol": tol}, {}
    for K in (1, 4):
        s = hosc.Solver(hosc.params(N, Ra=1e4, n_pl=1.0, Pr=1.0, dt=0.4 * h * h, solve_rtol=1e-11, p_iters=K),
                        device="cuda:0")
        s.init_fields(1, 1e-3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while True:
            info = s.run_to_steady(tol, 5000)
            if max(info.res) < tol or info.step >= 100000:
                break
        torch.cuda.synchronize()
        out[f"p_iters_{K}"] = {"steps": info.step, "seconds": time.perf_counter() - t0,
                               "nu_mean_hot": s.diagnostics(arrays=False)["nu_mean_hot"]}
        states[K] = s.get_state()
        s.close()
    out["max_rel_field_diff"] = max(float(np.max(np.abs(states[1][f] - states[4][f])) / np.max(np.abs(states[1][f])))
                                    for f in ("u", "v", "w", "T"))
    return out


def precision_check(hosc, W, kw, reset, steps):
    """Relative L2 difference of every field, and relative difference of the Nu, Be
    and entropy scalars, between the precision form and the FP64 path after `steps`
    steps from the same start state, with the wall time per step of each run (the
    first steps of a fresh solver, so a little above the timed figure)."""
    import numpy as np
    import torch
    res, ms = {}, {}
    for prec in (0, W["precision"]):
        s = hosc.Solver(hosc.params(W["N"], **dict(kw, precision=prec)), device="cuda:0")
        reset(s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.step(1)
            s.diagnostics(arrays=False)
        torch.cuda.synchronize()
        ms[prec] = (time.perf_counter() - t0) * 1e3 / steps
        res[prec] = (s.get_state(), s.diagnostics(arrays=False))
        s.close()
    (g0, d0), (g1, d1) = res[0], res[W["precision"]]
    out = {"steps": steps, "fp64_ms_per_step": ms[0], "this_form_ms_per_step": ms[W["precision"]],
           "field_rel_l2": {}, "scalar_rel": {}}
    for f in ("u", "v", "w", "T", "p"):
        out["field_rel_l2"][f] = float(np.linalg.norm(g1[f] - g0[f]) / np.linalg.norm(g0[f]))
    for k in ("nu_mean_hot", "nu_mean_cold", "nu_max_hot", "be_global", "e_total"):
        out["scalar_rel"][k] = float(abs(d1[k] - d0[k]) / abs(d0[k]))
    return out


# algorithmic bytes per interior node of the kernels of a step other than the
# implicit solves and the assembly (timed separately): viscosity 32, sources 72,
# update 88, divergence and pressure 40, entropy pass 40
OTHER_BYTES_PER_NODE = 32 + 72 + 88 + 40 + 40


def stream_sweep(hosc, torch, W, N):
    """Half-sweep bandwidth on a grid whose working set streams from HBM (the 129^3
    launch partly stays in the 256 MB Infinity Cache): the benchmark physics with the
    benchmark's dt/h^2, FP64, SOR, 2 untimed and 4 timed steps."""
    p = hosc.params(N, Ra=W["Ra"], n_pl=W["n_pl"], Pr=W["Pr"], dt=W["dt"] * (128.0 / (N - 1)) ** 2,
                    solve_rtol=W["solve_rtol"], solver=hosc.SOLVER_SOR)
    s = hosc.Solver(p, device="cuda:0")
    s.init_fields(W["seed"], W["noise"])
    s.step(2)
    s.perf_enable(True)
    s.step(4)
    torch.cuda.synchronize()
    c = s.perf()
    s.close()
    del s
    torch.cuda.empty_cache()
    n = max(c["sweep_launches"], 1)
    gbs = c["sweep_bytes"] / (c["sweep_ms"] * 1e-3) / 1e9
    mix = mix_probe(hosc, N)
    return {"grid": N, "kernel": "k_sweep", "half_sweeps": c["sweep_launches"],
            "bytes_per_launch": c["sweep_bytes"] / n, "avg_launch_us": c["sweep_ms"] / n * 1e3,
            "achieved": gbs, "frac": gbs / HBM_PEAK_GBS, "mix_probe_GBs": mix, "frac_of_mix_probe": gbs / mix}


def pcie_inclusive(s, reset, torch, M3, seg, reps=3):
    """The benchmark segment with its input handed over from host memory and its
    result read back to host memory: hosc_set_state from pageable numpy arrays (the
    segment's start state, u, v, w, theta, p), `seg` steps with the per-step
    diagnostics, hosc_get_state into pageable numpy arrays, timed end to end (best
    of `reps`); and the two transfers alone.  Then the same with page-locked host
    arrays."""
    reset(s)
    host = s.get_state()
    nbytes = sum(a.nbytes for a in host.values())
    best, best_xfer = float("inf"), float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.set_state(**host, apply_bc=False)
        s.get_state()
        best_xfer = min(best_xfer, time.perf_counter() - t0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.set_state(**host, apply_bc=False)
        for _ in range(seg):
            s.step(1)
            s.diagnostics(arrays=False)
        s.get_state()
        best = min(best, time.perf_counter() - t0)
    # the same with page-locked host arrays (torch's pinned allocation, viewed as numpy)
    pin = {f: torch.empty(a.shape, dtype=torch.float64, pin_memory=True).numpy() for f, a in host.items()}
    back = {f: torch.empty(a.shape, dtype=torch.float64, pin_memory=True).numpy() for f, a in host.items()}
    for f in host:
        pin[f][...] = host[f]
    best_pin, best_pin_xfer = float("inf"), float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.set_state(**pin, apply_bc=False)
        s.get_state(out=back)
        best_pin_xfer = min(best_pin_xfer, time.perf_counter() - t0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.set_state(**pin, apply_bc=False)
        for _ in range(seg):
            s.step(1)
            s.diagnostics(arrays=False)
        s.get_state(out=back)
        best_pin = min(best_pin, time.perf_counter() - t0)
    return {"segment_steps": seg, "state_bytes_each_way": nbytes,
            "pageable": {"ms_per_segment": best * 1e3, "cell_updates_per_s": M3 * seg / best,
                         "transfers_alone_ms": best_xfer * 1e3, "transfer_GBs": 2 * nbytes / best_xfer / 1e9},
            "pinned": {"ms_per_segment": best_pin * 1e3, "cell_updates_per_s": M3 * seg / best_pin,
                       "transfers_alone_ms": best_pin_xfer * 1e3, "transfer_GBs": 2 * nbytes / best_pin_xfer / 1e9}}


def mix_probe(hosc, N):
    """GB/s of the library's streaming probe with the half-sweep's access mix (15
    read-only arrays, 4 rewritten in place) on arrays of one colour half of the
    N^3 grid's interior: what a plain streaming kernel achieves with the sweep's
    reads, writes and working set."""
    return hosc.stream_mix_bandwidth(8 * ((N - 2) ** 3 // 2), 20)


def bench_sizes(args, W, hosc, torch):
    """Half-sweep bandwidth (algorithmic bytes / HIP-event launch time) for grids
    from 129^3, whose per-launch working set (about 150 MB) partly stays in the
    256 MB Infinity Cache between launches, to 385^3 (4.7 GB per launch), which
    streams from HBM; each beside the library's streaming probe with the
    half-sweep's access mix on arrays of that grid's size, plus the copy probe."""
    rows = []
    t0 = time.perf_counter()
    for N in W["grids"]:
        p = hosc.params(N, Ra=W["Ra"], n_pl=W["n_pl"], Pr=W["Pr"], dt=W["dt_over_h2"] / (N - 1) ** 2,
                        solve_rtol=W["solve_rtol"], solver=hosc.SOLVER_SOR)
        s = hosc.Solver(p, device="cuda:0")
        s.init_fields(W["seed"], W["noise"])
        s.step(3)
        s.perf_enable(True)
        s.step(6)
        torch.cuda.synchronize()
        c = s.perf()
        n = max(c["sweep_launches"], 1)
        rows.append({"grid": N, "half_sweeps": c["sweep_launches"], "mb_per_launch": c["sweep_bytes"] / n / 1e6,
                     "us_per_launch": c["sweep_ms"] / n * 1e3,
                     "gb_per_s": c["sweep_bytes"] / (c["sweep_ms"] * 1e-3) / 1e9})
        s.close()
        del s
        torch.cuda.empty_cache()
        mix = mix_probe(hosc, N)
        torch.cuda.empty_cache()
        rows[-1]["mix_probe_gb_per_s"] = mix
        rows[-1]["frac_of_mix_probe"] = rows[-1]["gb_per_s"] / mix
        print(f"[sizes] {rows[-1]}", file=sys.stderr, flush=True)
    el = time.perf_counter() - t0
    copy = hosc.copy_bandwidth()
    big = rows[-1]
    out = {
        "metric": METRIC, "value": big["gb_per_s"], "unit": "GB/s", "n_gpus": 1, "steps": 6, "warmup": 3,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": W["label"], "grids": list(W["grids"]), "wall_s": el},
        "roofline": {"bound": "hbm", "kernel": f"k_sweep at {big['grid']}^3", "achieved": big["gb_per_s"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": big["gb_per_s"] / HBM_PEAK_GBS, "traffic": None},
        "sizes": rows,
        "copy_probe_gb_per_s": copy,
    }
    print(json.dumps(out), flush=True)


def bench_batch(args, W, hosc, torch):
    """Batched form: all cavities advanced together (fused persistent solver
    launches, graph-captured phases, autotuned schedule).  Reports the aggregate
    cell-updates/s, the same segment stepped cavity by cavity with the
    single-cavity path (serial baseline), and the largest difference between each
    cavity's batched and single-cavity results (0 = bitwise equal)."""
    import numpy as np
    from paper_2411_06563_amd.inputs import batched_cavities
    cavs = batched_cavities(4)
    seg = args.segment if args.segment is not None else W["segment"]
    plist = [hosc.params(c["N"], Ra=c["Ra"], n_pl=c["n_pl"], Pr=W["Pr"], dt=max(W["dt"], W["dt_over_h2"] / (c["N"] - 1) ** 2),
                         solve_rtol=W["solve_rtol"], precision=W["precision"]) for c in cavs]
    seeds = [c["seed"] for c in cavs]
    b = hosc.Batch(plist)

    def reset():
        b.init_fields(seeds, W["noise"])

    reset()
    grid = b.tune()
    M3 = sum((c["N"] - 2) ** 3 for c in cavs)
    in_seg = 0
    for _ in range(args.warmup):
        if in_seg == seg:
            reset()
            in_seg = 0
        b.step(1)
        in_seg += 1
    reset()
    in_seg = 0
    b.perf_enable(True)
    torch.cuda.synchronize()
    el = 0.0
    t0 = time.perf_counter()
    sweeps = np.zeros(2)
    for q in range(args.steps):
        if in_seg == seg:
            torch.cuda.synchronize()
            el += time.perf_counter() - t0
            reset()
            in_seg = 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        infos = b.step(1)
        in_seg += 1
        sweeps += np.array([sum(i.sweeps[0] for i in infos), sum(i.sweeps[1] for i in infos)])
        if q % 10 == 0:
            print(f"batch step {q}: sweeps {[i.sweeps for i in infos]}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el += time.perf_counter() - t0
    perf = b.perf()
    b.perf_enable(False)
    graphs = b.graph_launches()
    # one segment batched vs cavity by cavity (single-cavity path, same stream kind)
    reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(seg)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    got = [cv.get_state() for cv in b.cavities]
    t_serial = 0.0
    worst = 0.0
    for i, p in enumerate(plist):
        s = hosc.Solver(p)
        s.init_fields(seeds[i], W["noise"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(seg)
        torch.cuda.synchronize()
        t_serial += time.perf_counter() - t0
        g = s.get_state()
        s.close()
        worst = max(worst, max(float(np.max(np.abs(g[f] - got[i][f]))) for f in ("u", "v", "w", "T", "p")))
    b.close()
    avg_ms = perf["sweep_ms"] / max(perf["sweep_launches"], 1)
    avg_bytes = perf["sweep_bytes"] / max(perf["sweep_launches"], 1)
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": M3 * args.steps / el,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{W['label']}; steps 1-{seg} from the start states, repeated",
                   "cavities": [(c["N"], c["Ra"], c["n_pl"]) for c in cavs], "interior_nodes": M3,
                   "cavity_steps_per_s": len(cavs) * args.steps / el, "tuned_grid": grid,
                   "graph_launches": graphs,
                   "mean_sor_sweeps_per_cavity_step": (sweeps / (args.steps * len(cavs))).tolist()},
        "roofline": {"bound": "hbm", "kernel": "k_sweep_fused (all cavities, one half-sweep)", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "avg_launch_us": avg_ms * 1e3, "launches": perf["sweep_launches"],
                     "bytes_per_launch": avg_bytes, "kernel_time_frac": perf["sweep_ms"] * 1e-3 / el,
                     "refine_time_frac": perf["refine_ms"] * 1e-3 / el},
        "batch_check": {"segment_steps": seg, "batched_s": t_batch, "cavity_by_cavity_s": t_serial,
                        "speedup": t_serial / t_batch, "max_abs_diff_vs_single_cavity": worst},
    }
    print(json.dumps(out), flush=True)


def bench_serve(args, W, hosc, torch):
    """Serving form: replay the first `requests` arrivals of the seeded trace in real
    time against the server (admission by HBM budget, continuous fused batching).
    Reports completed solves/s, p50/p99 of completion - arrival (and of the service
    time), and a mix-vs-alone check: sampled requests rerun as single cavities for
    the same number of steps must reproduce the served diagnostics bitwise."""
    import numpy as np
    from paper_2411_06563_amd.inputs import serving_trace
    nreq = args.requests if args.requests is not None else W["requests"]
    max_steps = args.max_steps if args.max_steps is not None else W["max_steps"]
    first = args.first
    trace = [dict(r) for r in serving_trace(500, W["rate"], W["trace_seed"])[first:first + nreq]]
    nreq = len(trace)
    t_first = trace[0]["arrival"]
    for r in trace:     # a later segment of the trace starts its clock at its own first arrival
        r["arrival"] -= t_first
    # --to-steady: every request marched to res_tol (the step cap only as a guard),
    # with the viscosity relaxation of the time-to-steady leg
    relax = (lambda n: steady_relax(n)) if args.to_steady else (lambda n: 1.0)
    plist = [hosc.params(r["N"], Ra=r["Ra"], n_pl=r["n_pl"], Pr=r["Pr"], dt=W["dt_over_h2"] / (r["N"] - 1) ** 2,
                         solve_rtol=W["solve_rtol"], precision=W["precision"], eta_relax=relax(r["n_pl"]))
             for r in trace]
    srv = hosc.Server(W["budget"], max_resident=W["max_resident"])
    t0 = srv.now()
    ids, results = {}, {}
    nxt = 0
    max_queued = 0
    next_report = 5000
    while len(results) < nreq:
        now = srv.now() - t0
        while nxt < nreq and trace[nxt]["arrival"] <= now:
            r = trace[nxt]
            ids[srv.submit(plist[nxt], r["seed"], W["noise"], W["res_tol"], max_steps, t0 + r["arrival"])] = nxt
            nxt += 1
        st = srv.stats()
        max_queued = max(max_queued, st["queued"])
        if st["resident"] or st["queued"]:
            srv.step()
        elif nxt < nreq:
            time.sleep(min(0.005, max(0.0, trace[nxt]["arrival"] - (srv.now() - t0))))
        for r in srv.poll():
            results[ids[r["id"]]] = r
            if len(results) % 20 == 0 or args.to_steady:
                print(f"serve: {len(results)}/{nreq} done", file=sys.stderr, flush=True)
        if args.to_steady and st["server_steps"] >= next_report:
            next_report += 5000
            print(f"serve: server step {st['server_steps']}, {st['resident']} resident, {len(results)} done",
                  file=sys.stderr, flush=True)
    st = srv.stats()
    srv.close()
    ok = [i for i in range(nreq) if results[i]["status"] == 0]
    steady = [i for i in ok if results[i]["steady"]]
    capped = [i for i in ok if not results[i]["steady"]]
    # the headline counts a request as solved only when it reached the steady residual
    lat = np.array([results[i]["t_done"] - results[i]["t_arrival"] for i in steady]) if steady else np.zeros(1)
    svc = np.array([results[i]["t_done"] - results[i]["t_admit"] for i in steady]) if steady else np.zeros(1)
    span = max(results[i]["t_done"] for i in range(nreq)) - (t0 + trace[0]["arrival"])
    # mix vs alone on sampled successful requests
    pool = steady if steady else ok
    nsample = args.sample if args.sample is not None else W["sample"]
    sample = pool[:: max(1, len(pool) // nsample)][:nsample] if nsample > 0 else []
    same = 0
    for i in sample:
        s = hosc.Solver(plist[i])
        s.init_fields(trace[i]["seed"], W["noise"])
        s.step(results[i]["steps"])
        d = s.diagnostics(arrays=False)
        s.close()
        same += int(d == results[i]["diag"])
    M3 = np.array([(trace[i]["N"] - 2) ** 3 for i in range(nreq)], dtype=float)
    cell_updates = float(sum(M3[i] * results[i]["steps"] for i in range(nreq)))
    out = {
        "metric": METRIC,
        "value": len(steady) / span,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": int(st["server_steps"]),
        "warmup": 0,
        "ms_per_step": st["busy_s"] * 1e3 / max(st["server_steps"], 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": W["label"].replace("or 200 steps", f"or {max_steps} steps")
                   + f"; requests {first}..{first + nreq - 1} of the 500-request trace",
                   "max_steps": max_steps,
                   "viscosity_relaxation": "0.1 for n < 1, 0.5 for n > 1" if args.to_steady else "none"},
        "steady_latencies_s": [round(float(x), 3) for x in lat] if args.to_steady else None,
        "latency_s": {"over": "requests that reached the steady residual",
                      "p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "mean": float(lat.mean())},
        "service_s": {"p50": float(np.percentile(svc, 50)), "p99": float(np.percentile(svc, 99))},
        "requests": {"completed": nreq, "steady": len(steady), "capped_at_max_steps": len(capped),
                     "failed": nreq - len(ok),
                     "failed_status": sorted({results[i]["status"] for i in range(nreq)} - {0})},
        "server": {"cavity_steps": int(st["cavity_steps"]), "server_steps": int(st["server_steps"]),
                   "busy_s": st["busy_s"], "span_s": span, "peak_bytes": int(st["peak"]),
                   "budget_bytes": int(st["budget"]), "max_queued": int(max_queued),
                   "cell_updates_per_busy_s": cell_updates / max(st["busy_s"], 1e-9)},
        "mix_vs_alone": {"sampled": len(sample), "bitwise_equal": same},
    }
    if args.capacity > 0:
        out["capacity"] = serve_capacity(hosc, W, trace, min(args.capacity, nreq), args.capacity_rtol)
    if args.steady > 0:
        out["time_to_steady"] = serve_steady(hosc, W, args.steady)
    print(json.dumps(out), flush=True)


def serve_capacity(hosc, W, trace, k, rtol=None):
    """Capacity on a saturated queue: the first k requests of the trace submitted at
    once, (a) through the server (continuous fused batching, FP32 refined and FP64),
    (b) through the plain path: one FP64 single-cavity solver after another.  Each
    request runs to res_tol or max_steps as in the replay.  Reports solves/s (ok
    solves / wall time) and p50/p99 of completion time."""
    import numpy as np
    rtol = W["solve_rtol"] if rtol is None else rtol
    out = {"requests": k, "solve_rtol": rtol}

    def plist(prec):
        return [hosc.params(r["N"], Ra=r["Ra"], n_pl=r["n_pl"], Pr=r["Pr"], dt=W["dt_over_h2"] / (r["N"] - 1) ** 2,
                            solve_rtol=rtol, precision=prec) for r in trace[:k]]

    for name, prec in (("served_fp32_refined", 1), ("served_fp64", 0)):
        pl = plist(prec)
        srv = hosc.Server(W["budget"], max_resident=W["max_resident"])
        t0 = srv.now()
        ids = {srv.submit(pl[i], trace[i]["seed"], W["noise"], W["res_tol"], W["max_steps"], t0): i for i in range(k)}
        res = {}
        while len(res) < k:
            srv.step()
            for r in srv.poll():
                res[ids[r["id"]]] = r
        wall = max(r["t_done"] for r in res.values()) - t0
        srv.close()
        ok = [i for i in range(k) if res[i]["status"] == 0]
        done = np.array([res[i]["t_done"] - t0 for i in ok])
        out[name] = {"solves_per_s": len(ok) / wall, "wall_s": wall, "ok": len(ok),
                     "p50_s": float(np.percentile(done, 50)), "p99_s": float(np.percentile(done, 99))}
        print(f"capacity {name}: {out[name]}", file=sys.stderr, flush=True)
    import torch
    pl = plist(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, ok = [], 0
    for i in range(k):
        s = hosc.Solver(pl[i])
        s.init_fields(trace[i]["seed"], W["noise"])
        try:
            s.run_to_steady(W["res_tol"], W["max_steps"])
            s.diagnostics(arrays=False)
            ok += 1
            torch.cuda.synchronize()
            done.append(time.perf_counter() - t0)
        except hosc.HoscError:
            pass
        s.close()
    wall = time.perf_counter() - t0
    out["plain_fp64_sequential"] = {"solves_per_s": ok / wall, "wall_s": wall, "ok": ok,
                                    "p50_s": float(np.percentile(done, 50)), "p99_s": float(np.percentile(done, 99))}
    print(f"capacity plain: {out['plain_fp64_sequential']}", file=sys.stderr, flush=True)
    return out


def steady_relax(n_pl: float) -> float:
    """Viscosity relaxation used for marching to steady state: strong for shear-
    thinning fluids (their lagged viscosity sustains a period-2 oscillation), mild
    otherwise (a shear-thickening fluid must leave its low rest-state viscosity)."""
    return 0.1 if n_pl < 1.0 else 0.5


def steady_requests(W, k):
    """The first k requests of the seeded trace with N <= 49 (the larger cavities need
    1e4-1e5 steps at the stable time steps)."""
    from paper_2411_06563_amd.inputs import serving_trace
    return [r for r in serving_trace(500, W["rate"], W["trace_seed"]) if r["N"] <= 49][:k]


def steady_params(hosc, W, r, prec):
    return hosc.params(r["N"], Ra=r["Ra"], n_pl=r["n_pl"], Pr=r["Pr"], dt=W["dt_over_h2"] / (r["N"] - 1) ** 2,
                       solve_rtol=W["solve_rtol"], precision=prec, eta_relax=steady_relax(r["n_pl"]))


def _pcts(x):
    import numpy as np
    if not x:
        return {"p50_s": None, "p99_s": None}
    return {"p50_s": float(np.percentile(x, 50)), "p99_s": float(np.percentile(x, 99))}


def serve_steady(hosc, W, k, sample=4):
    """Time to steady state: the first k small requests of the trace, each marched to
    res 1e-8 (at most 30000 steps) with the viscosity relaxation, submitted at once
    to the server (FP32 refined), and the same requests through the plain path (one
    FP64 single-cavity solver after another).  Reports steady solves, solves/s and
    p50/p99 time to steady state, and a mix-vs-alone check: sampled served requests
    rerun alone (same precision, single-cavity run to steady state) must take the
    same number of steps and give bitwise the same diagnostics."""
    import torch
    trace = steady_requests(W, k)
    out = {"requests": k, "sizes": sorted({r["N"] for r in trace}), "res_tol": 1e-8, "max_steps": 30000}
    srv = hosc.Server(W["budget"], max_resident=W["max_resident"])
    t0 = srv.now()
    ids = {srv.submit(steady_params(hosc, W, r, W["precision"]), r["seed"], W["noise"], 1e-8, 30000, t0): i
           for i, r in enumerate(trace)}
    res = {}
    while len(res) < k:
        srv.step()
        for q in srv.poll():
            res[ids[q["id"]]] = q
    srv.close()
    steady = [i for i in range(k) if res[i]["status"] == 0 and res[i]["steady"]]
    done = [res[i]["t_done"] - t0 for i in steady]
    wall = max(q["t_done"] for q in res.values()) - t0
    failed = sum(1 for i in range(k) if res[i]["status"] != 0)
    out["served_fp32_refined"] = dict({"steady": len(steady), "failed": failed,
                                       "capped": k - len(steady) - failed, "wall_s": wall,
                                       "solves_per_s": len(steady) / wall}, **_pcts(done))
    print(f"steady served: {out['served_fp32_refined']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, failed = [], 0
    for r in trace:
        sv = hosc.Solver(steady_params(hosc, W, r, 0))
        sv.init_fields(r["seed"], W["noise"])
        try:
            info = sv.run_to_steady(1e-8, 30000)
            torch.cuda.synchronize()
            if max(info.res) < 1e-8:
                done.append(time.perf_counter() - t0)
        except hosc.HoscError:
            failed += 1
        sv.close()
    wall = time.perf_counter() - t0
    out["plain_fp64_sequential"] = dict({"steady": len(done), "failed": failed, "wall_s": wall,
                                         "solves_per_s": len(done) / wall}, **_pcts(done))
    print(f"steady plain: {out['plain_fp64_sequential']}", file=sys.stderr, flush=True)
    same = 0
    picks = steady[:: max(1, len(steady) // sample)][:sample]
    for i in picks:
        sv = hosc.Solver(steady_params(hosc, W, trace[i], W["precision"]))
        sv.init_fields(trace[i]["seed"], W["noise"])
        info = sv.run_to_steady(1e-8, 30000)
        d = sv.diagnostics(arrays=False)
        sv.close()
        same += int(info.step == res[i]["steps"] and d == res[i]["diag"])
    out["mix_vs_alone"] = {"sampled": len(picks), "bitwise_equal": same}
    return out


def batch_leg(hosc, torch, seg=20, k=24):
    """Batched form, two views.  (a) The 12-cavity batch (sizes 33^3/65^3/97^3, the
    (Ra, n) grid, FP32 refined, autotuned schedule): one segment of `seg` steps from
    the seeded start with fused launches against the same steps cavity by cavity,
    and the largest difference of the results (0 = bitwise).  (b) Solves: the k
    small requests of the serving trace as one batch marched to res 1e-8
    (hosc_batch_run_to_steady, FP32 refined), solves/s and steps against each
    cavity's own run."""
    import numpy as np
    from paper_2411_06563_amd.inputs import batched_cavities
    W4 = WORKLOADS["batch12"]
    cavs = batched_cavities(4)
    plist = [hosc.params(c["N"], Ra=c["Ra"], n_pl=c["n_pl"], Pr=W4["Pr"],
                         dt=max(W4["dt"], W4["dt_over_h2"] / (c["N"] - 1) ** 2), solve_rtol=W4["solve_rtol"],
                         precision=W4["precision"]) for c in cavs]
    seeds = [c["seed"] for c in cavs]
    b = hosc.Batch(plist)
    b.init_fields(seeds, W4["noise"])
    grid = b.tune()
    b.init_fields(seeds, W4["noise"])
    b.step(2)                                   # captures the graphs of both level parities
    b.init_fields(seeds, W4["noise"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(seg)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    got = [cv.get_state() for cv in b.cavities]
    b.close()
    t_serial, worst = 0.0, 0.0
    for i, p in enumerate(plist):
        s = hosc.Solver(p)
        s.init_fields(seeds[i], W4["noise"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(seg)
        torch.cuda.synchronize()
        t_serial += time.perf_counter() - t0
        g = s.get_state()
        s.close()
        worst = max(worst, max(float(np.max(np.abs(g[f] - got[i][f]))) for f in ("u", "v", "w", "T", "p")))
    M3 = sum((c["N"] - 2) ** 3 for c in cavs)
    out = {"cavities": len(cavs), "segment_steps": seg, "tuned_grid": grid,
           "batched_cavity_steps_per_s": len(cavs) * seg / t_batch,
           "one_by_one_cavity_steps_per_s": len(cavs) * seg / t_serial,
           "batched_cell_updates_per_s": M3 * seg / t_batch, "speedup": t_serial / t_batch,
           "max_abs_diff_vs_single_cavity": worst}
    W5 = WORKLOADS["serve"]
    trace = steady_requests(W5, k)
    pl = [steady_params(hosc, W5, r, W5["precision"]) for r in trace]
    b = hosc.Batch(pl)
    b.init_fields([r["seed"] for r in trace], W5["noise"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, err = b.run_to_steady(1e-8, 30000, raise_on_error=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    steady = [i for i, inf in enumerate(infos) if inf.status == 0 and max(inf.res) < 1e-8]
    failed = [i for i, inf in enumerate(infos) if inf.status != 0]
    done = [i for i in steady]
    b.close()
    # each sampled steady cavity's own run (same precision) takes the same steps to the same residual
    picks = steady[:: max(1, len(steady) // 4)][:4]
    same = 0
    for i in picks:
        s = hosc.Solver(pl[i])
        s.init_fields(trace[i]["seed"], W5["noise"])
        si = s.run_to_steady(1e-8, 30000)
        same += int(si.step == infos[i].step and si.res == infos[i].res)
        s.close()
    out["to_steady"] = {"requests": k, "res_tol": 1e-8, "steady": len(done), "failed": len(failed), "wall_s": wall,
                        "solves_per_s": len(done) / wall, "first_error": None if err is None else str(err),
                        "sampled": len(picks), "sampled_same_as_alone": same}
    print(f"batch leg: {out}", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=120)
    ap.add_argument("--warmup", type=int, default=12)
    ap.add_argument("--segment", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--omega", type=float, default=None)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="fp64")
    ap.add_argument("--requests", type=int, default=None)
    ap.add_argument("--capacity", type=int, default=40,
                    help="serve: requests of the saturated-queue comparison (0 = skip)")
    ap.add_argument("--steady", type=int, default=24,
                    help="serve: small requests marched to steady state, served and plain (0 = skip)")
    ap.add_argument("--capacity-rtol", type=float, default=None,
                    help="serve: implicit-solve tolerance of the saturated-queue comparison (default: the workload's)")
    ap.add_argument("--serving", type=int, default=24,
                    help="default workload: small trace requests of the time-to-steady serving leg (0 = skip)")
    ap.add_argument("--batch-steady", type=int, default=24,
                    help="default workload: small trace requests of the batched time-to-steady leg (0 = skip the "
                         "batch object)")
    ap.add_argument("--max-steps", type=int, default=None,
                    help="serve: step cap of each replayed request (default: the workload's 200)")
    ap.add_argument("--first", type=int, default=0,
                    help="serve: first request of the replayed segment of the trace (its clock starts there)")
    ap.add_argument("--sample", type=int, default=None,
                    help="serve: served requests rerun alone for the mix-vs-alone check (default 20)")
    ap.add_argument("--to-steady", action="store_true",
                    help="serve: march every replayed request to res 1e-8 with the viscosity relaxation "
                         "(use with a large --max-steps)")
    ap.add_argument("--stream-grid", type=int, default=257,
                    help="default workload: grid of the HBM-streaming half-sweep measurement (0 = skip)")
    ap.add_argument("--pcie", type=int, default=1,
                    help="1: also time the segment with its state handed over through host memory")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the HOSC hot path is measured on one MI355X "
              "(sharding across GPUs is a design note, not a measured mode)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2411_06563_amd import hosc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    W = WORKLOADS[args.workload]
    if W.get("kind") == "batch":
        return bench_batch(args, W, hosc, torch)
    if W.get("kind") == "serve":
        return bench_serve(args, W, hosc, torch)
    if W.get("kind") == "sizes":
        return bench_sizes(args, W, hosc, torch)
    if args.segment is None:
        args.segment = W.get("segment", SEGMENT)
    kw = dict(Ra=W["Ra"], n_pl=W["n_pl"], Pr=W["Pr"], dt=W["dt"], solve_rtol=W["solve_rtol"],
              precision=W["precision"])
    if args.omega is not None:
        kw["omega"] = args.omega
    if W.get("p_iters"):
        kw["p_iters"] = W["p_iters"]
    start = None
    if W.get("newtonian_start"):
        w = hosc.Solver(hosc.params(W["N"], **dict(kw, n_pl=1.0, precision=0)), device="cuda:0")
        w.init_fields(W["seed"], W["noise"])
        w.step(W["newtonian_start"])
        start = w.get_state()
        w.close()
    s = hosc.Solver(hosc.params(W["N"], **kw), device="cuda:0")

    def reset(solver):
        if start is None:
            solver.init_fields(W["seed"], W["noise"])
        else:
            solver.set_state(**start, apply_bc=False)

    reset(s)

    def one_step():
        info = s.step(1)
        s.diagnostics(arrays=False)
        return info

    in_segment = 0
    for _ in range(args.warmup):
        if in_segment == args.segment:
            reset(s)
            in_segment = 0
        one_step()
        in_segment += 1
    reset(s)
    in_segment = 0
    s.perf_enable(True)
    torch.cuda.synchronize()
    el = 0.0
    sweeps = [0, 0, 0, 0]
    corrections = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        if in_segment == args.segment:
            torch.cuda.synchronize()
            el += time.perf_counter() - t0
            reset(s)
            in_segment = 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        info = one_step()
        in_segment += 1
        sweeps[0] += info.sweeps[0]
        sweeps[1] += info.sweeps[1]
        sweeps[2] += info.bicg_iters[0]
        sweeps[3] += info.bicg_iters[1]
        corrections += info.corrected
        print(f"step {info.step}: sweeps {info.sweeps} bicg {info.bicg_iters} omega "
              f"{info.omega[0]:.3f}/{info.omega[1]:.3f} dominance {info.dominance[0]:.3f}/{info.dominance[1]:.3f} "
              f"res {max(info.res):.3e}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el += time.perf_counter() - t0
    perf = s.perf()
    s.perf_enable(False)
    M3 = (W["N"] - 2) ** 3
    value = M3 * args.steps / el
    # dominant kernel: the red-black half-sweep, or BiCGSTAB if it took longer
    kind = "sweep" if perf["sweep_ms"] >= perf["bicg_ms"] else "bicg"
    kname = "k_sweep (red-black SOR half-sweep)" if kind == "sweep" else "k_bicg (BiCGSTAB phase)"
    avg_ms = perf[f"{kind}_ms"] / max(perf[f"{kind}_launches"], 1)
    avg_bytes = perf[f"{kind}_bytes"] / max(perf[f"{kind}_launches"], 1)
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if W["precision"] == 0 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{W['label']}; steps 1-{args.segment} from the start state, repeated",
                   "grid": W["N"], "interior_nodes": M3, "precision": args.workload, "segment_steps": args.segment,
                   "mean_sor_sweeps_per_step": [sweeps[0] / args.steps, sweeps[1] / args.steps],
                   "mean_bicgstab_iters_per_step": [sweeps[2] / args.steps, sweeps[3] / args.steps],
                   "p_iters": W.get("p_iters", 1), "mean_pressure_corrections_per_step": corrections / args.steps},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": sweep_traffic() if kind == "sweep" and args.workload == "fp64" else None,
                     "avg_launch_us": avg_ms * 1e3, "launches": perf[f"{kind}_launches"],
                     "bytes_per_launch": avg_bytes,
                     "kernel_time_frac": perf[f"{kind}_ms"] * 1e-3 / el,
                     "assemble_GBs": (perf["assemble_bytes"] / max(perf["assemble_ms"], 1e-12) / 1e6),
                     "assemble_us": perf["assemble_ms"] * 1e3 / max(perf["assemble_launches"], 1),
                     "refine_us": perf["refine_ms"] * 1e3 / max(perf["refine_launches"], 1),
                     "refine_time_frac": perf["refine_ms"] * 1e-3 / el},
    }
    if args.workload == "fp64" and args.pcie:
        out["pcie_inclusive"] = pcie_inclusive(s, reset, torch, M3, args.segment)
    s.close()
    if W["precision"] != 0:
        out["precision_check"] = precision_check(hosc, W, kw, reset, args.segment)
    if W.get("p_iters"):
        out["steady_comparison"] = steady_comparison(hosc, torch)
    # the whole step against the HBM roofline: the algorithmic bytes of every kernel
    # of the step (sweeps, BiCGSTAB and refinement as timed, the assembly, and per
    # interior node 32 B viscosity, 72 B sources, 88 B update, 40 B divergence and
    # pressure, 40 B entropy pass) over the measured time per step
    step_bytes = (perf["sweep_bytes"] + perf["bicg_bytes"] + perf["refine_bytes"] + perf["assemble_bytes"]) / args.steps \
        + OTHER_BYTES_PER_NODE * M3
    step_gbs = step_bytes / (el / args.steps) / 1e9
    out["roofline"]["step"] = {"bytes_per_step": step_bytes, "achieved": step_gbs, "frac": step_gbs / HBM_PEAK_GBS}
    out["roofline"]["copy_probe_GBs"] = hosc.copy_bandwidth(1 << 30, 10)
    if args.workload == "fp64":
        mix = mix_probe(hosc, W["N"])
        out["roofline"]["mix_probe_GBs"] = mix
        out["roofline"]["frac_of_mix_probe"] = out["roofline"]["achieved"] / mix
    if args.workload == "fp64" and args.stream_grid > 0:
        out["roofline"]["hbm_streaming"] = stream_sweep(hosc, torch, W, args.stream_grid)
    if args.workload == "fp64" and args.serving > 0:
        out["serving"] = serve_steady(hosc, WORKLOADS["serve"], args.serving)
    if args.workload == "fp64" and args.batch_steady > 0:
        out["batch"] = batch_leg(hosc, torch, k=args.batch_steady)
    if not args.no_cpu_baseline and args.workload == "fp64":
        out["cpu_baseline"] = cpu_baseline(args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
