"""Batched form: many cavities of different sizes and parameters advanced together
by fused solver launches (hosc_batch_*).  Every cavity must give the same result
as its single-cavity run: the fused kernels compute each tile exactly as the
single-cavity launch computes the block with the same index, and the solver
control is shared, so the comparison is bitwise.  From the second step on, the
phases around the solves replay captured graphs, with the eager fused solves and
host synchronisations between the replays; the sweep counts of every step and the
final fields and diagnostics are compared."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# (N, Ra, n, dt): mixed sizes, a ragged colour-row tail (even and odd N), shear
# thinning and thickening; all stable over the steps below
CASES = [(17, 1e3, 1.0, 1e-4), (20, 1e4, 0.75, 1e-4), (11, 1e4, 1.25, 5e-4), (33, 1e4, 1.25, 2e-4),
         (18, 1e5, 0.75, 5e-5)]
SEEDS = [11, 12, 13, 14, 15]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hosc():
    import torch
    assert torch.cuda.is_available()
    from paper_2411_06563_amd import hosc as h
    return h


def _plist(hosc, precision, **kw):
    return [hosc.params(N, Ra=Ra, n_pl=n, Pr=1.0, dt=dt, precision=precision, solve_rtol=1e-11, **kw)
            for (N, Ra, n, dt) in CASES]


def _solo(hosc, p, seed, steps):
    s = hosc.Solver(p)
    s.init_fields(seed, 1e-3)
    infos = [s.step(1) for _ in range(steps)]
    g = s.get_state()
    d = s.diagnostics(arrays=False)
    s.close()
    return g, d, infos


def _compare(hosc, precision, grid, steps=12, tune=False):
    plist = _plist(hosc, precision)
    b = hosc.Batch(plist)
    b.init_fields(SEEDS)
    if tune:
        grid = b.tune()
        say(f"[batch] tuned grid {grid}")
    elif grid is not None:
        b.set_grid(grid)
    binfo = [b.step(1) for _ in range(steps)]
    # steps 2..12 replay the captured pre- and post-solve phases (two each per step)
    say(f"[batch] graph launches {b.graph_launches()}")
    assert b.graph_launches() == 2 * (steps - 1)
    for i, p in enumerate(plist):
        g, d, infos = _solo(hosc, p, SEEDS[i], steps)
        gb = b.cavities[i].get_state()
        db = b.cavities[i].diagnostics(arrays=False)
        sweeps_b = [bi[i].sweeps for bi in binfo]
        sweeps_s = [si.sweeps for si in infos]
        same = all(np.array_equal(gb[f], g[f]) for f in ("u", "v", "w", "T", "p"))
        worst = max(float(np.max(np.abs(gb[f] - g[f]))) for f in ("u", "v", "w", "T", "p"))
        say(f"[batch] prec {precision} grid {grid} cavity {i} N={p.N}: bitwise {same}, max abs diff {worst:.3e}, "
            f"sweeps batch {sweeps_b[-1]} solo {sweeps_s[-1]}")
        assert sweeps_b == sweeps_s
        assert same, (i, worst)
        assert db == d
    b.close()


@pytest.mark.parametrize("grid", [None, 256, 0])
def test_batch_fp64_bitwise_equal_to_solo(hosc, grid):
    say(f"[batch] FP64, {len(CASES)} cavities, grid {grid}")
    _compare(hosc, hosc.HOSC_FP64, grid)


def test_batch_fp32_refined_bitwise_equal_to_solo(hosc):
    say(f"[batch] FP32 refined, {len(CASES)} cavities")
    _compare(hosc, hosc.HOSC_FP32_REFINED, None)


def test_batch_tuned_schedule_bitwise_equal_to_solo(hosc):
    say("[batch] autotuned schedule")
    _compare(hosc, hosc.HOSC_FP64, None, tune=True)


def test_batch_failure_is_isolated(hosc):
    """One cavity forced to fail from the host (SOR only, one sweep allowed) is
    reported by index; the other cavities' steps complete as if alone."""
    say("[batch] failure isolation")
    plist = _plist(hosc, hosc.HOSC_FP64)
    bad = 2
    plist[bad] = hosc.params(CASES[bad][0], Ra=CASES[bad][1], n_pl=CASES[bad][2], Pr=1.0, dt=CASES[bad][3],
                             solve_rtol=1e-11, solver=hosc.SOLVER_SOR, solve_maxit=1)
    b = hosc.Batch(plist)
    b.init_fields(SEEDS)
    with pytest.raises(hosc.HoscError) as e:
        b.step(1)
    say(f"[batch] error: {e.value}")
    assert f"cavity {bad}" in str(e.value)
    for i, p in enumerate(plist):
        if i == bad:
            continue
        g, _, _ = _solo(hosc, p, SEEDS[i], 1)
        gb = b.cavities[i].get_state()
        assert all(np.array_equal(gb[f], g[f]) for f in ("u", "v", "w", "T", "p")), i
    b.close()


def test_batch_benchmark_sizes_bitwise_equal_to_solo(hosc):
    """The batch benchmark's cavity sizes (97^3, 65^3, 33^3), FP32 refined, in the
    benchmark's launch configuration (autotuned schedule, graph-captured phases on
    side streams): four steps bitwise equal to each cavity alone."""
    cases = [(97, 1e5, 1.0), (65, 1e3, 1.25), (33, 1e4, 0.75)]
    plist = [hosc.params(N, Ra=Ra, n_pl=n, Pr=1.0, dt=max(5e-5, 0.2 / (N - 1) ** 2), precision=hosc.HOSC_FP32_REFINED,
                         solve_rtol=1e-10) for (N, Ra, n) in cases]
    seeds = [100, 101, 102]
    b = hosc.Batch(plist)
    b.init_fields(seeds)
    grid = b.tune()
    steps = 4
    for _ in range(steps):
        b.step(1)
    say(f"[batch] benchmark sizes, tuned grid {grid}, graph launches {b.graph_launches()}")
    assert b.graph_launches() == 2 * (steps - 1)
    for i, p in enumerate(plist):
        g, d, _ = _solo(hosc, p, seeds[i], steps)
        gb = b.cavities[i].get_state()
        worst = max(float(np.max(np.abs(gb[f] - g[f]))) for f in ("u", "v", "w", "T", "p"))
        say(f"[batch] N={p.N}: max abs diff {worst:.3e}")
        assert worst == 0.0, i
        assert b.cavities[i].diagnostics(arrays=False) == d
    b.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_with_relaxation_bitwise_equal_to_solo(hosc, precision):
    """Cavities with different viscosity relaxation factors in one batch (the relaxed
    viscosity is formed in the graph-captured entropy pass of each cavity): each
    cavity's fields, diagnostics and sweep counts equal its single-cavity run
    bitwise."""
    relax = [1.0, 0.3, 0.5, 0.7, 0.2]
    plist = [hosc.params(N, Ra=Ra, n_pl=n, Pr=1.0, dt=dt, precision=precision, solve_rtol=1e-11, eta_relax=r)
             for (N, Ra, n, dt), r in zip(CASES, relax)]
    steps = 10
    b = hosc.Batch(plist)
    b.init_fields(SEEDS)
    binfo = [b.step(1) for _ in range(steps)]
    assert b.graph_launches() == 2 * (steps - 1)
    for i, p in enumerate(plist):
        g, d, infos = _solo(hosc, p, SEEDS[i], steps)
        gb = b.cavities[i].get_state()
        for f in ("u", "v", "w", "T", "p"):
            assert np.array_equal(gb[f], g[f]), (i, f)
        assert b.cavities[i].diagnostics(arrays=False) == d
        assert [bi[i].sweeps for bi in binfo] == [si.sweeps for si in infos]
        say(f"[batch relax] precision {precision} cavity {i} r={relax[i]}: bitwise equal")
    b.close()


def test_batch_run_to_steady_equals_single_runs(hosc):
    """hosc_batch_run_to_steady: each cavity stops at its own steady residual (or
    step cap) and ends bitwise where hosc_run_to_steady alone ends, with the same
    number of steps, although the cavities finish at different steps."""
    cases = [(9, 1e3, 1.0, 2e-3), (11, 2e3, 0.8, 1e-3), (12, 5e2, 1.2, 2e-3)]
    plist = [hosc.params(N, Ra=Ra, n_pl=n, Pr=1.0, dt=dt, solve_rtol=1e-11) for (N, Ra, n, dt) in cases]
    seeds = [21, 22, 23]
    tol, cap = 1e-6, 3000
    say("[batch-steady] 3 cavities to res < 1e-6")
    b = hosc.Batch(plist)
    b.init_fields(seeds)
    binfo = b.run_to_steady(tol, cap)
    steps = []
    for i, p in enumerate(plist):
        s = hosc.Solver(p)
        s.init_fields(seeds[i], 1e-3)
        si = s.run_to_steady(tol, cap)
        g = s.get_state()
        gb = b.cavities[i].get_state()
        say(f"[batch-steady] cavity {i}: steps batch {binfo[i].step} solo {si.step}, res {max(binfo[i].res):.2e}")
        assert binfo[i].step == si.step and max(si.res) < tol
        assert binfo[i].res == si.res
        for f in ("u", "v", "w", "T", "p"):
            assert np.array_equal(gb[f], g[f]), (i, f)
        steps.append(si.step)
        s.close()
    assert len(set(steps)) == 3        # they really finish at different steps
    with pytest.raises(hosc.HoscError) as ei:
        b.run_to_steady(0.0, 10)
    assert ei.value.name == "HOSC_E_ARG"
    b.close()
