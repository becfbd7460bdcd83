"""Degenerate and failing calls through the C ABI: no state yet, zero steps, bad
counts and coordinates, and a non-finite state, which the library turns into
HOSC_E_NONFINITE (sticky until a new state is set).  Every failure here is forced
from the host through the inputs; every kernel runs to completion."""
import sys

import numpy as np
import pytest

from paper_2411_06563_amd.inputs import initial_state

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hosc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2411_06563_amd import hosc as h
    return h


def _err(hosc, fn):
    with pytest.raises(hosc.HoscError) as e:
        fn()
    return e.value.name


def test_calls_before_a_state(hosc):
    s = hosc.Solver(hosc.params(9, Ra=1e3, dt=1e-3))
    assert _err(hosc, lambda: s.step(1)) == "HOSC_E_STATE"
    assert _err(hosc, lambda: s.run_to_steady(1e-8, 10)) == "HOSC_E_STATE"
    assert _err(hosc, lambda: s.diagnostics(arrays=False)) == "HOSC_E_STATE"
    assert _err(hosc, lambda: s.probe([(0.5, 0.5, 0.5)])) == "HOSC_E_STATE"
    s.close()


def test_zero_steps_and_bad_arguments(hosc):
    N = 9
    s = hosc.Solver(hosc.params(N, Ra=1e3, dt=1e-3, solve_rtol=1e-11))
    s.init_fields(3, 1e-3)
    g0 = s.get_state()
    s.step(0)
    s.run_to_steady(1e-8, 0)
    g1 = s.get_state()
    for f in g0:
        assert np.array_equal(g0[f], g1[f]), f
    assert _err(hosc, lambda: s.step(-1)) == "HOSC_E_ARG"
    assert _err(hosc, lambda: s.run_to_steady(1e-8, -1)) == "HOSC_E_ARG"
    assert _err(hosc, lambda: s.run_to_steady(0.0, 5)) == "HOSC_E_ARG"
    assert _err(hosc, lambda: s.probe(np.zeros((0, 3)))) == "HOSC_E_ARG"
    assert _err(hosc, lambda: s.probe([(0.5, -0.1, 0.5)])) == "HOSC_E_ARG"
    assert _err(hosc, lambda: s.probe(np.full((N ** 3 // 8 + 1, 3), 0.5))) == "HOSC_E_ARG"
    with pytest.raises(ValueError):
        s.set_state(u=np.zeros(10))
    # the failed calls left the state alone: one step still matches a fresh solver's
    info = s.step(1)
    t = hosc.Solver(hosc.params(N, Ra=1e3, dt=1e-3, solve_rtol=1e-11))
    t.init_fields(3, 1e-3)
    t.step(1)
    a, b = s.get_state(), t.get_state()
    for f in a:
        assert np.array_equal(a[f], b[f]), f
    assert info.status == 0
    s.close()
    t.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_non_finite_state_is_reported_and_sticky(hosc, precision):
    N = 11
    s = hosc.Solver(hosc.params(N, Ra=1e4, n_pl=0.75, dt=5e-4, solve_rtol=1e-11, precision=precision))
    st = initial_state(N, 4, 1e-3)
    st["u"] = st["u"].copy()
    st["u"][5, 5, 5] = np.nan
    s.set_state(**st)
    assert _err(hosc, lambda: s.step(1)) == "HOSC_E_NONFINITE"
    assert _err(hosc, lambda: s.step(1)) == "HOSC_E_STATE"
    assert _err(hosc, lambda: s.run_to_steady(1e-8, 5)) == "HOSC_E_STATE"
    s.set_state(**initial_state(N, 4, 1e-3))
    info = s.step(2)
    assert info.status == 0
    g = s.get_state()
    assert all(np.all(np.isfinite(g[f])) for f in g)
    say(f"[edge] precision {precision}: NaN reported, sticky, cleared by a new state")
    s.close()


def test_binding_works_without_importing_torch_first():
    """A script that imports only the binding: the library must bind to the device
    runtime that torch (which provides the workspace) uses, whatever the order in
    which the two are first loaded."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("from paper_2411_06563_amd import hosc\n"
            "p = hosc.params(9, Ra=1e3, dt=1e-3)\n"
            "s = hosc.Solver(p)\n"
            "s.init_fields(1, 1e-3)\n"
            "print('status', s.step(2).status)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0 and "status 0" in r.stdout, r.stderr[-2000:]


def test_solvers_on_their_own_streams(hosc):
    """Two solvers on caller-made streams (default priority), their steps interleaved,
    give bitwise the results of the same runs on the default stream."""
    import torch
    plist = [hosc.params(13, Ra=1e4, n_pl=0.75, dt=5e-4, solve_rtol=1e-11),
             hosc.params(15, Ra=1e3, n_pl=1.25, dt=1e-3, solve_rtol=1e-11, precision=1)]
    ref = []
    for p, sd in zip(plist, (41, 42)):
        s = hosc.Solver(p)
        s.init_fields(sd, 1e-3)
        s.step(6)
        ref.append(s.get_state())
        s.close()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    solvers = [hosc.Solver(p, stream=st) for p, st in zip(plist, streams)]
    for s, sd in zip(solvers, (41, 42)):
        s.init_fields(sd, 1e-3)
    for _ in range(6):
        for s in solvers:
            assert s.step(1).status == 0
    for s, r in zip(solvers, ref):
        g = s.get_state()
        for f in g:
            assert np.array_equal(g[f], r[f]), f
        s.close()


def test_state_through_caller_and_page_locked_arrays(hosc):
    """get_state into caller arrays (page-locked ones included) equals get_state into
    its own arrays bitwise; a state set from page-locked arrays steps exactly like one
    set from pageable arrays; arrays of the wrong kind are refused before the call."""
    import torch
    N = 11
    say(f"[state arrays] N={N}")
    p = hosc.params(N, Ra=1e4, n_pl=0.75, dt=1e-3)
    st = initial_state(N, 3, 1e-3)
    pin = {f: torch.empty((N, N, N), dtype=torch.float64, pin_memory=True).numpy() for f in st}
    for f in st:
        pin[f][...] = st[f]
    a, b = hosc.Solver(p), hosc.Solver(p)
    a.set_state(**st)
    b.set_state(**pin)
    a.step(3)
    b.step(3)
    ga = a.get_state()
    out = {f: torch.empty((N, N, N), dtype=torch.float64, pin_memory=True).numpy() for f in ga}
    gb = b.get_state(out=out)
    assert gb is out
    for f in ga:
        assert np.array_equal(ga[f], gb[f]), f
    bad = dict(out)
    bad["T"] = np.empty((N, N, N), dtype=np.float32)
    with pytest.raises(ValueError):
        a.get_state(out=bad)
    bad["T"] = np.empty((N, N, N))[:, :, ::-1]
    with pytest.raises(ValueError):
        a.get_state(out=bad)
    a.close()
    b.close()
