"""Serving form: requests admitted by HBM budget, kept resident and advanced by
fused steps together with whatever else is resident.  A request's result must
equal its single-cavity run bitwise, however the mix around it changes."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# (N, Ra, n, dt): mixed sizes and parameters, stable over the steps used
REQS = [(17, 1e3, 1.0, 1e-4), (33, 1e4, 1.25, 2e-4), (20, 1e4, 0.75, 1e-4), (11, 1e4, 1.25, 5e-4),
        (33, 1e3, 0.75, 2e-4), (18, 1e5, 0.75, 5e-5), (25, 1e2, 1.1, 2e-4)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hosc():
    import torch
    assert torch.cuda.is_available()
    from paper_2411_06563_amd import hosc as h
    return h


def _solo_diag(hosc, p, seed, steps):
    s = hosc.Solver(p)
    s.init_fields(seed, 1e-3)
    s.step(steps)
    d = s.diagnostics(arrays=False)
    s.close()
    return d


@pytest.mark.parametrize("precision", [0, 1])
def test_server_results_equal_single_cavity_runs(hosc, precision):
    plist = [hosc.params(N, Ra=Ra, n_pl=n, Pr=1.0, dt=dt, solve_rtol=1e-11, precision=precision)
             for (N, Ra, n, dt) in REQS]
    sizes = sorted(hosc.workspace_bytes(p) for p in plist)
    budget = sizes[-1] + sizes[-2] + 4096     # at most two of the large ones at a time: forces queueing
    srv = hosc.Server(budget, max_resident=4)
    steps = [8 + 3 * i for i in range(len(plist))]
    ids = {}
    max_queued = 0
    # staggered submission: two now, the rest one per server step
    for i in range(2):
        ids[srv.submit(plist[i], 200 + i, res_tol=1e-30, max_steps=steps[i])] = i
    nxt = 2
    results = {}
    for _ in range(400):
        if nxt < len(plist):
            ids[srv.submit(plist[nxt], 200 + nxt, res_tol=1e-30, max_steps=steps[nxt])] = nxt
            nxt += 1
        srv.step()
        st = srv.stats()
        max_queued = max(max_queued, st["queued"])
        assert st["in_use"] <= budget
        for r in srv.poll():
            results[ids[r["id"]]] = r
        if len(results) == len(plist):
            break
    st = srv.stats()
    say(f"[server] precision {precision}: {st}; max queued {max_queued}")
    srv.close()
    assert len(results) == len(plist)
    assert max_queued > 0
    for i, p in enumerate(plist):
        r = results[i]
        assert r["status"] == 0, (i, r)
        assert r["steps"] == steps[i] and not r["steady"]
        assert r["t_arrival"] <= r["t_admit"] <= r["t_done"]
        d = _solo_diag(hosc, p, 200 + i, steps[i])
        say(f"[server] request {i} N={p.N}: Nu {r['diag']['nu_mean_hot']:.12f} solo {d['nu_mean_hot']:.12f}")
        assert r["diag"] == d, i


def test_server_steady_completion_and_budget(hosc):
    """Conduction (Ra = 0) relaxes to steady state: the request retires as steady
    after as many steps as the single-cavity run needs.  A request larger than the
    whole budget is refused at submission."""
    p = hosc.params(11, Ra=0.0, n_pl=1.0, Pr=1.0, dt=1e-3, solve_rtol=1e-11)
    srv = hosc.Server(hosc.workspace_bytes(p) + 4096, max_resident=2)
    big = hosc.params(65, Ra=1e3, n_pl=1.0, Pr=1.0, dt=1e-4)
    with pytest.raises(hosc.HoscError) as e:
        srv.submit(big, 1)
    assert "BUDGET" in str(e.value)
    srv.submit(p, 7, res_tol=1e-8, max_steps=5000)
    out = []
    for _ in range(5000):
        srv.step()
        out += srv.poll()
        if out:
            break
    srv.close()
    assert len(out) == 1 and out[0]["status"] == 0 and out[0]["steady"]
    s = hosc.Solver(p)
    s.init_fields(7, 1e-3)
    info = s.run_to_steady(1e-8, 5000)
    d = s.diagnostics(arrays=False)
    s.close()
    say(f"[server] steady after {out[0]['steps']} steps (single-cavity run {info.step})")
    assert out[0]["steps"] == info.step
    assert out[0]["diag"] == d


def test_server_failure_is_isolated(hosc):
    """A request forced to fail from the host (SOR only, one sweep allowed) retires
    with its error; the request resident beside it is unaffected."""
    good = hosc.params(17, Ra=1e3, n_pl=1.0, Pr=1.0, dt=1e-4, solve_rtol=1e-11)
    bad = hosc.params(17, Ra=1e3, n_pl=1.0, Pr=1.0, dt=1e-4, solve_rtol=1e-11, solver=hosc.SOLVER_SOR,
                      solve_maxit=1)
    srv = hosc.Server(4 * hosc.workspace_bytes(good), max_resident=4)
    ig = srv.submit(good, 3, res_tol=1e-30, max_steps=6)
    ib = srv.submit(bad, 4, res_tol=1e-30, max_steps=6)
    res = {}
    for _ in range(20):
        srv.step()
        for r in srv.poll():
            res[r["id"]] = r
        if len(res) == 2:
            break
    srv.close()
    say(f"[server] failure isolation: bad status {res[ib]['status']} after {res[ib]['steps']} steps")
    assert res[ib]["status"] == -4 and res[ib]["steps"] == 0
    assert res[ig]["status"] == 0 and res[ig]["steps"] == 6
    assert res[ig]["diag"] == _solo_diag(hosc, good, 3, 6)


@pytest.mark.parametrize("precision", [0, 1])
def test_server_relaxed_and_iterated_requests_equal_single_runs(hosc, precision):
    """Requests with different viscosity relaxation factors and pressure-iteration
    counts, admitted together and advanced in fused steps: each result's
    diagnostics equal its single-cavity run bitwise."""
    import numpy as np
    specs = [(17, 1e4, 0.75, 5e-4, 0.3, 1), (18, 1e4, 1.25, 5e-4, 0.5, 2), (13, 1e3, 1.0, 1e-3, 1.0, 3),
             (20, 1e4, 0.75, 2e-4, 0.6, 2)]
    plist = [hosc.params(N, Ra=Ra, n_pl=n, Pr=1.0, dt=dt, eta_relax=r, p_iters=K, precision=precision,
                         solve_rtol=1e-11) for (N, Ra, n, dt, r, K) in specs]
    seeds = [31, 32, 33, 34]
    steps = 8
    solo = []
    for p, sd in zip(plist, seeds):
        s = hosc.Solver(p)
        s.init_fields(sd, 1e-3)
        s.step(steps)
        solo.append(s.diagnostics(arrays=False))
        s.close()
    srv = hosc.Server(1 << 28, max_resident=4)
    ids = {srv.submit(p, sd, res_tol=1e-30, max_steps=steps): i for i, (p, sd) in enumerate(zip(plist, seeds))}
    res = {}
    for _ in range(100):
        srv.step()
        for r in srv.poll():
            res[ids[r["id"]]] = r
        if len(res) == len(plist):
            break
    srv.close()
    for i in range(len(plist)):
        assert res[i]["status"] == 0 and res[i]["steps"] == steps, res[i]
        assert res[i]["diag"] == solo[i], i
    assert np.isfinite(solo[0]["nu_mean_hot"])
