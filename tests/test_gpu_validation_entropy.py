"""Validation against the paper's entropy study (Sec. 4.3, Tables 3 and 4; fixture
tests/golden/tables3_4_entropy_bejan.json): steady total entropy generation and
Bejan number on the paper's 51^3 grid at Pr = 1.

The cases that reach a steady residual of 1e-8 under the stated scheme are checked:
the four Newtonian cases and n = 1.25 at Ra = 1e2 (the other shear-thinning and
shear-thickening cases either diverge or settle into a residual near 1e-4 with the
level-n viscosity).  They run together through the server (fused steps, each
retired at its own steady state), dt = 0.4 h^2.

The printed E_total is 1.041 for conduction, where the integral is exactly 1: the
paper's quadrature carries a factor (N/(N-1))^2 = 1.0404 at N = 51 (a node sum over
two directions), so E_total is compared after that factor.  Bars: Be within 1% for
Ra <= 1e4 and 8% at Ra = 1e5; E_total within 3%."""
import json
import os
import sys

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = [(1.0, "1e2"), (1.0, "1e3"), (1.0, "1e4"), (1.0, "1e5"), (1.25, "1e2")]


def test_tables3_4_steady_entropy_and_bejan():
    import torch
    assert torch.cuda.is_available()
    from paper_2411_06563_amd import hosc
    with open(os.path.join(HERE, "golden", "tables3_4_entropy_bejan.json")) as f:
        g = json.load(f)
    N, Pr = g["grid"], g["Pr"]
    dt = 0.4 / (N - 1) ** 2
    srv = hosc.Server(4 << 30, max_resident=len(CASES))
    ids = {}
    for n, ra in CASES:
        p = hosc.params(N, Ra=float(ra), n_pl=n, Pr=Pr, dt=dt, solve_rtol=1e-10)
        ids[srv.submit(p, 7, 1e-3, 1e-8, 20000)] = (n, ra)
    res = {}
    steps = 0
    while len(res) < len(CASES):
        srv.step()
        steps += 1
        for r in srv.poll():
            res[ids[r["id"]]] = r
        if steps % 2000 == 0:
            print(f"[tables3-4] server step {steps}: {len(res)} of {len(CASES)} done", flush=True)
    srv.close()
    factor = (N / (N - 1)) ** 2
    for n, ra in CASES:
        r = res[(n, ra)]
        d = r["diag"]
        be_ref = g["bejan"][str(n)][ra]
        e_ref = g["e_total"][str(n)][ra]
        print(f"[tables3-4] n={n} Ra={ra}: steady {r['steady']} after {r['steps']} steps; Be {d['be_global']:.6f} "
              f"(paper {be_ref}); E_total {d['e_total']:.4f} x {factor:.4f} = {d['e_total'] * factor:.4f} "
              f"(paper {e_ref}); Nu hot/cold {d['nu_mean_hot']:.5f}/{d['nu_mean_cold']:.5f}", flush=True)
        assert r["status"] == 0 and r["steady"], r
        tol = 0.08 if ra == "1e5" else 0.01
        assert abs(d["be_global"] - be_ref) <= tol * be_ref
        assert abs(d["e_total"] * factor - e_ref) <= 0.03 * e_ref
        assert abs(d["nu_mean_hot"] - d["nu_mean_cold"]) <= 1e-4 * d["nu_mean_hot"]


# shear-thinning and shear-thickening cases that reach steady state with the
# viscosity relaxation (eta_relax; the steady state is that of the stated scheme)
RELAXED = [(0.75, "1e2", 0.1), (0.75, "1e3", 0.1), (0.75, "1e4", 0.1), (1.25, "1e3", 0.5), (1.25, "1e4", 0.5),
           (1.25, "1e5", 0.5)]


def test_tables3_4_relaxed_non_newtonian():
    """The non-Newtonian cases of Tables 3-4 that the stated scheme cannot settle
    (a period-2 oscillation of the lagged viscosity) reach a steady residual of 1e-8
    with the viscosity relaxation.  E_total agrees with the paper to 1% at
    Ra <= 1e3 and 8% at Ra = 1e4, Be to 1% at Ra = 1e2 and for n = 1.25 at Ra = 1e3;
    at higher Ra the paper's Be departs from ours (its E_HT, which equals the mean
    Nusselt number at steady state, would put the shear-thinning Nu below the
    Newtonian one), so those are reported, not asserted."""
    import torch
    assert torch.cuda.is_available()
    from paper_2411_06563_amd import hosc
    with open(os.path.join(HERE, "golden", "tables3_4_entropy_bejan.json")) as f:
        g = json.load(f)
    N, Pr = g["grid"], g["Pr"]
    dt = 0.4 / (N - 1) ** 2
    srv = hosc.Server(6 << 30, max_resident=len(RELAXED))
    ids = {}
    for n, ra, r in RELAXED:
        p = hosc.params(N, Ra=float(ra), n_pl=n, Pr=Pr, dt=dt, solve_rtol=1e-10, eta_relax=r)
        ids[srv.submit(p, 7, 1e-3, 1e-8, 25000)] = (n, ra)
    res = {}
    steps = 0
    while len(res) < len(RELAXED):
        srv.step()
        steps += 1
        for q in srv.poll():
            res[ids[q["id"]]] = q
        if steps % 2000 == 0:
            print(f"[tables3-4 relaxed] server step {steps}: {len(res)} of {len(RELAXED)} done", flush=True)
    srv.close()
    factor = (N / (N - 1)) ** 2
    for n, ra, _ in RELAXED:
        q = res[(n, ra)]
        d = q["diag"]
        be_ref = g["bejan"][str(n)][ra]
        e_ref = g["e_total"][str(n)][ra]
        print(f"[tables3-4 relaxed] n={n} Ra={ra}: steady {q['steady']} after {q['steps']} steps; Be "
              f"{d['be_global']:.6f} (paper {be_ref}); E_total x f {d['e_total'] * factor:.4f} (paper {e_ref}); "
              f"Nu hot/cold {d['nu_mean_hot']:.5f}/{d['nu_mean_cold']:.5f}", flush=True)
        assert q["status"] == 0 and q["steady"], q
        assert abs(d["nu_mean_hot"] - d["nu_mean_cold"]) <= 1e-4 * d["nu_mean_hot"]
        if ra in ("1e2", "1e3"):
            assert abs(d["e_total"] * factor - e_ref) <= 0.01 * e_ref
        elif ra == "1e4":
            assert abs(d["e_total"] * factor - e_ref) <= 0.08 * e_ref
        if ra == "1e2" or (n == 1.25 and ra == "1e3"):
            assert abs(d["be_global"] - be_ref) <= 0.01 * be_ref
