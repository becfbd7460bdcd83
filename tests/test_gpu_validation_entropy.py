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


# every case with a steady state (n = 0.75 at Ra = 1e5 diverges under the stated
# scheme); the relaxation factor of each (1: the stated scheme, which settles the
# Newtonian cases and n = 1.25 at Ra = 1e2, where r = 0.5 keeps the rest-state
# viscosity long enough to lose the rows at start-up)
SETTLED = [(0.75, "1e2", 0.1), (0.75, "1e3", 0.1), (0.75, "1e4", 0.1), (1.0, "1e2", 1.0), (1.0, "1e3", 1.0),
           (1.0, "1e4", 1.0), (1.0, "1e5", 1.0), (1.25, "1e2", 1.0), (1.25, "1e3", 0.5), (1.25, "1e4", 0.5),
           (1.25, "1e5", 0.5)]


def test_nusselt_and_entropy_trends():
    """The paper's statements on its local and z-averaged Nusselt figures (Sec. 4.2),
    on the eleven steady states of the 51^3 study: Nu_local on the hot wall is nearly
    symmetric about y = 1/2 at Ra = 1e2 and grows asymmetric as Ra rises; its maximum
    rises with Ra at fixed n and falls as n rises at fixed Ra; Nu_avg(z) falls as n
    rises and rises with Ra, at every interior z; for Ra <= 1e4 Nu_avg(z) rises from
    the wall to a global maximum around z = 1/2 (within 0.1: for n = 0.75 at
    Ra = 1e4 the top is flat, with twin maxima at z = 0.46 and 0.54 that exceed the
    centre by 6e-6) and falls beyond it; at Ra = 1e2 the effect of n is small (the
    spread of max Nu_local over n is under 5% of the spread at Ra = 1e4) and the
    asymmetry about y = 1/2 is under a quarter of that at Ra = 1e3.  The paper's
    double peak of Nu_avg(z) at Ra = 1e5 is for n = 0.75, which diverges here.
    And its statements on entropy generation (Sec. 4.3): the largest local entropy
    generation and E_total rise with Ra and fall as n rises, E_total nearly
    independent of n at Ra = 1e2; entropy concentrates near the thermally active
    walls as Ra rises; E_local keeps the near-diagonal (half-turn) symmetry; Be falls
    with Ra, stays above 1/2 at Ra = 1e4 for n = 1 and 1.25 and falls below it at
    Ra = 1e5.  (The paper's Be below 1/2 for n = 0.75 at Ra = 1e4 is the departure
    of its Table 4, reported, not asserted.)  The rise of the largest local Nusselt
    number on the hot wall from Ra = 1e2 to 1e5 that the text gives (Sec. 4.2: 729 %
    for n = 1 and 385 % for n = 1.25; its 1948 % for n = 0.75 needs the Ra = 1e5 case
    that diverges here) is matched to 5 % of the printed rise (710 % and 402 % here).
    Both readings of the Bejan number (R18: ratio of the integrals, and volume mean
    of the local ratio) are compared with Table 4: the ratio of the integrals is the
    closer one (median gap 0.6 % against 3.5 % over the eleven cases)."""
    import numpy as np
    import torch
    assert torch.cuda.is_available()
    from paper_2411_06563_amd import hosc
    N = 51
    dt = 0.4 / (N - 1) ** 2
    out = {}
    for n, ra, r in SETTLED:
        s = hosc.Solver(hosc.params(N, Ra=float(ra), n_pl=n, Pr=1.0, dt=dt, solve_rtol=1e-10, eta_relax=r))
        s.init_fields(7, 1e-3)
        while True:
            info = s.run_to_steady(1e-8, 2500)
            assert info.status == 0 and info.step <= 30000, (n, ra, info)
            if max(info.res) < 1e-8:
                break
        d = s.diagnostics(arrays=True)
        nuh, avg = d["nu_hot"], d["nuavg_hot"]            # nu_hot indexed [k, j]
        asym = float(np.abs(nuh - nuh[:, ::-1]).max() / nuh.max())
        el, _ = s.entropy_fields()                          # E_local, indexed [k, j, i]
        emax = float(el.max())
        turn = float(np.abs(el - el[:, ::-1, ::-1]).max()) / emax
        near = (el[:, :, :6].sum() + el[:, :, -6:].sum()) / el.sum()    # within 0.1 of the x walls
        out[(n, ra)] = dict(nuh=nuh, avg=avg, numax=d["nu_local_max_hot"], asym=asym, emax=emax, turn=turn,
                            near=float(near), etot=d["e_total"], be=d["be_global"], be_mean=d["be_mean"])
        print(f"[Nu trends] n={n} Ra={ra}: steady after {info.step} steps; max Nu_local {d['nu_local_max_hot']:.5f}, "
              f"y-asymmetry {asym:.2e}, Nu_avg(z) centre {avg[N // 2]:.5f} range [{avg[1:-1].min():.5f}, "
              f"{avg[1:-1].max():.5f}]; max E_local {emax:.4f}, E_total {d['e_total']:.4f}, Be {d['be_global']:.4f}, "
              f"Be_mean {d['be_mean']:.6f}, entropy within 0.1 of the x walls {near:.3f}, half-turn asymmetry of "
              f"E_local {turn:.1e}", flush=True)
        s.close()
    ras = ["1e2", "1e3", "1e4", "1e5"]
    for n in (0.75, 1.0, 1.25):
        seq = [out[(n, ra)] for ra in ras if (n, ra) in out]
        for a, b in zip(seq, seq[1:]):
            assert b["numax"] > a["numax"]                                 # max Nu_local rises with Ra
            assert b["asym"] > a["asym"]                                   # asymmetry about y = 1/2 grows
            assert np.all(b["avg"][1:-1] > a["avg"][1:-1])                 # Nu_avg(z) rises with Ra
    for ra in ras:
        seq = [out[(n, ra)] for n in (0.75, 1.0, 1.25) if (n, ra) in out]
        for a, b in zip(seq, seq[1:]):
            assert b["numax"] < a["numax"]                                 # and falls as n rises
            assert np.all(b["avg"][1:-1] < a["avg"][1:-1])
        if ra != "1e5":
            lo, hi = round(0.4 * (N - 1)), round(0.6 * (N - 1))
            for q in seq:
                avg = q["avg"]
                km = int(np.argmax(avg))
                assert lo <= km <= hi                                      # global maximum around z = 1/2
                assert np.all(np.diff(avg[1:lo + 1]) > 0) and np.all(np.diff(avg[hi:-1]) < 0)
    for n in (0.75, 1.0, 1.25):
        a2, a3 = out[(n, "1e2")]["asym"], out[(n, "1e3")]["asym"]
        print(f"[Nu trends] n={n}: y-asymmetry at Ra = 1e2 / 1e3: {a2:.2e} / {a3:.2e}", flush=True)
        assert a2 < 0.25 * a3                                              # nearly symmetric at Ra = 1e2
    spread = {ra: (max(out[(n, ra)]["numax"] for n in (0.75, 1.0, 1.25))
                   - min(out[(n, ra)]["numax"] for n in (0.75, 1.0, 1.25))) for ra in ("1e2", "1e4")}
    print(f"[Nu trends] spread of max Nu_local over n: Ra = 1e2 {spread['1e2']:.4f}, Ra = 1e4 {spread['1e4']:.4f}")
    assert spread["1e2"] < 0.05 * spread["1e4"]                            # n hardly matters at Ra = 1e2
    # Sec. 4.3: local and total entropy generation and the Bejan number
    for n in (0.75, 1.0, 1.25):
        seq = [out[(n, ra)] for ra in ras if (n, ra) in out]
        for a, b in zip(seq, seq[1:]):
            assert b["emax"] > a["emax"] and b["etot"] > a["etot"]        # rise with Ra
            assert b["be"] < a["be"]                                       # Be falls with Ra
            assert b["near"] > a["near"]                                   # entropy moves to the active walls
    for ra in ras:
        seq = [out[(n, ra)] for n in (0.75, 1.0, 1.25) if (n, ra) in out]
        for a, b in zip(seq, seq[1:]):
            assert b["emax"] < a["emax"] and b["etot"] < a["etot"]        # fall as n rises
    # Sec. 4.2: the rise of max Nu_local on the hot wall from Ra = 1e2 to 1e5
    for n, printed in ((1.0, 729.0), (1.25, 385.0)):
        rise = 100.0 * (out[(n, "1e5")]["numax"] / out[(n, "1e2")]["numax"] - 1.0)
        print(f"[Nu trends] n={n}: max Nu_local rises {rise:.1f} % from Ra = 1e2 to 1e5 (paper {printed:.0f} %)",
              flush=True)
        assert abs(rise - printed) <= 0.05 * printed
    # Table 4 against both readings of the Bejan number (R18)
    with open(os.path.join(HERE, "golden", "tables3_4_entropy_bejan.json")) as f:
        tab = json.load(f)["bejan"]
    err = {"global": [], "mean": []}
    for (n, ra), q in sorted(out.items()):
        ref = tab[str(n)][ra]
        err["global"].append(abs(q["be"] - ref) / ref)
        err["mean"].append(abs(q["be_mean"] - ref) / ref)
        print(f"[Be readings] n={n} Ra={ra}: paper {ref:.6f}, Be_global {q['be']:.6f} ({err['global'][-1]:.2%}), "
              f"Be_mean {q['be_mean']:.6f} ({err['mean'][-1]:.2%})", flush=True)
    print(f"[Be readings] median relative gap to Table 4: Be_global {np.median(err['global']):.2%}, "
          f"Be_mean {np.median(err['mean']):.2%}", flush=True)
    # the ratio of the integrals is the reading closer to the printed table
    assert np.median(err["global"]) < np.median(err["mean"])
    et2 = [out[(n, "1e2")]["etot"] for n in (0.75, 1.0, 1.25)]
    assert (max(et2) - min(et2)) / min(et2) < 1e-3                        # E_total nearly equal at Ra = 1e2
    for key in out:
        assert out[key]["turn"] <= 1e-4                                    # near-diagonal (half-turn) symmetry
    assert out[(1.0, "1e4")]["be"] > 0.5 and out[(1.25, "1e4")]["be"] > 0.5
    assert out[(1.0, "1e5")]["be"] < 0.5 and out[(1.25, "1e5")]["be"] < 0.5
    print(f"[Nu trends] Be at Ra = 1e4 for n = 0.75: {out[(0.75, '1e4')]['be']:.4f} (the paper has it below 1/2)")


def test_shear_thinning_ra1e5_branch_by_continuation():
    """At Ra = 1e5 the shear-thinning steady states are reached by continuation in n
    from the Newtonian one on a grid finer than the paper's (65^3, Pr = 1,
    dt = 0.2 h^2, viscosity relaxation 0.1 after the Newtonian stage; from rest they
    diverge, and on 51^3 the branch ends below n = 0.875).  Along the branch n = 1,
    0.9, 0.875, 0.85 the paper's statements hold (Sec. 4.2, 4.3): the mean Nusselt
    number, the largest local Nusselt number on the hot wall and the total entropy
    generation rise as n falls, and max_z Nu_avg with them; each state has the
    hot/cold Nusselt balance of a steady state.  And the double peak of Nu_avg(z)
    that the paper shows for the shear-thinning fluid at Ra = 1e5 (Sec. 4.2, Fig. 9)
    appears along the branch: the Newtonian profile has its single maximum at
    z = 1/2, the shear-thinning ones two local maxima placed symmetrically about
    z = 1/2 with a dip between them that deepens, and maxima that move apart, as n
    falls (dip 0.27 % at n = 0.9 and 1.1 % at n = 0.85 here; 2.5 % at n = 0.8 and
    3.0 % at n = 0.7875 on 129^3)."""
    import numpy as np
    import torch
    assert torch.cuda.is_available()
    from paper_2411_06563_amd import hosc
    N = 65
    dt = 0.2 / (N - 1) ** 2
    state, rows = None, []
    for n in (1.0, 0.9, 0.875, 0.85):
        p = hosc.params(N, Ra=1e5, n_pl=n, Pr=1.0, dt=dt, solve_rtol=1e-10, eta_relax=1.0 if n == 1.0 else 0.1)
        s = hosc.Solver(p)
        if state is None:
            s.init_fields(7, 1e-3)
        else:
            s.set_state(**state)
        info = s.run_to_steady(1e-8, 20000)
        d = s.diagnostics(arrays=True)
        state = s.get_state()
        s.close()
        print(f"[Ra=1e5 branch] n={n}: {info.step} steps, res {max(info.res):.2e}, Nu {d['nu_mean_hot']:.5f}/"
              f"{d['nu_mean_cold']:.5f}, max Nu_local {d['nu_local_max_hot']:.4f}, max Nu_avg {d['nu_max_hot']:.4f}, "
              f"E_total {d['e_total']:.4f}, Be {d['be_global']:.5f}", flush=True)
        assert max(info.res) < 1e-8
        assert abs(d["nu_mean_hot"] - d["nu_mean_cold"]) <= 1e-4 * d["nu_mean_hot"]
        rows.append(d)
    for a, b in zip(rows, rows[1:]):     # n falling
        assert b["nu_mean_hot"] > a["nu_mean_hot"]
        assert b["nu_local_max_hot"] > a["nu_local_max_hot"]
        assert b["nu_max_hot"] > a["nu_max_hot"]
        assert b["e_total"] > a["e_total"]
    # local maxima of Nu_avg(z) over the interior z, and the dip between the outer two
    peaks = []
    for n, d in zip((1.0, 0.9, 0.875, 0.85), rows):
        avg = np.asarray(d["nuavg_hot"])[1:-1]
        mx = [i for i in range(1, len(avg) - 1) if avg[i] > avg[i - 1] and avg[i] >= avg[i + 1]]
        dip = 0.0
        if len(mx) == 2:
            lo = float(avg[mx[0]:mx[1] + 1].min())
            dip = (min(avg[mx[0]], avg[mx[1]]) - lo) / lo
        zs = [(i + 1) / (N - 1) for i in mx]
        print(f"[Ra=1e5 branch] n={n}: Nu_avg(z) local maxima at z = {[round(z, 4) for z in zs]}, dip {dip:.3e}",
              flush=True)
        peaks.append((zs, dip))
    assert peaks[0][0] == [0.5]                                        # Newtonian: one maximum, at z = 1/2
    for zs, dip in peaks[1:]:
        assert len(zs) == 2 and abs(zs[0] + zs[1] - 1.0) < 1e-12 and dip > 1e-3
    for (za, da), (zb, db) in zip(peaks[1:], peaks[2:]):
        assert db > da and zb[0] <= za[0]                              # deeper, and apart, as n falls
