"""Validation of the whole GPU path against numbers the paper prints: the maximum
over z of the hot-wall average Nusselt number for Newtonian natural convection at
Pr = 0.71 on the paper's 51^3 grid (Sec. 3.2, Table 2; fixture in
tests/golden/table2_max_nusselt.json).  The paper reports a deviation of at most
0.99% from two benchmark solutions; its own time step, quadrature and steady-state
test are not stated, so the bar is 2% of the printed value.  Each case is marched
from the seeded initial state to a steady residual of 1e-8; in increment form the
steady state does not depend on dt, so calmer flows use larger steps."""
import json
import os
import sys

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


DT = {1e3: 4e-4, 1e4: 2e-4, 1e5: 8e-5}


def _cases():
    with open(os.path.join(HERE, "golden", "table2_max_nusselt.json")) as f:
        g = json.load(f)
    return [(g["grid"], g["Pr"], c["Ra"], c["present"]) for c in g["cases"]]


@pytest.mark.parametrize("N,Pr,Ra,expected", _cases())
def test_table2_max_nusselt(N, Pr, Ra, expected):
    import torch
    assert torch.cuda.is_available()
    from paper_2411_06563_amd import hosc
    dt = DT[Ra]
    print(f"[table2] N={N} Pr={Pr} Ra={Ra:g} dt={dt}", flush=True)
    s = hosc.Solver(hosc.params(N, Ra=Ra, n_pl=1.0, Pr=Pr, dt=dt, solve_rtol=1e-10))
    s.init_fields(1, 1e-3)
    for _ in range(40):
        info = s.run_to_steady(1e-8, 1000)
        print(f"[table2] step {info.step} res {max(info.res):.3e} sweeps {info.sweeps}", flush=True)
        if max(info.res) < 1e-8:
            break
    assert max(info.res) < 1e-8, info
    d = s.diagnostics(arrays=False)
    print(f"[table2] Ra={Ra:g}: steps {info.step}, max_z Nu_avg {d['nu_max_hot']:.4f} (paper {expected}), "
          f"Nu_mean hot {d['nu_mean_hot']:.5f} cold {d['nu_mean_cold']:.5f}", flush=True)
    assert abs(d["nu_max_hot"] - expected) <= 0.02 * expected
    assert abs(d["nu_mean_hot"] - d["nu_mean_cold"]) <= 1e-4 * d["nu_mean_hot"]
    s.close()
