"""Pin: the oracle's iterative solve of the implicit 7-point systems (Sec. 2.2,
BiCGSTAB) equals a brute-force dense LU of the same operator on tiny grids,
including the temperature system whose y/z wall values are eliminated through
the zero-normal-derivative closure, and including an even N."""
import numpy as np
import pytest

from paper_2411_06563_amd.inputs import random_smooth_state


@pytest.mark.parametrize("N,n_pl", [(5, 0.75), (6, 1.25), (7, 1.0), (7, 0.75)])
def test_bicgstab_matches_dense_lu(oracle_lib, N, n_pl):
    orc = oracle_lib
    res = {}
    for dense in (False, True):
        p = orc.Params(N=N, Ra=3e4, n_pl=n_pl, Pr=1.0, dt=2e-3, dense=dense, solve_tol=1e-14)
        o = orc.Oracle(p)
        o.set_state(**random_smooth_state(N, seed=3, amp=5.0))
        infos = o.step(3)
        assert all(i.status == 0 for i in infos)
        res[dense] = o.state()
    for f in ("u", "v", "w", "T", "p"):
        a, b = res[False][f], res[True][f]
        assert np.linalg.norm(a - b) <= 1e-12 * max(np.linalg.norm(b), 1e-300), f


def test_solve_residual_reported(oracle_lib):
    orc = oracle_lib
    p = orc.Params(N=9, Ra=1e4, n_pl=0.75, dt=1e-3, solve_tol=1e-13)
    o = orc.Oracle(p)
    o.set_state(**random_smooth_state(9, seed=5, amp=2.0))
    info = o.step(1)[0]
    assert info.status == 0
    assert max(info.relres) <= 1e-13
