"""Pins of the oracle's viscosity relaxation (reading R27, an addition to the
paper's scheme for steady-state marching): the viscosity of level n is
r eta(v^n) + (1 - r) times that of level n-1.  A steady state of the stated scheme
(r = 1) is a fixed point of the relaxed march too, so both marches must reach the
same steady fields; the first step after a state is set has no history and is
unrelaxed; and the relaxation does change the transient (it is not a no-op)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2411_06563_amd import inputs


def _oracle(N, n_pl, r, Ra=1e3, c=0.4):
    h = 1.0 / (N - 1)
    o = O.Oracle(O.Params(N, Ra=Ra, n_pl=n_pl, dt=c * h * h, eta_relax=r, solve_tol=1e-14))
    o.set_state(**inputs.initial_state(N, 3, 1e-3))
    return o


def _march(o, tol=1e-11, maxs=4000):
    for _ in range(maxs):
        i = o.step(1)[0]
        assert i.status == 0
        if max(i.res) < tol:
            return
    raise AssertionError("no steady state")


@pytest.mark.parametrize("N,n_pl", [(11, 0.75), (9, 1.25)])
def test_relaxation_keeps_the_steady_state(N, n_pl):
    a, b = _oracle(N, n_pl, 1.0), _oracle(N, n_pl, 0.5)
    _march(a)
    _march(b)
    for f in ("u", "v", "w", "T"):
        scale = np.max(np.abs(a.a[f]))
        assert np.max(np.abs(a.a[f] - b.a[f])) <= 1e-8 * scale, f


def test_first_step_unrelaxed_and_transient_changed():
    N = 11
    a, b = _oracle(N, 0.75, 1.0, Ra=1e4), _oracle(N, 0.75, 0.5, Ra=1e4)
    a.step(1)
    b.step(1)
    for f in ("u", "v", "w", "T", "p"):
        assert np.array_equal(a.a[f], b.a[f]), f
    a.step(4)
    b.step(4)
    d = max(np.max(np.abs(a.a[f] - b.a[f])) / np.max(np.abs(a.a[f])) for f in ("u", "v", "w"))
    assert d > 1e-6



def test_relaxation_continuous_at_one():
    """The weight r belongs to the new viscosity: the relaxed march is continuous in
    r at r = 1, its departure from the stated scheme shrinking in proportion to
    1 - r (1e-6 and 1e-7 here, a ratio of 10).  With the weights the other way round
    the viscosity would stay frozen near its previous level for r near 1 and the
    march would depart by the size of the flow's change whatever 1 - r is."""
    N = 11
    a = _oracle(N, 0.75, 1.0, Ra=1e4)
    a.step(6)
    d = []
    for eps in (1e-6, 1e-7):
        b = _oracle(N, 0.75, 1.0 - eps, Ra=1e4)
        b.step(6)
        d.append(max(np.max(np.abs(a.a[f] - b.a[f])) / np.max(np.abs(a.a[f])) for f in ("u", "v", "w", "T")))
    assert 0.0 < d[1] < 1e-3, d
    assert 8.0 <= d[0] / d[1] <= 12.0, d
