"""Pins of the oracle's pressure iterations (modified artificial compressibility,
Sec. 2.2): within a step, after the momentum equations are solved the largest
|div v| is measured; above the tolerance the pressure is corrected by
p <- p - lambda div v and the momentum equations are solved again with the
pressure of that iteration, from the same level n.

The pins follow from that definition and from the linearity of the step in p:

- an iterated step equals a chain of single-correction steps, each restarted from
  the step's level-n state with the previous iteration's pressure (the last one
  keeps its correction); at the first step the level n-1 sources follow the iterate
  (reading R26);
- the iteration stops at the first solve whose divergence is within the tolerance,
  without correcting after it;
- the momentum increments are affine in the pressure and the energy solve does not
  depend on it;
- more iterations lower the divergence of the accepted velocity (a Richardson
  iteration with a small relaxation lambda = h^2 / (3 dt)).

Dense LU solves make the chain comparisons exact.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2411_06563_amd import inputs

ARRAYS = ("u", "v", "w", "T", "p", "up", "vp", "wp", "etap", "Eup", "Evp", "Ewp")


def _params(N, K, div_tol=0.0, dense=True, **kw):
    base = dict(Ra=1e4, n_pl=0.75, Pr=1.0, dt=5e-4)
    base.update(kw)
    return O.Params(N, div_tol=div_tol, p_iters=K, dense=dense, solve_tol=1e-14, **base)


def _start(N, history, **kw):
    """Level-n state: the seeded rest state, or the state after one step (so that
    level n-1 differs from level n)."""
    o = O.Oracle(_params(N, 1, **kw))
    o.set_state(**inputs.initial_state(N, 31, 1e-2))
    if history:
        o.step(1)
    return {f: o.a[f].copy() for f in ARRAYS}, o.first


def _from(snap, first, params, p=None):
    o = O.Oracle(params)
    for f in ARRAYS:
        o.a[f][...] = snap[f]
    if p is not None:
        o.a["p"][...] = p
    o.first = first
    return o


def _chain(snap, first, N, K, **kw):
    """K single-correction steps, each from the level-n state with the pressure the
    previous one left."""
    p = snap["p"]
    out = []
    for _ in range(K):
        o = _from(snap, first, _params(N, 1, **kw), p)
        info = o.step(1)[0]
        out.append((o, info))
        p = o.a["p"].copy()
    return out


@pytest.mark.parametrize("N,history,K", [(7, False, 3), (8, True, 3), (7, True, 2)])
def test_iterated_step_equals_restarted_single_steps(N, history, K):
    snap, first = _start(N, history)
    it = _from(snap, first, _params(N, K))
    info = it.step(1)[0]
    chain = _chain(snap, first, N, K)
    ref, rinfo = chain[-1]
    assert info.corrected == K
    assert info.maxdiv == rinfo.maxdiv
    for f in ARRAYS:
        assert np.array_equal(it.a[f], ref.a[f]), f
    # the divergence of successive iterates differs: the pressure really changed the solve
    assert chain[0][1].maxdiv != chain[1][1].maxdiv


def test_stops_at_first_solve_within_tolerance():
    N = 8
    snap, first = _start(N, True)
    chain = _chain(snap, first, N, 4)
    m = [c[1].maxdiv for c in chain]
    assert m[2] < m[0] and m[2] < m[1]
    tol = m[2]                       # the third solve is within tolerance (not above it)
    it = _from(snap, first, _params(N, 6, div_tol=tol))
    info = it.step(1)[0]
    assert info.corrected == 2 and info.maxdiv == m[2]
    third = chain[2][0]
    for f in ("u", "v", "w", "T"):
        assert np.array_equal(it.a[f], third.a[f]), f
    # no correction after the accepted solve: p is the pressure that solve used
    assert np.array_equal(it.a["p"], chain[1][0].a["p"])


def test_single_iteration_settings_agree():
    N = 7
    snap, first = _start(N, True)
    a = _from(snap, first, _params(N, 0))
    b = _from(snap, first, _params(N, 1))
    ia, ib = a.step(1)[0], b.step(1)[0]
    assert ia.corrected == ib.corrected == 1
    for f in ARRAYS:
        assert np.array_equal(a.a[f], b.a[f]), f


def test_momentum_affine_in_pressure_energy_independent():
    N = 8
    snap, first = _start(N, True)
    rng = np.random.default_rng(3)
    delta = np.zeros((N, N, N))
    delta[1:-1, 1:-1, 1:-1] = rng.standard_normal((N - 2,) * 3)
    outs = []
    for s in (0.0, 1.0, 2.0):
        o = _from(snap, first, _params(N, 1, div_tol=1e300), snap["p"] + s * delta)
        info = o.step(1)[0]
        assert info.corrected == 0
        outs.append(o)
    for f in ("u", "v", "w"):
        d1 = outs[1].a[f] - outs[0].a[f]
        d2 = outs[2].a[f] - outs[1].a[f]
        assert np.max(np.abs(d1)) > 1e-6                   # the pressure moves the velocity
        assert np.max(np.abs(d2 - d1)) <= 1e-10 * np.max(np.abs(d1)), f
    assert np.array_equal(outs[0].a["T"], outs[2].a["T"])


def test_more_iterations_lower_the_divergence():
    N = 12
    m = []
    for K in (1, 2, 4, 8):
        o = O.Oracle(_params(N, K, dense=False, Ra=1e3, n_pl=1.0, dt=1e-3))
        o.set_state(**inputs.initial_state(N, 7, 1e-3))
        info = o.step(2)
        assert info[-1].corrected == K
        m.append(info[-1].maxdiv)
    assert all(m[i + 1] < m[i] for i in range(3)), m
