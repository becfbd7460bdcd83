"""Pin: the oracle's HOSC step of the generic transport PDE (Sec. 2.2, Eq. 1 and the
compact scheme of Eq. 5) converges at 4th order in space and 2nd order in time on
a manufactured solution, as the paper claims (abstract; Sec. 2.2).

The solution, L and the convective coefficients are smooth, non-separable and
time dependent, so every term of the scheme (variable L, its time difference, the
cross-derivative terms p1, q1, r1, the bracket operator on the source) is
exercised: a dropped term or a wrong sign drops the observed order to 2 or less.
The source E* is obtained from the PDE by symbolic differentiation (sympy).
"""
import numpy as np
import pytest
import sympy as sp

x, y, z, t = sp.symbols("x y z t")
_CHI = sp.sin(sp.pi * x + t) * sp.sin(sp.pi * y) * sp.cos(sp.pi * z / 2) + sp.Rational(1, 10) * x * y * z
_L = 1 + sp.Rational(1, 2) * sp.sin(x + y + z + t)
_G = 2 * sp.cos(sp.pi * y) * (1 + sp.Rational(1, 5) * t)
_H = sp.Rational(3, 2) * sp.sin(sp.pi * z) * (1 - sp.Rational(3, 10) * t)
_I = -sp.cos(sp.pi * x) * (1 + sp.Rational(1, 10) * t * x)
_E = (_L * sp.diff(_CHI, t) + _G * sp.diff(_CHI, x) + _H * sp.diff(_CHI, y) + _I * sp.diff(_CHI, z)
      - (sp.diff(_CHI, x, 2) + sp.diff(_CHI, y, 2) + sp.diff(_CHI, z, 2)))
_F = {n: sp.lambdify((x, y, z, t), e, "numpy") for n, e in dict(chi=_CHI, L=_L, G=_G, H=_H, I=_I, E=_E).items()}


def _ev(name, X, Y, Z, tt):
    return np.ascontiguousarray(np.broadcast_to(_F[name](X, Y, Z, tt), X.shape).astype(np.float64))


def _run(orc, N, dt, T):
    g = np.linspace(0.0, 1.0, N)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    p = orc.Params(N=N, dt=dt, solve_tol=1e-14)
    nsteps = int(round(T / dt))
    c = _ev("chi", X, Y, Z, 0.0)
    for s in range(nsteps):
        tn = s * dt
        tp = tn - dt if s > 0 else tn          # level n-1 := level n at the first step
        co = {n: _ev(n, X, Y, Z, tn) for n in "LGHIE"}
        cp = {n: _ev(n, X, Y, Z, tp) for n in "LGHIE"}
        walls = _ev("chi", X, Y, Z, tn + dt)
        c, _, _ = orc.transport_step(p, co["L"], co["G"], co["H"], co["I"], co["E"], cp["L"], cp["G"], cp["H"],
                                     cp["I"], cp["E"], c, walls)
    exact = _ev("chi", X, Y, Z, nsteps * dt)
    return np.abs(c - exact)[1:-1, 1:-1, 1:-1].max(), c


def test_space_order_four(oracle_lib):
    T = 0.05
    errs = []
    for N in (9, 17, 33):
        h = 1.0 / (N - 1)
        n = int(np.ceil(T / (0.5 * h * h)))
        errs.append(_run(oracle_lib, N, T / n, T)[0])
    orders = [np.log2(errs[q] / errs[q + 1]) for q in range(2)]
    assert min(orders) >= 3.8, (errs, orders)


def test_time_order_two(oracle_lib):
    N, T = 33, 0.4
    sols = [_run(oracle_lib, N, dt, T)[1] for dt in (0.02, 0.01, 0.005, 0.0025)]
    d = [np.abs(sols[q] - sols[q + 1]).max() for q in range(3)]
    orders = [np.log2(d[q] / d[q + 1]) for q in range(2)]
    assert min(orders) >= 1.9, (d, orders)
