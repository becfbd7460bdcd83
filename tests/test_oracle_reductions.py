"""Pins of the oracle's Nusselt (Sec. 4.2) and entropy/Bejan (Sec. 4.3) reductions
on fields whose integrals are known in closed form.

- theta = 1 - x + (x - x^3) q(y, z), q = 0.3 + 0.2 y + 0.1 y^3 + 0.05 z^2: the 5-point
  one-sided difference is exact on this cubic in x, and Simpson is exact on the
  cubic in y and the quadratic in z, so
      Nu_hot(y, z) = 1 - q (largest, 0.7, at y = z = 0),  Nu_cold(y, z) = 1 + 2 q,
      Nu_avg,hot(z) = 0.575 - 0.05 z^2,  Nu_avg,cold(z) = 1.85 + 0.1 z^2.
- theta linear and u = y (1 - y): the gradients are exact, E_HT = |grad theta|^2 is
  constant and E_FF = phi (1 - 2y)^2 at n = 1 integrates to phi/3 (Simpson exact).
- Even N (Simpson with a 3/8 panel) gives the same exact integrals.
"""
import numpy as np
import pytest


@pytest.mark.parametrize("N", [17, 18])
def test_nusselt_exact_polynomial(oracle_lib, N):
    orc = oracle_lib
    g = np.linspace(0, 1, N)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    q = 0.3 + 0.2 * Y + 0.1 * Y ** 3 + 0.05 * Z ** 2
    T = np.ascontiguousarray(1 - X + (X - X ** 3) * q)
    zero = np.zeros_like(T)
    p = orc.Params(N=N)
    d = orc.diagnostics(p, zero, zero, zero, T)
    qw = q[:, :, 0]                       # nu arrays are indexed [k, j]
    assert np.allclose(d["nu_hot"], 1 - qw, rtol=0, atol=1e-11)
    assert np.allclose(d["nu_cold"], 1 + 2 * qw, rtol=0, atol=1e-11)
    assert np.allclose(d["nuavg_hot"], 0.575 - 0.05 * g ** 2, rtol=0, atol=1e-12)
    assert np.allclose(d["nuavg_cold"], 1.85 + 0.1 * g ** 2, rtol=0, atol=1e-12)
    assert abs(d["nu_mean_hot"] - (0.575 - 0.05 / 3)) <= 1e-12
    assert abs(d["nu_mean_cold"] - (1.85 + 0.1 / 3)) <= 1e-12
    assert abs(d["nu_max_hot"] - 0.575) <= 1e-12
    assert abs(d["nu_max_cold"] - 1.95) <= 1e-12
    # largest local Nusselt number on the hot wall: 1 - q is largest where q is
    # smallest, at y = z = 0 (q = 0.3)
    assert abs(d["nu_local_max_hot"] - 0.7) <= 1e-11


@pytest.mark.parametrize("N", [9, 12])
def test_entropy_and_bejan_exact(oracle_lib, N):
    orc = oracle_lib
    g = np.linspace(0, 1, N)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    T = np.ascontiguousarray(0.7 - 0.9 * X + 0.3 * Y - 0.2 * Z)
    u = np.ascontiguousarray(Y * (1 - Y))
    zero = np.zeros_like(T)
    phi = 1e-2
    p = orc.Params(N=N, n_pl=1.0, phi=phi)
    d = orc.diagnostics(p, u, zero, zero, T, fields=True)
    eht = 0.81 + 0.09 + 0.04
    eff = phi / 3.0
    assert abs(d["e_ht"] - eht) <= 1e-13
    assert abs(d["e_ff"] - eff) <= 1e-14
    assert abs(d["e_total"] - (eht + eff)) <= 1e-13
    assert abs(d["be_global"] - eht / (eht + eff)) <= 1e-14
    loc = eht + phi * (1 - 2 * Y) ** 2
    assert np.allclose(d["e_local"], loc, rtol=1e-13, atol=0)
    assert np.allclose(d["be_local"], eht / loc, rtol=1e-13, atol=0)
    # Be_mean: Simpson of eht/(eht + phi (1-2y)^2), compared with a fine quadrature
    yy = np.linspace(0, 1, 200001)
    fine = np.trapezoid(eht / (eht + phi * (1 - 2 * yy) ** 2), yy)
    assert abs(d["be_mean"] - fine) <= 1e-6


def test_entropy_shear_thickening_power(oracle_lib):
    """n = 3 gives eta = I2, E_FF = phi I2^2 = phi (1-2y)^4: Simpson error O(h^4)."""
    orc = oracle_lib
    errs = []
    for N in (17, 33):
        g = np.linspace(0, 1, N)
        Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
        u = np.ascontiguousarray(Y * (1 - Y))
        zero = np.zeros_like(u)
        T = np.ascontiguousarray(1 - X)
        p = orc.Params(N=N, n_pl=3.0, phi=1.0, i2_floor=0.0)
        d = orc.diagnostics(p, u, zero, zero, T)
        errs.append(abs(d["e_ff"] - 0.2))
    assert 14 < errs[0] / errs[1] < 18 and errs[1] < 5e-6      # Simpson: O(h^4)
