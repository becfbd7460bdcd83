"""Pin: closed form of the HOSC step for pure diffusion (Sec. 2.2, Eq. 5 with
constant L, zero convection and zero source).

A discrete sine mode chi = sin(a pi x) sin(b pi y) sin(c pi z) is an eigenvector of
every central second difference: delta_d^2 chi = -s_d chi, s_d = (4/h^2) sin^2(a_d pi h/2).
Then B chi = B_s chi and A chi = A_s chi with
    B_s = L0 + (dt/2 - L0 h^2/12) sum_d s_d
    A_s = sum_d s_d - M5 s_x s_y - M6 s_y s_z - M7 s_z s_x
so every step multiplies the mode by g = 1 - dt A_s / B_s.  (-A is the textbook
19-point Mehrstellen Laplacian sum delta^2 + (h^2/6) sum_pairs delta_i^2 delta_j^2.)
"""
import numpy as np
import pytest


# (mode, L0, dt): both signs of c = L0 h^2/12 - dt/2 occur; every case decays by
# a moderate factor over the 50 steps so the comparison is relative to a live mode.
@pytest.mark.parametrize("abc,L0,dt", [((1, 1, 1), 1.0, 2e-3), ((2, 1, 3), 1.0, 5e-4), ((1, 3, 2), 0.37, 2e-4),
                                       ((5, 2, 1), 0.37, 1e-4), ((5, 2, 1), 1.0, 2e-4)])
def test_diffusion_mode_decay(oracle_lib, abc, L0, dt):
    N, steps = 17, 50
    h = 1.0 / (N - 1)
    g1 = np.linspace(0.0, 1.0, N)
    Z, Y, X = np.meshgrid(g1, g1, g1, indexing="ij")
    a, b, c = abc
    chi0 = np.sin(a * np.pi * X) * np.sin(b * np.pi * Y) * np.sin(c * np.pi * Z)
    chi0[:, :, 0] = chi0[:, :, -1] = 0.0
    chi0[:, 0, :] = chi0[:, -1, :] = 0.0
    chi0[0, :, :] = chi0[-1, :, :] = 0.0
    L = np.full((N, N, N), L0)
    zero = np.zeros((N, N, N))
    p = oracle_lib.Params(N=N, dt=dt, solve_tol=1e-15, maxit=5000)
    chi = chi0.copy()
    for _ in range(steps):
        chi, _, _ = oracle_lib.transport_step(p, L, zero, zero, zero, None, L, zero, zero, zero, None, chi, zero)
    s = [4.0 / h ** 2 * np.sin(q * np.pi * h / 2) ** 2 for q in (a, b, c)]
    M5 = M6 = M7 = 2 * h * h / 12.0
    A_s = sum(s) - M5 * s[0] * s[1] - M6 * s[1] * s[2] - M7 * s[2] * s[0]
    B_s = L0 + (dt / 2 - L0 * h * h / 12.0) * sum(s)
    g = 1.0 - dt * A_s / B_s
    expect = g ** steps * chi0
    err = np.abs(chi - expect).max() / np.abs(expect).max()
    assert 1e-3 < g ** steps < 0.9
    assert err <= 1e-12, err

