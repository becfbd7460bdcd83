"""Pin: the oracle's operator-form assembly equals the paper's expanded (19,7)
stencil (Sec. 2.2, the weights L1..L7 and Q1..Q19 printed after Eq. (eq_implicit)).

The paper states the scheme twice: as the bracketed operators of Eq. 5 and as the
expanded point weights.  The oracle implements the first; this test transcribes the
second in numpy, with the print errors resolved as follows:
  - in Q1, Q3, Q4..Q7 the "+" between L*M25/(2h) and N1/h^2 (and alike) is lost;
  - in Q1 and Q3 the term -2 dt M7/(l^2 k^2) pairs z with x: -2 dt M7/(l^2 h^2);
  - in Q3 and Q5 the first-difference terms N4/(2h), N5/(2k) carry a minus sign
    (they are antisymmetric, as Q7 already shows for N6);
  - "2l^h" in Q16..Q19 is 2 l^2 h; "2K" in L3, L4 is 2k; p1*, q1*, r1* are p1, q1, r1;
  - M18 = [(dt/2) delta_t^- + sum (delta_d^2 - V_d delta_d) h_d^2/12] L (lost "+").
It then checks, at every interior node of a flowing state with distinct levels n
and n-1, that sum L_m x_m equals the oracle's B x for a random x, and that
sum Q_m chi_m + dt R equals the oracle's B chi + b (b = dt (R - A chi)).
"""
import numpy as np

from paper_2411_06563_amd.inputs import random_smooth_state, uniform01


def _sh(f, di, dj, dk):
    """f at interior nodes shifted by (di, dj, dk); arrays are indexed [k, j, i]."""
    N = f.shape[0]
    return f[1 + dk:N - 1 + dk, 1 + dj:N - 1 + dj, 1 + di:N - 1 + di]


def _d1(f, ax, h):
    e = [0, 0, 0]
    e[ax] = 1
    return (_sh(f, *e) - _sh(f, *[-q for q in e])) / (2 * h)


def _d2(f, ax, h):
    e = [0, 0, 0]
    e[ax] = 1
    return (_sh(f, *e) - 2 * _sh(f, 0, 0, 0) + _sh(f, *[-q for q in e])) / (h * h)


def expanded_weights(L, G, H, I, Lp, Gp, Hp, Ip, dt, h):
    """L1..L7 and Q1..Q19 of the paper at the interior nodes (K* = 0; h = k = l)."""
    k = l = h
    Lc, Gc, Hc, Ic = (_sh(a, 0, 0, 0) for a in (L, G, H, I))
    # bracket [1 + (dxx - G dx) h^2/12 + (dyy - H dy) k^2/12 + (dzz - I dz) l^2/12 + dt/2 delta_t^-] f
    def bracket(f, fp):
        return (_sh(f, 0, 0, 0) + (_d2(f, 0, h) - Gc * _d1(f, 0, h)) * h * h / 12
                + (_d2(f, 1, h) - Hc * _d1(f, 1, h)) * k * k / 12 + (_d2(f, 2, h) - Ic * _d1(f, 2, h)) * l * l / 12
                + dt / 2 * (_sh(f, 0, 0, 0) - _sh(fp, 0, 0, 0)) / dt)
    M_1 = -dt / (2 * Lc) + h * h / 12
    M_2 = -dt / (2 * Lc) + k * k / 12
    M_3 = -dt / (2 * Lc) + l * l / 12
    M_4 = dt / (2 * Lc)
    M15 = _d1(L, 0, h) * (h * h / (6 * Lc))
    M16 = _d1(L, 1, h) * (k * k / (6 * Lc))
    M17 = _d1(L, 2, h) * (l * l / (6 * Lc))
    M25, M26, M27 = M15, M16, M17
    M18 = (dt / 2 * (Lc - _sh(Lp, 0, 0, 0)) / dt + (_d2(L, 0, h) - Gc * _d1(L, 0, h)) * h * h / 12
           + (_d2(L, 1, h) - Hc * _d1(L, 1, h)) * k * k / 12 + (_d2(L, 2, h) - Ic * _d1(L, 2, h)) * l * l / 12)
    Lw = {}
    Lw[1] = (-M_1 * Gc / (2 * h) + M_1 / h ** 2 + M15 / (2 * h)) * Lc
    Lw[2] = (M_1 * Gc / (2 * h) + M_1 / h ** 2 - M15 / (2 * h)) * Lc
    Lw[3] = (-M_2 * Hc / (2 * k) + M_2 / k ** 2 + M16 / (2 * k)) * Lc
    Lw[4] = (M_2 * Hc / (2 * k) + M_2 / k ** 2 - M16 / (2 * k)) * Lc
    Lw[5] = (-M_3 * Ic / (2 * l) + M_3 / l ** 2 + M17 / (2 * l)) * Lc
    Lw[6] = (M_3 * Ic / (2 * l) + M_3 / l ** 2 - M17 / (2 * l)) * Lc
    Lw[7] = (1 - 2 * M_2 / k ** 2 - 2 * M_1 / h ** 2 + 2 * M_4 * M18 / dt - 2 * M_3 / l ** 2) * Lc

    alpha = (Gc ** 2 - 2 * _d1(G, 0, h)) * h * h / 12 + 1
    beta = (Hc ** 2 - 2 * _d1(H, 1, h)) * k * k / 12 + 1
    gamma = (Ic ** 2 - 2 * _d1(I, 2, h)) * l * l / 12 + 1
    M1 = bracket(G, Gp)
    M2 = bracket(H, Hp)
    M3 = bracket(I, Ip)
    p1 = -Gc * Hc + 2 / (h * h + k * k) * (k * k * _d1(G, 1, h) + h * h * _d1(H, 0, h))
    q1 = -Hc * Ic + 2 / (k * k + l * l) * (l * l * _d1(H, 2, h) + k * k * _d1(I, 1, h))
    r1 = -Ic * Gc + 2 / (l * l + h * h) * (h * h * _d1(I, 0, h) + l * l * _d1(G, 2, h))
    M5 = (h * h + k * k) / 12
    M6 = (k * k + l * l) / 12
    M7 = (l * l + h * h) / 12
    N1 = dt * alpha + Lc * M_1
    N2 = dt * beta + Lc * M_2
    N3 = dt * gamma + Lc * M_3
    N4 = -dt * M1 - Lc * M_1 * Gc
    N5 = -dt * M2 - Lc * M_2 * Hc
    N6 = -dt * M3 - Lc * M_3 * Ic
    N7 = M_4 * Lc
    Q = {}
    Q[1] = (Lc * M25 / (2 * h) + N1 / h ** 2 - 2 * dt * M5 / (h ** 2 * k ** 2) + 2 * dt * M5 * Gc / (2 * h * k ** 2)
            + N4 / (2 * h) - 2 * dt * M7 / (l ** 2 * h ** 2) + 2 * dt * M7 * Gc / (2 * h * l ** 2))
    Q[2] = (Lc - 2 * (N2 / k ** 2 + N1 / h ** 2 + N3 / l ** 2) + 4 * dt * M5 / (h ** 2 * k ** 2)
            + 4 * dt * M6 / (k ** 2 * l ** 2) + 2 * N7 * M18 / dt + 4 * dt * M7 / (h ** 2 * l ** 2))
    Q[3] = (-Lc * M25 / (2 * h) + N1 / h ** 2 - 2 * dt * M5 / (h ** 2 * k ** 2) - 2 * dt * M5 * Gc / (2 * h * k ** 2)
            - N4 / (2 * h) - 2 * dt * M7 / (l ** 2 * h ** 2) - 2 * dt * M7 * Gc / (2 * h * l ** 2))
    Q[4] = (Lc * M26 / (2 * k) + N2 / k ** 2 - 2 * dt * M5 / (h ** 2 * k ** 2) + N5 / (2 * k)
            + 2 * dt * M5 * Hc / (2 * h ** 2 * k) - 2 * dt * M6 / (l ** 2 * k ** 2) + 2 * dt * M6 * Hc / (2 * k * l ** 2))
    Q[5] = (-Lc * M26 / (2 * k) + N2 / k ** 2 - 2 * dt * M5 / (h ** 2 * k ** 2) - N5 / (2 * k)
            - 2 * dt * M5 * Hc / (2 * h ** 2 * k) - 2 * dt * M6 / (l ** 2 * k ** 2) - 2 * dt * M6 * Hc / (2 * k * l ** 2))
    Q[6] = (Lc * M27 / (2 * l) + N3 / l ** 2 - 2 * dt * M6 / (l ** 2 * k ** 2) + N6 / (2 * l)
            - 2 * dt * M7 / (l ** 2 * h ** 2) + 2 * dt * M6 * Ic / (2 * k ** 2 * l) + 2 * dt * M7 * Ic / (2 * l * h ** 2))
    Q[7] = (-2 * dt * M7 * Ic / (2 * l * h ** 2) - Lc * M27 / (2 * l) + N3 / l ** 2 - 2 * dt * M6 / (l ** 2 * k ** 2)
            - N6 / (2 * l) - 2 * dt * M6 * Ic / (2 * k ** 2 * l) - 2 * dt * M7 / (l ** 2 * h ** 2))
    Q[8] = (-dt * M5 * p1 / (4 * h * k) + dt * M5 / (h ** 2 * k ** 2) - dt * M5 * Hc / (2 * h ** 2 * k)
            - dt * M5 * Gc / (2 * h * k ** 2))
    Q[9] = (dt * M5 * p1 / (4 * h * k) + dt * M5 / (h ** 2 * k ** 2) - dt * M5 * Hc / (2 * h ** 2 * k)
            + dt * M5 * Gc / (2 * h * k ** 2))
    Q[10] = (dt * M5 * p1 / (4 * h * k) + dt * M5 / (h ** 2 * k ** 2) + dt * M5 * Hc / (2 * h ** 2 * k)
             - dt * M5 * Gc / (2 * h * k ** 2))
    Q[11] = (-dt * M5 * p1 / (4 * h * k) + dt * M5 / (h ** 2 * k ** 2) + dt * M5 * Hc / (2 * h ** 2 * k)
             + dt * M5 * Gc / (2 * h * k ** 2))
    Q[12] = (-dt * M6 * q1 / (4 * k * l) + dt * M6 / (l ** 2 * k ** 2) - dt * M6 * Ic / (2 * k ** 2 * l)
             - dt * M6 * Hc / (2 * k * l ** 2))
    Q[13] = (dt * M6 * q1 / (4 * k * l) + dt * M6 / (l ** 2 * k ** 2) - dt * M6 * Ic / (2 * k ** 2 * l)
             + dt * M6 * Hc / (2 * k * l ** 2))
    Q[14] = (dt * M6 * q1 / (4 * k * l) + dt * M6 / (l ** 2 * k ** 2) + dt * M6 * Ic / (2 * k ** 2 * l)
             - dt * M6 * Hc / (2 * k * l ** 2))
    Q[15] = (-dt * M6 * q1 / (4 * k * l) + dt * M6 / (l ** 2 * k ** 2) + dt * M6 * Ic / (2 * k ** 2 * l)
             + dt * M6 * Hc / (2 * k * l ** 2))
    Q[16] = (-dt * M7 * r1 / (4 * l * h) + dt * M7 / (l ** 2 * h ** 2) - dt * M7 * Gc / (2 * l ** 2 * h)
             - dt * M7 * Ic / (2 * l * h ** 2))
    Q[17] = (dt * M7 * r1 / (4 * l * h) + dt * M7 / (l ** 2 * h ** 2) - dt * M7 * Gc / (2 * l ** 2 * h)
             + dt * M7 * Ic / (2 * l * h ** 2))
    Q[18] = (dt * M7 * r1 / (4 * l * h) + dt * M7 / (l ** 2 * h ** 2) + dt * M7 * Gc / (2 * l ** 2 * h)
             - dt * M7 * Ic / (2 * l * h ** 2))
    Q[19] = (-dt * M7 * r1 / (4 * l * h) + dt * M7 / (l ** 2 * h ** 2) + dt * M7 * Gc / (2 * l ** 2 * h)
             + dt * M7 * Ic / (2 * l * h ** 2))
    return Lw, Q, bracket


# neighbour offsets (di, dj, dk) of the paper's point numbering
L_OFF = {1: (1, 0, 0), 2: (-1, 0, 0), 3: (0, 1, 0), 4: (0, -1, 0), 5: (0, 0, 1), 6: (0, 0, -1), 7: (0, 0, 0)}
Q_OFF = {1: (1, 0, 0), 2: (0, 0, 0), 3: (-1, 0, 0), 4: (0, 1, 0), 5: (0, -1, 0), 6: (0, 0, 1), 7: (0, 0, -1),
         8: (1, 1, 0), 9: (-1, 1, 0), 10: (1, -1, 0), 11: (-1, -1, 0), 12: (0, 1, 1), 13: (0, -1, 1),
         14: (0, 1, -1), 15: (0, -1, -1), 16: (1, 0, 1), 17: (1, 0, -1), 18: (-1, 0, 1), 19: (-1, 0, -1)}


def _flowing_oracle(orc, N, n_pl, Ra, dt):
    p = orc.Params(N=N, Ra=Ra, n_pl=n_pl, dt=dt, Pr=0.8)
    o = orc.Oracle(p)
    s = random_smooth_state(N, seed=7, amp=3.0)
    o.set_state(**s)
    o.step(2)          # levels n and n-1 now differ
    return p, o


def _check(orc, n_pl):
    N, dt = 11, 3e-3
    p, o = _flowing_oracle(orc, N, n_pl, 2e4, dt)
    h = p.h
    a = o.a
    eta, _ = orc.eta_field(p, a["u"], a["v"], a["w"])
    E = orc.estar_field(p, a["u"], a["v"], a["w"], a["T"], a["p"], eta)
    b4, eta_o, E3 = o.assemble()
    assert np.array_equal(eta, eta_o)
    Lm = 1.0 / (p.Pr * eta)
    Lmp = 1.0 / (p.Pr * a["etap"])
    one = np.ones_like(Lm)
    systems = {
        "mom": (Lm, a["u"] * Lm, a["v"] * Lm, a["w"] * Lm, Lmp, a["up"] * Lmp, a["vp"] * Lmp, a["wp"] * Lmp),
        "theta": (one, a["u"], a["v"], a["w"], one, a["up"], a["vp"], a["wp"]),
    }
    xr = uniform01(11, N ** 3).reshape(N, N, N) - 0.5
    for name, (L, G, H, I, Lp, Gp, Hp, Ip) in systems.items():
        Lw, Q, bracket = expanded_weights(L, G, H, I, Lp, Gp, Hp, Ip, dt, h)
        eq = 0 if name == "mom" else 1
        # implicit 7-point weights against the oracle's B
        Bx = sum(Lw[m] * _sh(xr, *L_OFF[m]) for m in Lw)
        ref = o.apply_B(eq, xr)[1:-1, 1:-1, 1:-1]
        scale = sum(np.abs(Lw[m] * _sh(xr, *L_OFF[m])) for m in Lw)
        assert np.max(np.abs(Bx - ref) / scale) < 1e-12, name
        # explicit 19-point side
        if name == "mom":
            rhs = [(a["u"], E[0], a["Eup"], b4[0]), (a["v"], E[1], a["Evp"], b4[1]), (a["w"], E[2], a["Ewp"], b4[2])]
        else:
            rhs = [(a["T"], None, None, b4[3])]
        for chi, Ef, Efp, b in rhs:
            R = bracket(Ef, Efp) if Ef is not None else 0.0
            lhs = sum(Q[m] * _sh(chi, *Q_OFF[m]) for m in Q) + dt * R
            ref = o.apply_B(eq, chi)[1:-1, 1:-1, 1:-1] + b[1:-1, 1:-1, 1:-1]
            scale = sum(np.abs(Q[m] * _sh(chi, *Q_OFF[m])) for m in Q) + np.abs(dt * R)
            assert np.max(np.abs(lhs - ref) / scale) < 1e-12, name


def test_expanded_equals_operator_form_shear_thinning(oracle_lib):
    _check(oracle_lib, 0.75)


def test_expanded_equals_operator_form_shear_thickening(oracle_lib):
    _check(oracle_lib, 1.25)
