"""Pins of the oracle's full cavity step against properties the equations fix
(Sec. 2.1 problem statement, Sec. 2.2 scheme, Secs. 4.2-4.3 reductions):

- conduction (Ra = 0) is an exact discrete fixed point for every power-law index:
  the linear temperature 1 - x makes A and R vanish and the wall closure keeps a
  y/z-constant field, so nothing moves; then Nu = 1 on both walls and the heat
  transfer entropy integrates to 1 (Simpson is exact on constants);
- noise on the conduction state decays;
- the cavity is symmetric under the half-turn (x, y) -> (1-x, 1-y) with
  (u, v, w, theta - 1/2, p) -> (-u, -v, w, -(theta - 1/2), p) and under the mirror
  z -> 1 - z with w -> -w: started symmetric, every step stays symmetric;
- Newtonian reduction: at n = 1 the viscosity is exactly 1 and the momentum source
  reduces to -grad p / Pr + Ra (theta - theta_ref); results depend smoothly on n;
- at steady state the hot and cold wall mean Nusselt numbers agree, and the
  volume integral of |grad theta|^2 equals the hot-wall Nusselt number (Green's
  identity with no-slip walls and a solenoidal field) up to an O(h^2) gap.
"""
import numpy as np
import pytest

from paper_2411_06563_amd.inputs import initial_state, random_smooth_state


@pytest.mark.parametrize("n_pl", [0.75, 1.0, 1.25])
def test_conduction_fixed_point(oracle_lib, n_pl):
    orc = oracle_lib
    N = 9
    p = orc.Params(N=N, Ra=0.0, n_pl=n_pl, dt=1e-3)
    o = orc.Oracle(p)
    o.set_state(**initial_state(N, 1, noise=0.0))
    T0 = o.a["T"].copy()
    x = np.linspace(0, 1, N)
    assert np.abs(T0 - (1 - x)[None, None, :]).max() <= 1e-15
    o.step(5)
    assert np.abs(o.a["T"] - T0).max() <= 1e-14
    for f in ("u", "v", "w", "p"):
        assert np.abs(o.a[f]).max() == 0.0
    d = o.diagnostics()
    for key in ("nu_mean_hot", "nu_mean_cold", "nu_max_hot", "nu_max_cold", "e_ht", "e_total", "be_global",
                "be_mean"):
        assert abs(d[key] - 1.0) <= 1e-13, key
    assert d["e_ff"] == 0.0


def test_conduction_noise_decays(oracle_lib):
    orc = oracle_lib
    N = 9
    p = orc.Params(N=N, Ra=0.0, n_pl=0.75, dt=2e-3)
    o = orc.Oracle(p)
    o.set_state(**initial_state(N, 9, noise=1e-2))
    lin = (1 - np.linspace(0, 1, N))[None, None, :]
    dist = [np.abs(o.a["T"] - lin).max()]
    for _ in range(4):
        o.step(10)
        dist.append(np.abs(o.a["T"] - lin).max())
    assert all(dist[q + 1] < dist[q] for q in range(4)), dist
    assert dist[-1] < 0.5 * dist[0]


def _centro(s):
    return dict(u=-s["u"][:, ::-1, ::-1], v=-s["v"][:, ::-1, ::-1], w=s["w"][:, ::-1, ::-1],
                T=1.0 - s["T"][:, ::-1, ::-1], p=s["p"][:, ::-1, ::-1])


def _mirror_z(s):
    return dict(u=s["u"][::-1], v=s["v"][::-1], w=-s["w"][::-1], T=s["T"][::-1], p=s["p"][::-1])


@pytest.mark.parametrize("n_pl", [0.75, 1.25])
def test_symmetry_every_step(oracle_lib, n_pl):
    orc = oracle_lib
    N = 9
    p = orc.Params(N=N, Ra=2e4, n_pl=n_pl, dt=2e-3, solve_tol=1e-14)
    o = orc.Oracle(p)
    o.set_state(**initial_state(N, 1, noise=0.0))
    for _ in range(6):
        o.step(1)
        s = o.state()
        assert np.abs(s["v"]).max() > 1e-3   # flow is developing
        for image in (_centro(s), _mirror_z(s)):
            for f in s:
                scale = max(np.abs(s[f]).max(), 1e-300)
                assert np.abs(image[f] - s[f]).max() <= 1e-12 * scale, f


def test_newtonian_reduction(oracle_lib):
    orc = oracle_lib
    N = 9
    s = random_smooth_state(N, seed=2, amp=3.0)
    p = orc.Params(N=N, Ra=5e3, n_pl=1.0, Pr=0.71, dt=1e-3)
    eta, I2 = orc.eta_field(p, s["u"], s["v"], s["w"])
    assert np.all(eta == 1.0) and I2.max() > 1.0
    E = orc.estar_field(p, s["u"], s["v"], s["w"], s["T"], s["p"], eta)
    # -grad p / Pr (zero wall-normal derivative) + Ra (theta - theta_ref) in the v equation
    h = p.h
    g = [np.zeros((N, N, N)) for _ in range(3)]
    g[0][:, :, 1:-1] = (s["p"][:, :, 2:] - s["p"][:, :, :-2]) / (2 * h)
    g[1][:, 1:-1, :] = (s["p"][:, 2:, :] - s["p"][:, :-2, :]) / (2 * h)
    g[2][1:-1, :, :] = (s["p"][2:, :, :] - s["p"][:-2, :, :]) / (2 * h)
    assert np.allclose(E[0], -g[0] / p.Pr, rtol=1e-13, atol=1e-12)
    assert np.allclose(E[1], -g[1] / p.Pr + p.Ra * (s["T"] - 0.5), rtol=1e-13, atol=1e-12)
    assert np.allclose(E[2], -g[2] / p.Pr, rtol=1e-13, atol=1e-12)
    # smooth dependence on n around 1
    out = {}
    for dn in (0.0, 1e-6, 2e-6):
        q = orc.Params(N=N, Ra=5e3, n_pl=1.0 + dn, Pr=0.71, dt=1e-3, solve_tol=1e-14)
        o = orc.Oracle(q)
        o.set_state(**s)
        o.step(3)
        out[dn] = o.state()
    for f in ("u", "v", "T"):
        d1 = np.linalg.norm(out[1e-6][f] - out[0.0][f])
        d2 = np.linalg.norm(out[2e-6][f] - out[0.0][f])
        assert 0 < d1 < 1e-4 * np.linalg.norm(out[0.0][f])
        assert abs(d2 / d1 - 2.0) < 1e-2, (f, d1, d2)


def _steady(orc, N, dt):
    p = orc.Params(N=N, Ra=1e3, n_pl=1.0, Pr=1.0, dt=dt, solve_tol=1e-12)
    o = orc.Oracle(p)
    o.set_state(**initial_state(N, 1, 1e-3))
    for _ in range(20000):
        info = o.step(1)[0]
        if max(info.res) < 1e-8:
            break
    assert max(info.res) < 1e-8
    return o.diagnostics()


def test_steady_state_wall_balance_and_green_identity(oracle_lib):
    d9 = _steady(oracle_lib, 9, 2e-3)
    d17 = _steady(oracle_lib, 17, 1e-3)
    for d in (d9, d17):
        assert abs(d["nu_mean_hot"] - d["nu_mean_cold"]) <= 1e-5 * d["nu_mean_hot"]
        assert d["nu_mean_hot"] > 1.05          # convection raises Nu above conduction
    gap9 = d9["e_ht"] / d9["nu_mean_hot"] - 1.0
    gap17 = d17["e_ht"] / d17["nu_mean_hot"] - 1.0
    assert 0 < gap17 < gap9 < 0.01
    assert 3.0 < gap9 / gap17 < 5.5             # O(h^2)


def _grad(f, h):
    """x, y, z derivatives of an array indexed [k, j, i]: central inside, second-order
    one-sided on the walls (numpy's gradient with second-order edges)."""
    gz, gy, gx = np.gradient(f, h, edge_order=2)
    return [gx, gy, gz]


def test_strain_invariant_is_twice_d_colon_d(oracle_lib):
    """I2 of the viscosity law (Sec. 2.1) is the second invariant 2 D:D of the rate
    of strain D = (grad v + grad v^T)/2: formed here as a tensor contraction of the
    velocity gradient, which the oracle writes out component by component."""
    orc = oracle_lib
    N = 9
    s = random_smooth_state(N, seed=3, amp=2.0)
    p = orc.Params(N=N, n_pl=0.6)
    _, I2 = orc.eta_field(p, s["u"], s["v"], s["w"])
    G = np.array([_grad(s[c], p.h) for c in ("u", "v", "w")])        # G[i, j] = d u_i / d x_j
    D = 0.5 * (G + G.transpose(1, 0, 2, 3, 4))
    ref = 2.0 * np.einsum("ij...,ij...->...", D, D)
    assert ref.max() > 1.0
    assert np.abs(I2 - ref).max() <= 1e-12 * ref.max()


def test_viscous_source_is_the_stress_divergence_part(oracle_lib):
    """The viscosity-gradient part of the momentum sources (Sec. 2.1, expanded
    stress divergence): div(2 eta D) = eta lap v + 2 D grad eta for a solenoidal
    velocity, so with p = 0 and theta = theta_ref, E*_i = sum_j (d_j u_i + d_i u_j)
    d_j eta / eta (L = 1/(Pr eta) cancels Pr), formed here as a contraction of the
    velocity gradient with grad eta for a non-uniform eta."""
    orc = oracle_lib
    N = 9
    s = random_smooth_state(N, seed=4, amp=2.0)
    t = random_smooth_state(N, seed=5, amp=1.0)["T"]
    eta = 1.0 + 0.5 * (t - t.min()) / (t.max() - t.min())
    p = orc.Params(N=N, Pr=0.71, Ra=1e4)
    E = orc.estar_field(p, s["u"], s["v"], s["w"], np.full((N, N, N), p.theta_ref), np.zeros((N, N, N)), eta)
    G = np.array([_grad(s[c], p.h) for c in ("u", "v", "w")])
    ge = _grad(eta, p.h)
    for i in range(3):
        ref = sum((G[i, j] + G[j, i]) * ge[j] for j in range(3)) / eta
        assert np.abs(ref).max() > 0.1
        assert np.abs(E[i] - ref).max() <= 1e-12 * np.abs(ref).max(), i


def test_theta_wall_closure_exact_on_quadratics(oracle_lib):
    """The zero-normal-derivative closure of theta on the y and z walls (reading R9)
    is second order: it reproduces exactly a field that is quadratic in the
    wall-normal coordinate with zero normal derivative on the wall.  With theta =
    1 - x + b q(y) + c q(z), q(s) = s^2 near s = 0 and (1 - s)^2 near s = 1, every
    y and z wall node (edges included) must get the field's value."""
    orc = oracle_lib
    N = 11
    x = np.linspace(0.0, 1.0, N)
    q = np.where(x <= 0.5, x ** 2, (1.0 - x) ** 2)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    Qz, Qy = q[:, None, None] * np.ones((N, N, N)), q[None, :, None] * np.ones((N, N, N))
    exact = 1.0 - X + 0.7 * Qy - 0.4 * Qz
    o = orc.Oracle(orc.Params(N=N))
    T = exact.copy()
    T[0], T[-1], T[:, 0], T[:, -1] = 99.0, 99.0, 99.0, 99.0     # wall values to be replaced
    o.set_state(T=T)
    got = o.a["T"]
    inner = slice(1, N - 1)                                       # x walls are Dirichlet
    for face in (got[0, :, inner] - exact[0, :, inner], got[-1, :, inner] - exact[-1, :, inner],
                 got[:, 0, inner] - exact[:, 0, inner], got[:, -1, inner] - exact[:, -1, inner]):
        assert np.abs(face).max() <= 1e-13


def test_pressure_wall_closure_exact_on_quadratics(oracle_lib):
    """The zero-normal-derivative closure of p on every wall (reading R9) reproduces
    exactly a field quadratic in each wall-normal coordinate with zero normal
    derivative on the walls: p = q(x) - 2 q(y) + 3 q(z) (q as for theta) gets its
    own value at every wall node, edges and corners included."""
    orc = oracle_lib
    N = 11
    x = np.linspace(0.0, 1.0, N)
    q = np.where(x <= 0.5, x ** 2, (1.0 - x) ** 2)
    exact = q[None, None, :] - 2.0 * q[None, :, None] + 3.0 * q[:, None, None] + np.zeros((N, N, N))
    o = orc.Oracle(orc.Params(N=N))
    p = exact.copy()
    for sl in ((0,), (-1,), (slice(None), 0), (slice(None), -1), (slice(None), slice(None), 0),
               (slice(None), slice(None), -1)):
        p[sl] = 99.0                                              # wall values to be replaced
    o.set_state(p=p)
    assert np.abs(o.a["p"] - exact).max() <= 1e-13


def test_first_step_takes_level_n_minus_1_equal_to_level_n(oracle_lib):
    """Reading R11: the first step after a state is set has no history, and takes
    level n-1 equal to level n (its time differences vanish).  The same step from
    an oracle whose level n-1 arrays were filled with level n's velocities,
    viscosity and sources must agree bitwise."""
    orc = oracle_lib
    N = 9
    s = random_smooth_state(N, seed=12, amp=3.0)
    prm = orc.Params(N=N, Ra=1e4, n_pl=0.75, dt=5e-4, solve_tol=1e-14)
    a = orc.Oracle(prm)
    a.set_state(**s)
    b = orc.Oracle(prm)
    b.set_state(**s)
    eta, _ = orc.eta_field(prm, b.a["u"], b.a["v"], b.a["w"])
    E = orc.estar_field(prm, b.a["u"], b.a["v"], b.a["w"], b.a["T"], b.a["p"], eta)
    for f, val in (("up", b.a["u"]), ("vp", b.a["v"]), ("wp", b.a["w"]), ("etap", eta), ("Eup", E[0]),
                   ("Evp", E[1]), ("Ewp", E[2])):
        b.a[f][...] = val
    b.first = 0
    a.step(1)
    b.step(1)
    for f in ("u", "v", "w", "T", "p"):
        assert np.array_equal(a.a[f], b.a[f]), f
    assert np.abs(a.a["v"]).max() > 1e-3


def _lap(f, h):
    """Seven-point Laplacian at interior nodes (zero on the walls)."""
    out = np.zeros_like(f)
    c = f[1:-1, 1:-1, 1:-1]
    out[1:-1, 1:-1, 1:-1] = (f[2:, 1:-1, 1:-1] + f[:-2, 1:-1, 1:-1] + f[1:-1, 2:, 1:-1] + f[1:-1, :-2, 1:-1]
                             + f[1:-1, 1:-1, 2:] + f[1:-1, 1:-1, :-2] - 6.0 * c) / (h * h)
    return out


def _pressure_grad(p, h):
    """Gradient of p: central inside; the component normal to a wall is the
    boundary condition dp/dn = 0 on that wall (tangential ones stay central)."""
    g = _grad(p, h)
    for ax, gi in enumerate(g):           # gi indexed [k, j, i]; axis 0 = x is the last array axis
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[2 - ax] = 0
        sl_hi[2 - ax] = -1
        gi[tuple(sl_lo)] = 0.0
        gi[tuple(sl_hi)] = 0.0
    return g


def test_momentum_sources_times_pr_eta_are_the_unnormalised_right_side(oracle_lib):
    """Reading R1.  The momentum equations (Sec. 2.1, expanded form) have the
    right-hand side -d_i p + Pr (eta lap u_i) + 2 Pr (D grad eta)_i + Ra Pr theta
    delta_iy; mapped onto the generic PDE (Eq. 1) with L = 1/(Pr eta) the whole
    non-Laplacian part is divided by Pr eta.  So Pr eta E*_i must equal
    -d_i p + Pr sum_j (d_j u_i + d_i u_j) d_j eta + Ra Pr (theta - theta_ref) delta_iy,
    formed here from numpy gradients with a non-uniform eta, a non-zero pressure
    and theta away from theta_ref: a source that leaves eta off its pressure or its
    buoyancy term gives Pr eta E* = -eta d_i p ... and fails."""
    orc = oracle_lib
    N = 11
    s = random_smooth_state(N, seed=31, amp=2.0)
    t = random_smooth_state(N, seed=32, amp=1.0)["T"]
    eta = 0.4 + 1.6 * (t - t.min()) / (t.max() - t.min())          # in [0.4, 2]
    T = random_smooth_state(N, seed=33, amp=1.0)["T"]
    p = orc.Params(N=N, Pr=0.71, Ra=3e3, theta_ref=0.5)
    pres = 5.0 * s["p"]
    E = orc.estar_field(p, s["u"], s["v"], s["w"], T, pres, eta)
    G = np.array([_grad(s[c], p.h) for c in ("u", "v", "w")])
    ge = _grad(eta, p.h)
    gp = _pressure_grad(pres, p.h)
    assert np.abs(T - 0.5).max() > 0.3 and np.abs(gp[1]).max() > 1.0
    for i in range(3):
        ref = -gp[i] + p.Pr * sum((G[i, j] + G[j, i]) * ge[j] for j in range(3))
        if i == 1:
            ref = ref + p.Ra * p.Pr * (T - p.theta_ref)
        assert np.abs(p.Pr * eta * E[i] - ref).max() <= 1e-12 * np.abs(ref).max(), i


def test_one_momentum_step_follows_the_momentum_equations(oracle_lib):
    """A full step of the scheme (Sec. 2.2), taken from a smooth flowing state with a
    tiny time step, must advance the velocity at the rate the momentum equations
    (Sec. 2.1, expanded form) give:
        u_i,t = -v.grad u_i - d_i p + Pr eta lap u_i + 2 Pr (D grad eta)_i
                + Ra Pr (theta - theta_ref) delta_iy,
    all terms formed here with numpy from the state (eta from the oracle's viscosity,
    itself pinned above).  The HOSC step is consistent with this to O(h^2) (about
    1.6 % at 17^3 away from the walls); the pressure and buoyancy terms carry eta
    variations of up to a factor 2.5 and each moves the rate by 10-20 % if the
    mapping of Sec. 2.2 leaves eta off them."""
    orc = oracle_lib
    N = 17
    s = random_smooth_state(N, seed=21, amp=2.0)
    s["p"] = 30.0 * s["p"]
    prm = orc.Params(N=N, Ra=2e3, Pr=0.7, n_pl=0.9, dt=1e-7, solve_tol=1e-14)
    o = orc.Oracle(prm)
    o.set_state(**s)
    s0 = o.state()
    eta, _ = orc.eta_field(prm, s0["u"], s0["v"], s0["w"])
    assert eta.max() / eta.min() > 2.0
    o.step(1)
    s1 = o.state()
    h = prm.h
    vel = [s0["u"], s0["v"], s0["w"]]
    G = np.array([_grad(c, h) for c in vel])
    ge = _grad(eta, h)
    gp = _pressure_grad(s0["p"], h)
    inner = (slice(2, -2),) * 3
    for i, name in enumerate(("u", "v", "w")):
        rate = (-gp[i] + prm.Pr * eta * _lap(vel[i], h) + prm.Pr * sum((G[i, j] + G[j, i]) * ge[j] for j in range(3))
                - sum(vel[j] * G[i, j] for j in range(3)))
        if i == 1:
            rate = rate + prm.Ra * prm.Pr * (s0["T"] - prm.theta_ref)
        got = (s1[name] - s0[name]) / prm.dt
        err = np.linalg.norm((got - rate)[inner]) / np.linalg.norm(rate[inner])
        assert err < 0.04, (name, err)


def test_steady_residual_is_the_relative_change_of_each_field(oracle_lib):
    """Reading R17 (the paper never defines its steady state): the residual the
    march stops on is, for each of u, v, w and theta, the 2-norm of the change over
    one step divided by the 2-norm of the new field, over all N^3 nodes.  Checked
    against numpy on the first step after a state is set and on a later one."""
    orc = oracle_lib
    N = 9
    prm = orc.Params(N=N, Ra=1e4, n_pl=0.8, dt=1e-3, solve_tol=1e-14)
    o = orc.Oracle(prm)
    o.set_state(**random_smooth_state(N, seed=41, amp=2.0))
    for _ in range(2):
        old = o.state()
        info = o.step(1)[0]
        new = o.state()
        for q, f in enumerate(("u", "v", "w", "T")):
            ref = np.linalg.norm(new[f] - old[f]) / np.linalg.norm(new[f])
            assert ref > 1e-6
            assert abs(info.res[q] - ref) <= 1e-13 * ref, f
