"""Spectral radius of the linearised HOSC step on the FP64 oracle (a measurement
tool of the test infrastructure, not collected by pytest).

The step maps the state of levels n and n-1 to the next one.  Its Jacobian is
applied by finite differences (a 1e-6 perturbation of every interior value, each
field weighted by its RMS), and a power iteration gives the spectral radius rho per
step, the growth per unit time sigma = ln(rho)/dt and the node where the growing
mode is largest.  The base state is marched from the seeded start of the cavity
runs.

    python tests/linearised_step.py N n Ra dt_march steps dt[,dt...] [iters]
           [--lam L] [--Ra-step R] [--frozen-coefficients]

--lam / --Ra-step change the pressure relaxation or the buoyancy of the linearised
step (ablations); --frozen-coefficients linearises the momentum transport step with
L, G*, H*, I* and E* held at the base state's values (the step is then linear in
the velocity; buoyancy and the pressure correction are left out).
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_2411_06563_amd.inputs import initial_state  # noqa: E402

INNER = (slice(1, -1),) * 3


def base_state(N, n_pl, Ra, dt, steps, seed=2):
    o = orc.Oracle(orc.Params(N=N, Ra=Ra, Pr=1.0, n_pl=n_pl, dt=dt, solve_tol=1e-13, maxit=20000))
    o.set_state(**initial_state(N, seed))
    o.step(steps)
    return {f: o.a[f].copy() for f in o.FIELDS}


def _power(apply, x0, weights, iters):
    def norm(d):
        return np.sqrt(sum(np.sum((d[f][INNER] / weights[f]) ** 2) for f in d))

    d = {f: v / norm(x0) for f, v in x0.items()}
    logs = []
    for _ in range(iters):
        jd = apply(d)
        g = norm(jd)
        logs.append(np.log(g))
        d = {f: v / g for f, v in jd.items()}
    return float(np.exp(np.mean(logs[iters // 2:]))), d


def full_step_radius(base, N, n_pl, Ra, dt, iters, lam=None, eps=1e-6, seed=0):
    """rho of the oracle's full step (all twelve state fields perturbed)."""
    fields = orc.Oracle.FIELDS
    kw = dict(N=N, Ra=Ra, Pr=1.0, n_pl=n_pl, dt=dt, solve_tol=1e-13, maxit=20000)
    if lam is not None:
        kw["lam"] = lam

    def F(Z):
        q = orc.Oracle(orc.Params(**kw))
        for f in fields:
            q.a[f][...] = Z[f]
        q.first = 0
        q.step(1)
        return {f: q.a[f].copy() for f in fields}

    F0 = F(base)
    W = {f: max(np.sqrt(np.mean(base[f][INNER] ** 2)), 1e-12) for f in fields}
    rng = np.random.default_rng(seed)
    x0 = {f: np.zeros_like(base[f]) for f in fields}
    for f in fields:
        x0[f][INNER] = rng.standard_normal(x0[f][INNER].shape) * W[f]

    def apply(d):
        F1 = F({f: base[f] + eps * d[f] for f in fields})
        out = {f: np.zeros_like(base[f]) for f in fields}
        for f in fields:
            out[f][INNER] = (F1[f][INNER] - F0[f][INNER]) / eps
        return out

    return _power(apply, x0, W, iters)


def frozen_coefficient_radius(base, N, n_pl, dt, iters, seed=0):
    """rho of the momentum transport step with every coefficient field (L, G*, H*,
    I*, E* at levels n and n-1) held at the base state's values."""
    P = orc.Params(N=N, n_pl=n_pl, Ra=0.0, dt=dt, solve_tol=1e-13, maxit=20000)
    eta, _ = orc.eta_field(P, base["u"], base["v"], base["w"])
    L = 1.0 / eta
    G, H, I = base["u"] * L, base["v"] * L, base["w"] * L
    Lp = 1.0 / base["etap"]
    Gp, Hp, Ip = base["up"] * Lp, base["vp"] * Lp, base["wp"] * Lp
    zero = np.zeros((N, N, N))
    W = {f: 1.0 for f in ("u", "v", "w")}
    rng = np.random.default_rng(seed)
    x0 = {f: np.zeros((N, N, N)) for f in W}
    for f in W:
        x0[f][INNER] = rng.standard_normal((N - 2,) * 3)

    def apply(d):
        out = {}
        for f in W:     # a linear step: zero source, zero walls
            out[f], _, _ = orc.transport_step(P, L, G, H, I, None, Lp, Gp, Hp, Ip, None, d[f], zero)
        return out

    return _power(apply, x0, W, iters)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("N", type=int)
    ap.add_argument("n_pl", type=float)
    ap.add_argument("Ra", type=float)
    ap.add_argument("dt_march", type=float)
    ap.add_argument("steps", type=int)
    ap.add_argument("dts")
    ap.add_argument("iters", type=int, nargs="?", default=100)
    ap.add_argument("--lam", type=float, default=None)
    ap.add_argument("--Ra-step", type=float, default=None)
    ap.add_argument("--frozen-coefficients", action="store_true")
    a = ap.parse_args()
    base = base_state(a.N, a.n_pl, a.Ra, a.dt_march, a.steps)
    for dt in (float(x) for x in a.dts.split(",")):
        if a.frozen_coefficients:
            rho, d = frozen_coefficient_radius(base, a.N, a.n_pl, dt, a.iters)
        else:
            Ra = a.Ra if a.Ra_step is None else a.Ra_step
            rho, d = full_step_radius(base, a.N, a.n_pl, Ra, dt, a.iters, lam=a.lam)
        mag = np.sqrt(sum(d[f] ** 2 for f in ("u", "v", "w")))
        k, j, i = np.unravel_index(np.argmax(mag), mag.shape)
        print(f"N={a.N} n={a.n_pl} Ra={a.Ra:g} t={a.steps * a.dt_march:g}: dt={dt:g} rho={rho:.4f} "
              f"sigma={np.log(rho) / dt:.3g} mode peak at (i,j,k)=({i},{j},{k})", flush=True)


if __name__ == "__main__":
    main()
