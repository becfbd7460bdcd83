"""The largest cavity one GPU holds.

The grid is the largest odd N whose workspace fits in 90% of the free device
memory (about 800^3 nodes in FP64 on a 288 GB device; odd N keeps the red-black
colouring symmetric).  The oracle cannot march a grid this size, so the check is
a property that holds at any size and that the oracle pins on small grids
(`test_symmetry_every_step`): the cavity is symmetric under the half-turn
(x, y) -> (1 - x, 1 - y) with (u, v, w, theta - 1/2, p) -> (-u, -v, w,
-(theta - 1/2), p) and under the mirror z -> 1 - z with w -> -w, so from the
noise-free conduction start every step stays symmetric to rounding.  An
indexing error anywhere in the step at this size (an offset past 2^31 bytes, a
grid that misses a tile, a partial record out of place) breaks that.  Also
checked: the wall values, the mirror symmetry of the local Nusselt numbers on the
hot wall and their half-turn image on the cold wall, and that every step
converged."""
import gc
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hosc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2411_06563_amd import hosc as h
    return h


def _largest_N(hosc, precision, budget):
    for N in range(1025, 4, -2):
        p = hosc.params(N, Ra=2e4, n_pl=0.75, Pr=1.0, dt=0.8 / (N - 1) ** 2, solve_rtol=1e-12, precision=precision)
        nbytes = hosc.workspace_bytes(p)
        if nbytes <= budget:
            return N, p, nbytes
    raise AssertionError("no grid fits")


def _check_symmetry(s, tol):
    u, v, w, T, p = s["u"], s["v"], s["w"], s["T"], s["p"]
    worst = {}
    # arrays are indexed [k, j, i]
    for name, f, image in (
        ("u", u, lambda a: -a[:, ::-1, ::-1]), ("v", v, lambda a: -a[:, ::-1, ::-1]),
        ("w", w, lambda a: a[:, ::-1, ::-1]), ("T", T, lambda a: 1.0 - a[:, ::-1, ::-1]),
        ("p", p, lambda a: a[:, ::-1, ::-1]),
    ):
        scale = max(float(np.abs(f).max()), 1e-300)
        d = float(np.abs(image(f) - f).max()) / scale
        worst["half-turn " + name] = d
        assert d <= tol, ("half-turn", name, d)
    for name, f, sign in (("u", u, 1.0), ("v", v, 1.0), ("w", w, -1.0), ("T", T, 1.0), ("p", p, 1.0)):
        scale = max(float(np.abs(f).max()), 1e-300)
        d = float(np.abs(sign * f[::-1] - f).max()) / scale
        worst["mirror " + name] = d
        assert d <= tol, ("mirror", name, d)
    return worst


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-10)])
def test_largest_grid_symmetric_steps(hosc, precision, tol):
    import torch
    gc.collect()
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    N, p, nbytes = _largest_N(hosc, precision, 0.9 * free)
    say(f"[max] precision {precision}: N = {N}, workspace {nbytes / 2**30:.1f} GiB of {free / 2**30:.1f} GiB free "
        f"({total / 2**30:.1f} GiB total)")
    assert nbytes >= 0.5 * total, "the largest grid should take most of the device memory"
    s = hosc.Solver(p)
    try:
        t = time.time()
        s.init_fields(1, 0.0)
        for step in range(2):
            info = s.step(1)
            say(f"[max] step {step + 1}: status {info.status} sweeps {info.sweeps} bicg {info.bicg_iters} "
                f"max|div| {info.maxdiv:.3e} res {info.res} ({time.time() - t:.1f} s)")
            assert info.status == 0
        st = s.get_state()
        assert np.abs(st["v"]).max() > 1e-6          # the flow is developing
        worst = _check_symmetry(st, tol)
        say(f"[max] worst relative asymmetry {max(worst.values()):.2e} ({max(worst, key=worst.get)})")
        # walls: no slip, fixed wall temperatures
        for f in ("u", "v", "w"):
            a = st[f]
            for face in (a[0], a[-1], a[:, 0], a[:, -1], a[:, :, 0], a[:, :, -1]):
                assert np.all(face == 0.0), f
        assert np.all(st["T"][:, :, 0] == p.theta_hot) and np.all(st["T"][:, :, -1] == p.theta_cold)
        del st
        d = s.diagnostics(arrays=True)
        nuh, nuc = d["nu_hot"], d["nu_cold"]       # indexed [k, j]
        assert np.all(np.isfinite(nuh)) and np.all(np.isfinite(nuc))
        # The wall flux is a five-point one-sided difference (weights 25, 48, 36, 16, 3
        # over 12h): it passes on the asymmetry of theta, and its own rounding, scaled by
        # 128/(12h), so its bound follows from the measured theta asymmetry.
        h = 1.0 / (N - 1)
        nu_tol = 128.0 / (12.0 * h) * (max(worst["half-turn T"], worst["mirror T"]) + 8.0 * 2.0 ** -53)
        a_mirror = float(np.abs(nuh[::-1] - nuh).max())                 # mirror z -> 1 - z
        a_turn = float(np.abs(nuc[:, ::-1] - nuh).max())                # the half-turn maps hot onto cold
        say(f"[max] local Nu asymmetry: mirror {a_mirror:.2e}, half-turn {a_turn:.2e} (bound {nu_tol:.2e})")
        assert a_mirror <= nu_tol and a_turn <= nu_tol
        assert abs(d["nu_mean_hot"] - d["nu_mean_cold"]) <= nu_tol
        say(f"[max] Nu hot {d['nu_mean_hot']:.9f}, E_total {d['e_total']:.6e}, Be {d['be_global']:.9f} "
            f"({time.time() - t:.1f} s)")
    finally:
        s.close()
        del s
        gc.collect()
        torch.cuda.empty_cache()
