"""Pins of the oracle's probe interpolation (the monitoring points of the grid-
independence study, Sec. 3.1, Table 1): trilinear interpolation reproduces every
trilinear polynomial exactly, returns node values at nodes (the paper's probes at
0.4 and 0.6 are nodes of its 11^3, 51^3 and 91^3 grids), and its error on a smooth
function stays within the classical bound (h^2/8)(|f_xx| + |f_yy| + |f_zz|)."""
import numpy as np
import pytest

from oracle import oracle as O


def _grid(N):
    x = np.linspace(0.0, 1.0, N)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return X, Y, Z


def _fields(fn, N):
    X, Y, Z = _grid(N)
    return {name: fn(X, Y, Z, q) for q, name in enumerate(("u", "v", "w", "T", "p"))}


def _trilinear(X, Y, Z, q):
    c = np.arange(8, dtype=float) + q
    return (c[0] + c[1] * X - c[2] * Y + c[3] * Z + c[4] * X * Y - c[5] * Y * Z + c[6] * X * Z
            + c[7] * X * Y * Z)


@pytest.mark.parametrize("N", [5, 8, 11])
def test_exact_on_trilinear_polynomials(N):
    rng = np.random.default_rng(N)
    pts = np.vstack([rng.random((40, 3)), [[0, 0, 0], [1, 1, 1], [1, 0, 0.5], [0.25, 1, 0]]])
    out = O.probe(_fields(_trilinear, N), pts)
    for q in range(5):
        ref = _trilinear(pts[:, 0], pts[:, 1], pts[:, 2], q)
        assert np.max(np.abs(out[:, q] - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("N", [11, 51, 91])
def test_paper_probes_are_nodes(N):
    rng = np.random.default_rng(7)
    f = {name: rng.standard_normal((N, N, N)) for name in ("u", "v", "w", "T", "p")}
    out = O.probe(f, [(0.6, 0.6, 0.6), (0.4, 0.4, 0.4)])
    for row, c in zip(out, (0.6, 0.4)):
        i = int(round(c * (N - 1)))
        assert abs(c * (N - 1) - i) < 1e-12
        for q, name in enumerate(("u", "v", "w", "T", "p")):
            assert abs(row[q] - f[name][i, i, i]) <= 1e-12 * max(1.0, np.max(np.abs(f[name])))


def test_error_bound_on_smooth_function():
    N = 17
    h = 1.0 / (N - 1)

    def fn(X, Y, Z, q):
        return np.sin(np.pi * (q + 1) * X / 2) * np.cos(np.pi * Y) * np.exp(Z)

    rng = np.random.default_rng(3)
    pts = rng.random((200, 3))
    out = O.probe(_fields(fn, N), pts)
    for q in range(5):
        ref = fn(pts[:, 0], pts[:, 1], pts[:, 2], q)
        a = np.pi * (q + 1) / 2
        bound = h * h / 8 * (a * a + np.pi ** 2 + 1.0) * np.e
        err = np.max(np.abs(out[:, q] - ref))
        assert err <= bound
        assert err >= 0.05 * bound          # an interpolant, not the exact function: the error is real
