"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module holds no arithmetic of the numerical method: only the random-number
generator, the initial-condition recipe and the workload generators (cavity sets
and request traces).  Boundary conditions are applied by whichever side consumes
the arrays.

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): output k of a stream seeded with s
is mix(s + (k+1)*0x9E3779B97F4A7C15) with the published mixing function, and a
uniform double in [0, 1) is (z >> 11) * 2^-53.  The GPU library implements the same
published generator on its own for ``hosc_init_fields``.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Outputs offset .. offset+count-1 of the SplitMix64 stream seeded with seed."""
    with np.errstate(over="ignore"):
        k = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform01(seed: int, count: int, offset: int = 0) -> np.ndarray:
    return (splitmix64(seed, count, offset) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def initial_state(N: int, seed: int, noise: float = 1e-3, theta_hot: float = 1.0, theta_cold: float = 0.0):
    """Initial condition of the cavity runs.

    u = v = w = p = 0; theta = theta_hot + (theta_cold - theta_hot) x + noise (2U - 1) at
    interior nodes, one U per interior node drawn in storage order (x fastest); the
    x walls hold theta_hot and theta_cold; the y/z wall values are placeholders
    (the linear profile) that the consumer replaces by its boundary closure.
    Arrays are (N, N, N) indexed [k, j, i]."""
    x = np.linspace(0.0, 1.0, N)
    T = np.broadcast_to(theta_hot + (theta_cold - theta_hot) * x, (N, N, N)).copy()
    M = N - 2
    if noise != 0.0 and M > 0:
        U = uniform01(seed, M * M * M).reshape(M, M, M)
        T[1:-1, 1:-1, 1:-1] += noise * (2.0 * U - 1.0)
    T[:, :, 0] = theta_hot
    T[:, :, -1] = theta_cold
    z = np.zeros((N, N, N))
    return dict(u=z.copy(), v=z.copy(), w=z.copy(), T=T, p=z.copy())


def random_smooth_state(N: int, seed: int, amp: float = 1.0):
    """A smooth non-trivial state (for assembly parity at a moving flow): sums of a
    few random Fourier modes, zero velocity on the walls, theta with the hot/cold
    x walls.  Arrays (N, N, N) indexed [k, j, i]."""
    x = np.linspace(0.0, 1.0, N)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    U = uniform01(seed, 64)
    out = {}
    bubble = np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z)
    q = 0
    for name in ("u", "v", "w", "p", "T"):
        f = np.zeros((N, N, N))
        for _ in range(3):
            a, b, c, ph = U[q:q + 4]
            q += 4
            f += np.cos(np.pi * (1 + 2 * a) * X + 2 * np.pi * ph) * np.cos(np.pi * (1 + 2 * b) * Y) \
                * np.cos(np.pi * (1 + 2 * c) * Z + np.pi * ph)
        if name in ("u", "v", "w"):
            f = amp * bubble * f
        elif name == "T":
            f = 1.0 - X + 0.1 * bubble * f
        else:
            f = amp * f
        out[name] = np.ascontiguousarray(f)
    out["T"][:, :, 0] = 1.0
    out["T"][:, :, -1] = 0.0
    return out


def batched_cavities(seed: int = 4):
    """The 12-cavity batch: (Ra, n) over {1e2,1e3,1e4,1e5} x {0.75,1.0,1.25} in
    lexicographic order, sizes {33 x4, 65 x4, 97 x4} shuffled by a seeded
    Fisher-Yates; cavity seeds 100 + index."""
    sizes = [33] * 4 + [65] * 4 + [97] * 4
    U = uniform01(seed, len(sizes))
    for q in range(len(sizes) - 1, 0, -1):
        r = int(U[q] * (q + 1))
        sizes[q], sizes[r] = sizes[r], sizes[q]
    out = []
    idx = 0
    for Ra in (1e2, 1e3, 1e4, 1e5):
        for n in (0.75, 1.0, 1.25):
            out.append(dict(N=sizes[idx], Ra=Ra, n_pl=n, Pr=1.0, seed=100 + idx))
            idx += 1
    return out


def serving_trace(count: int = 500, rate: float = 2.0, seed: int = 5, sizes=(33, 49, 65, 97, 129)):
    """Poisson arrivals (exponential gaps, mean 1/rate) of cavity solves with the
    grid size uniform over ``sizes``, Ra log-uniform in [1e2, 1e5] and n uniform in
    [0.7, 1.3]; request seeds 1000 + index."""
    U = uniform01(seed, 4 * count).reshape(count, 4)
    t = 0.0
    out = []
    for q in range(count):
        t += -math.log(1.0 - U[q, 0]) / rate
        N = sizes[min(int(U[q, 1] * len(sizes)), len(sizes) - 1)]
        Ra = 10.0 ** (2.0 + 3.0 * U[q, 2])
        n = 0.7 + 0.6 * U[q, 3]
        out.append(dict(arrival=t, N=N, Ra=Ra, n_pl=n, Pr=1.0, seed=1000 + q))
    return out
