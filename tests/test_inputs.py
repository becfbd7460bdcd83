"""The seeded input generators (no method arithmetic): SplitMix64 against its
published outputs for seed 0 (Steele, Lea & Flood 2014; reference implementation
by S. Vigna), and the initial-condition and workload recipes."""
import numpy as np

from paper_2411_06563_amd.inputs import batched_cavities, initial_state, serving_trace, splitmix64, uniform01


def test_splitmix64_published_values():
    assert [int(v) for v in splitmix64(0, 3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_splitmix64_counter_offsets():
    a = splitmix64(123, 10)
    b = splitmix64(123, 4, offset=6)
    assert np.array_equal(a[6:], b)
    u = uniform01(9, 1000)
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.05


def test_initial_state_recipe():
    N = 9
    s = initial_state(N, seed=1, noise=1e-3)
    x = np.linspace(0, 1, N)
    T = s["T"]
    assert np.all(T[:, :, 0] == 1.0) and np.all(T[:, :, -1] == 0.0)
    dev = T[1:-1, 1:-1, 1:-1] - (1 - x[1:-1])[None, None, :]
    U = uniform01(1, (N - 2) ** 3).reshape(N - 2, N - 2, N - 2)
    assert np.allclose(dev, 1e-3 * (2 * U - 1), rtol=0, atol=1e-15)
    for f in ("u", "v", "w", "p"):
        assert not s[f].any()


def test_workload_generators():
    cav = batched_cavities(4)
    assert len(cav) == 12
    assert sorted(c["N"] for c in cav) == [33] * 4 + [65] * 4 + [97] * 4
    assert [(c["Ra"], c["n_pl"]) for c in cav[:4]] == [(1e2, 0.75), (1e2, 1.0), (1e2, 1.25), (1e3, 0.75)]
    tr = serving_trace(500)
    t = np.array([r["arrival"] for r in tr])
    assert np.all(np.diff(t) > 0)
    assert 0.4 < np.mean(np.diff(t)) < 0.6
    assert {r["N"] for r in tr} == {33, 49, 65, 97, 129}
    assert all(1e2 <= r["Ra"] <= 1e5 and 0.7 <= r["n_pl"] <= 1.3 for r in tr)
