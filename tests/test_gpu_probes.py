"""The library's streaming probe with the half-sweep's access mix (a measurement aid
that bench.py reports beside the sweep's bandwidth): every launch updates every
element of the in-place arrays exactly once and touches nothing else."""
import ctypes

import pytest

from paper_2411_06563_amd import hosc

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("elems", [1000, 4096, 70001])    # 16-byte elements per array; ragged and whole blocks
def test_stream_mix_probe_updates(elems):
    import torch
    print(f"[stream-mix probe] {elems} elements per array", flush=True)
    nbytes = 16 * elems
    rd = torch.ones(15 * nbytes // 8, dtype=torch.float64, device="cuda:0")
    guard = 64
    up = torch.ones(4 * nbytes // 8 + guard, dtype=torch.float64, device="cuda:0")
    up[4 * nbytes // 8:] = -7.0
    ms = ctypes.c_double(0.0)
    reps = 10
    st = torch.cuda.current_stream().cuda_stream
    r = hosc.lib().hosc_stream_mix_bandwidth(ctypes.c_void_p(rd.data_ptr()), ctypes.c_void_p(up.data_ptr()), nbytes,
                                             reps, ctypes.c_void_p(st), ctypes.byref(ms))
    torch.cuda.synchronize()
    assert r == 0
    assert ms.value > 0.0
    # v <- v/2 + 15 per launch from v = 1, one warm-up launch and `reps` timed: 30 - 29 / 2^k, exact in binary
    k = reps + 1
    want = 30.0 - 29.0 / 2.0 ** k
    got = up[:4 * nbytes // 8].cpu()
    assert bool((got == want).all()), (float(got.min()), float(got.max()), want)
    assert bool((up[4 * nbytes // 8:].cpu() == -7.0).all())
    assert bool((rd.cpu() == 1.0).all())


def test_stream_mix_bandwidth_binding():
    gbs = hosc.stream_mix_bandwidth(8 * (127 ** 3 // 2), 5)
    print(f"[stream-mix probe] 129^3 colour-half arrays: {gbs:.0f} GB/s", flush=True)
    assert 500.0 < gbs < 20000.0
