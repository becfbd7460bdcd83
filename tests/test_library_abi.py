"""The C-ABI library loads on a host without a GPU and exports every function that
include/hosc.h declares; parameter validation and workspace sizing run on the
host (no compute call is made here)."""
import ctypes

import pytest

from paper_2411_06563_amd import hosc


def test_exports_every_declared_symbol():
    L = hosc.lib()
    names = hosc.library_exports()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n


def test_params_default_and_validation():
    p = hosc.params(17)
    assert p.N == 17 and p.Ra == 1e3 and p.Pr == 1.0 and p.n_pl == 1.0 and p.solve_rtol == 1e-10
    assert hosc.workspace_bytes(p) > 30 * 17 ** 3 * 8
    for N, bad in ((4, {}), (1026, {}), (17, dict(Pr=0.0)), (17, dict(dt=-1.0)), (17, dict(n_pl=0.0)),
                   (17, dict(n_pl=2.5)), (17, dict(omega=2.0)), (17, dict(omega=-0.5)), (17, dict(solve_rtol=0.0)),
                   (17, dict(solve_rtol=1.0)), (17, dict(Ra=float("nan"))), (17, dict(Ra=-1.0)),
                   (17, dict(p_iters=-1)), (17, dict(p_iters=65)), (17, dict(eta_relax=0.0)),
                   (17, dict(eta_relax=1.5)), (17, dict(i2_floor=0.0)), (17, dict(phi=-1e-4)),
                   (17, dict(precision=2)), (17, dict(solver=7)), (17, dict(check_every=-1)),
                   (17, dict(solve_maxit=0)), (17, dict(theta_hot=float("inf")))):
        q = hosc.params(N, **bad)
        with pytest.raises(hosc.HoscError) as e:
            hosc.workspace_bytes(q)
        assert e.value.name == "HOSC_E_ARG", (N, bad)
    for ok in (dict(p_iters=0), dict(p_iters=64), dict(eta_relax=1e-3), dict(eta_relax=1.0), dict(n_pl=2.0)):
        assert hosc.workspace_bytes(hosc.params(17, **ok)) > 0


def test_workspace_scales_with_grid():
    b65 = hosc.workspace_bytes(hosc.params(65))
    b129 = hosc.workspace_bytes(hosc.params(129))
    assert 6.0 < b129 / b65 < 9.0
    sor = hosc.workspace_bytes(hosc.params(129, solver=hosc.SOLVER_SOR))
    assert sor < 0.6e9 < b129 < 1.1e9    # BiCGSTAB vectors are carved only when that solver may run


def test_create_rejects_bad_workspace():
    L = hosc.lib()
    p = hosc.params(17)
    h = ctypes.c_void_p()
    st = L.hosc_create(ctypes.byref(p), None, 0, None, ctypes.byref(h))
    assert hosc.lib().hosc_status_string(st).decode() == "HOSC_E_ARG"
    st = L.hosc_create(ctypes.byref(p), ctypes.c_void_p(256), 10, None, ctypes.byref(h))
    assert hosc.lib().hosc_status_string(st).decode() == "HOSC_E_NOMEM"
    assert b"workspace" in L.hosc_last_error(None)


C_NAMES = {"lam": "lambda"}     # binding field names that differ from the C names (Python keywords)


def _c_layout(structs):
    """sizeof and every field offset of the ABI structs as a C compiler lays them
    out from include/hosc.h."""
    import os
    import subprocess
    import tempfile
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hosc.h"', "int main(void) {"]
    for cname, ct in structs:
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in ct._fields_:
            cf = C_NAMES.get(f, f)
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {cf}));')
    lines.append("return 0; }")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        with open(src, "w") as f:
            f.write("\n".join(lines))
        subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(root, "include"), "-I",
                        "/opt/rocm/include", src, "-o", exe], check=True, capture_output=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    return dict((k, int(v)) for k, v in (ln.split() for ln in out.splitlines()))


def test_binding_structs_match_the_c_layout():
    structs = [("hosc_params", hosc.CParams), ("hosc_step_info", hosc.CStepInfo), ("hosc_diag", hosc.CDiag),
               ("hosc_perf", hosc.CPerf), ("hosc_request", hosc.CRequest), ("hosc_result", hosc.CResult),
               ("hosc_server_stats", hosc.CServerStats)]
    c = _c_layout(structs)
    for cname, ct in structs:
        assert c[cname] == ctypes.sizeof(ct), cname
        for f, _ in ct._fields_:
            assert c[f"{cname}.{f}"] == getattr(ct, f).offset, (cname, f)


def test_server_workspace_sizing_and_create_validation():
    """The server takes its device memory from the caller: the workspace is the
    arena of the budget plus the fused-launch tables; bad sizes and a missing or
    misaligned workspace fail on the host, before any device call."""
    L = hosc.lib()
    n = ctypes.c_size_t(0)
    assert L.hosc_server_workspace_bytes(1 << 20, 4, ctypes.byref(n)) == 0
    base = n.value
    assert base > 1 << 20
    assert L.hosc_server_workspace_bytes((1 << 20) + 100, 4, ctypes.byref(n)) == 0 and n.value == base
    assert L.hosc_server_workspace_bytes(1 << 20, 8, ctypes.byref(n)) == 0 and n.value > base
    for budget, cap in ((100, 4), (1 << 20, 0), (1 << 20, 1025)):
        assert L.hosc_server_workspace_bytes(budget, cap, ctypes.byref(n)) == -1
    h = ctypes.c_void_p()
    assert L.hosc_server_create(None, 1 << 30, 1 << 20, 4, None, ctypes.byref(h)) == -1
    assert L.hosc_server_create(ctypes.c_void_p(256 * 1024 + 8), 1 << 30, 1 << 20, 4, None, ctypes.byref(h)) == -1
    assert L.hosc_server_create(ctypes.c_void_p(256 * 1024), 1000, 1 << 20, 4, None, ctypes.byref(h)) == -2
    assert not h.value


def test_stream_mix_probe_rejects_bad_arguments():
    """The measurement probe validates its buffers on the host before any HIP call."""
    L = hosc.lib()
    ms = ctypes.c_double(0.0)
    cases = [(None, 4096, 160, 1), (4096, None, 160, 1), (4096, 1 << 20, 0, 1), (4096, 1 << 20, 160, 0),
             (4104, 1 << 20, 160, 1), (4096, (1 << 20) + 8, 160, 1), (4096, 1 << 20, 168, 1),
             (4096, 4096 + 14 * 160, 160, 1),    # in-place arrays start inside the read arrays
             (1 << 20, (1 << 20) - 4 * 160 + 16, 160, 1)]    # read arrays start inside the in-place arrays
    for rd, up, nbytes, reps in cases:
        st = L.hosc_stream_mix_bandwidth(ctypes.c_void_p(rd) if rd else None, ctypes.c_void_p(up) if up else None,
                                         nbytes, reps, None, ctypes.byref(ms))
        assert L.hosc_status_string(st).decode() == "HOSC_E_ARG", (rd, up, nbytes, reps)
