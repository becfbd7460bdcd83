"""Python binding of libhosc (include/hosc.h): argument marshalling only.

Every step of the method runs in the HIP library; PyTorch only provides the
device workspace and the stream.  The library must be built (``build.py``); if the
shared object is missing it is built once, and if the build is impossible the
import fails loudly -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

import numpy as np

from . import build as _build

LIB_PATH = _build.LIB
HEADER = os.path.join(_build.ROOT, "include", "hosc.h")

HOSC_FP64 = 0
HOSC_FP32_REFINED = 1
SOLVER_AUTO = 0
SOLVER_SOR = 1
SOLVER_BICGSTAB = 2

_dp = ctypes.POINTER(ctypes.c_double)


class HoscError(RuntimeError):
    def __init__(self, status: int, name: str, msg: str):
        super().__init__(f"{name}: {msg}")
        self.status = status
        self.name = name


class CParams(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("precision", ctypes.c_int32), ("Ra", ctypes.c_double),
                ("Pr", ctypes.c_double), ("n_pl", ctypes.c_double), ("dt", ctypes.c_double),
                ("theta_hot", ctypes.c_double), ("theta_cold", ctypes.c_double), ("theta_ref", ctypes.c_double),
                ("lam", ctypes.c_double), ("div_tol", ctypes.c_double), ("solve_rtol", ctypes.c_double),
                ("solve_maxit", ctypes.c_int32), ("check_every", ctypes.c_int32), ("solver", ctypes.c_int32),
                ("p_iters", ctypes.c_int32), ("omega", ctypes.c_double),
                ("i2_floor", ctypes.c_double), ("phi", ctypes.c_double), ("eta_relax", ctypes.c_double)]


class CStepInfo(ctypes.Structure):
    _fields_ = [("res", ctypes.c_double * 4), ("relres", ctypes.c_double * 4), ("maxdiv", ctypes.c_double),
                ("step", ctypes.c_int64), ("sweeps", ctypes.c_int32 * 2), ("bicg_iters", ctypes.c_int32 * 2),
                ("omega", ctypes.c_double * 2), ("dominance", ctypes.c_double * 2), ("corrected", ctypes.c_int32),
                ("status", ctypes.c_int32)]


class CDiag(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("nu_mean_hot", "nu_mean_cold", "nu_max_hot", "nu_max_cold",
                                               "e_total", "e_ht", "e_ff", "be_global", "be_mean",
                                               "nu_local_max_hot")]


class CPerf(ctypes.Structure):
    _fields_ = [("sweep_launches", ctypes.c_int64), ("sweep_ms", ctypes.c_double), ("sweep_bytes", ctypes.c_double),
                ("assemble_launches", ctypes.c_int64), ("assemble_ms", ctypes.c_double),
                ("assemble_bytes", ctypes.c_double), ("bicg_launches", ctypes.c_int64), ("bicg_ms", ctypes.c_double),
                ("bicg_bytes", ctypes.c_double), ("refine_launches", ctypes.c_int64), ("refine_ms", ctypes.c_double),
                ("refine_bytes", ctypes.c_double)]


class CRequest(ctypes.Structure):
    _fields_ = [("params", CParams), ("seed", ctypes.c_uint64), ("noise_amp", ctypes.c_double),
                ("res_tol", ctypes.c_double), ("max_steps", ctypes.c_int64), ("t_arrival", ctypes.c_double)]


class CResult(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int32), ("steady", ctypes.c_int32),
                ("steps", ctypes.c_int64), ("res", ctypes.c_double), ("t_arrival", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double), ("diag", CDiag)]


class CServerStats(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int64), ("resident", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("server_steps", ctypes.c_int64), ("cavity_steps", ctypes.c_int64), ("budget", ctypes.c_size_t),
                ("in_use", ctypes.c_size_t), ("peak", ctypes.c_size_t), ("busy_s", ctypes.c_double)]


_lib = None


def library_exports() -> list[str]:
    """Function names declared in include/hosc.h."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:hosc_status|const char \*|void)\s*\*?\s*(hosc_\w+)\s*\(", text, re.M)))


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        _build.build()
    # torch provides the device memory and streams: its device runtime is loaded
    # first, so that the library binds to the same runtime as the tensors it is given
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    P = ctypes.POINTER(CParams)
    L.hosc_params_default.argtypes = [P]
    L.hosc_workspace_bytes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    L.hosc_create.argtypes = [P, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.hosc_destroy.argtypes = [vp]
    L.hosc_init_fields.argtypes = [vp, ctypes.c_uint64, ctypes.c_double]
    L.hosc_set_state.argtypes = [vp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int32]
    L.hosc_get_state.argtypes = [vp, _dp, _dp, _dp, _dp, _dp]
    L.hosc_step.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(CStepInfo)]
    L.hosc_run_to_steady.argtypes = [vp, ctypes.c_double, ctypes.c_int64, ctypes.POINTER(CStepInfo)]
    L.hosc_diagnostics.argtypes = [vp, ctypes.POINTER(CDiag), _dp, _dp, _dp, _dp]
    L.hosc_entropy_fields.argtypes = [vp, _dp, _dp]
    L.hosc_probe.argtypes = [vp, _dp, ctypes.c_int32, _dp]
    L.hosc_debug_assemble.argtypes = [vp, _dp, _dp, _dp, _dp, _dp]
    L.hosc_transport_step.argtypes = [vp] + [_dp] * 12 + [ctypes.POINTER(CStepInfo)]
    L.hosc_diagnostics_noalloc.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, vp]
    L.hosc_perf_enable.argtypes = [vp, ctypes.c_int32]
    L.hosc_perf_get.argtypes = [vp, ctypes.POINTER(CPerf)]
    L.hosc_copy_bandwidth.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_double)]
    L.hosc_stream_mix_bandwidth.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int32, vp,
                                            ctypes.POINTER(ctypes.c_double)]
    L.hosc_last_error.argtypes = [vp]
    L.hosc_last_error.restype = ctypes.c_char_p
    L.hosc_batch_workspace_bytes.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
    L.hosc_batch_create.argtypes = [P, ctypes.c_int32, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.hosc_batch_destroy.argtypes = [vp]
    L.hosc_batch_cavity.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(vp)]
    L.hosc_batch_init_fields.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), ctypes.c_double]
    L.hosc_batch_step.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(CStepInfo)]
    L.hosc_batch_run_to_steady.argtypes = [vp, ctypes.c_double, ctypes.c_int64, ctypes.POINTER(CStepInfo)]
    L.hosc_batch_tune.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.hosc_batch_set_grid.argtypes = [vp, ctypes.c_int32]
    L.hosc_batch_perf_enable.argtypes = [vp, ctypes.c_int32]
    L.hosc_batch_perf_get.argtypes = [vp, ctypes.POINTER(CPerf)]
    L.hosc_batch_graph_launches.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.hosc_server_workspace_bytes.argtypes = [ctypes.c_size_t, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
    L.hosc_server_create.argtypes = [vp, ctypes.c_size_t, ctypes.c_size_t, ctypes.c_int32, vp, ctypes.POINTER(vp)]
    L.hosc_server_destroy.argtypes = [vp]
    L.hosc_server_now.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.hosc_server_submit.argtypes = [vp, ctypes.POINTER(CRequest), ctypes.POINTER(ctypes.c_uint64)]
    L.hosc_server_step.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.hosc_server_poll.argtypes = [vp, ctypes.POINTER(CResult), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    L.hosc_server_stats_get.argtypes = [vp, ctypes.POINTER(CServerStats)]
    L.hosc_server_last_error.argtypes = [vp]
    L.hosc_server_last_error.restype = ctypes.c_char_p
    L.hosc_batch_last_error.argtypes = [vp]
    L.hosc_batch_last_error.restype = ctypes.c_char_p
    L.hosc_status_string.argtypes = [ctypes.c_int]
    L.hosc_status_string.restype = ctypes.c_char_p
    _lib = L
    return L


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _check(st: int, handle=None, batch=None, server=None):
    if st != 0:
        L = lib()
        if server is not None:
            msg = L.hosc_server_last_error(server)
        elif batch is not None:
            msg = L.hosc_batch_last_error(batch)
        else:
            msg = L.hosc_last_error(handle)
        raise HoscError(st, L.hosc_status_string(st).decode(), (msg or b"").decode())


def params(N: int, **kw) -> CParams:
    """hosc_params with the library defaults, overridden by keyword arguments
    (``lam`` is the artificial-compressibility lambda; 0 -> h^2/(3 dt))."""
    p = CParams()
    _check(lib().hosc_params_default(ctypes.byref(p)))
    p.N = N
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def workspace_bytes(p: CParams) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().hosc_workspace_bytes(ctypes.byref(p), ctypes.byref(n)))
    return n.value


def diagnostics_noalloc(p: CParams, u, v, w, T, out, nuavg_hot=None, nuavg_cold=None, stream=None):
    """hosc_diagnostics_noalloc on device tensors (float64, N^3 fields; out holds 10
    doubles; nuavg_* N doubles or None): launches only, on ``stream`` (default: torch's
    current stream of the tensors' device)."""
    import torch
    for t in (u, v, w, T, out) + tuple(x for x in (nuavg_hot, nuavg_cold) if x is not None):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("device float64 contiguous tensors are required")
    st = stream if stream is not None else torch.cuda.current_stream(u.device)
    ptr = [ctypes.c_void_p(t.data_ptr()) if t is not None else None for t in (u, v, w, T, out, nuavg_hot, nuavg_cold)]
    r = lib().hosc_diagnostics_noalloc(ctypes.byref(p), *ptr, ctypes.c_void_p(st.cuda_stream))
    _check(r)


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 10, device: str = "cuda:0") -> float:
    """Achievable HBM bandwidth (GB/s, read + write) of a plain copy kernel."""
    import torch
    with torch.cuda.device(torch.device(device)):
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=device)
        dst = torch.empty_like(src)
        ms = ctypes.c_double(0.0)
        st = torch.cuda.current_stream().cuda_stream
        _check(lib().hosc_copy_bandwidth(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nbytes,
                                         reps, ctypes.c_void_p(st), ctypes.byref(ms)))
        torch.cuda.synchronize()
    return 2.0 * nbytes / (ms.value * 1e-3) / 1e9



def stream_mix_bandwidth(nbytes: int, reps: int = 10, device: str = "cuda:0") -> float:
    """Bandwidth (GB/s, 23 * nbytes per launch) of a streaming kernel with a
    red-black half-sweep's mix: 15 read-only arrays and 4 rewritten in place, nbytes
    each (rounded down to a multiple of 16)."""
    import torch
    nbytes -= nbytes % 16
    with torch.cuda.device(torch.device(device)):
        rd = torch.ones(15 * nbytes // 8, dtype=torch.float64, device=device)
        up = torch.ones(4 * nbytes // 8, dtype=torch.float64, device=device)
        ms = ctypes.c_double(0.0)
        st = torch.cuda.current_stream().cuda_stream
        _check(lib().hosc_stream_mix_bandwidth(ctypes.c_void_p(rd.data_ptr()), ctypes.c_void_p(up.data_ptr()), nbytes,
                                               reps, ctypes.c_void_p(st), ctypes.byref(ms)))
        torch.cuda.synchronize()
        del rd, up
    return 23.0 * nbytes / (ms.value * 1e-3) / 1e9

@dataclass
class StepInfo:
    res: list
    relres: list
    maxdiv: float
    step: int
    sweeps: list
    bicg_iters: list
    omega: list
    dominance: list
    corrected: int
    status: int

    @classmethod
    def of(cls, c: CStepInfo):
        return cls(list(c.res), list(c.relres), c.maxdiv, c.step, list(c.sweeps), list(c.bicg_iters), list(c.omega),
                   list(c.dominance), c.corrected, c.status)


class Solver:
    """One cavity on one device; workspace and stream from torch."""

    def __init__(self, p: CParams, device: str = "cuda:0", stream=None):
        import torch
        self.p = p
        self.N = p.N
        self.device = torch.device(device)
        nbytes = workspace_bytes(p)
        with torch.cuda.device(self.device):
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            base = self.ws.data_ptr()
            off = (-base) % 256
            h = ctypes.c_void_p()
            _check(lib().hosc_create(ctypes.byref(p), ctypes.c_void_p(base + off), nbytes,
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h

    @classmethod
    def borrowed(cls, handle, p: CParams, owner):
        """A view of a solver owned by a batch (closing it does nothing)."""
        s = cls.__new__(cls)
        s.p, s.N, s.h, s._owner = p, p.N, handle, owner
        return s

    def close(self):
        if getattr(self, "_owner", None) is not None:
            return
        if getattr(self, "h", None):
            lib().hosc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def init_fields(self, seed: int, noise: float = 1e-3):
        _check(lib().hosc_init_fields(self.h, seed, noise), self.h)

    def set_state(self, u=None, v=None, w=None, T=None, p=None, apply_bc: bool = True):
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (u, v, w, T, p)]
        for a in arrs:
            if a is not None and a.size != self.N ** 3:
                raise ValueError("fields must hold N^3 values")
        _check(lib().hosc_set_state(self.h, *(_ptr(a) for a in arrs), int(apply_bc)), self.h)

    def get_state(self, out: dict = None) -> dict:
        """u, v, w, T, p as (N, N, N) arrays; `out` may hold the five arrays to fill
        (C-contiguous float64 of N^3 values each, e.g. views of page-locked memory)."""
        N = self.N
        names = ("u", "v", "w", "T", "p")
        if out is None:
            out = {f: np.empty((N, N, N)) for f in names}
        for f in names:
            a = out[f]
            if a.dtype != np.float64 or not a.flags["C_CONTIGUOUS"] or a.size != N ** 3 or not a.flags["WRITEABLE"]:
                raise ValueError(f"out[{f!r}] must be a writeable C-contiguous float64 array of N^3 values")
        _check(lib().hosc_get_state(self.h, *(_ptr(out[f]) for f in names)), self.h)
        return out

    def step(self, n: int = 1) -> StepInfo:
        info = CStepInfo()
        _check(lib().hosc_step(self.h, n, ctypes.byref(info)), self.h)
        return StepInfo.of(info)

    def run_to_steady(self, tol: float, max_steps: int) -> StepInfo:
        info = CStepInfo()
        _check(lib().hosc_run_to_steady(self.h, tol, max_steps, ctypes.byref(info)), self.h)
        return StepInfo.of(info)

    def diagnostics(self, arrays: bool = True) -> dict:
        N = self.N
        d = CDiag()
        if arrays:
            avh, avc = np.empty(N), np.empty(N)
            nuh, nuc = np.empty((N, N)), np.empty((N, N))
        else:
            avh = avc = nuh = nuc = None
        _check(lib().hosc_diagnostics(self.h, ctypes.byref(d), _ptr(avh), _ptr(avc), _ptr(nuh), _ptr(nuc)), self.h)
        out = {n: getattr(d, n) for n, _ in CDiag._fields_}
        if arrays:
            out.update(nuavg_hot=avh, nuavg_cold=avc, nu_hot=nuh, nu_cold=nuc)
        return out

    def perf_enable(self, on: bool = True):
        _check(lib().hosc_perf_enable(self.h, int(on)), self.h)

    def perf(self) -> dict:
        c = CPerf()
        _check(lib().hosc_perf_get(self.h, ctypes.byref(c)), self.h)
        return {n: getattr(c, n) for n, _ in CPerf._fields_}

    def entropy_fields(self):
        N = self.N
        el, bl = np.empty((N, N, N)), np.empty((N, N, N))
        _check(lib().hosc_entropy_fields(self.h, _ptr(el), _ptr(bl)), self.h)
        return el, bl

    def probe(self, points) -> np.ndarray:
        """u, v, w, theta, p at points (n x 3, coordinates in [0, 1]) by trilinear
        interpolation; returns n x 5."""
        xyz = np.ascontiguousarray(np.asarray(points, dtype=np.float64).reshape(-1, 3))
        out = np.empty((xyz.shape[0], 5))
        _check(lib().hosc_probe(self.h, _ptr(xyz), xyz.shape[0], _ptr(out)), self.h)
        return out

    def debug_assemble(self) -> dict:
        N = self.N
        eta = np.empty((N, N, N))
        E = np.empty((3, N, N, N))
        b = np.empty((4, N, N, N))
        Bm = np.empty((7, N, N, N))
        Bt = np.empty((7, N, N, N))
        _check(lib().hosc_debug_assemble(self.h, _ptr(eta), _ptr(E), _ptr(b), _ptr(Bm), _ptr(Bt)), self.h)
        return dict(eta=eta, E=E, b=b, Bmom=Bm, Btheta=Bt)

    def transport_step(self, L, G, H, I, E, Lp, Gp, Hp, Ip, Ep, chi, chi_new_walls):
        """One step of the generic transport PDE (hosc_transport_step): level n and
        n-1 coefficient fields, chi at level n, Dirichlet walls of level n+1 taken from
        ``chi_new_walls``.  Returns (chi_new, StepInfo).  The solver has no state
        afterwards."""
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64)
                for a in (L, G, H, I, E, Lp, Gp, Hp, Ip, Ep, chi)]
        for a in arrs:
            if a is not None and a.size != self.N ** 3:
                raise ValueError("fields must hold N^3 values")
        out = np.array(chi_new_walls, dtype=np.float64, copy=True, order="C")
        if out.size != self.N ** 3:
            raise ValueError("fields must hold N^3 values")
        info = CStepInfo()
        _check(lib().hosc_transport_step(self.h, *(_ptr(a) for a in arrs), _ptr(out), ctypes.byref(info)), self.h)
        return out, StepInfo.of(info)


class Batch:
    """Many cavities advanced together with fused solver launches (hosc_batch_*)."""

    def __init__(self, plist, device: str = "cuda:0", stream=None):
        import torch
        self.plist = list(plist)
        n = len(self.plist)
        arr = (CParams * n)(*self.plist)
        self._arr = arr
        nbytes = ctypes.c_size_t(0)
        _check(lib().hosc_batch_workspace_bytes(arr, n, ctypes.byref(nbytes)), batch=None)
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
            # a stream of its own (default priority): the per-step phases are captured
            # as graphs, which the null stream does not allow
            self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
            base = self.ws.data_ptr()
            off = (-base) % 256
            h = ctypes.c_void_p()
            _check(lib().hosc_batch_create(arr, n, ctypes.c_void_p(base + off), nbytes.value,
                                           ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), batch=None)
        self.b = h
        self.cavities = []
        for i in range(n):
            ch = ctypes.c_void_p()
            _check(lib().hosc_batch_cavity(self.b, i, ctypes.byref(ch)), batch=self.b)
            self.cavities.append(Solver.borrowed(ch, self.plist[i], self))

    def __len__(self):
        return len(self.cavities)

    def close(self):
        if getattr(self, "b", None):
            lib().hosc_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_fields(self, seeds, noise: float = 1e-3):
        arr = (ctypes.c_uint64 * len(self.cavities))(*seeds)
        _check(lib().hosc_batch_init_fields(self.b, arr, noise), batch=self.b)

    def step(self, n: int = 1) -> list:
        infos = (CStepInfo * len(self.cavities))()
        _check(lib().hosc_batch_step(self.b, n, infos), batch=self.b)
        return [StepInfo.of(c) for c in infos]

    def run_to_steady(self, tol: float, max_steps: int, raise_on_error: bool = True):
        """hosc_batch_run_to_steady.  A cavity that fails stops while the others go on;
        with raise_on_error the first failure is raised after the call, otherwise
        (infos, error or None) is returned, error being that HoscError."""
        infos = (CStepInfo * len(self.cavities))()
        st = lib().hosc_batch_run_to_steady(self.b, tol, max_steps, infos)
        out = [StepInfo.of(c) for c in infos]
        err = None
        try:
            _check(st, batch=self.b)
        except HoscError as e:
            if raise_on_error:
                raise
            err = e
        return out if raise_on_error else (out, err)

    def tune(self) -> int:
        g = ctypes.c_int32(0)
        _check(lib().hosc_batch_tune(self.b, ctypes.byref(g)), batch=self.b)
        return g.value

    def set_grid(self, grid: int):
        _check(lib().hosc_batch_set_grid(self.b, grid), batch=self.b)

    def graph_launches(self) -> int:
        c = ctypes.c_int64(0)
        _check(lib().hosc_batch_graph_launches(self.b, ctypes.byref(c)), batch=self.b)
        return c.value

    def synchronize(self):
        self.stream.synchronize()

    def perf_enable(self, on: bool = True):
        _check(lib().hosc_batch_perf_enable(self.b, int(on)), batch=self.b)

    def perf(self) -> dict:
        c = CPerf()
        _check(lib().hosc_batch_perf_get(self.b, ctypes.byref(c)), batch=self.b)
        return {n: getattr(c, n) for n, _ in CPerf._fields_}


class Server:
    """Request loop over resident cavities (hosc_server_*): admission by HBM budget,
    continuous fused batching, results with their arrival/admission/completion times."""

    def __init__(self, budget_bytes: int, max_resident: int = 64, device: str = "cuda:0", stream=None):
        import torch
        self.device = torch.device(device)
        nbytes = ctypes.c_size_t(0)
        _check(lib().hosc_server_workspace_bytes(budget_bytes, max_resident, ctypes.byref(nbytes)), server=None)
        with torch.cuda.device(self.device):
            # torch provides the server's device memory: the arena and its tables
            self.ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
            base = self.ws.data_ptr()
            off = (-base) % 256
            h = ctypes.c_void_p()
            _check(lib().hosc_server_create(ctypes.c_void_p(base + off), nbytes.value, budget_bytes, max_resident,
                                            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), server=None)
        self.v = h

    def close(self):
        if getattr(self, "v", None):
            lib().hosc_server_destroy(self.v)
            self.v = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def now(self) -> float:
        t = ctypes.c_double(0.0)
        _check(lib().hosc_server_now(self.v, ctypes.byref(t)), server=self.v)
        return t.value

    def submit(self, p: CParams, seed: int, noise: float = 1e-3, res_tol: float = 1e-8, max_steps: int = 1000,
               t_arrival: float = -1.0) -> int:
        rq = CRequest(p, seed, noise, res_tol, max_steps, t_arrival)
        rid = ctypes.c_uint64(0)
        _check(lib().hosc_server_submit(self.v, ctypes.byref(rq), ctypes.byref(rid)), server=self.v)
        return rid.value

    def step(self) -> int:
        n = ctypes.c_int32(0)
        _check(lib().hosc_server_step(self.v, ctypes.byref(n)), server=self.v)
        return n.value

    def poll(self, max_results: int = 256) -> list:
        out = (CResult * max_results)()
        n = ctypes.c_int32(0)
        _check(lib().hosc_server_poll(self.v, out, max_results, ctypes.byref(n)), server=self.v)
        res = []
        for q in range(n.value):
            c = out[q]
            res.append(dict(id=c.id, status=c.status, steady=bool(c.steady), steps=c.steps, res=c.res,
                            t_arrival=c.t_arrival, t_admit=c.t_admit, t_done=c.t_done,
                            diag={f: getattr(c.diag, f) for f, _ in CDiag._fields_}))
        return res

    def stats(self) -> dict:
        c = CServerStats()
        _check(lib().hosc_server_stats_get(self.v, ctypes.byref(c)), server=self.v)
        return {f: getattr(c, f) for f, _ in CServerStats._fields_}
