"""ctypes wrapper of the FP64 CPU oracle (``hosc_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and by
the CPU-baseline leg of the benchmark.  The product library never imports it and
shares no code with it.

Arrays are numpy float64 of shape (N, N, N) indexed [k, j, i] (x fastest in
memory), i.e. ``a[k, j, i]`` is node (x_i, y_j, z_k) with x_i = i h, h = 1/(N-1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hosc_oracle.c")
LIB = os.path.join(HERE, "libhosc_oracle.so")
# another build of the oracle (a copy with a planted mistake, for the tests that
# show the pins catch such mistakes); never compiled over by build()
ALT = os.environ.get("HOSC_ORACLE_LIB")
if ALT:
    LIB = ALT

_dp = ctypes.POINTER(ctypes.c_double)


class _Params(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int32), ("maxit", ctypes.c_int32), ("dense", ctypes.c_int32), ("p_iters", ctypes.c_int32),
        ("Ra", ctypes.c_double), ("Pr", ctypes.c_double), ("n_pl", ctypes.c_double), ("dt", ctypes.c_double),
        ("theta_hot", ctypes.c_double), ("theta_cold", ctypes.c_double), ("theta_ref", ctypes.c_double),
        ("lam", ctypes.c_double), ("div_tol", ctypes.c_double), ("i2_floor", ctypes.c_double),
        ("phi", ctypes.c_double), ("solve_tol", ctypes.c_double), ("eta_relax", ctypes.c_double),
    ]


class _State(ctypes.Structure):
    _fields_ = [(n, _dp) for n in ("u", "v", "w", "T", "p", "up", "vp", "wp", "etap", "Eup", "Evp", "Ewp")] + [
        ("first", ctypes.c_int32), ("pad", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("res", ctypes.c_double * 4), ("maxdiv", ctypes.c_double), ("relres", ctypes.c_double * 4),
                ("iters", ctypes.c_int32 * 4), ("corrected", ctypes.c_int32), ("status", ctypes.c_int32)]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, optional OpenMP)."""
    if ALT:
        return LIB
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P, S, I = ctypes.POINTER(_Params), ctypes.POINTER(_State), ctypes.POINTER(_Info)
        L.or_step.argtypes = [P, S, I]
        L.or_assemble.argtypes = [P, S, _dp, _dp, _dp]
        L.or_apply_B.argtypes = [P, S, ctypes.c_int, _dp, _dp]
        L.or_eta_field.argtypes = [P, _dp, _dp, _dp, _dp, _dp]
        L.or_estar_field.argtypes = [P, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_apply_bc.argtypes = [P, _dp, _dp, _dp, _dp, _dp]
        L.or_transport_step.argtypes = [P] + [_dp] * 12 + [_dp, ctypes.POINTER(ctypes.c_int)]
        L.or_diagnostics.argtypes = [P, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


@dataclass
class Params:
    """Problem parameters (Sec. 2.1: unit cube, Ra, Pr, power-law index n)."""
    N: int
    Ra: float = 1e3
    Pr: float = 1.0
    n_pl: float = 1.0
    dt: float = 1e-4
    theta_hot: float = 1.0
    theta_cold: float = 0.0
    theta_ref: float = 0.5
    lam: float | None = None           # None -> h^2 / (3 dt)
    div_tol: float = 0.0
    i2_floor: float = 1e-8
    phi: float = 1e-4
    solve_tol: float = 1e-13
    maxit: int = 20000
    dense: bool = False
    p_iters: int = 1                   # momentum solves per step at most (pressure iterations)
    eta_relax: float = 1.0             # weight of the new viscosity (1: the stated scheme)

    @property
    def h(self) -> float:
        return 1.0 / (self.N - 1)

    def c(self) -> _Params:
        lam = self.lam if self.lam is not None else self.h ** 2 / (3.0 * self.dt)
        return _Params(N=self.N, maxit=self.maxit, dense=int(self.dense), p_iters=self.p_iters, Ra=self.Ra, Pr=self.Pr,
                       n_pl=self.n_pl, dt=self.dt, theta_hot=self.theta_hot, theta_cold=self.theta_cold,
                       theta_ref=self.theta_ref, lam=lam, div_tol=self.div_tol, i2_floor=self.i2_floor,
                       phi=self.phi, solve_tol=self.solve_tol, eta_relax=self.eta_relax)


@dataclass
class StepInfo:
    res: list
    maxdiv: float
    relres: list
    iters: list
    corrected: int
    status: int


class Oracle:
    """Holds a state (levels n and n-1) and advances it with the oracle."""

    FIELDS = ("u", "v", "w", "T", "p", "up", "vp", "wp", "etap", "Eup", "Evp", "Ewp")

    def __init__(self, params: Params):
        self.params = params
        N = params.N
        self.a = {f: np.zeros((N, N, N)) for f in self.FIELDS}
        self.first = 1
        self._cp = params.c()

    def set_state(self, u=None, v=None, w=None, T=None, p=None, apply_bc=True):
        """Set level n (level n-1 is taken equal to it at the next step)."""
        for name, arr in (("u", u), ("v", v), ("w", w), ("T", T), ("p", p)):
            if arr is not None:
                self.a[name][...] = arr
        if apply_bc:
            lib().or_apply_bc(ctypes.byref(self._cp), *(_ptr(self.a[f]) for f in ("u", "v", "w", "T", "p")))
        self.first = 1

    def _cstate(self) -> _State:
        s = _State(*(_ptr(self.a[f]) for f in self.FIELDS), self.first, 0)
        return s

    def step(self, n: int = 1) -> list[StepInfo]:
        out = []
        for _ in range(n):
            st = self._cstate()
            info = _Info()
            lib().or_step(ctypes.byref(self._cp), ctypes.byref(st), ctypes.byref(info))
            self.first = st.first
            out.append(StepInfo(list(info.res), info.maxdiv, list(info.relres), list(info.iters), info.corrected,
                                info.status))
        return out

    def assemble(self):
        """Right-hand sides b of the u, v, w, T increment systems, eta and E* at
        level n (the state is not advanced)."""
        N = self.params.N
        b4 = np.zeros((4, N, N, N))
        eta = np.zeros((N, N, N))
        E3 = np.zeros((3, N, N, N))
        st = self._cstate()
        lib().or_assemble(ctypes.byref(self._cp), ctypes.byref(st), _ptr(b4), _ptr(eta), _ptr(E3))
        self.first = st.first
        return b4, eta, E3

    def apply_B(self, eq: int, x: np.ndarray) -> np.ndarray:
        """Raw 7-point implicit operator (eq 0 momentum, 1 energy) applied to x."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros_like(x)
        st = self._cstate()
        if self.first:
            raise RuntimeError("apply_B needs level n-1: call assemble() or step() first")
        lib().or_apply_B(ctypes.byref(self._cp), ctypes.byref(st), eq, _ptr(x), _ptr(y))
        return y

    def diagnostics(self, fields: bool = False):
        return diagnostics(self.params, self.a["u"], self.a["v"], self.a["w"], self.a["T"], fields=fields)

    def state(self):
        return {f: self.a[f].copy() for f in ("u", "v", "w", "T", "p")}


def probe(fields: dict, points) -> np.ndarray:
    """Trilinear interpolation of u, v, w, T, p (arrays [k, j, i]) at points
    (n x 3, x y z in [0, 1]) from the eight surrounding nodes; n x 5.  The cell of a
    point on the far wall is the last one (its upper weight is 1)."""
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    N = fields["u"].shape[0]
    out = np.zeros((pts.shape[0], 5))
    for q, (x, y, z) in enumerate(pts):
        lo, t = [], []
        for c in (x, y, z):
            f = c * (N - 1)
            i = min(max(int(np.floor(f)), 0), N - 2)
            lo.append(i)
            t.append(f - i)
        for fi, name in enumerate(("u", "v", "w", "T", "p")):
            a = fields[name]
            val = 0.0
            for dk in (0, 1):
                for dj in (0, 1):
                    for di in (0, 1):
                        wgt = ((t[0] if di else 1 - t[0]) * (t[1] if dj else 1 - t[1])
                               * (t[2] if dk else 1 - t[2]))
                        val += wgt * a[lo[2] + dk, lo[1] + dj, lo[0] + di]
            out[q, fi] = val
    return out


def num_threads() -> int:
    return int(lib().or_num_threads())


def eta_field(params: Params, u, v, w):
    N = params.N
    eta = np.zeros((N, N, N))
    I2 = np.zeros((N, N, N))
    cp = params.c()
    lib().or_eta_field(ctypes.byref(cp), _ptr(u), _ptr(v), _ptr(w), _ptr(eta), _ptr(I2))
    return eta, I2


def estar_field(params: Params, u, v, w, T, p, eta):
    N = params.N
    E = [np.zeros((N, N, N)) for _ in range(3)]
    cp = params.c()
    lib().or_estar_field(ctypes.byref(cp), _ptr(u), _ptr(v), _ptr(w), _ptr(T), _ptr(p), _ptr(eta),
                         *(_ptr(e) for e in E))
    return E


def diagnostics(params: Params, u, v, w, T, fields: bool = False) -> dict:
    N = params.N
    nuh = np.zeros((N, N))
    nuc = np.zeros((N, N))
    avh = np.zeros(N)
    avc = np.zeros(N)
    scal = np.zeros(10)
    el = np.zeros((N, N, N)) if fields else None
    bl = np.zeros((N, N, N)) if fields else None
    cp = params.c()
    lib().or_diagnostics(ctypes.byref(cp), _ptr(u), _ptr(v), _ptr(w), _ptr(T), _ptr(nuh), _ptr(nuc), _ptr(avh),
                         _ptr(avc), _ptr(scal), _ptr(el), _ptr(bl))
    out = dict(nu_hot=nuh, nu_cold=nuc, nuavg_hot=avh, nuavg_cold=avc, nu_mean_hot=scal[0], nu_mean_cold=scal[1],
               nu_max_hot=scal[2], nu_max_cold=scal[3], e_total=scal[4], e_ht=scal[5], e_ff=scal[6],
               be_global=scal[7], be_mean=scal[8], nu_local_max_hot=scal[9])
    if fields:
        out["e_local"] = el
        out["be_local"] = bl
    return out


def transport_step(params: Params, L, G, H, I, E, Lp, Gp, Hp, Ip, Ep, chi, chi_new_walls):
    """One HOSC step of the generic PDE (Eq. 1) with Dirichlet walls taken from
    ``chi_new_walls`` (its interior is ignored).  Returns (chi_new, relres, iters)."""
    arrs = [np.ascontiguousarray(a, dtype=np.float64) if a is not None else None
            for a in (L, G, H, I, E, Lp, Gp, Hp, Ip, Ep, chi)]
    out = np.array(chi_new_walls, dtype=np.float64, copy=True, order="C")
    relres = ctypes.c_double(0.0)
    iters = ctypes.c_int(0)
    cp = params.c()
    st = lib().or_transport_step(ctypes.byref(cp), *(_ptr(a) for a in arrs), _ptr(out), ctypes.byref(relres),
                                 ctypes.byref(iters))
    if st != 0:
        raise RuntimeError(f"oracle transport solve failed (status {st}, relres {relres.value})")
    return out, relres.value, iters.value
