"""ctypes wrapper of the CPU oracle (oracle/rhd_oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py, never by the product package. The oracle is a
plain FP64 implementation of the IMEX PD-ARS radiation step (He, Wibking &
Krumholz 2024, Sec. 3), shares no code with the HIP path, and is pinned by the
CPU tests against what the paper and the mathematics fix.

Where no closed form fixes a value (PPM face states in non-smooth fields), the
pins are the limiter's defining properties (flattening at an extremum, no
interior extremum of the parabola, edges within the neighbours' range, order
kept on monotone data) together with the invariants (conservation, symmetry,
translation invariance) and limits; the M1 closure is pinned at every flux
factor by the angular quadrature of its defining intensity.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# RHD_ORACLE_LIB names another build of the same source (the planted-mistake
# test loads deliberately broken copies this way); unset, the in-tree library.
_LIB_PATH = os.environ.get("RHD_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

OK, ENEWTON, ENONPHYS = 0, 1, 2


class OracleParams(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("closure", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("dx", ctypes.c_double),
        ("c", ctypes.c_double),
        ("chat", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("a_r", ctypes.c_double),
        ("kB_over_mu", ctypes.c_double),
        ("bc", ctypes.c_int32 * 3),
        ("v_order", ctypes.c_int32),
        ("newton_maxit", ctypes.c_int32),
        ("outer_maxit", ctypes.c_int32),
        ("newton_rtol", ctypes.c_double),
        ("outer_rtol", ctypes.c_double),
        ("scheme", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("hll_eps_cells", ctypes.c_double),
        ("kappa_T_power", ctypes.c_double),
        ("inflow_E", ctypes.c_double),
        ("inflow_F", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build_oracle
            build_oracle.build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(OracleParams)
        i64p = ctypes.POINTER(ctypes.c_int64)
        ip = ctypes.POINTER(ctypes.c_int)
        L.oracle_step.argtypes = [pp, dp, dp, dp, dp, dp, dp, ctypes.c_double, ctypes.c_int, i64p]
        L.oracle_step.restype = ctypes.c_int
        L.oracle_stage1.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp, ctypes.c_double, i64p]
        L.oracle_stage1.restype = ctypes.c_int
        L.oracle_transport.argtypes = [pp, dp, dp, dp, dp]
        L.oracle_transport.restype = None
        L.oracle_source.argtypes = [pp, dp, dp, dp, dp, dp, dp, ctypes.c_double, ip, ip, i64p]
        L.oracle_source.restype = ctypes.c_int
        L.oracle_ppm_edges.argtypes = [dp, ctypes.c_int64, dp, dp]
        L.oracle_ppm_edges.restype = None
        L.oracle_closure.argtypes = [pp, ctypes.c_int, ctypes.c_double, dp, dp]
        L.oracle_closure.restype = None
        L.oracle_hll.argtypes = [pp, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.oracle_hll.restype = None
        L.oracle_face_eps.argtypes = [pp, ctypes.c_double, ctypes.c_double]
        L.oracle_face_eps.restype = ctypes.c_double
        L.oracle_step_dual.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp, dp, dp, ctypes.c_double,
                                       ctypes.c_int, i64p]
        L.oracle_step_dual.restype = ctypes.c_int
        L.oracle_hydro_step.argtypes = [pp, dp, dp, ctypes.c_double, ctypes.c_int, i64p]
        L.oracle_hydro_step.restype = ctypes.c_int
        L.oracle_hydro_rhs.argtypes = [pp, dp, dp, dp, dp]
        L.oracle_hydro_rhs.restype = None
        L.oracle_hllc.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.oracle_hllc.restype = None
        L.oracle_rhd_step.argtypes = [pp, dp, dp, dp, dp, dp, dp, ctypes.c_double, ctypes.c_int,
                                      ctypes.c_int, i64p]
        L.oracle_rhd_step.restype = ctypes.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = None
        _lib = L
    return _lib


def make_params(p: dict) -> OracleParams:
    op = OracleParams()
    op.ndim = int(p["ndim"])
    op.closure = {"m1": 0, "eddington": 1}[p.get("closure", "m1")]
    n = tuple(p["n"]) + (1,) * (3 - len(p["n"]))
    for d in range(3):
        op.n[d] = int(n[d])
    op.dx = float(p["dx"])
    op.c = float(p["c"])
    op.chat = float(p["chat"])
    op.gamma = float(p["gamma"])
    op.a_r = float(p["a_r"])
    op.kB_over_mu = float(p["kB_over_mu"])
    bc = tuple(p.get("bc", (0, 0, 0))) + (0,) * 3
    for d in range(3):
        op.bc[d] = int(bc[d])
    op.v_order = int(p.get("v_order", 2))
    op.newton_maxit = int(p.get("newton_maxit", 50))
    op.outer_maxit = int(p.get("outer_maxit", 10))
    op.newton_rtol = float(p.get("newton_rtol", 1e-13))
    op.outer_rtol = float(p.get("outer_rtol", 1e-13))
    op.scheme = {"pdars": 0, "rk2ssp": 1}[p.get("scheme", "pdars")]
    op.pad_ = 0
    op.hll_eps_cells = float(p.get("hll_eps_cells", 0.0))
    op.kappa_T_power = float(p.get("kappa_T_power", 0.0))
    op.inflow_E = float(p.get("inflow_E", 0.0))
    op.inflow_F = float(p.get("inflow_F", 0.0))
    return op


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def step(p: dict, y: np.ndarray, rho, kP, kF, dt: float, nsteps: int, kE=None, jS=None):
    """Run nsteps steps. kE: energy-mean opacity (None: kP); jS: radiation
    injection rate per unit volume (None: no source). Returns (y_new, status,
    fail_cell)."""
    y = np.array(y, dtype=np.float64, order="C", copy=True)
    rho, kP, kF, kE, jS = _c(rho), _c(kP), _c(kF), _c(kE), _c(jS)
    fc = ctypes.c_int64(-1)
    st = lib().oracle_step(ctypes.byref(make_params(p)), _dp(y), _dp(rho), _dp(kP), _dp(kF),
                           _dp(kE), _dp(jS), float(dt), int(nsteps), ctypes.byref(fc))
    return y, st, fc.value


def stage1(p: dict, y: np.ndarray, rho, kP, kF, dt: float, kE=None, jS=None):
    y = _c(y)
    yh = np.empty_like(y)
    rho, kP, kF, kE, jS = _c(rho), _c(kP), _c(kF), _c(kE), _c(jS)
    fc = ctypes.c_int64(-1)
    st = lib().oracle_stage1(ctypes.byref(make_params(p)), _dp(y), _dp(yh), _dp(rho), _dp(kP),
                             _dp(kF), _dp(kE), _dp(jS), float(dt), ctypes.byref(fc))
    return yh, st, fc.value


def transport(p: dict, y: np.ndarray, rho=None, kF=None) -> np.ndarray:
    """s(y); rho and kF (chi_F = rho kF) are needed only with hll_eps_cells > 0."""
    y = _c(y)
    s = np.zeros_like(y)
    rho, kF = _c(rho), _c(kF)
    if float(p.get("hll_eps_cells", 0.0)) > 0.0 and (rho is None or kF is None):
        raise ValueError("hll_eps_cells > 0 needs rho and kF")
    lib().oracle_transport(ctypes.byref(make_params(p)), _dp(y), _dp(s), _dp(rho), _dp(kF))
    return s


def source(p: dict, y: np.ndarray, rho, kP, kF, tau: float, kE=None, jS=None):
    """Apply the local implicit source with theta*dt = tau to every cell (kE,
    jS as in step()). Returns (y_new, status, fail_cell, newton_iters,
    outer_iters)."""
    y = np.array(y, dtype=np.float64, order="C", copy=True)
    rho, kP, kF, kE, jS = _c(rho), _c(kP), _c(kF), _c(kE), _c(jS)
    N = rho.size
    it = np.zeros(N, dtype=np.int32)
    ou = np.zeros(N, dtype=np.int32)
    fc = ctypes.c_int64(-1)
    ip = ctypes.POINTER(ctypes.c_int)
    st = lib().oracle_source(ctypes.byref(make_params(p)), _dp(y), _dp(rho), _dp(kP), _dp(kF),
                             _dp(kE), _dp(jS), float(tau), it.ctypes.data_as(ip),
                             ou.ctypes.data_as(ip), ctypes.byref(fc))
    return y, st, fc.value, it.reshape(rho.shape), ou.reshape(rho.shape)


def ppm_edges(a: np.ndarray):
    a = _c(a)
    aL = np.full_like(a, np.nan)
    aR = np.full_like(a, np.nan)
    lib().oracle_ppm_edges(_dp(a), a.size, _dp(aL), _dp(aR))
    return aL, aR


def face_eps(p: dict, chi_a: float, chi_b: float) -> float:
    return float(lib().oracle_face_eps(ctypes.byref(make_params(p)), float(chi_a), float(chi_b)))


def closure(p: dict, ndim: int, E: float, F) -> np.ndarray:
    Fa = np.zeros(3)
    Fa[: len(F)] = F
    D = np.zeros(9)
    lib().oracle_closure(ctypes.byref(make_params(p)), int(ndim), float(E), _dp(Fa), _dp(D))
    return D.reshape(3, 3)


def hll(p: dict, ndim: int, d: int, Um, Up) -> np.ndarray:
    Um = _c(Um)
    Up = _c(Up)
    out = np.zeros(1 + ndim)
    lib().oracle_hll(ctypes.byref(make_params(p)), int(ndim), int(d), _dp(Um), _dp(Up), _dp(out))
    return out


def step_dual(p: dict, y, ty, rho, kP, tkP, kF, tkF, dt: float, nsteps: int, kE=None, jS=None):
    """Forward-mode tangent of nsteps steps (kE, jS without tangents). Returns (y,
    ty, status, fail_cell)."""
    y = np.array(y, dtype=np.float64, order="C", copy=True)
    ty = np.array(ty, dtype=np.float64, order="C", copy=True)
    rho, kP, tkP, kF, tkF, kE, jS = _c(rho), _c(kP), _c(tkP), _c(kF), _c(tkF), _c(kE), _c(jS)
    fc = ctypes.c_int64(-1)
    st = lib().oracle_step_dual(ctypes.byref(make_params(p)), _dp(y), _dp(ty), _dp(rho), _dp(kP),
                                _dp(tkP), _dp(kF), _dp(tkF), _dp(kE), _dp(jS), float(dt),
                                int(nsteps), ctypes.byref(fc))
    return y, ty, st, fc.value


def hydro_step(p: dict, y: np.ndarray, rho, dt: float, nsteps: int = 1):
    """nsteps RK2-SSP hydro steps (PPM + HLLC) of rho and of y's E_gas and
    momentum rows. Returns (y_new, rho_new, status, fail_cell)."""
    y = np.array(y, dtype=np.float64, order="C", copy=True)
    rho = np.array(rho, dtype=np.float64, order="C", copy=True)
    fc = ctypes.c_int64(-1)
    st = lib().oracle_hydro_step(ctypes.byref(make_params(p)), _dp(y), _dp(rho), float(dt),
                                 int(nsteps), ctypes.byref(fc))
    return y, rho, st, fc.value


def hydro_rhs(p: dict, y: np.ndarray, rho):
    """L(U) of the gas: (d rho/dt, d y/dt) with only the E_gas and momentum rows
    of the latter nonzero."""
    y, rho = _c(y), _c(rho)
    srho = np.zeros_like(rho)
    sy = np.zeros_like(y)
    lib().oracle_hydro_rhs(ctypes.byref(make_params(p)), _dp(y), _dp(rho), _dp(srho), _dp(sy))
    return srho, sy


def hllc(gamma: float, nd: int, d: int, WL, WR) -> np.ndarray:
    """HLLC flux along axis d between primitive states (rho, v_0..v_{nd-1}, p)."""
    WL, WR = _c(WL), _c(WR)
    out = np.zeros(2 + nd)
    lib().oracle_hllc(float(gamma), int(nd), int(d), _dp(WL), _dp(WR), _dp(out))
    return out


def rhd_step(p: dict, y: np.ndarray, rho, kP, kF, dt: float, nsub: int, nsteps: int, kE=None,
             jS=None):
    """Operator-split steps: each is one hydro step of dt, then nsub radiation
    steps of dt / nsub. Returns (y_new, rho_new, status, fail_cell)."""
    y = np.array(y, dtype=np.float64, order="C", copy=True)
    rho = np.array(rho, dtype=np.float64, order="C", copy=True)
    kP, kF, kE, jS = _c(kP), _c(kF), _c(kE), _c(jS)
    fc = ctypes.c_int64(-1)
    st = lib().oracle_rhd_step(ctypes.byref(make_params(p)), _dp(y), _dp(rho), _dp(kP), _dp(kF),
                               _dp(kE), _dp(jS), float(dt), int(nsub), int(nsteps),
                               ctypes.byref(fc))
    return y, rho, st, fc.value


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))
