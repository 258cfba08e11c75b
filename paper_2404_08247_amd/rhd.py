"""Python binding of librhd.so (the C ABI in include/rhd.h).

Argument marshalling only: every step of the radiation update runs in the HIP
kernels of the library. torch supplies device memory (the state, the scalar
fields and the workspace) and the stream. If the library is missing this module
raises on import; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librhd.so")

RHD_OK, RHD_EINVAL, RHD_ENEWTON, RHD_ENONPHYS, RHD_EHIP, RHD_EWORKSPACE = 0, -1, -2, -3, -4, -5
_STATUS = {0: "RHD_OK", -1: "RHD_EINVAL", -2: "RHD_ENEWTON", -3: "RHD_ENONPHYS", -4: "RHD_EHIP",
           -5: "RHD_EWORKSPACE"}
EXPORTED = ["rhd_workspace_bytes", "rhd_create", "rhd_step", "rhd_step_adjoint", "rhd_transport",
            "rhd_source", "rhd_stage1", "rhd_step_timed", "rhd_conserved_totals", "rhd_last_error",
            "rhd_destroy", "rhd_set_energy_opacity", "rhd_set_radiation_source",
            "rhd_hydro_step", "rhd_rhd_step", "rhd_hydro_signal_speed", "rhd_step_noalloc"]


class RHDParams(ctypes.Structure):
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
        ("precision", ctypes.c_int32),
        ("newton_maxit", ctypes.c_int32),
        ("outer_maxit", ctypes.c_int32),
        ("scheme", ctypes.c_int32),
        ("newton_rtol", ctypes.c_double),
        ("outer_rtol", ctypes.c_double),
        ("hll_eps_cells", ctypes.c_double),
        ("kappa_T_power", ctypes.c_double),
        ("inflow_E", ctypes.c_double),
        ("inflow_F", ctypes.c_double),
    ]


class RHDError(RuntimeError):
    def __init__(self, status: int, cell: int = -1, msg: str = ""):
        self.status = status
        self.cell = cell
        super().__init__(f"{_STATUS.get(status, status)}: {msg} (cell {cell})")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2404_08247_amd/build.py "
                          "(or __graft_entry__.build()); there is no fallback implementation")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    pp = ctypes.POINTER(RHDParams)
    L.rhd_workspace_bytes.argtypes = [pp, ctypes.c_int32]
    L.rhd_workspace_bytes.restype = ctypes.c_size_t
    L.rhd_create.argtypes = [pp, vp, vp, vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.rhd_create.restype = ctypes.c_int
    L.rhd_step.argtypes = [vp, vp, ctypes.c_double, ctypes.c_int32]
    L.rhd_step.restype = ctypes.c_int
    L.rhd_step_timed.argtypes = [vp, vp, ctypes.c_double, ctypes.c_int32,
                                 ctypes.POINTER(ctypes.c_double)]
    L.rhd_step_timed.restype = ctypes.c_int
    L.rhd_step_adjoint.argtypes = [vp, vp, ctypes.c_double, ctypes.c_int32, vp, vp, vp]
    L.rhd_step_adjoint.restype = ctypes.c_int
    L.rhd_transport.argtypes = [vp, vp, vp]
    L.rhd_transport.restype = ctypes.c_int
    L.rhd_source.argtypes = [vp, vp, ctypes.c_double]
    L.rhd_source.restype = ctypes.c_int
    L.rhd_stage1.argtypes = [vp, vp, vp, ctypes.c_double]
    L.rhd_stage1.restype = ctypes.c_int
    L.rhd_conserved_totals.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double)]
    L.rhd_conserved_totals.restype = ctypes.c_int
    L.rhd_last_error.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.c_char_p,
                                 ctypes.c_size_t]
    L.rhd_last_error.restype = ctypes.c_int
    L.rhd_destroy.argtypes = [vp]
    L.rhd_destroy.restype = None
    L.rhd_set_energy_opacity.argtypes = [vp, vp]
    L.rhd_set_energy_opacity.restype = ctypes.c_int
    L.rhd_set_radiation_source.argtypes = [vp, vp]
    L.rhd_set_radiation_source.restype = ctypes.c_int
    L.rhd_hydro_step.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_int32]
    L.rhd_hydro_step.restype = ctypes.c_int
    L.rhd_rhd_step.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_int32, ctypes.c_int32]
    L.rhd_rhd_step.restype = ctypes.c_int
    L.rhd_hydro_signal_speed.argtypes = [vp, vp, vp, ctypes.POINTER(ctypes.c_double)]
    L.rhd_hydro_signal_speed.restype = ctypes.c_int
    L.rhd_step_noalloc.argtypes = [pp, vp, vp, vp, vp, ctypes.c_double, ctypes.c_int32, vp,
                                   ctypes.POINTER(ctypes.c_int64)]
    L.rhd_step_noalloc.restype = ctypes.c_int
    return L


lib = _load()


def make_params(p: dict) -> RHDParams:
    rp = RHDParams()
    rp.ndim = int(p["ndim"])
    rp.closure = {"m1": 0, "eddington": 1}[p.get("closure", "m1")]
    n = tuple(p["n"]) + (1,) * (3 - len(p["n"]))
    for d in range(3):
        rp.n[d] = int(n[d])
    rp.dx = float(p["dx"])
    rp.c = float(p["c"])
    rp.chat = float(p["chat"])
    rp.gamma = float(p["gamma"])
    rp.a_r = float(p["a_r"])
    rp.kB_over_mu = float(p["kB_over_mu"])
    bc = tuple(p.get("bc", (0, 0, 0))) + (0, 0, 0)
    for d in range(3):
        rp.bc[d] = int(bc[d])
    rp.v_order = int(p.get("v_order", 2))
    rp.precision = {"fp64": 0, "mixed": 1}[p.get("precision", "fp64")]
    rp.newton_maxit = int(p.get("newton_maxit", 50))
    rp.outer_maxit = int(p.get("outer_maxit", 10))
    rp.scheme = {"pdars": 0, "rk2ssp": 1}[p.get("scheme", "pdars")]
    rp.newton_rtol = float(p.get("newton_rtol", 1e-13))
    rp.outer_rtol = float(p.get("outer_rtol", 1e-13))
    rp.hll_eps_cells = float(p.get("hll_eps_cells", 0.0))
    rp.kappa_T_power = float(p.get("kappa_T_power", 0.0))
    rp.inflow_E = float(p.get("inflow_E", 0.0))
    rp.inflow_F = float(p.get("inflow_F", 0.0))
    return rp


def step_noalloc(params: dict, state: torch.Tensor, rho: torch.Tensor, kappa_P: torch.Tensor,
                 kappa_F: Optional[torch.Tensor], dt: float, nsteps: int,
                 stream: Optional[torch.cuda.Stream] = None):
    """rhd_step_noalloc on torch's current stream (or `stream`): returns
    (status, fail_cell); raises nothing."""
    s = stream if stream is not None else torch.cuda.current_stream(state.device)
    cell = ctypes.c_int64(-1)
    st = lib.rhd_step_noalloc(ctypes.byref(make_params(params)), _ptr(rho), _ptr(kappa_P),
                              _ptr(kappa_F), _ptr(state), float(dt), int(nsteps),
                              ctypes.c_void_p(s.cuda_stream), ctypes.byref(cell))
    return int(st), int(cell.value)


def workspace_bytes(p: dict, adjoint_segment_len: int = 0) -> int:
    return int(lib.rhd_workspace_bytes(ctypes.byref(make_params(p)), int(adjoint_segment_len)))


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 tensor on the GPU")
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """A handle of the library bound to one parameter set, its scalar fields
    (rho, kappa_P, optional kappa_F; device float64 [nz, ny, nx]) and a
    workspace tensor, on the current torch stream of `device`."""

    def __init__(self, params: dict, rho: torch.Tensor, kappa_P: torch.Tensor,
                 kappa_F: Optional[torch.Tensor] = None, adjoint_segment_len: int = 0,
                 device: Optional[torch.device] = None):
        self.params = dict(params)
        self.rp = make_params(params)
        self.ndim = int(params["ndim"])
        self.nvar = 2 + 2 * self.ndim
        n = tuple(params["n"]) + (1,) * (3 - len(params["n"]))
        self.shape = (n[2], n[1], n[0])
        self.device = torch.device(device) if device is not None else rho.device
        self.rho, self.kappa_P, self.kappa_F = rho, kappa_P, kappa_F
        self.adj_len = int(adjoint_segment_len)
        nb = lib.rhd_workspace_bytes(ctypes.byref(self.rp), self.adj_len)
        if nb == 0:
            raise RHDError(RHD_EINVAL, -1, "invalid parameters")
        self.workspace = torch.empty(int(nb), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        st = lib.rhd_create(ctypes.byref(self.rp), _ptr(rho), _ptr(kappa_P), _ptr(kappa_F),
                            ctypes.c_void_p(self.workspace.data_ptr()), int(nb),
                            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != RHD_OK:
            raise RHDError(st, -1, "rhd_create failed")
        self._h = h

    # -- helpers --
    def _check(self, st: int, raise_on_error: bool = True) -> int:
        if st != RHD_OK and raise_on_error:
            cell = ctypes.c_int64(-1)
            buf = ctypes.create_string_buffer(256)
            lib.rhd_last_error(self._h, ctypes.byref(cell), buf, 256)
            raise RHDError(st, cell.value, buf.value.decode())
        return st

    def last_error(self):
        cell = ctypes.c_int64(-1)
        buf = ctypes.create_string_buffer(256)
        st = lib.rhd_last_error(self._h, ctypes.byref(cell), buf, 256)
        return st, cell.value, buf.value.decode()

    def _state(self, y: torch.Tensor):
        if tuple(y.shape) != (self.nvar,) + self.shape:
            raise ValueError(f"state shape {tuple(y.shape)} != {(self.nvar,) + self.shape}")
        return _ptr(y)

    # -- entry points --
    def step(self, y: torch.Tensor, dt: float, nsteps: int, raise_on_error: bool = True) -> int:
        return self._check(lib.rhd_step(self._h, self._state(y), float(dt), int(nsteps)),
                           raise_on_error)

    def step_timed(self, y: torch.Tensor, dt: float, nsteps: int):
        """rhd_step with the summed stage-1 / stage-2 kernel times (ms) measured
        by hipEvents on the handle's stream."""
        ms = (ctypes.c_double * 2)()
        self._check(lib.rhd_step_timed(self._h, self._state(y), float(dt), int(nsteps), ms))
        return float(ms[0]), float(ms[1])

    def stage1(self, y: torch.Tensor, yh: torch.Tensor, dt: float, raise_on_error=True) -> int:
        return self._check(lib.rhd_stage1(self._h, self._state(y), self._state(yh), float(dt)),
                           raise_on_error)

    def transport(self, y: torch.Tensor, s: torch.Tensor) -> int:
        return self._check(lib.rhd_transport(self._h, self._state(y), self._state(s)))

    def source(self, y: torch.Tensor, tau: float, raise_on_error=True) -> int:
        return self._check(lib.rhd_source(self._h, self._state(y), float(tau)), raise_on_error)

    def set_kappa_E(self, kappa_E: Optional[torch.Tensor]) -> int:
        """Energy-mean opacity field (None: kappa_E = kappa_P); kept referenced."""
        self.kappa_E = kappa_E
        return self._check(lib.rhd_set_energy_opacity(self._h, _ptr(kappa_E)))

    def set_radiation_source(self, j: Optional[torch.Tensor]) -> int:
        """Radiation injection rate per unit volume (None: no source); kept referenced."""
        self.j_source = j
        return self._check(lib.rhd_set_radiation_source(self._h, _ptr(j)))

    def hydro_step(self, y: torch.Tensor, dt: float, nsteps: int = 1,
                   raise_on_error: bool = True) -> int:
        """RK2-SSP hydro steps of the gas rows of y and of the bound density
        (self.rho, advanced in place)."""
        return self._check(lib.rhd_hydro_step(self._h, self._state(y), _ptr(self.rho), float(dt),
                                              int(nsteps)), raise_on_error)

    def rhd_step(self, y: torch.Tensor, dt: float, nsub: int, nsteps: int,
                 raise_on_error: bool = True) -> int:
        """Operator-split steps: one hydro step of dt, then nsub radiation steps
        of dt / nsub, nsteps times (self.rho advanced in place)."""
        return self._check(lib.rhd_rhd_step(self._h, self._state(y), _ptr(self.rho), float(dt),
                                            int(nsub), int(nsteps)), raise_on_error)

    def hydro_signal_speed(self, y: torch.Tensor) -> float:
        out = ctypes.c_double(0.0)
        self._check(lib.rhd_hydro_signal_speed(self._h, self._state(y), _ptr(self.rho),
                                               ctypes.byref(out)))
        return float(out.value)

    def conserved_totals(self, y: torch.Tensor):
        out = (ctypes.c_double * (1 + self.ndim))()
        self._check(lib.rhd_conserved_totals(self._h, self._state(y), out))
        return list(out)

    def step_adjoint(self, y0: torch.Tensor, dt: float, nsteps: int, lam: torch.Tensor,
                     g_kappa_P: torch.Tensor, g_kappa_F: Optional[torch.Tensor] = None) -> int:
        return self._check(lib.rhd_step_adjoint(self._h, self._state(y0), float(dt), int(nsteps),
                                                self._state(lam), _ptr(g_kappa_P),
                                                _ptr(g_kappa_F)))

    def close(self):
        if getattr(self, "_h", None):
            lib.rhd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
