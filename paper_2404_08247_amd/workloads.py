"""Seeded synthetic inputs for the radiation step (shared by the HIP path's tests
and benchmark and by the oracle's tests).

This module builds initial states, densities and opacity fields only. It holds
none of the method's arithmetic: no transport, no closure, no source update.

Units (code units, the same for every workload): c = 1, rho = 1, gamma = 5/3,
a_r = 1e-8, k_B/(mu m_H) = 1e-5 (so c_v = 1.5e-5 per unit mass), domain [0, 1]^d,
dx = 1/n, dt = 0.3 dx / chat. With these values the radiation energy density
stays far below rho c^2 and the sound speed far below c, so the v/c expansion of
the four-force (Sec. 2.1) holds and the gas is not driven relativistic by the
radiation force over the runs (no hydrodynamic step balances that force).

State layout: numpy float64 array of shape (nvar, nz, ny, nx), x fastest,
variables (E, F_1..F_d, E_gas, (rho v)_1..(rho v)_d), nvar = 2 + 2 d.
Unused axes have extent 1.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

SEED_BASE = 20240412

UNITS = dict(c=1.0, gamma=5.0 / 3.0, a_r=1.0e-8, kB_over_mu=1.0e-5)
CFL = 0.3


@dataclasses.dataclass
class Workload:
    name: str
    ndim: int
    n: tuple            # (nx, ny, nz)
    params: dict        # physical and numerical parameters of the step
    y0: np.ndarray      # (nvar, nz, ny, nx) float64
    rho: np.ndarray     # (nz, ny, nx)
    kappa_P: np.ndarray
    kappa_F: Optional[np.ndarray]   # None: flux mean equals Planck mean
    dt: float
    nsteps: int
    precision: str = "fp64"         # "fp64" | "mixed"
    objective_mask: Optional[np.ndarray] = None   # (nz, ny, nx) bool, J = sum E over mask
    ckpt_every: int = 0

    @property
    def ncells(self) -> int:
        return int(np.prod(self.n))

    @property
    def nvar(self) -> int:
        return 2 + 2 * self.ndim


def base_params(ndim, n, chat, bc, closure="m1", v_order=2, precision="fp64", **over):
    nn = tuple(int(x) for x in n) + (1,) * (3 - len(n))
    dx = 1.0 / nn[0]
    p = dict(ndim=ndim, n=nn, dx=dx, c=UNITS["c"], chat=float(chat), gamma=UNITS["gamma"],
             a_r=UNITS["a_r"], kB_over_mu=UNITS["kB_over_mu"],
             bc=tuple(bc) + (0,) * (3 - len(bc)), closure=closure, v_order=v_order,
             precision=precision, newton_rtol=1e-13, outer_rtol=1e-13, newton_maxit=50,
             outer_maxit=10)
    p.update(over)
    return p


def cell_centres(n: int) -> np.ndarray:
    return (np.arange(n) + 0.5) / n


def grf(shape: Sequence[int], ell: float, rng: np.random.Generator) -> np.ndarray:
    """Gaussian random field: white N(0,1) noise convolved (periodically, by FFT)
    with exp(-r^2 / (2 ell^2)) (r in cells), then shifted and scaled to zero mean
    and unit standard deviation."""
    shape = tuple(shape)
    w = rng.standard_normal(shape)
    axes = []
    for m in shape:
        d = np.arange(m)
        d = np.minimum(d, m - d).astype(np.float64)
        axes.append(d)
    r2 = np.zeros(shape)
    for ax, d in enumerate(axes):
        sh = [1] * len(shape)
        sh[ax] = shape[ax]
        r2 = r2 + (d ** 2).reshape(sh)
    ker = np.exp(-r2 / (2.0 * ell * ell))
    axes = tuple(range(len(shape)))
    f = np.fft.irfftn(np.fft.rfftn(w) * np.fft.rfftn(ker), s=shape, axes=axes)
    f = f - f.mean()
    sd = f.std()
    return f / sd if sd > 0 else f


def power_law_velocity(shape: Sequence[int], slope: float, rms: float,
                       rng: np.random.Generator) -> np.ndarray:
    """Random-phase vector field with |v_hat(k)| proportional to |k|^slope per
    component (k = 0 removed), scaled so that sqrt(<|v|^2>) = rms.
    Returns (3, *shape)."""
    shape = tuple(shape)
    kk = [np.fft.fftfreq(m) * m for m in shape[:-1]] + [np.fft.rfftfreq(shape[-1]) * shape[-1]]
    grids = np.meshgrid(*kk, indexing="ij")
    kmag = np.sqrt(sum(g * g for g in grids))
    amp = np.zeros_like(kmag)
    nz = kmag > 0
    amp[nz] = kmag[nz] ** slope
    out = np.empty((3,) + shape)
    for c in range(3):
        phase = rng.uniform(0.0, 2.0 * np.pi, size=kmag.shape)
        spec = amp * np.exp(1j * phase)
        out[c] = np.fft.irfftn(spec, s=shape, axes=tuple(range(len(shape))))
    vrms = np.sqrt(np.mean(np.sum(out ** 2, axis=0)))
    return out * (rms / vrms)


def _assemble(ndim, n, T_gas, E, F, v, rho, params):
    """State from temperatures, radiation moments and velocity (initial data).
    E_gas = C_v T + |rho v|^2 / (2 rho)."""
    nx, ny, nz = n
    nvar = 2 + 2 * ndim
    y = np.zeros((nvar, nz, ny, nx))
    cv = params["kB_over_mu"] / (params["gamma"] - 1.0)
    y[0] = E
    for d in range(ndim):
        y[1 + d] = F[d]
    mom = [rho * v[d] for d in range(ndim)]
    ke = sum(m * m for m in mom) / (2.0 * rho) if ndim > 0 else 0.0
    y[1 + ndim] = rho * cv * T_gas + ke
    for d in range(ndim):
        y[2 + ndim + d] = mom[d]
    return y


def _radial_r2_cells(n, ndim):
    nx, ny, nz = n
    ax = [np.arange(m) + 0.5 - m / 2.0 for m in (nz, ny, nx)]
    Z, Y, X = np.meshgrid(*ax, indexing="ij")
    r2 = X ** 2
    if ndim >= 2:
        r2 = r2 + Y ** 2
    if ndim >= 3:
        r2 = r2 + Z ** 2
    return r2


def config1(n: int = 256, nsteps: int = 1000, bc=(1,), **over) -> Workload:
    """1-D, reflecting walls, FP64: optically thick (tau_cell = 10) Gaussian
    radiation pulse T = 1 + 10 exp(-(x - 1/2)^2 / 0.05^2), gas in equilibrium,
    F = 0, v = 0, chat = c."""
    chat = 1.0
    p = base_params(1, (n,), chat, bc, **over)
    dx = p["dx"]
    x = cell_centres(n)
    T = 1.0 + 10.0 * np.exp(-((x - 0.5) ** 2) / 0.05 ** 2)
    T = T.reshape(1, 1, n)
    rho = np.ones((1, 1, n))
    kappa = np.full((1, 1, n), 10.0 / (1.0 * dx))
    E = p["a_r"] * T ** 4
    y = _assemble(1, p["n"], T, E, [np.zeros_like(T)], [np.zeros_like(T)], rho, p)
    return Workload("c1_1d_256_reflect_fp64", 1, p["n"], p, y, rho, kappa, None,
                    CFL * dx / chat, nsteps)


def config2(n: Sequence[int] = (128, 128, 128), nsteps: int = 200, precision="fp64",
            bc=(0, 0, 0), **over) -> Workload:
    """3-D static mixed-regime grid, periodic: log10 tau_cell = clip(N(0,1), -3, 3)
    i.i.d.; T = 1 + 0.1 GRF(8 cells); T_rad = T (1 + U(-0.2, 0.2)) i.i.d.;
    E = a_r T_rad^4; F = 0; v = 0; chat = c/100."""
    rng = np.random.default_rng(SEED_BASE + 2)
    chat = 0.01
    p = base_params(3, n, chat, bc, precision=precision, **over)
    nx, ny, nz = p["n"]
    dx = p["dx"]
    shape = (nz, ny, nx)
    tau = 10.0 ** np.clip(rng.standard_normal(shape), -3.0, 3.0)
    T = 1.0 + 0.1 * grf(shape, 8.0, rng)
    Trad = T * (1.0 + rng.uniform(-0.2, 0.2, size=shape))
    rho = np.ones(shape)
    kappa = tau / (rho * dx)
    zero = np.zeros(shape)
    y = _assemble(3, p["n"], T, p["a_r"] * Trad ** 4, [zero] * 3, [zero] * 3, rho, p)
    return Workload(f"c2_3d_{nx}x{ny}x{nz}_mixed_regime_{precision}", 3, p["n"], p, y, rho,
                    kappa, None, CFL * dx / chat, nsteps, precision=precision)


def config3(n: Sequence[int] = (256, 256, 256), nsteps: int = 300, precision="mixed",
            sigma_cells: Optional[float] = None, bc=(0, 0, 0), **over) -> Workload:
    """3-D dynamic diffusion, periodic: uniform v = 0.01 c along x; 8 x-slabs, each
    slab's tau_cell drawn from {0.1, 10, 1000}; T = 1 + exp(-r^2 / (2 sigma^2)),
    sigma = 16 cells (scaled with nx/256 on smaller grids), centred; E = a_r T^4;
    F = (4/3) v E (comoving equilibrium to O(v/c)); chat = c/50."""
    rng = np.random.default_rng(SEED_BASE + 3)
    chat = 0.02
    p = base_params(3, n, chat, bc, precision=precision, **over)
    nx, ny, nz = p["n"]
    dx = p["dx"]
    shape = (nz, ny, nx)
    choices = np.array([0.1, 10.0, 1000.0])
    slab_tau = choices[rng.integers(0, 3, size=8)]
    slab = np.minimum((np.arange(nx) * 8) // nx, 7)
    tau = np.broadcast_to(slab_tau[slab].reshape(1, 1, nx), shape).copy()
    if sigma_cells is None:
        sigma_cells = max(2.0, 16.0 * nx / 256.0)
    T = 1.0 + np.exp(-_radial_r2_cells(p["n"], 3) / (2.0 * sigma_cells ** 2))
    rho = np.ones(shape)
    kappa = tau / (rho * dx)
    vx = 0.01 * p["c"]
    E = p["a_r"] * T ** 4
    zero = np.zeros(shape)
    F = [(4.0 / 3.0) * vx * E, zero, zero]
    v = [np.full(shape, vx), zero, zero]
    y = _assemble(3, p["n"], T, E, F, v, rho, p)
    return Workload(f"c3_3d_{nx}x{ny}x{nz}_dynamic_diffusion_{precision}", 3, p["n"], p, y,
                    rho, kappa, None, CFL * dx / chat, nsteps, precision=precision)


def central_patch(n: Sequence[int], ndim: int, width: int) -> np.ndarray:
    nx, ny, nz = n
    m = np.zeros((nz, ny, nx), dtype=bool)
    sl = []
    for ax, size in enumerate((nz, ny, nx)):
        if (2 - ax) < ndim:
            lo = size // 2 - width // 2
            sl.append(slice(lo, lo + width))
        else:
            sl.append(slice(0, size))
    m[tuple(sl)] = True
    return m


def config4(n: Sequence[int] = (512, 512), nsteps: int = 200, ckpt_every: int = 20,
            bc=(0, 0), **over) -> Workload:
    """2-D adjoint run, FP64, periodic: log10 tau_cell = clip(N(0, 2/3), -2, 2)
    i.i.d.; v per component = GRF(8), scaled so max |v| = 0.005 c;
    T = 1 + exp(-r^2 / (2 (32 nx/512)^2)) centred; E = a_r T^4; F = 0; chat = c.
    Objective J = sum of E over the central (nx/8) x (ny/8) patch."""
    rng = np.random.default_rng(SEED_BASE + 4)
    chat = 1.0
    p = base_params(2, n, chat, bc, **over)
    nx, ny, nz = p["n"]
    dx = p["dx"]
    shape = (1, ny, nx)
    tau = 10.0 ** np.clip(rng.normal(0.0, 2.0 / 3.0, size=shape), -2.0, 2.0)
    vx = grf(shape, 8.0, rng)
    vy = grf(shape, 8.0, rng)
    vmag = np.sqrt(vx ** 2 + vy ** 2).max()
    vx, vy = vx * (0.005 / vmag), vy * (0.005 / vmag)
    sig = 32.0 * nx / 512.0
    T = 1.0 + np.exp(-_radial_r2_cells(p["n"], 2) / (2.0 * sig ** 2))
    rho = np.ones(shape)
    kappa = tau / (rho * dx)
    zero = np.zeros(shape)
    y = _assemble(2, p["n"], T, p["a_r"] * T ** 4, [zero, zero], [vx, vy], rho, p)
    return Workload(f"c4_2d_{nx}x{ny}_adjoint_fp64", 2, p["n"], p, y, rho, kappa, None,
                    CFL * dx / chat, nsteps, objective_mask=central_patch(p["n"], 2, max(2, nx // 8)),
                    ckpt_every=ckpt_every)


def config5(n: Sequence[int] = (320, 320, 320), nsteps: int = 100, ckpt_every: int = 10,
            precision="mixed", bc=(0, 0, 0), **over) -> Workload:
    """3-D forward + adjoint, periodic: tau_cell as config 2; velocity random-phase
    field with |v_hat(k)| ~ |k|^-2, rms |v| = 0.01 c; T = exp(0.1 GRF(8));
    E = a_r T^4; F = 0; chat = c/100. J = sum of E over the central (n/5)^3 block
    (64^3 at 320^3)."""
    rng = np.random.default_rng(SEED_BASE + 5)
    chat = 0.01
    p = base_params(3, n, chat, bc, precision=precision, **over)
    nx, ny, nz = p["n"]
    dx = p["dx"]
    shape = (nz, ny, nx)
    tau = 10.0 ** np.clip(rng.standard_normal(shape), -3.0, 3.0)
    v = power_law_velocity(shape, -2.0, 0.01 * p["c"], rng)
    T = np.exp(0.1 * grf(shape, 8.0, rng))
    rho = np.ones(shape)
    kappa = tau / (rho * dx)
    zero = np.zeros(shape)
    y = _assemble(3, p["n"], T, p["a_r"] * T ** 4, [zero] * 3, [v[0], v[1], v[2]], rho, p)
    return Workload(f"c5_3d_{nx}x{ny}x{nz}_fwd_adj_{precision}", 3, p["n"], p, y, rho, kappa,
                    None, CFL * dx / chat, nsteps, precision=precision,
                    objective_mask=central_patch(p["n"], 3, max(2, nx // 5)), ckpt_every=ckpt_every)


# The asymptotic Marshak wave (Sec. 5.2), in cgs with temperatures in keV.
MARSHAK = dict(a_r=7.5657e-15 * 1.160452e7 ** 4,   # erg cm^-3 keV^-4
               c=2.99792458e10, cv=3e15,            # erg cm^-3 keV^-1 (rho = 1)
               kappa=300.0, T_hot=1.0, T_cold=1e-3, length=0.66, t_end=2e-8)


def marshak(n: int = 60, cfl: float = 10.0, scheme: str = "pdars", t_end: Optional[float] = None,
            **over) -> Workload:
    """1-D Marshak wave: a cold (T = 1e-3 keV) static medium of density 1 with
    chi = 300 / T^3 cm^-1 (kappa = 300 scaled by T^-3 in the source) and
    C_v = 3e15 erg cm^-3 keV^-1, driven through x = 0 by radiation at 1 keV
    (inflow boundary; the far end reflects); Eddington closure, order-1 source,
    chat = c. dt = cfl dx / c, rounded so that an integer number of steps ends at
    t_end (default 2e-8 s)."""
    m = MARSHAK
    t_end = m["t_end"] if t_end is None else t_end
    dx = m["length"] / n
    p = dict(ndim=1, n=(n, 1, 1), dx=dx, c=m["c"], chat=m["c"], gamma=5.0 / 3.0, a_r=m["a_r"],
             kB_over_mu=m["cv"] * (2.0 / 3.0), bc=(2, 0, 0), closure="eddington", v_order=1,
             precision="fp64", scheme=scheme, newton_rtol=1e-13, outer_rtol=1e-13,
             newton_maxit=400, outer_maxit=10, kappa_T_power=-3.0,
             inflow_E=m["a_r"] * m["T_hot"] ** 4, inflow_F=0.0)
    p.update(over)
    shape = (1, 1, n)
    y = np.zeros((4,) + shape)
    y[0] = m["a_r"] * m["T_cold"] ** 4
    y[2] = m["cv"] * m["T_cold"]
    nsteps = max(1, int(round(t_end / (cfl * dx / m["c"]))))
    return Workload(f"marshak_1d_{n}_cfl{cfl:g}_{scheme}", 1, p["n"], p, y, np.ones(shape),
                    np.full(shape, m["kappa"]), None, t_end / nsteps, nsteps)


# The advecting radiation pulse (Sec. 5.4 static and Sec. 5.5 dynamic diffusion
# limit), in cgs.
PULSE = dict(a_r=7.5657e-15, c=2.99792458e10, k_B=1.380649e-16, mu=3.9e-24, T0=1e7, T1=2e7,
             width=24.0, rho0=1.2, half_length=512.0, t_end=4.8e-5)


@dataclasses.dataclass
class CoupledWorkload:
    """A radiation-hydrodynamics run: operator-split steps of dt (one hydro step,
    then nsub radiation steps of dt / nsub)."""
    name: str
    w: Workload          # state, density, opacities and radiation parameters
    dt: float            # hydro step
    nsub: int            # radiation steps per hydro step
    nsteps: int          # hydro steps to t_end
    shift_cells: int     # v0 t_end / dx (the advected run's displacement)


def advecting_pulse(regime: str = "static", advected: bool = True, hydro_cfl: float = 0.3,
                    rad_cfl: float = 4.0, t_end: Optional[float] = None, **over) -> CoupledWorkload:
    """1-D periodic radiation pulse on (-512, 512) cm in pressure balance:
    T = T0 + (T1 - T0) exp(-x^2 / (2 w^2)), rho = rho0 T0/T + (a_r mu / (3 k_B))
    (T0^4/T - T^3), T_rad = T_gas, mu = 3.9e-24 g, Eddington closure, chat = c,
    kappa_P = kappa_E = kappa_F. "static": 512 cells, kappa = 100 cm^2/g,
    v0 = 1e6 cm/s; "dynamic": 1024 cells, kappa = 500, v0 = 3e7. advected: the gas
    moves at v0 (with the comoving-equilibrium flux F = 4/3 v0 E), else it starts at
    rest. dt = hydro_cfl dx / max(|v| + c_s) of the initial state, rounded so that an
    integer number of steps ends at t_end (default 4.8e-5 s); the radiation is
    subcycled with nsub = ceil(dt c / (rad_cfl dx)) steps per hydro step."""
    m = PULSE
    n, kappa, v0 = (512, 100.0, 1e6) if regime == "static" else (1024, 500.0, 3e7)
    t_end = m["t_end"] if t_end is None else t_end
    L = 2.0 * m["half_length"]
    dx = L / n
    x = -m["half_length"] + (np.arange(n) + 0.5) * dx
    T = m["T0"] + (m["T1"] - m["T0"]) * np.exp(-x ** 2 / (2.0 * m["width"] ** 2))
    ar, kB, mu = m["a_r"], m["k_B"], m["mu"]
    rho = m["rho0"] * m["T0"] / T + ar * mu / (3.0 * kB) * (m["T0"] ** 4 / T - T ** 3)
    gamma = 5.0 / 3.0
    p = dict(ndim=1, n=(n, 1, 1), dx=dx, c=m["c"], chat=m["c"], gamma=gamma, a_r=ar,
             kB_over_mu=kB / mu, bc=(0, 0, 0), closure="eddington", v_order=2, precision="fp64",
             newton_rtol=1e-13, outer_rtol=1e-13, newton_maxit=50, outer_maxit=10)
    p.update(over)
    v = v0 if advected else 0.0
    cv = kB / mu / (gamma - 1.0)
    shape = (1, 1, n)
    E = ar * T ** 4
    y = np.zeros((4,) + shape)
    y[0] = E.reshape(shape)
    y[1] = (4.0 / 3.0 * v * E).reshape(shape)
    y[2] = (rho * cv * T + 0.5 * rho * v * v).reshape(shape)
    y[3] = (rho * v).reshape(shape)
    cs = np.sqrt(gamma * kB * T / mu)
    dt_max = hydro_cfl * dx / (np.abs(v) + cs).max()
    nsteps = int(np.ceil(t_end / dt_max))
    dt = t_end / nsteps
    nsub = int(np.ceil(dt * m["c"] / (rad_cfl * dx)))
    name = f"pulse_{regime}_{'advected' if advected else 'rest'}_{n}"
    w = Workload(name, 1, p["n"], p, y, rho.reshape(shape).copy(), np.full(shape, kappa), None,
                 dt / nsub, nsub * nsteps)
    return CoupledWorkload(name, w, dt, nsub, nsteps, int(round(v * t_end / dx)))


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}
