"""Pins of the oracle's whole PD-ARS step (transport + source, Sec. 3.2).

Anchors: the closed-form spreading of a Gaussian under the diffusion equation
(the static-diffusion limit, eq. diffu and the diffusion equation of Sec. 5.4),
Fick's-law flux in the thick limit (eq. f1 / flux_nhalf), exact conservation of
E_gas + (c/chat) E and of rho v + F/(c chat), and the dual-number tangent
against central finite differences.
"""
import numpy as np
import pytest

from paper_2404_08247_amd import workloads as W


def _diffusion_pulse(n, tau_cell_at_128=10.0, sigma0=0.0625, closure="m1"):
    """Radiation-dominated 1-D periodic Gaussian pulse at rest. A very heavy gas
    with a negligible heat capacity (C_v / (4 a_r T^3) ~ 1e-7) keeps the gas
    inert, so E obeys dE/dt = D d2E/dx2 with D = chat / (3 chi)."""
    chat = 1.0
    p = W.base_params(1, (n,), chat, (0,), closure=closure)
    p["a_r"] = 1.0
    rho = 1.0e14
    p["kB_over_mu"] = 1.0e-21          # C_v = 1.5e-7 per unit volume
    cv = p["kB_over_mu"] / (p["gamma"] - 1)
    chi = tau_cell_at_128 * 128.0       # fixed physical opacity across resolutions
    x = W.cell_centres(n)
    Ebg, A = 1.0, 1.0
    # cell averages of the Gaussian (the second moment then carries no h^2/12 bias)
    from scipy.special import erf
    h = 1.0 / n
    s2 = np.sqrt(2.0) * sigma0
    avg = 0.5 * s2 * np.sqrt(np.pi) * (erf((x + h / 2 - 0.5) / s2) - erf((x - h / 2 - 0.5) / s2)) / h
    E = Ebg + A * avg
    T = (E / p["a_r"]) ** 0.25
    y = np.zeros((4, 1, 1, n))
    y[0] = E
    y[2] = rho * cv * T
    return p, y, np.full((1, 1, n), rho), np.full((1, 1, n), chi / rho), chi, x, Ebg


def _second_moment(x, E, Ebg):
    w = E - Ebg
    m0 = w.sum()
    xc = (x * w).sum() / m0
    return ((x - xc) ** 2 * w).sum() / m0


@pytest.mark.slow
def test_gaussian_spreads_as_the_diffusion_equation(orc):
    # sigma^2(t) = sigma0^2 + 2 D t; the relative error of the variance increment
    # must be small and must fall with resolution.
    errs = []
    for n in (64, 128):
        p, y, rho, kap, chi, x, Ebg = _diffusion_pulse(n)
        D = p["chat"] / (3.0 * chi)
        dt = 0.3 * p["dx"] / p["chat"]
        t_end = 2.0
        nsteps = int(round(t_end / dt))
        s0 = _second_moment(x, y[0, 0, 0], Ebg)
        yo, st, _ = orc.step(p, y, rho, kap, None, dt, nsteps)
        assert st == 0
        s1 = _second_moment(x, yo[0, 0, 0], Ebg)
        t = nsteps * dt
        # the flux starts at 0 and relaxes over 1/(chat chi): telegraph-equation
        # variance 2 D (t - t_r (1 - exp(-t/t_r))), t_r = 1/(chat chi)
        tr = 1.0 / (p["chat"] * chi)
        pred = 2.0 * D * (t - tr * (1.0 - np.exp(-t / tr)))
        errs.append(abs((s1 - s0) - pred) / pred)
        # total energy conserved (gas + radiation)
        tot0 = (y[2] + y[0]).sum()
        assert abs((yo[2] + yo[0]).sum() - tot0) <= 1e-13 * tot0
    assert errs[-1] < 0.02, errs
    assert errs[1] < errs[0], errs


def test_thick_limit_flux_is_ficks_law(orc):
    # after a few steps in an optically thick, smooth, static problem,
    # F = -(c / (3 chi)) dE/dx (eq. f1). Away from the pulse peak (where PPM clips
    # the extremum) the agreement is second order in dx; everywhere it converges.
    out = []
    for n in (128, 256):
        p, y, rho, kap, chi, x, Ebg = _diffusion_pulse(n, tau_cell_at_128=50.0, sigma0=0.08)
        dt = 0.3 * p["dx"] / p["chat"]
        yo, st, _ = orc.step(p, y, rho, kap, None, dt, 20 * n // 128)
        assert st == 0
        E = yo[0, 0, 0]
        dEdx = (np.roll(E, -1) - np.roll(E, 1)) / (2 * p["dx"])
        fick = -p["c"] * dEdx / (3.0 * chi)
        e = np.abs(yo[1, 0, 0] - fick) / np.abs(fick).max()
        away = np.abs(x - 0.5) > 0.05
        out.append((e[away].max(), e.max()))
    assert out[0][0] < 5e-3 and out[1][0] < 0.3 * out[0][0], out
    assert out[1][1] < 0.5 * out[0][1], out


@pytest.mark.parametrize("cfg", ["c2", "c3", "c4", "c5"])
def test_energy_and_momentum_conserved_to_roundoff(orc, cfg):
    w = {"c2": lambda: W.config2(n=(16, 12, 10), nsteps=3),
         "c3": lambda: W.config3(n=(24, 12, 10), nsteps=3, precision="fp64"),
         "c4": lambda: W.config4(n=(40, 24), nsteps=3),
         "c5": lambda: W.config5(n=(16, 12, 10), nsteps=3, precision="fp64")}[cfg]()
    p = w.params
    yo, st, _ = orc.step(p, w.y0, w.rho, w.kappa_P, None, w.dt, w.nsteps)
    assert st == 0
    nd = w.ndim
    k = p["c"] / p["chat"]
    e0 = w.y0[1 + nd] + k * w.y0[0]
    e1 = yo[1 + nd] + k * yo[0]
    N = w.ncells
    assert abs(e1.sum() - e0.sum()) <= 4e-16 * np.sqrt(N) * np.abs(e0).sum() * 10
    for d in range(nd):
        m0 = w.y0[2 + nd + d] + w.y0[1 + d] / (p["c"] * p["chat"])
        m1 = yo[2 + nd + d] + yo[1 + d] / (p["c"] * p["chat"])
        scale = (np.abs(w.y0[2 + nd + d]) + np.abs(w.y0[1 + d] / (p["c"] * p["chat"]))
                 + np.abs(yo[1 + d] / (p["c"] * p["chat"]))).sum()
        assert abs(m1.sum() - m0.sum()) <= 1e-14 * np.sqrt(N) * scale


def test_reports_nonphysical_state(orc):
    # gas whose kinetic energy exceeds its total energy: flagged as non-physical
    w = W.config4(n=(16, 12), nsteps=1)
    y = w.y0.copy()
    y[3, 0, 5, 7] = 0.5 * (y[4, 0, 5, 7] ** 2 + y[5, 0, 5, 7] ** 2) * 0.5
    yo, st, cell = orc.step(w.params, y, w.rho, w.kappa_P, None, w.dt, 1)
    assert st == 2 and cell == 5 * 16 + 7


def test_reports_newton_failure(orc):
    w = W.config2(n=(8, 6, 4), nsteps=1)
    p = dict(w.params, newton_maxit=1)
    yo, st, cell = orc.step(p, w.y0, w.rho, w.kappa_P, None, w.dt, 1)
    assert st == 1 and cell >= 0


def _tie_free(y0):
    """A smooth, irregular 1 % modulation of E and E_gas: removes the exact ties
    (flat backgrounds, mirror-symmetric cells) at which the PPM limiter has a kink,
    so that the step is differentiable in a neighbourhood of the state."""
    y = y0.copy()
    nz, ny, nx = y.shape[1:]
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    y[0] *= 1.0 + 0.01 * np.sin(0.7 * X + 0.3 * Y + 0.2 * Z + 0.1)
    return y


@pytest.mark.parametrize("cfg", ["c1", "c4", "c3"])
def test_dual_tangent_matches_central_differences(orc, cfg):
    # Smooth perturbation directions and h = 1e-6: the step has kinks (limiter
    # branches, the Newton and outer stopping rules) that a larger h, or a
    # cell-by-cell random direction, would straddle.
    if cfg == "c1":
        w = W.config1(n=24, nsteps=2)
    elif cfg == "c4":
        w = W.config4(n=(12, 10), nsteps=2)
    else:
        w = W.config3(n=(10, 8, 6), nsteps=2, precision="fp64")
    p = w.params
    y0 = _tie_free(w.y0)
    sh = y0[0].shape
    Z, Y, X = np.meshgrid(*[np.arange(m) for m in sh], indexing="ij")
    ty = np.zeros_like(y0)
    ty[0] = y0[0] * np.sin(0.9 * X + 0.5 * Y - 0.4 * Z + 0.3)
    ty[1 + w.ndim] = y0[1 + w.ndim] * np.cos(0.6 * X - 0.8 * Y + 0.5 * Z) * 1e-2
    tk = w.kappa_P * np.sin(0.4 * X + 1.1 * Y + 0.7 * Z)
    y, t, st, _ = orc.step_dual(p, y0, ty, w.rho, w.kappa_P, tk, None, None, w.dt, w.nsteps)
    assert st == 0
    h = 1e-6
    yp, _, _ = orc.step(p, y0 + h * ty, w.rho, w.kappa_P + h * tk, None, w.dt, w.nsteps)
    ym, _, _ = orc.step(p, y0 - h * ty, w.rho, w.kappa_P - h * tk, None, w.dt, w.nsteps)
    fd = (yp - ym) / (2 * h)
    for v in range(w.nvar):
        sc = np.abs(fd[v]).max()
        if sc == 0:
            continue
        # rounding of y over 2h (momentum is large next to its variation)
        noise = 1000 * 2.2e-16 * np.abs(y[v]).max() / h
        err = np.abs(t[v] - fd[v]).max()
        assert err < 1e-6 * sc + noise, (v, err / sc, noise / sc)
    # values equal the FP64 oracle's (the dual run may take extra Newton/outer
    # passes until its tangent settles, which moves values by the tolerances)
    y2, _, _ = orc.step(p, y0, w.rho, w.kappa_P, None, w.dt, w.nsteps)
    np.testing.assert_allclose(y, y2, rtol=1e-10, atol=1e-12 * np.abs(y2).max())


@pytest.mark.parametrize("n", [64, 128])
def test_rk2ssp_comparator_has_the_numerical_diffusion_mode(orc, n):
    # Sec. 4.2 (eq. ssp-f1, ssp-f2, EErk2): a scheme whose first stage carries the
    # transport only gains, in the thick limit, a numerical diffusion coefficient
    # on top of the physical D = chat/(3 chi). With the RK2 average of the two
    # stages it is chat^2 dt / 6 (the non-dimensional C^2 dt/3 times the 1/2 of
    # eq. EErk2); PD-ARS has none.
    out = {}
    for scheme in ("pdars", "rk2ssp"):
        p, y, rho, kap, chi, x, Ebg = _diffusion_pulse(n)
        p["scheme"] = scheme
        D = p["chat"] / (3.0 * chi)
        dt = 0.3 * p["dx"] / p["chat"]
        nsteps = int(round(1.0 / dt))
        s0 = _second_moment(x, y[0, 0, 0], Ebg)
        yo, st, _ = orc.step(p, y, rho, kap, None, dt, nsteps)
        assert st == 0
        t = nsteps * dt
        out[scheme] = (_second_moment(x, yo[0, 0, 0], Ebg) - s0) / (2.0 * t) / D
        num = p["chat"] ** 2 * dt / 6.0 / D
    assert abs(out["pdars"] - 1.0) < 0.03, out
    assert abs(out["rk2ssp"] - (1.0 + num)) < 0.03 * (1.0 + num), (out, num)


def test_rk2ssp_equals_pdars_without_coupling(orc):
    # with chi = 0 the source is the identity and both schemes are RK2-SSP
    p = W.base_params(1, (48,), 1.0, (0,))
    x = W.cell_centres(48)
    y = np.zeros((4, 1, 1, 48))
    y[0] = 1.0 + np.exp(-((x - 0.4) ** 2) / 0.01)
    y[1] = 0.3 * y[0]
    y[2] = 1.0
    zero = np.zeros((1, 1, 48))
    a, _, _ = orc.step(p, y, np.ones((1, 1, 48)), zero, None, 0.3 / 48, 20)
    b, _, _ = orc.step(dict(p, scheme="rk2ssp"), y, np.ones((1, 1, 48)), zero, None, 0.3 / 48, 20)
    assert np.array_equal(a, b)


# ------------------------------------------ Skinner-type eps (Sec. 4.2) --
def test_eps_correction_is_plain_hll_when_optically_thin(orc):
    # tau = hll_eps_cells dx chi <= 1 everywhere: eps = 1 and the fluxes are HLL's
    w = W.config4(n=(20, 16))
    p = dict(w.params, hll_eps_cells=1.0)
    kap = np.full_like(w.kappa_P, 0.9 / (w.params["dx"] * w.rho.max()))
    y = w.y0.copy()
    a = orc.transport(w.params, y)
    b = orc.transport(p, y, w.rho, kap)
    assert np.array_equal(a, b)


def test_eps_correction_scales_only_the_energy_dissipation(orc):
    # With F = 0 the energy flux of HLL is pure dissipation, -S (E+ - E-)/2, so a
    # uniform eps = 1/tau scales s_E by 1/tau exactly and leaves s_F unchanged.
    w = W.config2(n=(12, 10, 8))
    y = w.y0.copy()
    y[1:4] = 0.0
    tau = 7.5
    p = dict(w.params, hll_eps_cells=2.0)
    kap = np.full_like(w.kappa_P, tau / (2.0 * w.params["dx"] * w.rho))
    a = orc.transport(w.params, y)
    b = orc.transport(p, y, w.rho, kap)
    np.testing.assert_allclose(b[0], a[0] / tau, rtol=1e-13, atol=1e-15 * np.abs(a[0]).max())
    assert np.array_equal(a[1:], b[1:])
    assert orc.face_eps(p, 3.0 / p["dx"], 3.0 / p["dx"]) == 1.0 / 6.0
    assert orc.face_eps(w.params, 1e9, 1e9) == 1.0   # correction off
    # With F != 0 the F rows still carry their full dissipation (bitwise the plain
    # HLL rows), and the energy row is affine in eps: s_E(eps) - s_E(1) =
    # (eps - 1) times the energy dissipation, the same for two values of eps.
    rng = np.random.default_rng(5)
    y[1:4] = 0.3 * rng.uniform(-1.0, 1.0, y[1:4].shape) * w.params["c"] * y[0]
    a = orc.transport(w.params, y)
    diss = []
    for t in (7.5, 30.0):
        kap_t = np.full_like(w.kappa_P, t / (2.0 * w.params["dx"] * w.rho))
        b = orc.transport(p, y, w.rho, kap_t)
        assert np.array_equal(a[1:], b[1:])
        diss.append((b[0] - a[0]) / (1.0 / t - 1.0))
    np.testing.assert_allclose(diss[1], diss[0], rtol=0, atol=1e-12 * np.abs(diss[0]).max())


def test_eps_correction_targets_the_hll_diffusion_not_the_rk2ssp_mode(orc):
    # Thick diffusion pulse at n = 64 (tau_cell = 20): the HLL dissipation adds a
    # small numerical diffusion to PD-ARS (about 2 %), which the eps correction
    # removes; RK2-SSP keeps its C^2 dt/3 mode with or without it (the mode comes
    # from the transport-only first stage, eq. ssp-f1, not from the Riemann solver).
    res = {}
    for scheme in ("pdars", "rk2ssp"):
        for eps in (0.0, 1.0):
            p, y, rho, kap, chi, x, Ebg = _diffusion_pulse(64)
            p["scheme"] = scheme
            p["hll_eps_cells"] = eps
            D = p["chat"] / (3.0 * chi)
            dt = 0.3 * p["dx"] / p["chat"]
            nsteps = int(round(1.0 / dt))
            s0 = _second_moment(x, y[0, 0, 0], Ebg)
            yo, st, _ = orc.step(p, y, rho, kap, None, dt, nsteps)
            assert st == 0
            res[(scheme, eps)] = (_second_moment(x, yo[0, 0, 0], Ebg) - s0) / (2.0 * nsteps * dt) / D
            num = p["chat"] ** 2 * dt / 6.0 / D
    assert abs(res[("pdars", 0.0)] - 1.0) > 0.015, res
    assert abs(res[("pdars", 1.0)] - 1.0) < 0.006, res
    for eps in (0.0, 1.0):
        assert abs(res[("rk2ssp", eps)] - (1.0 + num)) < 0.03 * (1.0 + num), res
