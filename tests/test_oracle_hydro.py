"""Oracle pins for the hydrodynamics half of the operator split (Sec. 3.1): the
RK2-SSP step of the Euler equations (PPM + HLLC), held against

- the exact solution of the Riemann problem (Sod's shock tube), from an exact
  Riemann solver written here (Toro, "Riemann Solvers and Numerical Methods for
  Fluid Dynamics", ch. 4), independently of the oracle;
- exact translation of a smooth density wave in a uniform flow (second-order
  convergence);
- conservation of mass, momentum and energy on periodic grids;
- a stationary contact, which HLLC keeps exactly;
- the same 1-D problem along x, y and z, and a reflecting wall against the
  mirror-symmetric periodic problem.
"""
import numpy as np
import pytest


def _params(nd, n, dx, gamma=1.4, bc=None):
    n = tuple(n) + (1,) * (3 - len(n))
    return dict(ndim=nd, n=n, dx=dx, c=1.0, chat=1.0, gamma=gamma, a_r=1.0, kB_over_mu=1.0,
                bc=tuple(bc) if bc is not None else (0, 0, 0), closure="eddington")


def _state(nd, rho, v, p, gamma):
    """y (E = F = 0) and rho from primitive fields of shape (nz, ny, nx)."""
    y = np.zeros((2 + 2 * nd,) + rho.shape)
    ke = 0.5 * rho * sum(vk ** 2 for vk in v)
    y[1 + nd] = p / (gamma - 1.0) + ke
    for k in range(nd):
        y[2 + nd + k] = rho * v[k]
    return y, rho.copy()


def _prim(nd, y, rho, gamma):
    v = [y[2 + nd + k] / rho for k in range(nd)]
    p = (gamma - 1.0) * (y[1 + nd] - 0.5 * rho * sum(vk ** 2 for vk in v))
    return v, p


# ------------------------------------------------------ exact Riemann solver --
def exact_riemann(WL, WR, gamma, xi):
    """Exact solution (rho, u, p) of the 1-D Riemann problem at x/t = xi."""
    rL, uL, pL = WL
    rR, uR, pR = WR
    aL, aR = np.sqrt(gamma * pL / rL), np.sqrt(gamma * pR / rR)
    g1 = (gamma - 1) / (2 * gamma)
    AL, AR = 2 / ((gamma + 1) * rL), 2 / ((gamma + 1) * rR)
    BL, BR = (gamma - 1) / (gamma + 1) * pL, (gamma - 1) / (gamma + 1) * pR

    def fK(p, pK, rK, aK, AK, BK):
        if p > pK:   # shock
            f = (p - pK) * np.sqrt(AK / (p + BK))
            df = np.sqrt(AK / (BK + p)) * (1 - (p - pK) / (2 * (BK + p)))
        else:        # rarefaction
            f = 2 * aK / (gamma - 1) * ((p / pK) ** g1 - 1)
            df = 1 / (rK * aK) * (p / pK) ** (-(gamma + 1) / (2 * gamma))
        return f, df

    p = max(1e-8, 0.5 * (pL + pR))
    for _ in range(100):
        f1, d1 = fK(p, pL, rL, aL, AL, BL)
        f2, d2 = fK(p, pR, rR, aR, AR, BR)
        pn = max(1e-12, p - (f1 + f2 + uR - uL) / (d1 + d2))
        if abs(pn - p) < 1e-15 * p:
            p = pn
            break
        p = pn
    ps = p
    us = 0.5 * (uL + uR) + 0.5 * (fK(ps, pR, rR, aR, AR, BR)[0] - fK(ps, pL, rL, aL, AL, BL)[0])
    out = np.zeros((3,) + np.shape(xi))
    for i, s in np.ndenumerate(np.asarray(xi)):
        if s <= us:   # left of the contact
            if ps > pL:
                SL = uL - aL * np.sqrt((gamma + 1) / (2 * gamma) * ps / pL + g1)
                w = (rL * ((ps / pL + (gamma - 1) / (gamma + 1)) / ((gamma - 1) / (gamma + 1) * ps / pL + 1)), us, ps) if s >= SL else (rL, uL, pL)
            else:
                SHL, STL = uL - aL, us - aL * (ps / pL) ** g1
                if s <= SHL:
                    w = (rL, uL, pL)
                elif s >= STL:
                    w = (rL * (ps / pL) ** (1 / gamma), us, ps)
                else:
                    fac = 2 / (gamma + 1) + (gamma - 1) / ((gamma + 1) * aL) * (uL - s)
                    w = (rL * fac ** (2 / (gamma - 1)), 2 / (gamma + 1) * (aL + (gamma - 1) / 2 * uL + s),
                         pL * fac ** (2 * gamma / (gamma - 1)))
        else:
            if ps > pR:
                SR = uR + aR * np.sqrt((gamma + 1) / (2 * gamma) * ps / pR + g1)
                w = (rR * ((ps / pR + (gamma - 1) / (gamma + 1)) / ((gamma - 1) / (gamma + 1) * ps / pR + 1)), us, ps) if s <= SR else (rR, uR, pR)
            else:
                SHR, STR = uR + aR, us + aR * (ps / pR) ** g1
                if s >= SHR:
                    w = (rR, uR, pR)
                elif s <= STR:
                    w = (rR * (ps / pR) ** (1 / gamma), us, ps)
                else:
                    fac = 2 / (gamma + 1) - (gamma - 1) / ((gamma + 1) * aR) * (uR - s)
                    w = (rR * fac ** (2 / (gamma - 1)), 2 / (gamma + 1) * (-aR + (gamma - 1) / 2 * uR + s),
                         pR * fac ** (2 * gamma / (gamma - 1)))
        out[(slice(None),) + i] = w
    return out, ps, us


SOD_L, SOD_R = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)


def test_exact_riemann_solver_reproduces_sod_star_state():
    # the textbook star state of Sod's problem (gamma = 1.4): p* = 0.30313, u* = 0.92745
    _, ps, us = exact_riemann(SOD_L, SOD_R, 1.4, np.array([0.0]))
    assert abs(ps - 0.30313) < 1e-5 and abs(us - 0.92745) < 1e-5


def _sod(orc, n, axis=0, nd=1, t_end=0.2, cfl=0.4):
    gamma = 1.4
    shape = [1, 1, 1]
    shape[2 - axis] = n
    nn = [1] * nd
    nn[axis] = n
    dx = 1.0 / n
    x = ((np.arange(n) + 0.5) * dx).reshape(shape)
    left = x < 0.5
    rho = np.where(left, SOD_L[0], SOD_R[0]) * np.ones(shape)
    pr = np.where(left, SOD_L[2], SOD_R[2]) * np.ones(shape)
    v = [np.zeros(shape) for _ in range(nd)]
    y, rho = _state(nd, rho, v, pr, gamma)
    bc = [0] * nd
    bc[axis] = 1
    p = _params(nd, nn, dx, gamma, bc=bc)
    nsteps = int(np.ceil(t_end / (cfl * dx / 2.0)))
    y, rho, st, _ = orc.hydro_step(p, y, rho, t_end / nsteps, nsteps)
    assert st == 0
    return x.ravel(), y, rho


@pytest.mark.parametrize("n", [200, 400])
def test_sod_shock_tube_against_exact_solution(orc, n):
    x, y, rho = _sod(orc, n)
    v, pr = _prim(1, y, rho, 1.4)
    ex, ps, us = exact_riemann(SOD_L, SOD_R, 1.4, (x - 0.5) / 0.2)
    l1 = [np.abs(a.ravel() - b).mean() for a, b in ((rho, ex[0]), (v[0], ex[1]), (pr, ex[2]))]
    assert max(l1) < (0.005 if n == 200 else 0.0025), l1
    # the star plateau between the rarefaction tail and the shock, away from both
    plateau = (x > 0.5 + 0.2 * 0.2) & (x < 0.5 + 0.2 * 1.6)
    assert abs(pr.ravel()[plateau].mean() - ps) < 2e-3 * ps
    assert abs(v[0].ravel()[plateau].mean() - us) < 2e-3 * us


def test_sod_error_falls_under_refinement(orc):
    errs = []
    for n in (100, 200, 400):
        x, y, rho = _sod(orc, n)
        ex, _, _ = exact_riemann(SOD_L, SOD_R, 1.4, (x - 0.5) / 0.2)
        errs.append(np.abs(rho.ravel() - ex[0]).mean())
    assert errs[1] < 0.75 * errs[0] and errs[2] < 0.75 * errs[1], errs


@pytest.mark.parametrize("axis,nd", [(1, 2), (2, 3)])
def test_sod_along_other_axes_matches_x(orc, axis, nd):
    x, y1, r1 = _sod(orc, 120)
    _, y2, r2 = _sod(orc, 120, axis=axis, nd=nd)
    np.testing.assert_allclose(r2.ravel(), r1.ravel(), rtol=1e-13, atol=0)
    np.testing.assert_allclose(y2[1 + nd].ravel(), y1[2].ravel(), rtol=1e-13, atol=0)
    np.testing.assert_allclose(y2[2 + nd + axis].ravel(), y1[3].ravel(), rtol=1e-12, atol=1e-14)
    for k in range(nd):
        if k != axis:
            assert np.all(y2[2 + nd + k] == 0.0)


def _advection(orc, n, periods=1.0):
    gamma = 1.4
    dx = 1.0 / n
    x = (np.arange(n) + 0.5) * dx
    shape = (1, 1, n)
    rho0 = (1.0 + 0.2 * np.sin(2 * np.pi * x)).reshape(shape)
    y, rho = _state(1, rho0, [np.ones(shape)], np.ones(shape), gamma)
    p = _params(1, (n,), dx, gamma)
    cfl = 0.4
    amax = 1.0 + np.sqrt(gamma / 0.8)
    nsteps = int(np.ceil(periods / (cfl * dx / amax)))
    y, rho, st, _ = orc.hydro_step(p, y, rho, periods / nsteps, nsteps)
    assert st == 0
    return np.abs(rho - rho0).mean()


def test_smooth_advection_converges_at_second_order(orc):
    e1, e2 = _advection(orc, 32), _advection(orc, 64)
    assert e2 < 1.5e-3
    assert e1 / e2 > 3.0, (e1, e2)


def test_stationary_contact_is_kept_exactly(orc):
    n = 64
    shape = (1, 1, n)
    rho0 = np.where(np.arange(n) < n // 2, 1.0, 0.1).reshape(shape) * np.ones(shape)
    y, rho = _state(1, rho0, [np.zeros(shape)], np.ones(shape), 1.4)
    y2, r2, st, _ = orc.hydro_step(_params(1, (n,), 1.0 / n, 1.4), y, rho, 0.2 / n, 50)
    assert st == 0
    np.testing.assert_allclose(r2, rho0, rtol=1e-14)
    assert np.abs(y2[3]).max() < 1e-14


@pytest.mark.parametrize("nd", [1, 2, 3])
def test_conservation_on_periodic_grids(orc, nd):
    rng = np.random.default_rng(5 + nd)
    nn = (24, 20, 16)[:nd]
    shape = (nn[2] if nd == 3 else 1, nn[1] if nd >= 2 else 1, nn[0])
    rho = 1.0 + 0.5 * rng.uniform(size=shape)
    v = [0.3 * rng.normal(size=shape) for _ in range(nd)]
    pr = 1.0 + 0.5 * rng.uniform(size=shape)
    y, rho = _state(nd, rho, v, pr, 5.0 / 3.0)
    p = _params(nd, nn, 1.0 / nn[0], 5.0 / 3.0)
    y2, r2, st, _ = orc.hydro_step(p, y, rho, 0.2 / nn[0], 20)
    assert st == 0
    assert abs(r2.sum() - rho.sum()) < 1e-13 * rho.sum()
    assert abs(y2[1 + nd].sum() - y[1 + nd].sum()) < 1e-13 * y[1 + nd].sum()
    for k in range(nd):
        assert abs(y2[2 + nd + k].sum() - y[2 + nd + k].sum()) < 1e-13 * np.abs(y[2 + nd + k]).sum()
    assert np.abs(r2 - rho).max() > 1e-3   # something happened
    assert np.all(y2[: 1 + nd] == 0.0)    # radiation rows untouched


def test_reflecting_wall_equals_mirror_symmetric_periodic_problem(orc):
    n = 50
    rng = np.random.default_rng(3)
    rho_h = 1.0 + rng.uniform(size=n)
    v_h = 0.5 * rng.normal(size=n)
    p_h = 1.0 + rng.uniform(size=n)
    # periodic domain of 2n cells: the half-state and its mirror image (v negated)
    rho_p = np.concatenate([rho_h, rho_h[::-1]]).reshape(1, 1, 2 * n)
    v_p = np.concatenate([v_h, -v_h[::-1]]).reshape(1, 1, 2 * n)
    p_p = np.concatenate([p_h, p_h[::-1]]).reshape(1, 1, 2 * n)
    yp, rp = _state(1, rho_p, [v_p], p_p, 1.4)
    yw, rw = _state(1, rho_h.reshape(1, 1, n), [v_h.reshape(1, 1, n)], p_h.reshape(1, 1, n), 1.4)
    dt = 0.2 / n
    yp2, rp2, st1, _ = orc.hydro_step(_params(1, (2 * n,), 1.0, 1.4), yp, rp, dt * n, 10)
    yw2, rw2, st2, _ = orc.hydro_step(_params(1, (n,), 1.0, 1.4, bc=(1,)), yw, rw, dt * n, 10)
    assert st1 == 0 and st2 == 0
    np.testing.assert_allclose(rw2.ravel(), rp2.ravel()[:n], rtol=1e-13)
    np.testing.assert_allclose(yw2[2].ravel(), yp2[2].ravel()[:n], rtol=1e-13)
    np.testing.assert_allclose(yw2[3].ravel(), yp2[3].ravel()[:n], rtol=1e-12, atol=1e-13)


def test_hllc_consistency_and_upwinding(orc):
    g = 1.4
    W = np.array([1.3, 0.2, -0.1, 0.7, 2.0])   # rho, v0, v1, v2, p
    # equal states: the physical flux
    f = orc.hllc(g, 3, 0, W, W)
    E = W[4] / (g - 1) + 0.5 * W[0] * (W[1:4] ** 2).sum()
    exact = [W[0] * W[1], W[0] * W[1] * W[1] + W[4], W[0] * W[1] * W[2], W[0] * W[1] * W[3],
             (E + W[4]) * W[1]]
    np.testing.assert_allclose(f, exact, rtol=1e-14)
    # supersonic to the right along axis 1: the left state's flux
    WL = np.array([1.0, 0.0, 5.0, 0.0, 1.0])
    WR = np.array([0.5, 0.0, 5.0, 0.0, 0.4])
    f = orc.hllc(g, 3, 1, WL, WR)
    EL = WL[4] / (g - 1) + 0.5 * WL[0] * 25.0
    np.testing.assert_allclose(f, [5.0, 0.0, 25.0 + 1.0, 0.0, (EL + 1.0) * 5.0], rtol=1e-14)


def _godunov_flux(WL, WR, gamma):
    """Flux of the exact Riemann solution at x/t = 0 (1-D primitive states)."""
    w, _, _ = exact_riemann(WL, WR, gamma, np.array([0.0]))
    r, u, p = w[:, 0]
    E = p / (gamma - 1) + 0.5 * r * u * u
    return np.array([r * u, r * u * u + p, (E + p) * u])


@pytest.mark.parametrize("base", [(1.0, 0.3, 1.0), (0.7, -0.4, 2.0), (1.2, 0.8, 0.8)])
def test_hllc_agrees_with_the_exact_godunov_flux_to_second_order_in_the_jump(orc, base):
    """For a jump of size delta in all three primitive variables the HLLC flux
    differs from the exact Godunov flux by O(delta^2) (both are consistent and
    upwind through the same wave fan)."""
    g = 1.4
    dirs = np.array([0.3, -0.5, 0.4])
    errs = []
    for delta in (4e-3, 2e-3, 1e-3):
        WL = np.array(base) * (1 - delta * dirs)
        WR = np.array(base) * (1 + delta * dirs)
        f = orc.hllc(g, 1, 0, WL, WR)
        errs.append(np.abs(f - _godunov_flux(WL, WR, g)).max())
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs
    # supersonic flow: both are the upwind state's flux
    WL, WR = np.array([1.2, 1.5, 0.8]), np.array([1.1, 1.6, 0.7])
    np.testing.assert_allclose(orc.hllc(g, 1, 0, WL, WR), _godunov_flux(WL, WR, g), rtol=1e-14)
