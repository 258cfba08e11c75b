"""Pins of the oracle's explicit transport (PPM + closure + HLL, RSLA form).

Every expected value here comes from mathematics independent of the oracle's
code: polynomial reconstruction identities, an angular quadrature of a boosted
isotropic intensity (the M1 closure's defining distribution), exact upwinding
in free streaming, mirror symmetry, translation invariance and the RSLA
time-rescaling of the transport equations.
"""
import numpy as np
import pytest

from paper_2404_08247_amd import workloads as W


def _p1d(n, chat=1.0, bc=0, closure="m1", **kw):
    p = W.base_params(1, (n,), chat, (bc,), closure=closure, **kw)
    return p


# ---------------------------------------------------------------- PPM (CW84) --
def test_ppm_constant_and_linear_exact(orc):
    rng = np.random.default_rng(1)
    for _ in range(5):
        a0, b = rng.normal(size=2)
        a = a0 + b * np.arange(12, dtype=float)
        aL, aR = orc.ppm_edges(a)
        i = np.arange(2, 10)
        np.testing.assert_allclose(aL[i], a[i] - 0.5 * b, rtol=0, atol=1e-13 * (abs(a0) + 12 * abs(b)))
        np.testing.assert_allclose(aR[i], a[i] + 0.5 * b, rtol=0, atol=1e-13 * (abs(a0) + 12 * abs(b)))
    c = np.full(9, 3.25)
    aL, aR = orc.ppm_edges(c)
    assert np.all(aL[2:7] == 3.25) and np.all(aR[2:7] == 3.25)


def test_ppm_cubic_cell_averages_give_exact_interface_values(orc):
    # Unlimited PPM interpolation is exact for cell averages of a cubic; on a
    # smooth, monotone, convex cubic the limiter and monotonicity steps are idle.
    f = lambda x: x ** 3 + x
    F = lambda x: x ** 4 / 4 + x ** 2 / 2            # antiderivative
    h = 0.01
    x = 1.0 + h * np.arange(16)
    avg = (F(x + h) - F(x)) / h
    aL, aR = orc.ppm_edges(avg)
    i = np.arange(2, 14)
    np.testing.assert_allclose(aR[i], f(x[i] + h), rtol=1e-12)
    np.testing.assert_allclose(aL[i], f(x[i]), rtol=1e-12)


def test_ppm_monotone_at_a_step(orc):
    a = np.array([0, 0, 0, 0, 1, 1, 1, 1], dtype=float)
    aL, aR = orc.ppm_edges(a)
    for i in range(2, 6):
        lo, hi = min(a[i - 1], a[i], a[i + 1]), max(a[i - 1], a[i], a[i + 1])
        assert lo <= aL[i] <= hi and lo <= aR[i] <= hi


def test_ppm_limiter_properties_on_rough_data(orc):
    """The limited parabola of each cell (CW84, as the transport uses it in
    Sec. 3.3) on rough data, where no polynomial identity applies. What the
    limiter is for fixes these properties: a cell whose average is a strict
    local extremum is flattened to its average; every other cell is flat or
    carries a parabola without an interior extremum (|a6| <= |aR - aL| with
    a6 = 6 a - 3 (aL + aR)); both edges stay within the range of the cell and
    its two neighbours; on increasing data the edges keep the order
    a[i-1] <= aL <= a[i] <= aR <= a[i+1]."""
    rng = np.random.default_rng(11)
    eps = np.finfo(float).eps
    n = 40
    for trial in range(160):
        kind = trial % 4
        if kind == 0:
            a = rng.normal(size=n)                                   # noise
        elif kind == 1:
            a = np.cumsum(rng.exponential(size=n))                   # increasing, rough
        elif kind == 2:
            a = np.where(rng.random(n) < 0.2, 5.0, 0.0) + 1e-3 * rng.normal(size=n)  # spikes
        else:
            a = np.round(3.0 * rng.normal(size=n)) / 3.0             # plateaus and steps
        aL, aR = orc.ppm_edges(a)
        for i in range(2, n - 2):
            ai, l, r = a[i], aL[i], aR[i]
            lo, hi = min(a[i - 1], ai, a[i + 1]), max(a[i - 1], ai, a[i + 1])
            assert lo <= l <= hi and lo <= r <= hi, (trial, i)
            flat = (l == ai and r == ai)
            if (ai > a[i - 1] and ai > a[i + 1]) or (ai < a[i - 1] and ai < a[i + 1]):
                assert flat, (trial, i)
            if not flat:
                a6 = 6.0 * ai - 3.0 * (l + r)
                tol = 8 * eps * (6 * abs(ai) + 3 * abs(l) + 3 * abs(r))
                assert abs(a6) <= abs(r - l) + tol, (trial, i, a6, r - l)
            if kind == 1:
                assert a[i - 1] <= l <= ai <= r <= a[i + 1], (trial, i)


# ------------------------------------------------------------------ closure --
def _m1_by_quadrature(f_target):
    """Eddington factor of the intensity I(mu) ~ (1 - b mu)^-4 (an isotropic
    distribution seen from a moving frame), the distribution that defines the M1
    closure; b is found so that F/(cE) = f_target. Gauss-Legendre quadrature."""
    mu, w = np.polynomial.legendre.leggauss(200)

    def moments(b):
        I = (1.0 - b * mu) ** -4
        return (w * I).sum(), (w * I * mu).sum(), (w * I * mu * mu).sum()

    lo, hi = 0.0, 1.0 - 1e-12
    for _ in range(200):
        b = 0.5 * (lo + hi)
        E, F, P = moments(b)
        if F / E < f_target:
            lo = b
        else:
            hi = b
    E, F, P = moments(0.5 * (lo + hi))
    return P / E


@pytest.mark.parametrize("f", [0.0, 0.2, 0.5, 0.8, 0.95])
def test_m1_closure_matches_boosted_isotropic_intensity(orc, f):
    p = _p1d(8)
    E = 2.0
    n = np.array([0.6, -0.48, 0.64])  # unit vector
    D = orc.closure(dict(p, ndim=3), 3, E, f * p["c"] * E * n)
    chi = _m1_by_quadrature(f) if f > 0 else 1.0 / 3.0
    # D = (1-chi)/2 I + (3chi-1)/2 n n
    Dref = 0.5 * (1 - chi) * np.eye(3) + 0.5 * (3 * chi - 1) * np.outer(n, n)
    np.testing.assert_allclose(D, Dref, rtol=0, atol=2e-9)
    assert abs(np.trace(D) - 1.0) < 1e-14


def test_closure_limits(orc):
    p = _p1d(8)
    D0 = orc.closure(dict(p, ndim=3), 3, 1.0, [0.0, 0.0, 0.0])
    np.testing.assert_allclose(D0, np.eye(3) / 3, atol=1e-16)
    D1 = orc.closure(dict(p, ndim=3), 3, 1.0, [0.0, 1.0, 0.0])     # |F| = cE
    np.testing.assert_allclose(D1, np.diag([0.0, 1.0, 0.0]), atol=1e-15)
    De = orc.closure(dict(p, ndim=3, closure="eddington"), 3, 1.0, [0.0, 0.9, 0.0])
    np.testing.assert_allclose(De, np.eye(3) / 3, atol=1e-16)


# ---------------------------------------------------------------------- HLL --
def test_hll_uniform_state_is_physical_flux(orc):
    chat = 0.1
    p = dict(_p1d(8, chat=chat), ndim=3)
    U = np.array([2.0, 0.3, -0.4, 0.5])
    for d in range(3):
        fl = orc.hll(p, 3, d, U, U)
        D = orc.closure(p, 3, U[0], U[1:])
        ref = np.concatenate([[chat / p["c"] * U[1 + d]], p["c"] * chat * U[0] * D[d]])
        np.testing.assert_allclose(fl, ref, rtol=1e-15, atol=1e-17)


def test_hll_dissipation_speed_eddington(orc):
    chat = 0.5
    p = dict(_p1d(8, chat=chat, closure="eddington"), ndim=1)
    Um, Up = np.array([1.0, 0.0]), np.array([3.0, 0.0])
    fl = orc.hll(p, 1, 0, Um, Up)
    S = chat / np.sqrt(3.0)
    # Phi_E = -S/2 (E+ - E-); Phi_F = c chat (E- + E+)/6
    np.testing.assert_allclose(fl, [-0.5 * S * 2.0, p["c"] * chat * 4.0 / 6.0], rtol=1e-15)


# ---------------------------------------------------------- free streaming --
def _streaming_state(n, ndim=1, axis=0):
    x = W.cell_centres(n)
    E = 1e-10 + np.exp(-((x - 0.3) ** 2) / (2 * 0.05 ** 2))
    return x, E


def _run_stream(orc, n, t_end, chat=1.0):
    p = _p1d(n, chat=chat)
    x, E = _streaming_state(n)
    y = np.zeros((4, 1, 1, n))
    y[0, 0, 0] = E
    y[1, 0, 0] = p["c"] * E         # F = cE: f = 1, pure streaming along +x
    y[2] = 1.0                      # gas energy (uncoupled, chi = 0)
    zero = np.zeros((1, 1, n))
    dt = 0.3 * p["dx"] / chat
    nsteps = int(round(t_end / dt))
    yo, st, _ = orc.step(p, y, np.ones((1, 1, n)), zero, None, dt, nsteps)
    assert st == 0
    return p, x, E, yo, nsteps * dt


def test_free_streaming_conserves_and_converges_to_translation(orc):
    errs = []
    for n in (64, 128, 256):
        p, x, E0, yo, t = _run_stream(orc, n, 0.3)
        E = yo[0, 0, 0]
        assert abs(E.sum() - E0.sum()) <= 1e-14 * E0.sum()
        # F stays equal to cE (both advect identically)
        np.testing.assert_allclose(yo[1, 0, 0], p["c"] * E, rtol=1e-12)
        xs = x - p["chat"] * t
        exact = 1e-10 + np.exp(-((xs - 0.3) ** 2) / (2 * 0.05 ** 2))
        errs.append(np.abs(E - exact).sum() / np.abs(exact).sum())
        cen = (x * E).sum() / E.sum()
        cen0 = (x * E0).sum() / E0.sum()
        if n == 256:
            assert abs((cen - cen0) / (p["chat"] * t) - 1.0) < 2e-3
    assert errs[1] < 0.5 * errs[0] and errs[2] < 0.5 * errs[1], errs


def test_streaming_with_reduced_chat_is_a_time_rescaling(orc):
    # RSLA transport: dE/dt = -(chat/c) div F, dF/dt = -c chat div P. With
    # t' = (chat/c) t these are the chat = c equations, so a step of dt at chat
    # equals a step of (chat/c) dt at chat = c (to rounding).
    n = 48
    rng = np.random.default_rng(7)
    y = np.zeros((4, 1, 1, n))
    y[0] = 1.0 + 0.5 * rng.random(n)
    y[1] = 0.3 * (rng.random(n) - 0.5)
    y[2] = 1.0
    s1 = orc.transport(_p1d(n, chat=0.01), y)
    s2 = orc.transport(_p1d(n, chat=1.0), y)
    np.testing.assert_allclose(s1[0] / 0.01, s2[0], rtol=1e-13, atol=1e-13 * np.abs(s2[0]).max())
    np.testing.assert_allclose(s1[1] / 0.01, s2[1], rtol=1e-13, atol=1e-13 * np.abs(s2[1]).max())


# --------------------------------------------------- symmetry / invariance --
def test_reflecting_walls_keep_mirror_symmetry(orc):
    w = W.config1(n=64, nsteps=40)
    y = w.y0.copy()
    y[..., 32:] = y[..., :32][..., ::-1]     # exact mirror image
    y[1, ..., 32:] = -y[1, ..., :32][..., ::-1]
    yo, st, _ = orc.step(w.params, y, w.rho, w.kappa_P, None, w.dt, w.nsteps)
    assert st == 0
    E = yo[0, 0, 0]
    np.testing.assert_array_equal(E, E[::-1])
    np.testing.assert_array_equal(yo[1, 0, 0], -yo[1, 0, 0][::-1])
    # no energy through the walls: E_gas + (c/chat) E summed is conserved
    tot0 = (y[2] + y[0]).sum()
    tot = (yo[2] + yo[0]).sum()
    assert abs(tot - tot0) <= 1e-14 * tot0


def test_translation_invariance_periodic_3d(orc):
    w = W.config2(n=(12, 10, 8), nsteps=2)
    shift = (3, -2, 5)
    ys = np.roll(w.y0, shift, axis=(1, 2, 3))
    kap = np.roll(w.kappa_P, shift, axis=(0, 1, 2))
    y1, s1, _ = orc.step(w.params, w.y0, w.rho, w.kappa_P, None, w.dt, 2)
    y2, s2, _ = orc.step(w.params, ys, w.rho, kap, None, w.dt, 2)
    assert s1 == 0 and s2 == 0
    np.testing.assert_array_equal(np.roll(y1, shift, axis=(1, 2, 3)), y2)


def test_1d_problem_embedded_in_3d_matches_1d(orc):
    # a field that varies only along x evolves identically on a 3-D periodic grid
    n = 32
    rng = np.random.default_rng(3)
    E = 1e-8 * (1.0 + rng.random(n))
    T = 1.0 + 0.2 * rng.random(n)
    kap = 10.0 ** rng.uniform(-1, 2, n) * n
    p1 = W.base_params(1, (n,), 0.1, (0,))
    p3 = W.base_params(3, (n, 4, 4), 0.1, (0, 0, 0))
    cv = p1["kB_over_mu"] / (p1["gamma"] - 1)
    y1 = np.zeros((4, 1, 1, n))
    y1[0] = E
    y1[1] = 0.1 * E * (rng.random(n) - 0.5)
    y1[2] = cv * T
    y3 = np.zeros((8, 4, 4, n))
    y3[0] = y1[0]
    y3[1] = y1[1]
    y3[4] = y1[2]
    dt = 0.3 * p1["dx"] / 0.1
    o1, a, _ = orc.step(p1, y1, np.ones((1, 1, n)), kap.reshape(1, 1, n), None, dt, 3)
    o3, b, _ = orc.step(p3, y3, np.ones((4, 4, n)), np.broadcast_to(kap, (4, 4, n)).copy(), None, dt, 3)
    assert a == 0 and b == 0
    for v1, v3 in ((0, 0), (1, 1), (2, 4), (3, 5)):
        for j in range(4):
            for k in range(4):
                np.testing.assert_allclose(o3[v3, k, j], o1[v1, 0, 0], rtol=1e-14,
                                           atol=1e-14 * np.abs(o1[v1]).max())
    assert np.abs(o3[[2, 3, 6, 7]]).max() == 0.0


def test_reflecting_walls_equal_the_mirrored_periodic_problem(orc):
    # Method of images: on [0, 1) with reflecting walls the solution equals the
    # restriction of the periodic problem on [-1, 1) started from the mirror
    # extension (E, E_gas even; F, rho v odd). A pulse sits on the wall at x = 0.
    n = 32
    rng = np.random.default_rng(4)
    p_ref = W.base_params(1, (n,), 0.5, (1,))
    p_per = W.base_params(1, (2 * n,), 0.5, (0,))
    p_per["dx"] = p_ref["dx"]
    cv = p_ref["kB_over_mu"] / (p_ref["gamma"] - 1)
    x = W.cell_centres(n)
    T = 1.0 + 3.0 * np.exp(-x ** 2 / 0.1 ** 2) + 0.1 * rng.random(n)
    E = p_ref["a_r"] * T ** 4 * (1 + 0.2 * rng.random(n))
    F = 0.3 * p_ref["c"] * E * (rng.random(n) - 0.3)
    mom = 1e-3 * (rng.random(n) - 0.5)
    half = np.zeros((4, 1, 1, n))
    half[0] = E
    half[1] = F
    half[2] = cv * T + 0.5 * mom ** 2
    half[3] = mom
    kap = 10.0 ** rng.uniform(-1, 2, n) * n
    full = np.zeros((4, 1, 1, 2 * n))
    full[:, 0, 0, n:] = half[:, 0, 0]
    full[:, 0, 0, :n] = half[:, 0, 0, ::-1]
    full[1, 0, 0, :n] *= -1
    full[3, 0, 0, :n] *= -1
    kfull = np.concatenate([kap[::-1], kap]).reshape(1, 1, -1)
    dt = 0.3 * p_ref["dx"] / 0.5
    a, s1, _ = orc.step(p_ref, half, np.ones((1, 1, n)), kap.reshape(1, 1, -1), None, dt, 25)
    b, s2, _ = orc.step(p_per, full, np.ones((1, 1, 2 * n)), kfull, None, dt, 25)
    assert s1 == 0 and s2 == 0
    for v in range(4):
        sc = np.abs(b[v]).max()
        np.testing.assert_allclose(a[v, 0, 0], b[v, 0, 0, n:], rtol=0, atol=1e-13 * sc)


# ------------------------------------------------------- transverse axes --
def _rotate_problem(p, y, rho, kap):
    """The same physical problem with the axes renamed cyclically: old z -> new
    x, old x -> new y, old y -> new z (a rotation of the grid). Arrays [z][y][x]
    become [y][x][z] (numpy axes (1, 2, 0)); the vector components F and rho v
    are permuted the same way; n and bc follow their axes."""
    n = p["n"]
    q = dict(p, n=(n[2], n[0], n[1]), bc=(p["bc"][2], p["bc"][0], p["bc"][1]))
    r = lambda a: np.ascontiguousarray(np.transpose(a, (1, 2, 0)))
    z = np.empty((8,) + r(y[0]).shape)
    z[0], z[4] = r(y[0]), r(y[4])
    for new, old in ((0, 2), (1, 0), (2, 1)):
        z[1 + new] = r(y[1 + old])
        z[5 + new] = r(y[5 + old])
    return q, z, r(rho), r(kap)


@pytest.mark.parametrize("closure", ["m1", "eddington"])
@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 1), (1, 0, 1), (0, 1, 1)])
def test_rotated_grid_gives_the_rotated_result(orc, closure, bc):
    """The method treats the three axes alike (Sec. 3.3 reconstructs and fluxes
    along every direction; the HLL speed along a direction is the Eddington-tensor
    component along it, Sec. 4.3): rotating a 3-D problem and its boundary kinds
    rotates the transport output and the result of whole steps, to round-off (the
    unsplit divergence sums the axes in another order). A wrong component, sign
    flip or signal speed on one of y or z moves the output of one of the two runs
    only. Extents differ per axis so that a swapped line mapping cannot match."""
    w = W.config5(n=(9, 7, 6), nsteps=2, precision="fp64", bc=bc, closure=closure)
    rng = np.random.default_rng(41)
    y = w.y0.copy()
    E = y[0]
    dirs = rng.normal(size=(3,) + E.shape)
    dirs /= np.linalg.norm(dirs, axis=0)
    f = rng.uniform(0.0, 0.9, E.shape)
    for d in range(3):
        y[1 + d] = f * w.params["c"] * E * dirs[d]
    q, z, rho_r, kap_r = _rotate_problem(w.params, y, w.rho, w.kappa_P)
    s = orc.transport(w.params, y)
    sr = orc.transport(q, z)
    q2, s_rot, _, _ = _rotate_problem(w.params, s, w.rho, w.kappa_P)
    for v in range(4):
        sc = np.abs(s_rot[v]).max()
        np.testing.assert_allclose(sr[v], s_rot[v], rtol=0, atol=1e-14 * sc)
    a, st1, _ = orc.step(w.params, y, w.rho, w.kappa_P, None, w.dt, w.nsteps)
    b, st2, _ = orc.step(q, z, rho_r, kap_r, None, w.dt, w.nsteps)
    assert st1 == 0 and st2 == 0
    _, a_rot, _, _ = _rotate_problem(w.params, a, w.rho, w.kappa_P)
    for v in range(8):
        sc = np.abs(a_rot[v]).max()
        np.testing.assert_allclose(b[v], a_rot[v], rtol=0, atol=1e-13 * sc)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_hll_dissipation_along_each_axis_m1(orc, d):
    """HLL along axis d with an oblique flux under M1 (Sec. 4.3): the dissipation
    speed is chat sqrt(max(D_dd-, D_dd+)), the Eddington-tensor component along
    d of each face state. The tensors come from the boosted-isotropic-intensity
    quadrature, not from the oracle's closure; D_xx, D_yy and D_zz all differ."""
    chat = 0.2
    p = dict(_p1d(8, chat=chat), ndim=3)
    c = p["c"]
    nm = np.array([0.36, -0.48, 0.8])                      # unit vectors
    npl = np.array([-0.6, 0.64, 0.48])
    Em, Ep, fm, fp = 1.5, 0.9, 0.7, 0.45
    Um = np.concatenate([[Em], fm * c * Em * nm])
    Up = np.concatenate([[Ep], fp * c * Ep * npl])

    def D_of(f, n):
        chi = _m1_by_quadrature(f)
        return 0.5 * (1 - chi) * np.eye(3) + 0.5 * (3 * chi - 1) * np.outer(n, n)

    Dm, Dp = D_of(fm, nm), D_of(fp, npl)
    S = chat * np.sqrt(max(Dm[d, d], Dp[d, d]))
    phys = lambda U, D: np.concatenate([[chat / c * U[1 + d]], c * chat * U[0] * D[d]])
    ref = 0.5 * (phys(Um, Dm) + phys(Up, Dp)) - 0.5 * S * (Up - Um)
    fl = orc.hll(p, 3, d, Um, Up)
    np.testing.assert_allclose(fl, ref, rtol=0, atol=5e-9 * np.abs(ref).max())
    # the speed is that of axis d: the other axes' speeds give another flux
    for e in range(3):
        if e != d and abs(max(Dm[e, e], Dp[e, e]) - max(Dm[d, d], Dp[d, d])) > 1e-3:
            Se = chat * np.sqrt(max(Dm[e, e], Dp[e, e]))
            wrong = 0.5 * (phys(Um, Dm) + phys(Up, Dp)) - 0.5 * Se * (Up - Um)
            assert np.abs(fl - wrong).max() > 1e-4 * np.abs(ref).max()
