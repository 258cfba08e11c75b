"""C-ABI checks that need no GPU: the library loads, exports every entry point
that include/rhd.h declares, and validates parameters on the host (no kernel
is launched by any call here)."""
import ctypes
import os
import re

import pytest

from paper_2404_08247_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rhd.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rhd_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2404_08247_amd import rhd
    names = _declared()
    assert len(names) >= 8
    for n in names:
        assert hasattr(rhd.lib, n), n
    assert sorted(rhd.EXPORTED) == names


def test_params_struct_layout_matches_header():
    from paper_2404_08247_amd import rhd
    # int32 ndim, closure; int64 n[3]; 6 doubles; int32 bc[3], v_order, precision,
    # newton_maxit, outer_maxit, scheme; 6 doubles
    assert ctypes.sizeof(rhd.RHDParams) == 8 + 24 + 48 + 32 + 48
    assert rhd.RHDParams.n.offset == 8
    assert rhd.RHDParams.bc.offset == 80
    assert rhd.RHDParams.newton_rtol.offset == 112
    assert rhd.RHDParams.hll_eps_cells.offset == 128
    assert rhd.RHDParams.inflow_F.offset == 152


def _ws(p, k=0):
    from paper_2404_08247_amd import rhd
    return rhd.workspace_bytes(p, k)


def test_workspace_size_and_validation():
    w = W.config2(n=(16, 12, 10))
    p = w.params
    nb = _ws(p)
    assert nb >= 8 * 8 * 16 * 12 * 10
    assert _ws(p, 4) > nb
    bad = [dict(p, chat=2.0), dict(p, chat=0.0), dict(p, dx=-1.0), dict(p, gamma=1.0),
           dict(p, v_order=3), dict(p, ndim=4), dict(p, n=(16, 12, 0)),
           dict(p, newton_maxit=0), dict(p, a_r=0.0), dict(p, newton_rtol=0.0),
           dict(p, hll_eps_cells=-1.0), dict(p, hll_eps_cells=float("inf")),
           dict(p, kappa_T_power=-3.0, hll_eps_cells=1.0), dict(p, bc=(3, 0, 0)),
           dict(p, inflow_E=float("nan"))]
    for b in bad:
        assert _ws(b) == 0, b
    # reflecting axis needs >= 3 cells; axes beyond ndim must be 1
    assert _ws(dict(p, n=(16, 2, 10), bc=(0, 1, 0))) == 0
    assert _ws(dict(W.config1(n=8).params, n=(8, 2, 1))) == 0


def test_create_rejects_bad_arguments_without_launching():
    from paper_2404_08247_amd import rhd
    L = rhd.lib
    p = W.config2(n=(16, 12, 10)).params
    rp = rhd.make_params(p)
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)           # never dereferenced on these paths
    nb = L.rhd_workspace_bytes(ctypes.byref(rp), 0)
    # NULL density
    assert L.rhd_create(ctypes.byref(rp), None, fake, None, fake, nb, None, ctypes.byref(h)) == -1
    # workspace too small / misaligned
    assert L.rhd_create(ctypes.byref(rp), fake, fake, None, fake, nb - 8, None, ctypes.byref(h)) == -5
    assert L.rhd_create(ctypes.byref(rp), fake, fake, None, ctypes.c_void_p((1 << 20) + 8), nb,
                        None, ctypes.byref(h)) == -5
    # order 2 with a distinct flux-mean opacity is accepted (3x3 flux solve)
    other = ctypes.c_void_p(1 << 21)
    assert L.rhd_create(ctypes.byref(rp), fake, fake, other, fake, nb, None, ctypes.byref(h)) == 0
    L.rhd_destroy(h)
    h = ctypes.c_void_p()
    # a valid create binds pointers only (no device work), destroy frees it
    assert L.rhd_create(ctypes.byref(rp), fake, fake, None, fake, nb, None, ctypes.byref(h)) == 0
    assert h.value is not None
    # invalid step arguments are rejected before any launch
    assert L.rhd_step(h, None, ctypes.c_double(0.1), 1) == -1
    assert L.rhd_step(h, fake, ctypes.c_double(-0.1), 1) == -1
    cell = ctypes.c_int64(0)
    buf = ctypes.create_string_buffer(64)
    assert L.rhd_last_error(h, ctypes.byref(cell), buf, 64) == -1
    L.rhd_destroy(h)
    L.rhd_destroy(None)


def test_adjoint_rejects_what_it_does_not_differentiate():
    """rhd_step_adjoint validates before any launch: reflecting axes, the RK2-SSP
    comparator and the HLL eps correction are rejected with RHD_EINVAL."""
    from paper_2404_08247_amd import rhd
    L = rhd.lib
    fake = ctypes.c_void_p(1 << 20)
    base = W.config4(n=(16, 12)).params
    for bad in (dict(base, bc=(1, 0)), dict(base, scheme="rk2ssp"), dict(base, hll_eps_cells=1.0),
                dict(base, bc=(2, 0)), dict(base, kappa_T_power=-3.0)):
        rp = rhd.make_params(bad)
        nb = L.rhd_workspace_bytes(ctypes.byref(rp), 2)
        assert nb > 0
        h = ctypes.c_void_p()
        assert L.rhd_create(ctypes.byref(rp), fake, fake, None, fake, nb, None, ctypes.byref(h)) == 0
        st = L.rhd_step_adjoint(h, ctypes.c_void_p(1 << 22), ctypes.c_double(0.1), 1,
                                ctypes.c_void_p(1 << 23), ctypes.c_void_p(1 << 24), None)
        assert st == -1, bad
        L.rhd_destroy(h)


def test_hydro_entry_points_validate_before_launching():
    """rhd_hydro_step / rhd_rhd_step reject a density other than the bound one,
    dt <= 0, nsteps < 0 and nsub < 1 with RHD_EINVAL (no launch)."""
    from paper_2404_08247_amd import rhd
    L = rhd.lib
    p = W.config2(n=(16, 12, 10)).params
    rp = rhd.make_params(p)
    nb = L.rhd_workspace_bytes(ctypes.byref(rp), 0)
    rho = ctypes.c_void_p(1 << 20)
    other = ctypes.c_void_p(1 << 21)
    y = ctypes.c_void_p(1 << 22)
    h = ctypes.c_void_p()
    assert L.rhd_create(ctypes.byref(rp), rho, other, None, ctypes.c_void_p(1 << 23), nb, None,
                        ctypes.byref(h)) == 0
    assert L.rhd_hydro_step(h, y, other, ctypes.c_double(1e-3), 1) == -1
    assert L.rhd_hydro_step(h, y, rho, ctypes.c_double(0.0), 1) == -1
    assert L.rhd_hydro_step(h, y, rho, ctypes.c_double(1e-3), -1) == -1
    assert L.rhd_hydro_step(h, None, rho, ctypes.c_double(1e-3), 1) == -1
    assert L.rhd_rhd_step(h, y, rho, ctypes.c_double(1e-3), 0, 1) == -1
    assert L.rhd_rhd_step(h, y, other, ctypes.c_double(1e-3), 2, 1) == -1
    assert L.rhd_hydro_signal_speed(h, y, rho, None) == -1
    L.rhd_destroy(h)


def test_adjoint_segment_capacity_follows_the_workspace_size():
    """rhd_create takes no segment length: a workspace of rhd_workspace_bytes(p, k)
    bytes admits adjoint segments of up to k steps (longer ones are rejected with
    RHD_EINVAL before any launch), and a forward-only workspace admits none."""
    from paper_2404_08247_amd import rhd
    L = rhd.lib
    fake = ctypes.c_void_p(1 << 20)
    p = W.config4(n=(16, 12)).params
    rp = rhd.make_params(p)
    for k in (0, 1, 2, 5):
        nb = L.rhd_workspace_bytes(ctypes.byref(rp), k)
        for slack in (0, 255):
            h = ctypes.c_void_p()
            assert L.rhd_create(ctypes.byref(rp), fake, fake, None, fake, nb + slack, None,
                                ctypes.byref(h)) == 0
            st = L.rhd_step_adjoint(h, ctypes.c_void_p(1 << 22), ctypes.c_double(0.1), k + 1,
                                    ctypes.c_void_p(1 << 23), ctypes.c_void_p(1 << 24), None)
            assert st == -1, (k, slack)
            L.rhd_destroy(h)


def test_adjoint_rejects_overlapping_arrays_before_touching_the_gpu():
    """rhd_step_adjoint reverses in lambda and reads state0 until it returns, so
    overlapping state0, lambda and gradient arrays are rejected with RHD_EINVAL
    before any HIP call (fake device addresses: this runs without a GPU)."""
    from paper_2404_08247_amd import rhd
    L = rhd.lib
    fake = ctypes.c_void_p(1 << 20)
    w = W.config4(n=(16, 12))
    rp = rhd.make_params(w.params)
    nb = L.rhd_workspace_bytes(ctypes.byref(rp), 2)
    h = ctypes.c_void_p()
    assert L.rhd_create(ctypes.byref(rp), fake, fake, None, fake, nb, None, ctypes.byref(h)) == 0
    nst = w.nvar * 16 * 12 * 8          # bytes of one state
    base = 1 << 30
    cases = [
        (base, base + 8 * 7, base + 4 * nst),                 # lambda starts inside state0
        (base + nst - 8, base, base + 4 * nst),               # state0 ends inside lambda
        (base, base + 2 * nst, base + 3 * nst - 64),          # g_kappa_P overlaps lambda's end
        (base, base + 2 * nst, base + 64),                    # g_kappa_P inside state0
    ]
    msg = ctypes.create_string_buffer(256)
    cell = ctypes.c_int64(0)
    for s0, lam, gk in cases:
        st = L.rhd_step_adjoint(h, ctypes.c_void_p(s0), ctypes.c_double(0.1), 1,
                                ctypes.c_void_p(lam), ctypes.c_void_p(gk), None)
        assert st == -1, (s0, lam, gk)
        L.rhd_last_error(h, ctypes.byref(cell), msg, 256)
        assert b"overlap" in msg.value
    L.rhd_destroy(h)


def test_noalloc_step_validates_before_touching_the_gpu():
    """rhd_step_noalloc rejects invalid parameters, pointers and dt with RHD_EINVAL
    and a grid whose y^{n+1/2} does not fit its 64 MiB static scratch with
    RHD_EWORKSPACE, before any HIP call (these calls run on a host without a GPU)."""
    from paper_2404_08247_amd import rhd
    L = rhd.lib
    fake = ctypes.c_void_p(1 << 20)
    cell = ctypes.c_int64(7)
    ok = W.config2(n=(16, 12, 10)).params
    big = W.config2(n=(128, 128, 64)).params        # 8 * 8 * 1048576 B > 64 MiB - 256
    fits = W.config2(n=(128, 128, 63)).params       # 66060288 + 256 B <= 64 MiB
    args = lambda p, y, dt: (ctypes.byref(rhd.make_params(p)), fake, fake, None, y,
                             ctypes.c_double(dt), 1, None, ctypes.byref(cell))
    assert L.rhd_step_noalloc(*args(dict(ok, chat=2.0), fake, 0.1)) == -1
    assert cell.value == -1
    assert L.rhd_step_noalloc(*args(ok, None, 0.1)) == -1
    assert L.rhd_step_noalloc(*args(ok, ctypes.c_void_p((1 << 20) + 4), 0.1)) == -1
    assert L.rhd_step_noalloc(*args(ok, fake, -0.1)) == -1
    assert L.rhd_step_noalloc(*args(big, fake, 0.1)) == -5
    # a grid that fits gets past the size check (and then needs a GPU)
    assert L.rhd_step_noalloc(*args(fits, fake, 0.1)) != -5


def test_binding_fails_loudly_without_the_library(tmp_path):
    """The product path has no fallback: importing the binding from a copy of the
    package that lacks librhd.so raises ImportError naming the missing file."""
    import shutil
    import subprocess
    import sys
    src = os.path.join(ROOT, "paper_2404_08247_amd")
    dst = tmp_path / "paper_2404_08247_amd"
    dst.mkdir()
    for f in os.listdir(src):
        if f.endswith(".py"):
            shutil.copy(os.path.join(src, f), dst / f)
    code = ("import sys; sys.path.insert(0, sys.argv[1])\n"
            "try:\n    import paper_2404_08247_amd.rhd\nexcept ImportError as e:\n"
            "    print('IMPORTERROR', e); sys.exit(3)\nprint('IMPORTED'); sys.exit(0)\n")
    r = subprocess.run([sys.executable, "-c", code, str(tmp_path)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 3 and "librhd.so is missing" in r.stdout, (r.returncode, r.stdout, r.stderr)
