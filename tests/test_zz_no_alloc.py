"""rhd_step_noalloc (the allocation-free step: no handle, no workspace, scratch
in a static device array) against rhd_step on a handle, through the C ABI, on
the same inputs: two calls in a row, the second on a smaller grid, then a 1-D
line and a mixed-precision grid. Same kernels and launch shapes, so the results
agree bitwise; the bar is the FP64 parity bar (1e-10, 1e-5 in mixed precision)."""
import sys

import numpy as np
import pytest

from paper_2404_08247_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


def _to(torch_dev, a):
    torch, dev = torch_dev
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)


def _compare(torch_dev, w, tol):
    from paper_2404_08247_amd import rhd
    torch, dev = torch_dev
    rho, kap = _to(torch_dev, w.rho), _to(torch_dev, w.kappa_P)
    S = rhd.Solver(w.params, rho, kap, None, 0, dev)
    ref = _to(torch_dev, w.y0)
    S.step(ref, w.dt, w.nsteps)
    y = _to(torch_dev, w.y0)
    st, cell = rhd.step_noalloc(w.params, y, rho, kap, None, w.dt, w.nsteps)
    torch.cuda.synchronize()
    assert st == rhd.RHD_OK and cell == -1, (st, cell)
    a, b = y.cpu().numpy(), ref.cpu().numpy()
    err = max(np.abs(a[v] - b[v]).max() / max(np.abs(b[v]).max(), 1e-300) for v in range(w.nvar))
    _say("  noalloc vs handle: max rel err", err, " bitwise", bool(np.array_equal(a, b)))
    assert err <= tol, err


def test_noalloc_step_matches_handle_step_on_two_calls(torch_dev):
    w1 = W.config2(n=(48, 40, 36), nsteps=3)
    _say("noalloc call 1", w1.n, w1.nsteps)
    _compare(torch_dev, w1, 1e-10)
    w2 = W.config5(n=(24, 16, 12), nsteps=2, precision="fp64")   # smaller, moving gas
    _say("noalloc call 2 (smaller)", w2.n, w2.nsteps)
    _compare(torch_dev, w2, 1e-10)


def test_noalloc_step_on_a_line_and_in_mixed_precision(torch_dev):
    w = W.config1(n=200, nsteps=40)
    _say("noalloc 1-D line", w.n, w.nsteps)
    _compare(torch_dev, w, 1e-10)
    w = W.config3(n=(40, 24, 20), nsteps=4, precision="mixed")
    _say("noalloc mixed", w.n, w.nsteps)
    _compare(torch_dev, w, 1e-5)


def test_noalloc_step_reports_failures_like_rhd_step(torch_dev, orc):
    from paper_2404_08247_amd import rhd
    w = W.config2(n=(20, 12, 10), nsteps=1, newton_maxit=1)
    _, st, cell = orc.step(w.params, w.y0, w.rho, w.kappa_P, None, w.dt, 1)
    assert st != 0
    y = _to(torch_dev, w.y0)
    got, gcell = rhd.step_noalloc(w.params, y, _to(torch_dev, w.rho), _to(torch_dev, w.kappa_P),
                                  None, w.dt, 1)
    assert got == rhd.RHD_ENEWTON and gcell == cell, (got, gcell, cell)


def test_noalloc_step_at_the_largest_grid_its_scratch_holds(torch_dev):
    # 256 + 8 nvar N <= 64 MiB: 128 x 128 x 63 = 1032192 cells in 3-D (64 planes,
    # 1048576 cells, would need 256 bytes more than the scratch holds and are
    # rejected, as the CPU test of the validation checks)
    w = W.config2(n=(128, 128, 63), nsteps=2)
    assert 256 + 8 * w.nvar * w.ncells <= 64 << 20 < 256 + 8 * w.nvar * 128 * 128 * 64
    _say("noalloc largest grid", w.n, w.nsteps)
    _compare(torch_dev, w, 1e-10)
