"""The allocation-free solve entry point (hps_solve_noalloc) against hps_solve: the same
factor, inputs and kernels, with the workspace carved from the library's fixed per-GPU
scratch array instead of allocated.  Two calls in a row, the second on a smaller
problem with fewer right-hand sides (the array keeps the first call's contents), in
complex128 and with the mixed-precision correction; a call whose workspace exceeds the
array is refused before anything is enqueued."""

import sys

import numpy as np
import pytest

from tests.hps_cases import Case, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1812_07167_amd import hps as H
    H.load()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _both(cs, f, with_s):
    import torch
    from paper_1812_07167_amd import hps as H
    t = torch.tensor(cs.t, dtype=torch.complex128, device="cuda")
    s = torch.tensor(cs.s, dtype=torch.complex128, device="cuda") if with_s else None
    u_ref = H.hps_solve(f, t, s)
    u_na = torch.full_like(u_ref, complex(np.nan, np.nan))
    H.hps_solve_noalloc(f, t, u_na, s)
    torch.cuda.synchronize()
    return u_na.cpu().numpy(), u_ref.cpu().numpy()


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_equals_solve_two_calls(precision):
    _say("noalloc, precision", precision)
    big = Case(8, 8, 10, 30.0, seed=31, nrhs=5)
    small = Case(4, 2, 7, 12.0, seed=32, nrhs=2)
    fb = big.gpu_build(precision=precision)
    fs = small.gpu_build(precision=precision)
    tol = 1e-13 if precision == 0 else 1e-11
    for cs, f, with_s in [(big, fb, True), (small, fs, True), (small, fs, False), (big, fb, False)]:
        _say("  case", cs.nx, cs.ny, cs.p, "nrhs", cs.t.shape[0], "s" if with_s else "s=0")
        u_na, u_ref = _both(cs, f, with_s)
        assert np.isfinite(u_na).all()
        assert rel(u_na, u_ref) < tol
        u_o = cs.oracle_solve(cs.oracle_build(), s=cs.s if with_s else None)
        assert rel(u_na, u_o) < 1e-10
    fb.free()
    fs.free()


def test_noalloc_refuses_oversized_workspace():
    import torch
    from paper_1812_07167_amd import hps as H
    _say("noalloc oversized")
    cs = Case(32, 32, 16, 40.0, seed=33, nrhs=1)
    f = cs.gpu_build()
    nrhs = 64  # the upward sweep's vectors alone exceed 64 MiB
    t = torch.zeros((nrhs, f.info.n_root), dtype=torch.complex128, device="cuda")
    s = torch.zeros((nrhs, f.info.n_interior), dtype=torch.complex128, device="cuda")
    u = torch.zeros((nrhs, f.info.n_leaf_nodes), dtype=torch.complex128, device="cuda")
    assert f.info.n_leaf_nodes * nrhs * 16 > H.NOALLOC_SCRATCH_BYTES
    with pytest.raises(H.HPSError) as e:
        H.hps_solve_noalloc(f, t, u, s)
    assert e.value.code == H.HPS_E_INVALID
    assert "allocation-free scratch" in str(e.value)
    torch.cuda.synchronize()
    # the refusal leaves the factor and the entry point usable
    cs1 = cs
    u_na, u_ref = _both(cs1, f, True)
    assert rel(u_na, u_ref) < 1e-13
    f.free()
