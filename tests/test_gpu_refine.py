"""GPU parity of the residual-correction path against the oracle: the FP64 residual of
the global collocation system, the solve with right-hand sides on the shared-edge rows
(interface jumps), and the correction loop.  Tolerance: rel. L2 1e-10 (complex128)."""

import numpy as np
import pytest

from oracle import hps_oracle as O
from tests.hps_cases import Case, rel

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _dev(a, dtype="complex128"):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=getattr(torch, dtype), device="cuda")


def _jumps(case, seed):
    rng = np.random.default_rng(seed)
    nb = case.prob.nb
    sh = (case.t.shape[0], case.prob.nleaf, nb)
    return rng.standard_normal(sh) + 1j * rng.standard_normal(sh)


@pytest.mark.parametrize("nx,ny,p,eta", [(2, 2, 6, None), (4, 2, 7, 5.0 - 3.0j), (2, 4, 16, None),
                                          (1, 1, 8, None), (8, 8, 12, None)])
def test_residual_matches_oracle(nx, ny, p, eta):
    from paper_1812_07167_amd import hps as H
    case = Case(nx, ny, p, 13.0, eta=eta, seed=nx * 10 + p, nrhs=3)
    rng = np.random.default_rng(p)
    u = rng.standard_normal((3, case.prob.nleaf * case.prob.n)) * (1 + 1j)
    u = u + 1j * rng.standard_normal(u.shape)
    j = _jumps(case, p)
    f = case.gpu_build()
    r = H.hps_residual(f, _dev(u), t=_dev(case.t), s=_dev(case.s), jumps=_dev(j))
    ro = O.global_residual(case.prob, case.c, case.s, case.t, u, jumps=j).reshape(3, -1)
    assert rel(r.cpu().numpy(), ro) < 1e-12
    f.free()


@pytest.mark.parametrize("nx,ny,p", [(2, 2, 6), (4, 4, 8), (2, 8, 10), (8, 4, 16)])
def test_jump_solve_matches_oracle(nx, ny, p):
    import torch
    from paper_1812_07167_amd import hps as H
    case = Case(nx, ny, p, 17.0, seed=p, nrhs=2)
    j = _jumps(case, 100 + p)
    f = case.gpu_build()
    u = H.hps_solve_jumps(f, _dev(case.t), _dev(case.s), _dev(j))
    torch.cuda.synchronize()
    uo = O.solve(case.prob, case.oracle_build(), case.s, case.t, jumps=j)
    assert rel(u.cpu().numpy(), uo) < TOL
    # jumps alone (s = NULL) run the upward pass too
    u0 = H.hps_solve_jumps(f, _dev(np.zeros_like(case.t)), None, _dev(j))
    uo0 = O.solve(case.prob, case.oracle_build(), None, np.zeros_like(case.t), jumps=j)
    assert rel(u0.cpu().numpy(), uo0) < TOL
    f.free()


def test_jump_solve_equals_dense_global_solve():
    import torch
    from paper_1812_07167_amd import hps as H
    case = Case(2, 4, 7, 9.0, eta=6.0 + 1.0j, seed=4, nrhs=2)
    j = _jumps(case, 8)
    f = case.gpu_build()
    u = H.hps_solve_jumps(f, _dev(case.t), _dev(case.s), _dev(j))
    torch.cuda.synchronize()
    ug = O.global_solve(case.prob, case.c, case.s, case.t, jumps=j)
    assert rel(u.cpu().numpy(), ug) < TOL
    f.free()


def test_fp64_correction_loop_converges_and_matches_oracle():
    """With correction on in complex128 the first step already meets the tolerance (the
    factorization is exact to round-off) and u still equals the oracle."""
    case = Case(8, 8, 10, 30.0, seed=5, nrhs=3)
    f = case.gpu_build(refine_max_iter=3, refine_tol=1e-11)
    u = case.gpu_solve(f)
    it, conv, corr = f.last_solve_info()
    assert conv and 1 <= it <= 2 and corr < 1e-11
    assert rel(u, case.oracle_solve(case.oracle_build())) < TOL
    f.free()


def test_residual_of_gpu_solution_is_roundoff():
    from paper_1812_07167_amd import hps as H
    case = Case(16, 16, 12, 40.0, seed=6, nrhs=2, rhs="manufactured")
    f = case.gpu_build()
    u = case.gpu_solve(f)
    r = H.hps_residual(f, _dev(u), t=_dev(case.t), s=_dev(case.s)).cpu().numpy()
    b = O.global_rhs(case.prob, case.s, case.t)
    assert np.linalg.norm(r) < 1e-10 * np.linalg.norm(b)
    f.free()
