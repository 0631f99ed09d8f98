"""Mixed precision (complex64 merges and solve products on the FP32 matrix cores, FP64
leaves and top-level interface inverses, FP64 residual correction) against the complex128
oracle.

Bars: the corrected solution meets the complex128 bar (rel. L2 1e-10 against the oracle);
the uncorrected complex64 pieces are checked at a complex64 bar (rel. 1e-4), which also
shows that they are really the reduced-precision ones (rel. > 1e-12)."""

import numpy as np
import pytest

from oracle import hps_oracle as O
from tests.hps_cases import Case, oracle_box_index, perm_to, canonical_keys, rel

pytestmark = pytest.mark.gpu
TOL = 1e-10
C64 = 1e-4


def _mixed(case, **kw):
    from paper_1812_07167_amd import hps as H
    return case.gpu_build(precision=H.HPS_PREC_MIXED, **kw)


@pytest.mark.parametrize("nx,ny,p,kappa,top", [(8, 8, 10, 40.0, 1), (16, 8, 12, 60.0, 3),
                                                (4, 4, 8, 20.0, 0), (8, 8, 16, 80.0, 2)])
def test_mixed_solve_corrected_to_complex128(nx, ny, p, kappa, top):
    case = Case(nx, ny, p, kappa, seed=nx + p, nrhs=3)
    f = _mixed(case, fp64_top_levels=top)
    u = case.gpu_solve(f)
    it, conv, corr = f.last_solve_info()
    assert conv and it >= 1 and corr <= 1e-12
    assert rel(u, case.oracle_solve(case.oracle_build())) < TOL
    f.free()


def test_uncorrected_mixed_solve_is_complex64_accurate():
    case = Case(8, 8, 12, 50.0, seed=3, nrhs=2)
    f = _mixed(case, fp64_top_levels=1, refine_max_iter=0)
    u = case.gpu_solve(f)
    e = rel(u, case.oracle_solve(case.oracle_build()))
    assert 1e-12 < e < C64
    f.free()


def test_mixed_merge_operators_complex64_accurate():
    """Operators of a complex64 level against the oracle's (every box of the level)."""
    from paper_1812_07167_amd import hps as H
    case = Case(4, 4, 8, 20.0, seed=5, nrhs=1)
    boxes = case.oracle_build()
    idx = oracle_box_index(boxes)
    f = _mixed(case, fp64_top_levels=1, keep_all_R=True)
    m = case.m
    for level in (1, 2, 3):
        for q in range(1 << level):
            ix0, ix1, iy0, iy1 = f.box(level, q)
            b = idx[(ix0, ix1, iy0, iy1)]
            keys = canonical_keys(ix0, ix1, iy0, iy1, m)
            P = perm_to(b.keys, keys)
            Rg = f.get(H.OP_R, level, q)
            Ro = b.ops["R"][np.ix_(P, P)]
            e = rel(Rg, Ro)
            assert e < C64, (level, q, e)
            assert e > 1e-12, (level, q, e)
    f.free()


def test_mixed_with_s_null_and_plane_wave():
    """s = NULL (downward sweep only) is corrected too; plane-wave closed form."""
    case = Case(8, 8, 12, 30.0, c="one", seed=2, nrhs=2, rhs="planewave")
    f = _mixed(case)
    u = case.gpu_solve(f, s=None)
    assert rel(u, case.oracle_solve(case.oracle_build(), s=None)) < TOL
    assert rel(u, case.exact) < 1e-7  # discretization error of p = 12, kappa h = 3.75
    f.free()
