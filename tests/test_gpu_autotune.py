"""The GEMM autotuner: a build with autotune on records a tile variant per merge GEMM
shape, and factorizations built with the tuned variants solve to the same result as the
default variants (rel. 1e-12) and as the oracle (rel. 1e-10)."""

import pytest

from tests.hps_cases import Case, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nx,ny,p,prec", [(8, 8, 10, 0), (16, 8, 8, 1), (4, 4, 12, 0)])
def test_tuned_build_matches_default_and_oracle(nx, ny, p, prec):
    from paper_1812_07167_amd import hps as H
    case = Case(nx, ny, p, 25.0, seed=nx + p, nrhs=2)
    H.autotune_clear()
    f0 = case.gpu_build(precision=prec)
    u0 = case.gpu_solve(f0)
    f0.free()
    f1 = case.gpu_build(precision=prec, autotune=True)
    n = H.autotune_entries()
    assert n >= 2
    u1 = case.gpu_solve(f1)
    f1.free()
    # a later build without the flag launches the recorded variants
    f2 = case.gpu_build(precision=prec)
    u2 = case.gpu_solve(f2)
    f2.free()
    assert H.autotune_entries() == n
    bar = 1e-12 if prec == 0 else 1e-10
    assert rel(u1, u0) < bar and rel(u2, u1) < bar
    assert rel(u1, case.oracle_solve(case.oracle_build())) < 1e-10
    H.autotune_clear()


def test_tuning_table_survives_a_save_and_load(tmp_path):
    from paper_1812_07167_amd import hps as H
    case = Case(8, 8, 8, 20.0, seed=3, nrhs=1)
    H.autotune_clear()
    case.gpu_build(autotune=True).free()
    n = H.autotune_entries()
    H.autotune_save(tmp_path / "tune.txt")
    H.autotune_clear()
    H.autotune_load(tmp_path / "tune.txt")
    assert H.autotune_entries() == n
    f = case.gpu_build()
    assert rel(case.gpu_solve(f), case.oracle_solve(case.oracle_build())) < 1e-10
    f.free()
    H.autotune_clear()
