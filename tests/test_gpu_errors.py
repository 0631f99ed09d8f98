"""Error paths and lifetimes on the device.  A coefficient that is not a number leaves
a leaf's interior matrix without a usable pivot: the build reports
HPS_E_SINGULAR (every kernel takes its own exit; the pivot checks run after the build's
one synchronization), hands back no factor, and the library keeps working.  A factor
keeps the shared plan of its shape alive after the plan cache has let it go."""

import numpy as np
import pytest

from tests.hps_cases import Case, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("p,node", [(8, 5), (16, 100)])
def test_nan_coefficient_is_a_singular_leaf(p, node):
    import torch
    from paper_1812_07167_amd import hps as H
    case = Case(4, 4, p, 20.0, seed=p, nrhs=1)
    c = np.array(case.c, dtype=np.float64)
    c[node] = np.nan
    dom = H.domain(case.nx, case.ny, case.box)
    cd = torch.tensor(c, dtype=torch.float64, device="cuda")
    with pytest.raises(H.HPSError) as e:
        H.hps_build(dom, case.p, case.kappa, case.eta, cd)
    assert e.value.code == H.HPS_E_SINGULAR
    assert "leaf interior" in str(e.value)
    # a clean build afterwards is unaffected
    f = case.gpu_build()
    assert rel(case.gpu_solve(f), case.oracle_solve(case.oracle_build())) < 1e-10
    f.free()


def test_factor_outlives_its_cached_plan():
    """The tree and index maps of a shape are shared through a cache of 32 shapes: a
    factor whose shape was evicted (33 other shapes planned since) or dropped by
    hps_release_cached still solves correctly, and its shape plans again on demand."""
    import torch
    from paper_1812_07167_amd import hps as H
    case = Case(4, 2, 10, 18.0, seed=21, nrhs=2)
    f = case.gpu_build()
    ref = case.oracle_solve(case.oracle_build())
    shapes = [(nx, ny, p) for p in (4, 5, 6, 7, 8, 9) for (nx, ny) in
              ((1, 1), (2, 1), (1, 2), (2, 2), (4, 1), (1, 4))][:33]
    for nx, ny, p in shapes:
        dom = H.domain(nx, ny)
        c = torch.ones(nx * ny * (p - 2) ** 2, dtype=torch.float64, device="cuda")
        H.hps_build(dom, p, 5.0, 5.0, c).free()
    H.hps_release_cached()
    assert rel(case.gpu_solve(f), ref) < 1e-10
    f.free()
    g = case.gpu_build()
    assert rel(case.gpu_solve(g), ref) < 1e-10
    g.free()
