"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on identical
seeded inputs.  Complex128 bar: relative L2 error <= 1e-10 on u and on every stored
operator (the stated tolerance for complex128)."""

import sys

import numpy as np
import pytest

from oracle import hps_oracle as O
from tests.hps_cases import Case, canonical_keys, oracle_box_index, perm_to, rel

pytestmark = pytest.mark.gpu

TOL = 1e-10


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


# ---------------------------------------------------------------- leaf operators (Sec. 2.1)


@pytest.mark.parametrize("nx,ny,p", [(2, 2, 4), (2, 1, 8), (2, 2, 9), (1, 1, 11), (2, 2, 12),
                                     (1, 2, 13), (2, 1, 14), (1, 2, 15), (2, 2, 16)])
def test_leaf_operators(nx, ny, p):
    from paper_1812_07167_amd import hps as H
    _say("leaf operators", nx, ny, p)
    cs = Case(nx, ny, p, 17.0, eta=17.0 + 2.0j, box=(0.0, 0.5, -0.25, 0.25), seed=p)
    f = cs.gpu_build(keep_all_R=True)
    L = f.info.levels
    for h in range(nx * ny):
        ix0, ix1, iy0, iy1 = f.box(L, h)
        g = iy0 * nx + ix0
        o = O.leaf_operators(*cs.prob.leaf_box(ix0, iy0), p, cs.kappa, cs.eta,
                             cs.c[g * (p - 2) ** 2:(g + 1) * (p - 2) ** 2])
        assert rel(f.get(H.OP_PSI, L, h), o["Psi"]) < TOL
        assert rel(f.get(H.OP_Y, L, h), o["Y"]) < TOL
        assert rel(f.get(H.OP_R, L, h), o["R"]) < TOL
    f.free()


def _leaf_route_taken(f):
    """'dirichlet' or 'impedance': the leaf kernels that ran in a profiled build."""
    names = {r[0].split("[")[0] for r in f.stage_times(0)}
    if "leaf_ainv" in names and "leaf_sinv" not in names:
        return "dirichlet"
    if "leaf_sinv" in names and "leaf_ainv" not in names:
        return "impedance"
    return "both"


@pytest.mark.parametrize("nx,ny,p", [(2, 2, 4), (2, 1, 5), (1, 2, 7), (2, 1, 8), (2, 2, 9),
                                     (2, 2, 10), (2, 2, 11), (2, 2, 12), (1, 2, 13),
                                     (2, 1, 14), (1, 2, 15), (2, 2, 16)])
def test_leaf_operators_dirichlet_route(nx, ny, p):
    """Leaves well inside a wavelength (kappa^2 max c below half the leaf's smallest
    Dirichlet eigenvalue): the automatic choice inverts the real interior block and
    eliminates the boundary afterwards.  Psi, Y and R against the oracle's dense B^{-1},
    and against the impedance-row elimination of the same leaves."""
    from paper_1812_07167_amd import hps as H
    _say("leaf operators, Dirichlet route", nx, ny, p)
    cs = Case(nx, ny, p, 6.0, eta=6.0 + 1.5j, box=(0.0, 0.5, -0.25, 0.25), seed=p)
    f = cs.gpu_build(keep_all_R=True, profile=True)
    assert _leaf_route_taken(f) == "dirichlet"
    fi = cs.gpu_build(keep_all_R=True, profile=True, leaf_route=1)
    assert _leaf_route_taken(fi) == "impedance"
    L = f.info.levels
    for h in range(nx * ny):
        ix0, ix1, iy0, iy1 = f.box(L, h)
        g = iy0 * nx + ix0
        o = O.leaf_operators(*cs.prob.leaf_box(ix0, iy0), p, cs.kappa, cs.eta,
                             cs.c[g * (p - 2) ** 2:(g + 1) * (p - 2) ** 2])
        for what, key in [(H.OP_PSI, "Psi"), (H.OP_Y, "Y"), (H.OP_R, "R")]:
            a = f.get(what, L, h)
            assert rel(a, o[key]) < TOL, (h, key)
            assert rel(a, fi.get(what, L, h)) < TOL, (h, key)
    u = cs.gpu_solve(f)
    assert rel(u, cs.oracle_solve(cs.oracle_build())) < TOL
    f.free()
    fi.free()


def test_leaf_routes_mixed_in_one_batch():
    """Problems of one shape built together, some below the Dirichlet-route bound (kappa
    3, 6) and some above it (kappa 40, 70): each problem takes its own route within the
    same launches, and every one matches the oracle; complex128 and mixed precision."""
    import torch
    from paper_1812_07167_amd import hps as H
    _say("leaf routes mixed in one batch")
    kappas = [3.0, 40.0, 6.0, 70.0]
    cases = [Case(4, 4, 10, k, seed=40 + i, nrhs=2) for i, k in enumerate(kappas)]
    for precision in (0, 1):
        doms = [H.domain(4, 4) for _ in cases]
        cs_d = [torch.tensor(cs.c, dtype=torch.float64, device="cuda") for cs in cases]
        fs = H.hps_build_batch(doms, [10] * 4, kappas, kappas, cs_d, precision=precision,
                               profile=True)
        assert _leaf_route_taken(fs[0]) == "both"
        for cs, f in zip(cases, fs):
            assert rel(cs.gpu_solve(f), cs.oracle_solve(cs.oracle_build())) < TOL
        for f in fs:
            f.free()


# ---------------------------------------------------------------- merge operators (Sec. 2.2)


# interface sizes n3: (4,4,8) 6..24; (8,8,5) 3..24; (8,8,11) 9, 18, 36, 72 (every width of
# the register-resident inverse, and the blocked ones with a ragged last block); (8,8,16)
# up to 112 and (4,8,14) up to 96 (two diagonal blocks of the block-pivot form); each
# with pivots on the diagonal blocks (0) and over whole columns (1)
@pytest.mark.parametrize("pivoting", [0, 1])
@pytest.mark.parametrize("nx,ny,p,kappa", [(4, 4, 8, 20.0), (4, 2, 6, 9.0), (2, 4, 10, 14.0),
                                           (8, 8, 5, 30.0), (8, 8, 11, 22.0), (8, 8, 16, 45.0),
                                           (4, 8, 14, 60.0)])
def test_merge_operators_every_level(nx, ny, p, kappa, pivoting):
    from paper_1812_07167_amd import hps as H
    _say("merge operators", nx, ny, p, "pivoting", pivoting)
    cs = Case(nx, ny, p, kappa, seed=3)
    boxes = cs.oracle_build()
    ob = oracle_box_index(boxes)
    f = cs.gpu_build(keep_all_R=True, interface_pivoting=pivoting)
    m = p - 2
    for l in range(f.info.levels + 1):
        for q in range(1 << l):
            geo = f.box(l, q)
            b = ob[geo]
            ck = canonical_keys(*geo, m)
            P = perm_to(b.keys, ck)
            assert rel(f.get(H.OP_R, l, q), b.ops["R"][np.ix_(P, P)]) < TOL, (l, q)
            if b.is_leaf:
                continue
            o = b.ops
            a, c = b.children
            ka = canonical_keys(a.ix0, a.ix1, a.iy0, a.iy1, m)
            setb = set(c.keys)
            lib_i3 = [k for k in ka if k in setb]
            lib_i1 = [k for k in ka if k not in setb]
            kb = canonical_keys(c.ix0, c.ix1, c.iy0, c.iy1, m)
            lib_i2 = [k for k in kb if k not in set(a.keys)]
            or_i3 = [a.keys[i] for i in o["i3a"]]
            or_i1 = [a.keys[i] for i in o["i1"]]
            or_i2 = [c.keys[i] for i in o["i2"]]
            P3, P1, P2 = perm_to(or_i3, lib_i3), perm_to(or_i1, lib_i1), perm_to(or_i2, lib_i2)
            Pp = perm_to(o["keys"], ck)
            assert rel(f.get(H.OP_WINV, l, q), o["Winv"][np.ix_(P3, P3)]) < TOL
            assert rel(f.get(H.OP_R33A, l, q), o["R33a"][np.ix_(P3, P3)]) < TOL
            assert rel(f.get(H.OP_R33B, l, q), o["R33b"][np.ix_(P3, P3)]) < TOL
            assert rel(f.get(H.OP_R13A, l, q), o["R13a"][np.ix_(P1, P3)]) < TOL
            assert rel(f.get(H.OP_R23B, l, q), o["R23b"][np.ix_(P2, P3)]) < TOL
            assert rel(f.get(H.OP_PHI_A, l, q), o["Phi_a"][np.ix_(P3, Pp)]) < TOL
            assert rel(f.get(H.OP_PHI_B, l, q), o["Phi_b"][np.ix_(P3, Pp)]) < TOL
    f.free()


# ---------------------------------------------------------------- full build + solve (Alg. 1-2)


@pytest.mark.parametrize("nx,ny,p,kappa,eta,box,nrhs", [
    (4, 4, 8, 20.0, 20.0, (0.0, 1.0, 0.0, 1.0), 2),
    (2, 1, 6, 5.0, 5.0, (0.0, 1.0, 0.0, 1.0), 1),
    (1, 2, 7, 5.0, 2.0 - 1.0j, (0.0, 1.0, 0.0, 2.0), 3),
    (4, 2, 6, 12.0, 12.0 + 3.0j, (-1.0, 1.0, 0.0, 0.5), 17),
    (2, 8, 5, 8.0, 8.0, (0.0, 0.5, 0.0, 2.0), 4),
    (1, 1, 9, 10.0, 10.0, (0.0, 1.0, 0.0, 1.0), 2),
    (8, 4, 12, 25.0, 25.0, (0.0, 1.0, 0.0, 0.5), 5),
])
def test_solve_random_rhs(nx, ny, p, kappa, eta, box, nrhs):
    _say("solve", nx, ny, p, nrhs)
    cs = Case(nx, ny, p, kappa, eta=eta, box=box, nrhs=nrhs, seed=nx + 7 * ny)
    u_o = cs.oracle_solve(cs.oracle_build())
    f = cs.gpu_build()
    u_g = cs.gpu_solve(f)
    assert rel(u_g, u_o) < TOL
    # body load zero: s = NULL skips the upward pass (Sec. 2) and equals s = 0
    u0 = cs.gpu_solve(f, s=None)
    uz = cs.gpu_solve(f, s=np.zeros_like(cs.s))
    assert rel(u0, uz) < 1e-13
    assert rel(u0, cs.oracle_solve(cs.oracle_build(), s=None)) < TOL
    f.free()


@pytest.mark.parametrize("nx,ny,p,kappa,seed", [(4, 4, 8, 17.0, 8), (8, 8, 8, 80.0, 1),
                                                 (8, 8, 12, 80.0, 2), (8, 8, 16, 80.0, 3),
                                                 (4, 8, 14, 60.0, 4), (8, 4, 15, 70.0, 5)])
def test_leaves_of_several_wavelengths(nx, ny, p, kappa, seed):
    """Leaves of a few wavelengths (kappa h up to 10 with c in [0.5, 1.5]): kappa^2 c
    crosses eigenvalues of the leaves' Dirichlet Laplacian, where a leaf's interior
    block alone is (nearly) singular; the impedance rows keep the leaf system well
    posed and the GPU path must still match the oracle.  Covers the register-resident
    (p <= 13) and the scratch-copy (p >= 14) leaf inverses."""
    _say("several wavelengths", nx, ny, p, kappa)
    cs = Case(nx, ny, p, kappa, seed=seed, nrhs=2)
    f = cs.gpu_build()
    assert rel(cs.gpu_solve(f), cs.oracle_solve(cs.oracle_build())) < TOL
    f.free()


def test_config1_plane_wave():
    """4x4 leaves, p = 8, kappa = eta = 20, c = 1, s = 0, plane wave with seeded angle."""
    _say("config 1")
    cs = Case(4, 4, 8, 20.0, c="one", rhs="planewave", nrhs=1, seed=0)
    u_o = cs.oracle_solve(cs.oracle_build())
    f = cs.gpu_build()
    u_g = cs.gpu_solve(f)
    assert rel(u_g, u_o) < TOL
    e_o, e_g = rel(u_o, cs.exact), rel(u_g, cs.exact)
    assert abs(e_g - e_o) < 1e-8 * max(e_o, 1e-12) + 1e-12
    assert e_g < 1e-3
    f.free()


def test_medium_manufactured_vs_oracle():
    """16 x 16 leaves at p = 16 (several GEMM tiles, ragged tails, blocked inversion at
    the top: n3 = 224), manufactured solution, 4 right-hand sides."""
    _say("medium 16x16 p16")
    cs = Case(16, 16, 16, 40.0, c="bump", rhs="manufactured", nrhs=4, seed=5)
    u_o = cs.oracle_solve(cs.oracle_build())
    f = cs.gpu_build()
    u_g = cs.gpu_solve(f)
    assert rel(u_g, u_o) < TOL
    assert rel(u_g, cs.exact) < 1e-8
    f.free()


def test_merge_order_independence_of_gpu_result():
    """The GPU result (x-first splits) equals the oracle built with y-first splits."""
    cs = Case(4, 4, 9, 15.0, seed=9)
    u_y = cs.oracle_solve(cs.oracle_build(tie="y"))
    f = cs.gpu_build()
    assert rel(cs.gpu_solve(f), u_y) < TOL
    f.free()


def test_shared_edge_nodes_agree_gpu():
    cs = Case(8, 8, 8, 22.0, seed=4, nrhs=1)
    f = cs.gpu_build()
    u = cs.gpu_solve(f)[0].reshape(64, cs.prob.n)
    m = cs.m
    seen, worst = {}, 0.0
    for iy in range(8):
        for ix in range(8):
            for r, k in enumerate(O.leaf_boundary_keys(ix, iy, m)):
                v = u[iy * 8 + ix, r]
                if k in seen:
                    worst = max(worst, abs(v - seen[k]))
                seen[k] = v
    assert worst < 1e-11 * np.abs(u).max()
    f.free()


def test_linearity_gpu():
    cs = Case(4, 4, 7, 11.0, seed=2, nrhs=2)
    f = cs.gpu_build()
    u = cs.gpu_solve(f)
    a, b = 0.5 - 2.0j, 1.5
    cs2 = Case(4, 4, 7, 11.0, seed=2, nrhs=2)
    cs2.s = a * cs.s[:1] + b * cs.s[1:]
    cs2.t = a * cs.t[:1] + b * cs.t[1:]
    ul = cs2.gpu_solve(f)
    assert rel(ul[0], a * u[0] + b * u[1]) < 1e-12
    f.free()


# ---------------------------------------------------------------- full size (64 x 64, p = 16)


@pytest.fixture(scope="module")
def config2():
    from paper_1812_07167_amd import hps as H
    _say("config 2 build (64x64 leaves, p=16, kappa=100)")
    cs = Case(64, 64, 16, 100.0, c="bump", rhs="polynomial", nrhs=2, seed=1)
    f = cs.gpu_build()
    yield cs, f
    f.free()


def test_config2_polynomial_reproduction(config2):
    """Exact result at full size: a polynomial of tensor degree <= 6 satisfies the
    discrete system exactly, so every level, both sweeps and all leaves must return its
    nodal values to round-off."""
    cs, f = config2
    u = cs.gpu_solve(f)
    _say("config2 poly rel", rel(u, cs.exact))
    assert rel(u, cs.exact) < 1e-10


def test_config2_sampled_leaves(config2):
    from paper_1812_07167_amd import hps as H
    cs, f = config2
    rng = np.random.default_rng(0)
    p = cs.p
    L = f.info.levels
    for h in rng.choice(f.info.nleaf, size=6, replace=False):
        ix0, ix1, iy0, iy1 = f.box(L, int(h))
        g = iy0 * cs.nx + ix0
        o = O.leaf_operators(*cs.prob.leaf_box(ix0, iy0), p, cs.kappa, cs.eta,
                             cs.c[g * (p - 2) ** 2:(g + 1) * (p - 2) ** 2])
        assert rel(f.get(H.OP_PSI, L, int(h)), o["Psi"]) < TOL
        assert rel(f.get(H.OP_Y, L, int(h)), o["Y"]) < TOL


@pytest.mark.parametrize("nrhs", [1, 16, 20, 37, 64, 70, 131])
@pytest.mark.parametrize("precision", [0, 1])
def test_many_right_hand_sides_in_ragged_passes(precision, nrhs):
    """The solve products take up to 64 right-hand sides per pass, in one, two or four
    16-column blocks (1, 16: one block; 20: two; 37, 64: four; 70 = 64 + 6 and
    131 = 64 + 64 + 3: several passes with a ragged tail), the paired launches of both
    sweeps included, with and without a body load, against the oracle."""
    _say(nrhs, "RHS, precision", precision)
    cs = Case(8, 8, 10, 30.0, seed=21, nrhs=nrhs)
    f = cs.gpu_build(precision=precision)
    boxes = cs.oracle_build()
    assert rel(cs.gpu_solve(f), cs.oracle_solve(boxes)) < TOL
    assert rel(cs.gpu_solve(f, s=None), cs.oracle_solve(boxes, s=None)) < TOL
    f.free()


def test_large_interfaces_polynomial_reproduction():
    """128 x 128 leaves at p = 16: the top interface (n = 1792) takes the blocked
    inverse's panels of two rows per lane over 16 waves, the next ones (n = 896) over 8;
    the polynomial must still come back to round-off."""
    _say("128x128 leaves, p=16, polynomial")
    cs = Case(128, 128, 16, 100.0, c="bump", rhs="polynomial", nrhs=1, seed=2)
    f = cs.gpu_build()
    u = cs.gpu_solve(f)
    f.free()
    _say("128x128 poly rel", rel(u, cs.exact))
    assert rel(u, cs.exact) < 1e-10


def test_largest_leaf_grid_polynomial_reproduction():
    """256 x 256 leaves (2^16, the most a domain takes) at p = 4: the leaf sweeps of the
    solve cover 65536 leaves, more than one launch's grid y extent, and run in slices;
    a polynomial of degree 3 must come back to round-off."""
    _say("256x256 leaves, p=4, polynomial")
    cs = Case(256, 256, 4, 3.0, rhs="polynomial", nrhs=2, seed=3)
    f = cs.gpu_build()
    u = cs.gpu_solve(f)
    _say("256x256 poly rel", rel(u, cs.exact))
    assert rel(u, cs.exact) < 1e-9
    f.free()


def test_config2_manufactured_solution(config2):
    cs, f = config2
    mf = Case(64, 64, 16, 100.0, c="bump", rhs="manufactured", nrhs=3, seed=11)
    u = mf.gpu_solve(f)
    err = rel(u, mf.exact)
    _say("config2 manufactured rel err", err)
    assert err < 1e-9
