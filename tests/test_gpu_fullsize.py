"""GPU parity at the benchmark's full size, against the oracle run on the same inputs.

The benchmark workload itself: Omega = [0,1]^2 in 64 x 64 leaves, p = 16, kappa = eta =
100, c = 1 - 0.5 exp(-160 |x - (1/2, 1/2)|^2), and the benchmark's 16 manufactured
right-hand sides u = e^{i kappa d.x}(1 + 0.1 sin 2 pi x sin 2 pi y) (directions from seed
0).  The solution u of all 16 right-hand sides, the stored top-level interface operators
W^{-1}, Phi^a and Phi^b (interfaces of 896 and 448 nodes, the blocked inverse's widest
shapes at this size), and the mixed-precision solve after FP64 correction are compared
entry by entry with the oracle (relative L2 <= 1e-10, the complex128 bar).  Both sides'
errors against the closed form are reported as relative L2 and as the paper's e_inf
(Sec. 4.1).

A second case reaches an interface of more than 1024 nodes at the root (128 x 128 leaves
at p = 11: 1152 nodes), compared the same way.

The oracle needs minutes of host time here; its progress goes straight to the terminal
(past pytest's capture) after every tree level.
"""

import sys
import time

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


def _sayer(request):
    capman = request.config.pluginmanager.getplugin("capturemanager")

    def say(*a):
        if capman is not None:
            with capman.global_and_fixture_disabled():
                print(*a, flush=True)
        else:
            print(*a, flush=True)
        sys.stdout.flush()
    return say


def _oracle(cs, say, tag):
    t0 = time.time()
    boxes = cs.oracle_build(progress=lambda lev, nb: say(
        "  oracle %s: level %d (%d boxes) done, %.0f s" % (tag, lev, nb, time.time() - t0)))
    u = cs.oracle_solve(boxes)
    say("  oracle %s: solve done, %.0f s" % (tag, time.time() - t0))
    return boxes, u


def _interface_ops(H, f, b, level, q, m):
    """GPU and oracle W^{-1}, Phi^a, Phi^b of merge q on level `level`, in one order."""
    geo = f.box(level, q)
    o = b.ops
    a, c = b.children
    ka = canonical_keys(a.ix0, a.ix1, a.iy0, a.iy1, m)
    setb = set(c.keys)
    lib_i3 = [k for k in ka if k in setb]
    or_i3 = [a.keys[i] for i in o["i3a"]]
    P3 = perm_to(or_i3, lib_i3)
    Pp = perm_to(o["keys"], canonical_keys(*geo, m))
    return [("Winv", f.get(H.OP_WINV, level, q), o["Winv"][np.ix_(P3, P3)]),
            ("Phi_a", f.get(H.OP_PHI_A, level, q), o["Phi_a"][np.ix_(P3, Pp)]),
            ("Phi_b", f.get(H.OP_PHI_B, level, q), o["Phi_b"][np.ix_(P3, Pp)])]


@pytest.fixture(scope="module")
def config2(request):
    say = _sayer(request)
    say("\nfull size: 64x64 leaves, p=16, kappa=eta=100, 16 manufactured RHS")
    cs = Case(64, 64, 16, 100.0, c="bump", rhs="manufactured", nrhs=16, seed=0)
    f = cs.gpu_build()
    u_g = cs.gpu_solve(f)
    say("  GPU complex128 build + solve done")
    fm = cs.gpu_build(precision=1)
    u_m = cs.gpu_solve(fm)
    info = fm.last_solve_info()
    fm.free()
    say("  GPU mixed build + corrected solve done")
    boxes, u_o = _oracle(cs, say, "64x64")
    yield cs, f, boxes, u_g, u_m, info, u_o, say
    f.free()


def test_config2_solution_vs_oracle(config2):
    cs, f, boxes, u_g, u_m, info, u_o, say = config2
    r = rel(u_g, u_o)
    say("  u: GPU vs oracle rel L2 %.3e, max |diff| %.3e (max |u| %.3e); vs closed form: "
        "GPU rel L2 %.3e e_inf %.3e, oracle rel L2 %.3e e_inf %.3e"
        % (r, O.e_inf(u_g, u_o), np.abs(u_o).max(), rel(u_g, cs.exact), O.e_inf(u_g, cs.exact),
           rel(u_o, cs.exact), O.e_inf(u_o, cs.exact)))
    assert r < TOL
    for k in range(u_g.shape[0]):  # every right-hand side on its own
        assert rel(u_g[k], u_o[k]) < TOL, k


def test_config2_top_interface_operators_vs_oracle(config2):
    from paper_1812_07167_amd import hps as H
    cs, f, boxes, u_g, u_m, info, u_o, say = config2
    ob = oracle_box_index(boxes)
    for level in range(3):
        for q in range(1 << level):
            b = ob[f.box(level, q)]
            for name, g, o in _interface_ops(H, f, b, level, q, cs.m):
                r = rel(g, o)
                say("  level %d box %d %s (%d x %d): rel %.3e" % (level, q, name, *g.shape, r))
                assert r < TOL, (level, q, name)


def test_config2_mixed_precision_vs_oracle(config2):
    cs, f, boxes, u_g, u_m, info, u_o, say = config2
    r = rel(u_m, u_o)
    iters, converged, corr = info
    say("  mixed: %d correction steps, last relative correction %.2e, vs oracle rel L2 %.3e, "
        "e_inf vs closed form %.3e" % (iters, corr, r, O.e_inf(u_m, cs.exact)))
    assert converged
    assert r < TOL


def test_root_interface_above_1024_nodes(request):
    """128 x 128 leaves at p = 11: the root interface has 1152 nodes."""
    from paper_1812_07167_amd import hps as H
    say = _sayer(request)
    say("\nfull size: 128x128 leaves, p=11, kappa=eta=60, 2 RHS")
    cs = Case(128, 128, 11, 60.0, seed=12, nrhs=2)
    f = cs.gpu_build()
    u_g = cs.gpu_solve(f)
    fp = cs.gpu_build(interface_pivoting=1)
    u_p = cs.gpu_solve(fp)
    fp.free()
    say("  GPU build + solve done (diagonal-block and whole-column pivots)")
    boxes, u_o = _oracle(cs, say, "128x128")
    say("  u: whole-column vs diagonal-block pivots rel L2 %.3e" % rel(u_p, u_g))
    assert rel(u_p, u_o) < TOL
    r = rel(u_g, u_o)
    say("  u: GPU vs oracle rel L2 %.3e" % r)
    assert r < TOL
    ob = oracle_box_index(boxes)
    for level, q in [(0, 0), (1, 0), (1, 1)]:
        b = ob[f.box(level, q)]
        for name, g, o in _interface_ops(H, f, b, level, q, cs.m):
            rr = rel(g, o)
            say("  level %d box %d %s (%d x %d): rel %.3e" % (level, q, name, *g.shape, rr))
            assert rr < TOL, (level, q, name)
    f.free()
