"""CPU checks of the C-ABI library: it loads, exports every entry point declared in
include/hps.h, its host-side node generator matches the oracle's coordinates exactly,
and argument validation fails cleanly before any device work."""

import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import hps_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hps.h")


def _lib():
    from paper_1812_07167_amd import hps as H
    if not os.path.exists(H.LIB_PATH):
        pytest.skip("libhps.so not built")
    return H, H.load()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hps_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    from paper_1812_07167_amd import hps as H
    assert declared_functions() == sorted(H.EXPORTS)


def test_library_exports_every_declared_symbol():
    H, lib = _lib()
    out = subprocess.run(["nm", "-D", "--defined-only", H.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r" T (hps_\w+)", out))
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(lib, name)


def test_version_and_default_opts():
    H, lib = _lib()
    assert lib.hps_version() >= 10000
    o = H.Opts()
    lib.hps_default_opts(C.byref(o))
    assert o.precision == 0 and o.store_root_R == 1 and o.keep_all_R == 0


@pytest.mark.parametrize("nx,ny,p,box", [(4, 2, 8, (0.0, 1.0, 0.0, 0.5)), (1, 1, 4, (0, 1, 0, 1)),
                                         (2, 8, 16, (-1.0, 2.0, 3.0, 5.0))])
def test_nodes_match_oracle_exactly(nx, ny, p, box):
    H, lib = _lib()
    xy, xyi, xyb, nrm = H.hps_nodes(H.domain(nx, ny, box), p)
    prob = O.Problem(*box, nx, ny, p, 1.0, 1.0)
    np.testing.assert_array_equal(xy, prob.leaf_nodes())
    np.testing.assert_array_equal(xyi, prob.interior_nodes())
    b, n = prob.root_boundary()
    np.testing.assert_array_equal(xyb, b)
    np.testing.assert_array_equal(nrm, n)


@pytest.mark.parametrize("nx,ny,p,kappa,eta,err", [
    (3, 2, 8, 1.0, 1.0, "powers of two"),
    (2, 2, 3, 1.0, 1.0, "p must be"),
    (2, 2, 17, 1.0, 1.0, "p must be"),
    (2, 2, 8, -1.0, 1.0, "kappa"),
    (2, 2, 8, float("nan"), 1.0, "kappa"),
    (2, 2, 8, 1.0, 1.0j, "Re(eta)"),
    (512, 256, 8, 1.0, 1.0, "65536"),
])
def test_build_rejects_invalid_arguments(nx, ny, p, kappa, eta, err):
    H, lib = _lib()
    dom = H.domain(nx, ny)
    out = C.c_void_p(123)
    code = lib.hps_build(C.byref(dom), p, kappa, float(np.real(eta)), float(np.imag(eta)),
                         C.c_void_p(16), None, C.byref(out))
    assert code == H.HPS_E_INVALID
    assert out.value is None
    assert err in lib.hps_last_error().decode()


def test_invalid_domain_bounds_and_nulls():
    H, lib = _lib()
    dom = H.Domain(1.0, 0.0, 0.0, 1.0, 2, 2)
    assert lib.hps_nodes(C.byref(dom), 8, None, None, None, None) == H.HPS_E_INVALID
    dom = H.domain(2, 2)
    out = C.c_void_p()
    assert lib.hps_build(C.byref(dom), 8, 1.0, 1.0, 0.0, None, None, C.byref(out)) == H.HPS_E_INVALID
    assert lib.hps_solve(None, 1, None, None, None) == H.HPS_E_INVALID
    assert lib.hps_nodes(None, 8, None, None, None, None) == H.HPS_E_INVALID
    lib.hps_free(None)  # no-op


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_1812_07167_amd import hps as H
    saved = H._lib
    try:
        H._lib = None
        with pytest.raises(RuntimeError, match="missing"):
            H.load(str(tmp_path / "nope.so"))
    finally:
        H._lib = saved


def _est(H, nx, ny, p, **kw):
    return H.hps_estimate_bytes(H.domain(nx, ny), p, **kw)


def test_estimate_of_a_single_leaf_is_its_operators():
    """One leaf, no merges: [Psi | Y] (n x n complex128), its ItI operator (n_b x n_b,
    kept as the root's), and the small tables (host arithmetic, no device)."""
    H, lib = _lib()
    p = 8
    n, nb, ni = p * p - 4, 4 * (p - 2), (p - 2) ** 2
    peak, res = _est(H, 1, 1, p)
    ops = n * n * 16 + nb * nb * 16
    small = 20 + ni * 8 + 32 * p * p + 32
    assert ops + small < res < ops + small + 16 * 2 * (p * p) * 4  # + the line tables
    assert peak > res


def test_estimate_of_one_merge():
    """2 x 1 leaves: two leaves' [Psi | Y] plus one merge's stored operators (n3 = m
    interface nodes, parent boundary 6m) and the root's ItI operator."""
    H, lib = _lib()
    p = 10
    m = p - 2
    n, n3, n1, nbp = p * p - 4, m, 3 * m, 6 * m
    peak, res = _est(H, 2, 1, p)
    merge = (3 * n3 * n3 + 2 * n1 * n3 + 2 * n3 * nbp) * 16
    core = 2 * n * n * 16 + merge + nbp * nbp * 16
    assert core < res < core + 64 * 1024
    # without the root's R it shrinks by exactly that operator
    _, res0 = _est(H, 2, 1, p, store_root_R=False)
    assert res - res0 == nbp * nbp * 16


def test_estimate_scales_and_orders():
    H, lib = _lib()
    pk1, r1 = _est(H, 32, 32, 12)
    pk2, r2 = _est(H, 64, 32, 12)
    assert 1.9 < r2 / r1 < 2.3 and pk2 > pk1 >= r1
    pkm, rm = _est(H, 32, 32, 12, precision=H.HPS_PREC_MIXED)
    assert rm < r1 and pkm > rm  # complex64 operators; the build stages complex128 leaves
    _, rk = _est(H, 32, 32, 12, keep_all_R=True)
    assert rk > r1


def test_estimate_rejects_invalid_arguments():
    H, lib = _lib()
    dom = H.domain(3, 2)
    pk = C.c_int64()
    assert lib.hps_estimate_bytes(C.byref(dom), 8, None, C.byref(pk), None) == H.HPS_E_INVALID
    dom = H.domain(2, 2)
    assert lib.hps_estimate_bytes(C.byref(dom), 8, None, None, None) == H.HPS_E_INVALID
    assert lib.hps_estimate_bytes(C.byref(dom), 20, None, C.byref(pk), None) == H.HPS_E_INVALID


def test_server_argument_checks_before_device_work():
    H, lib = _lib()
    o = H.ServerOpts()
    lib.hps_server_default_opts(C.byref(o))
    assert (o.slots, o.max_batch_rhs, o.max_pending_builds, o.evict_idle) == (4, 64, 64, 1)
    out = C.c_void_p(123)
    for field, bad in [("slots", 0), ("slots", 17), ("max_batch_rhs", 0), ("max_pending_builds", 0)]:
        b = H.ServerOpts()
        lib.hps_server_default_opts(C.byref(b))
        setattr(b, field, bad)
        assert lib.hps_server_create(1 << 30, C.byref(b), C.byref(out)) == H.HPS_E_INVALID
        assert out.value is None
    assert lib.hps_server_create(1 << 30, None, None) == H.HPS_E_INVALID
    n = C.c_int32()
    assert lib.hps_server_poll(None, None, 0, 0, C.byref(n)) == H.HPS_E_INVALID
    assert lib.hps_server_stats(None, None) == H.HPS_E_INVALID
    req = C.c_uint64()
    assert lib.hps_server_submit_solve(None, 1, 1, None, None, None, C.byref(req)) == H.HPS_E_INVALID
    assert lib.hps_server_release(None, 1) == H.HPS_E_INVALID
    lib.hps_server_destroy(None)  # no-op


def test_autotune_table_roundtrip(tmp_path):
    """The tuning table's text format: load merges lines, save writes them back (sorted by
    shape), clear empties it; malformed files are refused (host only)."""
    H, lib = _lib()
    H.autotune_clear()
    src = tmp_path / "t.txt"
    src.write_text("64 64 64 8 0 128x64\n\n14 84 14 2048 17 16x64\n")
    H.autotune_load(src)
    assert H.autotune_entries() == 2
    out = tmp_path / "o.txt"
    H.autotune_save(out)
    assert out.read_text().splitlines() == ["14 84 14 2048 17 16x64", "64 64 64 8 0 128x64"]
    H.autotune_load(out)  # merging the same shapes adds nothing
    assert H.autotune_entries() == 2
    for bad in ["1 2 3\n", "64 64 64 8 0 99x99\n"]:
        src.write_text(bad)
        with pytest.raises(H.HPSError) as e:
            H.autotune_load(src)
        assert e.value.code == H.HPS_E_INVALID
    assert H.autotune_entries() == 2  # a refused file changes nothing
    with pytest.raises(H.HPSError):
        H.autotune_load(tmp_path / "missing.txt")
    H.autotune_clear()
    assert H.autotune_entries() == 0


def test_allocator_hook_argument_checks():
    """Both functions or neither; a half-set hook is refused and changes nothing (host)."""
    H, lib = _lib()
    assert lib.hps_set_allocator(H.ALLOC_FN(lambda n, s, c: None), H.FREE_FN(), None) == H.HPS_E_INVALID
    assert "both" in lib.hps_last_error().decode()
    assert lib.hps_set_allocator(H.ALLOC_FN(), H.FREE_FN(lambda p, s, c: None), None) == H.HPS_E_INVALID
    assert lib.hps_set_allocator(H.ALLOC_FN(), H.FREE_FN(), None) == H.HPS_OK
    with pytest.raises(ValueError):
        H.set_allocator(lambda n, s: 0)
    H.set_allocator()


def test_bench_refuses_more_than_one_gpu():
    """bench.py has no multi-GPU path: --gpus above 1 exits with a message, before any
    device work."""
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
