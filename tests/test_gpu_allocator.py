"""The allocator hook (hps_set_allocator): with torch's caching allocator installed, every
device buffer of a build, a solve and the request loop comes from torch and goes back to
it, and results equal those under the library's own allocator (same kernels, same
order: rel. 1e-14)."""

import numpy as np
import pytest

from tests.hps_cases import Case, rel

pytestmark = pytest.mark.gpu
SAME = 1e-14


class Counting:
    """torch's caching allocator behind a ledger of the library's live buffers."""

    def __init__(self):
        import torch
        self.torch = torch
        self.dev = torch.cuda.current_device()
        self.live = {}
        self.allocs = 0
        self.streams = set()

    def alloc(self, n, st):
        p = self.torch.cuda.caching_allocator_alloc(n, self.dev, st)
        self.live[p] = n
        self.allocs += 1
        self.streams.add(st)
        return p

    def free(self, p, st):
        assert p in self.live, "freed memory the hook did not provide"
        del self.live[p]
        self.torch.cuda.caching_allocator_delete(p)


def _solve(case, f):
    import torch
    u = case.gpu_solve(f)
    torch.cuda.synchronize()
    return u


def test_build_and_solve_through_torch_allocator():
    import torch
    from paper_1812_07167_amd import hps as H
    case = Case(16, 8, 10, 30.0, seed=11, nrhs=3)
    f0 = case.gpu_build()
    u0 = _solve(case, f0)
    bytes0 = f0.info.device_bytes
    f0.free()
    hook = Counting()
    H.set_allocator(hook.alloc, hook.free)
    try:
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        f1 = case.gpu_build()
        held = torch.cuda.memory_allocated() - base
        u1 = _solve(case, f1)
        assert hook.allocs > 0 and 0 in hook.streams  # long-lived buffers: stream NULL
        # the factor's own buffers; the index maps of its shape are shared with the
        # earlier build of the same shape (plan cache) and were allocated then
        assert bytes0 - (1 << 20) <= held <= bytes0 + (64 << 20), (held, bytes0)
        f1.free()
        torch.cuda.synchronize()
        assert not hook.live, "buffers not returned: %d" % len(hook.live)
        assert torch.cuda.memory_allocated() == base
    finally:
        H.set_allocator()
    assert rel(u1, u0) < SAME
    assert rel(u1, case.oracle_solve(case.oracle_build())) < 1e-10
    # the library's own allocator again
    f2 = case.gpu_build()
    assert rel(_solve(case, f2), u0) < SAME
    f2.free()


def test_mixed_precision_and_server_through_torch_allocator():
    import torch
    from paper_1812_07167_amd import hps as H
    case = Case(8, 8, 12, 25.0, seed=12, nrhs=2)
    fa = case.gpu_build(precision=H.HPS_PREC_MIXED)
    ua = _solve(case, fa)
    fa.free()
    hook = Counting()
    H.set_allocator(hook.alloc, hook.free)
    try:
        fb = case.gpu_build(precision=H.HPS_PREC_MIXED)
        assert rel(_solve(case, fb), ua) < SAME
        fb.free()
        srv = H.Server(slots=2)
        try:
            pid, _ = srv.build(H.domain(case.nx, case.ny, case.box), case.p, case.kappa, case.eta,
                               torch.tensor(case.c, dtype=torch.float64, device="cuda"))
            t = torch.tensor(np.ascontiguousarray(case.t), dtype=torch.complex128, device="cuda")
            s = torch.tensor(np.ascontiguousarray(case.s), dtype=torch.complex128, device="cuda")
            r, u = srv.solve(pid, t, s)
            assert srv.wait([r])[r]["status"] == 0
            us = u.cpu().numpy()
        finally:
            srv.close()
        torch.cuda.synchronize()
        assert not hook.live, "buffers not returned: %d" % len(hook.live)
    finally:
        H.set_allocator()
    assert rel(us, case.oracle_solve(case.oracle_build())) < 1e-10
