"""Shared helpers of the test-suite: build seeded problems, run the GPU library and the
CPU oracle on identical inputs, and map operators between the two boundary orders.

The oracle keeps every box boundary as a list of node keys; the library stores box
boundaries in [S, E, N, W] order.  canonical_keys() writes the library's order as keys
so that any stored operator can be compared entry by entry.
"""

from __future__ import annotations

import numpy as np

from oracle import hps_oracle as O
from paper_1812_07167_amd import inputs as G


SAME = object()  # "use the case's own body load"


def canonical_keys(ix0, ix1, iy0, iy1, m):
    S = [("h", iy0, ix, i) for ix in range(ix0, ix1) for i in range(m)]
    E = [("v", ix1, iy, j) for iy in range(iy0, iy1) for j in range(m)]
    N = [("h", iy1, ix, i) for ix in range(ix0, ix1) for i in range(m)]
    W = [("v", ix0, iy, j) for iy in range(iy0, iy1) for j in range(m)]
    return S + E + N + W


def oracle_box_index(boxes):
    return {(b.ix0, b.ix1, b.iy0, b.iy1): b for b in boxes}


def perm_to(keys_from, keys_to):
    pos = {k: i for i, k in enumerate(keys_from)}
    return np.array([pos[k] for k in keys_to])


class Case:
    """A seeded problem: geometry, coefficient, right-hand sides, on both sides."""

    def __init__(self, nx, ny, p, kappa, eta=None, box=(0.0, 1.0, 0.0, 1.0), c="fourier",
                 seed=0, nrhs=2, rhs="random"):
        self.nx, self.ny, self.p, self.kappa = nx, ny, p, kappa
        self.eta = kappa if eta is None else eta
        self.box = box
        self.m = p - 2
        self.prob = O.Problem(*box, nx, ny, p, kappa, self.eta)
        self.xy = self.prob.leaf_nodes()
        self.xyi = self.prob.interior_nodes()
        self.xyb, self.nrm = self.prob.root_boundary()
        if c == "fourier":
            self.c = G.FourierField.seeded(seed)(self.xyi)
        elif c == "bump":
            self.c = G.c_gaussian_bump(self.xyi)
        elif c == "one":
            self.c = G.c_const(self.xyi)
        else:
            raise ValueError(c)
        rng = np.random.default_rng(seed + 1000)
        ni, nt = len(self.xyi), len(self.xyb)
        self.exact = None
        if rhs == "random":
            self.s = rng.standard_normal((nrhs, ni)) + 1j * rng.standard_normal((nrhs, ni))
            self.t = rng.standard_normal((nrhs, nt)) + 1j * rng.standard_normal((nrhs, nt))
        elif rhs == "manufactured":
            th = G.seeded_thetas(seed, nrhs)
            mfs = [G.Manufactured(kappa, float(a)) for a in th]
            self.s = np.stack([mf.s(self.xyi, self.c) for mf in mfs])
            self.t = np.stack([mf.t(self.xyb, self.nrm, self.eta) for mf in mfs])
            self.exact = np.stack([mf.u(self.xy) for mf in mfs])
        elif rhs == "planewave":
            th = G.seeded_thetas(seed, nrhs)
            pws = [G.PlaneWave(kappa, float(a)) for a in th]
            self.s = None
            self.t = np.stack([pw.t(self.xyb, self.nrm, self.eta) for pw in pws])
            self.exact = np.stack([pw.u(self.xy) for pw in pws])
        elif rhs == "polynomial":
            polys = [G.Polynomial.seeded(seed + k, min(p - 1, 6)) for k in range(nrhs)]
            self.s = np.stack([q.s(self.xyi, self.c, kappa) for q in polys])
            self.t = np.stack([q.t(self.xyb, self.nrm, self.eta) for q in polys])
            self.exact = np.stack([q.u(self.xy) for q in polys])
        else:
            raise ValueError(rhs)

    # ------------------------------------------------------------------ oracle side
    def oracle_build(self, tie="x", progress=None):
        return O.build(self.prob, self.c, tie=tie, progress=progress)

    def oracle_solve(self, boxes, s=SAME):
        s = self.s if s is SAME else s
        return O.solve(self.prob, boxes, s, self.t)

    # ------------------------------------------------------------------ GPU side
    def gpu_build(self, **kw):
        import torch
        from paper_1812_07167_amd import hps as H
        dom = H.domain(self.nx, self.ny, self.box)
        c = torch.tensor(self.c, dtype=torch.float64, device="cuda")
        f = H.hps_build(dom, self.p, self.kappa, self.eta, c, **kw)
        return f

    def gpu_solve(self, f, s=SAME):
        import torch
        from paper_1812_07167_amd import hps as H
        s = self.s if s is SAME else s
        t = torch.tensor(self.t, dtype=torch.complex128, device="cuda")
        sd = None if s is None else torch.tensor(s, dtype=torch.complex128, device="cuda")
        u = H.hps_solve(f, t, sd)
        torch.cuda.synchronize()
        return u.cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))
