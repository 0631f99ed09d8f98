"""Seeded synthetic inputs for the impedance Helmholtz problem
    -Lap u - kappa^2 c(x) u = s  in Omega,   du/dnu + i eta u = t  on dOmega
(eq. (basic) of the paper).

This module holds closed-form problem data only: coefficient fields c, exact solutions
u and the body load s / impedance data t that they imply.  It contains none of the
solver's arithmetic (no collocation, no merges); it is evaluated at coordinates that
the caller passes in, so the GPU library and the CPU oracle are fed identical arrays.
Pure numpy, no GPU.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


# ----------------------------------------------------------------------------- c(x)


def c_const(xy, value=1.0):
    return np.full(len(xy), float(value))


def c_gaussian_bump(xy, depth=0.5, width=160.0, x0=0.5, y0=0.5):
    """c = 1 - depth * exp(-width ((x-x0)^2 + (y-y0)^2)) (a smooth scatterer)."""
    x, y = xy[:, 0], xy[:, 1]
    return 1.0 - depth * np.exp(-width * ((x - x0) ** 2 + (y - y0) ** 2))


@dataclass
class FourierField:
    """c = 1 + sum_k a_k cos(2 pi (m_k x + n_k y) + phi_k), sum a_k = amp."""
    a: np.ndarray
    m: np.ndarray
    n: np.ndarray
    phi: np.ndarray

    @staticmethod
    def seeded(seed, nmodes=8, kmax=4, amp=0.5):
        rng = np.random.default_rng(seed)
        pairs = [(i, j) for i in range(-kmax, kmax + 1) for j in range(-kmax, kmax + 1)
                 if (i, j) != (0, 0)]
        idx = rng.integers(0, len(pairs), size=nmodes)
        m = np.array([pairs[i][0] for i in idx], dtype=float)
        n = np.array([pairs[i][1] for i in idx], dtype=float)
        phi = rng.uniform(0.0, 2 * np.pi, size=nmodes)
        w = rng.uniform(0.0, 1.0, size=nmodes)
        a = amp * w / w.sum()
        return FourierField(a, m, n, phi)

    def __call__(self, xy):
        x, y = xy[:, 0:1], xy[:, 1:2]
        arg = 2 * np.pi * (x * self.m[None] + y * self.n[None]) + self.phi[None]
        return 1.0 + (self.a[None] * np.cos(arg)).sum(axis=1)


# ------------------------------------------------------------------ exact solutions


@dataclass
class PlaneWave:
    """u = exp(i kappa d.x), d = (cos theta, sin theta).  With c = 1, s = 0 and
    t = i (kappa d.nu + eta) u."""
    kappa: float
    theta: float

    def u(self, xy):
        d = np.array([np.cos(self.theta), np.sin(self.theta)])
        return np.exp(1j * self.kappa * (xy @ d))

    def s(self, xy, c):
        x = xy
        return (self.kappa ** 2 * (1.0 - c)) * self.u(x)

    def t(self, xy, nrm, eta):
        d = np.array([np.cos(self.theta), np.sin(self.theta)])
        return 1j * (self.kappa * (nrm @ d) + eta) * self.u(xy)


@dataclass
class Manufactured:
    """u = exp(i kappa d.x) (1 + 0.1 sin 2 pi x sin 2 pi y).

    s = phi [kappa^2 (1 - c) w - 2 i kappa d.grad w - Lap w],
    t = phi [nu.grad w + i (kappa d.nu + eta) w],  phi = exp(i kappa d.x).
    """
    kappa: float
    theta: float
    amp: float = 0.1

    def _parts(self, xy):
        x, y = xy[:, 0], xy[:, 1]
        d = np.array([np.cos(self.theta), np.sin(self.theta)])
        phi = np.exp(1j * self.kappa * (xy @ d))
        sx, sy = np.sin(2 * np.pi * x), np.sin(2 * np.pi * y)
        cx, cy = np.cos(2 * np.pi * x), np.cos(2 * np.pi * y)
        w = 1.0 + self.amp * sx * sy
        gw = np.stack([2 * np.pi * self.amp * cx * sy, 2 * np.pi * self.amp * sx * cy], axis=1)
        lw = -8 * np.pi ** 2 * self.amp * sx * sy
        return d, phi, w, gw, lw

    def u(self, xy):
        _, phi, w, _, _ = self._parts(xy)
        return phi * w

    def s(self, xy, c):
        d, phi, w, gw, lw = self._parts(xy)
        return phi * (self.kappa ** 2 * (1.0 - c) * w - 2j * self.kappa * (gw @ d) - lw)

    def t(self, xy, nrm, eta):
        d, phi, w, gw, _ = self._parts(xy)
        return phi * ((gw * nrm).sum(axis=1) + 1j * (self.kappa * (nrm @ d) + eta) * w)


@dataclass
class Polynomial:
    """u = sum_{j,k <= deg} a_jk x^j y^k with complex coefficients (a global polynomial
    of tensor degree <= deg).  Its gradient and Laplacian are evaluated exactly."""
    coef: np.ndarray  # [deg+1, deg+1]

    @staticmethod
    def seeded(seed, deg):
        rng = np.random.default_rng(seed)
        a = rng.standard_normal((deg + 1, deg + 1)) + 1j * rng.standard_normal((deg + 1, deg + 1))
        return Polynomial(a / (deg + 1))

    def _eval(self, xy, dx=0, dy=0):
        x, y = xy[:, 0], xy[:, 1]
        deg = self.coef.shape[0] - 1
        out = np.zeros(len(xy), dtype=complex)
        for j in range(deg + 1):
            for k in range(deg + 1):
                if j < dx or k < dy:
                    continue
                cj = np.prod(np.arange(j - dx + 1, j + 1)) if dx else 1.0
                ck = np.prod(np.arange(k - dy + 1, k + 1)) if dy else 1.0
                out += self.coef[j, k] * cj * ck * x ** (j - dx) * y ** (k - dy)
        return out

    def u(self, xy):
        return self._eval(xy)

    def s(self, xy, c, kappa):
        lap = self._eval(xy, 2, 0) + self._eval(xy, 0, 2)
        return -lap - kappa ** 2 * c * self._eval(xy)

    def t(self, xy, nrm, eta):
        gx, gy = self._eval(xy, 1, 0), self._eval(xy, 0, 1)
        return nrm[:, 0] * gx + nrm[:, 1] * gy + 1j * eta * self._eval(xy)


def seeded_theta(seed):
    return float(np.random.default_rng(seed).uniform(0.0, 2 * np.pi))


def seeded_thetas(seed, k):
    return np.random.default_rng(seed).uniform(0.0, 2 * np.pi, size=k)


def root_normals(nx, ny, m):
    """Outward unit normals of the root boundary data in the external order
    (S side, E side, N side, W side; nx*m, ny*m, nx*m, ny*m nodes)."""
    return np.concatenate([
        np.tile([0.0, -1.0], (nx * m, 1)), np.tile([1.0, 0.0], (ny * m, 1)),
        np.tile([0.0, 1.0], (nx * m, 1)), np.tile([-1.0, 0.0], (ny * m, 1))])


def batch_problems(seed0=0, count=256):
    """Seeded parameters of a batch of independent problems on the unit square: leaf grid
    side from {8, 16, 32}, p from {8, 12, 16}, kappa ~ U[10, 80], eta = kappa, c a seeded
    Fourier field (8 modes, wave numbers <= 4, total amplitude 0.5) and one manufactured
    right-hand side with a seeded direction.  Returns a list of dicts."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        side = int(rng.choice([8, 16, 32]))
        p = int(rng.choice([8, 12, 16]))
        kappa = float(rng.uniform(10.0, 80.0))
        out.append({"seed": seed0 + i, "nx": side, "ny": side, "p": p, "kappa": kappa,
                    "theta": float(rng.uniform(0.0, 2 * np.pi))})
    return out


def serve_problems(seed0=0, count=32):
    """Seeded parameters of resident problems for a request stream on the unit square:
    leaf grid side from {32, 64, 128} (probabilities 0.4, 0.4, 0.2), p from {12, 14, 16},
    kappa ~ U[50, 300], eta = kappa, c a seeded Fourier field as in batch_problems, and
    two seeded smooth fields (Fourier fields of their own seeds) from which a problem's
    body loads are formed.  Returns a list of dicts."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(10_000 + seed0 + i)
        side = int(rng.choice([32, 64, 128], p=[0.4, 0.4, 0.2]))
        p = int(rng.choice([12, 14, 16]))
        kappa = float(rng.uniform(50.0, 300.0))
        out.append({"seed": 10_000 + seed0 + i, "nx": side, "ny": side, "p": p,
                    "kappa": kappa, "s_seeds": (20_000 + seed0 + 2 * i, 20_001 + seed0 + 2 * i)})
    return out


def poisson_requests(seed, count, max_rhs=64):
    """A seeded request stream: for each request a uniform draw in [0, 1) that picks its
    problem among those known when it arrives, its number of right-hand sides (uniform
    in 1..max_rhs; it solves the first nrhs of its problem's data) and unit-rate
    exponential inter-arrival gaps (scaled by 1/rate for a Poisson stream)."""
    rng = np.random.default_rng(seed)
    pick = rng.uniform(0.0, 1.0, size=count)
    nrhs = rng.integers(1, max_rhs + 1, size=count)
    gaps = rng.exponential(1.0, size=count)
    return pick, nrhs, gaps
