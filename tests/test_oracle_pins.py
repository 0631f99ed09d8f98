"""Pins for the CPU oracle: checks of oracle/hps_oracle.py against facts that do not
come from the oracle itself (closed forms, textbook values, exact discrete invariants,
a dense global solve, brute force).  CPU only.

Each pin is chosen so that a plausible mistake (dropped term, sign, index, transposed
operand, wrong side order) fails at least one of them; the mutation tests at the end
plant such mistakes in the oracle and check that the pins catch them.
"""

import os

import numpy as np
import pytest

from oracle import hps_oracle as O
from paper_1812_07167_amd import inputs as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#")


def _setup(nx, ny, p, kappa, eta, cfun, box=(0.0, 1.0, 0.0, 1.0)):
    prob = O.Problem(*box, nx, ny, p, kappa, eta)
    xy = prob.leaf_nodes()
    xyi = prob.interior_nodes()
    xyb, nrm = prob.root_boundary()
    return prob, xy, xyi, xyb, nrm, cfun(xyi)


# ------------------------------------------------------------------ P1: spectral primitives


@pytest.mark.parametrize("name,p", [("cheb_diff_N1.txt", 2), ("cheb_diff_N2.txt", 3)])
def test_cheb_diff_matches_textbook(name, p):
    """Trefethen's printed D (descending points) equals ours after reversing order."""
    Dd = _golden(name)
    J = np.eye(p)[::-1]
    np.testing.assert_allclose(O.cheb_diff(p), J @ Dd @ J, rtol=0, atol=1e-14)


@pytest.mark.parametrize("p", list(range(3, 19)))
def test_cheb_diff_exact_on_polynomials(p):
    x = O.cheb_points(p)
    assert np.all(np.diff(x) > 0) and x[0] == -1.0 and abs(x[-1] - 1.0) < 1e-15
    D = O.cheb_diff(p)
    nrm = np.abs(D).max()
    assert np.abs(D @ np.ones(p)).max() <= 1e-13 * nrm
    for k in range(1, p):
        err = np.abs(D @ x ** k - k * x ** (k - 1)).max()
        assert err <= 1e-12 * nrm * k, (p, k, err)
    N = p - 1
    # corner entries have the closed form -(2N^2+1)/6 (ascending order)
    assert abs(D[0, 0] + (2 * N * N + 1) / 6.0) <= 1e-12 * nrm
    assert abs(D[-1, -1] - (2 * N * N + 1) / 6.0) <= 1e-12 * nrm


# ------------------------------------------------------------------ P5 + leaf pins


@pytest.mark.parametrize("p,eta", [(6, 7.0), (8, 20.0), (12, 3.0 - 2.0j)])
def test_leaf_identities(p, eta):
    """F Psi = I, A(i,:) Psi = 0, F Y = 0, A(i,:) Y = I (definitions of Psi and Y),
    and the derived R = I - 2 i eta Psi_b, Gamma = -2 i eta Y_b (G = F - 2 i eta E_b)."""
    rng = np.random.default_rng(p)
    ni, nb = (p - 2) ** 2, 4 * p - 8
    c = 1.0 + 0.3 * rng.standard_normal(ni)
    ops = O.leaf_operators(0.1, 0.4, -0.2, 0.3, p, 11.0, eta, c)
    Psi, Y, F, A = ops["Psi"], ops["Y"], ops["F"], ops["Ahat_iI"]
    scale = np.abs(ops["B"]).max()
    assert np.abs(F @ Psi - np.eye(nb)).max() < 1e-11 * scale
    assert np.abs(A @ Psi).max() < 1e-9 * scale
    assert np.abs(F @ Y).max() < 1e-11 * scale
    assert np.abs(A @ Y - np.eye(ni)).max() < 1e-9 * scale
    np.testing.assert_allclose(ops["R"], np.eye(nb) - 2j * eta * Psi[:nb], atol=1e-11)
    np.testing.assert_allclose(ops["Gamma"], -2j * eta * Y[:nb], atol=1e-11)


@pytest.mark.parametrize("p", [5, 8, 11])
def test_leaf_reproduces_polynomials(p):
    """A polynomial of tensor degree <= p-1 is reproduced exactly by one leaf when t is
    its exact impedance trace (outward normal derivative + i eta u) and s its exact
    body load.  Pins the orientation and sign of the normal rows and of C."""
    x0, x1, y0, y1 = 0.2, 0.7, -0.1, 0.3
    kappa, eta = 9.0, 4.0 + 1.0j
    xy = O.leaf_coordinates(x0, x1, y0, y1, p)
    nb = 4 * p - 8
    m = p - 2
    nrm = np.concatenate([np.tile([0.0, -1.0], (m, 1)), np.tile([1.0, 0.0], (m, 1)),
                          np.tile([0.0, 1.0], (m, 1)), np.tile([-1.0, 0.0], (m, 1))])
    poly = G.Polynomial.seeded(p, p - 1)
    c = G.FourierField.seeded(p)(xy[nb:])
    ops = O.leaf_operators(x0, x1, y0, y1, p, kappa, eta, c)
    t = poly.t(xy[:nb], nrm, eta)
    s = poly.s(xy[nb:], c, kappa)
    u = ops["Psi"] @ t + ops["Y"] @ s
    assert O.rel_l2(u, poly.u(xy)) < 1e-11


def test_small_leaf_reproduces_polynomials_to_round_off():
    """A leaf of the size of the 64 x 64-leaf workload (h = 1/64, p = 16, kappa = eta =
    100): its collocation rows are about p^2/h times larger than its impedance rows.  The
    exact polynomial comes back to near machine precision, which an unequilibrated dense
    solve of B misses by two orders of magnitude."""
    p, h = 16, 1.0 / 64
    x0, y0 = 0.3, 0.6
    kappa = eta = 100.0
    xy = O.leaf_coordinates(x0, x0 + h, y0, y0 + h, p)
    m, nb = p - 2, 4 * p - 8
    nrm = np.concatenate([np.tile([0.0, -1.0], (m, 1)), np.tile([1.0, 0.0], (m, 1)),
                          np.tile([0.0, 1.0], (m, 1)), np.tile([-1.0, 0.0], (m, 1))])
    c = G.c_gaussian_bump(xy[nb:])
    ops = O.leaf_operators(x0, x0 + h, y0, y0 + h, p, kappa, eta, c)
    for seed in range(3):
        poly = G.Polynomial.seeded(seed, 6)
        u = ops["Psi"] @ poly.t(xy[:nb], nrm, eta) + ops["Y"] @ poly.s(xy[nb:], c, kappa)
        assert O.rel_l2(u, poly.u(xy)) < 3e-13


def test_leaf_plane_wave():
    """Psi applied to a plane wave's impedance data reproduces it to discretization
    error (closed form, c = 1, s = 0)."""
    p, kappa = 14, 25.0
    x0, x1, y0, y1 = 0.0, 0.25, 0.5, 0.75
    xy = O.leaf_coordinates(x0, x1, y0, y1, p)
    m, nb = p - 2, 4 * p - 8
    nrm = np.concatenate([np.tile([0.0, -1.0], (m, 1)), np.tile([1.0, 0.0], (m, 1)),
                          np.tile([0.0, 1.0], (m, 1)), np.tile([-1.0, 0.0], (m, 1))])
    pw = G.PlaneWave(kappa, 0.7)
    ops = O.leaf_operators(x0, x1, y0, y1, p, kappa, kappa, np.ones((p - 2) ** 2))
    u = ops["Psi"] @ pw.t(xy[:nb], nrm, kappa)
    assert O.rel_l2(u, pw.u(xy)) < 1e-8
    # the ItI map sends the incoming trace to the outgoing one: g = u_n - i eta u
    g = 1j * (kappa * (nrm @ [np.cos(0.7), np.sin(0.7)]) - kappa) * pw.u(xy[:nb])
    assert O.rel_l2(ops["R"] @ pw.t(xy[:nb], nrm, kappa), g) < 1e-7


# ------------------------------------------------------------------ P3: HPS == dense global solve


@pytest.mark.parametrize("nx,ny,p,kappa,eta,box", [
    (4, 4, 8, 20.0, 20.0, (0.0, 1.0, 0.0, 1.0)),
    (2, 1, 6, 5.0, 5.0, (0.0, 1.0, 0.0, 1.0)),
    (1, 2, 7, 5.0, 2.0 - 1.0j, (0.0, 1.0, 0.0, 2.0)),
    (4, 2, 6, 12.0, 12.0 + 3.0j, (-1.0, 1.0, 0.0, 0.5)),
    (2, 8, 5, 8.0, 8.0, (0.0, 0.5, 0.0, 2.0)),
    (1, 1, 9, 10.0, 10.0, (0.0, 1.0, 0.0, 1.0)),
])
def test_hps_equals_global_direct_solve(nx, ny, p, kappa, eta, box):
    prob, xy, xyi, xyb, nrm, c = _setup(nx, ny, p, kappa, eta, G.FourierField.seeded(nx * 10 + ny), box)
    rng = np.random.default_rng(1)
    s = rng.standard_normal((2, len(xyi))) + 1j * rng.standard_normal((2, len(xyi)))
    t = rng.standard_normal((2, len(xyb))) + 1j * rng.standard_normal((2, len(xyb)))
    u = O.solve(prob, O.build(prob, c), s, t)
    ug = O.global_solve(prob, c, s, t)
    assert O.rel_l2(u, ug) < 1e-11


def test_hps_equals_global_complex_c():
    prob, xy, xyi, xyb, nrm, c = _setup(2, 2, 7, 6.0, 6.0, G.FourierField.seeded(5))
    c = c + 0.2j * np.sin(3 * xyi[:, 0])
    rng = np.random.default_rng(2)
    s = rng.standard_normal(len(xyi)) + 0j
    t = rng.standard_normal(len(xyb)) + 1j * rng.standard_normal(len(xyb))
    assert O.rel_l2(O.solve(prob, O.build(prob, c), s[None], t[None]),
                    O.global_solve(prob, c, s[None], t[None])) < 1e-11


# ------------------------------------------------------------------ P2: polynomial reproduction


@pytest.mark.parametrize("nx,ny,p,kappa,box", [
    (4, 4, 8, 20.0, (0.0, 1.0, 0.0, 1.0)),
    (8, 4, 6, 30.0, (0.0, 2.0, 0.0, 1.0)),
    (2, 4, 10, 7.0, (-0.5, 0.5, 0.0, 1.5)),
])
def test_polynomial_reproduction_multilevel(nx, ny, p, kappa, box):
    deg = min(p - 1, 6)
    prob, xy, xyi, xyb, nrm, c = _setup(nx, ny, p, kappa, kappa, G.FourierField.seeded(7), box)
    poly = G.Polynomial.seeded(11, deg)
    u = O.solve(prob, O.build(prob, c), poly.s(xyi, c, kappa)[None], poly.t(xyb, nrm, kappa)[None])
    assert O.rel_l2(u[0], poly.u(xy)) < 1e-11


# ------------------------------------------------------------------ P4 + long/short forms


def test_merge_order_invariance():
    prob, xy, xyi, xyb, nrm, c = _setup(4, 4, 8, 15.0, 15.0, G.FourierField.seeded(9))
    mf = G.Manufactured(15.0, 0.4)
    s, t = mf.s(xyi, c)[None], mf.t(xyb, nrm, 15.0)[None]
    ux = O.solve(prob, O.build(prob, c, tie="x"), s, t)
    uy = O.solve(prob, O.build(prob, c, tie="y"), s, t)
    assert O.rel_l2(ux, uy) < 1e-12


def test_merge_short_forms_equal_paper_forms():
    """The oracle forms the merge maps by solving the stacked interface conditions of
    Sec. 2.2.  They must equal the paper's printed forms built on W = I - R33b R33a:
    Phi^a = W^{-1} [R33b R31a | -R32b] (eq. (talpha)), Phi^b = [-R31a - R33a W^{-1} R33b
    R31a | R33a W^{-1} R32b] (eq. (tbeta)), Ups^a = [W^{-1} R33b | -W^{-1}], Ups^b =
    [-(I + R33a W^{-1} R33b) | R33a W^{-1}]; and the short forms Phi^b = [-R31a, 0] -
    R33a Phi^a, Ups^b = [-I, 0] - R33a Ups^a (re-derived from the same conditions)."""
    prob, xy, xyi, xyb, nrm, c = _setup(4, 2, 7, 12.0, 12.0, G.FourierField.seeded(4))
    for b in O.build(prob, c):
        if b.is_leaf:
            continue
        o = b.ops
        n3 = len(o["i3a"])
        I3 = np.eye(n3)
        Wi = np.linalg.inv(I3 - o["R33b"] @ o["R33a"])
        np.testing.assert_allclose(o["Winv"], Wi, atol=1e-12)
        R33a, R33b, R31a, R32b = o["R33a"], o["R33b"], o["R31a"], o["R32b"]
        np.testing.assert_allclose(o["Phi_a"], Wi @ np.hstack([R33b @ R31a, -R32b]), atol=1e-12)
        np.testing.assert_allclose(
            o["Phi_b"], np.hstack([-R31a - R33a @ Wi @ R33b @ R31a, R33a @ Wi @ R32b]), atol=1e-12)
        np.testing.assert_allclose(o["Ups_a"], np.hstack([Wi @ R33b, -Wi]), atol=1e-12)
        np.testing.assert_allclose(
            o["Ups_b"], np.hstack([-(I3 + R33a @ Wi @ R33b), R33a @ Wi]), atol=1e-12)
        short_phi_b = -o["R33a"] @ o["Phi_a"]
        short_phi_b[:, :len(o["i1"])] -= o["R31a"]
        np.testing.assert_allclose(o["Phi_b"], short_phi_b, atol=1e-12)
        short_ups_b = -o["R33a"] @ o["Ups_a"]
        short_ups_b[:, :n3] -= np.eye(n3)
        np.testing.assert_allclose(o["Ups_b"], short_ups_b, atol=1e-12)


# ------------------------------------------------------------------ P6: shared edges


def test_shared_edge_values_agree():
    prob, xy, xyi, xyb, nrm, c = _setup(4, 4, 8, 18.0, 18.0, G.FourierField.seeded(2))
    rng = np.random.default_rng(5)
    s = rng.standard_normal(len(xyi)) + 1j * rng.standard_normal(len(xyi))
    t = rng.standard_normal(len(xyb)) + 1j * rng.standard_normal(len(xyb))
    u = O.solve(prob, O.build(prob, c), s[None], t[None])[0].reshape(16, prob.n)
    m = prob.m
    keyval = {}
    worst = 0.0
    for iy in range(4):
        for ix in range(4):
            for r, k in enumerate(O.leaf_boundary_keys(ix, iy, m)):
                v = u[iy * 4 + ix, r]
                if k in keyval:
                    worst = max(worst, abs(v - keyval[k]))
                keyval[k] = v
    assert worst < 1e-11 * np.abs(u).max()


# ------------------------------------------------------------------ P7, P8, P12: closed forms


def test_plane_wave_every_box():
    """For c = 1, every box's ItI operator maps the plane wave's incoming trace to its
    outgoing trace (to discretization error)."""
    kappa = 20.0
    prob, xy, xyi, xyb, nrm, c = _setup(4, 4, 12, kappa, kappa, G.c_const)
    th = 0.9
    d = np.array([np.cos(th), np.sin(th)])
    pw = G.PlaneWave(kappa, th)
    boxes = O.build(prob, c)
    # coordinates and normals of every boundary key
    coords, normals = {}, {}
    xyl = xy.reshape(prob.nleaf, prob.n, 2)
    side_n = [(0.0, -1.0), (1.0, 0.0), (0.0, 1.0), (-1.0, 0.0)]
    for iy in range(4):
        for ix in range(4):
            for r, k in enumerate(O.leaf_boundary_keys(ix, iy, prob.m)):
                coords[k] = xyl[iy * 4 + ix, r]
    for b in boxes:
        X = np.array([coords[k] for k in b.keys])
        nrm_b = []
        for k in b.keys:
            if k[0] == "h":
                nrm_b.append(side_n[0] if k[1] == b.iy0 else side_n[2])
            else:
                nrm_b.append(side_n[3] if k[1] == b.ix0 else side_n[1])
        nrm_b = np.array(nrm_b)
        f = 1j * (kappa * (nrm_b @ d) + kappa) * pw.u(X)
        g = 1j * (kappa * (nrm_b @ d) - kappa) * pw.u(X)
        assert O.rel_l2(b.ops["R"] @ f, g) < 1e-6, (b.level, b.ix0, b.iy0)


def test_config1_plane_wave_solution():
    """4x4 leaves, p = 8, kappa = eta = 20, c = 1, s = 0, plane wave (seed 0)."""
    kappa = 20.0
    prob, xy, xyi, xyb, nrm, c = _setup(4, 4, 8, kappa, kappa, G.c_const)
    pw = G.PlaneWave(kappa, G.seeded_theta(0))
    u = O.solve(prob, O.build(prob, c), None, pw.t(xyb, nrm, kappa)[None])
    assert O.rel_l2(u[0], pw.u(xy)) < 1e-3


def test_spectral_convergence_in_p():
    kappa = 20.0
    errs = []
    for p in (6, 8, 10, 12, 14):
        prob, xy, xyi, xyb, nrm, c = _setup(4, 4, p, kappa, kappa, G.c_gaussian_bump)
        mf = G.Manufactured(kappa, 0.3)
        u = O.solve(prob, O.build(prob, c), mf.s(xyi, c)[None], mf.t(xyb, nrm, kappa)[None])
        errs.append(O.rel_l2(u[0], mf.u(xy)))
    for a, b in zip(errs, errs[1:]):
        assert b < a / 5, errs
    assert errs[-1] < 1e-7


# ------------------------------------------------------------------ P9, P10: reciprocity, unitarity


def _edge_weights(p, length):
    """Interpolatory quadrature weights for the p-2 interior Lobatto nodes of an edge:
    exact for polynomials of degree <= p-3 (solved from the moment equations)."""
    x = O.cheb_points(p)[1:-1]
    k = np.arange(p - 2)
    V = x[None, :] ** k[:, None]
    mom = np.array([(1 - (-1) ** (j + 1)) / (j + 1) for j in k])
    return np.linalg.solve(V, mom) * length / 2.0


def _leaf_Q(p, hx, hy):
    wx, wy = _edge_weights(p, hx), _edge_weights(p, hy)
    return np.concatenate([wx, wy, wx, wy])


def test_reciprocity_and_unitarity_defects_decay():
    """Green's second identity makes Q R complex symmetric and, for real c and real
    eta > 0, energy conservation makes Q^(1/2) R Q^(-1/2) unitary.  Both hold for the
    discrete operator up to discretization error; at the matrix level that error is
    set by the corners (arbitrary edge data is not smooth there), so it decays
    algebraically with p.  A sign error in the i eta terms or a transposed block
    makes either defect O(1)."""
    kappa = 12.0
    hx = hy = 0.25

    def defects(pp):
        c = G.c_gaussian_bump(O.leaf_coordinates(0, hx, 0, hy, pp)[4 * pp - 8:], 0.3, 10.0, 0.1, 0.1)
        R = O.leaf_operators(0, hx, 0, hy, pp, kappa, kappa, c)["R"]
        Q = _leaf_Q(pp, hx, hy)
        QR = Q[:, None] * R
        recip = np.abs(QR - QR.T).max() / np.abs(QR).max()
        Uq = np.sqrt(Q)[:, None] * R / np.sqrt(Q)[None, :]
        sv = np.linalg.svd(Uq, compute_uv=False)
        return recip, np.abs(sv - 1).max()

    r1, u1 = defects(8)
    r2, u2 = defects(16)
    assert r2 < r1 / 3 and u2 < u1 / 1.5
    assert r2 < 0.015 and u2 < 0.07


@pytest.mark.parametrize("p", [8, 14])
def test_reciprocity_and_energy_on_smooth_data(p):
    """On traces of smooth exact solutions (plane waves, c = 1) the reciprocity form
    sum Q (g_a f_b - f_a g_b) and the energy balance |Q^(1/2) f| = |Q^(1/2) R f| hold
    to a spectrally small error."""
    kappa, hx, hy = 12.0, 0.25, 0.25
    xy = O.leaf_coordinates(0, hx, 0, hy, p)
    m, nb = p - 2, 4 * p - 8
    nrm = np.concatenate([np.tile([0.0, -1.0], (m, 1)), np.tile([1.0, 0.0], (m, 1)),
                          np.tile([0.0, 1.0], (m, 1)), np.tile([-1.0, 0.0], (m, 1))])
    R = O.leaf_operators(0, hx, 0, hy, p, kappa, kappa, np.ones(m * m))["R"]
    Q = _leaf_Q(p, hx, hy)
    fa = G.PlaneWave(kappa, 0.3).t(xy[:nb], nrm, kappa)
    fb = G.PlaneWave(kappa, 2.1).t(xy[:nb], nrm, kappa)
    ga, gb = R @ fa, R @ fb
    rec = abs(np.sum(Q * (ga * fb - fa * gb))) / np.sum(Q * np.abs(ga * fb))
    en = abs(np.sqrt(np.sum(Q * abs(ga) ** 2)) / np.sqrt(np.sum(Q * abs(fa) ** 2)) - 1)
    tol = 1e-3 if p == 8 else 1e-8
    assert rec < tol and en < tol, (rec, en)


# ------------------------------------------------------------------ P11: linearity, s = 0 shortcut


def test_linearity_and_zero_body_load_shortcut():
    prob, xy, xyi, xyb, nrm, c = _setup(4, 2, 7, 9.0, 9.0, G.FourierField.seeded(8))
    boxes = O.build(prob, c)
    rng = np.random.default_rng(3)
    s = rng.standard_normal((2, len(xyi))) + 1j * rng.standard_normal((2, len(xyi)))
    t = rng.standard_normal((2, len(xyb))) + 1j * rng.standard_normal((2, len(xyb)))
    u = O.solve(prob, boxes, s, t)
    a, b = 0.3 - 1.2j, 2.0
    ul = O.solve(prob, boxes, a * s[:1] + b * s[1:], a * t[:1] + b * t[1:])
    assert O.rel_l2(ul[0], a * u[0] + b * u[1]) < 1e-12
    u0 = O.solve(prob, boxes, None, t)
    uz = O.solve(prob, boxes, np.zeros_like(s), t)
    assert O.rel_l2(u0, uz) < 1e-14


# ------------------------------------------------------------------ mutation tests: the pins bite


def test_pins_catch_transposed_diff_matrix(monkeypatch):
    orig = O.cheb_diff
    monkeypatch.setattr(O, "cheb_diff", lambda p: orig(p).T)
    p = 7
    x = O.cheb_points(p)
    D = O.cheb_diff(p)
    assert np.abs(D @ x ** 2 - 2 * x).max() > 1e-3


def test_pins_catch_tangential_normal_rows(monkeypatch):
    """The literally printed N rows (tangential derivatives) fail the polynomial pin."""
    real_kron = np.kron

    def literal(x0, x1, y0, y1, p, kappa, eta, c_int):
        gg = O.LeafGrid(p)
        D = O.cheb_diff(p)
        Dx = real_kron(np.eye(p), 2.0 / (x1 - x0) * D)
        Dy = real_kron(2.0 / (y1 - y0) * D, np.eye(p))
        cfull = np.zeros(p * p, dtype=complex)
        cfull[gg.I_i] = c_int
        Ahat = -(Dx @ Dx) - (Dy @ Dy) - np.diag(kappa ** 2 * cfull)
        N = np.concatenate([-Dx[gg.I_s][:, gg.I], Dy[gg.I_e][:, gg.I],
                            Dx[gg.I_n][:, gg.I], -Dy[gg.I_w][:, gg.I]])
        Eb = np.eye(p * p)[gg.I_b][:, gg.I]
        F, Gm = N + 1j * eta * Eb, N - 1j * eta * Eb
        B = np.concatenate([F, Ahat[gg.I_i][:, gg.I]])
        Binv = np.linalg.inv(B)
        Psi, Y = Binv[:, :gg.nb], Binv[:, gg.nb:]
        return dict(Psi=Psi, Y=Y, R=Gm @ Psi, Gamma=Gm @ Y, F=F, G=Gm, N=N, B=B,
                    Ahat_iI=Ahat[gg.I_i][:, gg.I])

    monkeypatch.setattr(O, "leaf_operators", literal)
    prob, xy, xyi, xyb, nrm, c = _setup(2, 2, 8, 5.0, 5.0, G.c_const)
    poly = G.Polynomial.seeded(11, 5)
    u = O.solve(prob, O.build(prob, c), poly.s(xyi, c, 5.0)[None], poly.t(xyb, nrm, 5.0)[None])
    assert O.rel_l2(u[0], poly.u(xy)) > 1e-3


def test_pins_catch_misordered_side(monkeypatch):
    """Reversing the node order of one side of every leaf breaks the key matching of
    the merge; the dense global solve (which uses the same keys) then disagrees with
    the exact polynomial."""
    orig = O.leaf_boundary_keys

    def bad(ix, iy, m):
        k = orig(ix, iy, m)
        return k[:m][::-1] + k[m:]

    monkeypatch.setattr(O, "leaf_boundary_keys", bad)
    prob, xy, xyi, xyb, nrm, c = _setup(2, 2, 7, 5.0, 5.0, G.c_const)
    poly = G.Polynomial.seeded(11, 5)
    u = O.solve(prob, O.build(prob, c), poly.s(xyi, c, 5.0)[None], poly.t(xyb, nrm, 5.0)[None])
    assert O.rel_l2(u[0], poly.u(xy)) > 1e-3


def test_pins_catch_wrong_sign_in_W(monkeypatch):
    """W = I + R33b R33a instead of I - R33b R33a is caught by the dense global solve."""
    orig_inv = np.linalg.inv

    def merge_bad(Ra, ka, Rb, kb):
        mo = orig_merge(Ra, ka, Rb, kb)
        n3 = len(mo["i3a"])
        Wb = np.eye(n3) + mo["R33b"] @ mo["R33a"]
        Wi = orig_inv(Wb)
        mo["Phi_a"] = Wi @ np.hstack([mo["R33b"] @ mo["R31a"], -mo["R32b"]])
        mo["Ups_a"] = np.hstack([Wi @ mo["R33b"], -Wi])
        return mo

    orig_merge = O.merge_operators
    monkeypatch.setattr(O, "merge_operators", merge_bad)
    prob, xy, xyi, xyb, nrm, c = _setup(2, 1, 6, 5.0, 5.0, G.c_const)
    rng = np.random.default_rng(0)
    t = rng.standard_normal((1, len(xyb))) + 0j
    u = O.solve(prob, O.build(prob, c), None, t)
    monkeypatch.setattr(O, "merge_operators", orig_merge)
    ug = O.global_solve(prob, c, None, t)
    assert O.rel_l2(u, ug) > 1e-3


# ------------------------------------------------------------------ residual correction (jumps)
# Not in the paper: a reduced-precision solve is corrected with the FP64 residual of the
# global system, whose shared-edge rows then carry non-zero right-hand sides ("jumps").


def _jump_case(nx=2, ny=2, p=6, kappa=11.0, eta=7.0 - 2.0j, seed=3, nrhs=2):
    prob, xy, xyi, xyb, nrm, c = _setup(nx, ny, p, kappa, eta, G.FourierField.seeded(seed))
    rng = np.random.default_rng(seed)
    cn = lambda *sh: rng.standard_normal(sh) + 1j * rng.standard_normal(sh)
    s = cn(nrhs, prob.nleaf * prob.ni)
    t = cn(nrhs, len(xyb))
    j = cn(nrhs, prob.nleaf, prob.nb)
    return prob, c, s, t, j


@pytest.mark.parametrize("nx,ny,p", [(2, 2, 6), (4, 2, 5), (2, 4, 7)])
def test_jump_solve_equals_global_direct_solve(nx, ny, p):
    """With right-hand sides on the shared-edge rows, the HPS solve (jumps injected at
    every merge) equals the dense LU solve of the global system with those rows."""
    prob, c, s, t, j = _jump_case(nx, ny, p)
    u = O.solve(prob, O.build(prob, c), s, t, jumps=j)
    ug = O.global_solve(prob, c, s, t, jumps=j)
    assert O.rel_l2(u, ug) < 1e-11
    # and jumps alone (s = 0, t = 0) give a non-trivial field, also equal
    z = np.zeros_like(t)
    u0 = O.solve(prob, O.build(prob, c), None, z, jumps=j)
    assert np.linalg.norm(u0) > 1e-3 * np.linalg.norm(u)
    assert O.rel_l2(u0, O.global_solve(prob, c, None, z, jumps=j)) < 1e-11


def test_residual_vanishes_on_exact_solutions():
    """The residual is zero (to round-off) at the dense solution of the global system,
    and at the nodal values of a polynomial of degree <= p-1 with its exact s and t
    (the discrete system holds exactly for such u)."""
    prob, c, s, t, j = _jump_case(4, 2, 7)
    ug = O.global_solve(prob, c, s, t, jumps=j)
    r = O.global_residual(prob, c, s, t, ug, jumps=j)
    b = O.global_rhs(prob, s, t, jumps=j)
    assert np.linalg.norm(r) < 1e-11 * np.linalg.norm(b)
    prob, xy, xyi, xyb, nrm, c = _setup(4, 4, 8, 15.0, 15.0, G.FourierField.seeded(2))
    poly = G.Polynomial.seeded(5, 6)
    sp, tp = poly.s(xyi, c, 15.0)[None], poly.t(xyb, nrm, 15.0)[None]
    r = O.global_residual(prob, c, sp, tp, poly.u(xy)[None])
    assert np.linalg.norm(r) < 1e-10 * np.linalg.norm(O.global_rhs(prob, sp, tp))


def test_correction_solve_removes_a_perturbation():
    """u' = u + e: solving with the residual of u' as (s, t, jumps) returns -e, so one
    correction step restores u to round-off."""
    prob, c, s, t, j = _jump_case(4, 4, 6)
    boxes = O.build(prob, c)
    u = O.solve(prob, boxes, s, t)
    rng = np.random.default_rng(9)
    e = 1e-3 * (rng.standard_normal(u.shape) + 1j * rng.standard_normal(u.shape))
    r = O.global_residual(prob, c, s, t, u + e)
    sc, tc, jc = O.correction_rhs(prob, r)
    d = O.solve(prob, boxes, sc, tc, jumps=jc)
    assert O.rel_l2(d, -e) < 1e-9
    assert O.rel_l2(u + e + d, u) < 1e-12


def test_plane_wave_residual_decays_with_p():
    """The global residual of the sampled exact plane wave is a discretization error:
    it decays spectrally in p (c = 1, s = 0)."""
    res = []
    for p in (6, 8, 10, 12):
        prob, xy, xyi, xyb, nrm, c = _setup(2, 2, p, 12.0, 12.0, G.c_const)
        pw = G.PlaneWave(12.0, 0.7)
        r = O.global_residual(prob, c, None, pw.t(xyb, nrm, 12.0)[None], pw.u(xy)[None])
        res.append(np.linalg.norm(r) / np.linalg.norm(pw.t(xyb, nrm, 12.0)))
    assert all(b < a for a, b in zip(res, res[1:]))
    assert res[-1] < 1e-3 * res[0]


def test_pins_catch_swapped_jump_sides(monkeypatch):
    """Injecting j1 and j2 on the wrong sides of the interface fails the jump pin."""
    orig = O.solve

    def bad_solve(prob, boxes, s, t, upward=True, jumps=None):
        if jumps is None:
            return orig(prob, boxes, s, t, upward)
        # swap the roles: give every shared row the other side's right-hand side
        jj = np.asarray(jumps).reshape(-1, prob.nleaf, prob.nb).copy()
        for key, lst in O.shared_rows(prob).items():
            if len(lst) == 2:
                (l1, r1), (l2, r2) = lst
                jj[:, l1, r1], jj[:, l2, r2] = jumps[:, l2, r2].copy(), jumps[:, l1, r1].copy()
        return orig(prob, boxes, s, t, upward, jj)

    prob, c, s, t, j = _jump_case(2, 2, 6)
    u = bad_solve(prob, O.build(prob, c), s, t, jumps=j)
    assert O.rel_l2(u, O.global_solve(prob, c, s, t, jumps=j)) > 1e-3


def test_pins_catch_residual_with_F_for_G(monkeypatch):
    """A residual that uses the neighbour's F instead of G misses the exact solution."""
    prob, c, s, t, j = _jump_case(2, 2, 6)
    ug = O.global_solve(prob, c, s, t, jumps=j)
    orig = O.leaf_operators

    def swapped(*a, **k):
        ops = orig(*a, **k)
        ops = dict(ops)
        ops["G"] = ops["F"]
        return ops

    monkeypatch.setattr(O, "leaf_operators", swapped)
    r = O.global_residual(prob, c, s, t, ug, jumps=j)
    assert np.linalg.norm(r) > 1e-3 * np.linalg.norm(O.global_rhs(prob, s, t, jumps=j))


# ------------------------------------------------------------------ O14: the paper's e_inf (Sec. 4.1)


def test_e_inf_recovers_a_planted_error():
    """e_inf is the largest pointwise deviation (Sec. 4.1): a single complex error of known
    size planted at one node of an otherwise exact vector is returned, up to the rounding
    of adding it to that node, wherever it sits and whatever the vector's shape; zero for
    identical vectors."""
    rng = np.random.default_rng(7)
    b = rng.standard_normal((3, 41)) + 1j * rng.standard_normal((3, 41))
    assert O.e_inf(b, b) == 0.0
    for (r, k), d in [((0, 0), 3.0 - 4.0j), ((2, 40), -1e-9j), ((1, 17), 2.5)]:
        a = b.copy()
        a[r, k] += d
        ulp = 4.0 * np.finfo(float).eps * np.abs(b).max()
        assert O.e_inf(a, b) == pytest.approx(abs(d), rel=1e-12, abs=ulp)


def test_e_inf_norm_bounds_and_decay_in_p():
    """Norm equivalence with the 2-norm, ||d||_2 / sqrt(N) <= e_inf <= ||d||_2, on the
    discretization error of a solve; and e_inf of a plane-wave solve falls
    geometrically with p (the spectral convergence of Sec. 4.1)."""
    kappa = 20.0
    errs = []
    for p in (6, 8, 10, 12):
        prob, xy, xyi, xyb, nrm, c = _setup(2, 2, p, kappa, kappa, G.c_const)
        pw = G.PlaneWave(kappa, 0.7)
        u = O.solve(prob, O.build(prob, c), None, pw.t(xyb, nrm, kappa)[None])[0]
        ex = pw.u(xy)
        d2 = float(np.linalg.norm(u - ex))
        ei = O.e_inf(u, ex)
        assert d2 / np.sqrt(u.size) <= ei * (1 + 1e-12) and ei <= d2 * (1 + 1e-12)
        errs.append(ei)
    for a, b in zip(errs, errs[1:]):
        assert b < a / 5, errs
