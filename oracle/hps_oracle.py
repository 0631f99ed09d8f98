"""Plain FP64 complex CPU oracle of the HPS direct solver (Beams, Gillman, Hewett,
"A parallel shared-memory implementation of a high-order accurate solution technique
for variable coefficient Helmholtz problems", arXiv 1812.07167).

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously-correct reference that
the GPU library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or call it.  It shares no code with
the HIP path (no kernels, helpers, index maps or constants) and imports nothing from
the package.

Everything is complex128 / float64 numpy.  Library primitives used as single steps:
``numpy.linalg.solve`` / ``numpy.linalg.inv`` (dense LU with partial pivoting) and ``@``
(matrix product).  There is no blocking, fusion or reordering beyond the formulas of
the paper.  Each function cites the passage it follows.

Readings taken where the paper is silent, garbled or inconsistent:

* Sec. 2.1: the "classic product Chebyshev grid" is read as Chebyshev-Lobatto points,
  p = n_c per direction, stored in ascending coordinate order, with the standard
  (Trefethen) differentiation matrix.
* Sec. 2.1, definition of N: the printed rows (-D_x on the south edge, D_y on the east
  edge, ...) are tangential derivatives; the outward-normal reading (-D_y south,
  +D_x east, +D_y north, -D_x west) is the only one consistent with the ItI definition
  (Definition 2.1) and with dropping the corner points.  The oracle uses the normal
  reading.
* Sec. 2.1.2, eq. (particular): the printed block row [A(i,i) A(i,b)] is read as
  [A(i,b) A(i,i)] so that it multiplies u = [u_b; u_i] (same B as eq. (homogeneous)).
* The R^tau step of Algorithm 1 prints a stacked column [R13; R23]; the block-diagonal
  form of eq. (out) / eq. (flux_part) is used.
* Algorithm 2's downward pass gives only the t3 parts of the children's incoming data;
  the remaining parts are the parent's incoming data restricted to I_1 and I_2.
* The order of nodes within a side is not fixed by the paper; the oracle keeps every
  box boundary as a list of node keys and matches children by key, and maps the
  root boundary to the documented external order (S, E, N, W sides, each in
  ascending coordinate) only at the very end.
* Tree: each box is split in half across its longer side (ties split x).  The result
  of the method does not depend on this choice beyond round-off.
"""

from __future__ import annotations

import os

import numpy as np

# --------------------------------------------------------------------------------
# Spectral primitives: Sec. 2.1 (classic Chebyshev collocation, Trefethen 2000)
# --------------------------------------------------------------------------------


def cheb_points(p: int) -> np.ndarray:
    """Chebyshev-Lobatto points on [-1, 1] in ascending order (p points).

    Sec. 2.1: the leaf uses the classic n_c x n_c product Chebyshev grid.  The points
    cos(k pi/(p-1)) are listed descending in Trefethen's book; we use ascending order.
    """
    k = np.arange(p)
    return -np.cos(np.pi * k / (p - 1))


def cheb_diff(p: int) -> np.ndarray:
    """Spectral differentiation matrix on the ascending Chebyshev-Lobatto points.

    Off-diagonal entries (c_i/c_j)(-1)^(i+j)/(x_i - x_j), with c = 2 at both end points
    and 1 elsewhere; the diagonal is minus the row sum of the off-diagonal entries so
    that D applied to a constant is exactly zero (Trefethen, Spectral Methods in
    MATLAB, ch. 6).  The formula is unchanged by reversing the point order.
    """
    x = cheb_points(p)
    c = np.ones(p)
    c[0] = c[-1] = 2.0
    D = np.zeros((p, p))
    for i in range(p):
        for j in range(p):
            if i != j:
                D[i, j] = (c[i] / c[j]) * (-1.0) ** (i + j) / (x[i] - x[j])
    for i in range(p):
        D[i, i] = -np.sum(D[i, :])
    return D


# --------------------------------------------------------------------------------
# One leaf: Sec. 2.1, 2.1.1, 2.1.2
# --------------------------------------------------------------------------------


class LeafGrid:
    """Index sets of a p x p tensor grid with the corners removed (Sec. 2.1, Fig. 2).

    Full-grid index k = j*p + i, where i is the x index and j the y index.
    I_b = [I_s, I_e, I_n, I_w] (corners excluded), I_i = interior in j-major order.
    """

    def __init__(self, p: int):
        self.p = p
        m = p - 2
        self.m = m
        full = lambda i, j: j * p + i
        self.I_s = np.array([full(i, 0) for i in range(1, p - 1)])
        self.I_e = np.array([full(p - 1, j) for j in range(1, p - 1)])
        self.I_n = np.array([full(i, p - 1) for i in range(1, p - 1)])
        self.I_w = np.array([full(0, j) for j in range(1, p - 1)])
        self.I_b = np.concatenate([self.I_s, self.I_e, self.I_n, self.I_w])
        self.I_i = np.array([full(i, j) for j in range(1, p - 1) for i in range(1, p - 1)])
        self.I = np.concatenate([self.I_b, self.I_i])
        self.nb = 4 * p - 8
        self.ni = (p - 2) ** 2
        self.n = p * p - 4


def leaf_coordinates(x0: float, x1: float, y0: float, y1: float, p: int) -> np.ndarray:
    """Coordinates of the n = p^2-4 leaf nodes in the order I = [I_b, I_i] (Sec. 2.1)."""
    g = LeafGrid(p)
    xs = x0 + (x1 - x0) * (1.0 + cheb_points(p)) / 2.0
    ys = y0 + (y1 - y0) * (1.0 + cheb_points(p)) / 2.0
    X = np.array([xs[k % p] for k in range(p * p)])
    Y = np.array([ys[k // p] for k in range(p * p)])
    return np.stack([X[g.I], Y[g.I]], axis=1)


def leaf_operators(x0, x1, y0, y1, p, kappa, eta, c_interior):
    """Leaf solution and ItI operators of one box (Sec. 2.1, 2.1.1, 2.1.2).

    Returns a dict with
      Psi   (n x nb): homogeneous solution operator, B Psi = [I; 0]   eq. (hmgsolnopdef)
      Y     (n x ni): particular solution operator, B Y = [0; I]       eq. (prtsolnopdef)
      R     (nb x nb): ItI operator R = G Psi                           Sec. 2.1.1
      Gamma (nb x ni): outgoing particular impedance Gamma = G Y        Sec. 2.1.2
      and the pieces F, G, Ahat_iI, B for the identity pins.
    c_interior holds c at the n_i interior nodes (j-major); C only enters interior
    rows of B, so its boundary values are never used.
    """
    g = LeafGrid(p)
    hx, hy = x1 - x0, y1 - y0
    D = cheb_diff(p)
    Dx1 = (2.0 / hx) * D
    Dy1 = (2.0 / hy) * D
    Ip = np.eye(p)
    # k = j*p + i: x derivative acts on i (fast index), y derivative on j.
    Dx = np.kron(Ip, Dx1)
    Dy = np.kron(Dy1, Ip)
    # Ahat = -Dx^2 - Dy^2 - C  (Sec. 2.1), C = diag(kappa^2 c) on the full grid.
    cfull = np.zeros(p * p, dtype=complex)
    cfull[g.I_i] = c_interior
    Ahat = -(Dx @ Dx) - (Dy @ Dy) - np.diag(kappa ** 2 * cfull)
    # Outward normal derivative rows (normal reading of Sec. 2.1's N).
    N = np.concatenate([
        -Dy[g.I_s][:, g.I],
        +Dx[g.I_e][:, g.I],
        +Dy[g.I_n][:, g.I],
        -Dx[g.I_w][:, g.I],
    ])
    Eb = np.eye(p * p)[g.I_b][:, g.I]
    F = N + 1j * eta * Eb
    G = N - 1j * eta * Eb
    Ahat_iI = Ahat[g.I_i][:, g.I]
    B = np.concatenate([F, Ahat_iI])  # eq. (homogeneous)
    rhs_h = np.concatenate([np.eye(g.nb), np.zeros((g.ni, g.nb))])  # eq. (hmgsolnopdef)
    rhs_p = np.concatenate([np.zeros((g.nb, g.ni)), np.eye(g.ni)])  # eq. (prtsolnopdef)
    # Both systems are solved with every row of B and of its right-hand side divided by
    # the row's largest entry of B (row equilibration, which leaves the solutions
    # unchanged): the collocation rows carry second derivatives and the impedance rows
    # first derivatives, so their scales differ by about (p^2/h), and partial pivoting
    # only compares like-sized rows once they are equilibrated.
    d = 1.0 / np.abs(B).max(axis=1)
    Psi = np.linalg.solve(d[:, None] * B, d[:, None] * rhs_h)
    Y = np.linalg.solve(d[:, None] * B, d[:, None] * rhs_p)
    R = G @ Psi
    Gamma = G @ Y
    return dict(Psi=Psi, Y=Y, R=R, Gamma=Gamma, F=F, G=G, N=N, B=B, Ahat_iI=Ahat_iI)


# --------------------------------------------------------------------------------
# Tree and box boundaries: Sec. 2 (uniform partition, binary tree, parent < child)
# --------------------------------------------------------------------------------


class Box:
    __slots__ = ("ix0", "ix1", "iy0", "iy1", "children", "level", "keys", "ops")

    def __init__(self, ix0, ix1, iy0, iy1, level):
        self.ix0, self.ix1, self.iy0, self.iy1 = ix0, ix1, iy0, iy1
        self.children = None
        self.level = level
        self.keys = None
        self.ops = None

    @property
    def is_leaf(self):
        return self.children is None


def build_tree(nx: int, ny: int, tie: str = "x"):
    """Binary tree over an nx x ny uniform leaf grid (Sec. 2, Fig. 1).

    Boxes are listed so that a parent precedes its children (breadth first), root
    first.  A box of wx x wy leaves is halved across its longer side; ties split x
    (tie="y" splits y instead, used only to check that the result does not depend on
    the tree).  The first child (alpha) is the left / bottom half.
    """
    root = Box(0, nx, 0, ny, 0)
    boxes = [root]
    q = 0
    while q < len(boxes):
        b = boxes[q]
        q += 1
        wx, wy = b.ix1 - b.ix0, b.iy1 - b.iy0
        if wx == 1 and wy == 1:
            continue
        split_x = wx > wy or (wx == wy and tie == "x")
        if wy == 1:
            split_x = True
        if wx == 1:
            split_x = False
        if split_x:
            h = b.ix0 + wx // 2
            a = Box(b.ix0, h, b.iy0, b.iy1, b.level + 1)
            c = Box(h, b.ix1, b.iy0, b.iy1, b.level + 1)
        else:
            h = b.iy0 + wy // 2
            a = Box(b.ix0, b.ix1, b.iy0, h, b.level + 1)
            c = Box(b.ix0, b.ix1, h, b.iy1, b.level + 1)
        b.children = (a, c)
        boxes.extend([a, c])
    return boxes


def leaf_boundary_keys(ix: int, iy: int, m: int):
    """Global keys of a leaf's boundary nodes in the order [I_s, I_e, I_n, I_w].

    ('h', gy, ix, i): node i of the horizontal grid line gy inside leaf column ix;
    ('v', gx, iy, j): node j of the vertical grid line gx inside leaf row iy.
    Two leaves sharing an edge produce the same keys for its nodes.
    """
    S = [("h", iy, ix, i) for i in range(m)]
    E = [("v", ix + 1, iy, j) for j in range(m)]
    N = [("h", iy + 1, ix, i) for i in range(m)]
    W = [("v", ix, iy, j) for j in range(m)]
    return S + E + N + W


def root_boundary_keys(nx: int, ny: int, m: int):
    """External order of the root boundary data t: S side (leaves ix = 0..nx-1), E side
    (iy = 0..ny-1), N side (ix ascending), W side (iy ascending); each leaf edge in
    ascending coordinate."""
    S = [("h", 0, ix, i) for ix in range(nx) for i in range(m)]
    E = [("v", nx, iy, j) for iy in range(ny) for j in range(m)]
    N = [("h", ny, ix, i) for ix in range(nx) for i in range(m)]
    W = [("v", 0, iy, j) for iy in range(ny) for j in range(m)]
    return S + E + N + W


# --------------------------------------------------------------------------------
# Merge: Sec. 2.2, eqs. (talpha), (tbeta), (out), (flux_part); Algorithm 1
# --------------------------------------------------------------------------------


def merge_operators(Ra, keys_a, Rb, keys_b):
    """Merge two sibling ItI operators by eliminating the data on their shared edge
    (Sec. 2.2).

    I_1: alpha boundary nodes not on beta; I_2: beta nodes not on alpha; I_3: the shared
    nodes (alpha's order, beta's rows matched by key).  On I_3 the incoming data of one
    box is minus the outgoing data of the other (opposite normals): t3^a = -g3^b and
    t3^b = -g3^a, with g3^a = R31^a t1 + R33^a t3^a + h3^a and g3^b = R32^b t2 +
    R33^b t3^b + h3^b (eqs. (ItIalp), (ItIbet) restricted to I_3).  Stacked, the
    interface unknowns solve

        [[I, R33^b], [R33^a, I]] [t3^a; t3^b] = [[0, -R32^b], [-R31^a, 0]] [t1; t2]
                                                + [[0, -I], [-I, 0]] [h3^a; h3^b],

    so Phi = [Phi^a; Phi^b] (the maps of eqs. (talpha), (tbeta)) and Ups = [Ups^a; Ups^b]
    (their particular parts) come from one dense solve with that matrix.  The parent's
    outgoing data g1^a = R11^a t1 + R13^a t3^a + h1^a and g2^b = R22^b t2 + R23^b t3^b
    + h2^b give R^tau and Gamma^tau (eq. (out), block diagonal).  W = I - R33^b R33^a is
    the interface matrix of eq. (talpha); W^{-1} is stored as the paper's storage policy
    (Sec. 2.4) keeps it.  Returns the parent's R in the order I_b^tau = [I_1, I_2] with
    its keys, Phi^a, Phi^b, Ups^a, Ups^b, Gamma^tau, W, W^{-1} and the blocks of R^a, R^b.
    """
    set_a, set_b = set(keys_a), set(keys_b)
    pos_b = {k: i for i, k in enumerate(keys_b)}
    i1 = np.array([i for i, k in enumerate(keys_a) if k not in set_b], dtype=int)
    i3a = np.array([i for i, k in enumerate(keys_a) if k in set_b], dtype=int)
    i3b = np.array([pos_b[keys_a[i]] for i in i3a], dtype=int)
    i2 = np.array([i for i, k in enumerate(keys_b) if k not in set_a], dtype=int)
    R11a, R13a = Ra[np.ix_(i1, i1)], Ra[np.ix_(i1, i3a)]
    R31a, R33a = Ra[np.ix_(i3a, i1)], Ra[np.ix_(i3a, i3a)]
    R22b, R23b = Rb[np.ix_(i2, i2)], Rb[np.ix_(i2, i3b)]
    R32b, R33b = Rb[np.ix_(i3b, i2)], Rb[np.ix_(i3b, i3b)]
    n1, n2, n3 = len(i1), len(i2), len(i3a)
    I3 = np.eye(n3)
    # the stacked interface system: unknowns [t3^a; t3^b], data columns [t1, t2, h3^a, h3^b]
    M = np.block([[I3, R33b], [R33a, I3]])
    rhs = np.zeros((2 * n3, n1 + n2 + 2 * n3), dtype=complex)
    rhs[:n3, n1:n1 + n2] = -R32b
    rhs[n3:, :n1] = -R31a
    rhs[n3:, n1 + n2:n1 + n2 + n3] = -I3
    rhs[:n3, n1 + n2 + n3:] = -I3
    X = np.linalg.solve(M, rhs)
    Phi_a, Phi_b = X[:n3, :n1 + n2], X[n3:, :n1 + n2]
    Ups_a, Ups_b = X[:n3, n1 + n2:], X[n3:, n1 + n2:]
    W = I3 - R33b @ R33a
    Winv = np.linalg.inv(W)
    # eq. (out): R^tau = blockdiag(R11a, R22b) + blockdiag(R13a, R23b) [Phi^a; Phi^b]
    R_tau = np.zeros((n1 + n2, n1 + n2), dtype=complex)
    R_tau[:n1, :n1] = R11a
    R_tau[n1:, n1:] = R22b
    R_tau[:n1] += R13a @ Phi_a
    R_tau[n1:] += R23b @ Phi_b
    Gamma_tau = np.vstack([R13a @ Ups_a, R23b @ Ups_b])
    keys_tau = [keys_a[i] for i in i1] + [keys_b[i] for i in i2]
    return dict(R=R_tau, keys=keys_tau, Phi_a=Phi_a, Phi_b=Phi_b, Ups_a=Ups_a,
                Ups_b=Ups_b, Gamma=Gamma_tau, W=W, Winv=Winv, i1=i1, i2=i2, i3a=i3a,
                i3b=i3b, R33a=R33a, R33b=R33b, R13a=R13a, R23b=R23b, R31a=R31a,
                R32b=R32b, R11a=R11a, R22b=R22b)


# --------------------------------------------------------------------------------
# Whole problem: Algorithm 1 (build) and Algorithm 2 (solve)
# --------------------------------------------------------------------------------


class Problem:
    """Uniform nx x ny leaves on [x0,x1] x [y0,y1], p points per direction per leaf."""

    def __init__(self, x0, x1, y0, y1, nx, ny, p, kappa, eta):
        self.x0, self.x1, self.y0, self.y1 = x0, x1, y0, y1
        self.nx, self.ny, self.p = nx, ny, p
        self.kappa, self.eta = kappa, eta
        self.m = p - 2
        self.n = p * p - 4
        self.nb = 4 * p - 8
        self.ni = (p - 2) ** 2
        self.nleaf = nx * ny
        self.hx = (x1 - x0) / nx
        self.hy = (y1 - y0) / ny

    def leaf_box(self, ix, iy):
        return (self.x0 + ix * self.hx, self.x0 + (ix + 1) * self.hx,
                self.y0 + iy * self.hy, self.y0 + (iy + 1) * self.hy)

    def leaf_nodes(self) -> np.ndarray:
        """[nleaf*n, 2] leaf node coordinates, leaf l = iy*nx + ix, order I = [I_b, I_i].
        Computed once per problem (a copy is returned)."""
        if getattr(self, "_xy", None) is None:
            out = []
            for iy in range(self.ny):
                for ix in range(self.nx):
                    out.append(leaf_coordinates(*self.leaf_box(ix, iy), self.p))
            self._xy = np.concatenate(out)
        return self._xy.copy()

    def interior_nodes(self) -> np.ndarray:
        xy = self.leaf_nodes().reshape(self.nleaf, self.n, 2)
        return xy[:, self.nb:, :].reshape(-1, 2)

    def root_boundary(self):
        """Coordinates [nt, 2] and outward normals [nt, 2] of the root boundary nodes in
        the external order (S, E, N, W)."""
        xy = self.leaf_nodes().reshape(self.nleaf, self.n, 2)
        m, nx, ny = self.m, self.nx, self.ny
        pts, nrm = [], []
        for ix in range(nx):
            pts.append(xy[ix, 0:m]); nrm += [(0.0, -1.0)] * m
        for iy in range(ny):
            pts.append(xy[iy * nx + nx - 1, m:2 * m]); nrm += [(1.0, 0.0)] * m
        for ix in range(nx):
            pts.append(xy[(ny - 1) * nx + ix, 2 * m:3 * m]); nrm += [(0.0, 1.0)] * m
        for iy in range(ny):
            pts.append(xy[iy * nx, 3 * m:4 * m]); nrm += [(-1.0, 0.0)] * m
        return np.concatenate(pts), np.array(nrm)


# Keys of a leaf's operators that the merges and the solve read (the other pieces of
# leaf_operators are only for the identity pins).
_LEAF_KEEP = ("Psi", "Y", "R", "Gamma")


def _each(fn, items):
    """fn over independent items (the boxes of one tree level).  Wide levels run in a pool
    of host threads, each item's dense linear algebra single-threaded; narrow levels run
    one item at a time with the threaded BLAS.  Every item is computed by the same call
    either way, so the result does not depend on this choice."""
    items = list(items)
    workers = min(16, os.cpu_count() or 1)
    if len(items) < 2 * workers or workers == 1:
        return [fn(x) for x in items]
    from concurrent.futures import ThreadPoolExecutor
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # without the control the pool still gives the same results
        threadpool_limits = None
    if threadpool_limits is None:
        with ThreadPoolExecutor(workers) as ex:
            return list(ex.map(fn, items))
    with threadpool_limits(1), ThreadPoolExecutor(workers) as ex:
        return list(ex.map(fn, items))


def build(prob: Problem, c_interior: np.ndarray, tie: str = "x", progress=None):
    """Precomputation (Sec. 2, Algorithm 1): every leaf's operators (Sec. 2.1), then the
    merges of each tree level from the leaves up to the root (Sec. 2.2).

    c_interior: [nleaf * n_i] real or complex samples of c at the interior nodes,
    leaf-major in leaf order l = iy*nx + ix.  Returns the list of boxes (root first);
    each box carries its operators in box.ops and its boundary keys in box.keys.
    progress, if given, is called with (level, boxes on the level) after each level.
    """
    boxes = build_tree(prob.nx, prob.ny, tie)
    cI = np.asarray(c_interior).reshape(prob.nleaf, prob.ni)
    by_level = {}
    for b in boxes:
        by_level.setdefault(b.level, []).append(b)

    def leaf(b):
        ix, iy = b.ix0, b.iy0
        ops = leaf_operators(*prob.leaf_box(ix, iy), prob.p, prob.kappa, prob.eta,
                             cI[iy * prob.nx + ix])
        return {k: ops[k] for k in _LEAF_KEEP}

    def merge(b):
        a, c = b.children
        return merge_operators(a.ops["R"], a.keys, c.ops["R"], c.keys)

    for lev in sorted(by_level, reverse=True):
        level = by_level[lev]
        leaves = [b for b in level if b.is_leaf]
        for b, ops in zip(leaves, _each(leaf, leaves)):
            b.ops = ops
            b.keys = leaf_boundary_keys(b.ix0, b.iy0, prob.m)
        parents = [b for b in level if not b.is_leaf]
        for b, mo in zip(parents, _each(merge, parents)):
            b.ops = mo
            b.keys = mo["keys"]
        if progress is not None:
            progress(lev, len(level))
    return boxes


def shared_rows(prob: Problem):
    """Owners of every boundary node key: key -> [(leaf, position in I_b), ...] (two
    owners for a node on an edge shared by two leaves, one on the outer boundary)."""
    owner = {}
    for iy in range(prob.ny):
        for ix in range(prob.nx):
            l = iy * prob.nx + ix
            for r, k in enumerate(leaf_boundary_keys(ix, iy, prob.m)):
                owner.setdefault(k, []).append((l, r))
    return owner


def solve(prob: Problem, boxes, s, t, upward=True, jumps=None):
    """Solve stage (Sec. 2, Algorithm 2) for one or several right-hand sides: an upward
    pass that carries the body load's particular parts from the leaves to the root, then
    a downward pass that turns the root's boundary data into every box's incoming data
    and finally every leaf's solution.

    s: [nrhs, nleaf*n_i] body load at interior nodes (or None for s = 0, which skips
       the upward pass as Sec. 2 allows), t: [nrhs, nt] impedance data on the root
       boundary in the external order.  Returns u: [nrhs, nleaf*n] at all leaf nodes.

    jumps (not in the paper; used by residual correction): [nrhs, nleaf, nb] right-hand
    sides of the shared-edge rows of the global system, i.e. on a node shared by leaves
    l (position r) and l' the row F_l u_l + G_l' u_l' = jumps[:, l, r]; entries at outer
    boundary positions are ignored.  At a merge the interface conditions then read
    t3^a = -g3^b + j1 and t3^b = -g3^a + j2 (j1 from alpha's row, j2 from beta's), which is
    the elimination of eqs. (talpha)/(tbeta) with h3^b replaced by h3^b - j1 and h3^a by
    h3^a - j2 wherever the particular parts are formed.
    """
    t = np.atleast_2d(np.asarray(t, dtype=complex))
    nrhs = t.shape[0]
    if s is None:
        upward = jumps is not None
        s = np.zeros((nrhs, prob.nleaf * prob.ni), dtype=complex)
    s = np.atleast_2d(np.asarray(s, dtype=complex)).reshape(nrhs, prob.nleaf, prob.ni)
    if jumps is not None:
        jumps = np.asarray(jumps, dtype=complex).reshape(nrhs, prob.nleaf, prob.nb)
        owner = shared_rows(prob)
    utilde, h, ttil_a, ttil_b = {}, {}, {}, {}
    # Upward pass: particular solutions of the leaves (eq. (particular)), then at every
    # merge the particular parts of the shared-edge data and of the parent's outgoing data.
    for b in reversed(boxes):
        if b.is_leaf:
            l = b.iy0 * prob.nx + b.ix0
            sl = s[:, l, :].T                                      # [ni, nrhs]
            if upward:
                utilde[id(b)] = b.ops["Y"] @ sl                    # eq. (prtsolnopdef)
                h[id(b)] = b.ops["Gamma"] @ sl
            else:
                utilde[id(b)] = np.zeros((prob.n, nrhs), dtype=complex)
                h[id(b)] = np.zeros((prob.nb, nrhs), dtype=complex)
        else:
            a, c = b.children
            o = b.ops
            h3 = np.vstack([h[id(a)][o["i3a"]], h[id(c)][o["i3b"]]])
            if jumps is not None:
                n3 = len(o["i3a"])
                for q, ka in enumerate(o["i3a"]):
                    key = a.keys[ka]
                    (l1, r1), (l2, r2) = owner[key]
                    in_a = a.ix0 <= l1 % prob.nx < a.ix1 and a.iy0 <= l1 // prob.nx < a.iy1
                    (la, ra), (lb, rb) = ((l1, r1), (l2, r2)) if in_a else ((l2, r2), (l1, r1))
                    h3[q] -= jumps[:, lb, rb]                      # h3^a - j2
                    h3[n3 + q] -= jumps[:, la, ra]                 # h3^b - j1
            ttil_a[id(b)] = o["Ups_a"] @ h3                        # eqs. (talpha), (tbeta)
            ttil_b[id(b)] = o["Ups_b"] @ h3
            h12 = np.vstack([h[id(a)][o["i1"]], h[id(c)][o["i2"]]])
            h[id(b)] = h12 + o["Gamma"] @ h3                       # eq. (flux_part)
    # Downward pass: the root takes the boundary data; each merge maps its incoming data
    # to the children's shared-edge data (eqs. (talpha), (tbeta)); each leaf forms its
    # solution from its incoming data (eq. (hmgsolnopdef)) plus its particular part.
    root = boxes[0]
    rkeys = root_boundary_keys(prob.nx, prob.ny, prob.m)
    rpos = {k: i for i, k in enumerate(rkeys)}
    tin = {id(root): t.T[[rpos[k] for k in root.keys]]}            # root: the BVP data
    u = np.zeros((nrhs, prob.nleaf, prob.n), dtype=complex)
    for b in boxes:
        tb = tin[id(b)]
        if b.is_leaf:
            l = b.iy0 * prob.nx + b.ix0
            u[:, l, :] = (b.ops["Psi"] @ tb + utilde[id(b)]).T
        else:
            a, c = b.children
            o = b.ops
            n1 = len(o["i1"])
            t3a = o["Phi_a"] @ tb + ttil_a[id(b)]
            t3b = o["Phi_b"] @ tb + ttil_b[id(b)]
            ta = np.zeros((len(a.keys), nrhs), dtype=complex)
            ta[o["i1"]] = tb[:n1]
            ta[o["i3a"]] = t3a
            tc = np.zeros((len(c.keys), nrhs), dtype=complex)
            tc[o["i2"]] = tb[n1:]
            tc[o["i3b"]] = t3b
            tin[id(a)] = ta
            tin[id(c)] = tc
    return u.reshape(nrhs, -1)


# --------------------------------------------------------------------------------
# The global discrete system that HPS eliminates exactly (used for tiny grids)
# --------------------------------------------------------------------------------


def global_system(prob: Problem, c_interior):
    """Dense assembly of the discrete system whose solution HPS computes.

    Unknowns: every leaf's n nodal values (a node on a shared edge has one copy per
    adjacent leaf).  Rows of leaf l: its interior collocation rows Ahat(I_i, I) u_l = s;
    for each boundary node on the outer boundary, the impedance row F u_l = t; for
    each node of an edge shared with leaf l', the matching row F_l u_l + G_l' u_l' = 0
    (Sec. 2.2: incoming data of one box is minus the outgoing data of its neighbour,
    because the normals are opposite).  Returns (A, leaf ops list).
    """
    nl, n, nb, m = prob.nleaf, prob.n, prob.nb, prob.m
    cI = np.asarray(c_interior).reshape(nl, prob.ni)
    ops = []
    for iy in range(prob.ny):
        for ix in range(prob.nx):
            ops.append(leaf_operators(*prob.leaf_box(ix, iy), prob.p, prob.kappa, prob.eta,
                                      cI[iy * prob.nx + ix]))
    A = np.zeros((nl * n, nl * n), dtype=complex)
    owner = {}
    for iy in range(prob.ny):
        for ix in range(prob.nx):
            l = iy * prob.nx + ix
            for r, k in enumerate(leaf_boundary_keys(ix, iy, m)):
                owner.setdefault(k, []).append((l, r))
    for l in range(nl):
        A[l * n + nb:(l + 1) * n, l * n:(l + 1) * n] = ops[l]["Ahat_iI"]
    for k, lst in owner.items():
        if len(lst) == 1:
            l, r = lst[0]
            A[l * n + r, l * n:(l + 1) * n] = ops[l]["F"][r]
        else:
            (l1, r1), (l2, r2) = lst
            A[l1 * n + r1, l1 * n:(l1 + 1) * n] = ops[l1]["F"][r1]
            A[l1 * n + r1, l2 * n:(l2 + 1) * n] = ops[l2]["G"][r2]
            A[l2 * n + r2, l2 * n:(l2 + 1) * n] = ops[l2]["F"][r2]
            A[l2 * n + r2, l1 * n:(l1 + 1) * n] = ops[l1]["G"][r1]
    return A


def global_rhs(prob: Problem, s, t, jumps=None):
    """Right-hand side of the global system for body load s, root data t and (optional)
    right-hand sides of the shared-edge rows, jumps[:, l, r] as in solve()."""
    nl, n, nb, m = prob.nleaf, prob.n, prob.nb, prob.m
    t = np.atleast_2d(t)
    nrhs = t.shape[0]
    s = np.zeros((nrhs, nl * prob.ni), dtype=complex) if s is None else np.atleast_2d(s)
    s = s.reshape(nrhs, nl, prob.ni)
    rkeys = root_boundary_keys(prob.nx, prob.ny, m)
    rpos = {k: i for i, k in enumerate(rkeys)}
    b = np.zeros((nrhs, nl, n), dtype=complex)
    b[:, :, nb:] = s
    if jumps is not None:
        jumps = np.asarray(jumps, dtype=complex).reshape(nrhs, nl, nb)
    for iy in range(prob.ny):
        for ix in range(prob.nx):
            l = iy * prob.nx + ix
            for r, k in enumerate(leaf_boundary_keys(ix, iy, m)):
                if k in rpos:
                    b[:, l, r] = t[:, rpos[k]]
                elif jumps is not None:
                    b[:, l, r] = jumps[:, l, r]
    return b.reshape(nrhs, -1)


def global_solve(prob: Problem, c_interior, s, t, jumps=None):
    """Dense LU solve of the global system (tiny grids only)."""
    A = global_system(prob, c_interior)
    rhs = global_rhs(prob, s, t, jumps)
    return np.linalg.solve(A, rhs.T).T


def global_residual(prob: Problem, c_interior, s, t, u, jumps=None):
    """Residual b - A u of the global system, row by row and leaf by leaf (no dense
    assembly), in the layout of the global rows: [nrhs, nleaf, n] with positions
    [I_b, I_i] of each leaf.

    Interior rows: s - Ahat(I_i, I) u_l.  Outer boundary rows: t - F u_l.  Shared-edge
    rows (node shared by leaves l, l'): jumps - (F_l u_l + G_l' u_l') (jumps = 0 if not
    given).  Used for FP64 residual correction of a reduced-precision solve.
    """
    nl, n, nb, ni, m = prob.nleaf, prob.n, prob.nb, prob.ni, prob.m
    u = np.atleast_2d(np.asarray(u, dtype=complex))
    nrhs = u.shape[0]
    u = u.reshape(nrhs, nl, n)
    b = global_rhs(prob, s, t, jumps).reshape(nrhs, nl, n)
    cI = np.asarray(c_interior).reshape(nl, ni)
    ops = []
    for iy in range(prob.ny):
        for ix in range(prob.nx):
            ops.append(leaf_operators(*prob.leaf_box(ix, iy), prob.p, prob.kappa, prob.eta,
                                      cI[iy * prob.nx + ix]))
    r = np.zeros((nrhs, nl, n), dtype=complex)
    for l in range(nl):
        r[:, l, nb:] = b[:, l, nb:] - (ops[l]["Ahat_iI"] @ u[:, l, :].T).T
    for key, lst in shared_rows(prob).items():
        if len(lst) == 1:
            l, rr = lst[0]
            r[:, l, rr] = b[:, l, rr] - u[:, l, :] @ ops[l]["F"][rr]
        else:
            (l1, r1), (l2, r2) = lst
            r[:, l1, r1] = b[:, l1, r1] - (u[:, l1, :] @ ops[l1]["F"][r1] +
                                           u[:, l2, :] @ ops[l2]["G"][r2])
            r[:, l2, r2] = b[:, l2, r2] - (u[:, l2, :] @ ops[l2]["F"][r2] +
                                           u[:, l1, :] @ ops[l1]["G"][r1])
    return r


def correction_rhs(prob: Problem, r):
    """Split a global residual [nrhs, nleaf, n] into the (s, t, jumps) right-hand side of
    the correction solve: interior rows -> s, outer boundary rows -> t (external order),
    shared-edge rows -> jumps."""
    nl, n, nb, m = prob.nleaf, prob.n, prob.nb, prob.m
    r = np.asarray(r).reshape(-1, nl, n)
    s = r[:, :, nb:].reshape(r.shape[0], -1)
    rkeys = root_boundary_keys(prob.nx, prob.ny, m)
    t = np.zeros((r.shape[0], len(rkeys)), dtype=complex)
    owner = shared_rows(prob)
    for q, k in enumerate(rkeys):
        l, rr = owner[k][0]
        t[:, q] = r[:, l, rr]
    jumps = r[:, :, :nb].copy()
    return s, t, jumps


# --------------------------------------------------------------------------------
# Error measures (Sec. 4.1 defines e_inf; rel. L2 is the stated parity measure)
# --------------------------------------------------------------------------------


def rel_l2(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def e_inf(a, b):
    return float(np.max(np.abs(np.asarray(a).ravel() - np.asarray(b).ravel())))
