"""Oracle: embedded-boundary discretisation of -Laplace (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

What is computed, and where the paper defines it:

* mask m = [psi < 0]                                    Sec. 2, mask grid function
* boundary point (BP): inside with >= 1 of its 2d nearest
  neighbours outside; computational point: inside with all
  2d neighbours inside                                  Sec. 2, BP definition
* unknowns = computational points in lexicographic order,
  x fastest                                             Algorithm 2 step 1; Sec. 2.4
* the central difference (beta = 1)                     Sec. 2, Eq. (central_difference)
* the value at a BP used by a computational point is the
  linear interpolant between the computational point and
  the boundary crossing on the same grid line; only the
  diagonal and the right-hand side change             Sec. 2.1.1, interpolant and u_BP
* crossing location by linear interpolation of psi      Sec. 3.3, distance approximation
* RBF rows (2-D): the BP value is the polynomial-augmented
  RBF interpolant (phi(r) = r^3, linear polynomials) through
  the computational point and two boundary points chosen by
  the closest-point rule with the pi/4 rotation          Sec. 2.2, Eq. (rbf), (rbf_ubp);
                                                        Algorithm 1; phi from Sec. 3
* variable conductivity beta (Eq. (1)): each side of the stencil carries
  the face value beta_{i+-1/2}; a computational neighbour contributes
  beta_f to a_k and -beta_f / h^2 off the diagonal, a BP side beta_f times
  its interpolation weight(s) to a_k and to the records' c   Eq. (central_difference)
* strategy: "line" (extended line-by-line everywhere),
  "mixed" (line-by-line where the node two steps out is
  outside, RBF otherwise), "rbf" (RBF on every BP side)  Sec. 2.3; Algorithm 2 step 3

Readings taken where the paper leaves a choice:

* inside is psi < 0 strictly; psi == 0 is outside.
* the outer node layer must be outside (DomainError otherwise).
* mode "line": when the node two steps beyond the computational point is
  itself inside (Algorithm 2 would switch to RBF interpolation there), the
  grid line is walked on to the first outside node and the same two-point
  line interpolation is used ("extended line-by-line").  The weights stay in
  [0, 1], so the matrix stays symmetric and diagonally dominant.
* RBF rows are defined for 2-D only (the paper's method is 2-D).
* Gamma, for the closest-point and intersection searches of Algorithm 1, is
  the zero set of the piecewise-linear interpolant of the nodal psi on the
  triangles that split every grid cell along its diagonal from node (i, j)
  to node (i+1, j+1).  On grid lines it passes through the same crossings as
  the line-by-line rows.  Inside a triangle with one or two inside vertices
  it is one segment, from the first to the second crossed edge in the edge
  order (v0 v1), (v1 v2), (v2 v0).
* Gamma_l (the part of Gamma searched) is Gamma inside the 6h x 6h window of
  cells whose lower-left corners are at offsets -3..2 from the computational
  point.  The BP lies within h of Gamma (its outside neighbour's edge is
  crossed) and the computational point within 2h, so both closest points
  over all of Gamma lie in this window.  Ties go to the first segment in the
  order cell row, cell column, lower triangle (v (i,j), (i+1,j), (i+1,j+1))
  before upper ((i,j), (i+1,j+1), (i,j+1)).
* The rotated line of Algorithm 1 is taken as the ray from x_BP in the
  direction of x_Gamma1 - x_BP turned counterclockwise by pi/4; x_Gamma2 is
  its nearest crossing of Gamma anywhere on the grid (where the boundary
  turns, as between the arms of a star, the ray can run almost along it for
  many cells).  psi is negative at x_BP and the outer layer is outside, so a
  crossing always exists.  Three collinear interpolation points raise
  GeometryError.
* epsilon = 0.025 in the distinctness test (the value Sec. 2.3 reports).
* beta_{i+1/2,j} is beta at the face midpoint, sampled by the caller: `beta`
  is a (dim, *shape) array, beta[a] at a node holding the face toward +axis a
  (None: beta = 1).  a_k adds the regular sides' beta_f in direction order,
  then the records' c; with beta = 1 this is bit for bit the constant case.
* An RBF side keeps two cut records, one per boundary point, whose c is the
  interpolant's weight of that point; the side adds c_1 + c_2 (= 1 - w_ij by
  the reproduction of constants) to the diagonal and u(x_Gamma) c / h^2 per
  record to the right-hand side.  Records are sorted by (unknown, side,
  point).  A line-by-line record has steps = j >= 2; the two RBF records
  have steps = -1 and -2 and q = t = 0.

With x_Gamma at distance q*h from the computational point (q > 1), the
interpolation weights at the BP (distance h) are g_Gamma = 1/q and
g_1 = 1 - 1/q.  Substituting into the difference stencil turns the
neighbour term into a diagonal contribution c = 1/q and a right-hand-side
term u_Gamma / (q h^2).  The dimensionless diagonal is therefore

    a_k = (number of computational neighbours) + sum over BP sides of 1/q

and A = -L_h = (1/h^2) (diag(a) - adjacency) (+ sigma I for a shifted solve).

Floating-point order for a_k (so that an independent implementation can be
bit-exact): t = psi_in / (psi_in - psi_out); q = (j - 1) + t; c = 1 / q;
a_k = float(n_regular), then a_k += c for each record of the unknown in
record order (sides -x, +x, -y, +y, -z, +z; an RBF side's two points in
order).

Parity: pinned by tests/test_oracle_assembly.py (brute-force classification,
planar-boundary crossing exactness, exactness on linear functions, symmetry,
diagonal dominance, second-order convergence, small-cell spectrum bound) and
tests/test_oracle_rbf.py (RBF weights against barycentric coordinates and
linear reproduction; window closest points against a search over every
triangle of the grid and against the orthogonal projection onto a planar
boundary; the rotation step on a boundary perpendicular to the grid line;
exactness on linear functions and second-order convergence with RBF rows).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

OUTSIDE, BOUNDARY, COMPUTATIONAL = 0, 1, 2


class DomainError(ValueError):
    """The domain touches the outermost node layer."""


def directions(dim):
    """Direction list in the fixed order (-x, +x, -y, +y, -z, +z).

    Each entry is (numpy_axis, step, physical_axis); numpy axis order is
    [z, y, x] so physical axis a lives on numpy axis dim-1-a.
    """
    out = []
    for a in range(dim):
        for step in (-1, +1):
            out.append((dim - 1 - a, step, a))
    return out


def _strides(shape):
    """Element strides of a C-ordered array of this shape."""
    st = [1] * len(shape)
    for ax in range(len(shape) - 2, -1, -1):
        st[ax] = st[ax + 1] * shape[ax + 1]
    return st


def check_outer_layer(psi):
    """Raise DomainError if any node of the outermost layer is inside."""
    inside = psi < 0
    for ax in range(psi.ndim):
        lo = np.take(inside, 0, axis=ax)
        hi = np.take(inside, psi.shape[ax] - 1, axis=ax)
        if lo.any() or hi.any():
            raise DomainError("the domain reaches the outermost node layer")


def classify(psi):
    """kind[node] in {OUTSIDE, BOUNDARY, COMPUTATIONAL} (Sec. 2 definitions)."""
    check_outer_layer(psi)
    inside = psi < 0
    all_nbrs_inside = np.ones_like(inside)
    interior = tuple(slice(1, -1) for _ in range(psi.ndim))
    for ax in range(psi.ndim):
        for step in (-1, +1):
            shifted = np.zeros_like(inside)
            src = [slice(1, -1)] * psi.ndim
            src[ax] = slice(1 + step, psi.shape[ax] - 1 + step)
            shifted[interior] = inside[tuple(src)]
            all_nbrs_inside &= shifted
    kind = np.zeros(psi.shape, dtype=np.int8)
    kind[inside] = BOUNDARY
    kind[inside & all_nbrs_inside] = COMPUTATIONAL
    return kind


def number_unknowns(kind):
    """Lexicographic numbering of computational points (x fastest).

    Returns (nodes, index): nodes[k] is the flat node index of unknown k and
    index is a node field holding k at computational points, -1 elsewhere.
    """
    nodes = np.flatnonzero(kind.ravel() == COMPUTATIONAL)
    index = np.full(kind.size, -1, dtype=np.int64)
    index[nodes] = np.arange(nodes.size)
    return nodes, index.reshape(kind.shape)


class Assembly:
    """Result of assembling the line-by-line embedded-boundary operator."""

    def __init__(self, grid, psi, kind, nodes, index, a, n_regular, cuts, beta=None):
        self.beta = beta              # face conductivities or None (beta = 1)
        self.grid = grid
        self.psi = psi
        self.kind = kind
        self.nodes = nodes            # flat node index per unknown
        self.index = index            # node field -> unknown index or -1
        self.a = a                    # dimensionless diagonal per unknown
        self.n_regular = n_regular    # computational neighbours per unknown
        self.cuts = cuts              # dict of arrays, sorted by (unknown, dir)

    @property
    def n_unknowns(self):
        return self.nodes.size

    @property
    def n_cuts(self):
        return self.cuts["unknown"].size

    def a_field(self, fill=0.0):
        out = np.full(self.kind.size, fill)
        out[self.nodes] = self.a
        return out.reshape(self.kind.shape)


MODES = ("line", "mixed", "rbf")


class GeometryError(ValueError):
    """Algorithm 1 found no second boundary point, or collinear points."""


def assemble(grid, psi, mode="line", beta=None):
    """Classify, number and build the diagonal and cut records (Algorithm 2, steps 1-3).

    mode: "line" (extended line-by-line), "mixed" or "rbf" (Sec. 2.3);
    beta: face conductivities (dim, *shape) or None for beta = 1.
    """
    if mode not in MODES:
        raise ValueError(f"unknown mode {mode!r}")
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    dim = psi.ndim
    if mode != "line" and dim != 2:
        raise NotImplementedError("RBF rows are defined for 2-D grids")
    kind = classify(psi)
    nodes, index = number_unknowns(kind)
    strides = _strides(psi.shape)
    kflat = kind.ravel()
    pflat = psi.ravel()
    nc = nodes.size

    # pass 1: count computational neighbours (exact integers)
    n_regular = np.zeros(nc, dtype=np.int64)
    for (ax, step, _a) in directions(dim):
        nb = nodes + step * strides[ax]
        n_regular += (kflat[nb] == COMPUTATIONAL)
    if beta is not None:
        beta = np.ascontiguousarray(beta, dtype=np.float64).reshape((dim,) + psi.shape)

    # pass 2: every BP side, in direction order: its records
    cut_parts = []
    coords_of = np.unravel_index(nodes, psi.shape)   # numpy-axis coordinates
    for s, (ax, step, phys) in enumerate(directions(dim)):
        nb = nodes + step * strides[ax]
        sel = np.flatnonzero(kflat[nb] != COMPUTATIONAL)   # a BP neighbour
        if sel.size == 0:
            continue
        base = nodes[sel]
        if mode == "line":
            use_rbf = np.zeros(sel.size, dtype=bool)
        elif mode == "rbf":
            use_rbf = np.ones(sel.size, dtype=bool)
        else:   # Algorithm 2 step 3: RBF when the node two steps out is inside
            use_rbf = pflat[base + 2 * step * strides[ax]] < 0
        node_xyz = np.empty((sel.size, 3))
        for p in range(3):
            if p < dim:
                ipos = coords_of[dim - 1 - p][sel].astype(np.float64)
                node_xyz[:, p] = grid.x0[p] + ipos * grid.h
            else:
                node_xyz[:, p] = 0.0
        parts = []
        ln = np.flatnonzero(~use_rbf)
        if ln.size:
            parts.append(_line_records(pflat, strides, sel[ln], base[ln], node_xyz[ln],
                                       s, ax, step, phys, grid.h))
        rb = np.flatnonzero(use_rbf)
        if rb.size:
            ij = np.stack([coords_of[1][sel[rb]], coords_of[0][sel[rb]]], axis=1)   # (i, j)
            parts.extend(_rbf_records(psi, ij, sel[rb], base[rb], node_xyz[rb], s, grid.h))
        if beta is not None:
            for part in parts:   # the side's face: node + (step < 0 ? -e : 0)
                face = part["node"] + (step * strides[ax] if step < 0 else 0)
                part["c"] = beta[phys].ravel()[face] * part["c"]
        cut_parts.extend(parts)

    keys = ("unknown", "node", "dir", "point", "steps", "t", "q", "c", "xg")
    if cut_parts:
        cuts = {k: np.concatenate([p[k] for p in cut_parts]) for k in keys}
        order = np.lexsort((cuts["point"], cuts["dir"], cuts["unknown"]))
        cuts = {k: v[order] for k, v in cuts.items()}
    else:
        cuts = dict(unknown=np.zeros(0, np.int64), node=np.zeros(0, np.int64),
                    dir=np.zeros(0, np.int64), point=np.zeros(0, np.int64),
                    steps=np.zeros(0, np.int64), t=np.zeros(0), q=np.zeros(0), c=np.zeros(0),
                    xg=np.zeros((0, 3)))
    # a_k = the regular sides' beta_f in direction order (their count for
    # beta = 1), then + c of every record of k in record order
    if beta is None:
        a = n_regular.astype(np.float64)
    else:
        a = np.zeros(nc)
        for (ax, step, phys) in directions(dim):
            nb = nodes + step * strides[ax]
            reg = kflat[nb] == COMPUTATIONAL
            face = nodes + (step * strides[ax] if step < 0 else 0)
            a = np.where(reg, a + beta[phys].ravel()[face], a)
    for k, c in zip(cuts["unknown"], cuts["c"]):
        a[k] = a[k] + c
    return Assembly(grid, psi, kind, nodes, index, a, n_regular, cuts, beta)


def _line_records(pflat, strides, sel, base, node_xyz, s, ax, step, phys, h):
    """Line-by-line records (Sec. 2.1.1): walk to the first outside node j."""
    j = np.full(sel.size, 2, dtype=np.int64)
    while True:
        still_inside = pflat[base + j * step * strides[ax]] < 0
        if not still_inside.any():
            break
        j = np.where(still_inside, j + 1, j)
    psi_in = pflat[base + (j - 1) * step * strides[ax]]
    psi_out = pflat[base + j * step * strides[ax]]
    t = psi_in / (psi_in - psi_out)
    q = (j - 1).astype(np.float64) + t
    c = 1.0 / q
    xg = node_xyz.copy()
    xg[:, phys] = xg[:, phys] + step * (q * h)
    return dict(unknown=sel.astype(np.int64), node=base.astype(np.int64),
                dir=np.full(sel.size, s, dtype=np.int64), point=np.zeros(sel.size, np.int64),
                steps=j, t=t, q=q, c=c, xg=xg)


# ------------------------------------------------------------------ RBF rows
EPS_DISTINCT = 0.025            # epsilon of the distinctness test (Sec. 2.3)
COS45 = 0.7071067811865476      # cos(pi/4) = sin(pi/4), nearest double
WINDOW_LO, WINDOW_HI = -3, 2    # lower-left cell corners of Gamma_l, offsets from x_ij
SIDE_OFFSET = {0: (-1, 0), 1: (1, 0), 2: (0, -1), 3: (0, 1)}   # BP offset per side


def rbf_phi(r):
    """Polyharmonic spline phi(r) = r^3 (Sec. 3 preamble)."""
    return r * r * r


def rbf_weights(x_ij, x_g1, x_g2, x_bp):
    """Weights (w_ij, w_G1, w_G2) with u_BP = w . (u_ij, u_G1, u_G2).

    Eq. (rbf_ubp): u_BP = (phi_BP^T, pi_BP^T) B^-1 (u, 0); B is symmetric, so
    the weights are the first three entries of B^-1 (phi_BP, pi_BP).  Solves
    the 6 x 6 system of Eq. (rbf) as printed (phi(r) = r^3, linear
    polynomials).  Inputs are (M, 2) arrays; returns (M, 3).
    """
    pts = np.stack([x_ij, x_g1, x_g2], axis=1)                 # (M, 3, 2)
    M = pts.shape[0]
    B = np.zeros((M, 6, 6))
    for a in range(3):
        for b in range(3):
            d = pts[:, a] - pts[:, b]
            B[:, a, b] = rbf_phi(np.sqrt(d[:, 0] ** 2 + d[:, 1] ** 2))
        B[:, 3, a] = B[:, a, 3] = 1.0
        B[:, 4, a] = B[:, a, 4] = pts[:, a, 0]
        B[:, 5, a] = B[:, a, 5] = pts[:, a, 1]
    rhs = np.zeros((M, 6))
    for a in range(3):
        d = x_bp - pts[:, a]
        rhs[:, a] = rbf_phi(np.sqrt(d[:, 0] ** 2 + d[:, 1] ** 2))
    rhs[:, 3] = 1.0
    rhs[:, 4] = x_bp[:, 0]
    rhs[:, 5] = x_bp[:, 1]
    sol = np.linalg.solve(B, rhs[:, :, None])[:, :, 0]
    return sol[:, :3]


def _window_segments(psi, ij, oi, oj, upper):
    """Gamma's segment in one triangle of the cell at offset (oi, oj) from each
    computational point ij (M, 2), in coordinates relative to that point in
    units of h.  Returns (valid, S0 (M, 2), S1 (M, 2))."""
    ny, nx = psi.shape
    ci = ij[:, 0] + oi
    cj = ij[:, 1] + oj
    inside_grid = (ci >= 0) & (ci + 1 <= nx - 1) & (cj >= 0) & (cj + 1 <= ny - 1)
    cic = np.clip(ci, 0, nx - 2)
    cjc = np.clip(cj, 0, ny - 2)
    if upper:
        vs = [(0, 0), (1, 1), (0, 1)]
    else:
        vs = [(0, 0), (1, 0), (1, 1)]
    vpsi = [psi[cjc + vy, cic + vx] for (vx, vy) in vs]
    vloc = [np.array([oi + vx, oj + vy], dtype=np.float64) for (vx, vy) in vs]
    crossed, pts = [], []
    for (a, b) in ((0, 1), (1, 2), (2, 0)):
        ina = vpsi[a] < 0
        inb = vpsi[b] < 0
        cr = ina != inb
        p_in = np.where(ina, vpsi[a], vpsi[b])
        p_out = np.where(ina, vpsi[b], vpsi[a])
        with np.errstate(divide="ignore", invalid="ignore"):
            t = p_in / (p_in - p_out)
        t = np.where(cr, t, 0.0)
        v_in = np.where(ina[:, None], vloc[a][None, :], vloc[b][None, :])
        v_out = np.where(ina[:, None], vloc[b][None, :], vloc[a][None, :])
        pts.append(v_in + t[:, None] * (v_out - v_in))
        crossed.append(cr)
    valid = inside_grid & (crossed[0] | crossed[1] | crossed[2])
    S0 = np.where(crossed[0][:, None], pts[0], pts[1])
    S1 = np.where(crossed[2][:, None], pts[2], pts[1])
    return valid, S0, S1


def _window_triangles(lo=WINDOW_LO, hi=WINDOW_HI):
    """Triangles of Gamma_l in search order: cell row, cell column, lower then upper."""
    for oj in range(lo, hi + 1):
        for oi in range(lo, hi + 1):
            for upper in (False, True):
                yield oi, oj, upper


def closest_point_on_segment(P, S0, S1):
    """Point of the segment [S0, S1] nearest to P, and its squared distance."""
    ex = S1[:, 0] - S0[:, 0]
    ey = S1[:, 1] - S0[:, 1]
    wx = P[:, 0] - S0[:, 0]
    wy = P[:, 1] - S0[:, 1]
    den = ex * ex + ey * ey
    num = wx * ex + wy * ey
    with np.errstate(divide="ignore", invalid="ignore"):
        tau = np.where(den > 0, num / den, 0.0)
    tau = np.where(tau < 0, 0.0, np.where(tau > 1, 1.0, tau))
    Q = np.stack([S0[:, 0] + tau * ex, S0[:, 1] + tau * ey], axis=1)
    dx = P[:, 0] - Q[:, 0]
    dy = P[:, 1] - Q[:, 1]
    return Q, dx * dx + dy * dy


def closest_points(psi, ij, P):
    """argmin over Gamma_l of |x - P| for each point P (local coordinates, (M, 2)).
    Returns (found, Q)."""
    M = ij.shape[0]
    best = np.full(M, np.inf)
    Q = np.zeros((M, 2))
    for oi, oj, upper in _window_triangles():
        valid, S0, S1 = _window_segments(psi, ij, oi, oj, upper)
        q, d2 = closest_point_on_segment(P, S0, S1)
        better = valid & (d2 < best)
        best = np.where(better, d2, best)
        Q = np.where(better[:, None], q, Q)
    return np.isfinite(best), Q


def gamma_segments(psi):
    """Every segment of Gamma on the grid, in the order cell row, cell column,
    lower triangle before upper.  Each crossing point k (0, 1) is stored as its
    inside vertex (integer node coordinates i, j), the step to the outside
    vertex (components in {-1, 0, 1}) and t, so that it can be placed relative
    to any node without rounding the node coordinates: vin - node + t * step."""
    ny, nx = psi.shape
    cj, ci = np.meshgrid(np.arange(ny - 1), np.arange(nx - 1), indexing="ij")
    ci = ci.ravel()
    cj = cj.ravel()
    parts = []
    for upper in (False, True):
        vs = [(0, 0), (1, 1), (0, 1)] if upper else [(0, 0), (1, 0), (1, 1)]
        vpsi = [psi[cj + vy, ci + vx] for (vx, vy) in vs]
        edges = []
        for (a_, b_) in ((0, 1), (1, 2), (2, 0)):
            ina = vpsi[a_] < 0
            inb = vpsi[b_] < 0
            cr = ina != inb
            p_in = np.where(ina, vpsi[a_], vpsi[b_])
            p_out = np.where(ina, vpsi[b_], vpsi[a_])
            with np.errstate(divide="ignore", invalid="ignore"):
                t = np.where(cr, p_in / (p_in - p_out), 0.0)
            va, vb = np.array(vs[a_]), np.array(vs[b_])
            vin = np.where(ina[:, None], va[None, :], vb[None, :])
            vout = np.where(ina[:, None], vb[None, :], va[None, :])
            edges.append((cr, vin + np.stack([ci, cj], 1), vout - vin, t))
        has = edges[0][0] | edges[1][0] | edges[2][0]
        first = np.where(edges[0][0], 0, 1)
        second = np.where(edges[2][0], 2, 1)
        pick = lambda e, k: np.choose(e, [edges[0][k], edges[1][k], edges[2][k]]) if edges[0][k].ndim == 1 else \
            np.where((e == 0)[:, None], edges[0][k], np.where((e == 1)[:, None], edges[1][k], edges[2][k]))
        parts.append(dict(key=(cj * (nx - 1) + ci) * 2 + int(upper),
                          vin0=pick(first, 1), d0=pick(first, 2), t0=pick(first, 3),
                          vin1=pick(second, 1), d1=pick(second, 2), t1=pick(second, 3), has=has))
    seg = {k: np.concatenate([parts[0][k], parts[1][k]]) for k in parts[0]}
    keep = np.flatnonzero(seg["has"])
    order = keep[np.argsort(seg["key"][keep], kind="stable")]
    return {k: v[order] for k, v in seg.items() if k != "has"}


def ray_hit(segs, ij, O, D):
    """Nearest crossing of Gamma by the ray O + tau D, tau > 0, from the node
    ij (O, D and the result relative to ij, units of h).  None if there is none."""
    i, j = int(ij[0]), int(ij[1])
    base0 = (segs["vin0"] - np.array([i, j])).astype(np.float64)
    base1 = (segs["vin1"] - np.array([i, j])).astype(np.float64)
    S0 = base0 + segs["t0"][:, None] * segs["d0"].astype(np.float64)
    S1 = base1 + segs["t1"][:, None] * segs["d1"].astype(np.float64)
    ex = S1[:, 0] - S0[:, 0]
    ey = S1[:, 1] - S0[:, 1]
    wx = S0[:, 0] - O[0]
    wy = S0[:, 1] - O[1]
    denom = D[0] * ey - D[1] * ex
    with np.errstate(divide="ignore", invalid="ignore"):
        tau = (wx * ey - wy * ex) / denom
        mu = (wx * D[1] - wy * D[0]) / denom
    ok = (denom != 0) & (tau > 0) & (mu >= 0) & (mu <= 1)
    if not ok.any():
        return None
    k = int(np.argmin(np.where(ok, tau, np.inf)))     # first of equal minima
    return np.array([S0[k, 0] + mu[k] * ex[k], S0[k, 1] + mu[k] * ey[k]])


def rbf_points(psi, ij, side):
    """Algorithm 1 for each computational point ij (M, 2) and its BP side.

    Returns (x_G1, x_G2) in coordinates relative to x_ij, units of h.
    """
    M = ij.shape[0]
    P_bp = np.tile(np.array(SIDE_OFFSET[side], dtype=np.float64), (M, 1))
    P_ij = np.zeros((M, 2))
    f1, G1 = closest_points(psi, ij, P_bp)
    f2, G20 = closest_points(psi, ij, P_ij)
    if not (f1.all() and f2.all()):
        raise GeometryError("no boundary segment near a boundary point")
    d = G1 - G20
    distinct = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] > EPS_DISTINCT * EPS_DISTINCT
    G2 = G20.copy()
    rot = np.flatnonzero(~distinct)
    if rot.size:
        segs = gamma_segments(psi)
        for m in rot:
            v = G1[m] - P_bp[m]
            D = np.array([COS45 * v[0] - COS45 * v[1], COS45 * v[0] + COS45 * v[1]])
            X = ray_hit(segs, ij[m], P_bp[m], D)
            if X is None:          # cannot happen with an outside outer layer
                raise GeometryError("the rotated line of Algorithm 1 meets no boundary")
            G2[m] = X
    return G1, G2


def _rbf_records(psi, ij, sel, base, node_xyz, s, h):
    """The two records of each RBF side s (Sec. 2.2): weights of x_G1, x_G2."""
    G1, G2 = rbf_points(psi, ij, s)
    cross = G1[:, 0] * G2[:, 1] - G1[:, 1] * G2[:, 0]
    if np.any(cross == 0):
        raise GeometryError("collinear RBF interpolation points")
    M = sel.size
    P_bp = np.tile(np.array(SIDE_OFFSET[s], dtype=np.float64), (M, 1))
    w = rbf_weights(np.zeros((M, 2)), G1, G2, P_bp)
    out = []
    for pt, (G, wk) in enumerate(((G1, w[:, 1]), (G2, w[:, 2]))):
        xg = node_xyz.copy()
        xg[:, 0] = xg[:, 0] + G[:, 0] * h
        xg[:, 1] = xg[:, 1] + G[:, 1] * h
        out.append(dict(unknown=sel.astype(np.int64), node=base.astype(np.int64),
                        dir=np.full(M, s, dtype=np.int64), point=np.full(M, pt, dtype=np.int64),
                        steps=np.full(M, -1 - pt, dtype=np.int64), t=np.zeros(M), q=np.zeros(M),
                        c=wk.copy(), xg=xg))
    return out


def inv_h2(grid):
    return 1.0 / (grid.h * grid.h)


def rhs(asm, f, u_at_cuts):
    """b_k = f_k + sum over the cut sides of k of u_Gamma * c / h^2 (Sec. 2.1.1).

    f is a node field; u_at_cuts holds the Dirichlet data at each cut record's
    crossing point, in cut-record order.  Sign convention: the system solved
    is A u = b with A = -L_h, for -Lap u = f.
    """
    s = inv_h2(asm.grid)
    b = np.asarray(f, dtype=np.float64).ravel()[asm.nodes].copy()
    u_at_cuts = np.asarray(u_at_cuts, dtype=np.float64)
    for k, c, u in zip(asm.cuts["unknown"], asm.cuts["c"], u_at_cuts):
        b[k] = b[k] + u * (c * s)
    return b


def cut_coordinates(asm):
    """Tuple of crossing-coordinate arrays (x, y[, z]) in cut-record order."""
    return tuple(asm.cuts["xg"][:, p] for p in range(asm.psi.ndim))


def operator_csr(asm, sigma=0.0):
    """A = (1/h^2)(diag(a) - adjacency weighted by beta_f) + sigma I as scipy
    CSR (sorted columns)."""
    s = inv_h2(asm.grid)
    nc = asm.n_unknowns
    dim = asm.psi.ndim
    strides = _strides(asm.psi.shape)
    idx = asm.index.ravel()
    rows = [np.arange(nc)]
    cols = [np.arange(nc)]
    vals = [asm.a * s + sigma]
    for (ax, step, phys) in directions(dim):
        nb = idx[asm.nodes + step * strides[ax]]
        sel = nb >= 0
        rows.append(np.flatnonzero(sel))
        cols.append(nb[sel])
        if asm.beta is None:
            vals.append(np.full(int(sel.sum()), -s))
        else:   # -beta_f / h^2 on the face toward the neighbour
            face = asm.nodes[sel] + (step * strides[ax] if step < 0 else 0)
            vals.append(-(asm.beta[phys].ravel()[face] * s))
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nc, nc))
    A.sort_indices()
    return A


def apply_operator_field(asm, x_field, sigma=0.0):
    """y = A x on node fields (x ignored off unknowns; y = 0 there)."""
    A = operator_csr(asm, sigma)
    y = np.zeros(asm.kind.size)
    y[asm.nodes] = A @ np.asarray(x_field, dtype=np.float64).ravel()[asm.nodes]
    return y.reshape(asm.kind.shape)


def unknown_coords(asm):
    """Integer grid coordinates (x, y[, z]) of each unknown, shape (N_C, dim)."""
    c = np.unravel_index(asm.nodes, asm.psi.shape)
    return np.stack([c[asm.psi.ndim - 1 - p] for p in range(asm.psi.ndim)], axis=1)


def embed(asm, v, fill=0.0):
    """Scatter an unknown vector into a node field."""
    out = np.full(asm.kind.size, fill)
    out[asm.nodes] = v
    return out.reshape(asm.kind.shape)


# ------------------------------------------------------------------ contrast
def ghost_point_diagonal(grid, psi):
    """Dimensionless diagonal of the ghost-point (exterior) treatment.

    Prior art contrasted in the Introduction: every inside node is an unknown,
    and an outside neighbour is a ghost value extrapolated linearly through the
    unknown and the crossing at distance theta*h, theta in (0, 1].  Each such
    side contributes 1/theta to the diagonal (a 1-D end row becomes 1 + 1/theta),
    the source of small-cell stiffness.  Used only as a negative control.
    Returns (nodes, diagonal, offdiag_pairs) for building the matrix.
    """
    inside = (psi < 0).ravel()
    pflat = psi.ravel()
    nodes = np.flatnonzero(inside)
    index = np.full(psi.size, -1, dtype=np.int64)
    index[nodes] = np.arange(nodes.size)
    strides = _strides(psi.shape)
    diag = np.zeros(nodes.size)
    rows, cols = [], []
    for (ax, step, _a) in directions(psi.ndim):
        nb = nodes + step * strides[ax]
        reg = inside[nb]
        diag[reg] += 1.0
        rows.append(np.flatnonzero(reg))
        cols.append(index[nb[reg]])
        g = np.flatnonzero(~reg)
        p_in = pflat[nodes[g]]
        p_out = pflat[nb[g]]
        theta = p_in / (p_in - p_out)
        diag[g] += 1.0 / theta
    return nodes, diag, (np.concatenate(rows), np.concatenate(cols))


def ghost_point_csr(grid, psi):
    nodes, diag, (r, c) = ghost_point_diagonal(grid, psi)
    n = nodes.size
    s = inv_h2(grid)
    A = sp.csr_matrix((np.concatenate([diag * s, np.full(r.size, -s)]),
                       (np.concatenate([np.arange(n), r]), np.concatenate([np.arange(n), c]))),
                      shape=(n, n))
    A.sort_indices()
    return A
