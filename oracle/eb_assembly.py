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

Readings taken where the paper leaves a choice:

* inside is psi < 0 strictly; psi == 0 is outside.
* the outer node layer must be outside (DomainError otherwise).
* when the node two steps beyond the computational point is itself inside
  (Algorithm 2 would switch to RBF interpolation there), the grid line is
  walked on to the first outside node and the same two-point line
  interpolation is used ("extended line-by-line").  The weights stay in
  [0, 1], so the matrix stays symmetric and diagonally dominant.

With x_Gamma at distance q*h from the computational point (q > 1), the
interpolation weights at the BP (distance h) are g_Gamma = 1/q and
g_1 = 1 - 1/q.  Substituting into the difference stencil turns the
neighbour term into a diagonal contribution c = 1/q and a right-hand-side
term u_Gamma / (q h^2).  The dimensionless diagonal is therefore

    a_k = (number of computational neighbours) + sum over BP sides of 1/q

and A = -L_h = (1/h^2) (diag(a) - adjacency) (+ sigma I for a shifted solve).

Floating-point order for a_k (so that an independent implementation can be
bit-exact): t = psi_in / (psi_in - psi_out); q = (j - 1) + t; c = 1 / q;
a_k = float(n_regular), then a_k += c for each BP side in direction order
(-x, +x, -y, +y, -z, +z).

Parity: pinned by tests/test_oracle_assembly.py (brute-force classification,
planar-boundary crossing exactness, exactness on linear functions, symmetry,
diagonal dominance, second-order convergence, small-cell spectrum bound).
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

    def __init__(self, grid, psi, kind, nodes, index, a, n_regular, cuts):
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


def assemble(grid, psi):
    """Classify, number and build the diagonal and cut records (Algorithm 2, steps 1-3)."""
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    kind = classify(psi)
    nodes, index = number_unknowns(kind)
    dim = psi.ndim
    strides = _strides(psi.shape)
    kflat = kind.ravel()
    pflat = psi.ravel()
    nc = nodes.size

    # pass 1: count computational neighbours (exact integers)
    n_regular = np.zeros(nc, dtype=np.int64)
    for (ax, step, _a) in directions(dim):
        nb = nodes + step * strides[ax]
        n_regular += (kflat[nb] == COMPUTATIONAL)

    # pass 2: walk each BP side to the first outside node, in direction order
    a = n_regular.astype(np.float64)
    cut_parts = []
    coords_of = np.unravel_index(nodes, psi.shape)   # numpy-axis coordinates
    for s, (ax, step, phys) in enumerate(directions(dim)):
        nb = nodes + step * strides[ax]
        sel = np.flatnonzero(kflat[nb] != COMPUTATIONAL)   # a BP neighbour
        if sel.size == 0:
            continue
        base = nodes[sel]
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
        a[sel] = a[sel] + c
        # crossing coordinates: node coordinates, moved by q*h along the side
        xg = np.empty((sel.size, 3))
        for p in range(3):
            if p < dim:
                ipos = coords_of[dim - 1 - p][sel].astype(np.float64)
                xg[:, p] = grid.x0[p] + ipos * grid.h
            else:
                xg[:, p] = 0.0
        xg[:, phys] = xg[:, phys] + step * (q * grid.h)
        cut_parts.append(dict(unknown=sel.astype(np.int64),
                              node=base.astype(np.int64),
                              dir=np.full(sel.size, s, dtype=np.int64),
                              steps=j, t=t, q=q, c=c, xg=xg))

    if cut_parts:
        cuts = {k: np.concatenate([p[k] for p in cut_parts]) for k in cut_parts[0]}
        order = np.lexsort((cuts["dir"], cuts["unknown"]))
        cuts = {k: v[order] for k, v in cuts.items()}
    else:
        cuts = dict(unknown=np.zeros(0, np.int64), node=np.zeros(0, np.int64),
                    dir=np.zeros(0, np.int64), steps=np.zeros(0, np.int64),
                    t=np.zeros(0), q=np.zeros(0), c=np.zeros(0), xg=np.zeros((0, 3)))
    return Assembly(grid, psi, kind, nodes, index, a, n_regular, cuts)


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
    """A = (1/h^2)(diag(a) - adjacency) + sigma I as scipy CSR (sorted columns)."""
    s = inv_h2(asm.grid)
    nc = asm.n_unknowns
    dim = asm.psi.ndim
    strides = _strides(asm.psi.shape)
    idx = asm.index.ravel()
    rows = [np.arange(nc)]
    cols = [np.arange(nc)]
    vals = [asm.a * s + sigma]
    for (ax, step, _a) in directions(dim):
        nb = idx[asm.nodes + step * strides[ax]]
        sel = nb >= 0
        rows.append(np.flatnonzero(sel))
        cols.append(nb[sel])
        vals.append(np.full(int(sel.sum()), -s))
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
