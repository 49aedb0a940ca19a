"""Oracle: smoothed-aggregation AMG hierarchy and V(1,1) cycle (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper preconditions CG with algebraic multigrid (Sec. 3 preamble,
Algorithm 2 step 4) and names classical Ruge-Stueben AMG from a Julia
package; it fixes no AMG algorithm of its own.  The AMG built here is
aggregation based, and this module is the definition the GPU hierarchy is
checked against:

* Aggregates (level l -> l+1).  Every unknown carries integer grid
  coordinates (fine level: its node indices; coarse level: the box indices it
  was formed in).  Boxes are 3^d blocks of coordinates anchored at 0.  An
  aggregate is a connected component, in the graph of A_l (every stored
  off-diagonal entry is an edge), of the unknowns of one box.  Coarse
  unknowns are ordered by box (lexicographic, x fastest), then by the
  smallest member index; their coordinates are the box indices.
* P_tent(i, agg(i)) = 1.
* rho = max_i sum_j |a_ij| / a_ii (Gershgorin bound of D^-1 A, each row
  summed over its stored entries); omega = 4 / (3 rho).
* P = (I - omega D^-1 A) P_tent, with the sparsity pattern taken structurally
  (union of the patterns of P_tent and A P_tent; entries that happen to be
  zero are kept).
* R = P^T; A_{l+1} = R (A_l P), each product with structural patterns and
  sorted columns.
* Stop when n_l <= coarse_max (256), after max_levels levels, or when the next
  level would keep more than 0.6 n_l unknowns; the last level is solved by a
  dense Cholesky factorisation.
* V(1,1): z1 = omega D^-1 r; e_c = V_{l+1}(R (r - A z1)); z = z1 + P e_c;
  z = z + omega D^-1 (r - A z).  Coarsest: Cholesky solve.

Integer structures (aggregates, coarse numbering, CSR patterns) are the parity
target for the GPU bit for bit; floating-point entries are compared to a
relative tolerance.

Parity: pinned by tests/test_oracle_amg.py (brute-force connectivity and
box membership, dense products against the sparse ones, R = P^T, Galerkin
identity, symmetry, symmetric positive V-cycle).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

BOX = 3


def coo_sum_structural(rows, cols, vals, shape):
    """CSR matrix with one entry per distinct (row, col) pair, sum of its values.

    Every pair that occurs is kept even when its sum is exactly zero.  Columns
    are sorted within rows; duplicates are summed in their input order.
    """
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    if rows.size == 0:
        return sp.csr_matrix(shape)
    order = np.lexsort((cols, rows))            # stable: ties keep input order
    r, c, v = rows[order], cols[order], vals[order]
    first = np.ones(r.size, dtype=bool)
    first[1:] = (r[1:] != r[:-1]) | (c[1:] != c[:-1])
    starts = np.flatnonzero(first)
    # sequential summation of each run (plain loop over run lengths)
    sums = np.add.reduceat(v, starts)
    ur, uc = r[starts], c[starts]
    indptr = np.zeros(shape[0] + 1, dtype=np.int64)
    np.add.at(indptr, ur + 1, 1)
    indptr = np.cumsum(indptr)
    M = sp.csr_matrix((sums, uc, indptr), shape=shape)
    M.has_sorted_indices = True
    return M


def spgemm(A, B):
    """C = A B with the structural pattern (every product pair contributes).

    Row-wise expansion: entry (i, j) of C sums a_ik b_kj over k in
    ascending order.
    """
    A = sp.csr_matrix(A)
    B = sp.csr_matrix(B)
    A.sort_indices()
    B.sort_indices()
    Ac = A.tocoo()
    ai, ak, av = Ac.row.astype(np.int64), Ac.col.astype(np.int64), Ac.data
    # coo of a CSR matrix is row-major with sorted columns
    blen = np.diff(B.indptr)[ak]
    total = int(blen.sum())
    rows = np.repeat(ai, blen)
    avals = np.repeat(av, blen)
    start = np.repeat(B.indptr[ak], blen)
    seg_first = np.repeat(np.cumsum(blen) - blen, blen)
    pos = start + (np.arange(total) - seg_first)
    cols = B.indices[pos].astype(np.int64)
    vals = avals * B.data[pos]
    return coo_sum_structural(rows, cols, vals, (A.shape[0], B.shape[1]))


def box_keys(coords):
    """Box coordinates (coords // 3) per unknown."""
    return np.asarray(coords, dtype=np.int64) // BOX


def aggregate(A, coords):
    """Box-component aggregation.  Returns (agg, coarse_coords)."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    box = box_keys(coords)
    dim = box.shape[1]
    coo = A.tocoo()
    same = np.all(box[coo.row] == box[coo.col], axis=1) & (coo.row != coo.col)
    G = sp.csr_matrix((np.ones(int(same.sum())), (coo.row[same], coo.col[same])), shape=(n, n))
    ncomp, label = connected_components(G, directed=False)
    min_member = np.full(ncomp, n, dtype=np.int64)
    np.minimum.at(min_member, label, np.arange(n))
    rep_box = box[min_member]
    # order: box lexicographic with x fastest (z, then y, then x), then min member
    keys = [min_member] + [rep_box[:, p] for p in range(dim)]
    order = np.lexsort(tuple(keys))
    rank = np.empty(ncomp, dtype=np.int64)
    rank[order] = np.arange(ncomp)
    agg = rank[label]
    coarse_coords = rep_box[order]
    return agg, coarse_coords


def tentative_prolongator(agg, nc):
    n = agg.size
    return sp.csr_matrix((np.ones(n), (np.arange(n), agg)), shape=(n, nc))


def gershgorin_rho(A):
    """max_i sum_j |a_ij| / a_ii over stored entries."""
    A = sp.csr_matrix(A)
    diag = A.diagonal()
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    rowsum = np.zeros(A.shape[0])
    np.add.at(rowsum, rows, np.abs(A.data))
    return float(np.max(rowsum / diag))


def smoothed_prolongator(A, agg, nc, omega):
    """P = (I - omega D^-1 A) P_tent with the structural pattern."""
    A = sp.csr_matrix(A)
    A.sort_indices()
    n = A.shape[0]
    diag = A.diagonal()
    coo = A.tocoo()
    r = coo.row.astype(np.int64)
    c = coo.col.astype(np.int64)
    smooth_vals = -omega * (coo.data / diag[r])
    rows = np.concatenate([np.arange(n), r])
    cols = np.concatenate([agg, agg[c]])
    vals = np.concatenate([np.ones(n), smooth_vals])
    return coo_sum_structural(rows, cols, vals, (n, nc))


@dataclass
class Level:
    A: sp.csr_matrix
    coords: np.ndarray
    diag: np.ndarray
    omega: float = 0.0
    rho: float = 0.0
    agg: Optional[np.ndarray] = None
    P: Optional[sp.csr_matrix] = None
    R: Optional[sp.csr_matrix] = None
    chol: Optional[np.ndarray] = None      # lower Cholesky factor (coarsest only)

    @property
    def n(self):
        return self.A.shape[0]


@dataclass
class Hierarchy:
    levels: List[Level] = field(default_factory=list)

    @property
    def n_levels(self):
        return len(self.levels)


def build_hierarchy(A0, coords0, coarse_max=256, max_levels=16, min_reduction=0.6,
                    dense_limit=8192):
    """Build the smoothed-aggregation hierarchy of A0."""
    H = Hierarchy()
    A = sp.csr_matrix(A0)
    A.sort_indices()
    coords = np.asarray(coords0, dtype=np.int64)
    while True:
        lvl = Level(A=A, coords=coords, diag=A.diagonal().copy())
        H.levels.append(lvl)
        n = A.shape[0]
        coarsest = n <= coarse_max or len(H.levels) >= max_levels
        if not coarsest:
            agg, cc = aggregate(A, coords)
            nc = cc.shape[0]
            if nc > min_reduction * n:
                coarsest = True
        if coarsest:
            if n > dense_limit:
                raise RuntimeError(f"coarsest level too large for a dense solve ({n})")
            if n > 0:
                lvl.chol = sla.cholesky(A.toarray(), lower=True)
            return H
        lvl.rho = gershgorin_rho(A)
        lvl.omega = 4.0 / (3.0 * lvl.rho)
        lvl.agg = agg
        lvl.P = smoothed_prolongator(A, agg, nc, lvl.omega)
        lvl.R = lvl.P.T.tocsr()
        lvl.R.sort_indices()
        A = spgemm(lvl.R, spgemm(A, lvl.P))
        coords = cc


def coarse_solve(lvl, r):
    return sla.cho_solve((lvl.chol, True), r)


def vcycle(H, r, level=0):
    """One V(1,1) cycle with weighted Jacobi smoothing: returns z = M r."""
    lvl = H.levels[level]
    if lvl.chol is not None:
        return coarse_solve(lvl, r)
    if lvl.n == 0:
        return np.zeros(0)
    z1 = lvl.omega * (r / lvl.diag)
    rc = lvl.R @ (r - lvl.A @ z1)
    ec = vcycle(H, rc, level + 1)
    z = z1 + lvl.P @ ec
    z = z + lvl.omega * ((r - lvl.A @ z) / lvl.diag)
    return z


def hierarchy_summary(H):
    return [dict(n=l.n, nnz=int(l.A.nnz),
                 nnz_P=(int(l.P.nnz) if l.P is not None else 0),
                 rho=l.rho, omega=l.omega) for l in H.levels]
