"""Oracle: the SPD structure of the embedded-boundary operator (Sec. 2.4).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* D^(n)(a, b): the n x n 1-D segment matrix with end entries a, b, interior
  diagonal 2 and off-diagonals -1 (Sec. 2.4, Eq. (tridiag)).
* lemma_conditions(n, a, b): the sufficient conditions of Lemma 2.1 as stated
  in Sec. 2.4 (n = 1: a > 0; n = 2: a > 0 and ab > 1; n >= 3: a, b > (n-2)/(n-1)
  and a > ((n-2) b - (n-3)) / ((n-1) b - (n-2))).  The appendix restates the
  last inequality in a garbled form; the lemma statement is used.
* corollary_conditions(a, b): a > 1 and b > 1 (Corollary 1).
* axis_matrix(asm, axis): the block-diagonal matrix D_xx (or D_yy, D_zz) of
  Theorems 1-2: for every maximal run of consecutive unknowns along a grid
  line, the segment matrix whose diagonal is the part of a_k contributed by
  the two sides along that axis.  Theorem 2 states that h^2 A is the sum of
  these per-axis matrices (permuted back to lexicographic order).

* segment_check(kind, cut_node, cut_dir, cut_c): the a-priori test that
  Sec. 2.4 builds from these pieces: along every axis, every maximal run of
  computational points on a grid line is one segment; its length n and end
  entries a, b (the part of the diagonal from the two sides along that axis)
  must satisfy Lemma 2.1, and then the operator is SPD (Theorems 1-2).  Works
  from the node kinds and the cut records, so that records with altered c can
  be checked too.  Returns (segments, failing segments).

Parity: pinned by tests/test_oracle_spd.py (brute-force eigenvalues of random
segment matrices against the lemma; exact reconstruction of h^2 A from the
per-axis blocks; segment counts against a count of run starts; a passing
check on altered records against the eigenvalues of the per-axis operator it
describes; a hand-built failing segment that is indefinite).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .eb_assembly import COMPUTATIONAL, _strides, directions


def segment_matrix(n, a, b):
    """D^(n)(a, b) as a dense array."""
    if n == 1:
        return np.array([[float(a)]])
    D = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    D[0, 0] = a
    D[-1, -1] = b
    return D


def lemma_conditions(n, a, b):
    """Sufficient conditions of Lemma 2.1 for D^(n)(a, b) to be SPD."""
    if n == 1:
        return a > 0
    if n == 2:
        return a > 0 and a * b > 1
    lo = (n - 2) / (n - 1)
    if not (a > lo and b > lo):
        return False
    return a > ((n - 2) * b - (n - 3)) / ((n - 1) * b - (n - 2))


def corollary_conditions(a, b):
    """Corollary 1: a > 1 and b > 1 suffice."""
    return a > 1 and b > 1


def axis_part_of_diagonal(asm, phys_axis):
    """Contribution of the two sides along one axis to each a_k.

    A computational neighbour contributes 1, a BP side the sum of its records'
    c (c = 1/q for a line-by-line side; c_1 + c_2 for an RBF side).
    """
    dim = asm.psi.ndim
    strides = _strides(asm.psi.shape)
    kflat = asm.kind.ravel()
    part = np.zeros(asm.n_unknowns)
    cut_c = {}
    for k, s, c in zip(asm.cuts["unknown"], asm.cuts["dir"], asm.cuts["c"]):
        cut_c[(int(k), int(s))] = cut_c.get((int(k), int(s)), 0.0) + c
    for s, (ax, step, phys) in enumerate(directions(dim)):
        if phys != phys_axis:
            continue
        nb = asm.nodes + step * strides[ax]
        reg = kflat[nb] == COMPUTATIONAL
        part[reg] += 1.0
        for k in np.flatnonzero(~reg):
            part[k] += cut_c[(int(k), s)]
    return part


def line_segments(index, phys_axis):
    """Maximal runs of consecutive unknowns along grid lines of one axis.

    index is a node field holding the unknown number at computational points
    and -1 elsewhere.  Returns a list of arrays of unknown indices, each
    ordered along the axis (Sec. 2.4: the segments of D_line).
    """
    dim = index.ndim
    ax = dim - 1 - phys_axis
    idx = index
    moved = np.moveaxis(idx, ax, -1)            # lines along the last axis
    segs = []
    for line in moved.reshape(-1, moved.shape[-1]):
        run = []
        for v in line:
            if v >= 0:
                run.append(int(v))
            elif run:
                segs.append(np.array(run))
                run = []
        if run:
            segs.append(np.array(run))
    return segs


def axis_matrix(asm, phys_axis):
    """Per-axis operator D_axis in lexicographic unknown order (sparse).

    Equivalent to P^T D_line P of Theorem 2: assembled block by block from the
    1-D segment matrices D^(n)(a_seg, b_seg) of every grid-line segment.
    """
    part = axis_part_of_diagonal(asm, phys_axis)
    n = asm.n_unknowns
    rows, cols, vals = [], [], []
    blocks = []
    for seg in line_segments(asm.index, phys_axis):
        m = seg.size
        a_end, b_end = part[seg[0]], part[seg[-1]]
        D = segment_matrix(m, a_end, b_end)
        # interior diagonal entries of a segment are 2 by construction
        blocks.append((m, a_end, b_end))
        r, c = np.nonzero(D)
        rows.append(seg[r])
        cols.append(seg[c])
        vals.append(D[r, c])
    M = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return M, blocks, part


def segment_check(kind, cut_node, cut_dir, cut_c):
    """(segments, failing): Lemma 2.1 on every grid-line segment of every axis.

    kind: node field (COMPUTATIONAL marks unknowns); cut records as parallel
    arrays (flat node index, side in the order of directions(), c).
    The part of a diagonal along one axis is 0 + (minus side) + (plus side),
    each side 1 for a computational neighbour and, for a cut side, the sum of
    its records' c in record order (one record on a line-by-line side, two on
    an RBF side).
    """
    kind = np.asarray(kind)
    dim = kind.ndim
    dirs = directions(dim)
    strides = _strides(kind.shape)
    kflat = kind.ravel()
    cmap = {}
    for n, sd, c in zip(cut_node, cut_dir, cut_c):
        cmap[(int(n), int(sd))] = cmap.get((int(n), int(sd)), 0.0) + float(c)
    segments = 0
    failing = 0
    for phys in range(dim):
        sides = [sd for sd, (_, _, ph) in enumerate(dirs) if ph == phys]

        def part(node):
            v = 0.0
            for sd in sides:
                ax, step, _ = dirs[sd]
                nb = node + step * strides[ax]
                v = v + (1.0 if kflat[nb] == COMPUTATIONAL else cmap[(node, sd)])
            return v

        ax = dim - 1 - phys
        lines = np.moveaxis(np.arange(kind.size).reshape(kind.shape), ax, -1)
        for line in lines.reshape(-1, lines.shape[-1]):
            run = []
            for node in list(line) + [-1]:
                if node >= 0 and kflat[node] == COMPUTATIONAL:
                    run.append(int(node))
                    continue
                if run:
                    segments += 1
                    if not lemma_conditions(len(run), part(run[0]), part(run[-1])):
                        failing += 1
                    run = []
    return segments, failing
