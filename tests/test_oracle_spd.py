"""Pins of the SPD criteria (Sec. 2.4, Lemma 2.1, Corollary 1, Theorems 1-2)."""
import numpy as np
import pytest

from oracle import eb_assembly as E
from oracle import spd
from paper_2204_06083_amd import workloads as W


def test_lemma_conditions_imply_spd_brute_force():
    """Every (n, a, b) that satisfies Lemma 2.1 gives a positive definite D^(n)(a,b)."""
    rng = np.random.default_rng(7)
    checked = 0
    for _ in range(4000):
        n = int(rng.integers(1, 9))
        a, b = rng.uniform(-0.5, 2.5, size=2)
        if spd.lemma_conditions(n, a, b):
            lam = np.linalg.eigvalsh(spd.segment_matrix(n, a, b))
            assert lam[0] > 0, (n, a, b, lam[0])
            checked += 1
    assert checked > 1000


def test_lemma_is_sharp_near_boundary_for_n2():
    """n = 2: a > 0, ab > 1 is exactly positive definiteness."""
    for a, b in [(0.5, 2.0 + 1e-9), (0.5, 2.0 - 1e-9), (2.0, 0.6)]:
        pd = np.linalg.eigvalsh(spd.segment_matrix(2, a, b))[0] > 0
        assert pd == spd.lemma_conditions(2, a, b)


def test_corollary_implies_lemma():
    rng = np.random.default_rng(3)
    for _ in range(2000):
        n = int(rng.integers(1, 12))
        a, b = rng.uniform(1.0 + 1e-12, 3.0, size=2)
        assert spd.corollary_conditions(a, b)
        assert spd.lemma_conditions(n, a, b)
        assert np.linalg.eigvalsh(spd.segment_matrix(n, a, b))[0] > 0


@pytest.mark.parametrize("maker", [lambda: W.disk_mms(24), lambda: W.star_poisson(40),
                                   lambda: W.ellipsoid_poisson(14)])
def test_theorem2_decomposition_and_segment_ends(maker):
    """h^2 A equals the sum of per-axis block-diagonal segment matrices; every
    segment end entry exceeds 1 (Corollary 1), so each block is SPD (Theorem 1)."""
    p = maker()
    asm = E.assemble(p.grid, p.psi)
    h2A = E.operator_csr(asm) * p.grid.h ** 2
    total = None
    for axis in range(p.grid.dim):
        M, blocks, part = spd.axis_matrix(asm, axis)
        total = M if total is None else total + M
        for (m, a_end, b_end) in blocks:
            if m == 1:
                assert spd.lemma_conditions(1, a_end, a_end)
            else:
                assert a_end > 1 and b_end > 1
                assert spd.lemma_conditions(m, a_end, b_end)
    diff = (total - h2A).tocsr()
    diff.eliminate_zeros()
    assert abs(diff).max() < 1e-14 if diff.nnz else True
    # dense positive definiteness for the small cases
    if asm.n_unknowns <= 3000:
        lam = np.linalg.eigvalsh(h2A.toarray())
        assert lam[0] > 0


def _runs_by_starts(kind):
    """Segments counted as run starts: an unknown whose predecessor along the
    axis is not one (an independent count from the node kinds)."""
    comp = np.asarray(kind) == E.COMPUTATIONAL
    total = 0
    for ax in range(comp.ndim):
        prev = np.zeros_like(comp)
        sl_dst = [slice(None)] * comp.ndim
        sl_src = [slice(None)] * comp.ndim
        sl_dst[ax] = slice(1, None)
        sl_src[ax] = slice(None, -1)
        prev[tuple(sl_dst)] = comp[tuple(sl_src)]
        total += int(np.sum(comp & ~prev))
    return total


def _records(asm):
    nodes = asm.nodes[asm.cuts["unknown"]]
    return nodes, asm.cuts["dir"], asm.cuts["c"]


@pytest.mark.parametrize("maker", [lambda: W.disk_mms(24), lambda: W.star_poisson(40),
                                   lambda: W.ellipsoid_poisson(14)])
def test_segment_check_on_assemblies(maker):
    """Line-by-line rows always pass; the segment count is the number of run
    starts along every axis."""
    p = maker()
    asm = E.assemble(p.grid, p.psi)
    segs, fail = spd.segment_check(asm.kind, *_records(asm))
    assert segs == _runs_by_starts(asm.kind)
    assert fail == 0


def _axis_operator(kind, nodes_c, dirs_c, cs, asm):
    """Sum over axes of the block-diagonal segment matrices that the records
    describe (unknown order), built with the segment matrices directly."""
    n = asm.n_unknowns
    dims = kind.ndim
    dirs = E.directions(dims)
    strides = E._strides(kind.shape)
    kflat = np.asarray(kind).ravel()
    cmap = {(int(a), int(b)): float(c) for a, b, c in zip(nodes_c, dirs_c, cs)}
    M = np.zeros((n, n))
    for phys in range(dims):
        sides = [sd for sd, (_, _, ph) in enumerate(dirs) if ph == phys]
        for seg in spd.line_segments(asm.index, phys):
            ends = []
            for k in (seg[0], seg[-1]):
                node = int(asm.nodes[k])
                v = 0.0
                for sd in sides:
                    ax, step, _ = dirs[sd]
                    nb = node + step * strides[ax]
                    v = v + (1.0 if kflat[nb] == E.COMPUTATIONAL else cmap[(node, sd)])
                ends.append(v)
            D = spd.segment_matrix(seg.size, ends[0], ends[1])
            M[np.ix_(seg, seg)] += D
    return M


@pytest.mark.parametrize("scale", [0.9, -0.3, -0.9])
def test_segment_check_on_altered_records(scale):
    """Records with c rescaled: whenever the check passes, the per-axis
    operator the records describe is positive definite.  With positive c a
    segment end is at least 1 + c (Corollary 1 holds); negative side
    contributions (as interpolation rows with negative weights give) make
    segments fail."""
    p = W.disk_mms(16)
    asm = E.assemble(p.grid, p.psi)
    nodes, dirs, c = _records(asm)
    c2 = c * scale
    segs, fail = spd.segment_check(asm.kind, nodes, dirs, c2)
    assert segs == _runs_by_starts(asm.kind)
    lam = np.linalg.eigvalsh(_axis_operator(asm.kind, nodes, dirs, c2, asm))[0]
    if fail == 0:
        assert lam > 0
    if scale > 0:
        assert fail == 0
    if scale == -0.9:
        assert fail > 0


def test_segment_check_detects_an_indefinite_segment():
    """A column of three unknowns (y-segment, n = 3) whose outer y sides
    contribute -0.7, so both segment ends are -0.7 + 1 = 0.3 < 1/2: Lemma 2.1
    fails, and D^(3)(0.3, 0.3) indeed has a negative eigenvalue.  The three
    x-segments (single nodes, two cut sides of 0.5) pass."""
    kind = np.zeros((7, 3), dtype=np.int8)
    kind[2:5, 1] = E.COMPUTATIONAL
    nodes, dirs, cs = [], [], []
    for j in (2, 3, 4):
        for sd in (0, 1):                          # -x, +x: cut sides, c = 0.5
            nodes.append(j * 3 + 1)
            dirs.append(sd)
            cs.append(0.5)
    nodes += [2 * 3 + 1, 4 * 3 + 1]                # outer y sides of the end nodes
    dirs += [2, 3]
    cs += [-0.7, -0.7]
    segs, fail = spd.segment_check(kind, nodes, dirs, cs)
    assert segs == 4 and fail == 1
    assert np.linalg.eigvalsh(spd.segment_matrix(3, 0.3, 0.3))[0] < 0
