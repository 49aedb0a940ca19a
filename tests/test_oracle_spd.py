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
