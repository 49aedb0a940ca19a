"""Pins of the oracle's AMG hierarchy (aggregation, prolongator, Galerkin products, V-cycle)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import amg
from oracle import eb_assembly as E
from paper_2204_06083_amd import workloads as W


def _system(kind="star", n=48, sigma=0.0):
    p = {"star": lambda: W.star_poisson(n), "disk": lambda: W.disk_mms(n),
         "ell": lambda: W.ellipsoid_poisson(n)}[kind]()
    asm = E.assemble(p.grid, p.psi)
    return E.operator_csr(asm, sigma), E.unknown_coords(asm), asm


def _brute_aggregates_ok(A, coords, agg, cc):
    """Brute force: partition, within one box, connected, maximal, ordered."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    nc = cc.shape[0]
    box = [tuple(c // 3) for c in coords]
    assert agg.min() == 0 and agg.max() == nc - 1 and np.unique(agg).size == nc
    members = [[] for _ in range(nc)]
    for i in range(n):
        members[agg[i]].append(i)
    for J, mem in enumerate(members):
        boxes = {box[i] for i in mem}
        assert len(boxes) == 1
        assert tuple(cc[J]) == boxes.pop()
        # connected: BFS over edges inside the aggregate
        seen = {mem[0]}
        stack = [mem[0]]
        mset = set(mem)
        while stack:
            i = stack.pop()
            for j in A.indices[A.indptr[i]:A.indptr[i + 1]]:
                if j in mset and j not in seen:
                    seen.add(j)
                    stack.append(j)
        assert seen == mset
    # maximal: no edge joins two aggregates of the same box
    for i in range(n):
        for j in A.indices[A.indptr[i]:A.indptr[i + 1]]:
            if box[i] == box[j]:
                assert agg[i] == agg[j]
    # ordering: box lexicographic (x fastest), then smallest member
    keys = [tuple(reversed(tuple(cc[J]))) + (min(members[J]),) for J in range(nc)]
    assert keys == sorted(keys)


@pytest.mark.parametrize("kind,n", [("star", 40), ("disk", 30), ("ell", 12)])
def test_aggregation_brute_force_all_levels(kind, n):
    A, coords, _ = _system(kind, n)
    H = amg.build_hierarchy(A, coords, coarse_max=8)
    assert H.n_levels >= 2
    for lvl in H.levels[:-1]:
        agg, cc = amg.aggregate(lvl.A, lvl.coords)
        assert np.array_equal(agg, lvl.agg)
        _brute_aggregates_ok(lvl.A, lvl.coords, agg, cc)


def test_split_box_gives_several_aggregates():
    """An outside node at a box centre leaves the four box corners as separate
    computational points: four coarse unknowns share one box."""
    g = W.unit_box_grid(2, 30)
    X, Y = g.mesh()
    psi = np.maximum(np.abs(Y) - 0.3, np.abs(X) - 0.4)
    psi[13, 13] = 1.0            # node (13, 13) is the centre of box (4, 4)
    asm = E.assemble(g, psi)
    A = E.operator_csr(asm)
    coords = E.unknown_coords(asm)
    agg, cc = amg.aggregate(A, coords)
    _brute_aggregates_ok(A, coords, agg, cc)
    boxes, counts = np.unique(cc, axis=0, return_counts=True)
    assert counts.max() == 4
    assert tuple(boxes[np.argmax(counts)]) == (4, 4)


def test_spgemm_matches_dense_and_structural_pattern():
    rng = np.random.default_rng(0)
    A = sp.random(40, 30, density=0.1, random_state=1, format="csr")
    B = sp.random(30, 25, density=0.15, random_state=2, format="csr")
    # force an exact cancellation to check that structural zeros survive
    C = amg.spgemm(A, B)
    dense = A.toarray() @ B.toarray()
    assert np.allclose(C.toarray(), dense, rtol=0, atol=1e-14)
    pattern = (abs(A).toarray() > 0).astype(float) @ (abs(B).toarray() > 0).astype(float) > 0
    got = np.zeros_like(pattern)
    got[np.repeat(np.arange(C.shape[0]), np.diff(C.indptr)), C.indices] = True
    assert np.array_equal(got, pattern)
    # structural zero kept
    A2 = sp.csr_matrix(np.array([[1.0, 1.0]]))
    B2 = sp.csr_matrix(np.array([[1.0], [-1.0]]))
    C2 = amg.spgemm(A2, B2)
    assert C2.nnz == 1 and C2.data[0] == 0.0
    assert rng is not None


@pytest.mark.parametrize("sigma", [0.0, 128.0])
def test_prolongator_dense_definition(sigma):
    A, coords, _ = _system("disk", 24, sigma)
    agg, cc = amg.aggregate(A, coords)
    nc = cc.shape[0]
    rho = amg.gershgorin_rho(A)
    omega = 4.0 / (3.0 * rho)
    P = amg.smoothed_prolongator(A, agg, nc, omega)
    Ad = A.toarray()
    Pt = np.zeros((A.shape[0], nc))
    Pt[np.arange(A.shape[0]), agg] = 1.0
    Pd = (np.eye(A.shape[0]) - omega * Ad / np.diag(Ad)[:, None]) @ Pt
    assert np.max(np.abs(P.toarray() - Pd)) < 1e-14
    # pattern is structural: (|A| + I) P_tent > 0
    patt = ((np.abs(Ad) > 0) | np.eye(A.shape[0], dtype=bool)).astype(float) @ Pt > 0
    got = np.zeros_like(patt)
    got[np.repeat(np.arange(P.shape[0]), np.diff(P.indptr)), P.indices] = True
    assert np.array_equal(got, patt)
    # Gershgorin bound dominates the spectrum of D^-1 A; fine level has rho = 2 when sigma = 0
    lam = np.linalg.eigvals(Ad / np.diag(Ad)[:, None]).real.max()
    assert lam <= rho + 1e-12
    if sigma == 0.0:
        assert rho == 2.0


@pytest.mark.parametrize("kind,n", [("star", 64), ("ell", 16)])
def test_galerkin_identity_symmetry_and_transpose(kind, n):
    A, coords, _ = _system(kind, n)
    H = amg.build_hierarchy(A, coords, coarse_max=16)
    rng = np.random.default_rng(5)
    for l, lvl in enumerate(H.levels[:-1]):
        Ac = H.levels[l + 1].A
        assert (lvl.R != lvl.P.T.tocsr()).nnz == 0
        xc, yc = rng.normal(size=(2, Ac.shape[0]))
        lhs = xc @ (Ac @ yc)
        rhs = (lvl.P @ xc) @ (lvl.A @ (lvl.P @ yc))
        assert abs(lhs - rhs) <= 1e-12 * abs(rhs) + 1e-12 * np.linalg.norm(xc) * np.linalg.norm(yc) * abs(Ac).max()
        asym = abs(Ac - Ac.T).max()
        assert asym <= 1e-14 * abs(Ac).max()


def test_hierarchy_stop_rules_and_coarsest_cholesky():
    A, coords, _ = _system("star", 96)
    H = amg.build_hierarchy(A, coords)
    sizes = [l.n for l in H.levels]
    assert sizes[-1] <= 256 and all(s > 256 for s in sizes[:-1])
    for a, b in zip(sizes[:-1], sizes[1:]):
        assert b <= 0.6 * a
    L = H.levels[-1].chol
    Ac = H.levels[-1].A.toarray()
    assert np.allclose(L @ L.T, Ac, rtol=1e-13, atol=1e-13 * abs(Ac).max())


@pytest.mark.parametrize("kind,n,sigma", [("star", 80, 0.0), ("disk", 64, 64.0), ("ell", 16, 0.0)])
def test_vcycle_symmetric_positive(kind, n, sigma):
    A, coords, _ = _system(kind, n, sigma)
    H = amg.build_hierarchy(A, coords, coarse_max=32)
    rng = np.random.default_rng(11)
    r1, r2 = rng.normal(size=(2, A.shape[0]))
    m1, m2 = amg.vcycle(H, r1), amg.vcycle(H, r2)
    assert abs(m1 @ r2 - r1 @ m2) <= 1e-12 * abs(m1 @ r2)
    assert m1 @ r1 > 0 and m2 @ r2 > 0


def test_vcycle_is_linear_and_reduces_error():
    A, coords, _ = _system("star", 96)
    H = amg.build_hierarchy(A, coords)
    rng = np.random.default_rng(2)
    e = rng.normal(size=A.shape[0])
    r = A @ e
    z = amg.vcycle(H, r)
    # two-grid-like contraction in the energy norm: ||e - M A e||_A < ||e||_A
    d = e - z
    assert d @ (A @ d) < 0.5 * (e @ (A @ e))
    z2 = amg.vcycle(H, 2.0 * r)
    assert np.allclose(z2, 2.0 * z, rtol=1e-13, atol=0)
