"""Pins of the oracle's assembly against what the paper and mathematics fix.

CPU only.  Each test names what would catch a plausible mistake.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import eb_assembly as E
from oracle import pcg as OP
from paper_2204_06083_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _brute_kind(psi):
    """Per-node loop straight from the definitions of Sec. 2."""
    inside = psi < 0
    kind = np.zeros(psi.shape, dtype=np.int8)
    it = np.nditer(psi, flags=["multi_index"])
    for _ in it:
        idx = it.multi_index
        if not inside[idx]:
            continue
        n_in = 0
        for ax in range(psi.ndim):
            for st in (-1, 1):
                j = list(idx)
                j[ax] += st
                n_in += int(inside[tuple(j)])
        kind[idx] = 2 if n_in == 2 * psi.ndim else 1
    return kind


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("dim", [2, 3])
def test_classification_brute_force(seed, dim):
    rng = np.random.default_rng(seed)
    shape = (9, 11) if dim == 2 else (7, 8, 9)
    psi = rng.normal(size=shape)
    psi[tuple(slice(None) for _ in shape)] += 0.3
    # outer layer outside
    for ax in range(dim):
        sl = [slice(None)] * dim
        sl[ax] = 0
        psi[tuple(sl)] = 1.0
        sl[ax] = -1
        psi[tuple(sl)] = 1.0
    assert np.array_equal(E.classify(psi), _brute_kind(psi))


def test_psi_zero_counts_as_outside_and_domain_error():
    g = W.unit_box_grid(2, 8)
    psi = np.ones(g.shape)
    psi[3:6, 3:6] = -1.0
    psi[4, 5] = 0.0
    kind = E.classify(psi)
    assert kind[4, 5] == E.OUTSIDE
    psi2 = psi.copy()
    psi2[0, 4] = -1.0
    with pytest.raises(E.DomainError):
        E.classify(psi2)


def test_census_configs():
    """Regression constants of the benchmark geometries (mask counts)."""
    asm = E.assemble(W.disk_poisson(128).grid, W.disk_poisson(128).psi)
    assert asm.n_unknowns == 7948 and asm.n_cuts == 400
    assert int((asm.kind == E.BOUNDARY).sum()) == 288
    assert int((asm.cuts["steps"] > 2).sum()) == 68
    p = W.star_poisson(1024)
    asm = E.assemble(p.grid, p.psi)
    assert asm.n_unknowns == 310308 and asm.n_cuts == 3722


def test_numbering_is_lexicographic_x_fastest():
    p = W.disk_poisson(32)
    asm = E.assemble(p.grid, p.psi)
    c = E.unknown_coords(asm)
    key = c[:, 1] * 10_000 + c[:, 0]
    assert np.all(np.diff(key) > 0)


def test_golden_spd_geometry_numbering_and_segments():
    """Fixture transcribed from the Sec. 2.4 figure: labels and x-block sizes."""
    from oracle import spd
    fx = json.load(open(os.path.join(GOLDEN, "fig_spd_geometry.json")))
    rows = fx["grid"]["rows"]
    kind = np.array([[2 if ch == "S" else 0 for ch in r] for r in rows], dtype=np.int8)
    nodes, index = E.number_unknowns(kind)
    labels = np.where(index >= 0, index + 1, 0)
    assert labels.tolist() == fx["grid"]["expected_labels"]
    sizes = [s.size for s in spd.line_segments(index, 0)]
    assert sizes == fx["grid"]["expected_x_block_sizes"]
    line = np.array([[0 if ch == "E" else 1 for ch in fx["line"]["points"]]])
    idx = np.where(line > 0, np.cumsum(line) - 1, -1)
    assert [s.size for s in spd.line_segments(idx, 0)] == fx["line"]["expected_segment_sizes"]


def test_planar_boundary_crossing_is_exact():
    """Linear interpolation of a linear psi locates the crossing exactly (Sec. 3.3)."""
    g = W.unit_box_grid(2, 40)
    nrm = np.array([0.6, 0.8])
    off = 0.0731
    psi = W.psi_halfplane_box(g, nrm, off)
    asm = E.assemble(g, psi)
    xg = asm.cuts["xg"]
    lin = xg[:, 0] * nrm[0] + xg[:, 1] * nrm[1] - off
    box = np.max(np.abs(xg[:, :2]), axis=1) - 0.35
    on_tilted = box < -2.5 * g.h          # far from the box faces
    assert on_tilted.sum() > 10
    assert np.max(np.abs(lin[on_tilted])) < 1e-14


@pytest.mark.parametrize("n", [24, 64])
def test_diagonal_bounds_and_weights(n):
    """n_regular <= a_k <= 2d, strict on cut rows; 0 < g_Gamma, g_1 < 1 (Sec. 2.1.1)."""
    fx = json.load(open(os.path.join(GOLDEN, "paper_closed_forms.json")))["interior_bp_weights"]
    for p in (W.disk_mms(n), W.star_poisson(n)):
        asm = E.assemble(p.grid, p.psi)
        nreg = asm.n_regular
        has_cut = np.zeros(asm.n_unknowns, bool)
        has_cut[asm.cuts["unknown"]] = True
        assert np.all(asm.a >= nreg) and np.all(asm.a <= 4)
        assert np.all(asm.a[has_cut] > nreg[has_cut])
        assert np.all(asm.a[~has_cut] == 4.0)
        q = asm.cuts["q"]
        assert np.all(q > 1.0)
        g_gamma, g_1 = 1.0 / q, 1.0 - 1.0 / q
        assert np.all(np.abs(g_gamma) <= fx["bound"]) and np.all(np.abs(g_1) <= fx["bound"])


def test_symmetry_exact():
    p = W.star_poisson(96)
    A = E.operator_csr(E.assemble(p.grid, p.psi))
    assert (A - A.T).count_nonzero() == 0


@pytest.mark.parametrize("dim,n", [(2, 48), (3, 20)])
def test_exact_on_linear_functions(dim, n):
    """Central differences and the line interpolant are exact on P1 data."""
    if dim == 2:
        p = W.star_poisson(n)
        coef = (0.7, -1.3, 2.1)
    else:
        p = W.ellipsoid_poisson(n)
        coef = (0.7, -1.3, 2.1, 0.4)
    asm = E.assemble(p.grid, p.psi)
    u = W.linear_field(coef)
    A = E.operator_csr(asm)
    b = E.rhs(asm, np.zeros(p.grid.shape), u(*E.cut_coordinates(asm)))
    x = OP.direct_solve(A, b)
    ue = u(*p.grid.mesh()).ravel()[asm.nodes]
    assert np.max(np.abs(x - ue)) / np.max(np.abs(ue)) < 1e-11


def test_rhs_and_operator_are_consistent_for_manufactured_solution():
    """A u_exact - b is the truncation error: O(1) in the interior of the unit-scaled operator, small relative to b."""
    p = W.disk_mms(64)
    asm = E.assemble(p.grid, p.psi)
    A = E.operator_csr(asm)
    b = E.rhs(asm, p.f, p.u_dirichlet(*E.cut_coordinates(asm)))
    ue = p.u_exact(*p.grid.mesh()).ravel()[asm.nodes]
    tau = A @ ue - b
    interior = asm.a == 4.0
    assert np.max(np.abs(tau[interior])) < 0.05 * np.max(np.abs(b))


@pytest.mark.slow
def test_second_order_convergence_l2():
    """Manufactured solution on the disk: fitted l2 slope >= 1.9 over N = 32..512 (Sec. 3: O(h^2))."""
    errs, hs = [], []
    for n in (32, 64, 128, 256, 512):
        p = W.disk_mms(n)
        asm = E.assemble(p.grid, p.psi)
        A = E.operator_csr(asm)
        b = E.rhs(asm, p.f, p.u_dirichlet(*E.cut_coordinates(asm)))
        x = OP.direct_solve(A, b)
        ue = p.u_exact(*p.grid.mesh()).ravel()[asm.nodes]
        errs.append(math.sqrt(np.sum((x - ue) ** 2) * p.grid.h ** 2))
        hs.append(p.grid.h)
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert slope >= 1.9, slope


def _disk_with_theta(theta, n=16, radius=0.3):
    """Disk whose rightmost node on the centre row sits theta*h inside the circle."""
    g = W.unit_box_grid(2, n)
    xs = g.axis_coords(0)
    cy = g.axis_coords(1)[n // 2]
    i_m = n // 2 + int(round(radius / g.h))      # rightmost inside node
    cx = xs[i_m] + theta * g.h - radius
    X, Y = g.mesh()
    psi = np.sqrt((X - cx) ** 2 + (Y - cy) ** 2) - radius
    return g, psi, (n // 2, i_m)


@pytest.mark.parametrize("theta", [1e-12, 1e-6, 0.5, 1.0 - 1e-9])
def test_no_small_cell_stiffness(theta):
    """h^2 lambda_max(A) <= 4d for any cut fraction, while the ghost-point
    treatment (Introduction) grows like 1/theta (negative control)."""
    g, psi, (j, i_m) = _disk_with_theta(theta)
    asm = E.assemble(g, psi)
    A = E.operator_csr(asm).toarray() * g.h ** 2
    lam = np.linalg.eigvalsh(A)
    assert lam[0] > 0 and lam[-1] <= 8.0 + 1e-12
    Ag = E.ghost_point_csr(g, psi).toarray() * g.h ** 2
    lam_g = np.linalg.eigvalsh(Ag)
    if theta < 1e-3:
        assert lam_g[-1] > 0.5 / theta
    # the chosen node is a BP whose crossing has fraction theta
    sel = (asm.cuts["t"] - theta)
    assert np.min(np.abs(sel)) < 1e-9


def _rectangle_with_theta(theta, n=16):
    """Rectangle whose right face sits theta*h beyond the node column i_m."""
    g = W.unit_box_grid(2, n)
    i_m = n // 2 + 4
    xr = g.axis_coords(0)[i_m] + theta * g.h
    X, Y = g.mesh()
    psi = np.maximum(np.maximum(X - xr, -0.3 - X), np.abs(Y) - 0.3)
    return g, psi, i_m


def test_ghost_point_end_diagonal_golden():
    """The 1-D end entry of the ghost-point treatment is 1 + 1/theta (Introduction)."""
    fx = json.load(open(os.path.join(GOLDEN, "paper_closed_forms.json")))["ghost_point_end_diagonal"]
    for theta, expect in zip(fx["theta"], fx["expected_negated_diagonal"]):
        if theta == 1.0:
            theta = 1.0 - 1e-15
        g, psi, i_m = _rectangle_with_theta(theta)
        nodes, diag, _ = E.ghost_point_diagonal(g, psi)
        j = g.n[1] // 2
        k = np.flatnonzero(nodes == j * (g.n[0] + 1) + i_m)[0]
        # both y-neighbours are inside and contribute 1 each; the x part is the 1-D end entry
        assert abs((diag[k] - 2.0) - expect) <= 1e-6 * expect
        # the interior-boundary-point treatment of the same geometry stays bounded:
        # the computational point left of the BP gets 1 + 1/(1 + theta) <= 2 along x
        asm = E.assemble(g, psi)
        kk = asm.index.ravel()[j * (g.n[0] + 1) + i_m - 1]
        assert kk >= 0 and 3.5 <= asm.a[kk] < 4.0


def test_spectrum_bound_golden_and_smallest_eigenvalue():
    """h^2 lambda in (0, 8 beta_max] (Sec. 3.3.1 bound, beta = 1), and the smallest
    eigenvalue approaches the continuous j_{0,1}^2 / R^2 of the disk."""
    from scipy.special import jn_zeros
    fx = json.load(open(os.path.join(GOLDEN, "paper_closed_forms.json")))["periodic_spectrum_bound"]
    p = W.disk_poisson(128)
    asm = E.assemble(p.grid, p.psi)
    A = E.operator_csr(asm)
    lmax = spla.eigsh(A, k=1, which="LA", return_eigenvectors=False)[0]
    assert lmax * p.grid.h ** 2 <= fx["bound_times_h2"] / fx["beta_max"] + 1e-9
    lmin = spla.eigsh(A, k=1, sigma=0.0, which="LM", return_eigenvectors=False)[0]
    exact = jn_zeros(0, 1)[0] ** 2 / 0.4 ** 2
    assert abs(lmin - exact) / exact < 2e-2


def test_three_d_assembly_basic():
    p = W.ellipsoid_poisson(32)
    asm = E.assemble(p.grid, p.psi)
    assert np.array_equal(asm.kind, _brute_kind(p.psi))
    assert np.all(asm.a <= 6.0) and np.all(asm.a >= asm.n_regular)
    A = E.operator_csr(asm)
    assert (A - A.T).count_nonzero() == 0
