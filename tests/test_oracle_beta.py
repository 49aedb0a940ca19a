"""Pins of the oracle's variable-conductivity operator (Eq. (1), Eq.
(central_difference) with face values beta_{i+-1/2}; Sec. 3.3.1 and Sec. 3.4).

CPU only.  Each test names the mistake it would catch.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import eb_assembly as E
from oracle import steppers as ST
from paper_2204_06083_amd import workloads as W


def test_beta_one_is_the_constant_case_bit_for_bit():
    # beta = 1 must reproduce the constant-coefficient assembly exactly (a
    # wrong accumulation order or a stray factor would show here).
    for prob, mode in ((W.star_poisson(128), "line"), (W.star_poisson(128), "mixed"), (W.ellipsoid_poisson(24), "line")):
        ones = np.ones((prob.grid.dim,) + prob.psi.shape)
        a0 = E.assemble(prob.grid, prob.psi, mode=mode)
        a1 = E.assemble(prob.grid, prob.psi, mode=mode, beta=ones)
        assert np.array_equal(a0.a, a1.a)
        assert np.array_equal(a0.cuts["c"], a1.cuts["c"])
        assert (E.operator_csr(a0) != E.operator_csr(a1)).nnz == 0


@pytest.mark.parametrize("mode", ["line", "mixed"])
def test_operator_entries_from_the_difference_formula(mode):
    # Per-node loop straight from Eq. (central_difference): the entry between
    # neighbouring unknowns is -beta_face / h^2 with the face between them;
    # the diagonal is the sum over the 2d sides of beta_face times 1 (a
    # computational neighbour) or times the side's interpolation weights
    # (taken from the beta = 1 assembly).  Catches a face taken on the wrong
    # side, a missing beta on a cut side, a transposed off-diagonal.
    pb = W.bone_beta_poisson(48)
    beta = W.beta_faces(pb.grid, pb.meta["beta"])
    asm = E.assemble(pb.grid, pb.psi, mode=mode, beta=beta)
    asm1 = E.assemble(pb.grid, pb.psi, mode=mode)
    A = E.operator_csr(asm).tocsr()
    s = 1.0 / pb.grid.h ** 2
    ny, nx = pb.psi.shape
    idx = asm.index
    weights = {}
    for k, d, c in zip(asm1.cuts["unknown"], asm1.cuts["dir"], asm1.cuts["c"]):
        weights[(int(k), int(d))] = weights.get((int(k), int(d)), 0.0) + c
    for k, node in enumerate(asm.nodes):
        j, i = divmod(int(node), nx)
        diag = 0.0
        for d, (di, dj, face) in enumerate(((-1, 0, beta[0][j, i - 1]), (1, 0, beta[0][j, i]),
                                            (0, -1, beta[1][j - 1, i]), (0, 1, beta[1][j, i]))):
            m = idx[j + dj, i + di]
            if m >= 0:
                assert A[k, m] == -(face * s)
                diag += face
            else:
                diag += face * weights[(k, d)]
        assert abs(A[k, k] - diag * s) <= 1e-13 * diag * s
    assert (A != A.T).nnz == 0


def test_spectrum_bounded_by_the_largest_conductivity():
    # Reading of Sec. 3.3.1: every eigenvalue of h^2 A lies in (0, 4 d beta_max]
    # (the paper's bound 24 for beta_max = 3 in 2-D).
    pb = W.bone_beta_poisson(40)
    beta = W.beta_faces(pb.grid, pb.meta["beta"])
    asm = E.assemble(pb.grid, pb.psi, beta=beta)
    A = E.operator_csr(asm).toarray() * pb.grid.h ** 2
    lam = np.linalg.eigvalsh(A)
    bmax = beta.max()
    assert lam.min() > 0 and lam.max() <= 8.0 * bmax


def test_bone_coefficient_second_order_convergence():
    # Sec. 3.3.1's beta and exact solution: second order (mixed rows).  A
    # face beta sampled at the node instead of the midpoint drops the order.
    def errs(n):
        pb = W.bone_beta_poisson(n)
        beta = W.beta_faces(pb.grid, pb.meta["beta"])
        asm = E.assemble(pb.grid, pb.psi, mode="mixed", beta=beta)
        A = E.operator_csr(asm)
        b = E.rhs(asm, pb.f, pb.u_dirichlet(*E.cut_coordinates(asm)))
        x = spla.spsolve(A.tocsc(), b)
        X, Y = pb.grid.mesh()
        e = x - pb.u_exact(X, Y).ravel()[asm.nodes]
        return np.sqrt(np.mean(e * e)), np.abs(e).max()
    Ns = [128, 256, 512]
    E_ = np.array([errs(n) for n in Ns])
    lh = np.log(1.0 / np.array(Ns))
    s2 = np.polyfit(lh, np.log(E_[:, 0]), 1)[0]
    si = np.polyfit(lh, np.log(E_[:, 1]), 1)[0]
    print(f"bone beta: l2 slope {s2:.2f}, linf slope {si:.2f}")
    assert s2 >= 1.85 and si >= 1.7


def test_heat_example_with_variable_beta_second_order():
    # Sec. 3.4: u_t = div(beta grad u) + f on the disk of radius 1/2, beta =
    # 1/4 - x^2 - y^2, u = exp(-t)(x^2 + y^2 - 1/4), Crank-Nicolson with
    # dt = h to t = 0.5, the mixed rows.  The l2 and max errors at t = 0.5
    # fall about 4x per refinement; with the face beta dropped (beta = 1) the
    # source no longer matches and the error stays O(1).
    def err(n, use_beta=True):
        g = W.heat_cn_grid(n)
        psi = W.psi_heat_disk(g)
        beta = W.beta_faces(g, W.beta_heat) if use_beta else None
        asm = E.assemble(g, psi, mode="mixed", beta=beta)
        X, Y = g.mesh()
        dt = g.h
        ns = int(round(0.5 / dt))
        xg = E.cut_coordinates(asm)
        u0 = W.heat_cn_exact(X, Y, 0.0).ravel()[asm.nodes]
        u = ST.heat_cn(asm, u0, dt, ns, lambda k: E.rhs(asm, W.heat_beta_source(X, Y, k * dt),
                                                          W.heat_cn_exact(xg[0], xg[1], k * dt)))
        ee = u - W.heat_cn_exact(X, Y, ns * dt).ravel()[asm.nodes]
        return np.sqrt(np.mean(ee * ee)), np.abs(ee).max()
    e = np.array([err(n) for n in (32, 64, 128)])
    rates = np.log2(e[:-1] / e[1:])
    print("heat beta errors", e.tolist(), "rates", rates.tolist())
    assert np.all(rates[:, 0] >= 1.9) and np.all(rates[:, 1] >= 1.8)
    assert err(64, use_beta=False)[1] > 20 * e[1, 1]
