"""Pins of the oracle's PCG and direct references."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import amg
from oracle import eb_assembly as E
from oracle import pcg as OP
from paper_2204_06083_amd import workloads as W


def _problem(p, sigma=0.0):
    asm = E.assemble(p.grid, p.psi)
    A = E.operator_csr(asm, sigma)
    b = E.rhs(asm, p.f, p.u_dirichlet(*E.cut_coordinates(asm)))
    return asm, A, b


def test_unpreconditioned_matches_library_cg_iterates():
    """With M = I, PCG is textbook CG: iterates agree with an independent CG routine."""
    asm, A, b = _problem(W.disk_mms(24))
    for k in (1, 3, 7):
        mine = OP.pcg(A, b, precond=None, tol=1e-300, maxit=k, restart_on_drift=False)
        lib, _ = spla.cg(A, b, x0=np.zeros_like(b), rtol=1e-300, atol=0.0, maxiter=k)
        assert np.linalg.norm(mine.x - lib) <= 1e-11 * np.linalg.norm(lib)


def test_one_level_hierarchy_converges_in_one_iteration():
    asm, A, b = _problem(W.disk_mms(16))
    assert A.shape[0] <= 256
    res, H = OP.amg_pcg(A, E.unknown_coords(asm), b, tol=1e-12)
    assert H.n_levels == 1 and res.iterations == 1


@pytest.mark.parametrize("n", [10, 12, 16])
def test_dense_solve_small_grids(n):
    """Brute-force dense solve on grids up to 16^2 (the reference solution)."""
    p = W.disk_mms(n, radius=0.3)
    asm, A, b = _problem(p)
    xd = np.linalg.solve(A.toarray(), b)
    res, _ = OP.amg_pcg(A, E.unknown_coords(asm), b, tol=1e-13)
    assert np.linalg.norm(res.x - xd) <= 1e-11 * np.linalg.norm(xd)


def test_amg_pcg_matches_sparse_direct_config1():
    """Config-1 sizes: AMG-PCG at tol 1e-13 agrees with a sparse direct solve to 1e-10."""
    p = W.disk_poisson(128)
    asm, A, b = _problem(p)
    res, H = OP.amg_pcg(A, E.unknown_coords(asm), b, tol=1e-13)
    xs = OP.direct_solve(A, b)
    assert np.linalg.norm(res.x - xs) <= 1e-10 * np.linalg.norm(xs)
    assert res.converged and res.rel_res_true <= 1e-12


def test_shifted_heat_solve_and_warm_start():
    p = W.star_heat(128, rhs_id=3)
    asm = E.assemble(p.grid, p.psi)
    A = E.operator_csr(asm, p.sigma)
    b = np.asarray(p.f).ravel()[asm.nodes]
    res, H = OP.amg_pcg(A, E.unknown_coords(asm), b, tol=1e-10)
    xs = OP.direct_solve(A, b)
    assert np.linalg.norm(res.x - xs) <= 1e-8 * np.linalg.norm(xs)
    # warm start from the solution converges immediately
    res2 = OP.pcg(A, b, precond=lambda r: amg.vcycle(H, r), tol=1e-8, x0=res.x)
    assert res2.iterations == 0


def test_zero_rhs_and_empty_system():
    asm, A, b = _problem(W.disk_mms(20))
    res = OP.pcg(A, np.zeros_like(b), tol=1e-8)
    assert res.iterations == 0 and not np.any(res.x)
    import scipy.sparse as sp
    res0 = OP.pcg(sp.csr_matrix((0, 0)), np.zeros(0))
    assert res0.x.size == 0


def test_maxit_reports_not_converged():
    asm, A, b = _problem(W.disk_mms(40))
    res = OP.pcg(A, b, precond=None, tol=1e-12, maxit=2)
    assert not res.converged and res.iterations == 2


def test_restart_when_the_true_residual_drifts():
    # a tolerance below what the true residual can reach (about eps kappa):
    # the recursive residual still falls below it, the true one does not, so
    # PCG restarts once from the current iterate with r = b - A x recomputed
    # (the history jumps back up to the true residual there), and no more
    from oracle import eb_assembly as E
    from oracle import pcg as OP
    from paper_2204_06083_amd import workloads as W
    p = W.disk_poisson(64)
    asm = E.assemble(p.grid, p.psi)
    A = E.operator_csr(asm)
    b = E.rhs(asm, p.f, p.u_dirichlet(*E.cut_coordinates(asm)))
    res = OP.pcg(A, b, tol=1e-19, maxit=400)
    assert res.restarts == 1
    # the entry after the restart is the recomputed true residual, far above
    # the recursive residual it replaced
    k = int(np.argmax(np.diff(np.log10(np.asarray(res.history)))))
    assert res.history[k + 1] > 1e3 * res.history[k]
    plain = OP.pcg(A, b, tol=1e-19, maxit=400, restart_on_drift=False)
    assert plain.restarts == 0
