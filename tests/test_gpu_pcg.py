"""GPU PCG parity: same hierarchy and algorithm as the oracle, direct-solve parity, error paths."""
import numpy as np
import pytest
import torch

from oracle import amg as OA
from oracle import eb_assembly as E
from oracle import pcg as OP
from paper_2204_06083_amd import _lib as L
from paper_2204_06083_amd import solver as S
from paper_2204_06083_amd import workloads as W

from gpu_common import DEV, gpu_system, oracle_system, rel, to_dev

pytestmark = pytest.mark.gpu

ITER_CASES = {
    "disk128_1e-10": (lambda: W.disk_poisson(128), 1e-10),
    "star512": (lambda: W.star_poisson(512), 1e-8),
    "star1000_ragged": (lambda: W.star_poisson(1000), 1e-8),
    "heat512_sigma": (lambda: W.star_heat(512, 5), 1e-8),
    "ell48": (lambda: W.ellipsoid_poisson(48), 1e-8),
    "ell64": (lambda: W.ellipsoid_poisson(64), 1e-8),
    "disk16_onelevel": (lambda: W.disk_mms(16, radius=0.3), 1e-10),
    "star2048_full": (lambda: W.star_poisson(2048), 1e-8),
    "staircases512": (lambda: W.staircase_poisson(512), 1e-10),
}


@pytest.mark.parametrize("name", list(ITER_CASES))
def test_iterate_parity(name):
    mk, tol = ITER_CASES[name]
    prob = mk()
    print(f"[gpu] pcg {name} grid={prob.grid.shape}", flush=True)
    asm_o, A, b_o, u = oracle_system(prob)
    res_o, Ho = OP.amg_pcg(A, E.unknown_coords(asm_o), b_o, tol=tol)
    asm_g, b_g = gpu_system(prob, u)
    H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a, prob.sigma)
    x_g, info = H.solve(b_g, tol=tol)
    x = x_g.cpu().numpy().ravel()
    assert info["status"] == 0
    assert abs(info["iterations"] - res_o.iterations) <= 1, (info, res_o.iterations)
    assert rel(x[asm_o.nodes], res_o.x) <= 1e-10
    assert not np.any(x[asm_o.kind.ravel() != 2])
    # residual recomputed by the oracle's own operator
    assert np.linalg.norm(b_o - A @ x[asm_o.nodes]) <= tol * np.linalg.norm(b_o) * 1.0001
    assert info["rel_res_true"] <= tol
    H.free()


def test_direct_solve_parity_config1():
    """S-parity: tight tolerance against a sparse direct solve."""
    prob = W.disk_poisson(128)
    asm_o, A, b_o, u = oracle_system(prob)
    xs = OP.direct_solve(A, b_o)
    asm_g, b_g = gpu_system(prob, u)
    H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a)
    x_g, info = H.solve(b_g, tol=1e-13)
    assert rel(x_g.cpu().numpy().ravel()[asm_o.nodes], xs) <= 1e-10
    H.free()


@pytest.mark.parametrize("n", [10, 13, 16])
def test_dense_small_grids(n):
    prob = W.disk_mms(n, radius=0.3)
    asm_o, A, b_o, u = oracle_system(prob)
    xd = np.linalg.solve(A.toarray(), b_o)
    asm_g, b_g = gpu_system(prob, u)
    H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a, coarse_max=4)
    x_g, info = H.solve(b_g, tol=1e-13)
    assert rel(x_g.cpu().numpy().ravel()[asm_o.nodes], xd) <= 1e-10
    H.free()


def test_full_size_ellipsoid_iterate_parity():
    """Full 257^3 grid (2,868,149 unknowns): the GPU AMG-PCG against the
    oracle's AMG-PCG on the host (same hierarchy rules, tol 1e-8): iterations
    within one, iterates within 1e-10; and the residual recomputed by the
    oracle's operator."""
    prob = W.ellipsoid_poisson(256)
    print("[gpu] pcg ell256 full: oracle on the host (about half a minute)", flush=True)
    asm_o, A, b_o, u = oracle_system(prob)
    ref, Ho = OP.amg_pcg(A, E.unknown_coords(asm_o), b_o, tol=1e-8)
    asm_g, b_g = gpu_system(prob, u)
    H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a)
    assert H.n_levels == Ho.n_levels
    x_g, info = H.solve(b_g, tol=1e-8)
    x = x_g.cpu().numpy().ravel()[asm_o.nodes]
    print(f"  iterations gpu {info['iterations']} oracle {ref.iterations}, rel diff {rel(x, ref.x):.2e}", flush=True)
    assert abs(info["iterations"] - ref.iterations) <= 1
    assert rel(x, ref.x) <= 1e-10
    assert np.linalg.norm(b_o - A @ x) <= 1e-8 * np.linalg.norm(b_o) * 1.0001
    ue = W.u_ellipsoid(*prob.grid.mesh()).ravel()[asm_o.nodes]
    assert np.max(np.abs(x - ue)) < 5e-3            # discretisation error at h = 1/256
    H.free()


def test_determinism_and_warm_start():
    prob = W.star_poisson(600)
    asm_o, A, b_o, u = oracle_system(prob)
    asm_g, b_g = gpu_system(prob, u)
    H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a)
    x1, i1 = H.solve(b_g, tol=1e-8)
    x2, i2 = H.solve(b_g, tol=1e-8)
    assert torch.equal(x1, x2) and i1["iterations"] == i2["iterations"]
    x3, i3 = H.solve(b_g, tol=1e-8, x0=x1)
    assert i3["iterations"] == 0
    x4, i4 = H.solve(b_g, tol=1e-10, x0=x1)
    assert 0 < i4["iterations"] < i1["iterations"] + 5
    H.free()


@pytest.mark.parametrize("make", [lambda: W.star_poisson(600), lambda: W.ellipsoid_poisson(40)],
                         ids=["star600", "ell40"])
def test_zero_guess_start(make):
    """Without a guess the solve starts in one kernel from r0 = b; an explicit
    zero guess takes the general start, r0 = b - A 0, which is b bit for bit.
    alpha and beta do not depend on ||r||^2, so the iteration count and the
    solution agree exactly.  A zero right-hand side after a solve returns
    exactly zero (x is cleared at every unknown, not only where the last
    iterate was small)."""
    prob = make()
    asm_o, A, b_o, u = oracle_system(prob)
    asm_g, b_g = gpu_system(prob, u)
    H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a)
    print(f"[gpu] zero-guess start {prob.name} grid={prob.grid.shape}", flush=True)
    H.solve(b_g, tol=1e-8, x0=torch.ones_like(b_g))       # leaves a non-zero iterate behind
    xa, ia = H.solve(b_g, tol=1e-8)
    xb, ib = H.solve(b_g, tol=1e-8, x0=torch.zeros_like(b_g))
    assert ia["iterations"] == ib["iterations"] > 0
    assert torch.equal(xa, xb)
    x = xa.cpu().numpy().ravel()[asm_o.nodes]
    assert np.linalg.norm(b_o - A @ x) <= 1e-8 * np.linalg.norm(b_o) * 1.0001
    xz, iz = H.solve(torch.zeros_like(b_g), tol=1e-8)
    assert iz["iterations"] == 0 and iz["status"] == 0
    assert not torch.any(xz)
    H.free()


def test_error_paths():
    prob = W.star_poisson(256)
    asm_o, A, b_o, u = oracle_system(prob)
    asm_g, b_g = gpu_system(prob, u)
    H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a)
    with pytest.raises(L.EbError) as ei:
        H.solve(b_g, tol=1e-12, maxit=1)
    assert ei.value.code == L.EB_ENOCONV
    x, info = H.solve(b_g, tol=1e-12, maxit=1, allow_noconv=True)
    assert info["status"] == L.EB_ENOCONV and info["iterations"] == 1
    xz, iz = H.solve(torch.zeros_like(b_g), tol=1e-8)
    assert iz["iterations"] == 0 and not torch.any(xz).item()
    with pytest.raises(L.EbError) as ei:
        H.solve(b_g, tol=-1.0)
    assert ei.value.code == L.EB_EINVAL
    H.free()
    # negative shift is rejected; a kind with an unknown on the outer layer is rejected
    with pytest.raises(L.EbError):
        S.Hierarchy(prob.grid, asm_g.kind, asm_g.a, sigma=-1.0)
    bad = asm_g.kind.clone()
    bad[0, 5] = 2
    with pytest.raises(L.EbError) as ei:
        S.Hierarchy(prob.grid, bad, asm_g.a)
    assert ei.value.code == L.EB_EDOMAIN


def test_empty_system():
    g = W.unit_box_grid(2, 32)
    psi = np.ones(g.shape)
    asm = S.assemble_diag(g, to_dev(psi))
    H = S.Hierarchy(g, asm.kind, asm.a)
    x, info = H.solve(torch.zeros(g.shape, dtype=torch.float64, device=DEV))
    assert info["iterations"] == 0 and not torch.any(x).item()
    H.free()


@pytest.mark.parametrize("name,prec", [("star512", "fp64"), ("star512", "fp32"), ("ell48", "fp64"),
                                       ("disk128", "fp64")])
def test_iteration_graphs_match_kernel_launches(name, prec):
    """Captured iteration pairs run the same kernels with the same arguments:
    bitwise the same solution and iteration count as launching kernel by
    kernel, on the first graph launch and on later solves that replay it, on
    the default stream and on a stream of the caller's."""
    mk = {"star512": lambda: W.star_poisson(512), "ell48": lambda: W.ellipsoid_poisson(48),
          "disk128": lambda: W.disk_poisson(128)}[name]
    prob = mk()
    asm_o, A, b_o, u = oracle_system(prob)
    asm_g, b_g = gpu_system(prob, u)
    H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a, prob.sigma)
    try:
        S.set_iteration_graphs(False)
        x0, i0 = H.solve(b_g, tol=1e-10, precision=prec)
        S.set_iteration_graphs(True)
        x1, i1 = H.solve(b_g, tol=1e-10, precision=prec)
        x2, i2 = H.solve(b_g, tol=1e-10, precision=prec)
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            x3, i3 = H.solve(b_g, tol=1e-10, precision=prec)
        st.synchronize()
        print(f"[gpu] graphs {name} {prec}: iterations {i0['iterations']} {i1['iterations']} "
              f"solve ms {i0['solve_ms']:.2f} -> {i2['solve_ms']:.2f}", flush=True)
        assert i0["iterations"] >= 4
        for x, i in ((x1, i1), (x2, i2), (x3, i3)):
            assert torch.equal(x, x0) and i["iterations"] == i0["iterations"] and i["status"] == 0
    finally:
        S.set_iteration_graphs(True)
        H.free()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_poll_cadence_does_not_change_the_solve(precision):
    """The host sizes the chunks of iterations between polls from the
    residual's reduction rate and may queue the true residual early; the
    device work per iteration is the same, so solution and iteration count
    are bitwise independent of the polling cadence."""
    prob = W.star_poisson(400)
    asm_o, A, b_o, u = oracle_system(prob)
    asm_g, b_g = gpu_system(prob, u)
    print(f"[gpu] poll cadence {precision}", flush=True)
    H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a)
    x_ref, i_ref = H.solve(b_g, tol=1e-9, precision=precision)
    for ce in (1, 2, 5, 64):
        x, i = H.solve(b_g, tol=1e-9, precision=precision, check_every=ce)
        assert torch.equal(x, x_ref), ce
        assert i["iterations"] == i_ref["iterations"] and i["status"] == 0, ce
        assert i["rel_res_true"] == i_ref["rel_res_true"], ce
    H.free()


def test_handle_memory_through_caller_allocator():
    # amg_params_t alloc / free: every device block of the handle comes from
    # the caller's allocator (here torch's caching allocator) and goes back to
    # it by amg_free; results are bitwise those of the library's own cache.
    prob = W.star_poisson(512)
    asm_o, A, b_o, u = oracle_system(prob)
    asm_g, b_g = gpu_system(prob, u)
    H1 = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a)
    x1, i1 = H1.solve(b_g, tol=1e-8)
    x1f, _ = H1.solve(b_g, tol=1e-8, precision="fp32")
    H1.free()
    before = torch.cuda.memory_allocated()
    H2 = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a, allocator="torch")
    assert H2.alloc_calls[0] > 0
    held = torch.cuda.memory_allocated() - before
    assert held > 0
    x2, i2 = H2.solve(b_g, tol=1e-8)
    x2f, _ = H2.solve(b_g, tol=1e-8, precision="fp32")
    xb, _ = H2.solve_batched(torch.stack([b_g, 2.0 * b_g]).contiguous(), tol=1e-8)
    assert torch.equal(x1, x2) and torch.equal(x1f, x2f) and i1["iterations"] == i2["iterations"]
    assert rel(xb[0].cpu().numpy(), x1.cpu().numpy()) <= 1e-10
    after_solves = torch.cuda.memory_allocated()
    H2.free()
    torch.cuda.synchronize()
    assert H2.alloc_calls[0] == H2.alloc_calls[1]
    assert torch.cuda.memory_allocated() < after_solves - held // 2
