"""Single-precision V-cycle inside FP64 PCG, against the FP64 oracle.

The oracle has no reduced-precision variant: the FP32 cycle is checked against
the oracle's FP64 cycle within a bound derived from FP32 rounding, and the
mixed solve against the oracle's FP64 solution with the 1e-6 relative bound
asked of the mixed path after its FP64 true-residual check."""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle import amg as OA
from oracle import eb_assembly as E
from oracle import pcg as OP
from paper_2204_06083_amd import _lib as L
from paper_2204_06083_amd import solver as S
from paper_2204_06083_amd import workloads as W

from gpu_common import gpu_system, oracle_system, rel, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    "disk128": (lambda: W.disk_poisson(128), 1e-10),
    "star512": (lambda: W.star_poisson(512), 1e-8),
    "star1000_ragged": (lambda: W.star_poisson(1000), 1e-8),
    "heat512_sigma": (lambda: W.star_heat(512, 3), 1e-8),
    "ell48": (lambda: W.ellipsoid_poisson(48), 1e-8),
    "ell64": (lambda: W.ellipsoid_poisson(64), 1e-8),
    "disk16_onelevel": (lambda: W.disk_mms(16, radius=0.3), 1e-10),
}

# One FP32 V-cycle: each level loses a few units of 2^-24 relative to the
# magnitude of its own vectors; with up to ~6 levels and the smoother's
# cancellation (r - A z with A z ~ r/2) the cycle stays well inside 2e-5.
VCYCLE_FP32_REL = 2e-5


@pytest.mark.parametrize("name", [k for k in CASES if k != "disk16_onelevel"])
def test_vcycle_fp32_against_oracle(name):
    mk, _ = CASES[name]
    prob = mk()
    print(f"[gpu] fp32 vcycle {name} grid={prob.grid.shape}", flush=True)
    asm_o, A, b_o, u = oracle_system(prob)
    Ho = OA.build_hierarchy(A, E.unknown_coords(asm_o))
    asm_g, _ = gpu_system(prob, u)
    H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a, prob.sigma)
    assert H.n_levels == len(Ho.levels) and H.n_levels > 1
    rng = np.random.default_rng(7)
    for trial in range(2):
        r = rng.standard_normal(asm_o.n_unknowns) * (1.0 + 1e3 * trial)
        field = np.zeros(prob.grid.shape).ravel()
        field[asm_o.nodes] = r
        zo = OA.vcycle(Ho, r)
        z32 = H.vcycle(to_dev(field.reshape(prob.grid.shape)), precision="fp32").cpu().numpy().ravel()
        z64 = H.vcycle(to_dev(field.reshape(prob.grid.shape)), precision="fp64").cpu().numpy().ravel()
        e32 = rel(z32[asm_o.nodes], zo)
        e64 = rel(z64[asm_o.nodes], zo)
        print(f"  trial {trial}: fp32 rel {e32:.3e}  fp64 rel {e64:.3e}", flush=True)
        assert e64 <= 1e-12
        assert e32 <= VCYCLE_FP32_REL
        assert e32 > 0.0            # the cycle really ran in single precision
        assert not np.any(z32[asm_o.kind.ravel() != 2])
    H.free()


@pytest.mark.parametrize("name", list(CASES))
def test_mixed_solve_against_oracle(name):
    mk, tol = CASES[name]
    prob = mk()
    print(f"[gpu] mixed pcg {name} grid={prob.grid.shape}", flush=True)
    asm_o, A, b_o, u = oracle_system(prob)
    ref, _ = OP.amg_pcg(A, E.unknown_coords(asm_o), b_o, tol=1e-12)
    asm_g, b_g = gpu_system(prob, u)
    H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a, prob.sigma)
    x64, i64 = H.solve(b_g, tol=tol)
    x32, i32 = H.solve(b_g, tol=tol, precision="fp32")
    xs = x32.cpu().numpy().ravel()
    e32 = rel(xs[asm_o.nodes], ref.x)
    e64 = rel(x64.cpu().numpy().ravel()[asm_o.nodes], ref.x)
    print(f"  iters fp64 {i64['iterations']} fp32 {i32['iterations']} (restarts {i32['restarts']}); "
          f"err fp64 {e64:.2e} fp32 {e32:.2e}", flush=True)
    assert i32["status"] == 0
    assert i32["rel_res_true"] <= tol
    assert np.linalg.norm(b_o - A @ xs[asm_o.nodes]) <= tol * np.linalg.norm(b_o) * 1.0001
    assert e32 <= 1e-6
    assert i32["iterations"] <= i64["iterations"] + 3
    assert not np.any(xs[asm_o.kind.ravel() != 2])
    H.free()


def test_mixed_full_size_star2048():
    """Full 2049^2 star: mixed solve against the FP64 solve and the oracle operator."""
    prob = W.star_poisson(2048)
    print("[gpu] mixed pcg star2048 full", flush=True)
    asm_o, A, b_o, u = oracle_system(prob)
    asm_g, b_g = gpu_system(prob, u)
    H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a)
    x64, i64 = H.solve(b_g, tol=1e-8)
    x32, i32 = H.solve(b_g, tol=1e-8, precision="fp32")
    xs = x32.cpu().numpy().ravel()[asm_o.nodes]
    x6 = x64.cpu().numpy().ravel()[asm_o.nodes]
    print(f"  iters fp64 {i64['iterations']} fp32 {i32['iterations']} rel diff {rel(xs, x6):.2e}", flush=True)
    assert np.linalg.norm(b_o - A @ xs) <= 1e-8 * np.linalg.norm(b_o) * 1.0001
    assert rel(xs, x6) <= 1e-6
    assert i32["iterations"] <= i64["iterations"] + 3
    H.free()


def test_mixed_determinism_and_errors():
    prob = W.star_poisson(300)
    asm_o, A, b_o, u = oracle_system(prob)
    asm_g, b_g = gpu_system(prob, u)
    H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a)
    x1, i1 = H.solve(b_g, tol=1e-8, precision="fp32")
    x2, i2 = H.solve(b_g, tol=1e-8, precision="fp32")
    assert torch.equal(x1, x2) and i1["iterations"] == i2["iterations"]
    # an FP64 solve after the FP32 copies exist is unchanged
    xa, ia = H.solve(b_g, tol=1e-8)
    H2 = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a)
    xb, ib = H2.solve(b_g, tol=1e-8)
    assert torch.equal(xa, xb) and ia["iterations"] == ib["iterations"]
    prm = L.PcgParams(1e-8, 100, 0, 8, 7)
    res = L.PcgResult()
    x = torch.empty_like(b_g)
    rc = L.lib().pcg_solve(H.handle, C.c_void_p(b_g.data_ptr()), C.c_void_p(x.data_ptr()), C.byref(prm),
                           C.byref(res), None)
    torch.cuda.synchronize()
    assert rc == L.EB_EINVAL
    H.free()
    H2.free()


# --------------------------------------------------------------- BF16 smoother
# The BF16 smoother stores the preconditioned residual z in BF16 (relative
# rounding at most 2^-9 per entry) and scales its post-smoothing sweep by a
# BF16 copy of 1/d (again at most 2^-9 on the terms it scales, which are of
# the size of z).  Against the oracle's FP64 cycle that is a few times 2^-9
# in the 2-norm on top of the FP32 cycle's 2e-5: bounded by 1e-2.  The solve
# keeps the FP64 outer CG with its true-residual check, so the answer must
# still be within 1e-6 of the oracle's FP64 solution.
VCYCLE_BF16_REL = 1e-2


@pytest.mark.parametrize("name", ["disk128", "star512", "ell48"])
def test_vcycle_bf16_against_oracle(name):
    mk, _ = CASES[name]
    prob = mk()
    print(f"[gpu] bf16 vcycle {name} grid={prob.grid.shape}", flush=True)
    asm_o, A, b_o, u = oracle_system(prob)
    Ho = OA.build_hierarchy(A, E.unknown_coords(asm_o))
    asm_g, _ = gpu_system(prob, u)
    H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a, prob.sigma)
    rng = np.random.default_rng(11)
    r = rng.standard_normal(asm_o.n_unknowns)
    field = np.zeros(prob.grid.shape).ravel()
    field[asm_o.nodes] = r
    zo = OA.vcycle(Ho, r)
    z16 = H.vcycle(to_dev(field.reshape(prob.grid.shape)), precision="bf16").cpu().numpy().ravel()
    e16 = rel(z16[asm_o.nodes], zo)
    print(f"  bf16 cycle rel {e16:.3e}", flush=True)
    assert 1e-5 < e16 <= VCYCLE_BF16_REL
    assert not np.any(z16[asm_o.kind.ravel() != 2])
    H.free()


@pytest.mark.parametrize("name", ["disk128", "star512", "star1000_ragged", "heat512_sigma", "ell48"])
def test_bf16_smoother_solve_against_oracle(name):
    mk, tol = CASES[name]
    prob = mk()
    print(f"[gpu] bf16-smoother pcg {name} grid={prob.grid.shape}", flush=True)
    asm_o, A, b_o, u = oracle_system(prob)
    ref, _ = OP.amg_pcg(A, E.unknown_coords(asm_o), b_o, tol=1e-12)
    asm_g, b_g = gpu_system(prob, u)
    H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a, prob.sigma)
    x64, i64 = H.solve(b_g, tol=tol)
    x16, i16 = H.solve(b_g, tol=tol, precision="bf16")
    xs = x16.cpu().numpy().ravel()
    e16 = rel(xs[asm_o.nodes], ref.x)
    print(f"  iters fp64 {i64['iterations']} bf16 {i16['iterations']} (restarts {i16['restarts']}); "
          f"err {e16:.2e}", flush=True)
    assert i16["status"] == 0
    assert i16["rel_res_true"] <= tol
    assert np.linalg.norm(b_o - A @ xs[asm_o.nodes]) <= tol * np.linalg.norm(b_o) * 1.0001
    assert e16 <= 1e-6
    assert i16["iterations"] <= i64["iterations"] + 5
    H.free()


def test_bf16_smoother_full_size_star2048_and_errors():
    prob = W.star_poisson(2048)
    print("[gpu] bf16-smoother pcg star2048 full", flush=True)
    asm_o, A, b_o, u = oracle_system(prob)
    asm_g, b_g = gpu_system(prob, u)
    H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a)
    x64, i64 = H.solve(b_g, tol=1e-8)
    x16, i16 = H.solve(b_g, tol=1e-8, precision="bf16")
    x16b, i16b = H.solve(b_g, tol=1e-8, precision="bf16")
    assert torch.equal(x16, x16b) and i16["iterations"] == i16b["iterations"]
    xs = x16.cpu().numpy().ravel()[asm_o.nodes]
    x6 = x64.cpu().numpy().ravel()[asm_o.nodes]
    print(f"  iters fp64 {i64['iterations']} bf16 {i16['iterations']} rel diff {rel(xs, x6):.2e}", flush=True)
    assert np.linalg.norm(b_o - A @ xs) <= 1e-8 * np.linalg.norm(b_o) * 1.0001
    assert rel(xs, x6) <= 1e-6
    # per-point smoother weights are not taken by the BF16 smoother
    w = torch.full_like(b_g, 0.5)
    assert L.lib().amg_set_fine_weights(H.handle, C.c_void_p(w.data_ptr()), None) == L.EB_OK
    prm = L.PcgParams(1e-8, 100, 0, 8, L.PRECISION["bf16"])
    res = L.PcgResult()
    x = torch.empty_like(b_g)
    rc = L.lib().pcg_solve(H.handle, C.c_void_p(b_g.data_ptr()), C.c_void_p(x.data_ptr()), C.byref(prm),
                           C.byref(res), None)
    assert rc == L.EB_ENOTIMPL
    assert L.lib().amg_clear_fine_weights(H.handle) == L.EB_OK
    x16c, _ = H.solve(b_g, tol=1e-8, precision="bf16")
    assert torch.equal(x16c, x16)
    # batched solves do not take it
    with pytest.raises(L.EbError) as ei:
        H.solve_batched(torch.stack([b_g, b_g]).contiguous(), tol=1e-8, precision="bf16")
    assert ei.value.code == L.EB_EINVAL
    H.free()
