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
