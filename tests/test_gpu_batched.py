"""Batched PCG (several right-hand sides, one hierarchy, one launch sequence)
against the oracle's AMG-PCG per right-hand side and against the single
solve of the library."""
import numpy as np
import pytest
import torch

from oracle import eb_assembly as E
from oracle import pcg as OP
from paper_2204_06083_amd import _lib as L
from paper_2204_06083_amd import solver as S
from paper_2204_06083_amd import workloads as W

from gpu_common import gpu_system, oracle_system, rel, to_dev

pytestmark = pytest.mark.gpu


def _rhs_family(prob, nrhs, seed):
    """Right-hand sides on the problem's system: b0 = the problem's own RHS,
    then seeded mixtures of it with random smooth and rough node fields
    (zero off unknowns, as the library ignores them)."""
    asm_o, A, b_o, u = oracle_system(prob)
    rng = np.random.default_rng(seed)
    fields = []
    asm_g, _ = gpu_system(prob, u)
    coords = E.unknown_coords(asm_o)
    for j in range(nrhs):
        if j == 0:
            bj = b_o.copy()
        else:
            smooth = np.cos((j + 1) * np.pi * coords[:, 0] / max(coords[:, 0].max(), 1)) * np.sin(
                (j + 2) * np.pi * coords[:, 1] / max(coords[:, 1].max(), 1))
            bj = rng.standard_normal(1) * b_o + rng.uniform(0.5, 2.0) * smooth * np.abs(b_o).max() \
                + 0.1 * rng.standard_normal(b_o.size) * np.abs(b_o).max()
        fields.append(bj)
    B = np.zeros((nrhs,) + prob.grid.shape)
    for j, bj in enumerate(fields):
        B[j].ravel()[asm_o.nodes] = bj
    return asm_o, A, fields, asm_g, B


CASES = {
    "disk128_x3": (lambda: W.disk_poisson(128), 1e-10, 3),
    "star512_x5": (lambda: W.star_poisson(512), 1e-8, 5),
    "heat512_x8": (lambda: W.star_heat(512, 0), 1e-8, 8),
    "ell48_x4": (lambda: W.ellipsoid_poisson(48), 1e-8, 4),
    "disk16_onelevel_x2": (lambda: W.disk_mms(16, radius=0.3), 1e-10, 2),
    "star300_x1": (lambda: W.star_poisson(300), 1e-8, 1),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_against_oracle(name, precision):
    mk, tol, nrhs = CASES[name]
    prob = mk()
    print(f"[gpu] batched {name} {precision} grid={prob.grid.shape}", flush=True)
    asm_o, A, fields, asm_g, B = _rhs_family(prob, nrhs, seed=11)
    H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a, prob.sigma)
    X, infos = H.solve_batched(to_dev(B), tol=tol, precision=precision)
    X = X.cpu().numpy()
    coords = E.unknown_coords(asm_o)
    for j in range(nrhs):
        ref, _ = OP.amg_pcg(A, coords, fields[j], tol=tol)
        xj = X[j].ravel()
        err = rel(xj[asm_o.nodes], ref.x)
        print(f"  rhs {j}: iters {infos[j]['iterations']} (oracle {ref.iterations}) err {err:.2e}", flush=True)
        assert infos[j]["status"] == 0
        assert infos[j]["rel_res_true"] <= tol
        assert np.linalg.norm(fields[j] - A @ xj[asm_o.nodes]) <= tol * np.linalg.norm(fields[j]) * 1.0001
        assert not np.any(xj[asm_o.kind.ravel() != 2])
        if precision == "fp64":
            assert abs(infos[j]["iterations"] - ref.iterations) <= 1
            assert err <= 1e-10
        else:
            assert infos[j]["iterations"] <= ref.iterations + 3
            ref12, _ = OP.amg_pcg(A, coords, fields[j], tol=1e-12)
            assert rel(xj[asm_o.nodes], ref12.x) <= 1e-6
    H.free()


def test_batched_matches_single_solves():
    prob = W.star_poisson(600)
    asm_o, A, fields, asm_g, B = _rhs_family(prob, 4, seed=3)
    H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a)
    Bd = to_dev(B)
    X, infos = H.solve_batched(Bd, tol=1e-8)
    for j in range(4):
        xj, ij = H.solve(Bd[j].contiguous(), tol=1e-8)
        assert abs(ij["iterations"] - infos[j]["iterations"]) <= 1
        assert rel(X[j].cpu().numpy().ravel(), xj.cpu().numpy().ravel()) <= 1e-10
    # bitwise reproducible
    X2, infos2 = H.solve_batched(Bd, tol=1e-8)
    assert torch.equal(X, X2) and [i["iterations"] for i in infos] == [i["iterations"] for i in infos2]
    H.free()


def test_batched_edge_cases():
    prob = W.star_poisson(256)
    asm_o, A, fields, asm_g, B = _rhs_family(prob, 3, seed=5)
    B[1] = 0.0                                   # a zero right-hand side inside the batch
    H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a)
    Bd = to_dev(B)
    X, infos = H.solve_batched(Bd, tol=1e-8)
    assert infos[1]["iterations"] == 0 and not torch.any(X[1]).item()
    assert infos[0]["status"] == 0 and infos[2]["status"] == 0
    # warm start from the solution: nothing to do
    X3, infos3 = H.solve_batched(Bd, tol=1e-8, x0=X)
    assert all(i["iterations"] == 0 for i in infos3)
    # iteration limit reported per right-hand side
    with pytest.raises(L.EbError) as ei:
        H.solve_batched(Bd, tol=1e-12, maxit=2)
    assert ei.value.code == L.EB_ENOCONV
    Xn, infon = H.solve_batched(Bd, tol=1e-12, maxit=2, allow_noconv=True)
    assert infon[0]["status"] == L.EB_ENOCONV and infon[0]["iterations"] == 2
    # slot count limits
    big = torch.zeros((65,) + prob.grid.shape, dtype=torch.float64, device=Bd.device)
    with pytest.raises(L.EbError) as ei:
        H.solve_batched(big, tol=1e-8)
    assert ei.value.code == L.EB_EINVAL
    H.free()


def test_batched_heat1024_64rhs():
    """The heat workload at full size: 64 seeded initial conditions, one batch."""
    print("[gpu] batched heat1024 x64", flush=True)
    probs = [W.star_heat(1024, j) for j in range(64)]
    p0 = probs[0]
    asm_g, _ = gpu_system(p0)
    B = torch.stack([S.assemble_rhs(asm_g, to_dev(p.f), torch.zeros(asm_g.n_cuts, dtype=torch.float64,
                                                                      device=asm_g.kind.device)) for p in probs])
    H = S.Hierarchy(p0.grid, asm_g.kind, asm_g.a, p0.sigma)
    for precision in ("fp64", "fp32"):
        X, infos = H.solve_batched(B.contiguous(), tol=1e-8, precision=precision)
        assert all(i["status"] == 0 and i["rel_res_true"] <= 1e-8 for i in infos)
        for j in (0, 17, 63):
            xj, ij = H.solve(B[j].contiguous(), tol=1e-8, precision=precision)
            assert abs(ij["iterations"] - infos[j]["iterations"]) <= 1
            assert rel(X[j].cpu().numpy().ravel(), xj.cpu().numpy().ravel()) <= (1e-10 if precision == "fp64" else 1e-6)
    # oracle operator residual for a sample
    asm_o, A, b_o, _ = oracle_system(probs[5])
    x5 = X[5].cpu().numpy().ravel()[asm_o.nodes]
    assert np.linalg.norm(b_o - A @ x5) <= 1e-8 * np.linalg.norm(b_o) * 1.0001
    H.free()


def test_launch_shapes_agree_and_autotuner_reports():
    """Every fixed launch shape of the batched fine kernels gives the same
    solutions as the autotuned one; the autotuner reports its candidates."""
    prob = W.star_heat(512, 0)
    asm_o, A, fields, asm_g, B = _rhs_family(prob, 16, seed=9)
    Bd = to_dev(B)
    S.set_batched_launch_shape(0, 0)
    H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a, prob.sigma)
    Xa, ia = H.solve_batched(Bd, tol=1e-10)
    rep = S.batched_launch_shape(H)
    print(f"[gpu] autotuned shape {rep['plane_width']} x {rep['planes_per_block']}: "
          + ", ".join(f"{c['plane_width']}x{c['planes_per_block']} {c['ms']:.3f} ms" for c in rep["candidates"]),
          flush=True)
    assert len(rep["candidates"]) >= 2
    assert (rep["plane_width"], rep["planes_per_block"]) in [(c["plane_width"], c["planes_per_block"])
                                                            for c in rep["candidates"]]
    H.free()
    try:
        for w, n in ((8, 1), (8, 4), (16, 2), (32, 1), (64, 1)):
            S.set_batched_launch_shape(w, n)
            H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a, prob.sigma)
            X, infos = H.solve_batched(Bd, tol=1e-10)
            r = S.batched_launch_shape(H)
            assert r["plane_width"] == min(w, 16) and r["planes_per_block"] == n
            for j in range(16):
                assert abs(infos[j]["iterations"] - ia[j]["iterations"]) <= 1
                assert rel(X[j].cpu().numpy().ravel(), Xa[j].cpu().numpy().ravel()) <= 1e-12
            H.free()
        with pytest.raises(L.EbError):
            S.set_batched_launch_shape(12, 1)
    finally:
        S.set_batched_launch_shape(0, 0)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_iteration_graphs_match_kernel_launches(precision):
    """Batched solves replay a captured pair of iterations: bitwise the same
    solutions and iteration counts as launching kernel by kernel, on the
    first replay, on a later solve, after a change of launch shape (the graph
    is captured again) and on a stream of the caller's."""
    prob = W.star_heat(512, 0)
    asm_o, A, fields, asm_g, B = _rhs_family(prob, 6, seed=21)
    Bd = to_dev(B)
    H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a, prob.sigma)
    try:
        S.set_iteration_graphs(False)
        X0, i0 = H.solve_batched(Bd, tol=1e-10, precision=precision)
        S.set_iteration_graphs(True)
        X1, i1 = H.solve_batched(Bd, tol=1e-10, precision=precision)
        X2, i2 = H.solve_batched(Bd, tol=1e-10, precision=precision)
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            X3, i3 = H.solve_batched(Bd, tol=1e-10, precision=precision)
        st.synchronize()
        print(f"[gpu] batched graphs {precision}: iterations {[i['iterations'] for i in i0]} "
              f"solve ms {i0[0]['solve_ms']:.2f} -> {i2[0]['solve_ms']:.2f}", flush=True)
        assert min(i["iterations"] for i in i0) >= 4
        for X, ii in ((X1, i1), (X2, i2), (X3, i3)):
            assert torch.equal(X, X0)
            assert [i["iterations"] for i in ii] == [i["iterations"] for i in i0]
            assert all(i["status"] == 0 for i in ii)
        H.free()
        # another launch shape: kernel by kernel against a fresh capture
        S.set_batched_launch_shape(8, 2)
        H = S.Hierarchy(prob.grid, asm_g.kind, asm_g.a, prob.sigma)
        S.set_iteration_graphs(False)
        X4, i4 = H.solve_batched(Bd, tol=1e-10, precision=precision)
        S.set_iteration_graphs(True)
        X5, i5 = H.solve_batched(Bd, tol=1e-10, precision=precision)
        assert torch.equal(X5, X4) and [i["iterations"] for i in i5] == [i["iterations"] for i in i4]
        assert rel(X4.cpu().numpy().ravel(), X0.cpu().numpy().ravel()) <= (1e-12 if precision == "fp64" else 1e-6)
    finally:
        S.set_iteration_graphs(True)
        S.set_batched_launch_shape(0, 0)
        H.free()
