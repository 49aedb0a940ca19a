"""Island batches (pcg_solve_islands): several geometries of different sizes
stacked in one canvas, one hierarchy and one launch sequence, each system
with its own PCG; against the oracle's direct solve of every island and
against the single-geometry solves."""
import math

import numpy as np
import pytest
import torch

from oracle import eb_assembly as E
from oracle import pcg as OP
from paper_2204_06083_amd import _lib as L
from paper_2204_06083_amd import solver as S
from paper_2204_06083_amd import workloads as W

from gpu_common import rel, to_dev

pytestmark = pytest.mark.gpu


def _stars(sizes, seed):
    """Random star geometries (the shape-optimisation family) on grids of the
    given sizes, resampled until they keep two node layers from the box."""
    rng = np.random.default_rng(seed)
    out = []
    for n in sizes:
        while True:
            c = rng.uniform(0.0, 0.04, size=5)
            ph = rng.uniform(0.0, 2.0 * math.pi, size=5)
            if 0.3 + c.sum() <= 0.5 - 2.0 / n:
                break
        g = W.unit_box_grid(2, n)
        out.append((g, W.psi_random_star(g, c, ph)))
    return out


def _sources(g, j):
    """Right-hand-side sources: f = 1 (j = 0), otherwise a seeded sine sum."""
    if j == 0:
        return np.ones(g.shape)
    return W.heat_initial(g, 1000 + j)


def _canvas_system(geoms, nrhs, fill_psi=1.0):
    canvas = S.stack_islands([g for g, _ in geoms])
    psi_c = canvas.pack([p for _, p in geoms], fill=fill_psi)
    asm_c = S.assemble_diag(canvas.grid, to_dev(psi_c))
    B = torch.stack([S.assemble_rhs_islands(asm_c, canvas, to_dev(canvas.pack([_sources(g, j) for g, _ in geoms])))
                     for j in range(nrhs)]).contiguous()
    return canvas, asm_c, B


@pytest.mark.parametrize("island_hierarchy", [True, False])
def test_islands_against_oracle_direct_solves(island_hierarchy):
    geoms = _stars([48, 64, 80], seed=3)
    nrhs = 2
    canvas, asm_c, B = _canvas_system(geoms, nrhs)
    print(f"[gpu] islands 3 x {nrhs}, canvas {canvas.grid.shape}, island hierarchy {island_hierarchy}", flush=True)
    H = S.Hierarchy(canvas.grid, asm_c.kind, asm_c.a, 0.0, islands=canvas.rows if island_hierarchy else None)
    assert H.n_levels > 1
    X, infos = S.solve_islands(H, B, canvas.rows, tol=1e-13)
    kinds = canvas.unpack(asm_c.kind.cpu().numpy())
    avals = canvas.unpack(asm_c.a.cpu().numpy())
    xs = canvas.unpack(X.cpu().numpy())
    for i, (g, psi) in enumerate(geoms):
        asm_o = E.assemble(g, psi)
        # the canvas assembly is the island's own (translation and h invariant)
        assert np.array_equal(kinds[i].ravel(), asm_o.kind.ravel())
        assert np.array_equal(avals[i].ravel()[asm_o.nodes], asm_o.a)
        A = E.operator_csr(asm_o)
        for j in range(nrhs):
            b = E.rhs(asm_o, _sources(g, j), np.zeros(asm_o.n_cuts))
            xstar = OP.direct_solve(A, b)
            xi = xs[i][j].ravel()[asm_o.nodes]
            info = infos[i][j]
            print(f"  island {i} rhs {j}: iters {info['iterations']} err {rel(xi, xstar):.2e}", flush=True)
            assert info["status"] == 0 and info["rel_res_true"] <= 1e-13
            assert rel(xi, xstar) <= 1e-10
            assert np.linalg.norm(b - A @ xi) <= 1e-13 * np.linalg.norm(b) * 1.0001
    H.free()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_single_island_matches_batched_solve(precision):
    (g, psi), = _stars([200], seed=5)
    canvas, asm_c, B = _canvas_system([(g, psi)], 3)
    Hc = S.Hierarchy(canvas.grid, asm_c.kind, asm_c.a, 0.0, islands=canvas.rows)
    Xc, ic = S.solve_islands(Hc, B, canvas.rows, tol=1e-12, precision=precision)
    asm_g = S.assemble_diag(g, to_dev(psi))
    zero = torch.zeros(asm_g.n_cuts, dtype=torch.float64, device=asm_g.kind.device)
    Bg = torch.stack([S.assemble_rhs(asm_g, to_dev(_sources(g, j)), zero) for j in range(3)]).contiguous()
    Hg = S.Hierarchy(g, asm_g.kind, asm_g.a, 0.0)
    Xg, ig = Hg.solve_batched(Bg, tol=1e-12, precision=precision)
    assert Hc.n_levels == Hg.n_levels
    for j in range(3):
        assert abs(ic[0][j]["iterations"] - ig[j]["iterations"]) <= 1
        assert rel(canvas.unpack(Xc[j].cpu().numpy())[0].ravel(), Xg[j].cpu().numpy().ravel()) <= 1e-9
    Hc.free()
    Hg.free()


def test_island_edge_cases():
    geoms = _stars([40, 56], seed=7)
    empty = W.unit_box_grid(2, 24)
    geoms.insert(1, (empty, np.ones(empty.shape)))          # an island with no unknowns
    canvas, asm_c, B = _canvas_system(geoms, 2)
    H = S.Hierarchy(canvas.grid, asm_c.kind, asm_c.a, 0.0, islands=canvas.rows)
    X, infos = S.solve_islands(H, B, canvas.rows, tol=1e-10)
    assert all(i["iterations"] == 0 and i["status"] == 0 for i in infos[1])
    assert not torch.any(X[:, int(canvas.rows[1]):int(canvas.rows[2])]).item()
    assert all(i["status"] == 0 and i["rel_res_true"] <= 1e-10 for k in (0, 2) for i in infos[k])
    # segments must increase and cover every unknown
    bad = [canvas.rows[::-1].copy(), np.array([0, canvas.rows[1]], dtype=np.int32),
           np.array([0, canvas.rows[-1] + 5], dtype=np.int32)]
    for rows in bad:
        with pytest.raises(L.EbError) as ei:
            S.solve_islands(H, B, rows, tol=1e-10)
        assert ei.value.code == L.EB_EINVAL
    # too many systems: 1025 segments
    with pytest.raises(L.EbError) as ei:
        S.solve_islands(H, B, np.arange(1026, dtype=np.int32), tol=1e-10)
    assert ei.value.code == L.EB_EINVAL
    # warm start from the solution: nothing to do
    X2, infos2 = S.solve_islands(H, B, canvas.rows, x0=X, tol=1e-10)
    assert all(i["iterations"] == 0 for row in infos2 for i in row)
    H.free()


def test_shape_optimisation_batch_sample():
    """24 random stars on grids of 256 .. 512 cells, 4 right-hand sides each,
    one island solve to 1e-8: every system converges; sampled islands checked
    with the oracle's operator and against their own batched solves."""
    rng = np.random.default_rng(11)
    sizes = [int(rng.choice([256, 384, 512])) for _ in range(24)]
    geoms = _stars(sizes, seed=13)
    canvas, asm_c, B = _canvas_system(geoms, 4)
    print(f"[gpu] islands 24 x 4, canvas {canvas.grid.shape}", flush=True)
    H = S.Hierarchy(canvas.grid, asm_c.kind, asm_c.a, 0.0, islands=canvas.rows)
    X, infos = S.solve_islands(H, B, canvas.rows, tol=1e-8)
    its = [i["iterations"] for row in infos for i in row]
    print(f"  levels {H.n_levels}, iterations {min(its)}..{max(its)}", flush=True)
    assert all(i["status"] == 0 and i["rel_res_true"] <= 1e-8 for row in infos for i in row)
    xs = canvas.unpack(X.cpu().numpy())
    for i in (0, 9, 23):
        g, psi = geoms[i]
        asm_o = E.assemble(g, psi)
        A = E.operator_csr(asm_o)
        for j in range(4):
            b = E.rhs(asm_o, _sources(g, j), np.zeros(asm_o.n_cuts))
            xi = xs[i][j].ravel()[asm_o.nodes]
            assert np.linalg.norm(b - A @ xi) <= 1e-8 * np.linalg.norm(b) * 1.0001
    # tight solves agree with each island's own batched solve (1e-11: near the
    # rounding floor kappa * eps of the 512^2 islands; two solutions with that
    # residual differ by at most 2 kappa tol ~ 4e-7 relative)
    Xt, _ = S.solve_islands(H, B, canvas.rows, tol=1e-11)
    xt = canvas.unpack(Xt.cpu().numpy())
    for i in (4, 17):
        g, psi = geoms[i]
        asm_g = S.assemble_diag(g, to_dev(psi))
        zero = torch.zeros(asm_g.n_cuts, dtype=torch.float64, device=asm_g.kind.device)
        Bg = torch.stack([S.assemble_rhs(asm_g, to_dev(_sources(g, j)), zero) for j in range(4)]).contiguous()
        Hg = S.Hierarchy(g, asm_g.kind, asm_g.a, 0.0)
        Xg, _ = Hg.solve_batched(Bg, tol=1e-11)
        for j in range(4):
            d = rel(xt[i][j].ravel(), Xg[j].cpu().numpy().ravel())
            print(f"  island {i} rhs {j}: vs own solve {d:.2e}", flush=True)
            assert d <= 4e-7
        Hg.free()
    H.free()


def test_island_iteration_graphs_match_kernel_launches():
    """Island batches replay captured iteration pairs: bitwise the same
    solutions and iteration counts as launching kernel by kernel."""
    geoms = _stars([64, 96, 128], seed=13)
    canvas, asm_c, B = _canvas_system(geoms, 4)
    H = S.Hierarchy(canvas.grid, asm_c.kind, asm_c.a, 0.0, islands=canvas.rows)
    try:
        S.set_iteration_graphs(False)
        X0, i0 = S.solve_islands(H, B, canvas.rows, tol=1e-10)
        S.set_iteration_graphs(True)
        X1, i1 = S.solve_islands(H, B, canvas.rows, tol=1e-10)
        X2, i2 = S.solve_islands(H, B, canvas.rows, tol=1e-10)
        its = [[i["iterations"] for i in seg] for seg in i0]
        print(f"[gpu] island graphs: iterations {its}", flush=True)
        assert min(min(r) for r in its) >= 4
        for X, ii in ((X1, i1), (X2, i2)):
            assert torch.equal(X, X0)
            assert [[i["iterations"] for i in seg] for seg in ii] == its
    finally:
        S.set_iteration_graphs(True)
        H.free()


def test_island_rhs_scales_each_source_by_its_h2():
    # eb_assemble_rhs_islands multiplies island k's source by h_k^2 on the
    # device; the same right-hand side as scaling the packed sources first
    # and calling eb_assemble_rhs, bit for bit (one product, then the
    # boundary terms in record order), with nonzero boundary data.
    geoms = _stars([40, 56, 72], seed=9)
    canvas = S.stack_islands([g for g, _ in geoms])
    asm_c = S.assemble_diag(canvas.grid, to_dev(canvas.pack([p for _, p in geoms], fill=1.0)))
    src = [_sources(g, 1) for g, _ in geoms]
    u = torch.linspace(-1.0, 2.0, asm_c.n_cuts, dtype=torch.float64, device=asm_c.kind.device)
    b1 = S.assemble_rhs_islands(asm_c, canvas, to_dev(canvas.pack(src)), u)
    scaled = canvas.pack([f * (g.h * g.h) for f, (g, _) in zip(src, geoms)])
    b2 = S.assemble_rhs(asm_c, to_dev(scaled), u)
    assert torch.equal(b1, b2)
    # segments that do not cover the canvas rows are refused
    from types import SimpleNamespace
    bad = SimpleNamespace(rows=canvas.rows[:-1], h=canvas.h[:-1])
    with pytest.raises(L.EbError) as ei:
        S.assemble_rhs_islands(asm_c, bad, to_dev(canvas.pack(src)), u)
    assert ei.value.code == L.EB_EINVAL


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_island_hierarchy_iterations_match_single_geometries(precision):
    """Each island's part of the island hierarchy ends where its own
    hierarchy would and smooths with its own weight, so every (island, rhs)
    takes the iterations of the same geometry solved alone (allowed: one
    more or less, from rounding; measured: equal), including islands whose
    own hierarchy has fewer levels than the others'."""
    rng = np.random.default_rng(21)
    sizes = [int(rng.choice([256, 384, 512, 768])) for _ in range(10)] + [160, 1024]
    geoms = _stars(sizes, seed=23)
    canvas, asm_c, B = _canvas_system(geoms, 2)
    H = S.Hierarchy(canvas.grid, asm_c.kind, asm_c.a, 0.0, islands=canvas.rows)
    X, infos = S.solve_islands(H, B, canvas.rows, tol=1e-8, precision=precision)
    print(f"[gpu] island hierarchy {len(geoms)} islands, {H.n_levels} levels", flush=True)
    xs = canvas.unpack(X.cpu().numpy())
    worst = 0
    for i, (g, psi) in enumerate(geoms):
        asm_g = S.assemble_diag(g, to_dev(psi))
        zero = torch.zeros(asm_g.n_cuts, dtype=torch.float64, device=asm_g.kind.device)
        Bg = torch.stack([S.assemble_rhs(asm_g, to_dev(_sources(g, j)), zero) for j in range(2)]).contiguous()
        Hg = S.Hierarchy(g, asm_g.kind, asm_g.a, 0.0)
        Xg, ig = Hg.solve_batched(Bg, tol=1e-8, precision=precision)
        for j in range(2):
            a, b = infos[i][j]["iterations"], ig[j]["iterations"]
            print(f"  island {i} (N = {sizes[i]}, {Hg.n_levels} levels) rhs {j}: {a} vs alone {b}", flush=True)
            worst = max(worst, abs(a - b))
            assert infos[i][j]["status"] == 0 and infos[i][j]["rel_res_true"] <= 1e-8
            assert rel(xs[i][j].ravel(), Xg[j].cpu().numpy().ravel()) <= 1e-6
        Hg.free()
    assert worst <= 1
    H.free()


def test_island_hierarchy_refuses_misaligned_islands():
    # islands that do not start on a multiple of 3^l cannot end as one row
    # range on level l
    # two disks reaching to 3 node rows from their boxes' edges, stacked
    # without alignment: their coarse unknowns share box rows
    geoms = []
    for n in (256, 256):
        g = W.unit_box_grid(2, n)
        geoms.append((g, W.psi_disk(g, center=(0.0, 0.0), radius=0.5 - 2.5 / n)))
    canvas = S.stack_islands([g for g, _ in geoms], align=1)
    psi_c = canvas.pack([p for _, p in geoms], fill=1.0)
    asm_c = S.assemble_diag(canvas.grid, to_dev(psi_c))
    with pytest.raises(L.EbError) as ei:
        S.Hierarchy(canvas.grid, asm_c.kind, asm_c.a, 0.0, islands=canvas.rows)
    assert ei.value.code == L.EB_EINVAL
    with pytest.raises(L.EbError) as ei:
        S.Hierarchy(canvas.grid, asm_c.kind, asm_c.a, 0.0, islands=np.array([0, 5], dtype=np.int32))
    assert ei.value.code == L.EB_EINVAL
