"""Time-stepper right-hand sides and drivers on the GPU against the oracle's
steppers (wave theta-scheme, Crank-Nicolson heat), and the paper's Table 1
runs at full size."""
import json
import math
import os

import numpy as np
import pytest
import torch

from oracle import eb_assembly as E
from oracle import steppers as ST
from paper_2204_06083_amd import solver as S
from paper_2204_06083_amd import workloads as W

from gpu_common import rel, to_dev

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _wave_setup(n):
    g = W.wave_disk_grid(n)
    psi = W.psi_unit_disk(g)
    asm_o = E.assemble(g, psi)
    A = E.operator_csr(asm_o)
    asm_g = S.assemble_diag(g, to_dev(psi))
    X, Y = g.mesh()
    return g, asm_o, A, asm_g, X, Y


@pytest.mark.parametrize("theta,scale", [(0.0, 1.0), (1.0 / 12.0, 37.5), (0.5, 2.0)])
def test_wave_rhs_against_oracle(theta, scale):
    g, asm_o, A, asm_g, X, Y = _wave_setup(200)
    print(f"[gpu] wave_rhs theta={theta}", flush=True)
    rng = np.random.default_rng(1)
    u = rng.standard_normal(g.shape)
    um = rng.standard_normal(g.shape)
    dt = 0.7 * g.h
    out = S.wave_rhs(asm_g, theta, dt, scale, to_dev(u), to_dev(um)).cpu().numpy().ravel()
    nodes = asm_o.nodes
    un, unm = u.ravel()[nodes], um.ravel()[nodes]
    ref = scale * (2.0 * un - unm - dt * dt * (A @ ((1.0 - 2.0 * theta) * un + theta * unm)))
    assert np.abs(out[nodes] - ref).max() <= 1e-13 * np.abs(ref).max()
    mask = np.ones(out.size, bool)
    mask[nodes] = False
    assert not np.any(out[mask])


def test_stencil_combine_against_oracle():
    g, asm_o, A, asm_g, X, Y = _wave_setup(160)
    rng = np.random.default_rng(2)
    x, y, z = (rng.standard_normal(g.shape) for _ in range(3))
    sigma, alpha, beta, gamma = -3.0e4, -1.0, 0.5, 2.0
    out = S.stencil_combine(asm_g, sigma, alpha, to_dev(x), beta, to_dev(y), gamma, to_dev(z)).cpu().numpy().ravel()
    nodes = asm_o.nodes
    ref = alpha * (E.operator_csr(asm_o, sigma) @ x.ravel()[nodes]) + beta * y.ravel()[nodes] + gamma * z.ravel()[nodes]
    assert np.abs(out[nodes] - ref).max() <= 1e-13 * np.abs(ref).max()
    # y and z may be left out
    out2 = S.stencil_combine(asm_g, 0.0, 1.0, to_dev(x)).cpu().numpy().ravel()
    assert np.abs(out2[nodes] - A @ x.ravel()[nodes]).max() <= 1e-13 * np.abs(A @ x.ravel()[nodes]).max()


def test_leapfrog_matches_oracle():
    g, asm_o, A, asm_g, X, Y = _wave_setup(200)
    print("[gpu] leap-frog 200, 120 steps", flush=True)
    dt = 0.7 * g.h
    u0, u1 = W.standing_mode(X, Y, 0.0), W.standing_mode(X, Y, dt)
    ug, umg, st = S.wave_theta(asm_g, to_dev(u0), to_dev(u1), dt, 0.0, 120)
    nodes = asm_o.nodes
    uo, umo = ST.wave_theta(A, u0.ravel()[nodes], u1.ravel()[nodes], dt, 0.0, 120)
    assert rel(ug.cpu().numpy().ravel()[nodes], uo) <= 1e-11
    assert rel(umg.cpu().numpy().ravel()[nodes], umo) <= 1e-11
    # the discrete energy is conserved by the GPU trajectory too
    e0 = ST.wave_energy(A, u1.ravel()[nodes], u0.ravel()[nodes], dt, 0.0)
    e1 = ST.wave_energy(A, ug.cpu().numpy().ravel()[nodes], umg.cpu().numpy().ravel()[nodes], dt, 0.0)
    assert abs(e1 - e0) <= 1e-9 * abs(e0)


@pytest.mark.parametrize("theta", [1.0 / 12.0, 0.25, 0.5])
def test_implicit_theta_scheme_matches_oracle(theta):
    g, asm_o, A, asm_g, X, Y = _wave_setup(100)
    print(f"[gpu] theta-scheme {theta}, 100, 40 steps", flush=True)
    dt = (0.85 if theta < 0.25 else 2.0) * g.h
    u0, u1 = W.standing_mode(X, Y, 0.0), W.standing_mode(X, Y, dt)
    ug, umg, st = S.wave_theta(asm_g, to_dev(u0), to_dev(u1), dt, theta, 40, tol=1e-13)
    nodes = asm_o.nodes
    uo, _ = ST.wave_theta(A, u0.ravel()[nodes], u1.ravel()[nodes], dt, theta, 40)
    print(f"  mean PCG iterations {st['mean_iterations']:.2f}", flush=True)
    assert rel(ug.cpu().numpy().ravel()[nodes], uo) <= 1e-9
    assert st["steps"] == 39 and st["mean_iterations"] > 0


def test_crank_nicolson_matches_oracle():
    n = 64
    g = W.heat_cn_grid(n)
    psi = W.psi_heat_disk(g)
    asm_o = E.assemble(g, psi)
    asm_g = S.assemble_diag(g, to_dev(psi))
    X, Y = g.mesh()
    dt = g.h
    ns = int(round(0.5 / dt))
    xg_o = E.cut_coordinates(asm_o)
    xg_g = asm_g.cut_coordinates()

    def b_o(k):
        t = k * dt
        return E.rhs(asm_o, W.heat_cn_source(X, Y, t), W.heat_cn_exact(xg_o[0], xg_o[1], t))

    def b_g(k):
        t = k * dt
        return S.assemble_rhs(asm_g, to_dev(W.heat_cn_source(X, Y, t)), W.heat_cn_exact(xg_g[0], xg_g[1], t))

    H = S.Hierarchy(g, asm_g.kind, asm_g.a, 2.0 / dt)
    u0 = W.heat_cn_exact(X, Y, 0.0)
    ug, st = S.heat_cn(asm_g, H, to_dev(u0), dt, ns, b_g, tol=1e-13)
    uo = ST.heat_cn(asm_o, u0.ravel()[asm_o.nodes], dt, ns, b_o)
    nodes = asm_o.nodes
    assert rel(ug.cpu().numpy().ravel()[nodes], uo) <= 1e-9
    ex = W.heat_cn_exact(X, Y, ns * dt).ravel()[nodes]
    eg = np.abs(ug.cpu().numpy().ravel()[nodes] - ex).max()
    assert abs(eg - ST.max_error(uo, ex)) <= 1e-8
    with pytest.raises(ValueError):
        S.heat_cn(asm_g, H, to_dev(u0), 2.0 * dt, 1, b_g)
    H.free()


def test_table1_full_size():
    """Table 1 rows h = 2.75e-3 and 1.375e-3 (800 and 1600 cells): leap-frog
    and theta = 1/12 max-errors within a factor 4 (5) of the paper's and
    convergence of order about 2; PCG iterations per implicit step reported."""
    gold = json.load(open(os.path.join(GOLDEN, "wave_table1.json")))
    for key, theta, fac in (("theta_0", 0.0, 4.0), ("theta_1_12", 1.0 / 12.0, 5.0)):
        ref = gold[key]["max_error"][3:]
        errs = []
        for n in (800, 1600):
            g = W.wave_disk_grid(n)
            psi = W.psi_unit_disk(g)
            asm_g = S.assemble_diag(g, to_dev(psi))
            X, Y = g.mesh()
            dt, ns = W.wave_schedule(n, gold[key]["dt_over_h"], gold["periods"])
            print(f"[gpu] Table 1 {key} n={n} steps={ns}", flush=True)
            u, _, st = S.wave_theta(asm_g, to_dev(W.standing_mode(X, Y, 0.0)), to_dev(W.standing_mode(X, Y, dt)), dt,
                                    theta, ns, tol=1e-10)
            kind = asm_g.kind.cpu().numpy().ravel() == 2
            e = float(np.abs(u.cpu().numpy().ravel()[kind] - W.standing_mode(X, Y, ns * dt).ravel()[kind]).max())
            print(f"  max error {e:.3e} (paper {ref[len(errs)]:.1e}), mean PCG iterations "
                  f"{st['mean_iterations']:.2f}", flush=True)
            errs.append(e)
            assert ref[len(errs) - 1] / fac <= e <= fac * ref[len(errs) - 1]
        assert 1.6 <= math.log2(errs[0] / errs[1]) <= 2.4


def test_table1_theta_half_and_quarter_full_size():
    """Table 1's theta = 1/2 and 1/4 columns (dt/h = 2) at h = 2.2e-2 ..
    1.375e-3 (100 .. 1600 cells).  Every row follows the single-mode phase
    model of the oracle's pins (the rows wrap around in phase, as the paper's
    do); on the two finest rows, where the phase error is below one radian,
    the max-errors are within a factor 4 of the paper's and converge with order
    about 2.  Each implicit step (PCG to 1e-10, warm-started) takes at most 16
    iterations of the aggregation V(1,1) cycle; the paper reports 5-6 with
    classical AMG (its V- and W-cycles)."""
    gold = json.load(open(os.path.join(GOLDEN, "wave_table1.json")))
    kappa = W.bessel_zero(7, 7)
    for key, theta in (("theta_1_2", 0.5), ("theta_1_4", 0.25)):
        errs = []
        for i, n in enumerate((100, 200, 400, 800, 1600)):
            g = W.wave_disk_grid(n)
            asm_g = S.assemble_diag(g, to_dev(W.psi_unit_disk(g)))
            X, Y = g.mesh()
            dt, ns = W.wave_schedule(n, gold[key]["dt_over_h"], gold["periods"])
            print(f"[gpu] Table 1 {key} n={n} steps={ns}", flush=True)
            v = to_dev(W.standing_mode(X, Y, 0.0))
            u, _, st = S.wave_theta(asm_g, v, to_dev(W.standing_mode(X, Y, dt)), dt, theta, ns, tol=1e-10)
            kind = asm_g.kind.reshape(v.shape) == 2
            vin = torch.where(kind, v, torch.zeros_like(v))
            Av = S.stencil_apply(g, asm_g.kind, asm_g.a, 0.0, vin)
            lam = (torch.sum(vin * Av) / torch.sum(vin * vin)).item()
            k = dt * dt * lam
            phi = math.acos(1.0 - k / (2.0 * (1.0 + theta * k)))
            b1 = (math.cos(kappa * dt) - math.cos(phi)) / math.sin(phi)
            a_n = math.cos(ns * phi) + b1 * math.sin(ns * phi)
            pred = vin.abs().max().item() * abs(math.cos(kappa * ns * dt) - a_n)
            exact = to_dev(W.standing_mode(X, Y, ns * dt))
            e = (u - exact).abs()[kind].max().item()
            ref = gold[key]["max_error"][i]
            print(f"  max error {e:.3e} (paper {ref:.1e}, single-mode model {pred:.3e}), "
                  f"mean PCG iterations {st['mean_iterations']:.2f} (paper {gold[key]['iter'][i]})", flush=True)
            assert abs(e - pred) <= 0.2 * pred + 5e-3
            if n >= 800:
                assert ref / 4.0 <= e <= 4.0 * ref
                assert abs(e - pred) <= 0.05 * pred
                assert st["mean_iterations"] <= 16.0
            errs.append(e)
        assert 1.6 <= math.log2(errs[3] / errs[4]) <= 2.4
