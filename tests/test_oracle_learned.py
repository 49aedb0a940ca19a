"""Pins of the oracle's learned-smoother extension (network, weighted cycle, gradients)."""
import numpy as np
import pytest

from oracle import amg
from oracle import eb_assembly as E
from oracle import learned as LN
from paper_2204_06083_amd import workloads as W


def _small(kind="star", n=48):
    p = {"star": lambda: W.star_poisson(n), "disk": lambda: W.disk_mms(n),
         "ell": lambda: W.ellipsoid_poisson(n)}[kind]()
    asm = E.assemble(p.grid, p.psi)
    A = E.operator_csr(asm)
    H = amg.build_hierarchy(A, E.unknown_coords(asm), coarse_max=32)
    f = LN.features_of(asm, p.psi, p.grid.h, p.grid.dim)
    return p, asm, A, H, f


def test_bf16_rounding_known_values():
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -7, -2.5, 3.0e38, 1.0 + 2.0 ** -9])
    y = LN.bf16_round(x)
    # ties go to the even mantissa; 2^-9 above 1 rounds down
    np.testing.assert_array_equal(y[:4], np.float32([1.0, 1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7]))
    assert y[4] == np.float32(-2.5)
    assert y[6] == np.float32(1.0)
    # every result has 16 zero low bits
    assert not np.any(y.view(np.uint32) & 0xFFFF)


@pytest.mark.parametrize("dim", [2, 3])
def test_conv_against_brute_force(dim):
    rng = np.random.default_rng(1)
    shape = (5, 6) if dim == 2 else (3, 4, 5)
    x = rng.standard_normal((3,) + shape)
    nt = 3 ** dim
    w = rng.standard_normal((4, 3, nt))
    b = rng.standard_normal(4)
    out = LN.conv(x, w, b, dim)
    taps = LN.taps(dim)
    ref = np.zeros((4,) + shape)
    for idx in np.ndindex(*shape):
        for c in range(4):
            s = b[c]
            for t, off in enumerate(taps):
                o = off if dim == 3 else off[1:]
                q = tuple(i + d for i, d in zip(idx, o))
                if all(0 <= qi < n for qi, n in zip(q, shape)):
                    for cp in range(3):
                        s += w[c, cp, t] * x[(cp,) + q]
            ref[(c,) + idx] = s
    np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_network_gradients_finite_differences(dim):
    rng = np.random.default_rng(2)
    shape = (6, 7) if dim == 2 else (4, 5, 4)
    f = rng.standard_normal((2,) + shape)
    net = LN.init_net(dim, seed=3)
    net["w3"] = rng.standard_normal(net["w3"].shape) * 0.3
    net["b3"] = np.array([0.1])
    go = rng.standard_normal(shape)
    o, cache = LN.forward(net, f, dim)
    g = LN.backward(cache, go, dim)
    eps = 1e-6
    for k in ("w1", "b1", "w2", "b2", "w3", "b3"):
        for _ in range(3):
            idx = tuple(rng.integers(0, s) for s in net[k].shape)
            net2 = {kk: v.copy() for kk, v in net.items()}
            net2[k][idx] += eps
            lp = float(np.sum(go * LN.forward(net2, f, dim)[0]))
            net2[k][idx] -= 2 * eps
            lm = float(np.sum(go * LN.forward(net2, f, dim)[0]))
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - g[k][idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx, fd, g[k][idx])


def test_weighted_cycle_constant_weights_is_plain_cycle():
    p, asm, A, H, f = _small("star", 64)
    assert H.n_levels >= 3
    rng = np.random.default_rng(4)
    r = rng.standard_normal(A.shape[0])
    z0 = amg.vcycle(H, r)
    z1 = LN.vcycle_weighted(H, r, np.full(A.shape[0], H.levels[0].omega))
    assert np.linalg.norm(z1 - z0) <= 1e-14 * np.linalg.norm(z0)
    # a zero last layer gives exactly omega_0 everywhere
    net = LN.init_net(2, seed=0)
    o, _ = LN.forward(net, f, 2)
    assert np.all(LN.omega_of(o, H.levels[0].omega) == H.levels[0].omega)


def test_weighted_cycle_symmetric_positive():
    p, asm, A, H, f = _small("disk", 40)
    rng = np.random.default_rng(5)
    n = A.shape[0]
    om = H.levels[0].omega * (1.0 + 0.5 * np.tanh(rng.standard_normal(n)))
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    mx, my = LN.vcycle_weighted(H, x, om), LN.vcycle_weighted(H, y, om)
    assert abs(x @ my - y @ mx) <= 1e-12 * abs(x @ my)
    assert x @ mx > 0 and y @ my > 0


@pytest.mark.parametrize("kind,n", [("star", 48), ("ell", 14)])
def test_loss_gradient_finite_differences(kind, n):
    p, asm, A, H, f = _small(kind, n)
    assert H.n_levels >= 2
    rng = np.random.default_rng(6)
    E_ = LN.error_samples(H, 2, seed=7)
    om = H.levels[0].omega * (1.0 + 0.3 * np.tanh(rng.standard_normal(A.shape[0])))
    L, g = LN.loss_and_grad(H, om, E_)
    assert 0.0 < L < 0.5
    eps = 1e-6
    for k in rng.integers(0, A.shape[0], size=6):
        o2 = om.copy()
        o2[k] += eps
        lp = LN.loss_and_grad(H, o2, E_)[0]
        o2[k] -= 2 * eps
        lm = LN.loss_and_grad(H, o2, E_)[0]
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(g).max()), (k, fd, g[k])
    # directional derivative along a random direction
    dvec = rng.standard_normal(A.shape[0]) * 1e-3
    lp = LN.loss_and_grad(H, om + dvec * 1e-3, E_)[0]
    lm = LN.loss_and_grad(H, om - dvec * 1e-3, E_)[0]
    fd = (lp - lm) / 2e-3
    assert abs(fd - g @ dvec) <= 1e-5 * abs(fd)


def test_full_gradient_finite_differences():
    p, asm, A, H, f = _small("star", 40)
    rng = np.random.default_rng(8)
    net = LN.init_net(2, seed=9)
    net["w3"] = rng.standard_normal(net["w3"].shape) * 0.2
    E_ = LN.error_samples(H, 2, seed=10)
    L, grads, om = LN.full_grad(net, f, 2, H, asm.nodes, asm.kind, E_)
    eps = 1e-6
    for k in ("w1", "w2", "w3", "b3"):
        idx = tuple(rng.integers(0, s) for s in net[k].shape)
        n2 = {kk: v.copy() for kk, v in net.items()}
        n2[k][idx] += eps
        lp = LN.full_grad(n2, f, 2, H, asm.nodes, asm.kind, E_)[0]
        n2[k][idx] -= 2 * eps
        lm = LN.full_grad(n2, f, 2, H, asm.nodes, asm.kind, E_)[0]
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - grads[k][idx]) <= 1e-5 * max(abs(fd), 1e-4), (k, idx, fd, grads[k][idx])


def test_training_lowers_the_loss():
    """A few Adam steps on the oracle lower the loss from the plain smoother's."""
    p, asm, A, H, f = _small("star", 64)
    net = LN.init_net(2, seed=11)
    opt = LN.Adam(net, lr=5e-3)
    E_ = LN.error_samples(H, 4, seed=12)
    L0 = LN.full_grad(net, f, 2, H, asm.nodes, asm.kind, E_)[0]
    for it in range(15):
        L, g, _ = LN.full_grad(net, f, 2, H, asm.nodes, asm.kind, E_)
        net = opt.step(net, g)
    L1 = LN.full_grad(net, f, 2, H, asm.nodes, asm.kind, E_)[0]
    assert L1 < L0
