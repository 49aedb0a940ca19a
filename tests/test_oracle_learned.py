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


# ------------------------------------------------------------------ Adam
# Adam (Kingma and Ba): m_t = b1 m + (1 - b1) g, v_t = b2 v + (1 - b2) g^2,
# m^ = m_t / (1 - b1^t), v^ = v_t / (1 - b2^t), w -= lr m^ / (sqrt(v^) + eps).
# The pins below are consequences of that definition worked out by hand, not
# a second copy of the update.

def _adam_run(grads, lr):
    net = {"w": np.zeros(len(grads[0]))}
    opt = LN.Adam(net, lr=lr)
    steps = []
    for g in grads:
        before = net["w"].copy()
        opt.step(net, {"w": np.asarray(g, dtype=np.float64)})
        steps.append(net["w"] - before)
    return steps


def test_adam_first_step_is_lr_times_the_sign():
    # after one step m^ = g and v^ = g^2 exactly, so the move is
    # -lr g / (|g| + eps): lr in the direction of -g, whatever b1 and b2
    g = [0.5, -2.0, 1e-3, 0.0]
    (d,) = _adam_run([g], lr=0.05)
    expect = [-0.05 * 0.5 / (0.5 + 1e-8), 0.05 * 2.0 / (2.0 + 1e-8), -0.05 * 1e-3 / (1e-3 + 1e-8), 0.0]
    np.testing.assert_allclose(d, expect, rtol=1e-15, atol=0)
    # 5e-2 to 1e-10 relative for the three non-zero gradients
    assert abs(abs(d[0]) - 0.05) < 1e-9 and abs(abs(d[1]) - 0.05) < 1e-9


def test_adam_constant_gradient_moves_lr_each_step():
    # with a constant gradient, m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so
    # the bias corrections give m^ = g, v^ = g^2 at every step
    g = [3.0, -0.25]
    steps = _adam_run([g] * 6, lr=0.01)
    for d in steps:
        np.testing.assert_allclose(d, [-0.01 * 3.0 / (3.0 + 1e-8), 0.01 * 0.25 / (0.25 + 1e-8)], rtol=1e-13)


def test_adam_second_step_after_a_zero_gradient():
    # g_1 = g, g_2 = 0: m_2 = b1 (1 - b1) g, v_2 = b2 (1 - b2) g^2, so
    # m^ = b1 / (1 + b1) g = 0.47368... g and sqrt(v^) = sqrt(b2 / (1 + b2)) |g|
    # = 0.70692... |g|; the second move is -lr 0.6700582541365435 sign(g)
    # (|g| >> eps)
    g = [4.0, -1.5]
    d1, d2 = _adam_run([g, [0.0, 0.0]], lr=0.2)
    np.testing.assert_allclose(d2, [-0.2 * 0.6700582541365435, 0.2 * 0.6700582541365435], rtol=1e-8)


# ------------------------------------------------------------------ features
def test_features_on_a_hand_built_grid():
    # 5 x 5 nodes, h = 0.25; kinds, diagonal and psi chosen by hand
    kind = np.array([[0, 0, 0, 0, 0],
                     [0, 1, 1, 1, 0],
                     [0, 1, 2, 2, 0],
                     [0, 1, 2, 1, 0],
                     [0, 0, 0, 0, 0]], dtype=np.int8)
    a = np.zeros((5, 5))
    a[2, 2], a[2, 3], a[3, 2] = 4.0, 3.5, 2.75          # only read at kind 2
    a[1, 1] = 9.0                                       # a boundary point: ignored
    psi = np.array([[1.0, 0.5, 0.3, 0.5, 1.0],
                    [0.5, -0.05, -0.1, -0.05, 0.5],
                    [0.3, -0.1, -0.5, -0.25, 0.3],
                    [0.5, -0.05, -0.3, -0.1, 0.5],
                    [1.0, 0.5, 0.3, 0.5, 1.0]])
    f = LN.features(kind, a, psi, 0.25, 2)
    assert f.shape == (2, 5, 5)
    f0 = np.zeros((5, 5))
    f0[2, 2], f0[2, 3], f0[3, 2] = 1.0, 0.875, 0.6875   # a / (2 d), d = 2
    np.testing.assert_array_equal(f[0], f0)
    # psi / h clipped to [-3, 3], then / 3:  1.0/0.25 = 4 -> 1; 0.5/0.25 = 2 -> 2/3;
    # 0.3/0.25 = 1.2 -> 0.4; -0.05/0.25 = -0.2 -> -1/15; -0.1/0.25 = -0.4 -> -2/15;
    # -0.5/0.25 = -2 -> -2/3; -0.25/0.25 = -1 -> -1/3; -0.3/0.25 = -1.2 -> -0.4
    f1 = np.array([[1.0, 2 / 3, 0.4, 2 / 3, 1.0],
                   [2 / 3, -1 / 15, -2 / 15, -1 / 15, 2 / 3],
                   [0.4, -2 / 15, -2 / 3, -1 / 3, 0.4],
                   [2 / 3, -1 / 15, -0.4, -2 / 15, 2 / 3],
                   [1.0, 2 / 3, 0.4, 2 / 3, 1.0]])
    np.testing.assert_allclose(f[1], f1, rtol=1e-15, atol=1e-16)
    # a level set far below -3h saturates at -1
    f = LN.features(kind, a, np.full((5, 5), -7.0), 0.25, 2)
    assert np.all(f[1] == -1.0)


# ------------------------------------------------------------ error samples
def test_error_samples_against_the_dense_error_propagator():
    # on a 12^2 disk the cycle M is formed column by column as a dense matrix;
    # the samples must be (I - M A)^s xi with the seeded xi, in unit 2-norm
    p, asm, A, H, _ = _small("disk", 12)
    n = A.shape[0]
    M = np.column_stack([amg.vcycle(H, np.eye(n)[:, i]) for i in range(n)])
    Ad = A.toarray()
    T = np.eye(n) - M @ Ad
    for sweeps in (1, 3):
        Es = LN.error_samples(H, 4, seed=7, sweeps=sweeps)
        xi = np.random.default_rng(7).standard_normal((n, 4))
        ref = np.linalg.matrix_power(T, sweeps) @ xi
        ref /= np.linalg.norm(ref, axis=0)
        np.testing.assert_allclose(Es, ref, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(np.linalg.norm(Es, axis=0), 1.0, rtol=1e-14)
