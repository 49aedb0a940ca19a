"""Oracle: learned per-point smoothing weights for the fine level (CPU).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

This is an extension of the method, not a step of the paper: the paper
preconditions CG with an AMG package (Sec. 3 preamble, Algorithm 2 step 4)
and fixes no smoother.  The extension replaces the fine-level Jacobi weight
omega (the same for every point) by a weight omega_k per computational point,
produced by a small convolutional network from local geometry, so that the
points next to the boundary, whose diagonal a_k the line-by-line treatment
changes (Sec. 2.1.1), can be smoothed with their own weight.  What is
computed, written out plainly:

* Features per node (2 channels), zero outside the node grid:
    f0 = a_k / (2d) at computational points, 0 elsewhere;
    f1 = clip(psi / h, -3, 3) / 3.
* Network: three convolutions with 3^d taps and zero padding,
    y1 = relu(conv(f; W1, b1))      2 -> 16 channels
    y2 = relu(conv(y1; W2, b2))    16 -> 16
    o  = conv(y2; W3, b3)          16 -> 1
  conv(x; W, b)[c, p] = b[c] + sum_{c', t} W[c, c', t] x[c', p + off_t], the
  taps off_t in {-1, 0, 1}^d in lexicographic order with x fastest.
  omega_k = omega_0 (1 + 0.35 tanh(o_k)) in (0.65 omega_0, 1.35 omega_0),
  omega_0 the level's own weight 4 / (3 rho).  With W3 = 0 and b3 = 0 the
  weights equal omega_0: the plain smoother.  The span is a reading: the
  operator is diagonally dominant (rho <= 2, omega_0 <= 2/3), so the weight
  stays below 0.9, short of 1, where a Jacobi sweep stops damping the
  oscillatory error; the loss below, measured on smooth error samples,
  keeps falling up to that edge.
* Precision of the GPU network: every convolution takes its weights and its
  input rounded to bfloat16 (round to nearest even); products and sums are
  FP32, biases FP32.  `forward(..., precision="bf16")` does the same here (the
  cache then holds the rounded inputs, so the weight gradients are those of
  the rounded computation and input gradients pass straight through the
  rounding); "fp64" keeps everything in FP64 (used for the finite-difference
  pins).
* Smoother: on the fine level only, pre- and post-smoothing use
  W = diag(omega_k / A_kk); the prolongator and every coarser level keep
  their own omega.  One V(1,1) cycle:
    z1 = W r;  z2 = z1 + P E_c R (r - A z1);  z = z2 + W (r - A z2)
  with E_c the V-cycle of the coarser levels (a fixed symmetric operator).
  W is the same before and after, so the cycle stays symmetric.
* Loss for error samples e (columns of E): the A-norm of the error after one
  cycle, relative to before,  L = mean_e  (e'^T A e') / (2 e^T A e),
  e' = e - M A e.  Its gradient with respect to W follows from the chain
  rule of the three lines above (A and E_c symmetric, R = P^T):
    g = -A e' / (e^T A e)
    dL/dW = g * (r - A z2) + v * r,
    u = g - A (W g),   v = u - A P E_c R u.
  dL/domega_k = dL/dW_k / A_kk, then through tanh and the three convolutions.
* Training: Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 weights.
  Error samples are errors a cycle leaves: starting from seeded xi ~ N(0, 1)
  at the unknowns, e = (I - M A)^sweeps xi scaled to unit 2-norm (scaling
  after every sweep or once at the end gives the same vector up to
  rounding).  error_samples below uses the plain cycle M_0; the GPU training
  loop draws them with the cycle of the current weights (the same sweep with
  vcycle_weighted).

Parity: pinned by tests/test_oracle_learned.py (convolution against a dense
brute-force sum; network gradients and dL/domega against central finite
differences; the weighted cycle with constant weights against the plain
cycle; symmetry of the weighted cycle; a zero last layer reproduces the
plain smoother; the features on a hand-built 5 x 5 grid; the error samples
against the dense error propagator (I - M A)^s; Adam against hand-derived
moves: the first is -lr g / (|g| + eps), a constant gradient moves lr every
step, and after g then 0 the move is lr b1 / (1 + b1) / sqrt(b2 / (1 + b2))).
"""
from __future__ import annotations

import numpy as np

from . import amg

NCH = 16


# ------------------------------------------------------------------ features
def features(kind, a_node, psi, h, dim):
    """kind, a_node (a_k at computational points), psi: node fields."""
    f0 = np.where(kind == 2, a_node / (2.0 * dim), 0.0)
    f1 = np.clip(psi / h, -3.0, 3.0) / 3.0
    return np.stack([f0, f1]).astype(np.float64)


def features_of(asm, psi, h, dim):
    a_node = np.zeros(asm.kind.size)
    a_node[asm.nodes] = asm.a
    return features(asm.kind, a_node.reshape(asm.kind.shape), psi, h, dim)


# ------------------------------------------------------------------ bfloat16
def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float32."""
    x32 = np.asarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


# ------------------------------------------------------------------ network
def taps(dim):
    """Tap offsets (dz, dy, dx) in lexicographic order, x fastest."""
    rng = (-1, 0, 1)
    if dim == 2:
        return [(0, dy, dx) for dy in rng for dx in rng]
    return [(dz, dy, dx) for dz in rng for dy in rng for dx in rng]


def init_net(dim, seed=0):
    """He-normal first two layers, zero last layer (starts at the plain smoother)."""
    rng = np.random.default_rng(seed)
    nt = 3 ** dim
    w1 = rng.normal(0.0, np.sqrt(2.0 / (2 * nt)), size=(NCH, 2, nt))
    w2 = rng.normal(0.0, np.sqrt(2.0 / (NCH * nt)), size=(NCH, NCH, nt))
    return {"w1": w1, "b1": np.zeros(NCH), "w2": w2, "b2": np.zeros(NCH),
            "w3": np.zeros((1, NCH, nt)), "b3": np.zeros(1)}


def _shift(x, off, dim):
    """y[p] = x[p + off] with zeros outside (x: (c, *shape))."""
    y = np.zeros_like(x)
    shape = x.shape[1:]
    offs = off if dim == 3 else off[1:]
    src, dst = [slice(None)], [slice(None)]
    for o, n in zip(offs, shape):
        if o >= 0:
            src.append(slice(o, n))
            dst.append(slice(0, n - o))
        else:
            src.append(slice(0, n + o))
            dst.append(slice(-o, n))
    y[tuple(dst)] = x[tuple(src)]
    return y


def conv(x, w, b, dim):
    cout = w.shape[0]
    out = np.zeros((cout,) + x.shape[1:], dtype=x.dtype)
    for t, off in enumerate(taps(dim)):
        xs = _shift(x, off, dim)
        out += np.tensordot(w[:, :, t].astype(x.dtype), xs, axes=(1, 0))
    out += b.astype(x.dtype).reshape((cout,) + (1,) * (x.ndim - 1))
    return out


def conv_backward(x, w, gout, dim):
    """Gradients of sum(gout * conv(x; w, b)) with respect to x, w and b."""
    gx = np.zeros_like(x)
    gw = np.zeros(w.shape, dtype=np.float64)
    for t, off in enumerate(taps(dim)):
        xs = _shift(x, off, dim)
        gw[:, :, t] = np.tensordot(gout, xs, axes=(tuple(range(1, x.ndim)), tuple(range(1, x.ndim))))
        neg = tuple(-o for o in off)
        gx += _shift(np.tensordot(w[:, :, t].T.astype(x.dtype), gout, axes=(1, 0)), neg, dim)
    gb = gout.sum(axis=tuple(range(1, x.ndim))).astype(np.float64)
    return gx, gw, gb


def forward(net, f, dim, precision="fp64"):
    """Network output o (the tanh argument) and the activations for backward."""
    if precision == "bf16":
        dt = np.float32
        W = {k: (bf16_round(v) if k[0] == "w" else np.asarray(v, dtype=np.float32)) for k, v in net.items()}
    else:
        dt = np.float64
        W = {k: np.asarray(v, dtype=np.float64) for k, v in net.items()}
    rnd = bf16_round if precision == "bf16" else (lambda v: v)
    x0 = rnd(f.astype(dt))
    z1 = conv(x0, W["w1"], W["b1"], dim)
    y1 = rnd(np.maximum(z1, 0))
    z2 = conv(y1, W["w2"], W["b2"], dim)
    y2 = rnd(np.maximum(z2, 0))
    o = conv(y2, W["w3"], W["b3"], dim)[0]
    return o, {"x0": x0, "z1": z1, "y1": y1, "z2": z2, "y2": y2, "W": W}


def backward(cache, go, dim):
    """Gradients of sum(go * o) with respect to every weight."""
    W = cache["W"]
    g3 = go[None].astype(cache["y2"].dtype)
    gy2, gw3, gb3 = conv_backward(cache["y2"], W["w3"], g3, dim)
    gz2 = gy2 * (cache["z2"] > 0)
    gy1, gw2, gb2 = conv_backward(cache["y1"], W["w2"], gz2, dim)
    gz1 = gy1 * (cache["z1"] > 0)
    _, gw1, gb1 = conv_backward(cache["x0"], W["w1"], gz1, dim)
    return {"w1": gw1, "b1": gb1, "w2": gw2, "b2": gb2, "w3": gw3, "b3": gb3}


OMEGA_SPAN = 0.35


def omega_of(o, omega0):
    return omega0 * (1.0 + OMEGA_SPAN * np.tanh(o))


# ------------------------------------------------------------ weighted cycle
def vcycle_weighted(H, r, omega):
    """One V(1,1) cycle whose fine smoother uses W = diag(omega / A_kk)."""
    lvl = H.levels[0]
    if lvl.chol is not None:
        return amg.coarse_solve(lvl, r)
    w = omega / lvl.diag
    z1 = w * r
    ec = amg.vcycle(H, lvl.R @ (r - lvl.A @ z1), 1)
    z2 = z1 + lvl.P @ ec
    return z2 + w * (r - lvl.A @ z2)


def loss_and_grad(H, omega, E):
    """L and dL/domega (per unknown) for the error samples in the columns of E."""
    lvl = H.levels[0]
    A, d = lvl.A, lvl.diag
    w = omega / d
    m = E.shape[1]
    L = 0.0
    gw = np.zeros(A.shape[0])
    for s in range(m):
        e = E[:, s]
        r = A @ e
        nrm = float(e @ r)
        z1 = w * r
        ec = amg.vcycle(H, lvl.R @ (r - A @ z1), 1)
        z2 = z1 + lvl.P @ ec
        t2 = r - A @ z2
        z = z2 + w * t2
        ep = e - z
        Aep = A @ ep
        L += 0.5 * float(ep @ Aep) / nrm
        g = -Aep / nrm
        u = g - A @ (w * g)
        v = u - A @ (lvl.P @ amg.vcycle(H, lvl.R @ u, 1))
        gw += g * t2 + v * r
    return L / m, (gw / m) / d


def error_samples(H, m, seed, sweeps=2):
    """e = (I - M_0 A)^sweeps xi, columns normalised in the 2-norm."""
    A = H.levels[0].A
    rng = np.random.default_rng(seed)
    E = rng.standard_normal((A.shape[0], m))
    for s in range(m):
        e = E[:, s]
        for _ in range(sweeps):
            e = e - amg.vcycle(H, A @ e)
        E[:, s] = e / np.linalg.norm(e)
    return E


def full_grad(net, f, dim, H, nodes, kind, E, precision="fp64"):
    """Loss and gradients with respect to the network weights.

    nodes: flat node index of every unknown (level-0 order); kind: node kinds.
    """
    o, cache = forward(net, f, dim, precision)
    omega0 = H.levels[0].omega
    oo = o.ravel()[nodes].astype(np.float64)
    om = omega_of(oo, omega0)
    L, gom = loss_and_grad(H, om, E)
    go = np.zeros(o.size)
    go[nodes] = gom * omega0 * OMEGA_SPAN * (1.0 - np.tanh(oo) ** 2)
    grads = backward(cache, go.reshape(o.shape).astype(o.dtype), dim)
    return L, grads, om


class Adam:
    def __init__(self, net, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = {k: np.zeros_like(v) for k, v in net.items()}
        self.v = {k: np.zeros_like(v) for k, v in net.items()}
        self.t = 0

    def step(self, net, grads):
        self.t += 1
        for k in net:
            g = grads[k]
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * g
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * g * g
            mh = self.m[k] / (1 - self.b1 ** self.t)
            vh = self.v[k] / (1 - self.b2 ** self.t)
            net[k] = net[k] - self.lr * mh / (np.sqrt(vh) + self.eps)
        return net
