"""Seeded synthetic inputs: grids, level sets, manufactured solutions.

This module only *samples* the problem data that a user of the solver would
hand in: the node grid, the level-set function psi at the nodes (negative
inside the domain), the source f, the Dirichlet data u_D and, for the heat
problem, random smooth initial data.  It contains none of the method's
arithmetic (no classification, interpolation weights, operator or solver), so
both the CPU oracle and the GPU path may consume its arrays.

Geometries follow the level-set description of Sec. 2 (the mask is the sign of
psi) and the workloads of Sec. 3: a disk, a five-armed star, an ellipsoid and
random perturbed stars standing in for the shape-optimisation batch of
Sec. 3.6.  No dataset is involved anywhere; every input is analytic or drawn
from a seeded numpy generator.

The node grid puts node i of axis a at x0[a] + i*h, i = 0..n[a] (so n[a]+1
nodes per axis; the box [-0.5, 0.5]^d with n cells per side gives h = 1/n).
Arrays are numpy C-order with index order [z, y, x] (x fastest), i.e. the
lexicographic numbering of Sec. 2.4.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional, Tuple

import numpy as np

SEED_BASE = 220406083


@dataclass(frozen=True)
class Grid:
    dim: int
    n: Tuple[int, ...]          # cells per axis, x first
    x0: Tuple[float, ...]       # coordinate of node 0 per axis, x first
    h: float

    @property
    def shape(self) -> Tuple[int, ...]:
        """numpy array shape of a node field, [z, y, x] order."""
        return tuple(m + 1 for m in reversed(self.n))

    @property
    def n_nodes(self) -> int:
        return int(np.prod(self.shape))

    def axis_coords(self, axis: int) -> np.ndarray:
        """Node coordinates along physical axis (0 = x, 1 = y, 2 = z)."""
        i = np.arange(self.n[axis] + 1, dtype=np.float64)
        return self.x0[axis] + i * self.h

    def mesh(self):
        """Coordinate arrays (X, Y[, Z]) broadcast to the node field shape."""
        axes = [self.axis_coords(a) for a in range(self.dim)]
        grids = np.meshgrid(*reversed(axes), indexing="ij")  # [z,y,x] order
        return tuple(reversed(grids))                          # X, Y[, Z]


def unit_box_grid(dim: int, n: int) -> Grid:
    """Box [-0.5, 0.5]^dim with n cells per side, h = 1/n."""
    return Grid(dim=dim, n=(n,) * dim, x0=(-0.5,) * dim, h=1.0 / n)


@dataclass
class Problem:
    """One Poisson / shifted-Poisson problem instance."""
    name: str
    grid: Grid
    psi: np.ndarray                              # node field, < 0 inside
    f: np.ndarray                                # node field (source of -Lap u = f)
    u_exact: Optional[Callable] = None           # u(X, Y[, Z], xp) or None
    u_dirichlet: Optional[Callable] = None       # boundary data u_D(X, Y[, Z], xp)
    sigma: float = 0.0                           # diagonal shift (heat: 1/dt)
    tol: float = 1e-8
    meta: dict = field(default_factory=dict)


# ---------------------------------------------------------------- geometries

def psi_disk(grid: Grid, center=(0.013, 0.021), radius=0.4) -> np.ndarray:
    X, Y = grid.mesh()
    return np.sqrt((X - center[0]) ** 2 + (Y - center[1]) ** 2) - radius


def psi_star(grid: Grid, r0=0.3, amp=0.1, arms=5) -> np.ndarray:
    """psi = |x| - (r0 + amp cos(arms*phi))."""
    X, Y = grid.mesh()
    phi = np.arctan2(Y, X)
    return np.sqrt(X * X + Y * Y) - (r0 + amp * np.cos(arms * phi))


def psi_ellipsoid(grid: Grid, semi=(0.4, 0.3, 0.35)) -> np.ndarray:
    X, Y, Z = grid.mesh()
    return (X / semi[0]) ** 2 + (Y / semi[1]) ** 2 + (Z / semi[2]) ** 2 - 1.0


def psi_random_star(grid: Grid, c, phase, r0=0.3) -> np.ndarray:
    """psi = |x| - (r0 + sum_m c_m cos(m phi + phase_m)), m = 2..2+len(c)-1."""
    X, Y = grid.mesh()
    phi = np.arctan2(Y, X)
    r = np.full_like(X, r0)
    for m, (cm, pm) in enumerate(zip(c, phase), start=2):
        r = r + cm * np.cos(m * phi + pm)
    return np.sqrt(X * X + Y * Y) - r


def psi_halfplane_box(grid: Grid, normal, offset, half_width=0.35) -> np.ndarray:
    """Intersection of a tilted half-plane {n.x < offset} with a centred box.

    Piecewise linear: along any grid line whose two nodes straddle the tilted
    face and lie away from the box faces, linear interpolation of psi is exact.
    """
    comps = grid.mesh()
    lin = sum(nc * X for nc, X in zip(normal, comps)) - offset
    box = np.max(np.stack([np.abs(X) for X in comps]), axis=0) - half_width
    return np.maximum(lin, box)


# ------------------------------------------------------ manufactured solutions

def _xp_of(a):
    try:
        import torch
        if isinstance(a, torch.Tensor):
            return torch
    except ImportError:  # pragma: no cover
        pass
    return np


def u_disk(X, Y):
    xp = _xp_of(X)
    return xp.sin(2 * math.pi * X) * xp.cos(3 * math.pi * Y)


def u_star(X, Y):
    xp = _xp_of(X)
    return xp.exp(X) * xp.sin(4 * math.pi * Y)


def u_ellipsoid(X, Y, Z):
    xp = _xp_of(X)
    return xp.sin(math.pi * X) * xp.sin(2 * math.pi * Y) * xp.sin(3 * math.pi * Z)


def zero_data(*coords):
    return 0.0 * coords[0]


def linear_field(coef):
    """u = coef[0] + coef[1] x + coef[2] y (+ coef[3] z); -Lap u = 0."""
    def u(*coords):
        out = coef[0] + 0.0 * coords[0]
        for c, X in zip(coef[1:], coords):
            out = out + c * X
        return out
    return u


# -------------------------------------------------------------- the workloads

def disk_poisson(n: int = 128) -> Problem:
    """2-D Poisson on the disk r = 0.4 centred at (0.013, 0.021); u = sin(2 pi x) cos(3 pi y)."""
    g = unit_box_grid(2, n)
    X, Y = g.mesh()
    return Problem("disk2d", g, psi_disk(g), 13.0 * math.pi ** 2 * u_disk(X, Y),
                   u_exact=u_disk, u_dirichlet=u_disk, tol=1e-10)


def star_poisson(n: int = 2048) -> Problem:
    """2-D Poisson on the star r = 0.3 + 0.1 cos(5 phi); u = exp(x) sin(4 pi y)."""
    g = unit_box_grid(2, n)
    X, Y = g.mesh()
    return Problem("star2d", g, psi_star(g), (16.0 * math.pi ** 2 - 1.0) * u_star(X, Y),
                   u_exact=u_star, u_dirichlet=u_star, tol=1e-8)


def ellipsoid_poisson(n: int = 256) -> Problem:
    """3-D Poisson on the ellipsoid (0.4, 0.3, 0.35); u = sin(pi x) sin(2 pi y) sin(3 pi z)."""
    g = unit_box_grid(3, n)
    X, Y, Z = g.mesh()
    return Problem("ellipsoid3d", g, psi_ellipsoid(g),
                   14.0 * math.pi ** 2 * u_ellipsoid(X, Y, Z),
                   u_exact=u_ellipsoid, u_dirichlet=u_ellipsoid, tol=1e-8)


def heat_initial(grid: Grid, rhs_id: int, kmax: int = 8) -> np.ndarray:
    """u0 = sum_{kx,ky in 1..kmax} a_k sin(kx pi x) sin(ky pi y), a_k ~ N(0, 1/|k|^2)."""
    rng = np.random.default_rng(SEED_BASE + rhs_id)
    X, Y = grid.mesh()
    u0 = np.zeros_like(X)
    for kx in range(1, kmax + 1):
        for ky in range(1, kmax + 1):
            std = 1.0 / math.sqrt(kx * kx + ky * ky)
            a = rng.normal(0.0, std)
            u0 += a * np.sin(kx * math.pi * X) * np.sin(ky * math.pi * Y)
    return u0


def heat_coefficients(rhs_id: int, kmax: int = 8) -> np.ndarray:
    """The a_k of heat_initial for one rhs_id, as a [kx-1, ky-1] array (same draws, same order)."""
    rng = np.random.default_rng(SEED_BASE + rhs_id)
    a = np.zeros((kmax, kmax))
    for kx in range(1, kmax + 1):
        for ky in range(1, kmax + 1):
            a[kx - 1, ky - 1] = rng.normal(0.0, 1.0 / math.sqrt(kx * kx + ky * ky))
    return a


def heat_initial_batch(grid: Grid, rhs_ids, device, kmax: int = 8):
    """heat_initial for several rhs_ids at once as a torch tensor (nrhs, ny+1, nx+1) on
    `device`: u0 = S_y A^T S_x^T per right-hand side (separable sine modes), FP64.
    Equal to heat_initial up to summation order."""
    import torch
    x = torch.as_tensor(grid.axis_coords(0), dtype=torch.float64, device=device)
    y = torch.as_tensor(grid.axis_coords(1), dtype=torch.float64, device=device)
    k = torch.arange(1, kmax + 1, dtype=torch.float64, device=device)
    sx = torch.sin(math.pi * x[:, None] * k[None, :])          # (nx+1, K)
    sy = torch.sin(math.pi * y[:, None] * k[None, :])          # (ny+1, K)
    A = torch.as_tensor(np.stack([heat_coefficients(r, kmax) for r in rhs_ids]), device=device)  # (R, kx, ky)
    return torch.matmul(torch.matmul(sy, A.transpose(1, 2).contiguous()), sx.t().contiguous())


def star_heat(n: int = 1024, rhs_id: int = 0) -> Problem:
    """One backward-Euler heat step on the star: (A + I/dt) u1 = u0/dt, dt = h, u_D = 0."""
    g = unit_box_grid(2, n)
    dt = g.h
    u0 = heat_initial(g, rhs_id)
    return Problem("star2d_heat", g, psi_star(g), u0 / dt, u_exact=None,
                   u_dirichlet=zero_data, sigma=1.0 / dt, tol=1e-8,
                   meta={"dt": dt, "u0": u0, "rhs_id": rhs_id})


def random_star_params(count: int = 256, seed: int = SEED_BASE):
    """Parameters of the shape-optimisation batch: (N, c[5], phase[5]) per geometry."""
    rng = np.random.default_rng(seed)
    sizes = (256, 384, 512, 768, 1024)
    out = []
    while len(out) < count:
        n = int(rng.choice(sizes))
        c = rng.uniform(0.0, 0.04, size=5)
        ph = rng.uniform(0.0, 2.0 * math.pi, size=5)
        h = 1.0 / n
        if 0.3 + c.sum() > 0.5 - 2.0 * h:      # keep the outer node layer outside
            continue
        out.append((n, c, ph))
    return out


def random_star_poisson(n: int, c, phase) -> Problem:
    g = unit_box_grid(2, n)
    return Problem("random_star2d", g, psi_random_star(g, c, phase),
                   np.ones(g.shape), u_exact=None, u_dirichlet=zero_data, tol=1e-8)


def disk_mms(n: int, center=(0.013, 0.021), radius=0.4) -> Problem:
    """Manufactured-solution disk used for convergence sweeps (config-1 data at any n)."""
    g = unit_box_grid(2, n)
    X, Y = g.mesh()
    return Problem("disk2d_mms", g, psi_disk(g, center, radius),
                   13.0 * math.pi ** 2 * u_disk(X, Y),
                   u_exact=u_disk, u_dirichlet=u_disk, tol=1e-10)


def ellipsoid_mms(n: int) -> Problem:
    return ellipsoid_poisson(n)


WORKLOADS = {
    "disk2d_128": lambda: disk_poisson(128),
    "star2d_2048": lambda: star_poisson(2048),
    "star2d_heat_1024": lambda: star_heat(1024, 0),
    "ellipsoid3d_256": lambda: ellipsoid_poisson(256),
}


# ------------------------------------------------------- time-dependent inputs

def wave_disk_grid(n: int) -> Grid:
    """Box [-1.1, 1.1]^2 with n cells per side (the wave example's grid)."""
    return Grid(dim=2, n=(n, n), x0=(-1.1, -1.1), h=2.2 / n)


def psi_unit_disk(grid: Grid) -> np.ndarray:
    X, Y = grid.mesh()
    return np.sqrt(X * X + Y * Y) - 1.0


def bessel_zero(m: int = 7, k: int = 7) -> float:
    """k-th positive zero of J_m."""
    from scipy.special import jn_zeros
    return float(jn_zeros(m, k)[-1])


def standing_mode(X, Y, t: float, m: int = 7, k: int = 7) -> np.ndarray:
    """u = J_m(kappa r) cos(m theta) cos(kappa t), kappa the k-th zero of J_m
    (vanishes on the unit circle)."""
    from scipy.special import jv
    kappa = bessel_zero(m, k)
    r = np.sqrt(X * X + Y * Y)
    th = np.arctan2(Y, X)
    return jv(m, kappa * r) * np.cos(m * th) * np.cos(kappa * t)


def wave_schedule(n: int, dt_over_h: float, periods: float = 10.2, m: int = 7, k: int = 7):
    """(dt, nsteps) reaching `periods` periods of the standing mode exactly with
    dt at most dt_over_h * h."""
    h = 2.2 / n
    T = periods * 2.0 * math.pi / bessel_zero(m, k)
    nsteps = int(math.ceil(T / (dt_over_h * h)))
    return T / nsteps, nsteps


def heat_cn_grid(n: int) -> Grid:
    """Box [-1, 1]^2 with n cells per side (the heat example's grid)."""
    return Grid(dim=2, n=(n, n), x0=(-1.0, -1.0), h=2.0 / n)


def psi_heat_disk(grid: Grid) -> np.ndarray:
    """Disk of radius 1/2, psi = x^2 + y^2 - 1/4 (< 0 inside)."""
    X, Y = grid.mesh()
    return X * X + Y * Y - 0.25


def heat_cn_exact(X, Y, t: float):
    """u = exp(-t) (x^2 + y^2 - 1/4); with beta = 1 its source is
    f = u_t - Lap u = -u - 4 exp(-t)."""
    return math.exp(-t) * (X * X + Y * Y - 0.25)


def heat_cn_source(X, Y, t: float):
    return -heat_cn_exact(X, Y, t) - 4.0 * math.exp(-t)


# ------------------------------------------------------- variable coefficient
#
# Eq. (1) with a variable conductivity beta: the scheme of Eq.
# (central_difference) takes beta at the cell faces, beta_{i+1/2,j} between
# nodes (i, j) and (i+1, j).  The caller samples beta there; these helpers
# give the face fields as the library takes them: face[a] is a node field
# holding beta at the midpoint between each node and its neighbour in +axis a
# (the last node of each line holds beta one half step beyond the grid; it
# borders no unknown).

def beta_faces(grid: Grid, beta) -> np.ndarray:
    """(dim, *grid.shape) array: beta at the +axis face midpoint of every node."""
    comps = grid.mesh()
    out = np.empty((grid.dim,) + tuple(grid.shape))
    for a in range(grid.dim):
        moved = [c + (0.5 * grid.h if b == a else 0.0) for b, c in enumerate(comps)]
        out[a] = beta(*moved)
    return out


def beta_heat(X, Y):
    """Sec. 3.4 conductivity beta = 0.25 - x^2 - y^2 (vanishes on the disk's edge)."""
    return 0.25 - X * X - Y * Y


def heat_beta_source(X, Y, t: float):
    """Sec. 3.4: u = exp(-t) (x^2 + y^2 - 1/4) with beta = 1/4 - x^2 - y^2;
    div(beta grad u) = exp(-t) (1 - 8 r^2), so u_t = div(beta grad u) + f needs
    f = exp(-t) (7 r^2 - 3/4)."""
    return math.exp(-t) * (7.0 * (X * X + Y * Y) - 0.75)


def beta_bone(X, Y):
    """Sec. 3.3.1 conductivity beta = 2 + sin(x y)."""
    xp = _xp_of(X)
    return 2.0 + xp.sin(X * Y)


def u_bone(X, Y):
    """Sec. 3.3.1 exact solution u = e^x (x^2 sin y + y^2)."""
    xp = _xp_of(X)
    return xp.exp(X) * (X * X * xp.sin(Y) + Y * Y)


def f_bone(X, Y):
    """-div(beta grad u) for beta_bone and u_bone:
    beta Lap u + grad beta . grad u with Lap u = e^x (4x sin y + 2 sin y + y^2 + 2),
    u_x = e^x (x^2 sin y + 2x sin y + y^2), u_y = e^x (x^2 cos y + 2y),
    grad beta = cos(xy) (y, x)."""
    xp = _xp_of(X)
    ex = xp.exp(X)
    s, c = xp.sin(Y), xp.cos(Y)
    lap = ex * (4.0 * X * s + 2.0 * s + Y * Y + 2.0)
    ux = ex * (X * X * s + 2.0 * X * s + Y * Y)
    uy = ex * (X * X * c + 2.0 * Y)
    cxy = xp.cos(X * Y)
    return -((2.0 + xp.sin(X * Y)) * lap + cxy * (Y * ux + X * uy))


def bone_beta_poisson(n: int) -> Problem:
    """The bone example's beta and exact solution (Sec. 3.3.1) on a five-armed
    star around (0, 1.5) in the example's box [-2, 2] x [-1, 3] (the bone's
    parametric boundary itself is not used): -div(beta grad u) = f."""
    g = Grid(dim=2, n=(n, n), x0=(-2.0, -1.0), h=4.0 / n)
    X, Y = g.mesh()
    Yc = Y - 1.5
    phi = np.arctan2(Yc, X)
    psi = np.sqrt(X * X + Yc * Yc) - (1.1 + 0.3 * np.cos(5 * phi))
    return Problem("bone_beta_star", g, psi, f_bone(X, Y), u_exact=u_bone, u_dirichlet=u_bone, tol=1e-10,
                   meta={"beta": beta_bone})


# ------------------------------------------------- shape-parameter QOI studies
#
# Sec. 3.6: Poisson problems (beta = 1, zero Dirichlet data, source 3 in the
# paper's convention div(beta grad u) = f, i.e. f = -3 for -Lap u = f here)
# on one grid for a family of geometries, each giving one quantity of interest.

QOI_SOURCE = -3.0


def qoi_ellipse_grid(n: int = 1024) -> Grid:
    """Box [-2.2, 2.2]^2 with n (even) cells per side: the origin is a node and
    every ellipse of the family (semi-axes up to 2) lies inside."""
    if n % 2:
        raise ValueError("n must be even")
    return Grid(dim=2, n=(n, n), x0=(-2.2, -2.2), h=4.4 / n)


def psi_area_ellipse(grid: Grid, a: float) -> np.ndarray:
    """x^2/a^2 + y^2 a^2 - 1 (semi-axes a and 1/a, area pi for every a)."""
    X, Y = grid.mesh()
    return X * X / (a * a) + Y * Y * (a * a) - 1.0


def qoi_ellipse_params(count: int = 61):
    """a on [0.5, 2], equally spaced."""
    return np.linspace(0.5, 2.0, count)


def qoi_rotated_grid() -> Grid:
    """501 x 501 nodes on [-5, 5]^2 (h = 0.02; the origin is node (250, 250))."""
    return Grid(dim=2, n=(500, 500), x0=(-5.0, -5.0), h=0.02)


def psi_rotated_ellipse(grid: Grid, theta: float) -> np.ndarray:
    """Ellipse with semi-axes 4 and 2 rotated by theta."""
    X, Y = grid.mesh()
    c, s = math.cos(theta), math.sin(theta)
    return (X * c - Y * s) ** 2 / 16.0 + (X * s + Y * c) ** 2 / 4.0 - 1.0


def qoi_rotated_params(count: int = 64):
    """theta on [0, 2 pi), equally spaced."""
    return np.arange(count) * (2.0 * math.pi / count)


def qoi_rectangle_weights(grid: Grid, rect=((-1.0, 1.0), (-0.5, 0.5))) -> np.ndarray:
    """Node weights of the composite trapezoid rule over an axis-aligned
    rectangle whose sides lie on grid lines (h^2 times 1, 1/2 on an edge, 1/4 at
    a corner; zero outside).  The quantity of interest int u is w . u."""
    h = grid.h
    w1 = []
    for axis, (lo, hi) in enumerate(rect):
        i0 = (lo - grid.x0[axis]) / h
        i1 = (hi - grid.x0[axis]) / h
        if abs(i0 - round(i0)) > 1e-9 or abs(i1 - round(i1)) > 1e-9:
            raise ValueError("rectangle sides must lie on grid lines")
        i0, i1 = int(round(i0)), int(round(i1))
        w = np.zeros(grid.n[axis] + 1)
        w[i0:i1 + 1] = 1.0
        w[i0] = w[i1] = 0.5
        w1.append(w * h)
    return w1[1][:, None] * w1[0][None, :]


def psi_staircases(grid: Grid, stripe: int = 12, step: int = 20, margin: int = 4) -> np.ndarray:
    """Horizontal stripes whose upper boundary descends one node row every
    `step` columns (a sawtooth of staircases), in node units scaled by h.  An
    unknown at the foot of each step sees the grid line continue inside for
    about `step` nodes beyond its boundary point: thousands of long walks
    along grid lines.  (2-D; psi is never zero at a node.)"""
    X, Y = grid.mesh()
    c = np.rint((X - grid.x0[0]) / grid.h)
    r = np.rint((Y - grid.x0[1]) / grid.h)
    k = np.floor((r - margin) / stripe)
    rr = (r - margin) - k * stripe
    per_tooth = stripe - 4
    s = np.floor(np.mod(c, per_tooth * step) / step)
    top = (stripe - 1.5) - s
    psi = np.maximum(1.5 - rr, rr - top)
    edge = (r < margin) | (r > grid.n[1] - margin) | (c < margin) | (c > grid.n[0] - margin)
    return np.where(edge, 1.0, psi) * grid.h


def staircase_poisson(n: int = 512) -> Problem:
    """Poisson problem on the staircase stripes (psi_staircases): f = 1 and
    Dirichlet data sin 3x + y; many disconnected thin components."""
    g = unit_box_grid(2, n)

    def u_d(X, Y, xp=np):
        return xp.sin(3.0 * X) + Y

    return Problem("staircases2d", g, psi_staircases(g), np.ones(g.shape), u_dirichlet=u_d, tol=1e-10)
