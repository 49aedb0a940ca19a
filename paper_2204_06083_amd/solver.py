"""Python entry points over the C ABI, taking torch tensors on the GPU.

Each function checks shapes and dtypes, passes raw device pointers and the
current HIP stream to libebamg.so and wraps the outputs.  All arithmetic runs
in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib as L


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _field(t: torch.Tensor, shape, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP tensor")
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous {dtype} of shape {tuple(shape)}, got "
                         f"{t.dtype} {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


@dataclass
class Assembly:
    grid: object
    kind: torch.Tensor          # int8 node field
    a: torch.Tensor             # float64 node field
    cuts: torch.Tensor          # uint8 [cap*56] device buffer of eb_cut_t records
    n_unknowns: int
    n_cuts: int
    beta: Optional[torch.Tensor] = None   # face conductivities (variable beta), else None

    def cuts_host(self) -> np.ndarray:
        raw = self.cuts[: self.n_cuts * 56].cpu().numpy()
        return raw.view(L.CUT_DTYPE)

    def cut_coordinates(self):
        """Crossing coordinates as device tensors (x, y[, z]) in record order:
        strided views into the records (no copy; read them, do not write)."""
        if self.n_cuts == 0:
            z = torch.zeros(0, dtype=torch.float64, device=self.kind.device)
            return tuple(z for _ in range(self.grid.dim))
        rec = self.cuts[: self.n_cuts * 56].view(torch.float64).view(self.n_cuts, 7)
        return tuple(rec[:, 4 + p] for p in range(self.grid.dim))


def assemble_diag(grid, psi: torch.Tensor, cuts_cap: Optional[int] = None, mode: str = "line",
                  beta: Optional[torch.Tensor] = None) -> Assembly:
    """Classify nodes and build a_k and the cut records (eb_assemble_diag_mode;
    mode "line", "mixed" or "rbf"; with beta, the face conductivities of shape
    (dim, *grid.shape), eb_assemble_diag_beta)."""
    lib = L.lib()
    if mode not in L.BC_MODES:
        raise ValueError(f"unknown boundary mode {mode!r}")
    m = L.BC_MODES[mode]
    g = L.make_grid(grid)
    shape = grid.shape
    dev = psi.device
    psi_p = _field(psi, shape, torch.float64, "psi")
    beta_p = None
    if beta is not None:
        beta = beta.contiguous()
        beta_p = _field(beta, (grid.dim,) + tuple(shape), torch.float64, "beta")
    kind = torch.empty(shape, dtype=torch.int8, device=dev)
    a = torch.empty(shape, dtype=torch.float64, device=dev)
    nu, nc = C.c_int64(0), C.c_int64(0)

    def call(cuts_ptr, cap):
        if beta_p is not None:
            return lib.eb_assemble_diag_beta(C.byref(g), psi_p, beta_p, m, C.c_void_p(kind.data_ptr()),
                                             C.c_void_p(a.data_ptr()), cuts_ptr, cap, C.byref(nu), C.byref(nc),
                                             _stream())
        return lib.eb_assemble_diag_mode(C.byref(g), psi_p, m, C.c_void_p(kind.data_ptr()), C.c_void_p(a.data_ptr()),
                                         cuts_ptr, cap, C.byref(nu), C.byref(nc), _stream())

    if cuts_cap is None:
        # counts first (capacity 0 reports the required size), then the records
        L.check(call(None, 0), "eb_assemble_diag", ok=(L.EB_OK, L.EB_ENOSPC))
        cuts_cap = nc.value
    cuts = torch.empty(max(cuts_cap, 1) * 56, dtype=torch.uint8, device=dev)
    L.check(call(C.c_void_p(cuts.data_ptr()), int(cuts_cap)), "eb_assemble_diag")
    return Assembly(grid, kind, a, cuts, nu.value, nc.value, beta)


def check_spd(asm: Assembly, cuts: Optional[torch.Tensor] = None) -> tuple:
    """A-priori SPD test of the operator (eb_check_spd): (segments, failing).

    cuts: the assembly's record buffer (default) or a copy with altered c."""
    lib = L.lib()
    g = L.make_grid(asm.grid)
    buf = asm.cuts if cuts is None else cuts
    ns, nf = C.c_int64(0), C.c_int64(0)
    rc = lib.eb_check_spd(C.byref(g), C.c_void_p(asm.kind.data_ptr()), C.c_void_p(buf.data_ptr()),
                          int(asm.n_cuts), C.byref(ns), C.byref(nf), _stream())
    L.check(rc, "eb_check_spd")
    return ns.value, nf.value


def assemble_rhs(asm: Assembly, f: torch.Tensor, u_at_cuts: torch.Tensor) -> torch.Tensor:
    lib = L.lib()
    g = L.make_grid(asm.grid)
    shape = asm.grid.shape
    f_p = _field(f, shape, torch.float64, "f")
    u = u_at_cuts.contiguous().to(torch.float64)
    if u.numel() != asm.n_cuts:
        raise ValueError("u_at_cuts must hold one value per cut record")
    b = torch.empty(shape, dtype=torch.float64, device=f.device)
    rc = lib.eb_assemble_rhs(C.byref(g), C.c_void_p(asm.kind.data_ptr()), f_p, C.c_void_p(asm.cuts.data_ptr()),
                             asm.n_cuts, C.c_void_p(u.data_ptr()), C.c_void_p(b.data_ptr()), _stream())
    L.check(rc, "eb_assemble_rhs")
    return b


def assemble_rhs_islands(asm: Assembly, canvas: "IslandCanvas", f: torch.Tensor,
                         u_at_cuts: Optional[torch.Tensor] = None) -> torch.Tensor:
    """eb_assemble_rhs_islands: the right-hand side of an island canvas, each
    island's source in its own units (the library scales it by that island's h^2)."""
    lib = L.lib()
    g = L.make_grid(asm.grid)
    shape = asm.grid.shape
    f_p = _field(f, shape, torch.float64, "f")
    if u_at_cuts is None:
        u_at_cuts = torch.zeros(asm.n_cuts, dtype=torch.float64, device=f.device)
    u = u_at_cuts.contiguous().to(torch.float64)
    if u.numel() != asm.n_cuts:
        raise ValueError("u_at_cuts must hold one value per cut record")
    rows = np.ascontiguousarray(np.asarray(canvas.rows, dtype=np.int32))
    hs = np.ascontiguousarray(np.asarray(canvas.h, dtype=np.float64))
    b = torch.empty(shape, dtype=torch.float64, device=f.device)
    rc = lib.eb_assemble_rhs_islands(C.byref(g), C.c_void_p(asm.kind.data_ptr()), f_p, C.c_void_p(asm.cuts.data_ptr()),
                                     asm.n_cuts, C.c_void_p(u.data_ptr()), int(rows.size - 1),
                                     rows.ctypes.data_as(C.POINTER(C.c_int32)), hs.ctypes.data_as(C.POINTER(C.c_double)),
                                     C.c_void_p(b.data_ptr()), _stream())
    L.check(rc, "eb_assemble_rhs_islands")
    return b


def stencil_apply(grid, kind: torch.Tensor, a: torch.Tensor, sigma: float, x: torch.Tensor,
                  out: Optional[torch.Tensor] = None, beta: Optional[torch.Tensor] = None) -> torch.Tensor:
    lib = L.lib()
    g = L.make_grid(grid)
    shape = grid.shape
    y = out if out is not None else torch.empty(shape, dtype=torch.float64, device=x.device)
    kp, ap = _field(kind, shape, torch.int8, "kind"), _field(a, shape, torch.float64, "a")
    xp, yp = _field(x, shape, torch.float64, "x"), _field(y, shape, torch.float64, "y")
    if beta is not None:
        bp = _field(beta, (grid.dim,) + tuple(shape), torch.float64, "beta")
        rc = lib.stencil_apply_beta(C.byref(g), kp, ap, bp, float(sigma), xp, yp, _stream())
    else:
        rc = lib.stencil_apply(C.byref(g), kp, ap, float(sigma), xp, yp, _stream())
    L.check(rc, "stencil_apply")
    return y


def wave_rhs(asm: "Assembly", theta: float, dt: float, scale: float, un: torch.Tensor, unm1: torch.Tensor,
             out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """eb_wave_rhs: scale (2 u^n - u^{n-1} - dt^2 A ((1 - 2 theta) u^n + theta u^{n-1}))."""
    shape = asm.grid.shape
    g = L.make_grid(asm.grid)
    y = out if out is not None else torch.empty(shape, dtype=torch.float64, device=un.device)
    kp, ap = _field(asm.kind, shape, torch.int8, "kind"), _field(asm.a, shape, torch.float64, "a")
    up, ump = _field(un, shape, torch.float64, "un"), _field(unm1, shape, torch.float64, "unm1")
    yp = _field(y, shape, torch.float64, "out")
    if asm.beta is not None:
        bp = _field(asm.beta, (asm.grid.dim,) + tuple(shape), torch.float64, "beta")
        rc = L.lib().eb_wave_rhs_beta(C.byref(g), kp, ap, bp, float(theta), float(dt), float(scale), up, ump, yp,
                                      _stream())
    else:
        rc = L.lib().eb_wave_rhs(C.byref(g), kp, ap, float(theta), float(dt), float(scale), up, ump, yp, _stream())
    L.check(rc, "eb_wave_rhs")
    return y


def stencil_combine(asm: "Assembly", sigma: float, alpha: float, x: torch.Tensor, beta: float = 0.0,
                    y: Optional[torch.Tensor] = None, gamma: float = 0.0, z: Optional[torch.Tensor] = None,
                    out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """eb_stencil_combine: alpha (A + sigma I) x + beta y + gamma z."""
    shape = asm.grid.shape
    g = L.make_grid(asm.grid)
    o = out if out is not None else torch.empty(shape, dtype=torch.float64, device=x.device)
    yp = _field(y, shape, torch.float64, "y") if y is not None else None
    zp = _field(z, shape, torch.float64, "z") if z is not None else None
    kp, ap = _field(asm.kind, shape, torch.int8, "kind"), _field(asm.a, shape, torch.float64, "a")
    xp, op = _field(x, shape, torch.float64, "x"), _field(o, shape, torch.float64, "out")
    if asm.beta is not None:
        cp = _field(asm.beta, (asm.grid.dim,) + tuple(shape), torch.float64, "beta")
        rc = L.lib().eb_stencil_combine_beta(C.byref(g), kp, ap, cp, float(sigma), float(alpha), xp, float(beta), yp,
                                             float(gamma), zp, op, _stream())
    else:
        rc = L.lib().eb_stencil_combine(C.byref(g), kp, ap, float(sigma), float(alpha), xp, float(beta), yp,
                                        float(gamma), zp, op, _stream())
    L.check(rc, "eb_stencil_combine")
    return o


def heat_backward_euler_batched(asm: "Assembly", H: "Hierarchy", u0: torch.Tensor, dt: float, nsteps: int,
                                tol: float = 1e-8, precision: str = "fp64"):
    """Backward-Euler steps (A + I/dt) u^{n+1} = u^n / dt of the heat equation
    with homogeneous Dirichlet data for a batch of initial conditions u0
    (shape (nrhs, *grid.shape)); H must be set up with sigma = 1/dt.  Every
    step forms its right-hand sides with eb_stencil_combine (beta = 1/dt) and
    solves them in one pcg_solve_batched call warm-started from u^n.  Returns
    (u^nsteps, iterations per step and right-hand side)."""
    nrhs = u0.shape[0]
    u = u0.clone()
    b = torch.empty_like(u)
    nxt = torch.empty_like(u)
    its = []
    for _ in range(nsteps):
        for j in range(nrhs):
            stencil_combine(asm, 0.0, 0.0, u[j], beta=1.0 / dt, y=u[j], out=b[j])
        _, infos = solve_batched(H, b, x0=u, tol=tol, precision=precision, out=nxt)
        u, nxt = nxt, u
        its.append([i["iterations"] for i in infos])
    return u, its


def wave_theta(asm: "Assembly", u0: torch.Tensor, u1: torch.Tensor, dt: float, theta: float, nsteps: int,
               tol: float = 1e-10, precision: str = "fp64", H: Optional["Hierarchy"] = None):
    """theta-scheme for u_tt = Lap u with homogeneous Dirichlet data (Sec. 3.5),
    from u^0 = u0 and u^1 = u1 to u^nsteps.  theta = 0 is the explicit leap-frog
    scheme (one eb_wave_rhs per step); theta > 0 solves
    (A + sigma I) u^{n+1} = sigma w, sigma = 1/(theta dt^2), by PCG warm-started
    from u^n on a hierarchy with that shift (made here unless given).
    Returns (u^nsteps, u^{nsteps-1}, stats)."""
    if theta < 0.0 or nsteps < 1:
        raise ValueError("theta must be >= 0 and nsteps >= 1")
    if nsteps == 1:
        return u1.clone(), u0.clone(), {"steps": 0, "pcg_iterations": 0}
    sigma = 1.0 / (theta * dt * dt) if theta > 0.0 else 0.0
    own = False
    if theta > 0.0 and H is None:
        H = Hierarchy(asm.grid, asm.kind, asm.a, sigma)
        own = True
    bufs = [u0.clone(), u1.clone(), torch.empty_like(u0)]
    rhs = torch.empty_like(u0) if theta > 0.0 else None
    iters = []
    for n in range(2, nsteps + 1):
        um, u, un = bufs[(n - 2) % 3], bufs[(n - 1) % 3], bufs[n % 3]
        if theta == 0.0:
            wave_rhs(asm, 0.0, dt, 1.0, u, um, out=un)
        else:
            wave_rhs(asm, theta, dt, sigma, u, um, out=rhs)
            _, info = H.solve(rhs, x0=u, tol=tol, out=un, precision=precision)
            iters.append(info["iterations"])
    if own:
        H.free()
    stats = {"steps": nsteps - 1, "pcg_iterations": int(sum(iters)),
             "mean_iterations": float(np.mean(iters)) if iters else 0.0}
    return bufs[nsteps % 3], bufs[(nsteps - 1) % 3], stats


def heat_cn(asm: "Assembly", H: "Hierarchy", u0: torch.Tensor, dt: float, nsteps: int, rhs_of_step,
            tol: float = 1e-10, precision: str = "fp64"):
    """Crank-Nicolson for u_t = div(beta grad u) + f (Sec. 3.4; beta from the
    assembly, 1 if it has none):
    (A + (2/dt) I) u^{n+1} = ((2/dt) I - A) u^n + b^n + b^{n+1}, with
    b^n = rhs_of_step(n) (assemble_rhs of the source and Dirichlet data at t_n)
    and H set up with sigma = 2/dt.  PCG warm-started from u^n.
    Returns (u^nsteps, stats)."""
    s2 = 2.0 / dt
    if abs(H.sigma - s2) > 1e-12 * s2:
        raise ValueError("heat_cn: the hierarchy must be set up with sigma = 2/dt")
    u = u0.clone()
    un = torch.empty_like(u0)
    rhs = torch.empty_like(u0)
    b_prev = rhs_of_step(0)
    iters = []
    for k in range(1, nsteps + 1):
        b_next = rhs_of_step(k)
        stencil_combine(asm, -s2, -1.0, u, 1.0, b_prev, 1.0, b_next, out=rhs)
        _, info = H.solve(rhs, x0=u, tol=tol, out=un, precision=precision)
        iters.append(info["iterations"])
        u, un = un, u
        b_prev = b_next
    return u, {"steps": nsteps, "pcg_iterations": int(sum(iters)),
               "mean_iterations": float(np.mean(iters)) if iters else 0.0}


@dataclass
class LevelArrays:
    n: int
    nnz_a: int
    nnz_p: int
    nnz_r: int
    rho: float
    omega: float
    is_coarsest: bool
    max_comp: int
    info: object


class Hierarchy:
    """amg_setup / pcg_solve / amg_free around one handle."""

    def __init__(self, grid, kind: torch.Tensor, a: torch.Tensor, sigma: float = 0.0, coarse_max: int = 256,
                 max_levels: int = 16, min_reduction: float = 0.6, dense_limit: int = 1200,
                 allocator: Optional[str] = None, beta: Optional[torch.Tensor] = None, islands=None):
        """allocator: None (the library's own cache) or "torch": every device
        block of the handle comes from torch's caching allocator.  beta: face
        conductivities (dim, *grid.shape) of a variable-coefficient assembly
        (amg_setup_beta).  islands: the node-row bounds of a canvas of islands
        (IslandCanvas.rows): each island's part of the hierarchy ends where
        its own hierarchy would (amg_setup_islands)."""
        lib = L.lib()
        self.grid = grid
        self.sigma = float(sigma)
        g = L.make_grid(grid)
        p = L.AmgParams(coarse_max, max_levels, min_reduction, dense_limit, 0)
        self.alloc_calls = [0, 0]
        if allocator == "torch":
            dev = torch.cuda.current_device()
            calls = self.alloc_calls

            def _alloc(nbytes, stream, ctx):
                calls[0] += 1
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev, int(stream or 0))

            def _free(ptr, stream, ctx):
                calls[1] += 1
                torch.cuda.caching_allocator_delete(int(ptr))

            # the C callbacks must outlive the handle
            self._alloc_cb = (L.ALLOC_FN(_alloc), L.FREE_FN(_free))
            p.alloc, p.free = self._alloc_cb
        elif allocator is not None:
            raise ValueError(f"unknown allocator {allocator!r}")
        self._params = p
        h = C.c_void_p()
        shape = grid.shape
        if islands is not None:
            if beta is not None:
                raise ValueError("islands and beta cannot be combined")
            rows = np.ascontiguousarray(np.asarray(islands, dtype=np.int32))
            rc = lib.amg_setup_islands(C.byref(g), _field(kind, shape, torch.int8, "kind"),
                                       _field(a, shape, torch.float64, "a"), self.sigma, int(rows.size - 1),
                                       rows.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(p), C.byref(h), _stream())
        elif beta is not None:
            bp = _field(beta, (grid.dim,) + tuple(shape), torch.float64, "beta")
            rc = lib.amg_setup_beta(C.byref(g), _field(kind, shape, torch.int8, "kind"),
                                    _field(a, shape, torch.float64, "a"), bp, self.sigma, C.byref(p), C.byref(h),
                                    _stream())
        else:
            rc = lib.amg_setup(C.byref(g), _field(kind, shape, torch.int8, "kind"),
                               _field(a, shape, torch.float64, "a"), self.sigma, C.byref(p), C.byref(h), _stream())
        L.check(rc, "amg_setup")
        self.handle = h
        self._keep = (kind, a)

    def free(self):
        if getattr(self, "handle", None) and self.handle.value:
            L.lib().amg_free(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    @property
    def n_levels(self) -> int:
        return L.lib().amg_num_levels(self.handle)

    def level(self, l: int) -> LevelArrays:
        info = L.LevelInfo()
        L.check(L.lib().amg_level_info(self.handle, l, C.byref(info)), "amg_level_info")
        return LevelArrays(info.n, info.nnz_a, info.nnz_p, info.nnz_r, info.rho, info.omega,
                           bool(info.is_coarsest), info.max_comp, info)

    def export_level(self, l: int) -> dict:
        """Copy one level's arrays to host numpy (parity tests)."""
        torch.cuda.synchronize()
        lv = self.level(l)
        i = lv.info
        out = dict(n=lv.n, rho=lv.rho, omega=lv.omega, is_coarsest=lv.is_coarsest, max_comp=lv.max_comp)

        def get(ptr, count, dtype):
            arr = np.empty(max(count, 0), dtype=dtype)
            if ptr and count > 0:
                L.copy_device_to_host(ptr, arr.nbytes, arr)
            return arr

        out["a_rowptr"] = get(i.a_rowptr, lv.n + 1, np.int32)
        out["a_col"] = get(i.a_col, lv.nnz_a, np.int32)
        out["a_val"] = get(i.a_val, lv.nnz_a, np.float64)
        out["coords"] = get(i.coords, 3 * lv.n, np.int32).reshape(-1, 3)
        if not lv.is_coarsest:
            nc = self.level(l + 1).n
            out["agg"] = get(i.agg, lv.n, np.int32)
            out["p_rowptr"] = get(i.p_rowptr, lv.n + 1, np.int32)
            out["p_col"] = get(i.p_col, lv.nnz_p, np.int32)
            out["p_val"] = get(i.p_val, lv.nnz_p, np.float64)
            out["r_rowptr"] = get(i.r_rowptr, nc + 1, np.int32)
            out["r_col"] = get(i.r_col, lv.nnz_r, np.int32)
            out["r_val"] = get(i.r_val, lv.nnz_r, np.float64)
        elif i.dense_inv:
            out["dense_inv"] = get(i.dense_inv, lv.n * lv.n, np.float64).reshape(lv.n, lv.n)
        return out

    def fine_nodes(self) -> np.ndarray:
        torch.cuda.synchronize()
        n = self.level(0).n
        arr = np.empty(n, dtype=np.int64)
        ptr = L.lib().amg_fine_nodes(self.handle)
        if n > 0:
            L.copy_device_to_host(ptr, arr.nbytes, arr)
        return arr

    def time_kernel(self, name: Optional[str]):
        """Bracket every launch of one solve kernel with HIP events (None disables)."""
        kid = -1 if name is None else L.KERNEL_IDS[name]
        L.check(L.lib().eb_timing_select(self.handle, kid), "eb_timing_select")

    def kernel_time(self):
        """(launches, total ms) of the selected kernel since the last read."""
        n, ms = C.c_int64(0), C.c_double(0.0)
        L.check(L.lib().eb_timing_read(self.handle, C.byref(n), C.byref(ms)), "eb_timing_read")
        return n.value, ms.value

    def vcycle(self, r: torch.Tensor, precision: str = "fp64") -> torch.Tensor:
        """One V(1,1) cycle z = M r; precision "fp64", "fp32" (single-precision
        cycle) or "bf16" (that cycle with the BF16 fine smoother)."""
        shape = self.grid.shape
        z = torch.empty(shape, dtype=torch.float64, device=r.device)
        rc = L.lib().amg_vcycle_apply_prec(self.handle, _field(r, shape, torch.float64, "r"), C.c_void_p(z.data_ptr()),
                                           L.PRECISION[precision], _stream())
        L.check(rc, "amg_vcycle_apply_prec")
        return z

    def set_level_weight(self, level: int, factor: float = 1.0):
        """amg_set_level_weight: V-cycle smoothing weight of a coarse level,
        `factor` times the set-up 4 / (3 rho) (1 restores it)."""
        L.check(L.lib().amg_set_level_weight(self.handle, int(level), float(factor), _stream()),
                "amg_set_level_weight")

    def smoothed_levels(self) -> list:
        """Coarse levels with a smoother (1 .. levels - 2)."""
        return [l for l in range(1, self.n_levels) if not self.level(l).is_coarsest]

    def solve(self, b: torch.Tensor, x0: Optional[torch.Tensor] = None, tol: float = 1e-8, maxit: int = 1000,
              check_every: int = 8, out: Optional[torch.Tensor] = None, allow_noconv: bool = False,
              precision: str = "fp64"):
        """PCG to ||r|| <= tol ||b||; precision selects the V-cycle's ("fp64" or "fp32")."""
        shape = self.grid.shape
        x = out if out is not None else torch.empty(shape, dtype=torch.float64, device=b.device)
        if x0 is not None:
            x.copy_(x0)
        prm = L.PcgParams(float(tol), int(maxit), 1 if x0 is not None else 0, int(check_every),
                          L.PRECISION[precision])
        res = L.PcgResult()
        rc = L.lib().pcg_solve(self.handle, _field(b, shape, torch.float64, "b"), _field(x, shape, torch.float64, "x"),
                               C.byref(prm), C.byref(res), _stream())
        ok = (L.EB_OK, L.EB_ENOCONV) if allow_noconv else (L.EB_OK,)
        L.check(rc, "pcg_solve", ok=ok)
        return x, _result_dict(res)

    def solve_batched(self, b: torch.Tensor, **kw):
        """Several right-hand sides in one batched solve (see solve_batched)."""
        return solve_batched(self, b, **kw)


def _result_dict(res):
    return dict(iterations=res.iterations, status=res.status, restarts=res.restarts, levels=res.levels,
                rel_res_true=res.rel_res_true, solve_ms=res.solve_ms)


def solve_batched(H: "Hierarchy", b: torch.Tensor, x0: Optional[torch.Tensor] = None, tol: float = 1e-8,
                  maxit: int = 1000, check_every: int = 8, out: Optional[torch.Tensor] = None,
                  allow_noconv: bool = False, precision: str = "fp64"):
    """pcg_solve_batched: b of shape (nrhs, *grid.shape); returns (x, [info per rhs])."""
    shape = tuple(H.grid.shape)
    if b.dim() != len(shape) + 1:
        raise ValueError("b must have shape (nrhs, *grid.shape)")
    nrhs = b.shape[0]
    bp = _field(b, (nrhs,) + shape, torch.float64, "b")
    x = out if out is not None else torch.empty((nrhs,) + shape, dtype=torch.float64, device=b.device)
    if x0 is not None:
        x.copy_(x0)
    xp = _field(x, (nrhs,) + shape, torch.float64, "x")
    prm = L.PcgParams(float(tol), int(maxit), 1 if x0 is not None else 0, int(check_every), L.PRECISION[precision])
    res = (L.PcgResult * max(nrhs, 1))()
    rc = L.lib().pcg_solve_batched(H.handle, int(nrhs), bp, xp, C.byref(prm), res, _stream())
    ok = (L.EB_OK, L.EB_ENOCONV) if allow_noconv else (L.EB_OK,)
    L.check(rc, "pcg_solve_batched", ok=ok)
    return x, [_result_dict(res[j]) for j in range(nrhs)]


@dataclass
class IslandCanvas:
    """Placement of several 2-D geometries' node grids one above the other in
    one node grid (the canvas, h = 1) for pcg_solve_islands."""
    grid: object                 # canvas grid (workloads.Grid-like: dim, n, x0, h = 1)
    rows: np.ndarray             # int32 [nseg + 1]: first node row of each island, then the total
    shapes: list                 # node-field shape (ny + 1, nx + 1) of each island
    h: np.ndarray                # each island's own grid spacing

    @property
    def nseg(self) -> int:
        return len(self.shapes)

    def pack(self, fields, fill: float = 0.0) -> np.ndarray:
        """Canvas node field from one field per island (numpy), values copied."""
        out = np.full(self.grid.shape, fill, dtype=np.float64)
        for i, (f, sh) in enumerate(zip(fields, self.shapes)):
            f = np.asarray(f, dtype=np.float64).reshape(sh)
            r0 = int(self.rows[i])
            out[r0:r0 + sh[0], :sh[1]] = f
        return out

    def unpack(self, field):
        """Per-island views of a canvas node field (numpy or torch, last two axes)."""
        return [field[..., int(self.rows[i]):int(self.rows[i]) + sh[0], :sh[1]] for i, sh in enumerate(self.shapes)]


ISLAND_ROW_ALIGN = 81   # 3^4: islands stay whole row ranges on up to five levels


def stack_islands(grids, align: int = ISLAND_ROW_ALIGN) -> IslandCanvas:
    """Canvas for 2-D geometries given by their grids (each with its own n and
    h): island i's node rows start at rows[i], a multiple of `align` (rows of
    outside nodes fill the gaps and belong to the island above), so that the
    island hierarchy (Hierarchy(islands=rows)) keeps each island one row range
    on every level it can end on."""
    shapes = [tuple(g.shape) for g in grids]
    if any(len(sh) != 2 for sh in shapes):
        raise ValueError("stack_islands: 2-D grids only")
    width = max(sh[1] for sh in shapes)
    rows = np.zeros(len(shapes) + 1, dtype=np.int32)
    for i, sh in enumerate(shapes):
        end = int(rows[i]) + sh[0]
        rows[i + 1] = end if i + 1 == len(shapes) else -(-end // align) * align
    from types import SimpleNamespace
    n = (width - 1, int(rows[-1]) - 1)
    canvas = SimpleNamespace(dim=2, n=n, x0=(0.0, 0.0), h=1.0, shape=(n[1] + 1, n[0] + 1))
    return IslandCanvas(canvas, rows, shapes, np.array([g.h for g in grids], dtype=np.float64))


def solve_islands(H: "Hierarchy", b: torch.Tensor, rows, x0: Optional[torch.Tensor] = None, tol: float = 1e-8,
                  maxit: int = 1000, check_every: int = 8, allow_noconv: bool = False, precision: str = "fp64"):
    """pcg_solve_islands: b of shape (nrhs, *canvas shape), rows the segments'
    node-row bounds; returns (x, infos) with infos[s][j] for island s, rhs j."""
    shape = tuple(H.grid.shape)
    if b.dim() != len(shape) + 1:
        raise ValueError("b must have shape (nrhs, *grid.shape)")
    nrhs = b.shape[0]
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int32))
    nseg = rows.size - 1
    bp = _field(b, (nrhs,) + shape, torch.float64, "b")
    x = torch.empty((nrhs,) + shape, dtype=torch.float64, device=b.device)
    if x0 is not None:
        x.copy_(x0)
    xp = _field(x, (nrhs,) + shape, torch.float64, "x")
    prm = L.PcgParams(float(tol), int(maxit), 1 if x0 is not None else 0, int(check_every), L.PRECISION[precision])
    res = (L.PcgResult * max(nrhs * nseg, 1))()
    rc = L.lib().pcg_solve_islands(H.handle, int(nrhs), int(nseg), rows.ctypes.data_as(C.POINTER(C.c_int32)), bp, xp,
                                   C.byref(prm), res, _stream())
    ok = (L.EB_OK, L.EB_ENOCONV) if allow_noconv else (L.EB_OK,)
    L.check(rc, "pcg_solve_islands", ok=ok)
    return x, [[_result_dict(res[s * nrhs + j]) for j in range(nrhs)] for s in range(nseg)]


def segment_dots(w: torch.Tensor, x: torch.Tensor, rows) -> np.ndarray:
    """eb_segment_dots: w . x_j over the node rows of every island for every
    field x_j of x (shape (nfields, *canvas shape)); w is one canvas node
    field.  Returns a numpy array [nfields, nseg]."""
    if x.dim() != w.dim() + 1:
        raise ValueError("x must have shape (nfields, *w.shape)")
    shape = tuple(w.shape)
    nf = x.shape[0]
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int32))
    nseg = rows.size - 1
    wp = _field(w, shape, torch.float64, "w")
    xp = _field(x, (nf,) + shape, torch.float64, "x")
    out = np.zeros(nf * nseg, dtype=np.float64)
    rc = L.lib().eb_segment_dots(wp, xp, int(nf), int(np.prod(shape)), int(shape[-1]), int(nseg),
                                 rows.ctypes.data_as(C.POINTER(C.c_int32)),
                                 out.ctypes.data_as(C.POINTER(C.c_double)), _stream())
    L.check(rc, "eb_segment_dots")
    return out.reshape(nf, nseg)


def qoi_study(grid, psis, f, weights, tol: float = 1e-10, precision: str = "fp64", device="cuda"):
    """Quantity of interest of a family of geometries on one 2-D grid (Sec. 3.6):
    Q_k = w . u_k, u_k the solution of -Lap u = f on {psis[k] < 0} with zero
    Dirichlet data.  The geometries are stacked as islands of one canvas and
    solved together (eb_assemble_diag, eb_assemble_rhs, amg_setup,
    pcg_solve_islands); the functional is eb_segment_dots.  Returns (Q, infos)
    with infos[k] the solve result of geometry k and the phase times."""
    import time
    K = len(psis)
    canvas = stack_islands([grid] * K)
    t0 = time.perf_counter()
    psi_c = torch.from_numpy(canvas.pack(psis, fill=1.0)).to(device)
    f_c = torch.from_numpy(canvas.pack([f] * K)).to(device)
    w_c = torch.from_numpy(canvas.pack([weights] * K)).to(device)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    asm = assemble_diag(canvas.grid, psi_c)
    b = assemble_rhs_islands(asm, canvas, f_c)
    H = Hierarchy(canvas.grid, asm.kind, asm.a, 0.0, islands=canvas.rows)
    try:
        X, infos = solve_islands(H, b[None].contiguous(), canvas.rows, tol=tol, precision=precision)
        Q = segment_dots(w_c, X, canvas.rows)[0]
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        levels = H.n_levels
    finally:
        H.free()
    times = {"upload_ms": 1e3 * (t1 - t0), "device_ms": 1e3 * (t2 - t1), "levels": levels,
             "n_unknowns": int(asm.n_unknowns)}
    return Q, [i[0] for i in infos], times


def set_iteration_graphs(enabled: bool = True):
    """Launch steady-state PCG iterations as captured HIP graphs (default) or
    kernel by kernel (process-wide switch; results are identical)."""
    L.check(L.lib().eb_set_iteration_graphs(1 if enabled else 0), "eb_set_iteration_graphs")


def set_batched_launch_shape(plane_width: int = 0, planes_per_block: int = 0):
    """Fix the batched fine kernels' launch shape for batch buffers made from
    now on (0, 0: the autotuner chooses)."""
    L.check(L.lib().pcg_batched_set_launch_shape(int(plane_width), int(planes_per_block)),
            "pcg_batched_set_launch_shape")


def batched_launch_shape(H: "Hierarchy") -> dict:
    """Launch shape in use on H and the autotuner's timed candidates."""
    w, n, nc = C.c_int32(0), C.c_int32(0), C.c_int32(0)
    cw, cn, cm = (C.c_int32 * 8)(), (C.c_int32 * 8)(), (C.c_float * 8)()
    L.check(L.lib().pcg_batched_launch_shape(H.handle, C.byref(w), C.byref(n), C.byref(nc), cw, cn, cm),
            "pcg_batched_launch_shape")
    return {"plane_width": w.value, "planes_per_block": n.value,
            "candidates": [{"plane_width": cw[i], "planes_per_block": cn[i], "ms": cm[i]} for i in range(nc.value)]}


def solve_problem(problem, device="cuda", tol=None, coarse_max=256, precision="fp64"):
    """Full path for one workloads.Problem: assemble, RHS, setup, solve."""
    g = problem.grid
    psi = torch.as_tensor(problem.psi, device=device)
    f = torch.as_tensor(problem.f, device=device)
    asm = assemble_diag(g, psi)
    coords = asm.cut_coordinates()
    u_cut = problem.u_dirichlet(*coords) if problem.u_dirichlet is not None else torch.zeros_like(coords[0])
    b = assemble_rhs(asm, f, torch.as_tensor(u_cut, device=device, dtype=torch.float64))
    H = Hierarchy(g, asm.kind, asm.a, problem.sigma, coarse_max=coarse_max)
    x, info = H.solve(b, tol=problem.tol if tol is None else tol, precision=precision)
    return dict(asm=asm, b=b, H=H, x=x, info=info)


# ------------------------------------------------------- learned smoother
NET_CH = 16


def init_smoother_params(dim: int, seed: int = 0) -> np.ndarray:
    """Initial FP32 parameters: He-normal first two layers, zero last layer, so the
    network starts at the plain smoother (omega_k = omega0).  Packed in the
    library's order W1, b1, W2, b2, W3, b3."""
    rng = np.random.default_rng(seed)
    T = 3 ** dim
    w1 = rng.normal(0.0, np.sqrt(2.0 / (2 * T)), size=(NET_CH, 2, T))
    w2 = rng.normal(0.0, np.sqrt(2.0 / (NET_CH * T)), size=(NET_CH, NET_CH, T))
    parts = [w1.ravel(), np.zeros(NET_CH), w2.ravel(), np.zeros(NET_CH), np.zeros(NET_CH * T), np.zeros(1)]
    out = np.concatenate(parts).astype(np.float32)
    assert out.size == L.lib().eb_smoother_net_size(dim)
    return out


class LearnedSmoother:
    """Per-point fine smoother weights from the library's network, trained on the GPU.

    Every step is a library call: forward pass, error samples, loss and
    dL/domega (adjoint of the V-cycle), backward pass, Adam.  This class holds
    the device buffers and the loop."""

    def __init__(self, H: "Hierarchy", asm: "Assembly", psi: torch.Tensor, params: Optional[np.ndarray] = None,
                 seed: int = 0):
        self.H, self.asm, self.grid = H, asm, asm.grid
        self.psi = psi.contiguous()
        dev = psi.device
        dim = self.grid.dim
        self.P = int(L.lib().eb_smoother_net_size(dim))
        p0 = init_smoother_params(dim, seed) if params is None else np.asarray(params, dtype=np.float32)
        self.params = torch.as_tensor(p0, device=dev).contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        n = int(np.prod(self.grid.shape))
        self.z1 = torch.empty(n * NET_CH, dtype=torch.float32, device=dev)
        self.z2 = torch.empty(n * NET_CH, dtype=torch.float32, device=dev)
        self.o = torch.empty(n, dtype=torch.float32, device=dev)
        self.omega = torch.empty(self.grid.shape, dtype=torch.float64, device=dev)
        g = L.make_grid(self.grid)
        self.scratch = torch.empty(int(L.lib().eb_smoother_scratch_floats(C.byref(g))), dtype=torch.float32,
                                   device=dev)
        self.grads = torch.zeros(self.P, dtype=torch.float32, device=dev)
        self.omega0 = H.level(0).omega
        self.g = {}             # per-level multipliers of the coarse smoothing weights

    def forward(self) -> torch.Tensor:
        g = L.make_grid(self.grid)
        rc = L.lib().eb_smoother_forward(C.byref(g), C.c_void_p(self.asm.kind.data_ptr()),
                                         C.c_void_p(self.asm.a.data_ptr()), C.c_void_p(self.psi.data_ptr()),
                                         C.c_void_p(self.params.data_ptr()), self.omega0,
                                         C.c_void_p(self.z1.data_ptr()), C.c_void_p(self.z2.data_ptr()),
                                         C.c_void_p(self.o.data_ptr()), C.c_void_p(self.omega.data_ptr()), _stream())
        L.check(rc, "eb_smoother_forward")
        return self.omega

    def backward(self, grad_omega: torch.Tensor) -> torch.Tensor:
        g = L.make_grid(self.grid)
        rc = L.lib().eb_smoother_backward(C.byref(g), C.c_void_p(self.asm.kind.data_ptr()),
                                          C.c_void_p(self.asm.a.data_ptr()), C.c_void_p(self.psi.data_ptr()),
                                          C.c_void_p(self.params.data_ptr()), self.omega0,
                                          C.c_void_p(self.z1.data_ptr()), C.c_void_p(self.z2.data_ptr()),
                                          C.c_void_p(self.o.data_ptr()),
                                          _field(grad_omega, self.grid.shape, torch.float64, "grad_omega"),
                                          C.c_void_p(self.scratch.data_ptr()), C.c_void_p(self.grads.data_ptr()),
                                          _stream())
        L.check(rc, "eb_smoother_backward")
        return self.grads

    def apply(self):
        """Evaluate the network and install its weights in the hierarchy's fine smoother."""
        om = self.forward()
        L.check(L.lib().amg_set_fine_weights(self.H.handle, C.c_void_p(om.data_ptr()), _stream()),
                "amg_set_fine_weights")
        return om

    def samples(self, xi: torch.Tensor, sweeps: int) -> torch.Tensor:
        m = xi.shape[0]
        e = torch.empty_like(xi)
        rc = L.lib().amg_smoother_samples(self.H.handle, int(m), int(sweeps),
                                          _field(xi, (m,) + tuple(self.grid.shape), torch.float64, "xi"),
                                          C.c_void_p(e.data_ptr()), _stream())
        L.check(rc, "amg_smoother_samples")
        return e

    def loss_grad(self, e: torch.Tensor):
        m = e.shape[0]
        gom = torch.empty(self.grid.shape, dtype=torch.float64, device=e.device)
        loss = C.c_double(0.0)
        rc = L.lib().amg_smoother_loss_grad(self.H.handle, int(m),
                                            _field(e, (m,) + tuple(self.grid.shape), torch.float64, "e"),
                                            C.byref(loss), C.c_void_p(gom.data_ptr()), _stream())
        L.check(rc, "amg_smoother_loss_grad")
        return loss.value, gom

    def step(self, lr: float):
        self.t += 1
        rc = L.lib().eb_adam_step(C.c_void_p(self.params.data_ptr()), C.c_void_p(self.grads.data_ptr()),
                                  C.c_void_p(self.m.data_ptr()), C.c_void_p(self.v.data_ptr()), self.P, self.t,
                                  float(lr), _stream())
        L.check(rc, "eb_adam_step")

    def train(self, steps: int = 100, samples: int = 4, sweeps: int = 6, lr: float = 3e-3, seed: int = 0):
        """Adam on the loss of error samples left by the current cycle (xi seeded per step)."""
        gen = torch.Generator(device=self.params.device)
        gen.manual_seed(int(seed))
        mask = (self.asm.kind == 2).to(torch.float64)
        history = []
        for it in range(steps):
            self.apply()
            xi = torch.randn((samples,) + tuple(self.grid.shape), dtype=torch.float64, device=self.params.device,
                             generator=gen) * mask
            e = self.samples(xi.contiguous(), sweeps)
            loss, gom = self.loss_grad(e)
            self.backward(gom)
            self.step(lr)
            history.append(loss)
        self.apply()
        return history

    def level_search(self, samples: int = 4, sweeps: int = 4, seed: int = 0, gmax: float = 3.0,
                     evals: int = 10, passes: int = 2) -> dict:
        """Per-level smoothing weights of the coarse levels: g_l times the
        set-up 4 / (3 rho_l), g_l in [1, gmax].  Each level in turn (finest
        coarse level first, `passes` times) takes the g minimising the same
        loss as the network, by golden-section search over `evals` loss
        evaluations, on fixed error samples: `samples` seeded N(0, 1) fields
        (rough errors) and as many left by `sweeps` cycles (smooth errors),
        drawn with the cycle as it stands at the start of each pass.  Leaves
        the weights installed; returns {level: g}."""
        levels = self.H.smoothed_levels()
        gen = torch.Generator(device=self.params.device)
        gen.manual_seed(int(seed))
        mask = (self.asm.kind == 2).to(torch.float64)
        shape = (samples,) + tuple(self.grid.shape)
        for l in levels:
            self.g.setdefault(l, 1.0)
        phi = (math.sqrt(5.0) - 1.0) / 2.0
        for _ in range(passes):
            xi = (torch.randn(shape, dtype=torch.float64, device=self.params.device, generator=gen) * mask)
            xs = (torch.randn(shape, dtype=torch.float64, device=self.params.device, generator=gen) * mask)
            e = torch.cat([self.samples(xi.contiguous(), 0), self.samples(xs.contiguous(), sweeps)]).contiguous()
            for l in levels:
                def loss_at(g):
                    self.H.set_level_weight(l, g)
                    return self.loss_grad(e)[0]
                a, b = 1.0, gmax
                c, d = b - phi * (b - a), a + phi * (b - a)
                fc, fd = loss_at(c), loss_at(d)
                for _ in range(max(evals - 2, 0)):
                    if fc <= fd:
                        b, d, fd = d, c, fc
                        c = b - phi * (b - a)
                        fc = loss_at(c)
                    else:
                        a, c, fc = c, d, fd
                        d = a + phi * (b - a)
                        fd = loss_at(d)
                self.g[l] = c if fc <= fd else d
                self.H.set_level_weight(l, self.g[l])
        return dict(self.g)

    def apply_levels(self, g_by_level: dict):
        """Install per-level multipliers {level: g} on this hierarchy; its levels
        beyond the given ones take the multiplier of the deepest given level."""
        last = 1.0
        for l in self.H.smoothed_levels():
            last = g_by_level.get(l, last)
            self.g[l] = last
            self.H.set_level_weight(l, last)

    def clear_levels(self):
        for l in self.H.smoothed_levels():
            self.H.set_level_weight(l, 1.0)

    def clear(self):
        L.check(L.lib().amg_clear_fine_weights(self.H.handle), "amg_clear_fine_weights")

    def select(self, b: torch.Tensor, tol: float = 1e-8, precision: str = "fp64") -> dict:
        """Keep the learned weights only if they solve b in fewer iterations than the
        plain smoother; otherwise fall back to the plain smoother.  Returns both
        counts and the choice."""
        self.apply()
        self.apply_levels(self.g)
        _, il = self.H.solve(b, tol=tol, precision=precision, allow_noconv=True)
        self.clear()
        self.clear_levels()
        _, ip = self.H.solve(b, tol=tol, precision=precision, allow_noconv=True)
        use = il["status"] == 0 and il["iterations"] < ip["iterations"]
        if use:
            self.apply()
            self.apply_levels(self.g)
        return {"plain_iterations": ip["iterations"], "learned_iterations": il["iterations"],
                "learned_status": il["status"], "use_learned": bool(use)}

    def fit(self, steps: int = 100, samples: int = 4, sweeps: int = 6, lr: float = 3e-3, seed: int = 0):
        """The whole training: per-level weights (level_search), the network
        (train) with them in place, the per-level weights again.  Returns the
        network's loss history."""
        self.level_search(samples=samples, sweeps=4, seed=seed + 101, passes=1)
        hist = self.train(steps=steps, samples=samples, sweeps=sweeps, lr=lr, seed=seed)
        self.level_search(samples=samples, sweeps=4, seed=seed + 202, passes=1)
        return hist
