"""Oracle: preconditioned conjugate gradients and direct references (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Algorithm 2 step 4 solves the SPD system with conjugate gradients and an AMG
preconditioner; the paper stops on the relative residual (Sec. 3 preamble).
Textbook PCG is written out here with the stopping rule
||r_k||_2 <= tol * ||b||_2 on the recursively updated residual, followed by a
recomputation of the true residual b - A x; if that exceeds the tolerance,
PCG restarts once from the current iterate.

Iteration order (one iteration = one product with A):
    q = A p;  alpha = rho / (p, q);  x += alpha p;  r -= alpha q
    stop if ||r|| <= tol ||b||
    z = M r;  rho' = (r, z);  beta = rho' / rho;  p = z + beta p

Parity: pinned by tests/test_oracle_pcg.py (M = I against an independent CG
library routine; one-level hierarchy converges in one iteration; dense
solves on grids up to 16^2; sparse direct solves at larger sizes).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse.linalg as spla

from . import amg


@dataclass
class PCGResult:
    x: np.ndarray
    iterations: int
    rel_res_recursive: float
    rel_res_true: float
    converged: bool
    restarts: int
    history: list


def pcg(A, b, precond=None, tol=1e-8, maxit=1000, x0=None, restart_on_drift=True):
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    M = precond if precond is not None else (lambda r: r.copy())
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    if n == 0 or bnorm == 0.0:
        return PCGResult(np.zeros(n), 0, 0.0, 0.0, True, 0, [])
    total_its = 0
    restarts = 0
    history = []
    while True:
        r = b - A @ x if np.any(x) else b.copy()
        rnorm = float(np.linalg.norm(r))
        history.append(rnorm / bnorm)
        converged = rnorm <= tol * bnorm
        if not converged:
            z = M(r)
            rho = float(r @ z)
            p = z.copy()
            while total_its < maxit:
                q = A @ p
                alpha = rho / float(p @ q)
                x = x + alpha * p
                r = r - alpha * q
                total_its += 1
                rnorm = float(np.linalg.norm(r))
                history.append(rnorm / bnorm)
                if rnorm <= tol * bnorm:
                    converged = True
                    break
                z = M(r)
                rho_new = float(r @ z)
                beta = rho_new / rho
                rho = rho_new
                p = z + beta * p
        true_rel = float(np.linalg.norm(b - A @ x)) / bnorm
        if converged and true_rel > tol and restart_on_drift and restarts == 0 \
                and total_its < maxit:
            restarts += 1
            continue
        return PCGResult(x, total_its, rnorm / bnorm, true_rel, converged,
                         restarts, history)


def amg_pcg(A, coords, b, tol=1e-8, maxit=1000, x0=None, **amg_params):
    H = amg.build_hierarchy(A, coords, **amg_params)
    res = pcg(A, b, precond=lambda r: amg.vcycle(H, r), tol=tol, maxit=maxit, x0=x0)
    return res, H


def direct_solve(A, b):
    """Reference solution: dense solve for small systems, sparse LU otherwise."""
    n = A.shape[0]
    if n <= 400:
        return np.linalg.solve(A.toarray(), b)
    return spla.spsolve(A.tocsc(), b)
