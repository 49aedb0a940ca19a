"""Oracle: time steppers on the line-by-line operator (CPU).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper uses its spatial discretisation inside two time integrators.  With
A = -L_h the SPD operator of eb_assembly (homogeneous or inhomogeneous
Dirichlet data entering through the right-hand side), written out plainly:

* Wave equation u_tt = Lap u, theta-scheme (Sec. 3.5):
      (I + theta dt^2 A) u^{n+1} = 2 u^n - u^{n-1}
                                   - dt^2 A ((1 - 2 theta) u^n + theta u^{n-1}).
  Reading: the printed scheme lacks the Laplacian on its (1 - 2 theta) term;
  with it the scheme is the standard theta-scheme, theta = 0 is the explicit
  leap-frog scheme the text names, theta = 1/12 the fourth-order one.
  Homogeneous Dirichlet data, as in the paper's example.  The implicit steps
  are solved directly (sparse LU).
* Heat equation u_t = Lap u + f, Crank-Nicolson (Sec. 3.4), multiplied by 2:
      (A + (2/dt) I) u^{n+1} = ((2/dt) I - A) u^n + b^n + b^{n+1},
  b^n = eb_assembly.rhs(f(t_n), u_D(t_n)) the source plus boundary terms at
  t_n.  Reading: written for beta = 1 (the paper's example has a variable
  beta, which is not treated here).

Pins (tests/test_oracle_steppers.py): closed forms on an eigenvector of A
(the theta-scheme's mode recurrence a^n = cos(n phi), the Crank-Nicolson
amplification factor), the exactly conserved discrete energy of the
theta-scheme, the Bessel-zero constants the paper prints, the leap-frog
max-errors of the paper's Table 1 and the second-order decay of the
Crank-Nicolson error on a manufactured solution.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import eb_assembly as E


def theta_step_matrix(A, dt, theta):
    """I + theta dt^2 A (CSC, for the direct solves)."""
    n = A.shape[0]
    return (sp.identity(n, format="csc") + (theta * dt * dt) * A.tocsc()).tocsc()


def wave_theta(A, u0, u1, dt, theta, nsteps, callback=None):
    """u^0 = u0, u^1 = u1 (unknown vectors); returns (u^{nsteps}, u^{nsteps-1}).

    callback(n, u_n, u_{n-1}) is called after each new u^n (n = 2..nsteps).
    """
    um, u = np.asarray(u0, dtype=np.float64).copy(), np.asarray(u1, dtype=np.float64).copy()
    dt2 = dt * dt
    lu = spla.splu(theta_step_matrix(A, dt, theta)) if theta != 0.0 else None
    for n in range(2, nsteps + 1):
        v = (1.0 - 2.0 * theta) * u + theta * um
        w = 2.0 * u - um - dt2 * (A @ v)
        un = w if lu is None else lu.solve(w)
        um, u = u, un
        if callback is not None:
            callback(n, u, um)
    return u, um


def wave_energy(A, u_new, u_old, dt, theta):
    """E = d^T (I + theta dt^2 A) d / dt^2 + u_new^T A u_old, d = u_new - u_old.

    Constant along theta-scheme trajectories: subtracting consecutive values
    leaves (d+ - d-)^T (I + theta dt^2 A)(d+ + d-)/dt^2
    + u^T A (u^{n+1} - u^{n-1}), zero by the scheme and the symmetry of A.
    """
    d = u_new - u_old
    return float(d @ d + theta * dt * dt * (d @ (A @ d))) / (dt * dt) + float(u_new @ (A @ u_old))


def heat_cn(asm, u0, dt, nsteps, b_of_step):
    """Crank-Nicolson steps; b_of_step(n) = right-hand side vector at t_n."""
    A = E.operator_csr(asm)
    n = A.shape[0]
    s2 = 2.0 / dt
    M = (A + s2 * sp.identity(n, format="csr")).tocsc()
    lu = spla.splu(M)
    u = np.asarray(u0, dtype=np.float64).copy()
    b_prev = b_of_step(0)
    for k in range(1, nsteps + 1):
        b_next = b_of_step(k)
        rhs = s2 * u - A @ u + b_prev + b_next
        u = lu.solve(rhs)
        b_prev = b_next
    return u


def max_error(u, exact):
    return float(np.max(np.abs(u - exact)))
