"""Oracle: quantities of interest over a family of geometries (CPU).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. 3.6 computes a quantity of interest (QOI) from the solution of a Poisson
problem for each value of a geometry parameter and differentiates it in the
parameter by central differences.  Written out plainly here: for every level
set of the family, assemble the line-by-line system on the common grid
(eb_assembly), solve it directly (sparse LU), put the solution back on the
node field (zero off the unknowns) and evaluate

* the value at one node (the paper's u(0, 0)), or
* a linear functional w . u with node weights w (the paper's integral of u
  over a rectangle, by the composite trapezoid rule; the weights are the
  caller's).

The derivative in the parameter is the central difference of neighbouring
QOI values of an equally spaced parameter sweep.

Pins (tests/test_oracle_qoi.py): the closed-form QOI of the fixed-area
ellipse (u = C (x^2/a^2 + y^2 a^2 - 1) solves the problem exactly) with its
second-order convergence and the central-difference derivative against the
closed-form derivative; the a <-> 1/a and theta <-> -theta, theta + pi
symmetries, which the discrete problems inherit from the grid; the trapezoid
weights against exact integrals of bilinear fields.
"""
from __future__ import annotations

import numpy as np

from oracle import eb_assembly as E
from oracle import pcg as OP


def solve_field(grid, psi, f):
    """Solution node field of -Lap u = f on {psi < 0}, u = 0 on the boundary."""
    asm = E.assemble(grid, psi)
    A = E.operator_csr(asm)
    b = E.rhs(asm, f, np.zeros(len(asm.cuts["c"])))
    x = OP.direct_solve(A, b)
    return E.embed(asm, x).reshape(psi.shape)


def node_value(grid, u, point):
    """u at the node with the given coordinates (which must be a node)."""
    idx = []
    for axis in reversed(range(grid.dim)):
        t = (point[axis] - grid.x0[axis]) / grid.h
        i = int(round(t))
        if abs(t - i) > 1e-9:
            raise ValueError("point is not a node")
        idx.append(i)
    return float(u[tuple(idx)])


def weighted_sum(w, u):
    """w . u, in plain order."""
    return float(np.sum(np.asarray(w, dtype=np.float64) * u))


def sweep(grid, psis, f, qoi):
    """QOI of every geometry of a family: qoi(u) for u = solve_field(psi)."""
    return np.array([qoi(solve_field(grid, psi, f)) for psi in psis])


def central_differences(values, step):
    """(Q_{k+1} - Q_{k-1}) / (2 step) at the interior parameters."""
    v = np.asarray(values, dtype=np.float64)
    return (v[2:] - v[:-2]) / (2.0 * step)
