"""Helpers shared by the GPU parity tests (inputs from the workload generators,
expected values from the oracle only)."""
import numpy as np
import torch

from oracle import amg as OA
from oracle import eb_assembly as E
from oracle import pcg as OP
from paper_2204_06083_amd import solver as S

DEV = "cuda:0"


def to_dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


def oracle_system(prob, sigma=None, mode="line"):
    sig = prob.sigma if sigma is None else sigma
    asm = E.assemble(prob.grid, prob.psi, mode=mode)
    A = E.operator_csr(asm, sig)
    if prob.u_dirichlet is not None:
        u = np.asarray(prob.u_dirichlet(*E.cut_coordinates(asm)), dtype=np.float64) * np.ones(asm.n_cuts)
    else:
        u = np.zeros(asm.n_cuts)
    b = E.rhs(asm, prob.f, u)
    return asm, A, b, u


def gpu_system(prob, u_host=None, mode="line"):
    """GPU assembly + RHS; the Dirichlet data are passed in (same values as the oracle)."""
    asm = S.assemble_diag(prob.grid, to_dev(prob.psi), mode=mode)
    if u_host is None:
        u_host = np.zeros(asm.n_cuts)
    b = S.assemble_rhs(asm, to_dev(prob.f), to_dev(np.asarray(u_host, dtype=np.float64)))
    return asm, b


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
