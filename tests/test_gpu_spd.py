"""The a-priori SPD test (eb_check_spd, Sec. 2.4) on the GPU against the
oracle's segment_check: integer counts equal on real assemblies and on
records with altered c; the full-size star by properties."""
import numpy as np
import pytest
import torch

from oracle import eb_assembly as E
from oracle import spd
from paper_2204_06083_amd import _lib as L
from paper_2204_06083_amd import solver as S
from paper_2204_06083_amd import workloads as W

from gpu_common import to_dev

pytestmark = pytest.mark.gpu


def _runs_by_starts(kind):
    comp = np.asarray(kind) == 2
    total = 0
    for ax in range(comp.ndim):
        prev = np.zeros_like(comp)
        dst = [slice(None)] * comp.ndim
        src = [slice(None)] * comp.ndim
        dst[ax] = slice(1, None)
        src[ax] = slice(None, -1)
        prev[tuple(dst)] = comp[tuple(src)]
        total += int(np.sum(comp & ~prev))
    return total


def _oracle_counts(asm_g, c=None):
    rec = asm_g.cuts_host()
    kind = asm_g.kind.cpu().numpy()
    cc = rec["c"] if c is None else c
    return spd.segment_check(kind, rec["node"], rec["dir"], cc)


CASES = {
    "disk128": lambda: W.disk_poisson(128),
    "star300": lambda: W.star_poisson(300),
    "ell40": lambda: W.ellipsoid_poisson(40),
}


@pytest.mark.parametrize("name", list(CASES))
def test_check_spd_against_oracle(name):
    p = CASES[name]()
    print(f"[gpu] check_spd {name}", flush=True)
    asm_g = S.assemble_diag(p.grid, to_dev(p.psi))
    segs, fail = S.check_spd(asm_g)
    assert (segs, fail) == _oracle_counts(asm_g)
    assert fail == 0 and segs == _runs_by_starts(asm_g.kind.cpu().numpy())


@pytest.mark.parametrize("scale", [0.5, -0.3, -0.9])
def test_check_spd_altered_records(scale):
    p = W.disk_poisson(96)
    asm_g = S.assemble_diag(p.grid, to_dev(p.psi))
    cuts = asm_g.cuts.clone()
    rec = cuts[: asm_g.n_cuts * 56].view(torch.float64).view(asm_g.n_cuts, 7)
    rec[:, 3] *= scale                       # c of every record
    c_host = rec[:, 3].cpu().numpy()
    segs, fail = S.check_spd(asm_g, cuts)
    assert (segs, fail) == _oracle_counts(asm_g, c_host)
    if scale > 0:
        assert fail == 0
    if scale == -0.9:
        assert fail > 0


def test_check_spd_edge_cases():
    g = W.unit_box_grid(2, 24)
    asm_g = S.assemble_diag(g, to_dev(np.ones(g.shape)))
    assert S.check_spd(asm_g) == (0, 0)
    # a missing record is refused
    p = W.disk_poisson(64)
    asm_g = S.assemble_diag(p.grid, to_dev(p.psi))
    short = S.Assembly(asm_g.grid, asm_g.kind, asm_g.a, asm_g.cuts, asm_g.n_unknowns, asm_g.n_cuts - 1)
    with pytest.raises(L.EbError) as ei:
        S.check_spd(short)
    assert ei.value.code == L.EB_EINVAL


def test_check_spd_full_size_star():
    p = W.star_poisson(2048)
    print("[gpu] check_spd star2048", flush=True)
    asm_g = S.assemble_diag(p.grid, to_dev(p.psi))
    segs, fail = S.check_spd(asm_g)
    assert fail == 0 and segs == _runs_by_starts(asm_g.kind.cpu().numpy())


def test_check_spd_on_staircases():
    """Staircase stripes (321 k grid-line segments, many with long walks and
    both ends cut): counts equal to the oracle's, unchanged and with the c of
    every third record made negative."""
    g = W.unit_box_grid(2, 2048)
    print("[gpu] check_spd staircases 2049^2", flush=True)
    asm_g = S.assemble_diag(g, to_dev(W.psi_staircases(g)))
    segs, fail = S.check_spd(asm_g)
    assert (segs, fail) == _oracle_counts(asm_g)
    assert fail == 0 and segs == _runs_by_starts(asm_g.kind.cpu().numpy())
    cuts = asm_g.cuts.clone()
    rec = cuts[: asm_g.n_cuts * 56].view(torch.float64).view(asm_g.n_cuts, 7)
    rec[::3, 3] *= -0.7
    c_host = rec[:, 3].cpu().numpy()
    segs2, fail2 = S.check_spd(asm_g, cuts)
    assert (segs2, fail2) == _oracle_counts(asm_g, c_host)
    assert segs2 == segs and fail2 > 0
