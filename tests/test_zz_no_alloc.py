"""eb_segment_dots_noalloc (the allocation-free variant of eb_segment_dots)
against eb_segment_dots through the C ABI: bit-for-bit equal results on two
calls in a row (the second with a smaller input, so the fixed scratch still
holds the first call's contents), and the size limit.  Inputs are seeded
random node fields and ragged island segments."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2204_06083_amd import _lib as L

DEV = "cuda:0"


def _call(name, w, x, nf, row_len, rows):
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    nseg = rows.size - 1
    out = np.full(nf * nseg, np.nan)
    stream = torch.cuda.current_stream().cuda_stream
    rc = getattr(L.lib(), name)(C.c_void_p(w.data_ptr()), C.c_void_p(x.data_ptr()), nf, w.numel(), row_len, nseg,
                                rows.ctypes.data_as(C.POINTER(C.c_int32)),
                                out.ctypes.data_as(C.POINTER(C.c_double)), C.c_void_p(stream))
    return rc, out.reshape(nf, nseg)


def _case(seed, nf, ny, nx, rows):
    g = np.random.default_rng(seed)
    w = torch.as_tensor(g.standard_normal((ny, nx)), device=DEV)
    x = torch.as_tensor(g.standard_normal((nf, ny, nx)), device=DEV)
    return w, x, np.asarray(rows, dtype=np.int32)


@pytest.mark.gpu
def test_noalloc_matches_allocating_entry_point_twice():
    # first call: 3 fields, 5 ragged segments (one empty, one longer than a
    # 2048-node chunk); second call: 2 fields, 3 shorter segments
    cases = [(_case(11, 3, 300, 257, [0, 17, 17, 140, 299, 300]), 257),
             (_case(12, 2, 90, 64, [0, 5, 40, 90]), 64)]
    for (w, x, rows), row_len in cases:
        nf = x.shape[0]
        print(f"[gpu] segment dots noalloc: {nf} fields, {rows.size - 1} segments, {w.shape}", flush=True)
        rc_a, ref = _call("eb_segment_dots", w, x, nf, row_len, rows)
        rc_b, got = _call("eb_segment_dots_noalloc", w, x, nf, row_len, rows)
        assert rc_a == 0 and rc_b == 0, (rc_a, rc_b, L.lib().eb_last_error())
        assert np.array_equal(got, ref), np.abs(got - ref).max()
        # and a plain host sum (the same sums in another order)
        wh, xh = w.cpu().numpy().ravel(), x.cpu().numpy().reshape(nf, -1)
        for j in range(nf):
            for s in range(rows.size - 1):
                lo, hi = rows[s] * row_len, rows[s + 1] * row_len
                host = float(np.dot(wh[lo:hi], xh[j, lo:hi]))
                assert abs(got[j, s] - host) <= 1e-12 * (1.0 + np.abs(wh[lo:hi] * xh[j, lo:hi]).sum())


@pytest.mark.gpu
def test_noalloc_rejects_inputs_beyond_its_scratch():
    # 1000 fields x 1000 one-node segments need 16 kB + 16 MB of scratch (> 8 MiB)
    nf, nseg = 1000, 1000
    w = torch.ones(nseg, dtype=torch.float64, device=DEV)
    x = torch.ones((nf, nseg), dtype=torch.float64, device=DEV)
    rows = np.arange(nseg + 1, dtype=np.int32)
    print("[gpu] segment dots noalloc: oversized request", flush=True)
    rc, _ = _call("eb_segment_dots_noalloc", w, x, nf, 1, rows)
    assert rc == L.EB_ENOSPC
    assert b"scratch" in L.lib().eb_last_error()
    # the allocating entry point takes the same input
    rc, out = _call("eb_segment_dots", w, x, nf, 1, rows)
    assert rc == 0 and np.all(out == 1.0)
