"""gq_points_near_noalloc (the proximity query with its device buffers in the library's
fixed scratch) against gq_points_near (which allocates its own), through the C ABI: two
calls in a row, the second smaller, both bit-equal to the allocating entry point; and the
documented error for a query larger than the scratch."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _lib():
    import torch

    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_1805_06106_amd import _capi as C

    C.lib()
    return C


def _case(rng, n_q, n_p, scale):
    pts = rng.uniform(-1.0, 1.0, (n_p, 3))
    q = rng.uniform(-1.1, 1.1, (n_q, 3))
    r = rng.uniform(0.0, scale, n_q)
    # a few radii exactly at a point's distance (on the boundary: hit unless strict)
    k = min(n_q, n_p, 16)
    d = q[:k] - pts[:k]
    r[:k] = np.sqrt((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2])
    return q, r, pts


def test_noalloc_matches_allocating_entry_point():
    C = _lib()
    rng = np.random.default_rng(77)
    for n_q, n_p, scale in ((60_000, 200_000, 0.02), (3_000, 10_000, 0.05)):
        q, r, pts = _case(rng, n_q, n_p, scale)
        for strict in (False, True):
            print(f"[gpu] points_near_noalloc n_q={n_q} n_p={n_p} strict={strict}", flush=True)
            want = C.gq_points_near(q, r, pts, strict=strict)
            got = C.gq_points_near(q, r, pts, strict=strict, noalloc=True)
            assert got.dtype == want.dtype and np.array_equal(got, want)
            assert 0 < int(want.sum()) < n_q  # both outcomes occur


def test_noalloc_rejects_queries_beyond_the_scratch():
    C = _lib()
    rng = np.random.default_rng(78)
    n = 1_000_000  # 24 MB of points plus 33 MB of query buffers: above 32 MiB
    pts = np.ascontiguousarray(rng.uniform(-1.0, 1.0, (n, 3)))
    q = np.ascontiguousarray(rng.uniform(-1.0, 1.0, (n, 3)))
    radius = np.full(n, 0.01)
    hit = np.full(n, 7, dtype=np.uint8)
    # every array passed by address stays referenced until the call returns
    st = C.lib().gq_points_near_noalloc(n, C._ptr(q), C._ptr(radius), 0, n, C._ptr(pts),
                                        C._ptr(hit), None)
    assert st == C.GQ_EINVAL
    assert "scratch" in C.gq_last_error()
    assert np.all(hit == 7)  # outputs untouched
