"""CPU check of the device-staged serving schedule in bench.py: chunks of whole
requests and the release of pairs no chunk needs for `keep` chunks, against a
brute-force walk over the chunks."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _trace(seed, n_req):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(1, 50, n_req)
    starts = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    ids = rng.integers(0, 30, int(starts[-1])).astype(np.uint32)
    lods = rng.integers(0, 4, int(starts[-1])).astype(np.uint8)
    return ids, lods, starts


def test_chunks_and_releases_match_brute_force():
    for seed, n_warm, chunk, keep in ((1, 10, 100, 2), (2, 0, 64, 1), (3, 25, 300, 4), (4, 5, 1, 3)):
        ids, lods, starts = _trace(seed, 60)
        pb, first, rk, rel_b = bench.chunk_schedule(ids, lods, starts, n_warm, chunk, keep)
        req_edges = set(int(v) for v in starts)
        assert pb[0] == 0 and pb[-1] == int(starts[-1]) and all(p in req_edges for p in pb)
        assert all(b > a for a, b in zip(pb, pb[1:]))
        n_chunks = len(pb) - 1
        assert pb[first] == int(starts[n_warm])
        for a, b in zip(pb, pb[1:]):  # over the cap only when one request alone is
            if b - a > chunk:
                assert np.searchsorted(starts, a, "right") == np.searchsorted(starts, b, "left")
        keys = [set((ids[pb[c]:pb[c + 1]].astype(np.int64) * 8 + lods[pb[c]:pb[c + 1]]).tolist())
                for c in range(n_chunks)]
        for r in range(n_chunks):
            got = sorted(rk[rel_b[r]:rel_b[r + 1]].tolist())
            want = set()
            c = r - keep
            if c >= 0:
                later = set().union(*keys[c + 1:r + 1])
                want = keys[c] - later
            assert got == sorted(want), (seed, r)
