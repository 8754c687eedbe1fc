"""Host logic of the served decode: the request / provision / assign scheduler
(serve_core.h) driven by a simulated backend on the CPU (tests/serve_sim.cpp).

The simulation records which (brick, LOD) pair was decoded into every cache
range and checks, for every completed request, that each of its pairs is
still in the slot it was decoded into (nothing pinned was evicted or
overwritten), that slots stay inside the cache and that admission follows
arrival order."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from synth import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "_serve_sim.so")


@pytest.fixture(scope="module")
def sim():
    src = os.path.join(HERE, "serve_sim.cpp")
    hdr = os.path.join(HERE, "..", "paper_2609_36898_amd", "csrc", "serve_core.h")
    if not os.path.exists(SO) or os.path.getmtime(SO) < max(os.path.getmtime(src), os.path.getmtime(hdr)):
        subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread", src, "-o", SO + ".tmp"],
                       check=True)
        os.replace(SO + ".tmp", SO)
    lib = ctypes.CDLL(SO)
    P = ctypes.c_void_p
    lib.sim_run.argtypes = [P, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32, ctypes.c_int,
                            ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_uint32, P, ctypes.c_double,
                            P, P, P, P, P, P, ctypes.c_char_p, ctypes.c_int]
    return lib


STATS = ["requests_done", "pairs_requested", "hits", "decoded", "evictions", "resets", "batches",
         "decoded_elements", "requested_elements", "top", "pinned", "max_batch_seen", "joined", "splits"]


def run(lib, l2, cache, ids, lods, starts, arrival, streams=2, max_batch=64, keep_pinned=0, delay=3, dt=1e-3,
        shards=1, threaded=0, with_pairs=False):
    n_req = len(starts) - 1
    l2 = np.ascontiguousarray(l2, dtype=np.uint8)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    lods = np.ascontiguousarray(lods, dtype=np.uint8)
    starts = np.ascontiguousarray(starts, dtype=np.uint64)
    arrival = np.ascontiguousarray(arrival, dtype=np.float64)
    t_adm = np.zeros(n_req)
    t_done = np.zeros(n_req)
    status = np.zeros(n_req, dtype=np.int32)
    ndec = np.zeros(n_req, dtype=np.uint32)
    npairs = np.zeros(n_req, dtype=np.uint32)
    stats = np.zeros(14, dtype=np.uint64)
    err = ctypes.create_string_buffer(512)
    rc = lib.sim_run(l2.ctypes.data, len(l2), cache, streams, max_batch, keep_pinned, delay, shards, threaded,
                     ids.ctypes.data, lods.ctypes.data, starts.ctypes.data, n_req, arrival.ctypes.data, dt,
                     t_adm.ctypes.data, t_done.ctypes.data, status.ctypes.data, ndec.ctypes.data, npairs.ctypes.data,
                     stats.ctypes.data, err, 512)
    assert rc == 0, err.value.decode()
    out = (t_adm, t_done, status, ndec, dict(zip(STATS, (int(x) for x in stats))))
    return out + (npairs,) if with_pairs else out


def _frustum_trace(n, grid, rate, seed):
    return workloads.frustum_requests(n, grid, rate, seed=seed, n_max=512)


def test_frustum_stream_every_request_served_from_its_own_slots(sim):
    grid = (16, 16, 16)
    ids, lods, starts, arr = _frustum_trace(300, grid, 500.0, seed=1)
    l2 = np.full(16 ** 3, 5, np.uint8)
    elems = (np.int64(1) << (3 * (5 - lods.astype(np.int64))))
    per_req = np.add.reduceat(elems, starts[:-1].astype(np.int64))
    cache = int(1.5 * per_req.max())  # the largest request fits, the stream does not: heavy eviction
    assert cache < per_req.sum() / 4
    t_adm, t_done, st, ndec, s = run(sim, l2, cache, ids, lods, starts, arr)
    assert (st == 0).all()
    assert (t_done >= arr - 1e-12).all() and (t_adm >= arr - 1e-12).all() and (t_done >= t_adm).all()
    assert s["requests_done"] == 300
    assert s["hits"] + s["joined"] + s["decoded"] == s["pairs_requested"]
    assert s["evictions"] > 0 and s["top"] <= cache and s["pinned"] == 0
    assert int(ndec.sum()) == s["decoded"]


def test_continuous_batching_overlaps_requests(sim):
    grid = (16, 16, 16)
    ids, lods, starts, arr = _frustum_trace(200, grid, 5000.0, seed=2)  # arrivals faster than batches finish
    l2 = np.full(16 ** 3, 5, np.uint8)
    t_adm, t_done, st, _, s = run(sim, l2, 1 << 26, ids, lods, starts, arr, streams=3, max_batch=256, delay=20)
    assert (st == 0).all()
    # requests admitted while earlier ones were still pending
    overlap = sum(1 for r in range(1, 200) if t_adm[r] < t_done[r - 1])
    assert overlap > 50
    assert s["batches"] < s["decoded"]  # tasks of several requests shared batches
    assert s["max_batch_seen"] <= 256


def test_keep_pinned_and_mixed_brick_sides(sim):
    rng = np.random.default_rng(3)
    l2 = rng.choice(np.array([5, 6], np.uint8), size=512)
    reqs = []
    for r in range(120):
        n = int(rng.integers(1, 40))
        b = rng.choice(512, size=n, replace=False)
        lod = np.array([rng.integers(0, l2[x] + 1) for x in b], np.uint8)
        reqs.append((b, lod))
    ids = np.concatenate([r[0] for r in reqs])
    lods = np.concatenate([r[1] for r in reqs])
    starts = np.concatenate([[0], np.cumsum([len(r[0]) for r in reqs])])
    arr = np.arange(120) * 1e-3
    for keep in (0, 1):
        _, _, st, _, s = run(sim, l2, 40 * 64 ** 3, ids, lods, starts, arr, keep_pinned=keep, delay=2)
        assert (st == 0).all() and s["requests_done"] == 120


def test_request_larger_than_cache_is_rejected_and_others_proceed(sim):
    l2 = np.full(64, 5, np.uint8)
    ids = np.array([0, 1, 2, 3, 4, 5, 6], np.uint32)
    lods = np.zeros(7, np.uint8)
    starts = np.array([0, 1, 6, 7], np.uint64)  # requests of 1, 5 and 1 full bricks
    arr = np.array([0.0, 0.001, 0.002])
    _, _, st, _, s = run(sim, l2, 4 * 32 ** 3, ids, lods, starts, arr)
    assert list(st) == [0, -1, 0]
    assert s["resets"] >= 1


def test_hits_do_not_decode_again(sim):
    l2 = np.full(8, 5, np.uint8)
    ids = np.array([0, 1, 0, 1, 1, 0], np.uint32)
    lods = np.array([0, 1, 0, 1, 1, 0], np.uint8)
    starts = np.array([0, 2, 4, 6], np.uint64)
    arr = np.array([0.0, 0.5, 1.0])
    _, _, st, ndec, s = run(sim, l2, 1 << 20, ids, lods, starts, arr)
    assert (st == 0).all()
    assert list(ndec) == [2, 0, 0] and s["decoded"] == 2 and s["hits"] == 4


def test_smaller_class_splits_a_larger_slot_instead_of_resetting(sim):
    # two full bricks fill the cache; later requests for smaller LODs take
    # slots split out of the least recently used full brick
    l2 = np.full(8, 5, np.uint8)
    ids = np.array([0, 1, 2, 3, 4, 1], np.uint32)
    lods = np.array([0, 0, 1, 2, 1, 0], np.uint8)
    starts = np.array([0, 2, 3, 4, 5, 6], np.uint64)
    arr = np.array([0.0, 1.0, 2.0, 3.0, 4.0])
    _, _, st, ndec, s = run(sim, l2, 2 * 32 ** 3, ids, lods, starts, arr, delay=2)
    assert (st == 0).all()
    assert s["resets"] == 0 and s["splits"] >= 1
    # brick 0 (least recently used) was split; brick 1 stayed resident
    assert list(ndec) == [2, 1, 1, 1, 0]


def test_random_traces_keep_every_invariant(sim):
    # small caches, brick sides 8..64, duplicate pairs, one to three streams,
    # tiny batches, keep_pinned on and off: the simulation's own checks
    # (no completed pair overwritten, slots inside the cache, arrival-order
    # admission) must hold and every request must end served or rejected
    rng = np.random.default_rng(0)
    for trial in range(24):
        nb = int(rng.integers(8, 200))
        l2 = rng.choice(np.array([3, 4, 5, 6], np.uint8), size=nb)
        reqs = []
        for _ in range(int(rng.integers(20, 150))):
            b = rng.integers(0, nb, size=int(rng.integers(1, 30))).astype(np.uint32)
            reqs.append((b, np.array([rng.integers(0, l2[x] + 1) for x in b], np.uint8)))
        ids = np.concatenate([a for a, _ in reqs])
        lods = np.concatenate([b for _, b in reqs])
        starts = np.concatenate([[0], np.cumsum([len(a) for a, _ in reqs])]).astype(np.uint64)
        arr = np.sort(rng.uniform(0, 0.05, size=len(reqs)))
        cache = int(rng.integers(1, 6)) * 64 ** 3
        _, _, st, ndec, s = run(sim, l2, cache, ids, lods, starts, arr, streams=int(rng.integers(1, 4)),
                                max_batch=int(rng.integers(1, 64)), keep_pinned=trial % 2,
                                delay=int(rng.integers(1, 5)))
        assert set(np.unique(st)) <= {0, -1}
        assert s["requests_done"] == int((st == 0).sum())
        assert s["hits"] + s["joined"] + s["decoded"] == s["pairs_requested"]
        assert s["pinned"] == 0 and s["top"] <= cache


def test_eviction_follows_least_recent_use(sim):
    # three full bricks fill the cache; a hit on brick 0 makes brick 1 the least
    # recently used, so brick 3 evicts brick 1 and brick 0 stays resident
    l2 = np.full(8, 5, np.uint8)
    ids = np.array([0, 1, 2, 0, 3, 0, 1], np.uint32)
    lods = np.zeros(7, np.uint8)
    starts = np.array([0, 3, 4, 5, 6, 7], np.uint64)
    arr = np.array([0.0, 1.0, 2.0, 3.0, 4.0])
    _, _, st, ndec, s = run(sim, l2, 3 * 32 ** 3, ids, lods, starts, arr, delay=2)
    assert (st == 0).all()
    assert list(ndec) == [3, 0, 1, 0, 1]
    assert s["evictions"] == 2 and s["resets"] == 0


def _distinct_pairs(ids, lods, starts):
    return np.array([len(set(zip(ids[a:b].tolist(), lods[a:b].tolist())))
                     for a, b in zip(starts[:-1].astype(np.int64), starts[1:].astype(np.int64))])


def test_sharded_cache_keeps_every_invariant(sim):
    # brick shards stepped in turn: every pair of a completed request sits in
    # its shard's range where it was decoded, admission times stay in arrival
    # order, and a request's pair counts are the sums over its parts
    grid = (16, 16, 16)
    ids, lods, starts, arr = _frustum_trace(300, grid, 500.0, seed=4)
    l2 = np.full(16 ** 3, 5, np.uint8)
    per_req = np.add.reduceat(np.int64(1) << (3 * (5 - lods.astype(np.int64))), starts[:-1].astype(np.int64))
    for shards in (2, 3, 8):
        cache = int(3 * per_req.max())
        t_adm, t_done, st, ndec, s, npairs = run(sim, l2, cache, ids, lods, starts, arr, shards=shards,
                                                 with_pairs=True)
        assert (st == 0).all() and s["requests_done"] == 300
        assert (t_done >= t_adm).all() and (t_adm >= arr - 1e-12).all()
        assert np.array_equal(npairs, _distinct_pairs(ids, lods, starts))
        assert s["hits"] + s["joined"] + s["decoded"] == s["pairs_requested"] == int(npairs.sum())
        assert int(ndec.sum()) == s["decoded"] and s["evictions"] > 0 and s["pinned"] == 0
        assert s["top"] <= cache


def test_sharded_threads_serve_a_trace(sim):
    # one host thread per shard on the real clock: every request completes,
    # each record is its own request's, and the counts add up
    grid = (16, 16, 16)
    ids, lods, starts, arr = _frustum_trace(400, grid, 20000.0, seed=6)
    l2 = np.full(16 ** 3, 5, np.uint8)
    want = _distinct_pairs(ids, lods, starts)
    # (with keep_pinned nothing is released during the run: the cache holds the whole trace)
    for shards, keep, cache in ((1, 0, 1 << 27), (4, 0, 1 << 27), (8, 1, 1 << 31)):
        t_adm, t_done, st, ndec, s, npairs = run(sim, l2, cache, ids, lods, starts, arr * 0.02, streams=2,
                                                 max_batch=128, keep_pinned=keep, delay=2, shards=shards,
                                                 threaded=1, with_pairs=True)
        assert (st == 0).all() and s["requests_done"] == 400
        assert np.array_equal(npairs, want)
        assert (t_done >= t_adm).all() and (t_adm >= arr * 0.02 - 1e-9).all()
        assert s["hits"] + s["joined"] + s["decoded"] == s["pairs_requested"] == int(want.sum())
        assert int(ndec.sum()) == s["decoded"] and s["pinned"] == 0


def test_sharded_rejection_of_an_oversized_part(sim):
    # a part larger than its shard's range rejects the whole request; the
    # others proceed
    l2 = np.full(64, 5, np.uint8)
    ids = np.array([0, 0, 2, 4, 6, 8, 1], np.uint32)  # request 1: five bricks of shard 0
    lods = np.zeros(7, np.uint8)
    starts = np.array([0, 1, 6, 7], np.uint64)
    arr = np.array([0.0, 0.001, 0.002])
    _, _, st, _, s = run(sim, l2, 2 * 4 * 32 ** 3, ids, lods, starts, arr, shards=2)
    assert list(st) == [0, -1, 0]
    assert s["requests_done"] == 2
