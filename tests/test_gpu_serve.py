"""Served decode on the GPU: a stream of frustum requests through the server
(cache, admission, continuous batching on two streams), with the cache whole
or split into brick shards.  Every completed request's cache slots must equal
(a) the same pairs decoded alone with the plain one-launch-per-brick form and
(b) the CPU oracle -- the result of a request is the same alone and in the
mix, bit for bit."""
import sys

import numpy as np
import pytest

import oracle
import synth
from synth import workloads

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_36898_amd
    return paper_2609_36898_amd


def _alone(P, dv, ids, lods):
    import torch
    out, st, offs = dv.decode(ids, lods, mode=P.MODE_PLAIN)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    return out.cpu().numpy().view(np.uint32), offs


def _cache_for(ids, lods, starts, shards, slack):
    """Cache elements that hold `slack` times the largest part any shard gets."""
    el = np.int64(1) << (3 * (5 - lods.astype(np.int64)))
    part = 0
    for w in range(shards):
        m = (ids % shards) == w
        part = max(part, int(np.add.reduceat(np.where(m, el, 0), starts[:-1].astype(np.int64)).max()))
    return shards * (int(slack * part) + 64)


@pytest.mark.parametrize("shards", [1, 4])
def test_served_requests_equal_alone_and_oracle(P, shards):
    import torch
    vol = synth.neurite_u32(256, 600, seed=12)
    c = oracle.encode_volume(vol, 5, nthreads=8)
    dv = P.DeviceVolume(c)
    grid = (8, 8, 8)
    ids, lods, starts, arr = workloads.frustum_requests(60, grid, 2000.0, seed=5, n_max=256, orbit=(0.75, 3.0))
    cache_elems = _cache_for(ids, lods, starts, shards, 1.1)  # well under the volume: eviction and slot reuse
    assert cache_elems < 0.6 * 512 * 32 ** 3
    cache = torch.zeros(cache_elems, dtype=torch.int32, device="cuda")
    _say("shards", shards, "cache elements", cache_elems)
    srv = P.csgv.csgv_server(dv.info, dv.tensor, cache, cache_elems, n_streams=2, max_batch=512, keep_pinned=True,
                             n_shards=shards)
    t0 = srv.clock()
    for r in range(60):
        a, b = int(starts[r]), int(starts[r + 1])
        srv.submit(ids[a:b], lods[a:b], t0 + float(arr[r]) * 0.2)
    done = 0
    checked = 0
    while done < 60:
        srv.step()
        for d in srv.drain():
            done += 1
            assert d.status == 0, d.status
            r = int(d.req)
            a, b = int(starts[r]), int(starts[r + 1])
            rid, rl = ids[a:b], lods[a:b]
            torch.cuda.synchronize()
            host = cache.cpu().numpy().view(np.uint32)
            got = np.concatenate([host[srv.where(int(i), int(l)):srv.where(int(i), int(l)) + (32 >> int(l)) ** 3]
                                  for i, l in zip(rid, rl)])
            alone, offs = _alone(P, dv, rid, rl)
            want, wst = oracle.decode_tasks(c, rid, rl, offs, len(alone), 4, nthreads=8)
            assert (wst == 0).all()
            assert np.array_equal(got, alone), "request %d differs from its alone decode" % r
            assert np.array_equal(got, want), "request %d differs from the oracle" % r
            srv.release(r)
            checked += 1
    s = srv.stats()
    _say("served", checked, "requests;", s)
    assert s["evictions"] > 0 and s["batches"] >= 2 and s["failed_tasks"] == 0
    srv.destroy()


@pytest.mark.parametrize("shards", [1, 4])
def test_served_trace_run_completes(P, shards):
    import torch
    vol = synth.voronoi_voids(256, 2500, seed=6)
    c = oracle.encode_volume(vol, 5, nthreads=8)
    dv = P.DeviceVolume(c)
    ids, lods, starts, arr = workloads.frustum_requests(300, (8, 8, 8), 3000.0, seed=9, n_max=512)
    cache_elems = _cache_for(ids, lods, starts, shards, 1.5)
    cache = torch.zeros(cache_elems, dtype=torch.int32, device="cuda")
    _say("shards", shards, "cache elements", cache_elems)
    srv = P.csgv.csgv_server(dv.info, dv.tensor, cache, cache_elems, n_streams=3, max_batch=1024, n_shards=shards)
    rec = srv.run(ids, lods, starts, arr)
    lat = rec["t_done"] - rec["t_arrival"]
    _say("trace: p50 %.3f ms p99 %.3f ms" % (1e3 * np.percentile(lat, 50), 1e3 * np.percentile(lat, 99)))
    assert (rec["status"] == 0).all() and (lat >= 0).all()
    assert (rec["t_admit"] >= rec["t_arrival"] - 1e-9).all()
    s = srv.stats()
    assert s["requests_done"] == 300 and s["failed_tasks"] == 0
    assert s["hits"] + s["joined"] + s["decoded"] == s["pairs_requested"]
    distinct = [len(set(zip(ids[a:b].tolist(), lods[a:b].tolist()))) for a, b in zip(starts[:-1], starts[1:])]
    assert rec["n_pairs"].tolist() == distinct and int(rec["n_decoded"].sum()) == s["decoded"]
    # after the run, every pair of the trace's last request is resident where the oracle puts its labels
    a, b = int(starts[-2]), int(starts[-1])
    torch.cuda.synchronize()
    host = cache.cpu().numpy().view(np.uint32)
    got = np.concatenate([host[srv.where(int(i), int(l)):srv.where(int(i), int(l)) + (32 >> int(l)) ** 3]
                          for i, l in zip(ids[a:b], lods[a:b])])
    offs, total = P.dense_offsets(np.full(b - a, 5, np.uint8), lods[a:b])
    want, wst = oracle.decode_tasks(c, ids[a:b], lods[a:b], offs, total, 4, nthreads=8)
    assert (wst == 0).all() and np.array_equal(got, want)
    srv.destroy()
