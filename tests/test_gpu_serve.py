"""Served decode on the GPU: a stream of frustum requests through the server
(cache, admission, continuous batching on two streams).  Every completed
request's cache slots must equal (a) the same pairs decoded alone with the
plain one-launch-per-brick form and (b) the CPU oracle -- the result of a
request is the same alone and in the mix, bit for bit."""
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


def test_served_requests_equal_alone_and_oracle(P):
    import torch
    vol = synth.neurite_u32(256, 600, seed=12)
    c = oracle.encode_volume(vol, 5, nthreads=8)
    dv = P.DeviceVolume(c)
    grid = (8, 8, 8)
    ids, lods, starts, arr = workloads.frustum_requests(60, grid, 2000.0, seed=5, n_max=256, orbit=(0.75, 3.0))
    per = np.add.reduceat(np.int64(1) << (3 * (5 - lods.astype(np.int64))), starts[:-1].astype(np.int64))
    cache_elems = int(1.1 * per.max())  # well under the volume: eviction and slot reuse across the stream
    assert cache_elems < 0.6 * 512 * 32 ** 3
    cache = torch.zeros(cache_elems, dtype=torch.int32, device="cuda")
    srv = P.csgv.csgv_server(dv.info, dv.tensor, cache, cache_elems, n_streams=2, max_batch=512, keep_pinned=True)
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


def test_served_trace_run_completes(P):
    import torch
    vol = synth.voronoi_voids(256, 2500, seed=6)
    c = oracle.encode_volume(vol, 5, nthreads=8)
    dv = P.DeviceVolume(c)
    ids, lods, starts, arr = workloads.frustum_requests(300, (8, 8, 8), 3000.0, seed=9, n_max=512)
    per = np.add.reduceat(np.int64(1) << (3 * (5 - lods.astype(np.int64))), starts[:-1].astype(np.int64))
    cache_elems = int(1.5 * per.max())
    cache = torch.zeros(cache_elems, dtype=torch.int32, device="cuda")
    srv = P.csgv.csgv_server(dv.info, dv.tensor, cache, cache_elems, n_streams=3, max_batch=1024)
    rec = srv.run(ids, lods, starts, arr)
    lat = rec["t_done"] - rec["t_arrival"]
    _say("trace: p50 %.3f ms p99 %.3f ms" % (1e3 * np.percentile(lat, 50), 1e3 * np.percentile(lat, 99)))
    assert (rec["status"] == 0).all() and (lat >= 0).all()
    assert (rec["t_admit"] >= rec["t_arrival"] - 1e-9).all()
    s = srv.stats()
    assert s["requests_done"] == 300 and s["failed_tasks"] == 0
    assert s["hits"] + s["joined"] + s["decoded"] == s["pairs_requested"]
    srv.destroy()
