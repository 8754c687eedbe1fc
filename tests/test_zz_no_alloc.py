"""The decode entry point that allocates nothing (its scratch is a fixed
device array inside the library) against csgv_decode_bricks, through the C
ABI: two calls in a row, the second with a smaller input, each bit-identical
to the allocating entry point (labels and task status) on the same tasks, in
both launch forms, for 32^3 and 64^3 bricks; the device's free memory does
not change across a call (after the first one in the process, which places
the array); requests beyond the fixed limits are refused."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_36898_amd as P
    # the first use of the fixed array on a device makes the runtime place it
    # (the library's one-time cost on that GPU); later calls must allocate nothing
    c = P.encode_volume(synth.voronoi_voids(64, 40, seed=3), 5)
    dv = P.DeviceVolume(c)
    ids = np.zeros(1, np.uint32)
    lods = np.zeros(1, np.uint8)
    offs, total = P.dense_offsets(np.full(1, 5), lods)
    _, st, _ = _decode(P, P.csgv.csgv_decode_bricks_noalloc, dv, ids, lods, offs, total, P.MODE_PERSISTENT, False)
    assert (st == 0).all()
    return P


def _decode(P, fn, dv, ids, lods, offs, total, mode, dense):
    import torch
    lb = int(dv.info.label_bytes)
    d_ids = torch.from_numpy(np.ascontiguousarray(ids, np.uint32).view(np.int32)).cuda()
    d_lods = torch.from_numpy(np.ascontiguousarray(lods, np.uint8)).cuda()
    d_offs = None if dense else torch.from_numpy(np.ascontiguousarray(offs, np.uint64).view(np.int64)).cuda()
    out = torch.full((total,), 0x5A5A5A5A, dtype=torch.int64 if lb == 8 else torch.int32, device="cuda")
    status = torch.full((len(ids),), -1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    fn(None, dv.info, dv.tensor, d_ids, d_lods, d_offs, len(ids), out, total, status, mode=mode)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    return out.cpu().numpy(), status.cpu().numpy(), free1 - free0


def _two_calls(P, container, calls):
    dv = P.DeviceVolume(container)
    log2b = P.brick_log2b(container, dv.info)
    for mode in (P.MODE_PERSISTENT, P.MODE_PLAIN):
        for k, (ids, lods, dense) in enumerate(calls):
            offs, total = P.dense_offsets(log2b[ids.astype(np.int64)], lods)
            _say("noalloc mode", mode, "call", k, "tasks", len(ids), "dense", dense)
            want, wst, _ = _decode(P, P.csgv.csgv_decode_bricks, dv, ids, lods, offs, total, mode, dense)
            got, gst, dfree = _decode(P, P.csgv.csgv_decode_bricks_noalloc, dv, ids, lods, offs, total, mode, dense)
            assert (wst == 0).all()
            assert np.array_equal(gst, wst)
            assert np.array_equal(got, want), "call %d mode %d differs from csgv_decode_bricks" % (k, mode)
            assert dfree == 0, "free device memory changed by %d bytes across the call" % dfree
    return dv


def test_noalloc_matches_allocating_entry_point_32(P):
    vol = synth.voronoi_voids(256, 1500, seed=21)  # 512 bricks of 32^3
    c = P.encode_volume(vol, 5)
    rng = np.random.default_rng(4)
    ids1 = rng.permutation(512).astype(np.uint32)  # more tasks than the fixed scratch has work-groups
    lods1 = rng.integers(0, 6, size=512).astype(np.uint8)
    ids2 = rng.choice(512, size=40, replace=False).astype(np.uint32)
    lods2 = rng.integers(0, 3, size=40).astype(np.uint8)
    _two_calls(P, c, [(ids1, lods1, False), (ids2, lods2, True)])
    # the second call's labels are also the oracle's
    log2b = P.brick_log2b(c)
    offs, total = P.dense_offsets(log2b[ids2.astype(np.int64)], lods2)
    want, wst = oracle.decode_tasks(c, ids2, lods2, offs, total, 4, nthreads=8)
    dv = P.DeviceVolume(c)
    got, gst, _ = _decode(P, P.csgv.csgv_decode_bricks_noalloc, dv, ids2, lods2, offs, total, P.MODE_PERSISTENT, True)
    assert (wst == 0).all() and np.array_equal(gst, wst) and np.array_equal(got.view(np.uint32), want)


def test_noalloc_matches_allocating_entry_point_64(P):
    bricks, l2 = [], []
    for i in range(6):
        side = 64 if i % 2 == 0 else 32
        b, _ = synth.uneven_brick_u64(side, 17, i)
        bricks.append(b.reshape(-1))
        l2.append(6 if side == 64 else 5)
    c = P.csgv_encode_bricks(np.concatenate(bricks), l2, 8, origins=np.zeros((6, 3), np.uint32))
    ids1 = np.repeat(np.arange(6), 2).astype(np.uint32)
    lods1 = np.tile([0, 1], 6).astype(np.uint8)
    ids2 = np.array([4, 1, 0], np.uint32)
    lods2 = np.array([0, 2, 3], np.uint8)
    _two_calls(P, c, [(ids1, lods1, False), (ids2, lods2, True)])


def test_noalloc_refuses_beyond_its_limits(P):
    import torch
    vol = synth.voronoi_voids(64, 40, seed=2)
    c = P.encode_volume(vol, 5)
    dv = P.DeviceVolume(c)
    d = torch.zeros(16, dtype=torch.int32, device="cuda")
    with pytest.raises(RuntimeError, match="fixed scratch"):
        P.csgv.csgv_decode_bricks_noalloc(None, dv.info, dv.tensor, d, d, None, 262145, d, 16, None,
                                          mode=P.MODE_PERSISTENT)
