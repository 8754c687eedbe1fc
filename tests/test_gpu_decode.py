"""GPU parity: the HIP decoder (through the C ABI) against the CPU oracle,
bit for bit, on the same seeded inputs.  Status words and, for damaged
records, the zero-filled outputs must match too."""
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import streams

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


def _compare(P, container, ids, lods, modes=(0, 2), sentinel=0x5A5A5A5A, **kw):
    """Decode on the GPU in each mode and with the oracle; assert identical outputs and status."""
    import torch
    info = P.csgv_volume_parse(container)
    lb = int(info.label_bytes)
    log2b = P.brick_log2b(container, info)
    ids = np.asarray(ids, dtype=np.uint32)
    lods = np.asarray(lods, dtype=np.uint8)
    safe_ids = np.minimum(ids, info.n_bricks - 1).astype(np.int64)
    l2 = log2b[safe_ids]
    offs, total = P.dense_offsets(np.maximum(l2, lods), lods)
    total = max(total, 1)
    fill = np.uint64(sentinel) if lb == 8 else np.uint32(sentinel)
    want, wst = oracle.decode_tasks(container, ids, lods, offs, total, lb,
                                    out=np.full(total, fill, dtype=np.uint64 if lb == 8 else np.uint32),
                                    nthreads=8)
    dv = P.DeviceVolume(container)
    for mode in modes:
        _say("decode mode", mode, "tasks", len(ids), kw)
        d_ids = torch.from_numpy(ids.view(np.int32)).cuda()
        d_lods = torch.from_numpy(lods).cuda()
        d_offs = torch.from_numpy(offs.view(np.int64)).cuda()
        out = torch.full((total,), 0, dtype=dv.dtype, device="cuda")
        out.view(torch.int32).fill_(sentinel if lb == 4 else 0)
        if lb == 8:
            out.copy_(torch.from_numpy(np.full(total, fill, dtype=np.uint64).view(np.int64)).cuda())
        status = torch.full((max(len(ids), 1),), -1, dtype=torch.int32, device="cuda")
        P.csgv_decode_bricks(None, info, dv.tensor, d_ids, d_lods, d_offs, len(ids), out, total, status,
                             mode=mode, **kw)
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint64 if lb == 8 else np.uint32)
        gst = status[:len(ids)].cpu().numpy().view(np.uint32)
        assert np.array_equal(gst, wst), (mode, np.nonzero(gst != wst)[0][:10], gst[gst != wst][:10], wst[gst != wst][:10])
        if not np.array_equal(got, want):
            bad = np.nonzero(got != want)[0]
            task = np.searchsorted(offs.astype(np.int64), bad[0], side="right") - 1
            raise AssertionError("mode %d: %d mismatches, first at %d (task %d id %d lod %d): got %d want %d" %
                                 (mode, len(bad), bad[0], task, ids[task], lods[task], got[bad[0]], want[bad[0]]))
    return want, wst


def test_voronoi_small_every_lod(P):
    v = synth.voronoi_small(0)
    c = P.encode_volume(v, 5)
    n = 64
    for lod in range(6):
        _compare(P, c, np.arange(n), [lod] * n)
    # full resolution equals the raw bricks
    want, st = _compare(P, c, np.arange(n), [0] * n, modes=(2,))
    assert np.array_equal(want, P.bricks_of_volume(v, 5))


@pytest.mark.parametrize("policy", [1, 2])
def test_coders_and_mixed_lods(P, policy):
    v = synth.voronoi_voids(128, 312, seed=3)
    c = P.encode_volume(v, 5, coder_policy=policy, lane_syms=16)
    rng = np.random.default_rng(policy)
    ids = rng.permutation(64)
    lods = rng.integers(0, 6, size=64)
    _compare(P, c, ids, lods)


def test_op_masks_and_neighbor_modes(P):
    v = synth.neurite_u32(128, 200, seed=4)
    for mask in (0, 1, 15, 31, 63, 127):  # 127: back references limited to 16 entries (palette duplicates)
        for nm in (0, 1):
            c = P.encode_volume(v, 5, op_mask=mask, neighbor_mode=nm)
            _compare(P, c, np.arange(64), np.arange(64) % 4, modes=(2,))


def _random_stream_container(seed, n, lb, Ls=(1, 2, 3, 4, 5), coder_mix=True):
    rng = np.random.default_rng(seed)
    recs, all_syms, infos = [], [], []
    for k in range(n):
        L = int(Ls[k % len(Ls)])
        pool = 6 if k % 3 == 0 else None
        syms, se, pal, grids = streams.random_stream(rng, L, lb, n_label_pool=pool, p_stop=0.2 + 0.1 * (k % 4))
        infos.append((L, syms, se, pal))
        all_syms.extend(syms)
    freq = streams.freq_from_counts(np.bincount(all_syms, minlength=16))
    for k, (L, syms, se, pal) in enumerate(infos):
        coder = (k % 2) if coder_mix else 0
        recs.append(streams.record_bytes(L, lb, syms, se, pal, coder=coder, freq=freq, log2W=k % 9))
    # the header's brick side must cover every record: output offsets are sized from it
    return streams.container(recs, lb, freq=freq, log2b=max(Ls)), [i[0] for i in infos]


@pytest.mark.parametrize("lb", [4, 8])
def test_random_valid_streams(P, lb):
    c, Ls = _random_stream_container(10 + lb, 40, lb)
    ids, lods = [], []
    for k, L in enumerate(Ls):
        for lod in range(L + 1):
            ids.append(k)
            lods.append(lod)
    _compare(P, c, ids, lods)


@pytest.mark.parametrize("lb", [4, 8])
def test_random_valid_streams_64_bricks(P, lb):
    # 64^3 bricks: the level-6 grids, long neighbour chains and delta chains of a random grammar walk
    c, Ls = _random_stream_container(30 + lb, 3, lb, Ls=(6,))
    ids = [k for k in range(3) for lod in range(7)]
    lods = [lod for k in range(3) for lod in range(7)]
    _compare(P, c, ids, lods)


def test_big_bricks_and_uneven_content(P):
    bricks, l2 = [], []
    for i in range(10):
        side = 64 if i % 3 == 0 else 32
        b, kind = synth.uneven_brick_u64(side, 11, i)
        bricks.append(b.reshape(-1))
        l2.append(6 if side == 64 else 5)
    c = P.csgv_encode_bricks(np.concatenate(bricks), l2, 8, origins=np.zeros((10, 3), np.uint32))
    ids = np.repeat(np.arange(10), 3)
    lods = np.tile([0, 1, 2], 10)
    want, st = _compare(P, c, ids, lods)
    assert (st == 0).all()


def test_large_palette_without_back_references(P):
    # palette-only coding of a 32^3 noise brick: every node is an ADV, 37449 palette entries
    b = synth.test_brick_u64(32, 0, 1 << 30, base=1, seed=9).astype(np.uint32)
    c = P.csgv_encode_bricks(b.reshape(-1), [5], 4, op_mask=0)
    info = P.csgv_volume_parse(c)
    sym, se, inf = oracle.record_symbols(c, 0)
    assert inf[4] > 32768
    _compare(P, c, [0, 0, 0], [0, 1, 2])


def test_corrupt_records_match_oracle_verdicts(P):
    base, Ls = _random_stream_container(77, 24, 4, Ls=(2, 3))
    offs = oracle.brick_offsets(base)
    rng = np.random.default_rng(5)
    c = bytearray(base)
    for k in range(24):
        if k % 4 == 3:
            continue  # keep some records intact
        for _ in range(int(rng.integers(1, 4))):
            p = int(rng.integers(offs[k], offs[k + 1]))
            c[p] ^= 1 << int(rng.integers(8))
    c = bytes(c)
    ids, lods = [], []
    for k, L in enumerate(Ls):
        for lod in range(L + 1):
            ids.append(k)
            lods.append(lod)
    want, st = _compare(P, c, ids, lods)
    assert (st == 2).sum() > 10


def test_invalid_tasks(P):
    v = synth.voronoi_u32(64, 20, seed=1)
    c = P.encode_volume(v, 5)
    _compare(P, c, [0, 9, 3, 1000], [0, 0, 6, 1])


def test_persistent_runs_are_repeatable(P):
    import torch
    v = synth.voronoi_voids(256, 2500, seed=6)
    c = P.encode_volume(v, 5)
    dv = P.DeviceVolume(c)
    rng = np.random.default_rng(0)
    ids = rng.permutation(512)
    lods = rng.integers(0, 4, 512)
    ref = None
    for wg in (256, 512, 1024):
        for sort in (0, 1):
            out, st, offs = dv.decode(ids, lods, mode=P.MODE_PERSISTENT, wg_size=wg, sort_tasks=sort)
            torch.cuda.synchronize()
            o = out.cpu().numpy()
            assert (st.cpu().numpy() == 0).all()
            if ref is None:
                ref = o
            assert np.array_equal(o, ref), (wg, sort)
    want, st = oracle.decode_tasks(c, ids, lods, offs, len(ref), 4, nthreads=8)
    assert np.array_equal(ref.view(np.uint32), want)


def test_plan_graph_replays(P):
    import torch
    v = synth.voronoi_voids(128, 312, seed=8)
    c = P.encode_volume(v, 5)
    dv = P.DeviceVolume(c)
    ids = np.arange(64)
    lods = np.arange(64) % 3
    d_ids, d_lods, d_offs, offs, total = dv.tasks(ids, lods)
    plan = P.csgv_plan(dv.info, 64)
    want, wst = oracle.decode_tasks(c, ids, lods, offs, total, 4)
    for rep in range(4):
        out = torch.zeros(total, dtype=torch.int32, device="cuda")
        st = torch.full((64,), -1, dtype=torch.int32, device="cuda")
        plan.launch(None, dv.tensor, d_ids, d_lods, d_offs, 64, out, total, st)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().view(np.uint32), want), rep
        assert (st.cpu().numpy() == 0).all()
    plan.set_timing(True)
    out = torch.zeros(total, dtype=torch.int32, device="cuda")
    plan.launch(None, dv.tensor, d_ids, d_lods, d_offs, 64, out, total, None)
    assert plan.last_kernel_ms() > 0
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint32), want)
    plan.destroy()
