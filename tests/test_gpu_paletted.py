"""GPU parity of cache-paletted output (Methods > Memory management > Cache
paletting): the decoder writing packed palette indices (I bits, floor(32/I)
per 32-bit word) against the CPU oracle's paletted decode, word for word,
with the same task status (palettes beyond 2^I entries and 64^3 cubes are
INVALID and untouched; damaged records zero-fill their words)."""
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
    import paper_2609_36898_amd
    return paper_2609_36898_amd


def _layout(P, c, ids, lods, bits):
    info = P.csgv_volume_parse(c)
    l2 = P.brick_log2b(c, info)[np.minimum(ids, info.n_bricks - 1).astype(np.int64)]
    voxels = np.int64(1) << (3 * (np.maximum(l2, lods) - lods).astype(np.int64))
    words = P.csgv.paletted_words(voxels, bits)
    offs = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    return offs, int(words.sum())


def _compare(P, c, ids, lods, bits, modes=(0, 2), dense=False, **kw):
    import torch
    ids = np.asarray(ids, np.uint32)
    lods = np.asarray(lods, np.uint8)
    offs, total = _layout(P, c, ids, lods, bits)
    total = max(total, 1)
    want, wst = oracle.decode_tasks_paletted(c, ids, lods, offs, total, bits, nthreads=8,
                                             out=np.full(total, 0x5A5A5A5A, np.uint32))
    dv = P.DeviceVolume(c)
    d_ids = torch.from_numpy(ids.view(np.int32)).cuda()
    d_lods = torch.from_numpy(lods).cuda()
    d_offs = None if dense else torch.from_numpy(offs.view(np.int64)).cuda()
    for mode in modes:
        _say("paletted mode", mode, "tasks", len(ids), "bits", bits, "dense", dense)
        out = torch.full((total,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
        status = torch.full((len(ids),), -1, dtype=torch.int32, device="cuda")
        P.csgv_decode_bricks(None, dv.info, dv.tensor, d_ids, d_lods, d_offs, len(ids), out, total, status,
                             mode=mode, palette_bits=bits, **kw)
        torch.cuda.synchronize()
        gst = status.cpu().numpy().view(np.uint32)
        got = out.cpu().numpy().view(np.uint32)
        assert np.array_equal(gst, wst), (gst[:8], wst[:8])
        if dense:  # packed back to back in task order: compare the tasks that wrote
            ok = wst == 0
            assert ok.all()
        assert np.array_equal(got, want), "mode %d: first mismatch at word %d" % (mode, int(np.nonzero(got != want)[0][0]))
    return wst


def test_paletted_voronoi_every_lod_and_width(P):
    c = P.encode_volume(synth.voronoi_small(0), 5)  # 128^3, 64 bricks
    info = P.csgv_volume_parse(c)
    I = P.csgv.palette_bits_for(info.max_palette)
    ids = np.repeat(np.arange(64), 6)
    lods = np.tile(np.arange(6), 64)
    for bits in (I, I + 1, 7, 16, 31):
        st = _compare(P, c, ids, lods, bits)
        assert (st == 0).all()
    # too narrow for the largest palettes: those tasks are refused, the rest decode
    st = _compare(P, c, ids, lods, max(1, I - 2))
    assert (st == 1).any() and (st == 0).any()


def test_paletted_dense_offsets(P):
    c = P.encode_volume(synth.voronoi_voids(128, 312, seed=3), 5)
    info = P.csgv_volume_parse(c)
    I = P.csgv.palette_bits_for(info.max_palette)
    rng = np.random.default_rng(2)
    ids = rng.permutation(64).astype(np.uint32)
    lods = rng.integers(0, 6, size=64).astype(np.uint8)
    _compare(P, c, ids, lods, I, dense=True)


def test_paletted_neurite_and_two_labels(P):
    c = P.encode_volume(synth.neurite_u32(256, 600, seed=12), 5)
    info = P.csgv_volume_parse(c)
    rng = np.random.default_rng(3)
    ids = rng.permutation(512).astype(np.uint32)
    lods = rng.integers(0, 4, size=512).astype(np.uint8)
    _compare(P, c, ids, lods, P.csgv.palette_bits_for(info.max_palette))
    # two labels per brick at most: one bit per voxel, 32 voxels per word
    v = (synth.voronoi_u32(64, 2, seed=4) % 2 + 1).astype(np.uint32)
    c2 = P.encode_volume(v, 5)
    assert P.csgv_volume_parse(c2).max_palette <= 2
    st = _compare(P, c2, np.arange(8), np.zeros(8), 1)
    assert (st == 0).all()


def test_paletted_u64_mixed_sides(P):
    bricks, l2 = [], []
    for i in range(8):
        side = 64 if i % 2 == 0 else 32
        b, _ = synth.uneven_brick_u64(side, 21, i)
        bricks.append(b.reshape(-1))
        l2.append(6 if side == 64 else 5)
    c = P.csgv_encode_bricks(np.concatenate(bricks), l2, 8, origins=np.zeros((8, 3), np.uint32))
    ids = np.repeat(np.arange(8), 3).astype(np.uint32)
    lods = np.tile([0, 1, 3], 8).astype(np.uint8)
    for bits in (18, 9, 4):
        st = _compare(P, c, ids, lods, bits)
        # 64^3 cubes (even bricks at LOD 0) have no paletted form
        assert (st[(ids % 2 == 0) & (lods == 0)] == 1).all()


def test_paletted_corrupt_records(P):
    c = P.encode_volume(synth.voronoi_voids(128, 312, seed=3), 5)
    offs = oracle.brick_offsets(c)
    bad = bytearray(c)
    rng = np.random.default_rng(9)
    for k in range(0, 64, 3):  # damage payload bytes of every third record
        a, b = int(offs[k]), int(offs[k + 1])
        for _ in range(6):
            bad[int(rng.integers(a + 64, b))] ^= int(rng.integers(1, 256))
    bad = bytes(bad)
    info = P.csgv_volume_parse(bad)
    st = _compare(P, bad, np.arange(64), np.zeros(64), P.csgv.palette_bits_for(info.max_palette))
    assert (st == 2).any()


def test_paletted_plan_graph_replays(P):
    import torch
    c = P.encode_volume(synth.voronoi_voids(128, 312, seed=5), 5)
    info = P.csgv_volume_parse(c)
    bits = P.csgv.palette_bits_for(info.max_palette)
    ids = np.arange(64, dtype=np.uint32)
    lods = (np.arange(64) % 3).astype(np.uint8)
    offs, total = _layout(P, c, ids, lods, bits)
    want, wst = oracle.decode_tasks_paletted(c, ids, lods, offs, total, bits, nthreads=8)
    dv = P.DeviceVolume(c)
    d_ids = torch.from_numpy(ids.view(np.int32)).cuda()
    d_lods = torch.from_numpy(lods).cuda()
    d_offs = torch.from_numpy(offs.view(np.int64)).cuda()
    out = torch.zeros(total, dtype=torch.int32, device="cuda")
    status = torch.zeros(64, dtype=torch.int32, device="cuda")
    plan = P.csgv_plan(info, 64, palette_bits=bits)
    for r in range(3):
        out.fill_(-1)
        torch.cuda.synchronize()
        plan.launch(None, dv.tensor, d_ids, d_lods, d_offs, 64, out, total, status)
        torch.cuda.synchronize()
        assert (status.cpu().numpy() == 0).all()
        assert np.array_equal(out.cpu().numpy().view(np.uint32), want), "replay %d" % r
    plan.destroy()
