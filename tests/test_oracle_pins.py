"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests retypes the oracle's own formulas: they compare it with
hand-worked fixtures (tests/golden), brute force over tiny bricks, a
Counter-based mode, an independent Python decoder, construction-side answers
of a random stream generator, and closed forms.
"""
from collections import Counter
import itertools
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import streams
from tests import micro_decoder

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [l.strip() for l in f if l.strip() and not l.startswith("#")]


def _mode_min(vals):
    c = Counter(vals)
    top = max(c.values())
    return min(v for v, k in c.items() if k == top)


def _brick_labels(brick, lod):
    """Recursive mode-of-8 by Counter (independent of the oracle's C code)."""
    cur = brick.astype(object)
    for _ in range(lod):
        s = cur.shape[0] // 2
        nxt = np.empty((s, s, s), dtype=object)
        for z, y, x in itertools.product(range(s), repeat=3):
            nxt[z, y, x] = _mode_min(list(cur[2 * z:2 * z + 2, 2 * y:2 * y + 2, 2 * x:2 * x + 2].reshape(-1)))
        cur = nxt
    return cur


def _encode_one(brick, **kw):
    b = brick.shape[0]
    return oracle.encode_bricks(brick.reshape(-1), [b.bit_length() - 1], brick.dtype.itemsize, **kw)


def _decode_one(c, lod, lb):
    L = oracle.header(c)
    sym, se, info = oracle.record_symbols(c, 0)
    S = 1 << (int(info[1]) - lod)
    out, st = oracle.decode_tasks(c, [0], [lod], [0], S ** 3, lb)
    return st[0], out[:S ** 3].reshape(S, S, S)


# ------------------------------------------------------------------ golden
def test_delta_chains_golden():
    for line in _lines("delta_chains.txt"):
        parts = line.split()
        delta, entries = int(parts[0]), [int(p, 16) for p in parts[1:]]
        assert oracle.delta_entries(delta) == entries, delta
        # decoding side: the chain folds back to delta
        d = 0
        for e in entries:
            d = (d << 3) | (e & 7)
        assert d == delta
    # the paper's worst case for a 64^3 brick is 7 entries
    assert len(oracle.delta_entries(sum(8 ** i for i in range(7)))) == 7


def test_encoder_golden_examples():
    for line in _lines("encode_examples.txt"):
        name, side, vox, syms, ends, pal = [p.strip() for p in line.split("|")]
        side = int(side)
        if vox.startswith("slabx"):
            _, a, b = vox.split()
            brick = np.empty((side,) * 3, dtype=np.uint32)
            brick[:, :, : side // 2] = int(a)
            brick[:, :, side // 2:] = int(b)
        else:
            brick = np.array([int(v) for v in vox.split()], dtype=np.uint32).reshape(side, side, side)
        c = _encode_one(brick, coder=1)
        sym, se, info = oracle.record_symbols(c, 0)
        assert [int(s) for s in sym] == [int(s, 16) for s in syms.split()], name
        assert [int(s) for s in se] == [int(s) for s in ends.split()], name
        assert int(info[4]) == len(pal.split())
        st, out = _decode_one(c, 0, 4)
        assert st == 0 and np.array_equal(out, brick), name


def test_rans_golden():
    for line in _lines("rans_examples.txt"):
        freq, syms, state, words = [p.strip() for p in line.split("|")]
        freq = np.array([int(v) for v in freq.split()], dtype=np.uint16)
        syms = np.array([int(v) for v in syms.split()], dtype=np.uint8)
        words = [int(w) for w in words.split()]
        st, gw, w = oracle.rans_encode(syms, freq, 0)
        assert int(st[0]) == int(state) and [int(x) for x in w] == words
        rc, dec = oracle.rans_decode(len(syms), freq, 0, st, gw, w)
        assert rc == 0 and list(dec) == list(syms)


def test_freq_table_golden():
    for line in _lines("freq_tables.txt"):
        counts, freq = [p.strip() for p in line.split("|")]
        counts = [int(v) for v in counts.split()]
        want = [int(v) for v in freq.split()]
        got = [int(v) for v in oracle.make_freq(counts)]
        assert got == want, (counts, got)
        assert sum(got) in (0, 4096)


# ----------------------------------------------------- mode / downsample
def test_mode_rule_all_two_and_three_label_cubes():
    # every 2^3 brick over {0,1} and over {0,1,2}: LOD 1 = mode with ties to the smaller label
    for nlab in (2, 3):
        for combo in itertools.product(range(nlab), repeat=8):
            brick = (np.array(combo, dtype=np.uint32) * 7 + 3).reshape(2, 2, 2)
            got = oracle.downsample(brick, 1)[0, 0, 0]
            assert got == _mode_min(list(brick.reshape(-1))), combo


def test_downsample_matches_counter_mode_on_random_bricks():
    for seed in range(6):
        b = synth.test_brick_u64(8, seed % 3, 3 + seed, base=10, seed=seed)
        for lod in range(4):
            assert np.array_equal(oracle.downsample(b, lod), _brick_labels(b, lod).astype(np.uint64))


def test_constant_brick_everywhere_constant():
    for lb, dt in ((4, np.uint32), (8, np.uint64)):
        brick = np.full((32, 32, 32), 123456789 if lb == 4 else 2 ** 63 + 5, dtype=dt)
        c = _encode_one(brick)
        sym, se, info = oracle.record_symbols(c, 0)
        assert list(sym) == [0xC] and int(info[4]) == 1      # one ADV with stop, one palette entry
        assert list(se) == [1] * 6
        for lod in range(6):
            st, out = _decode_one(c, lod, lb)
            assert st == 0 and (out == brick[0, 0, 0]).all()


# -------------------------------------------------------------- round trip
def test_exhaustive_tiny_bricks_roundtrip():
    # all 2^3 bricks over 2 and 3 labels, both LODs, through encode -> decode
    bricks = []
    for nlab in (2, 3):
        for combo in itertools.product(range(nlab), repeat=8):
            bricks.append(np.array(combo, dtype=np.uint32) + 1)
    flat = np.concatenate(bricks)
    n = len(bricks)
    for mask in (63, 1 | 16 | 32, 0):
        c = oracle.encode_bricks(flat, [1] * n, 4, op_mask=mask)
        for lod in (0, 1):
            offs, tot = oracle.dense_offsets([1] * n, [lod] * n)
            out, st = oracle.decode_tasks(c, np.arange(n), [lod] * n, offs, tot, 4)
            assert (st == 0).all()
            if lod == 0:
                assert np.array_equal(out, flat)
            else:
                want = [_mode_min(list(b)) for b in bricks]
                assert list(out) == want


@pytest.mark.parametrize("log2b", [2, 3])
def test_random_bricks_every_op_set_and_coder(log2b):
    b = 1 << log2b
    prefixes = [0, 1, 3, 7, 15, 31, 63]  # palette-only, then the ablation order of the paper
    kinds = [(0, 2), (0, 5), (1, 4), (2, 3), (0, 40)]
    for (kind, nlab), mask, nmode, coder, lane in itertools.product(kinds, prefixes, (0, 1), (1, 2), (1, 8)):
        brick = synth.test_brick_u64(b, kind, nlab, base=1000, seed=kind * 7 + nlab + mask).astype(np.uint64)
        c = _encode_one(brick, op_mask=mask, neighbor_mode=nmode, coder=coder, lane_syms=lane)
        for lod in range(log2b + 1):
            st, out = _decode_one(c, lod, 8)
            assert st == 0
            assert np.array_equal(out, oracle.downsample(brick, lod)), (kind, nlab, mask, lod)


def test_volume_roundtrip_every_lod():
    v = synth.voronoi_u32(64, 40, seed=3)
    c = oracle.encode_volume(v, 5)
    n = 8
    flat = oracle._bricks_of_volume(v, 5)
    for lod in range(6):
        offs, tot = oracle.dense_offsets([5] * n, [lod] * n)
        out, st = oracle.decode_tasks(c, np.arange(n), [lod] * n, offs, tot, 4, nthreads=4)
        assert (st == 0).all()
        S = 32 >> lod
        for k in range(n):
            want = oracle.downsample(flat[k * 32768:(k + 1) * 32768].reshape(32, 32, 32), lod)
            assert np.array_equal(out[offs[k]:offs[k] + S ** 3].reshape(S, S, S), want)


# ------------------------------------------------------------- invariants
def test_palette_without_duplicates_when_delta_enabled():
    # With unlimited back references a brick's palette holds each label once
    # (paper, Results > "CSGV" and Methods > "Cache paletting").
    for seed in range(5):
        brick = synth.test_brick_u64(16, seed % 3, 20 + 10 * seed, base=1, seed=seed)
        c = _encode_one(brick, op_mask=63)
        h = oracle.header(c)
        offs = oracle.brick_offsets(c)
        sym, se, info = oracle.record_symbols(c, 0)
        pc = int(info[4])
        rec = np.frombuffer(c, dtype=np.uint8, count=int(offs[1] - offs[0]), offset=int(offs[0]))
        hdr = 8 + 4 * 5 + (4 * ((2 ** int(info[3]) + 63) // 64) + 4 * 2 ** int(info[3]) if info[0] == 1 else 0)
        hdr = (hdr + 7) // 8 * 8
        pal = rec[hdr:hdr + 8 * pc].view(np.uint64)
        assert len(set(pal.tolist())) == pc
        assert set(pal.tolist()) == set(np.unique(brick).tolist())
        # palette order = first use in decode order: scan the level grids
        assert h["label_bytes"] == 8


def test_label_set_preserved_and_lod_shrinks_by_eight():
    brick = synth.test_brick_u64(16, 1, 9, base=77, seed=1)
    c = _encode_one(brick)
    st, out0 = _decode_one(c, 0, 8)
    assert set(np.unique(out0)) == set(np.unique(brick))
    for lod in range(1, 5):
        st, out = _decode_one(c, lod, 8)
        assert out.size * 8 ** lod == brick.size


def _level_counts(sym, se, L):
    """(ops, entries, open) per level from a symbol stream (2-state automaton)."""
    res = []
    pos = 0
    for i in range(L + 1):
        ops = ents = opened = 0
        in_chain = False
        while pos < se[i]:
            s = int(sym[pos])
            pos += 1
            if in_chain:
                ents += 1
                in_chain = bool(s & 8)
            else:
                ops += 1
                opened += 0 if (s & 8) else 1
                in_chain = (s & 7) == 6
        res.append((ops, ents, opened))
    return res


def test_counting_invariant():
    # explicit nodes of level i = 8 x (explicit, non-stopped nodes of level i-1);
    # symbols = explicit nodes + delta entries
    for seed in range(4):
        brick = synth.test_brick_u64(32, seed % 3, 12, base=5, seed=seed)
        c = _encode_one(brick, op_mask=63)
        sym, se, info = oracle.record_symbols(c, 0)
        counts = _level_counts(sym, se, 5)
        assert counts[0][0] == 1
        for i in range(1, 6):
            assert counts[i][0] == 8 * counts[i - 1][2]
        assert sum(o + e for o, e, _ in counts) == len(sym)


# -------------------------------------------------------------------- rANS
@pytest.mark.parametrize("log2W", list(range(9)))
def test_rans_roundtrip_every_lane_count(log2W):
    rng = np.random.default_rng(log2W)
    p = rng.dirichlet(np.ones(16) * 0.5)
    for n in (0, 1, 5, 63, 64, 65, 1000, 5000):
        sym = rng.choice(16, size=n, p=p).astype(np.uint8)
        counts = np.bincount(sym, minlength=16) if n else np.ones(16)
        freq = oracle.make_freq(counts)
        assert int(freq.sum()) == 4096 and all(freq[s] >= 1 for s in range(16) if counts[s])
        st, gw, w = oracle.rans_encode(sym, freq, log2W)
        rc, dec = oracle.rans_decode(n, freq, log2W, st, gw, w)
        assert rc == 0 and np.array_equal(dec, sym)
        # python encoder of the same definition agrees word for word
        x, gw2, w2 = streams.rans_encode_py(list(sym), [int(f) for f in freq], log2W)
        assert list(x) == list(st) and list(gw2) == list(gw) and list(w2) == list(w)
        if n >= 1000:
            # size: within 0.1 bit/symbol of the entropy under the table, plus 48 bits per lane
            bits = -np.sum(np.log2(freq[sym] / 4096.0))
            assert 16 * len(w) <= bits + 0.1 * n + 48 * (1 << log2W)
        # the final decoder state returns to the encoder's start state
        if n:
            assert rc == 0


def test_raw4_and_rans_carry_identical_symbols():
    v = synth.voronoi_u32(64, 60, seed=5)
    c_raw = oracle.encode_volume(v, 5, coder=1)
    c_rans = oracle.encode_volume(v, 5, coder=2)
    for k in range(8):
        s1, e1, i1 = oracle.record_symbols(c_raw, k)
        s2, e2, i2 = oracle.record_symbols(c_rans, k)
        assert i1[0] == 0 and i2[0] == 1
        assert np.array_equal(s1, s2) and np.array_equal(e1, e2)


# --------------------------------------------------- random valid streams
def _three_way(c, L, grids, lb, nbricks=1):
    for lod in range(L + 1):
        S = 1 << (L - lod)
        out, st = oracle.decode_tasks(c, [0], [lod], [0], S ** 3, lb)
        assert st[0] == 0, lod
        got = out[:S ** 3].reshape(S, S, S)
        verdict, py = micro_decoder.decode(c, 0, lod)
        assert verdict == "ok"
        assert np.array_equal(np.array(py, dtype=np.uint64), got.astype(np.uint64))
        assert np.array_equal(streams.grid_to_linear(grids[L - lod], L - lod), got.astype(np.uint64))


@pytest.mark.parametrize("seed", range(12))
def test_random_valid_streams_three_way(seed):
    rng = np.random.default_rng(seed)
    L = 1 + seed % 3
    lb = 8 if seed % 2 else 4
    syms, se, pal, grids = streams.random_stream(rng, L, lb, n_label_pool=(5 if seed % 4 == 0 else None))
    if seed % 3 == 0:
        rec = streams.record_bytes(L, lb, syms, se, pal)
        c = streams.container([rec], lb)
    else:
        freq = streams.freq_from_counts(np.bincount(syms, minlength=16))
        rec = streams.record_bytes(L, lb, syms, se, pal, coder=1, freq=freq, log2W=seed % 7)
        c = streams.container([rec], lb, freq=freq)
    _three_way(c, L, grids, lb)


# ------------------------------------------------------------ error paths
def _valid_small(seed=0, coder=0):
    rng = np.random.default_rng(seed)
    syms, se, pal, grids = streams.random_stream(rng, 2, 4)
    freq = streams.freq_from_counts(np.bincount(syms, minlength=16))
    rec = streams.record_bytes(2, 4, syms, se, pal, coder=coder, freq=freq, log2W=1)
    return syms, se, pal, streams.container([rec], 4, freq=freq)


def _verdicts(c, lod=0, L=2):
    S = 1 << (L - lod)
    out, st = oracle.decode_tasks(c, [0], [lod], [0], S ** 3, 4)
    v, py = micro_decoder.decode(c, 0, lod)
    return int(st[0]), v, out[:S ** 3]


def _corrupt_record(syms, se, pal, L=2):
    return streams.container([streams.record_bytes(L, 4, syms, se, pal)], 4)


def test_targeted_corruptions():
    cases = []
    cases.append(([0], [1, 1], [5], 1))                        # PARENT at the root
    cases.append(([1], [1, 1], [5], 1))                        # NX at x = 0
    cases.append(([5], [1, 1], [5], 1))                        # LAST with an empty palette so far
    cases.append(([4, 0, 0, 0, 0, 0, 0, 0, 6, 0], [1, 10], [5], 1))  # delta = 0
    cases.append(([4, 0, 0, 0, 0, 0, 0, 0, 6, 2], [1, 10], [5], 1))  # delta > n
    cases.append(([4, 0, 0, 0, 0, 0, 0, 0, 7], [1, 9], [5], 1))     # op 7
    cases.append(([4, 0, 0, 0, 0, 0, 0, 0, 4], [1, 9], [5], 1))     # ADV past the palette
    cases.append(([4, 0, 0, 0, 0, 0, 0, 0], [1, 8], [5], 1))        # level 1 one symbol short
    cases.append(([4, 0, 0, 0, 0, 0, 0, 0, 0, 0], [1, 10], [5], 1))  # one symbol too many
    cases.append(([4, 0, 0, 0, 0, 0, 0, 0, 6, 9], [1, 10], [5], 1))  # delta chain runs off the level
    cases.append(([4, 0, 0, 0, 0, 0, 0, 0, 0], [1, 9], [5, 6], 1))  # palette entry never read (t = L)
    cases.append(([4, 0, 0, 0, 0, 0, 0, 0, 0], [2, 9], [5], 1))     # level 0 end past its symbols
    for syms, se, pal, L in cases:
        c = _corrupt_record(syms, se, pal, L)
        st, v, out = _verdicts(c, 0, L)
        assert st == oracle.ST_CORRUPT and v == "corrupt", (syms, se, pal)
        assert (out == 0).all()
    # a palette entry left over is fine when decoding a coarser LOD
    c = _corrupt_record([4, 0, 0, 0, 0, 0, 0, 0, 0], [1, 9], [5, 6], 1)
    st, v, out = _verdicts(c, 1, 1)
    assert st == 0 and v == "ok" and out[0] == 5


def test_invalid_tasks_leave_output_untouched():
    syms, se, pal, c = _valid_small()
    out, st = oracle.decode_tasks(c, [1], [0], [0], 64, 4)           # brick id out of range
    assert st[0] == oracle.ST_INVALID and (out[:64] == 0xA5A5A5A5).all()
    out, st = oracle.decode_tasks(c, [0], [3], [0], 64, 4)           # LOD beyond the brick
    assert st[0] == oracle.ST_INVALID and (out[:64] == 0xA5A5A5A5).all()
    out, st = oracle.decode_tasks(c, [0], [0], [1], 64, 4)           # output range too short
    assert st[0] == oracle.ST_INVALID and (out[:64] == 0xA5A5A5A5).all()


@pytest.mark.parametrize("coder", [0, 1])
def test_random_byte_flips_agree_with_python_decoder(coder):
    rng = np.random.default_rng(100 + coder)
    base_syms, base_se, base_pal, c0 = _valid_small(seed=coder + 3, coder=coder)
    offs = oracle.brick_offsets(c0)
    n_corrupt = 0
    for trial in range(300):
        c = bytearray(c0)
        for _ in range(int(rng.integers(1, 4))):
            p = int(rng.integers(offs[0], offs[1]))
            c[p] ^= 1 << int(rng.integers(8))
        c = bytes(c)
        for lod in (0, 1, 2):
            S = 1 << (2 - lod)
            out, st = oracle.decode_tasks(c, [0], [lod], [0], S ** 3, 4)
            v, py = micro_decoder.decode(c, 0, lod, S ** 3)
            want = {"ok": 0, "invalid": 1, "corrupt": 2}[v]
            assert int(st[0]) == want, (trial, lod)
            if v == "ok":
                assert np.array_equal(out[:S ** 3].reshape(S, S, S).astype(np.uint64), np.array(py, dtype=np.uint64))
            elif v == "corrupt":
                n_corrupt += 1
    assert n_corrupt > 50


# ------------------------------------------------------------- generators
def test_pcg32_reference_value():
    # O'Neill's pcg32 demo (seed 42, sequence 54) starts with 0xa15c02b7
    assert synth.pcg32_first(42, 54) == 0xA15C02B7


def test_workload_generators_shape():
    v = synth.voronoi_small(0)
    assert v.shape == (128, 128, 128) and v.min() == 1 and v.max() == 500
    w = synth.voronoi_voids(128, 312, 0)
    assert 0.10 <= (w == 0).mean() < 0.2
    t = synth.neurite_u32(256, 1562, 0)
    assert 0.2 < (t == 0).mean() < 0.4
    a = synth.neurite_u32(128, 200, 1)
    b = np.concatenate([synth.neurite_u32(128, 200, 1, 0, 40), synth.neurite_u32(128, 200, 1, 40, 128)])
    assert np.array_equal(a, b)  # slab-wise generation is exact
    kinds = [synth.uneven_brick_u64(32, 0, i)[1] for i in range(200)]
    assert 0.25 < kinds.count(0) / 200 < 0.55 and kinds.count(2) > 10


# ------------------------------------------------- cache-paletted output
def _unpack(words, n, bits):
    """Plain unpacking of the cache-paletted form, written out here."""
    e = 32 // bits
    return np.array([(int(words[k // e]) >> ((k % e) * bits)) & ((1 << bits) - 1) for k in range(n)], dtype=np.uint32)


def test_palette_packing_golden():
    # Methods > Memory management > Cache paletting: floor(32/I) entries per word
    for line in _lines("palette_pack.txt"):
        b, idx, words = (x.strip() for x in line.split("|"))
        got = oracle.pack_indices([int(v) for v in idx.split()], int(b))
        assert [int(w, 16) for w in words.split()] == got.tolist()


def test_palette_packing_roundtrip_every_width():
    rng = np.random.default_rng(0)
    for bits in range(1, 32):
        idx = rng.integers(0, 1 << bits, size=int(rng.integers(1, 300)), dtype=np.uint64).astype(np.uint32)
        words = oracle.pack_indices(idx, bits)
        e = 32 // bits
        assert len(words) == -(-len(idx) // e)
        assert np.array_equal(_unpack(words, len(idx), bits), idx)
        # bits above the last entry of every word stay zero
        if e * bits < 32:
            assert (words >> np.uint32(e * bits) == 0).all()


@pytest.mark.parametrize("lb", [4, 8])
def test_paletted_decode_is_the_first_occurrence_index(lb):
    # With unlimited back references (DELTA on) a palette holds each label once,
    # so a voxel's index is the position of its label in its brick's palette;
    # unpacked through the palette the paletted decode is the label decode.
    if lb == 4:
        c = oracle.encode_volume(synth.voronoi_voids(64, 60, seed=5), 5)
    else:
        bricks = [synth.test_brick_u64(32, k % 3, 2 + 9 * k, base=1, seed=k).reshape(-1) for k in range(4)]
        c = oracle.encode_bricks(np.concatenate(bricks), [5] * 4, 8)
    n = oracle.header(c)["n_bricks"]
    pmax = max(len(oracle.record_palette(c, k)) for k in range(n))
    bits = max(1, int(np.ceil(np.log2(pmax))))
    for lod in (0, 1, 2, 5):
        ids = np.arange(n)
        lods = np.full(n, lod)
        S3 = (32 >> lod) ** 3
        offs, tot = oracle.dense_offsets([5] * n, lods)
        labels, st = oracle.decode_tasks(c, ids, lods, offs, tot, lb, nthreads=4)
        assert (st == 0).all()
        wcount = oracle.paletted_words(np.full(n, S3), bits)
        woffs = np.concatenate([[0], np.cumsum(wcount)[:-1]]).astype(np.uint64)
        words, pst = oracle.decode_tasks_paletted(c, ids, lods, woffs, int(wcount.sum()), bits, nthreads=4)
        assert (pst == 0).all()
        for k in range(n):
            pal = oracle.record_palette(c, k)
            a = int(woffs[k])
            idx = _unpack(words[a:a + int(wcount[k])], S3, bits)
            lab = labels[offs[k]:offs[k] + S3].astype(np.uint64)
            assert np.array_equal(pal[idx], lab)
            first = {int(v): i for i, v in reversed(list(enumerate(pal.tolist())))}
            assert np.array_equal(idx, np.array([first[int(v)] for v in lab], dtype=np.uint32))


def test_paletted_duplicates_keep_the_stream_index():
    # without back references a palette repeats labels; the index is the one the
    # operation stream designates, and it still maps to the decoded label
    brick = synth.test_brick_u64(16, 1, 6, base=1, seed=3).astype(np.uint32)
    c = oracle.encode_bricks(brick.reshape(-1), [4], 4, op_mask=0)
    pal = oracle.record_palette(c, 0)
    assert len(pal) > len(set(pal.tolist()))
    bits = int(np.ceil(np.log2(len(pal))))
    words, st = oracle.decode_tasks_paletted(c, [0], [0], [0], int(oracle.paletted_words(4096, bits)), bits)
    assert st[0] == 0
    idx = _unpack(words, 4096, bits)
    assert np.array_equal(pal[idx], brick.reshape(-1).astype(np.uint64))
    # ... and is not simply the label's first palette position
    first = {int(v): i for i, v in reversed(list(enumerate(pal.tolist())))}
    assert any(first[int(pal[i])] != i for i in set(idx.tolist()))


def test_paletted_invalid_and_corrupt_tasks():
    c = oracle.encode_volume(synth.voronoi_voids(64, 60, seed=5), 5)
    pmax = max(len(oracle.record_palette(c, k)) for k in range(8))
    small = max(1, int(np.ceil(np.log2(pmax))) - 1)  # too few bits for the largest palette
    ids = np.arange(8)
    wcount = oracle.paletted_words(np.full(8, 32768), small)
    woffs = np.concatenate([[0], np.cumsum(wcount)[:-1]]).astype(np.uint64)
    words, st = oracle.decode_tasks_paletted(c, ids, np.zeros(8), woffs, int(wcount.sum()), small)
    pcs = np.array([len(oracle.record_palette(c, k)) for k in range(8)])
    assert np.array_equal(st == 1, pcs > (1 << small))
    for k in np.nonzero(st == 1)[0]:  # untouched
        a = int(woffs[k])
        assert (words[a:a + int(wcount[k])] == 0xA5A5A5A5).all()
    # 64^3 bricks at full resolution have no paletted form
    b, _ = synth.uneven_brick_u64(64, 3, 1)
    c64 = oracle.encode_bricks(b.reshape(-1), [6], 8)
    _, st = oracle.decode_tasks_paletted(c64, [0, 0], [0, 1], [0, 100000], 200000, 18)
    assert list(st) == [1, 0]
    # a damaged record zero-fills its words
    offs = oracle.brick_offsets(c)
    bad = bytearray(c)
    bad[int(offs[2]) + 8] = 0xFF  # sym_end[0] of brick 2: no longer ordered
    nw = int(oracle.paletted_words(32768, small + 1))
    words, st = oracle.decode_tasks_paletted(bytes(bad), [2], [0], [0], nw, small + 1)
    assert st[0] == 2 and (words[:nw] == 0).all()
