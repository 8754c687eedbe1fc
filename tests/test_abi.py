"""CPU checks of the C-ABI library: it loads, exports what include/csgv.h
declares, rejects bad arguments before touching the GPU, and its host encoder
writes the same bytes as the oracle's encoder."""
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    lib = os.path.join(ROOT, "paper_2609_36898_amd", "libcsgv.so")
    if not os.path.exists(lib):
        from paper_2609_36898_amd import _build
        _build.build()
    import paper_2609_36898_amd
    return paper_2609_36898_amd


def _declared():
    src = open(os.path.join(ROOT, "include", "csgv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(csgv_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(P):
    lib = os.path.join(ROOT, "paper_2609_36898_amd", "libcsgv.so")
    out = subprocess.run(["nm", "-D", "--defined-only", lib], capture_output=True, text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    declared = _declared()
    assert declared, "no declarations found"
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    assert set(P.csgv.EXPORTED) == set(declared)


def test_volume_parse_rejects_bad_headers(P):
    v = synth.voronoi_u32(64, 20, seed=1)
    c = P.encode_volume(v, 5)
    info = P.csgv_volume_parse(c)
    assert info.n_bricks == 8 and info.label_bytes == 4 and list(info.grid) == [2, 2, 2]
    bad = bytearray(c)
    bad[0] ^= 1
    with pytest.raises(P.CsgvError):
        P.csgv_volume_parse(bytes(bad))
    bad = bytearray(c)
    bad[24] = 3  # label width 3
    with pytest.raises(P.CsgvError):
        P.csgv_volume_parse(bytes(bad))
    with pytest.raises(P.CsgvError):
        P.csgv_volume_parse(c[:100])


def test_decode_rejects_null_arguments_synchronously(P):
    c = P.encode_volume(synth.voronoi_u32(64, 20, seed=1), 5)
    info = P.csgv_volume_parse(c)
    with pytest.raises(P.CsgvError) as e:
        P.csgv_decode_bricks(0, info, None, None, None, None, 4, None, 0, None)
    assert e.value.code == P.csgv.CSGV_EINVAL
    # n = 0 is a no-op
    P.csgv_decode_bricks(0, info, None, None, None, None, 0, None, 0, None)


@pytest.mark.parametrize("case", ["voronoi", "neurite", "uneven64", "masks"])
def test_host_encoder_matches_oracle_encoder(P, case):
    if case == "voronoi":
        v = synth.voronoi_voids(128, 312, seed=2)
        assert P.encode_volume(v, 5) == oracle.encode_volume(v, 5)
    elif case == "neurite":
        v = synth.neurite_u32(128, 200, seed=4)
        for cp in (0, 1, 2):
            assert P.encode_volume(v, 5, coder_policy=cp) == oracle.encode_volume(v, 5, coder=cp)
    elif case == "uneven64":
        bricks, l2 = [], []
        for i in range(6):
            b, kind = synth.uneven_brick_u64(64 if i % 2 else 32, 7, i)
            bricks.append(b.reshape(-1))
            l2.append(6 if i % 2 else 5)
        flat = np.concatenate(bricks)
        org = np.arange(18, dtype=np.uint32).reshape(6, 3)
        a = P.csgv_encode_bricks(flat, l2, 8, origins=org)
        b = oracle.encode_bricks(flat, l2, 8, origins=org)
        assert a == b
    else:
        v = synth.voronoi_u32(64, 30, seed=5)
        for mask in (0, 1, 7, 31, 63):
            for nm in (0, 1):
                assert P.encode_volume(v, 5, op_mask=mask, neighbor_mode=nm, lane_syms=8) == \
                    oracle.encode_volume(v, 5, op_mask=mask, neighbor_mode=nm, lane_syms=8)


def test_volume_parse_bounds_by_given_bytes(P):
    c = P.encode_volume(synth.voronoi_u32(64, 20, seed=1), 5)
    info = P.csgv_volume_parse(c)
    assert info.total_bytes == len(c) and info.max_log2b == 5
    # truncated container: header claims more bytes than were given
    with pytest.raises(P.CsgvError) as e:
        P.csgv_volume_parse(c[:-8])
    assert e.value.code == P.csgv.CSGV_EINVAL
    # inflated total_bytes in the header
    bad = bytearray(c)
    bad[96:104] = np.uint64(len(c) + 4096).tobytes()
    with pytest.raises(P.CsgvError):
        P.csgv_volume_parse(bytes(bad))
    # offset table running past the container
    bad = bytearray(c)
    bad[32:36] = np.uint32(1 << 20).tobytes()
    with pytest.raises(P.CsgvError):
        P.csgv_volume_parse(bytes(bad))


def test_volume_parse_max_brick_side_from_records(P):
    bricks, l2 = [], []
    for i in range(4):
        b, _ = synth.uneven_brick_u64(64 if i == 2 else 32, 3, i)
        bricks.append(b.reshape(-1))
        l2.append(6 if i == 2 else 5)
    c = P.csgv_encode_bricks(np.concatenate(bricks), l2, 8, origins=np.zeros((4, 3), np.uint32))
    assert P.csgv_volume_parse(c).max_log2b == 6
    c = P.encode_volume(synth.voronoi_u32(32, 9, seed=2), 4)
    assert P.csgv_volume_parse(c).max_log2b == 4


def test_streaming_encoder_matches_one_shot(P):
    v = synth.voronoi_voids(128, 312, seed=2)
    flat = P.bricks_of_volume(v, 5)
    whole = P.encode_volume(v, 5)
    enc = P.csgv.csgv_encoder(4, dims=(128, 128, 128), default_log2b=5, grid=(4, 4, 4))
    per = 32 ** 3
    for k0 in range(0, 64, 24):  # three uneven slabs of bricks
        k1 = min(64, k0 + 24)
        enc.add(flat[k0 * per:k1 * per], [5] * (k1 - k0))
    assert enc.finish() == whole
    enc.destroy()


def _max_delta(sym):
    """Largest palette back reference in a symbol stream (sequential walk)."""
    best, j = 0, 0
    while j < len(sym):
        s = int(sym[j])
        j += 1
        if (s & 7) == 6:
            d, e = 0, 8
            while e & 8:
                e = int(sym[j])
                j += 1
                d = (d << 3) | (e & 7)
            best = max(best, d)
    return best


def test_legacy_back_reference_limit(P):
    # op_mask bit 6: DELTA only within 16 palette entries; labels further back are
    # appended again, so palettes carry duplicates; decoding is unchanged
    rng = np.random.default_rng(7)
    brick = rng.integers(1, 40, size=(16, 16, 16), dtype=np.uint64).astype(np.uint32)
    for mask, limited in ((63, False), (127, True)):
        c = P.csgv_encode_bricks(brick.reshape(-1), [4], 4, op_mask=mask)
        sym, se, info = oracle.record_symbols(c, 0)
        pal = oracle.record_palette(c, 0)
        md = _max_delta(sym)
        if limited:
            assert md <= 16 and len(pal) > len(set(pal.tolist()))
        else:
            assert md > 16 and len(pal) == len(set(pal.tolist()))
        out, st = oracle.decode_tasks(c, [0], [0], [0], 4096, 4)
        assert st[0] == 0 and np.array_equal(out, brick.reshape(-1))


def test_dcache_rejects_null_arguments_synchronously(P):
    c = P.encode_volume(synth.voronoi_u32(64, 20, seed=1), 5)
    info = P.csgv_volume_parse(c)
    with pytest.raises(P.CsgvError) as e:
        P.csgv.csgv_dcache(info, None, 1 << 20, stream=0)
    assert e.value.code == P.csgv.CSGV_EINVAL
    for rc in (P.csgv._lib.csgv_dcache_request(None, None, None, None, 4, None, None, None),
               P.csgv._lib.csgv_dcache_free(None, None, None, None, 4),
               P.csgv._lib.csgv_dcache_reset(None, None),
               P.csgv._lib.csgv_dcache_query(None, None, None, None)):
        assert rc == P.csgv.CSGV_EINVAL
    assert b"null" in P.csgv._lib.csgv_dcache_last_error()


def test_dcache_state_codes_match_header(P):
    src = open(os.path.join(ROOT, "include", "csgv.h")).read()
    codes = dict((k, int(v)) for k, v in re.findall(r"\bCSGV_DC_([A-Z]+)\s*=\s*(\d+)", src))
    assert codes == {"NEW": P.csgv.DC_NEW, "HIT": P.csgv.DC_HIT, "JOINED": P.csgv.DC_JOINED,
                     "FULL": P.csgv.DC_FULL, "INVALID": P.csgv.DC_INVALID}
