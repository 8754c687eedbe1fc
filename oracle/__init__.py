"""Plain CPU oracle of the CSGV brick codec (ctypes wrapper around csgv_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may use it; the product path never does.  It shares no code
with the GPU decoder.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_oracle.so")
_lib = None

# op codes and encoder op-mask bits (the oracle's own copy of the format)
PARENT, NX, NY, NZ, ADV, LAST, DELTA = range(7)
M_PARENT, M_NX, M_NY, M_NZ, M_LAST, M_DELTA = 1, 2, 4, 8, 16, 32
ALL_OPS = 63
ST_OK, ST_INVALID, ST_CORRUPT = 0, 1, 2


def build(verbose: bool = False) -> str:
    src = os.path.join(_HERE, "csgv_oracle.c")
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", src, "-o", LIB_PATH + ".tmp"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    P, U32, U64, I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    lib.oracle_downsample.argtypes = [P, I, I, I, P]
    lib.oracle_delta_entries.argtypes = [U32, P]
    lib.oracle_make_freq.argtypes = [P, P]
    lib.oracle_rans_encode.argtypes = [P, U32, P, I, P, P, P, U32]
    lib.oracle_rans_encode.restype = U32
    lib.oracle_rans_decode.argtypes = [P, U32, P, I, P, P, P]
    lib.oracle_encode_volume.argtypes = [P, P, U32, I, P, I, P, P, I, I, I, I, I,
                                         ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(U64)]
    lib.oracle_free.argtypes = [P]
    lib.oracle_decode_tasks.argtypes = [P, U64, P, P, P, U32, P, U64, P, I]
    lib.oracle_decode_tasks_paletted.argtypes = [P, U64, P, P, P, U32, P, U64, P, I, I]
    lib.oracle_pack_indices.argtypes = [P, U64, I, P]
    lib.oracle_record_palette.argtypes = [P, U64, U32, P, U32]
    lib.oracle_record_palette.restype = ctypes.c_int64
    lib.oracle_record_symbols.argtypes = [P, U64, U32, P, U32, P, P]
    lib.oracle_record_symbols.restype = ctypes.c_int64
    _lib = lib
    return lib


def _ldtype(lb: int):
    return np.uint64 if lb == 8 else np.uint32


def downsample(brick: np.ndarray, lod: int) -> np.ndarray:
    """LOD `lod` of a b^3 brick by the recursive mode-of-8 rule (ties -> smallest label)."""
    b = brick.shape[0]
    assert brick.shape == (b, b, b) and b & (b - 1) == 0
    L = b.bit_length() - 1
    lb = brick.dtype.itemsize
    brick = np.ascontiguousarray(brick)
    S = b >> lod
    out = np.empty((S, S, S), dtype=brick.dtype)
    if _load().oracle_downsample(brick.ctypes.data, lb, L, lod, out.ctypes.data) != 0:
        raise ValueError("bad downsample arguments")
    return out


def delta_entries(delta: int) -> list[int]:
    buf = (ctypes.c_uint8 * 16)()
    n = _load().oracle_delta_entries(delta, buf)
    return list(buf[:n])


def make_freq(counts) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(counts, dtype=np.uint64))
    f = np.zeros(16, dtype=np.uint16)
    _load().oracle_make_freq(c.ctypes.data, f.ctypes.data)
    return f


def rans_encode(sym: np.ndarray, freq: np.ndarray, log2W: int):
    sym = np.ascontiguousarray(sym, dtype=np.uint8)
    freq = np.ascontiguousarray(freq, dtype=np.uint16)
    W = 1 << log2W
    G = (W + 63) // 64
    states = np.zeros(W, dtype=np.uint32)
    gw = np.zeros(G, dtype=np.uint32)
    cap = len(sym) + 64 * G + 16
    words = np.zeros(cap, dtype=np.uint16)
    n = _load().oracle_rans_encode(sym.ctypes.data, len(sym), freq.ctypes.data, log2W, states.ctypes.data,
                                   gw.ctypes.data, words.ctypes.data, cap)
    return states, gw, words[:n].copy()


def rans_decode(n: int, freq, log2W: int, states, gw, words):
    out = np.zeros(max(n, 1), dtype=np.uint8)
    freq = np.ascontiguousarray(freq, dtype=np.uint16)
    states = np.ascontiguousarray(states, dtype=np.uint32)
    gw = np.ascontiguousarray(gw, dtype=np.uint32)
    words = np.ascontiguousarray(words, dtype=np.uint16)
    if len(words) == 0:
        words = np.zeros(1, dtype=np.uint16)
    rc = _load().oracle_rans_decode(out.ctypes.data, n, freq.ctypes.data, log2W, states.ctypes.data, gw.ctypes.data,
                                    words.ctypes.data)
    return rc, out[:n]


def _bricks_of_volume(vol: np.ndarray, log2b: int) -> np.ndarray:
    """Reorder a [z,y,x] volume into concatenated b^3 bricks (brick id = bx + nbx*(by + nby*bz))."""
    b = 1 << log2b
    nz, ny, nx = vol.shape
    assert nx % b == 0 and ny % b == 0 and nz % b == 0
    v = vol.reshape(nz // b, b, ny // b, b, nx // b, b)
    return np.ascontiguousarray(v.transpose(0, 2, 4, 1, 3, 5)).reshape(-1)


def encode_bricks(bricks: np.ndarray, log2bs, label_bytes: int, dims=(0, 0, 0), default_log2b: int = 5,
                  grid=None, origins=None, op_mask: int = ALL_OPS, neighbor_mode: int = 0, coder: int = 0,
                  lane_syms: int = 64, nthreads: int | None = None) -> bytes:
    """Encode concatenated bricks (flat array, brick k of (2^log2bs[k])^3 labels, x fastest)."""
    lib = _load()
    bricks = np.ascontiguousarray(bricks, dtype=_ldtype(label_bytes))
    l2 = np.ascontiguousarray(np.asarray(log2bs, dtype=np.uint8))
    dims_a = np.ascontiguousarray(np.asarray(dims, dtype=np.uint32))
    grid_a = None if grid is None else np.ascontiguousarray(np.asarray(grid, dtype=np.uint32))
    org_a = None if origins is None else np.ascontiguousarray(np.asarray(origins, dtype=np.uint32).reshape(-1))
    out = ctypes.c_void_p()
    nbytes = ctypes.c_uint64()
    nt = nthreads if nthreads is not None else min(16, os.cpu_count() or 1)
    rc = lib.oracle_encode_volume(bricks.ctypes.data, l2.ctypes.data, len(l2), label_bytes, dims_a.ctypes.data,
                                  default_log2b, None if grid_a is None else grid_a.ctypes.data,
                                  None if org_a is None else org_a.ctypes.data, op_mask, neighbor_mode, coder,
                                  lane_syms, nt, ctypes.byref(out), ctypes.byref(nbytes))
    if rc != 0:
        raise ValueError("oracle encode failed")
    data = ctypes.string_at(out.value, nbytes.value)
    lib.oracle_free(out)
    return data


def encode_volume(vol: np.ndarray, log2b: int = 5, **kw) -> bytes:
    """Encode a [z,y,x] label volume (u32 or u64) with a regular brick grid."""
    b = 1 << log2b
    nz, ny, nx = vol.shape
    grid = (nx // b, ny // b, nz // b)
    flat = _bricks_of_volume(vol, log2b)
    n = grid[0] * grid[1] * grid[2]
    return encode_bricks(flat, [log2b] * n, vol.dtype.itemsize, dims=(nx, ny, nz), default_log2b=log2b,
                         grid=grid, **kw)


def decode_tasks(container: bytes, ids, lods, out_offsets, out_cap: int, label_bytes: int,
                 nthreads: int = 1, out: np.ndarray | None = None):
    """Decode tasks (brick id, LOD, element offset) into a flat label array; returns (out, status)."""
    lib = _load()
    ids = np.ascontiguousarray(np.asarray(ids, dtype=np.uint32))
    lods = np.ascontiguousarray(np.asarray(lods, dtype=np.uint8))
    offs = np.ascontiguousarray(np.asarray(out_offsets, dtype=np.uint64))
    if out is None:
        out = np.full(max(out_cap, 1), 0xA5A5A5A5, dtype=_ldtype(label_bytes))
    status = np.zeros(max(len(ids), 1), dtype=np.uint32)
    buf = np.frombuffer(container, dtype=np.uint8)
    rc = lib.oracle_decode_tasks(buf.ctypes.data, len(container), ids.ctypes.data, lods.ctypes.data, offs.ctypes.data,
                                 len(ids), out.ctypes.data, out_cap, status.ctypes.data, nthreads)
    if rc != 0:
        raise ValueError("unusable container header")
    return out, status[:len(ids)]


def pack_indices(idx, bits: int) -> np.ndarray:
    """Palette indices packed floor(32/bits) to a 32-bit word (cache paletting)."""
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.uint32))
    e = 32 // bits
    out = np.empty(max((len(idx) + e - 1) // e, 1), dtype=np.uint32)
    _load().oracle_pack_indices(idx.ctypes.data, len(idx), bits, out.ctypes.data)
    return out[:(len(idx) + e - 1) // e]


def paletted_words(n_voxels, bits: int):
    """32-bit words one task's packed indices occupy."""
    e = 32 // bits
    return (np.asarray(n_voxels, dtype=np.int64) + e - 1) // e


def decode_tasks_paletted(container: bytes, ids, lods, word_offsets, out_words: int, bits: int,
                          nthreads: int = 1, out: np.ndarray | None = None):
    """Decode tasks to cache-paletted form (packed palette indices, bits each,
    floor(32/bits) per 32-bit word) at word offsets; returns (words, status)."""
    lib = _load()
    ids = np.ascontiguousarray(np.asarray(ids, dtype=np.uint32))
    lods = np.ascontiguousarray(np.asarray(lods, dtype=np.uint8))
    offs = np.ascontiguousarray(np.asarray(word_offsets, dtype=np.uint64))
    if out is None:
        out = np.full(max(out_words, 1), 0xA5A5A5A5, dtype=np.uint32)
    status = np.zeros(max(len(ids), 1), dtype=np.uint32)
    buf = np.frombuffer(container, dtype=np.uint8)
    rc = lib.oracle_decode_tasks_paletted(buf.ctypes.data, len(container), ids.ctypes.data, lods.ctypes.data,
                                          offs.ctypes.data, len(ids), out.ctypes.data, out_words,
                                          status.ctypes.data, bits, nthreads)
    if rc != 0:
        raise ValueError("unusable container header or bits")
    return out, status[:len(ids)]


def record_palette(container: bytes, brick_id: int) -> np.ndarray:
    """Palette entries of one record (u64 values of the volume's label width)."""
    buf = np.frombuffer(container, dtype=np.uint8)
    out = np.zeros(1 << 18, dtype=np.uint64)
    n = _load().oracle_record_palette(buf.ctypes.data, len(container), brick_id, out.ctypes.data, len(out))
    if n < 0:
        raise ValueError("unreadable record")
    return out[:n].copy()


def record_symbols(container: bytes, brick_id: int):
    """(symbols, sym_end, info) of one record; info = coder, log2b, label_bytes, log2W, pc, extent."""
    lib = _load()
    buf = np.frombuffer(container, dtype=np.uint8)
    cap = 8 * 299593 + 16
    sym = np.zeros(cap, dtype=np.uint8)
    se = np.zeros(7, dtype=np.uint32)
    info = np.zeros(6, dtype=np.uint32)
    n = lib.oracle_record_symbols(buf.ctypes.data, len(container), brick_id, sym.ctypes.data, cap, se.ctypes.data,
                                  info.ctypes.data)
    if n < 0:
        raise ValueError("unreadable record")
    L = int(info[1])
    return sym[:n].copy(), se[:L + 1].copy(), info


def header(container: bytes) -> dict:
    """Fields of the volume container header."""
    h = np.frombuffer(container[:128], dtype=np.uint8)
    u32 = h[:48].view(np.uint32)
    return {
        "magic": int(u32[0]), "version": int(u32[1]), "dims": tuple(int(x) for x in u32[2:5]),
        "log2b": int(u32[5]), "label_bytes": int(u32[6]), "op_mask": int(u32[7]), "n_bricks": int(u32[8]),
        "grid": tuple(int(x) for x in u32[9:12]),
        "freq": h[48:80].view(np.uint16).copy(),
        "offsets_pos": int(h[80:88].view(np.uint64)[0]), "dir_pos": int(h[88:96].view(np.uint64)[0]),
        "total_bytes": int(h[96:104].view(np.uint64)[0]),
    }


def brick_offsets(container: bytes) -> np.ndarray:
    h = header(container)
    return np.frombuffer(container, dtype=np.uint64, count=h["n_bricks"] + 1, offset=h["offsets_pos"]).copy()


def dense_offsets(log2bs, lods) -> tuple[np.ndarray, int]:
    """Element offsets that pack the tasks' outputs back to back, and the total."""
    sizes = np.array([(1 << (int(l2) - int(ld))) ** 3 for l2, ld in zip(log2bs, lods)], dtype=np.uint64)
    offs = np.zeros(len(sizes), dtype=np.uint64)
    if len(sizes) > 1:
        offs[1:] = np.cumsum(sizes)[:-1]
    return offs, int(sizes.sum())
