"""Random valid CSGV streams and a pure-Python container writer (test inputs).

TEST INFRASTRUCTURE ONLY.  The generator walks the decoder's grammar (levels
coarse to fine, Morton order, one operation per explicit node) and picks a
random *valid* operation at every node, so it emits streams that the encoder
never would: long neighbour chains, LAST/DELTA with duplicate palettes, delta
chains with leading zero entries, stop bits set on the finest level (which a
decoder must ignore).  It records the label grid of every level as it goes,
which gives a third, construction-side answer next to the two decoders.
"""
from __future__ import annotations

import struct

import numpy as np

PARENT, NX, NY, NZ, ADV, LAST, DELTA = range(7)


def morton(x: int, y: int, z: int, bits: int) -> int:
    m = 0
    for k in range(bits):
        m |= ((x >> k) & 1) << (3 * k) | ((y >> k) & 1) << (3 * k + 1) | ((z >> k) & 1) << (3 * k + 2)
    return m


def demorton(m: int, bits: int):
    x = y = z = 0
    for k in range(bits):
        x |= ((m >> (3 * k)) & 1) << k
        y |= ((m >> (3 * k + 1)) & 1) << k
        z |= ((m >> (3 * k + 2)) & 1) << k
    return x, y, z


def delta_chain(delta: int, extra_zero_groups: int = 0) -> list[int]:
    """Entries for delta: 3-bit groups MSB first, bit 3 = more follow; optional leading zero groups."""
    groups = []
    d = delta
    while True:
        groups.append(d & 7)
        d >>= 3
        if d == 0:
            break
    groups = groups[::-1]
    groups = [0] * extra_zero_groups + groups
    return [g | (8 if i + 1 < len(groups) else 0) for i, g in enumerate(groups)]


def random_stream(rng: np.random.Generator, L: int, label_bytes: int = 4, p_stop: float = 0.35,
                  weights=(3, 2, 2, 2, 2, 1, 1), n_label_pool: int | None = None, nonminimal: float = 0.1,
                  stop_at_finest: float = 0.2):
    """A random valid stream for a 2^L brick.

    Returns (symbols, sym_end, palette, grids) where grids[i] is level i's
    label grid in Morton order (the decoded result of every LOD).
    """
    pool_hi = (1 << (8 * label_bytes)) - 1
    pool = None
    if n_label_pool is not None:
        pool = rng.integers(0, pool_hi, size=n_label_pool, dtype=np.uint64, endpoint=True)
    syms: list[int] = []
    sym_end = []
    pal: list[int] = []
    grids = []
    expand_prev = None
    for i in range(L + 1):
        n = 1 << (3 * i)
        G = [0] * n
        expand = [False] * n
        for m in range(n):
            if i > 0 and not expand_prev[m >> 3]:
                G[m] = grids[i - 1][m >> 3]
                continue
            x, y, z = demorton(m, i)
            choices = [ADV]
            if i > 0:
                choices.append(PARENT)
            if x > 0:
                choices.append(NX)
            if y > 0:
                choices.append(NY)
            if z > 0:
                choices.append(NZ)
            if pal:
                choices += [LAST, DELTA]
            w = np.array([weights[c] for c in choices], dtype=float)
            op = int(choices[rng.choice(len(choices), p=w / w.sum())])
            extra = []
            if op == PARENT:
                v = grids[i - 1][m >> 3]
            elif op == NX:
                v = G[morton(x - 1, y, z, i)]
            elif op == NY:
                v = G[morton(x, y - 1, z, i)]
            elif op == NZ:
                v = G[morton(x, y, z - 1, i)]
            elif op == ADV:
                v = int(pool[rng.integers(len(pool))]) if pool is not None else int(rng.integers(0, pool_hi, endpoint=True, dtype=np.uint64))
                pal.append(v)
            elif op == LAST:
                v = pal[-1]
            else:
                d = int(rng.integers(1, len(pal) + 1))
                v = pal[len(pal) - d]
                extra = delta_chain(d, int(rng.integers(1, 3)) if rng.random() < nonminimal else 0)
            if i < L:
                stop = rng.random() < p_stop
            else:
                stop = rng.random() < stop_at_finest  # ignored by decoders at the finest level
            syms.append(op | (8 if stop else 0))
            syms.extend(extra)
            G[m] = v
            expand[m] = not stop
        sym_end.append(len(syms))
        grids.append(G)
        expand_prev = expand
    return syms, sym_end, pal, grids


def grid_to_linear(G, level: int) -> np.ndarray:
    """Morton-ordered level grid -> [z,y,x] array."""
    s = 1 << level
    out = np.zeros((s, s, s), dtype=np.uint64)
    for m, v in enumerate(G):
        x, y, z = demorton(m, level)
        out[z, y, x] = v
    return out


# ------------------------------------------------------------- rANS (Python)
def _cum(freq):
    c = [0]
    for f in freq:
        c.append(c[-1] + int(f))
    return c


def rans_encode_py(sym, freq, log2W: int):
    """Interleaved rANS (12-bit table, 32-bit state in [2^16, 2^32), 16-bit words, lane groups of 64)."""
    W = 1 << log2W
    G = (W + 63) // 64
    cum = _cum(freq)
    x = [1 << 16] * W
    stacks = [[] for _ in range(G)]
    for j in range(len(sym) - 1, -1, -1):
        l = j % W
        s = sym[j]
        f = int(freq[s])
        if x[l] >= (f << 20):
            stacks[l // 64].append(x[l] & 0xFFFF)
            x[l] >>= 16
        x[l] = ((x[l] // f) << 12) + (x[l] % f) + cum[s]
    words = []
    gw = []
    for g in range(G):
        gw.append(len(stacks[g]))
        words.extend(stacks[g][::-1])
    return x, gw, words


def freq_from_counts(counts) -> list[int]:
    """Any valid table: every used symbol gets >= 1, sum 4096 (largest symbol absorbs the rest)."""
    counts = [int(c) for c in counts]
    tot = sum(counts)
    f = [max(1, c * 4096 // tot) if c else 0 for c in counts]
    big = max(range(16), key=lambda s: counts[s])
    f[big] += 4096 - sum(f)
    assert f[big] >= 1
    return f


# -------------------------------------------------------- container writer
def _align(v: int, a: int) -> int:
    return (v + a - 1) // a * a


def record_bytes(L: int, label_bytes: int, syms, sym_end, pal, coder: int = 0, freq=None, log2W: int = 0) -> bytes:
    hdr = bytearray(struct.pack("<BBBBI", coder, L, label_bytes, log2W if coder else 0, len(pal)))
    hdr += struct.pack("<%dI" % (L + 1), *sym_end)
    if coder == 1:
        x, gw, words = rans_encode_py(syms, freq, log2W)
        hdr += struct.pack("<%dI" % len(gw), *gw)
        hdr += struct.pack("<%dI" % len(x), *x)
        payload = struct.pack("<%dH" % len(words), *words)
    else:
        pb = bytearray((len(syms) + 1) // 2)
        for j, s in enumerate(syms):
            pb[j // 2] |= (s & 15) << (4 * (j & 1))
        payload = bytes(pb)
    rec = bytes(hdr)
    rec += b"\0" * (_align(len(rec), 8 if label_bytes == 8 else 4) - len(rec))
    fmt = "<Q" if label_bytes == 8 else "<I"
    for v in pal:
        rec += struct.pack(fmt, int(v))
    rec += payload
    rec += b"\0" * (_align(len(rec), 8) - len(rec))
    return rec


def container(records, label_bytes: int, freq=None, dims=(0, 0, 0), log2b: int = 5) -> bytes:
    """Volume container around already-built records."""
    n = len(records)
    freq = list(freq) if freq is not None else [0] * 16
    off_pos = 128
    rec0 = _align(off_pos + 8 * (n + 1), 8)
    offs = []
    pos = rec0
    for r in records:
        offs.append(pos)
        pos += len(r)
    offs.append(pos)
    h = bytearray(128)
    struct.pack_into("<IIIIIIIII", h, 0, 0x56475343, 1, dims[0], dims[1], dims[2], log2b, label_bytes, 63, n)
    struct.pack_into("<16H", h, 48, *freq)
    struct.pack_into("<QQQ", h, 80, off_pos, 0, pos)
    body = bytes(h) + struct.pack("<%dQ" % (n + 1), *offs)
    body += b"\0" * (rec0 - len(body))
    return body + b"".join(records)
