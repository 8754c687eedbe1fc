"""An independent pure-Python CSGV decoder for tiny bricks.

It re-reads the byte layout and the decoding rules from scratch (no code in
common with the C oracle) so that the two can be checked against each other
on random and corrupted streams.  Slow: meant for bricks up to 8^3.

Rules (paper, Results > "CSGV" and the supplementary operation list; Methods >
"Compressed segmentation volumes" for the delta chain): levels are decoded
coarse to fine, nodes in Morton order; a node is explicit when it is the root
or its parent was explicit with a clear stop bit; explicit nodes copy from the
parent, from the -x/-y/-z neighbour on their level, or from the palette
(next entry, the last entry, or delta entries back).
"""
from __future__ import annotations

import struct


class Corrupt(Exception):
    pass


def _bits3(v: int, bits: int, axis: int) -> int:
    out = 0
    for k in range(bits):
        out |= ((v >> k) & 1) << (3 * k + axis)
    return out


def _coord(m: int, bits: int, axis: int) -> int:
    out = 0
    for k in range(bits):
        out |= ((m >> (3 * k + axis)) & 1) << k
    return out


def _node(x: int, y: int, z: int, bits: int) -> int:
    return _bits3(x, bits, 0) | _bits3(y, bits, 1) | _bits3(z, bits, 2)


def _symbols(rec: bytes, coder: int, log2W: int, L: int, count: int, payload_off: int, freq):
    if coder == 0:
        out = []
        for j in range(count):
            byte = rec[payload_off + j // 2]
            out.append((byte >> 4) if (j % 2) else (byte & 15))
        return out
    W = 1 << log2W
    ngroups = (W + 63) // 64
    base = 8 + 4 * (L + 1)
    gw = list(struct.unpack_from("<%dI" % ngroups, rec, base))
    states = list(struct.unpack_from("<%dI" % W, rec, base + 4 * ngroups))
    starts = []
    acc = 0
    for g in gw:
        starts.append(acc)
        acc += g
    used = [0] * ngroups
    cum = [0]
    for f in freq:
        cum.append(cum[-1] + f)
    out = []
    for j in range(count):
        lane = j % W
        grp = lane // 64
        x = states[lane]
        slot = x % 4096
        s = next(k for k in range(16) if cum[k] <= slot < cum[k + 1])
        x = freq[s] * (x >> 12) + slot - cum[s]
        if x < 65536:
            if used[grp] >= gw[grp]:
                raise Corrupt("rANS words exhausted")
            (w,) = struct.unpack_from("<H", rec, payload_off + 2 * (starts[grp] + used[grp]))
            used[grp] += 1
            x = (x << 16) | w
        states[lane] = x
        out.append(s)
    return out


def decode(container: bytes, brick: int, lod: int, out_room: int | None = None):
    """Returns ('ok', [z][y][x] nested list) or ('invalid', None) or ('corrupt', None).

    out_room: output elements available to the task (None = unlimited).
    """
    magic, version = struct.unpack_from("<II", container, 0)
    assert magic == 0x56475343 and version == 1
    (vol_lb,) = struct.unpack_from("<I", container, 24)
    (nbricks,) = struct.unpack_from("<I", container, 32)
    freq = list(struct.unpack_from("<16H", container, 48))
    (offpos,) = struct.unpack_from("<Q", container, 80)
    if brick >= nbricks:
        return "invalid", None
    start, end = struct.unpack_from("<QQ", container, offpos + 8 * brick)
    if start > end or end > len(container) or start % 8 or end - start < 8:
        return "corrupt", None
    rec = container[start:end]
    coder, L, lb, log2W, pc = struct.unpack_from("<BBBBI", rec, 0)
    if not 1 <= L <= 6:
        return "corrupt", None
    if lod > L:
        return "invalid", None
    if out_room is not None and (1 << (L - lod)) ** 3 > out_room:
        return "invalid", None
    try:
        t = L - lod
        if lb != vol_lb or coder not in (0, 1) or (coder == 0 and log2W) or (coder == 1 and log2W > 8):
            raise Corrupt("record header")
        hdr = 8 + 4 * (L + 1)
        if coder == 1:
            W = 1 << log2W
            hdr += 4 * ((W + 63) // 64) + 4 * W
        if hdr > len(rec):
            raise Corrupt("header past record")
        pal_off = -(-hdr // (8 if lb == 8 else 4)) * (8 if lb == 8 else 4)
        if pal_off + pc * lb > len(rec):
            raise Corrupt("palette past record")
        fmt = "<Q" if lb == 8 else "<I"
        palette = [struct.unpack_from(fmt, rec, pal_off + lb * k)[0] for k in range(pc)]
        payload_off = pal_off + pc * lb
        payload_len = len(rec) - payload_off
        ends = list(struct.unpack_from("<%dI" % (L + 1), rec, 8))
        if any(ends[i] < ends[i - 1] for i in range(1, L + 1)):
            raise Corrupt("sym_end order")
        if ends[L] > 8 * sum(8 ** i for i in range(L + 1)):
            raise Corrupt("too many symbols")
        if coder == 0 and ends[L] > 2 * payload_len:
            raise Corrupt("raw payload short")
        if coder == 1:
            W = 1 << log2W
            ng = (W + 63) // 64
            if 2 * sum(struct.unpack_from("<%dI" % ng, rec, 8 + 4 * (L + 1))) > payload_len:
                raise Corrupt("rANS payload short")
            if sum(freq) != 4096:
                raise Corrupt("bad table")
        syms = _symbols(rec, coder, log2W, L, ends[t], payload_off, freq)
        pos = 0
        nadv = 0
        prev = None      # level i-1 labels by Morton index
        prev_open = None  # level i-1: explicit and not stopped
        for level in range(t + 1):
            cur = {}
            cur_open = {}
            for m in range(8 ** level):
                if level > 0 and not prev_open[m // 8]:
                    cur[m] = prev[m // 8]
                    cur_open[m] = False
                    continue
                if pos >= ends[level]:
                    raise Corrupt("level overrun")
                s = syms[pos]
                pos += 1
                op, stop = s % 8, s // 8
                x, y, z = (_coord(m, level, a) for a in range(3))
                if op == 0:
                    if level == 0:
                        raise Corrupt("parent of root")
                    val = prev[m // 8]
                elif op in (1, 2, 3):
                    c = (x, y, z)[op - 1]
                    if c == 0:
                        raise Corrupt("neighbour outside")
                    nb = [x, y, z]
                    nb[op - 1] -= 1
                    val = cur[_node(nb[0], nb[1], nb[2], level)]
                elif op == 4:
                    if nadv >= pc:
                        raise Corrupt("palette overrun")
                    val = palette[nadv]
                    nadv += 1
                elif op == 5:
                    if nadv == 0:
                        raise Corrupt("last without palette")
                    val = palette[nadv - 1]
                elif op == 6:
                    delta = 0
                    while True:
                        if pos >= ends[level]:
                            raise Corrupt("delta overrun")
                        e = syms[pos]
                        pos += 1
                        delta = min((delta << 3) | (e & 7), 0xFFFFFFFF)
                        if not e & 8:
                            break
                    if delta == 0 or delta > nadv:
                        raise Corrupt("delta range")
                    val = palette[nadv - delta]
                else:
                    raise Corrupt("op 7")
                cur[m] = val
                cur_open[m] = not stop
            if pos != ends[level]:
                raise Corrupt("level end mismatch")
            prev, prev_open = cur, cur_open
        if t == L and nadv != pc:
            raise Corrupt("palette not consumed")
        S = 1 << t
        return "ok", [[[prev[_node(x, y, z, t)] for x in range(S)] for y in range(S)] for z in range(S)]
    except Corrupt:
        return "corrupt", None
