// CSGV brick decoder for gfx950 (MI355X).
//
// One work-group decodes one task = (brick id, LOD, output offset): it
// rebuilds the brick's multi-resolution levels coarse to fine and writes the
// level of the requested LOD as a cube of labels, linear with x fastest
// (paper: Results > "CSGV" for the encoding -- one operation per node of a
// multi-resolution grid, copy from parent / neighbour / palette, stop bits for
// all-constant children; Methods > "GPU rendering pipeline" for the decode
// stage; Methods > "Memory management" for LODs).
//
// Per level i (side 2^i, nodes in Morton order):
//   1. compaction of the parents that expand (explicit, stop bit clear) into a
//      list; children of every other parent are filled with the parent's value
//      (the 8 children of a parent are contiguous in Morton order, so one
//      16-byte LDS store);
//   2. the level's symbol segment [sym_end[i-1], sym_end[i]) is processed in
//      chunks of 16 symbols per thread: a block-wide scan over 2-state
//      automata separates operations from the 4-bit delta entries that follow
//      PALETTE_DELTA (Methods > "Compressed segmentation volumes"), a second
//      scan counts operations and PALETTE_ADV operations, and every operation
//      is written to its node: the k-th operation of the level belongs to
//      child k & 7 of the (k >> 3)-th expanding parent;
//   3. neighbour references are resolved by pointer chasing: a node's slot holds
//      either a final palette index (top bit set) or the index of the node it
//      copies from; targets always precede their source in Morton order and
//      every slot changes at most once (reference -> final), so concurrent
//      chasing without barriers is safe and terminates.
// Levels live in LDS as 16-bit slots for bricks up to 32^3 whose palette
// indices fit 15 bits; 64^3 bricks (and 32^3 bricks with larger palettes)
// keep their level grids in a per-work-group global scratch area with 32-bit
// slots.  rANS-coded streams are first decoded into symbol bytes in the same
// scratch area: each 64-lane group of the interleaved coder is one wavefront,
// and the lanes that renormalise in a round find their word offsets with a
// ballot and a masked bit count.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "csgv_format.h"
#include "decode_kernel.h"

// Phase markers: empty unless a build defines CSGV_PHASE (timing probes).
#ifndef CSGV_PHASE
#define CSGV_PHASE(k) ((void)0)
#endif

namespace csgv {

// ------------------------------------------------------------------ limits
constexpr int kLdsMaxL = 5;                // levels held in LDS: up to side 32
constexpr uint32_t kLdsOdd = 1u << 15;     // slots for levels 1, 3, 5
constexpr uint32_t kLdsEven = 1u << 12;    // slots for levels 0, 2, 4
constexpr uint32_t kListMax = 1u << 15;    // expanding parents (level 5 of a 64^3 brick)
constexpr uint32_t kEOddWords = 1024;      // expansion bits, level 5 (64^3) / 3 / 1
constexpr uint32_t kEEvenWords = 128;      // expansion bits, level 4 / 2 / 0
constexpr uint32_t kPalLdsBytes = 8192;    // palette staging

// ------------------------------------------------------ wave/block helpers
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t lanemask_lt_popc(uint64_t mask) {
    // number of set bits of mask below this lane
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

struct Shared;

// Morton helpers: bit k of x/y/z goes to bit 3k / 3k+1 / 3k+2
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// ------------------------------------------------------------ LDS layout
struct Shared {
    uint16_t gOdd[kLdsOdd];
    uint16_t gEven[kLdsEven];
    uint16_t list[kListMax / 8 > 4096 ? 4096 : kListMax / 8];  // LDS path: <= 4096 parents
    uint32_t eOdd[kEOddWords];
    uint32_t eEven[kEEvenWords];
    uint32_t wpre[kEOddWords];  // exclusive prefix of expansion-bit popcounts per word
    uint32_t rans_tab[kRansM];  // slot -> symbol | freq << 4 | (slot - cum) << 17
    uint64_t pal[kPalLdsBytes / 8];
    uint32_t scan[64];
    uint32_t scan2[64];
    // task header
    uint32_t task, status, write_ok, coder, L, lb, log2W, pc, t, big, pal_lds, err;
    uint32_t sym_end[8];
    uint32_t gw[4], gstart[4];
    uint64_t out_off, rec, pal_off, pay_off, pay_bytes, states_off;
    // level carries
    uint32_t adv_total, carry_state, carry_ops, carry_adv, slow;
};

// ------------------------------------------------------------- block scans
// Exclusive sum over the block; returns this thread's prefix, *total = sum.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_sum(uint32_t v, uint32_t* total, uint32_t* scratch) {
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(incl, d, 64);
        if (lane >= (uint32_t)d) incl += o;
    }
    if (lane == 63) scratch[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int w = 0; w < NT / 64; ++w) {
            uint32_t t = scratch[w];
            scratch[w] = acc;
            acc += t;
        }
        scratch[NT / 64] = acc;
    }
    __syncthreads();
    uint32_t r = scratch[wave] + incl - v;
    *total = scratch[NT / 64];
    __syncthreads();
    return r;
}

// 2-state transfer functions: bit0 = exit state for entry 0, bit1 = for entry 1.
__device__ __forceinline__ uint32_t fn_then(uint32_t first, uint32_t second) {
    uint32_t r0 = (second >> (first & 1u)) & 1u, r1 = (second >> ((first >> 1) & 1u)) & 1u;
    return r0 | (r1 << 1);
}

// entry state of this thread given the block's entry state `carry`
template <int NT>
__device__ __forceinline__ uint32_t block_entry_state(uint32_t f, uint32_t carry, uint32_t* scratch) {
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    uint32_t incl = f;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(incl, d, 64);
        if (lane >= (uint32_t)d) incl = fn_then(o, incl);
    }
    uint32_t excl = __shfl_up(incl, 1, 64);
    if (lane == 0) excl = 2u;  // identity
    if (lane == 63) scratch[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t st = carry;
        for (int w = 0; w < NT / 64; ++w) {
            uint32_t t = scratch[w];
            scratch[w] = st;
            st = (t >> st) & 1u;
        }
    }
    __syncthreads();
    uint32_t e = (excl >> scratch[wave]) & 1u;
    __syncthreads();
    return e;
}

// ---------------------------------------------------------- symbol access
struct SymSrc {
    const uint32_t* raw;   // RAW4 payload (dword aligned) or nullptr
    uint32_t raw_dwords;
    const uint8_t* bytes;  // decoded rANS symbols, one per byte
};

__device__ __forceinline__ uint32_t raw_dword(const SymSrc& s, uint32_t d) { return d < s.raw_dwords ? s.raw[d] : 0u; }

// symbols j0 .. j0+15 as 16 nibbles (nibble q = symbol j0 + q)
__device__ __forceinline__ uint64_t load16(const SymSrc& s, uint32_t j0) {
    if (s.raw) {
        uint32_t d = j0 >> 3, sh = 4u * (j0 & 7u);
        uint64_t lo = (uint64_t)raw_dword(s, d) | ((uint64_t)raw_dword(s, d + 1) << 32);
        uint64_t hi = raw_dword(s, d + 2);
        return sh ? ((lo >> sh) | (hi << (64 - sh))) : lo;
    }
    const uint32_t* w = (const uint32_t*)(s.bytes + (j0 & ~3u));
    uint32_t sh = 8u * (j0 & 3u);
    uint64_t r = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint64_t a = w[k], b = w[k + 1];
        uint32_t v = (uint32_t)(sh ? ((a >> sh) | (b << (32 - sh))) : a);
        uint32_t n = (v & 0xFu) | ((v >> 4) & 0xF0u) | ((v >> 8) & 0xF00u) | ((v >> 12) & 0xF000u);
        r |= (uint64_t)n << (16 * k);
    }
    return r;
}

__device__ __forceinline__ uint32_t sym_at(const SymSrc& s, uint32_t j) {
    if (s.raw) return (raw_dword(s, j >> 3) >> (4u * (j & 7u))) & 15u;
    return s.bytes[j];
}

// ------------------------------------------------------------- header parse
__device__ __forceinline__ uint32_t rd32(const uint8_t* p) { return *(const uint32_t*)p; }

// Thread 0: validate the task and its record (same checks and order as the
// reference decoder) and fill the task header in LDS.
__device__ void parse_task(const Params& P, uint32_t task, Shared& sh) {
    sh.status = kTaskOk;
    sh.write_ok = 0;
    sh.err = 0;
    sh.big = 0;
    uint32_t id = P.ids[task];
    uint32_t lod = P.lods[task];
    uint64_t out_off = P.out_offs[task];
    sh.out_off = out_off;
    if (id >= P.n_bricks) { sh.status = kTaskInvalid; return; }
    const uint64_t* offs = (const uint64_t*)(P.vol + P.off_pos);
    uint64_t a = offs[id], b = offs[id + 1];
    if (a > b || b > P.vol_bytes || (a & 7) || b - a < 8) { sh.status = kTaskCorrupt; return; }
    const uint8_t* rec = P.vol + a;
    uint32_t w0 = rd32(rec);
    uint32_t coder = w0 & 0xFF, L = (w0 >> 8) & 0xFF, lb = (w0 >> 16) & 0xFF, log2W = w0 >> 24;
    uint32_t pc = rd32(rec + 4);
    uint64_t extent = b - a;
    if (L < 1 || L > kMaxLog2b) { sh.status = kTaskCorrupt; return; }
    if (lod > L) { sh.status = kTaskInvalid; return; }
    uint32_t t = L - lod;
    uint64_t S = 1ull << t, n_out = S * S * S;
    if (out_off > P.out_cap || n_out > P.out_cap - out_off) { sh.status = kTaskInvalid; return; }
    sh.write_ok = 1;
    sh.L = L;
    sh.t = t;
    sh.lb = P.label_bytes;
    if (lb != P.label_bytes || coder > 1 || (coder == kRaw4 && log2W != 0) || (coder == kRans && log2W > 8)) {
        sh.status = kTaskCorrupt;
        return;
    }
    uint64_t hdr = record_header_bytes(L, coder, log2W);
    if (hdr > extent) { sh.status = kTaskCorrupt; return; }
    uint64_t al = lb == 8 ? 8 : 4;
    uint64_t pal_rel = (hdr + al - 1) / al * al;
    if (pal_rel > extent || (uint64_t)pc * lb > extent - pal_rel) { sh.status = kTaskCorrupt; return; }
    uint64_t pay_rel = pal_rel + (uint64_t)pc * lb;
    uint64_t pay_bytes = extent - pay_rel;
    uint32_t prev = 0;
    for (uint32_t i = 0; i <= L; ++i) {
        uint32_t e = rd32(rec + 8 + 4 * i);
        sh.sym_end[i] = e;
        if (i > 0 && e < prev) { sh.status = kTaskCorrupt; return; }
        prev = e;
    }
    if ((uint64_t)prev > 8 * total_nodes(L)) { sh.status = kTaskCorrupt; return; }
    if (coder == kRaw4) {
        if ((uint64_t)prev > 2 * pay_bytes) { sh.status = kTaskCorrupt; return; }
    } else {
        uint32_t W = 1u << log2W, G = (W + 63) / 64;
        uint64_t tw = 0;
        for (uint32_t g = 0; g < G; ++g) {
            uint32_t c = rd32(rec + 8 + 4 * (L + 1) + 4 * g);
            sh.gw[g] = c;
            sh.gstart[g] = (uint32_t)tw;
            tw += c;
        }
        if (2 * tw > pay_bytes) { sh.status = kTaskCorrupt; return; }
        if (!P.freq_ok) { sh.status = kTaskCorrupt; return; }
        sh.states_off = a + 8 + 4 * (L + 1) + 4 * G;
    }
    sh.coder = coder;
    sh.log2W = log2W;
    sh.pc = pc;
    sh.rec = a;
    sh.pal_off = a + pal_rel;
    sh.pay_off = a + pay_rel;
    sh.pay_bytes = pay_bytes;
    sh.big = (t > kLdsMaxL) || (t == kLdsMaxL && pc > 32768u);
    sh.pal_lds = (uint64_t)pc * lb <= kPalLdsBytes;
}

// ----------------------------------------------------------------- rANS
// Decode the first `nsym` symbols into sym[] (one byte each).  Wavefront w
// handles lane groups w, w + NW, ...; returns nothing, sets sh.err on
// exhausted words.
template <int NT>
__device__ void rans_decode(const Params& P, Shared& sh, uint32_t nsym, uint8_t* sym) {
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    const uint32_t W = 1u << sh.log2W, G = (W + 63) / 64, lanes = W < 64 ? W : 64;
    const uint16_t* words = (const uint16_t*)(P.vol + sh.pay_off);
    const uint32_t* states = (const uint32_t*)(P.vol + sh.states_off);
    for (uint32_t g = wave; g < G; g += NT / 64) {
        const bool active = lane < lanes;
        const uint32_t gl = 64 * g + lane;
        const uint32_t gcount = sh.gw[g], gbase = sh.gstart[g];
        uint32_t x = active ? states[gl] : 0u;
        // word window: win0 holds words [wbase, wbase+64), win1 the next 64
        uint32_t wbase = 0;
        uint32_t win0 = lane < gcount ? words[gbase + lane] : 0u;
        uint32_t win1 = 64 + lane < gcount ? words[gbase + 64 + lane] : 0u;
        uint32_t gpos = 0;
        bool bad = false;
        for (uint32_t r0 = 64 * g; r0 < nsym; r0 += W) {
            const uint32_t j = r0 + lane;
            const bool act = active && j < nsym;
            uint32_t s = 0;
            if (act) {
                uint32_t e = sh.rans_tab[x & (kRansM - 1)];
                s = e & 15u;
                x = ((e >> 4) & 0x1FFFu) * (x >> kRansBits) + (e >> 17);
            }
            const bool need = act && x < kRansL;
            const uint64_t m = __ballot(need);
            const uint32_t widx = gpos + lanemask_lt_popc(m);
            const uint32_t rel = widx - wbase;
            const uint32_t w0 = __shfl(win0, rel & 63, 64), w1 = __shfl(win1, rel & 63, 64);
            if (need) {
                if (widx >= gcount) bad = true;
                x = (x << 16) | (rel < 64 ? w0 : w1);
            }
            gpos += (uint32_t)__popcll(m);
            if (act) sym[j] = (uint8_t)s;
            if (gpos - wbase >= 64) {
                wbase += 64;
                win0 = win1;
                uint32_t p = wbase + 64 + lane;
                win1 = p < gcount ? words[gbase + p] : 0u;
            }
        }
        if (__ballot(bad)) {
            if (lane == 0) atomicOr(&sh.err, 1u);
        }
    }
}

// ------------------------------------------------------------ level decode
template <typename V>
struct Slot {
    static constexpr V kFinal = (V)(V(1) << (sizeof(V) * 8 - 1));
    static constexpr V kIdx = (V)(kFinal - 1);
};

__device__ __forceinline__ void fill8(uint16_t* p, uint16_t v) {
    uint32_t w = (uint32_t)v | ((uint32_t)v << 16);
    *(uint4*)p = make_uint4(w, w, w, w);
}
__device__ __forceinline__ void fill8(uint32_t* p, uint32_t v) {
    ((uint4*)p)[0] = make_uint4(v, v, v, v);
    ((uint4*)p)[1] = make_uint4(v, v, v, v);
}

// Resolve neighbour references of a level (all nodes final afterwards).
template <int NT, typename V>
__device__ __forceinline__ void resolve_level(V* cur, uint32_t nodes, Shared& sh) {
    for (uint32_t p = threadIdx.x; p < nodes; p += NT) {
        V v = cur[p];
        if (!(v & Slot<V>::kFinal)) {
            uint32_t it = 0;
            while (!(v & Slot<V>::kFinal) && it < nodes) {
                v = cur[v];
                ++it;
            }
            if (!(v & Slot<V>::kFinal)) {
                atomicOr(&sh.err, 1u);
                v = Slot<V>::kFinal;
            }
            cur[p] = v;
        }
    }
}

// Decode levels 0..t.  gOdd/gEven: slot arrays for odd/even levels; list:
// expanding parents of the previous level.  On return the slots of level t
// are final unless sh.err is set.
template <int NT, typename V>
__device__ void decode_levels(const SymSrc& src, Shared& sh, V* gOdd, V* gEven, uint16_t* list) {
    const uint32_t tid = threadIdx.x;
    const uint32_t t = sh.t;
    uint32_t expected = 1;
    for (uint32_t i = 0; i <= t; ++i) {
        V* cur = (i & 1) ? gOdd : gEven;
        V* prev = (i & 1) ? gEven : gOdd;
        uint32_t* Ecur = (i & 1) ? sh.eOdd : sh.eEven;
        uint32_t* Eprev = (i & 1) ? sh.eEven : sh.eOdd;
        const uint32_t nodes = 1u << (3 * i);
        const uint32_t mx = 0x09249249u & (nodes - 1u), my = mx << 1, mz = mx << 2;
        if (i < t)
            for (uint32_t w = tid; w < (nodes + 31) / 32; w += NT) Ecur[w] = 0;
        if (i > 0) {
            // compaction of expanding parents + fill of implied children
            const uint32_t pn = nodes >> 3, pw = (pn + 31) / 32;
            uint32_t total = 0, base = 0;
            for (uint32_t w0 = 0; w0 < pw; w0 += NT) {
                uint32_t w = w0 + tid;
                uint32_t bits = w < pw ? Eprev[w] : 0u;
                if (pn < 32) bits &= (1u << pn) - 1u;
                uint32_t tot;
                uint32_t pre = block_excl_sum<NT>((uint32_t)__popc(bits), &tot, sh.scan);
                if (w < pw) sh.wpre[w] = base + pre;
                base += tot;
            }
            total = base;
            __syncthreads();
            for (uint32_t q = tid; q < pn; q += NT) {
                uint32_t bits = Eprev[q >> 5];
                if ((bits >> (q & 31)) & 1u) {
                    list[sh.wpre[q >> 5] + __popc(bits & ((1u << (q & 31)) - 1u))] = (uint16_t)q;
                } else {
                    fill8(cur + 8 * q, prev[q]);
                }
            }
            expected = 8 * total;
        }
        __syncthreads();
        CSGV_PHASE(3 + 3 * i);
        // ------------------------------------------------ symbol chunks
        const uint32_t seg0 = i ? sh.sym_end[i - 1] : 0u, seg1 = sh.sym_end[i];
        uint32_t carry_state = 0, ops_done = 0, adv_done = sh.adv_total;
        for (uint32_t c = seg0; c < seg1; c += NT * 16) {
            const uint32_t j0 = c + 16 * tid;
            const uint32_t nv = j0 < seg1 ? (seg1 - j0 < 16 ? seg1 - j0 : 16) : 0;
            uint64_t nib = nv ? load16(src, j0) : 0ull;
            const uint64_t vmask = nv == 16 ? ~0ull : ((1ull << (4 * nv)) - 1ull);
            nib &= vmask;
            const uint64_t lowbits = 0x1111111111111111ull & vmask;
            // positions whose low 3 bits are 110b: a PALETTE_DELTA op if read in op state
            const uint64_t cand = (nib >> 2) & (nib >> 1) & ~nib & lowbits;
            const bool slow = __syncthreads_or(cand != 0) || carry_state != 0;
            uint32_t entry = 0;
            if (slow) {
                uint32_t f = 0;
#pragma unroll
                for (uint32_t e = 0; e < 2; ++e) {
                    uint32_t st = e;
                    for (uint32_t q = 0; q < nv; ++q) {
                        uint32_t s = (uint32_t)(nib >> (4 * q)) & 15u;
                        st = st ? (s >> 3) : ((s & 7u) == kDelta);
                    }
                    f |= st << e;
                }
                if (nv == 0) f = 2u;
                entry = block_entry_state<NT>(f, carry_state, sh.scan);
            }
            // operations of this thread's symbols given its entry state
            uint32_t opmask, nops, nadv, exit_state;
            if (!slow) {
                opmask = nv == 16 ? 0xFFFFu : ((1u << nv) - 1u);
                nops = nv;
                const uint64_t adv = (nib >> 2) & ~(nib >> 1) & ~nib & lowbits;  // op == 100b
                nadv = (uint32_t)__popcll(adv);
                exit_state = 0;
            } else {
                uint32_t st = entry;
                opmask = 0;
                nops = 0;
                nadv = 0;
                for (uint32_t q = 0; q < nv; ++q) {
                    uint32_t s = (uint32_t)(nib >> (4 * q)) & 15u;
                    if (!st) {
                        opmask |= 1u << q;
                        ++nops;
                        nadv += (s & 7u) == kAdv;
                        st = (s & 7u) == kDelta;
                    } else {
                        st = s >> 3;
                    }
                }
                exit_state = st;
            }
            uint32_t tot;
            const uint32_t pre = block_excl_sum<NT>(nops | (nadv << 16), &tot, sh.scan);
            uint32_t k = ops_done + (pre & 0xFFFFu);
            uint32_t a = adv_done + (pre >> 16);
            // emit operations
            uint32_t m = opmask;
            bool bad = false;
            while (m) {
                const uint32_t q = __builtin_ctz(m);
                m &= m - 1;
                const uint32_t s = (uint32_t)(nib >> (4 * q)) & 15u, op = s & 7u, stop = s >> 3;
                if (k >= expected) { bad = true; break; }
                const uint32_t p = i ? (((uint32_t)list[k >> 3] << 3) | (k & 7u)) : 0u;
                V v = Slot<V>::kFinal;
                switch (op) {
                case kParent:
                    if (i == 0) bad = true;
                    else v = prev[p >> 3];
                    break;
                case kNX:
                    if (!(p & mx)) bad = true;
                    else v = (V)((((p & mx) - 1u) & mx) | (p & ~mx));
                    break;
                case kNY:
                    if (!(p & my)) bad = true;
                    else v = (V)((((p & my) - 1u) & my) | (p & ~my));
                    break;
                case kNZ:
                    if (!(p & mz)) bad = true;
                    else v = (V)((((p & mz) - 1u) & mz) | (p & ~mz));
                    break;
                case kAdv:
                    if (a >= sh.pc) bad = true;
                    else v = (V)(Slot<V>::kFinal | a);
                    ++a;
                    break;
                case kLast:
                    if (a == 0) bad = true;
                    else v = (V)(Slot<V>::kFinal | (a - 1));
                    break;
                case kDelta: {
                    uint32_t d = 0, jj = j0 + q + 1, e = 8;
                    while (e & 8u) {
                        if (jj >= seg1) { bad = true; break; }
                        e = (jj < j0 + nv) ? (uint32_t)(nib >> (4 * (jj - j0))) & 15u : sym_at(src, jj);
                        d = d >= (1u << 29) ? 0xFFFFFFFFu : ((d << 3) | (e & 7u));
                        ++jj;
                    }
                    if (d == 0 || d > a) bad = true;
                    else v = (V)(Slot<V>::kFinal | (a - d));
                    break;
                }
                default:
                    bad = true;
                }
                cur[p] = v;
                if (i < t && !stop) atomicOr(&Ecur[p >> 5], 1u << (p & 31));
                ++k;
            }
            if (bad) atomicOr(&sh.err, 1u);
            // chunk carry: exit state of the last thread holding symbols
            const uint32_t last = (seg1 - c - 1) / 16 < (uint32_t)NT ? (seg1 - c - 1) / 16 : NT - 1;
            if (tid == last) sh.carry_state = exit_state;
            __syncthreads();
            carry_state = sh.carry_state;
            ops_done += tot & 0xFFFFu;
            adv_done += tot >> 16;
        }
        if (tid == 0) {
            if (ops_done != expected || carry_state != 0) sh.err = 1;
            sh.adv_total = adv_done;
        }
        __syncthreads();
        CSGV_PHASE(4 + 3 * i);
        if (sh.err) return;
        resolve_level<NT, V>(cur, nodes, sh);
        __syncthreads();
        CSGV_PHASE(5 + 3 * i);
        if (sh.err) return;
    }
    if (t == sh.L && sh.adv_total != sh.pc) {
        if (tid == 0) sh.err = 1;
    }
    __syncthreads();
}

// ------------------------------------------------------------------ output
template <typename V>
__device__ __forceinline__ uint64_t pal_get(const Params& P, const Shared& sh, V v) {
    const uint32_t idx = (uint32_t)(v & Slot<V>::kIdx);
    if (sh.lb == 4) {
        if (sh.pal_lds) return ((const uint32_t*)sh.pal)[idx];
        return ((const uint32_t*)(P.vol + sh.pal_off))[idx];
    }
    if (sh.pal_lds) return sh.pal[idx];
    return ((const uint64_t*)(P.vol + sh.pal_off))[idx];
}

template <int NT, typename V>
__device__ void write_output(const Params& P, const Shared& sh, const V* cur, bool zero) {
    const uint32_t t = sh.t, S = 1u << t;
    const uint64_t n_out = (uint64_t)S * S * S;
    uint8_t* out = P.out + sh.out_off * sh.lb;
    const bool vec = S >= 4 && (((uintptr_t)out & 15u) == 0);
    if (vec) {
        const uint32_t units = (uint32_t)(n_out >> 2);
        for (uint32_t u = threadIdx.x; u < units; u += NT) {
            const uint32_t lin = u << 2;
            const uint32_t x = lin & (S - 1), y = (lin >> t) & (S - 1), z = lin >> (2 * t);
            uint64_t l0 = 0, l1 = 0, l2 = 0, l3 = 0;
            if (!zero) {
                const uint32_t m = spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
                l0 = pal_get<V>(P, sh, cur[m]);
                l1 = pal_get<V>(P, sh, cur[m + 1]);
                l2 = pal_get<V>(P, sh, cur[m + 8]);
                l3 = pal_get<V>(P, sh, cur[m + 9]);
            }
            if (sh.lb == 4) {
                ((uint4*)out)[u] = make_uint4((uint32_t)l0, (uint32_t)l1, (uint32_t)l2, (uint32_t)l3);
            } else {
                uint4* o = (uint4*)out + 2 * u;
                o[0] = make_uint4((uint32_t)l0, (uint32_t)(l0 >> 32), (uint32_t)l1, (uint32_t)(l1 >> 32));
                o[1] = make_uint4((uint32_t)l2, (uint32_t)(l2 >> 32), (uint32_t)l3, (uint32_t)(l3 >> 32));
            }
        }
    } else {
        for (uint64_t lin = threadIdx.x; lin < n_out; lin += NT) {
            const uint32_t x = (uint32_t)lin & (S - 1), y = ((uint32_t)lin >> t) & (S - 1), z = (uint32_t)lin >> (2 * t);
            uint64_t l = 0;
            if (!zero) l = pal_get<V>(P, sh, cur[spread3(x) | (spread3(y) << 1) | (spread3(z) << 2)]);
            if (sh.lb == 4) ((uint32_t*)out)[lin] = (uint32_t)l;
            else ((uint64_t*)out)[lin] = l;
        }
    }
}

// ------------------------------------------------------------------ a task
template <int NT>
__device__ void decode_task(const Params& P, Shared& sh, uint8_t* scratch) {
    const uint32_t tid = threadIdx.x;
    if (sh.status != kTaskOk) {
        if (sh.status == kTaskCorrupt && sh.write_ok) write_output<NT, uint16_t>(P, sh, nullptr, true);
        return;
    }
    // palette staging
    if (sh.pal_lds) {
        const uint32_t words = (sh.pc * sh.lb + 3) / 4;
        const uint32_t* src = (const uint32_t*)(P.vol + sh.pal_off);
        for (uint32_t w = tid; w < words; w += NT) ((uint32_t*)sh.pal)[w] = src[w];
    }
    // symbol source
    SymSrc src;
    uint8_t* symbuf = scratch;
    uint8_t* bigbuf = scratch + kScratchSymBytes;
    if (sh.coder == kRaw4) {
        src.raw = (const uint32_t*)(P.vol + sh.pay_off);
        src.raw_dwords = (uint32_t)(sh.pay_bytes / 4);
        src.bytes = nullptr;
    } else {
        src.raw = nullptr;
        src.raw_dwords = 0;
        src.bytes = symbuf;
        rans_decode<NT>(P, sh, sh.sym_end[sh.t], symbuf);
    }
    __syncthreads();
    CSGV_PHASE(2);
    if (!sh.err) {
        if (!sh.big) {
            decode_levels<NT, uint16_t>(src, sh, sh.gOdd, sh.gEven, sh.list);
            if (!sh.err) {
                write_output<NT, uint16_t>(P, sh, (sh.t & 1) ? sh.gOdd : sh.gEven, false);
                CSGV_PHASE(24);
                return;
            }
        } else {
            uint32_t* gOdd = (uint32_t*)bigbuf;
            uint32_t* gEven = gOdd + kBigOddSlots;
            uint16_t* list = (uint16_t*)(gEven + kBigEvenSlots);
            decode_levels<NT, uint32_t>(src, sh, gOdd, gEven, list);
            if (!sh.err) {
                write_output<NT, uint32_t>(P, sh, (sh.t & 1) ? gOdd : gEven, false);
                return;
            }
        }
    }
    if (tid == 0) sh.status = kTaskCorrupt;
    write_output<NT, uint16_t>(P, sh, nullptr, true);
}

template <int NT>
__global__ void __launch_bounds__(NT) decode_kernel(Params P) {
    extern __shared__ uint8_t dyn_smem[];
    Shared& sh = *reinterpret_cast<Shared*>(dyn_smem);
    const uint32_t tid = threadIdx.x;
    // rANS lookup table for the volume's frequency table
    if (P.freq_ok) {
        for (uint32_t slot = tid; slot < kRansM; slot += NT) {
            uint32_t cum = 0, s = 0;
            for (uint32_t k = 0; k < 16; ++k) {
                const uint32_t f = (P.freq[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
                if (slot >= cum && slot < cum + f) { s = k; break; }
                cum += f;
            }
            const uint32_t f = (P.freq[s >> 1] >> (16 * (s & 1))) & 0xFFFFu;
            sh.rans_tab[slot] = s | (f << 4) | ((slot - cum) << 17);
        }
    }
    uint8_t* scratch = P.scratch ? P.scratch + (uint64_t)blockIdx.x * P.scratch_stride : nullptr;
    uint32_t iter = 0;
    for (;;) {
        __syncthreads();
        CSGV_PHASE(0);
        if (tid == 0) {
            uint32_t jt;
            if (P.queue) jt = atomicAdd(P.queue, 1u);
            else jt = iter == 0 ? P.task0 + blockIdx.x : P.n_tasks;
            sh.task = jt;
            if (jt < P.n_tasks) {
                const uint32_t task = P.order ? P.order[jt] : jt;
                sh.task = task;
                sh.adv_total = 0;
                parse_task(P, task, sh);
                sh.task = task;
            } else {
                sh.task = 0xFFFFFFFFu;
            }
        }
        __syncthreads();
        CSGV_PHASE(1);
        ++iter;
        const uint32_t task = sh.task;
        if (task == 0xFFFFFFFFu) break;
        decode_task<NT>(P, sh, scratch);
        __syncthreads();
        if (tid == 0 && P.status) P.status[task] = sh.status;
    }
}

// ------------------------------------------------------------ small kernels
__global__ void reset_queue_kernel(uint32_t* q) {
    if (threadIdx.x == 0) q[0] = 0;
}

// task cost classes for a decreasing-cost pop order: cls = 63 - clz(cost)
__global__ void cost_class_kernel(Params P, uint32_t* cls, uint32_t* hist) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= P.n_tasks) return;
    const uint32_t id = P.ids[j];
    uint64_t cost = 1;
    if (id < P.n_bricks) {
        const uint64_t* offs = (const uint64_t*)(P.vol + P.off_pos);
        const uint64_t a = offs[id], b = offs[id + 1];
        uint64_t rec = b > a ? b - a : 0;
        const uint32_t lod = P.lods[j];
        uint32_t L = 5;
        if (b >= a + 8 && b <= P.vol_bytes && !(a & 7)) L = P.vol[a + 1] & 7u;
        const uint32_t t = lod <= L ? L - lod : 0;
        cost = rec + (((uint64_t)1 << (3 * t)) * P.label_bytes) + 1;
    }
    const uint32_t c = 63u - (uint32_t)__clzll(cost);
    cls[j] = c;
    atomicAdd(&hist[c], 1u);
}

// exclusive scan of the 64-bin histogram in decreasing class order (one wave)
__global__ void cost_scan_kernel(uint32_t* hist, uint32_t* cursor) {
    const uint32_t lane = threadIdx.x;
    const uint32_t c = 63 - lane;  // lane 0 = most expensive class
    const uint32_t v = hist[c];
    uint32_t incl = v;
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(incl, d, 64);
        if (lane >= (uint32_t)d) incl += o;
    }
    cursor[c] = incl - v;
}

__global__ void cost_scatter_kernel(uint32_t n, const uint32_t* cls, uint32_t* cursor, uint32_t* order) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    order[atomicAdd(&cursor[cls[j]], 1u)] = j;
}

__global__ void zero_u32_kernel(uint32_t* p, uint32_t n) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) p[j] = 0;
}

// ------------------------------------------------------------ host launch
size_t shared_bytes() { return sizeof(Shared); }

template <int NT>
static hipError_t launch_nt(const Params& P, uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL(decode_kernel<NT>, dim3(grid), dim3(NT), sizeof(Shared), s, P);
    return hipGetLastError();
}

hipError_t set_kernel_attrs() {
    hipError_t e = hipFuncSetAttribute((const void*)decode_kernel<256>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)sizeof(Shared));
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)decode_kernel<512>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)sizeof(Shared));
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)decode_kernel<1024>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)sizeof(Shared));
}

hipError_t launch_decode(const Params& P, int wg_size, uint32_t grid, hipStream_t s) {
    switch (wg_size) {
    case 256: return launch_nt<256>(P, grid, s);
    case 512: return launch_nt<512>(P, grid, s);
    case 1024: return launch_nt<1024>(P, grid, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_reset(uint32_t* q, hipStream_t s) {
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, s, q);
    return hipGetLastError();
}

hipError_t launch_sort(const Params& P, uint32_t* cls, uint32_t* hist, uint32_t* order, hipStream_t s) {
    hipLaunchKernelGGL(zero_u32_kernel, dim3(2), dim3(64), 0, s, hist, 128u);
    const uint32_t blocks = (P.n_tasks + 255) / 256;
    hipLaunchKernelGGL(cost_class_kernel, dim3(blocks), dim3(256), 0, s, P, cls, hist);
    hipLaunchKernelGGL(cost_scan_kernel, dim3(1), dim3(64), 0, s, hist, hist + 64);
    hipLaunchKernelGGL(cost_scatter_kernel, dim3(blocks), dim3(256), 0, s, P.n_tasks, cls, hist + 64, order);
    return hipGetLastError();
}

}  // namespace csgv
