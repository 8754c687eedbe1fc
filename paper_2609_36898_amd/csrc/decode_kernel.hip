// CSGV brick decoder for gfx950 (MI355X).
//
// A work-group decodes one task = (brick id, LOD, output offset): it rebuilds
// the brick's multi-resolution levels coarse to fine and writes the level of
// the requested LOD as a cube of labels, linear with x fastest (paper:
// Results > "CSGV" for the encoding -- one operation per explicit node of the
// multi-resolution grid, copying from the parent, a neighbour or the palette,
// with stop bits for all-constant children; Methods > "GPU rendering
// pipeline" for the decode stage; Methods > "Memory management" for LODs).
//
// Storage of the levels of a task (node order within a level is Morton):
//   levels 0..3   full grids (585 nodes): implied nodes are filled with their
//                 parent's value when the level starts;
//   levels 4, 5   explicit nodes only, indexed by their operation rank k
//                 (the k-th operation of a level is the k-th explicit node in
//                 Morton order); an implied node is looked up through its
//                 parent: rank of an expanding parent = prefix popcount of the
//                 parent level's expansion bitmap;
//   level 6       (64^3 bricks at full resolution) explicit nodes are kept at
//                 their voxel position in the task's own output range, which
//                 the output pass then overwrites in place with labels.
// A slot holds either a final palette index (top bit set) or a reference to
// a same-level slot whose value it copies (a neighbour operation whose target
// was decoded in the same pass).  Fast path: 16-bit slots, levels 0..5 in
// LDS.  Big path (palettes above 2^15 entries or more explicit nodes than the
// LDS share holds): 32-bit slots in a per-work-group global scratch area.
//
// A level's symbol segment is consumed in passes of one symbol per thread.
// Per wavefront, ballots classify each symbol as an operation or a 4-bit
// delta entry for both possible entry states of the 2-state automaton
// (inside a delta chain or not), count operations and PALETTE_ADV operations
// (Methods > "Compressed segmentation volumes" for the delta chains); one
// barrier later every wave folds the earlier waves' summaries and knows its
// entry state, its first operation rank and its palette (ADV) rank, and every
// lane then ranks itself with mbcnt.  Neighbour targets decoded in an earlier
// pass are already final; references within a pass are resolved right after
// it by chasing, which terminates because every target precedes its source
// in Morton order.
//
// rANS-coded records are first decoded into 4-bit symbols in the work-group's
// scratch: every 64-lane group of the interleaved coder is one wavefront, and
// the lanes that renormalise in a round find their word offsets with a ballot
// and a masked bit count.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "csgv_format.h"
#include "decode_kernel.h"

namespace csgv {

// ------------------------------------------------------------------ layout
__device__ __forceinline__ uint32_t fbase(uint32_t i) { return i == 0 ? 0u : i == 1 ? 8u : i == 2 ? 16u : 80u; }
__device__ __forceinline__ uint32_t ebase(uint32_t i) { return i == 0 ? 0u : i == 1 ? 1u : i == 2 ? 2u : i == 3 ? 4u : 20u; }
__host__ __device__ constexpr uint32_t ewords(uint32_t i) { return i <= 1 ? 1u : i == 2 ? 2u : (1u << (3 * i - 5)); }

struct TaskHdr {
    uint32_t task, status, write_ok, coder, L, t, log2W, pc, big, pal_lds, c5base, nsym;
    uint32_t sym_end[7];
    uint32_t gw[4], gstart[4];
    uint64_t out_off, pal_off, pay_off, states_off;
};

struct Shared {
    TaskHdr h;
    uint32_t err;
    uint32_t pub[2][kMaxWaves];
    uint32_t red[kMaxWaves + 2];
    uint32_t E[kEWords];       // expansion bitmaps of levels 0..4
    uint16_t wpre[kEWords];    // exclusive popcount prefix of each bitmap word
    alignas(16) uint16_t G[kFullSlots];  // full grids of levels 0..3 (fast path)
    alignas(16) uint8_t U[kUBytes];      // rANS table | parent list + values | palette
};
static_assert(sizeof(Shared) % 16 == 0, "compact slots follow Shared 16-byte aligned");

// ------------------------------------------------------ wave/block helpers
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t mbcnt(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__device__ __forceinline__ uint32_t compact3(uint32_t v) {
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030C30C3u;
    v = (v | (v >> 4)) & 0x0300F00Fu;
    v = (v | (v >> 8)) & 0x030000FFu;
    v = (v | (v >> 16)) & 0x000003FFu;
    return v;
}

// Exclusive sum over the block; *total = sum.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_sum(uint32_t v, uint32_t* total, uint32_t* red) {
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(incl, d, 64);
        if (lane >= (uint32_t)d) incl += o;
    }
    if (NT == 64) {
        *total = __shfl(incl, 63, 64);
        return incl - v;
    }
    if (lane == 63) red[wave] = incl;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        uint32_t x = red[w];
        base += (uint32_t)w < wave ? x : 0u;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return base + incl - v;
}

// 2-state transfer function of one symbol, or of a run of symbols:
// bit e = state after the run when it was entered in state e
// (state 0: the next symbol is an operation; state 1: it is a delta entry).
__device__ __forceinline__ uint32_t fn_then(uint32_t first, uint32_t second) {
    return ((second >> (first & 1u)) & 1u) | (((second >> ((first >> 1) & 1u)) & 1u) << 1);
}

// -------------------------------------------------------------- palette
__device__ __forceinline__ uint64_t pal_read(const Params& P, const TaskHdr& h, const uint8_t* U, uint32_t idx) {
    if (P.label_bytes == 4) {
        if (h.pal_lds) return ((const uint32_t*)U)[idx];
        return idx < h.pc ? ((const uint32_t*)(P.vol + h.pal_off))[idx] : 0u;
    }
    if (h.pal_lds) return ((const uint64_t*)U)[idx];
    return idx < h.pc ? ((const uint64_t*)(P.vol + h.pal_off))[idx] : 0u;
}

// -------------------------------------------------------------- task parse
__device__ __forceinline__ uint32_t ld32(const uint8_t* p) { return *(const uint32_t*)p; }

// Validate task j and its record with the same checks, in the same order, as
// the CPU decoder; fills the header (thread 0 only).
__device__ void parse_task(const Params& P, uint32_t task, TaskHdr& h) {
    h.task = task;
    h.status = kTaskOk;
    h.write_ok = 0;
    h.big = 0;
    const uint32_t id = P.ids[task];
    const uint32_t lod = P.lods[task];
    const uint64_t out_off = P.out_offs ? P.out_offs[task] : P.dense_offs[task];
    h.out_off = out_off;
    if (id >= P.n_bricks) { h.status = kTaskInvalid; return; }
    const uint64_t* offs = (const uint64_t*)(P.vol + P.off_pos);
    const uint64_t a = offs[id], b = offs[id + 1];
    if (a > b || b > P.vol_bytes || (a & 7) || b - a < 8) { h.status = kTaskCorrupt; return; }
    const uint8_t* rec = P.vol + a;
    const uint32_t w0 = ld32(rec);
    const uint32_t coder = w0 & 0xFF, L = (w0 >> 8) & 0xFF, lb = (w0 >> 16) & 0xFF, log2W = w0 >> 24;
    const uint32_t pc = ld32(rec + 4);
    const uint64_t extent = b - a;
    // (a record larger than every brick the container was parsed with cannot
    // occur for the parsed bytes; it is refused because scratch is sized by them)
    if (L < 1 || L > kMaxLog2b || L > P.max_log2b) { h.status = kTaskCorrupt; return; }
    if (lod > L) { h.status = kTaskInvalid; return; }
    const uint32_t t = L - lod;
    const uint64_t S = 1ull << t, n_out = S * S * S;
    if (out_off > P.out_cap || n_out > P.out_cap - out_off) { h.status = kTaskInvalid; return; }
    h.write_ok = 1;
    h.L = L;
    h.t = t;
    if (lb != P.label_bytes || coder > 1 || (coder == kRaw4 && log2W != 0) || (coder == kRans && log2W > 8)) {
        h.status = kTaskCorrupt;
        return;
    }
    const uint64_t hdr = record_header_bytes(L, coder, log2W);
    if (hdr > extent) { h.status = kTaskCorrupt; return; }
    const uint64_t al = lb == 8 ? 8 : 4;
    const uint64_t pal_rel = (hdr + al - 1) / al * al;
    if (pal_rel > extent || (uint64_t)pc * lb > extent - pal_rel) { h.status = kTaskCorrupt; return; }
    const uint64_t pay_rel = pal_rel + (uint64_t)pc * lb;
    const uint64_t pay_bytes = extent - pay_rel;
    uint32_t prev = 0;
    for (uint32_t i = 0; i <= L; ++i) {
        const uint32_t e = ld32(rec + 8 + 4 * i);
        h.sym_end[i] = e;
        if (i > 0 && e < prev) { h.status = kTaskCorrupt; return; }
        prev = e;
    }
    if ((uint64_t)prev > 8 * total_nodes(L)) { h.status = kTaskCorrupt; return; }
    if (coder == kRaw4) {
        if ((uint64_t)prev > 2 * pay_bytes) { h.status = kTaskCorrupt; return; }
    } else {
        const uint32_t W = 1u << log2W, G = (W + 63) / 64;
        uint64_t tw = 0;
        for (uint32_t g = 0; g < G; ++g) {
            const uint32_t c = ld32(rec + 8 + 4 * (L + 1) + 4 * g);
            h.gw[g] = c;
            h.gstart[g] = (uint32_t)tw;
            tw += c;
        }
        if (2 * tw > pay_bytes) { h.status = kTaskCorrupt; return; }
        if (!P.freq_ok) { h.status = kTaskCorrupt; return; }
        h.states_off = a + 8 + 4 * (L + 1) + 4 * G;
    }
    h.coder = coder;
    h.log2W = log2W;
    h.pc = pc;
    h.pal_off = a + pal_rel;
    h.pay_off = a + pay_rel;
    h.nsym = h.sym_end[t];
    // the explicit nodes of levels 4 and 5 are at most their segments' symbol counts
    uint32_t need = 0, c5 = 0;
    if (t >= 4) {
        c5 = (h.sym_end[4] - h.sym_end[3] + 7u) & ~7u;
        need = c5;
        if (t >= 5) need += h.sym_end[5] - h.sym_end[4];
    }
    h.c5base = c5;
    h.big = pc > 32768u || need > P.cap16;
    h.pal_lds = (uint64_t)pc * lb <= kUBytes;
}

// ----------------------------------------------------------------- rANS
// Decode the first h.nsym symbols of the record into 4-bit symbols at nib[]
// (low nibble first).  Wavefront w handles lane groups w, w + NW, ...
template <int NT>
__device__ void rans_decode(const Params& P, Shared& sh, uint8_t* nib) {
    const TaskHdr& h = sh.h;
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    const uint32_t W = 1u << h.log2W, G = (W + 63) / 64, lanes = W < 64 ? W : 64;
    const uint32_t nsym = h.nsym;
    const uint16_t* words = (const uint16_t*)(P.vol + h.pay_off);
    const uint32_t* states = (const uint32_t*)(P.vol + h.states_off);
    const uint32_t* tab = (const uint32_t*)sh.U;
    for (uint32_t g = wave; g < G; g += NT / 64) {
        const bool active = lane < lanes;
        const uint32_t gl = 64 * g + lane;
        const uint32_t gcount = h.gw[g], gbase = h.gstart[g];
        uint32_t x = active ? states[gl] : 0u;
        // word window: win0 holds words [wbase, wbase+64), win1 the next 64
        uint32_t wbase = 0;
        uint32_t win0 = lane < gcount ? words[gbase + lane] : 0u;
        uint32_t win1 = 64 + lane < gcount ? words[gbase + 64 + lane] : 0u;
        uint32_t gpos = 0, pend = 0;
        bool bad = false;
        for (uint32_t r0 = 64 * g; r0 < nsym; r0 += W) {
            const uint32_t j = r0 + lane;
            const bool act = active && j < nsym;
            uint32_t s = 0;
            if (act) {
                const uint32_t e = tab[x & (kRansM - 1)];
                s = e & 15u;
                x = ((e >> 4) & 0x1FFFu) * (x >> kRansBits) + (e >> 17);
            }
            const bool need = act && x < kRansL;
            const uint64_t m = __ballot(need);
            const uint32_t widx = gpos + mbcnt(m);
            const uint32_t rel = widx - wbase;
            const uint32_t v0 = __shfl(win0, rel & 63, 64), v1 = __shfl(win1, rel & 63, 64);
            if (need) {
                if (widx >= gcount) bad = true;
                x = (x << 16) | (rel < 64 ? v0 : v1);
            }
            gpos += (uint32_t)__popcll(m);
            // two consecutive symbols per output byte
            if (W >= 2) {
                const uint32_t hi = __shfl_xor(s, 1, 64);
                if (act && !(lane & 1)) nib[j >> 1] = (uint8_t)(s | (j + 1 < nsym ? hi << 4 : 0u));
            } else if (lane == 0) {
                if (!(j & 1)) {
                    pend = s;
                    if (j + 1 == nsym) nib[j >> 1] = (uint8_t)pend;
                } else {
                    nib[j >> 1] = (uint8_t)(pend | (s << 4));
                }
            }
            if (gpos - wbase >= 64) {
                wbase += 64;
                win0 = win1;
                const uint32_t p = wbase + 64 + lane;
                win1 = p < gcount ? words[gbase + p] : 0u;
            }
        }
        if (__ballot(bad) && lane == 0) atomicOr(&sh.err, 1u);
    }
}

// ------------------------------------------------------------ level store
// Where the levels of one task live.  V: slot type (u16 fast path, u32 big
// path).  Full grids of levels 0..3 and compact slots of levels 4 and 5 are
// LDS (fast) or scratch (big); level 6 slots are u32 at the voxel position in
// the output; parent lists are LDS for levels <= 5 on the fast path.
template <typename V>
struct Slot {
    static constexpr V kFinal = (V)(V(1) << (sizeof(V) * 8 - 1));
    static constexpr V kIdx = (V)(kFinal - 1);
};

template <typename V, bool BIG>
struct Store {
    V* full;          // levels 0..3 at fbase(i)
    V* c4;            // compact slots of level 4
    V* c5;            // compact slots of level 5
    uint32_t* out6;   // level-6 slots (u32 at voxel v: out6[v * lb / 4])
    uint32_t lb4;     // label_bytes / 4
    uint32_t* E;      // bitmaps of levels 0..4 (LDS)
    uint16_t* wpre;
    uint32_t* E5;     // bitmap of level 5 (scratch)
    uint16_t* wpre5;
    uint16_t* list_l;  // parent lists in LDS (fast path, levels <= 5)
    V* pval_l;
    uint16_t* list_g;  // parent lists in scratch
    uint32_t* pval_g;
    bool list_in_lds;

    __device__ __forceinline__ uint32_t* ebits(uint32_t lvl) const { return lvl <= 4 ? E + ebase(lvl) : E5; }
    __device__ __forceinline__ const uint16_t* epre(uint32_t lvl) const { return lvl <= 4 ? wpre + ebase(lvl) : wpre5; }
    __device__ __forceinline__ bool ebit(uint32_t lvl, uint32_t q) const {
        if (lvl <= 4) return (E[ebase(lvl) + (q >> 5)] >> (q & 31)) & 1u;
        return (E5[q >> 5] >> (q & 31)) & 1u;
    }
    __device__ __forceinline__ uint32_t rank(uint32_t lvl, uint32_t q) const {
        uint32_t w, p;
        if (lvl <= 4) {
            w = E[ebase(lvl) + (q >> 5)];
            p = wpre[ebase(lvl) + (q >> 5)];
        } else {
            w = E5[q >> 5];
            p = wpre5[q >> 5];
        }
        return p + (uint32_t)__popc(w & ((1u << (q & 31)) - 1u));
    }
    // value of node `node` of level lvl (<= 5), all levels up to lvl final
    __device__ __forceinline__ uint32_t value_at(uint32_t lvl, uint32_t node) const {
        while (lvl >= 4) {
            const uint32_t q = node >> 3;
            if (ebit(lvl - 1, q)) {
                const uint32_t k = 8 * rank(lvl - 1, q) + (node & 7);
                return lvl == 4 ? (uint32_t)c4[k] : (uint32_t)c5[k];
            }
            lvl -= 1;
            node = q;
        }
        return full[fbase(lvl) + node];
    }
    // slot of level lvl at index idx (full: node; compact: rank; level 6: voxel)
    __device__ __forceinline__ uint32_t get(uint32_t lvl, uint32_t idx) const {
        if (lvl <= 3) return full[fbase(lvl) + idx];
        if (lvl == 4) return c4[idx];
        if (lvl == 5) return c5[idx];
        return out6[(uint64_t)idx * lb4];
    }
    __device__ __forceinline__ void set(uint32_t lvl, uint32_t idx, uint32_t v) const {
        if (lvl <= 3) full[fbase(lvl) + idx] = (V)v;
        else if (lvl == 4) c4[idx] = (V)v;
        else if (lvl == 5) c5[idx] = (V)v;
        else out6[(uint64_t)idx * lb4] = v;
    }
    __device__ __forceinline__ uint32_t list(uint32_t r) const { return list_in_lds ? list_l[r] : list_g[r]; }
    __device__ __forceinline__ uint32_t pval(uint32_t r) const { return list_in_lds ? (uint32_t)pval_l[r] : pval_g[r]; }
    __device__ __forceinline__ void set_list(uint32_t r, uint32_t q, uint32_t v) const {
        if (list_in_lds) {
            list_l[r] = (uint16_t)q;
            pval_l[r] = (V)v;
        } else {
            list_g[r] = (uint16_t)q;
            pval_g[r] = v;
        }
    }
};

// final flag / index mask of a level's slots (level 6 slots are always u32)
template <typename V>
__device__ __forceinline__ uint32_t fin_bit(uint32_t lvl) { return lvl == 6 ? 0x80000000u : (uint32_t)Slot<V>::kFinal; }

// index of node p (Morton, level i) in the level's slot storage given its op rank k
__device__ __forceinline__ uint32_t slot_index(uint32_t i, uint32_t p, uint32_t k) {
    if (i <= 3) return p;
    if (i <= 5) return k;
    return (compact3(p >> 2) << 12) | (compact3(p >> 1) << 6) | compact3(p);  // (z*64 + y)*64 + x
}

// ------------------------------------------------------------ level decode
template <int NT, typename V, bool BIG>
__device__ void decode_levels(const Params& P, Shared& sh, const Store<V, BIG>& st, const uint8_t* nib) {
    constexpr uint32_t NW = NT / 64;
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const uint32_t t = sh.h.t, pc = sh.h.pc;
    uint32_t adv_done = 0;
    uint32_t pbuf = 0;
    for (uint32_t i = 0; i <= t; ++i) {
        const uint32_t nodes = 1u << (3 * i);
        const uint32_t FIN = fin_bit<V>(i), IDX = FIN - 1u;
        // final values of lower levels carry V's flag; level-6 slots are u32 with their own
        const auto refin = [FIN](uint32_t x) { return (x & (uint32_t)Slot<V>::kIdx) | FIN; };
        // references of this level point below this bound (full: nodes; compact: ops; level 6: voxels)
        const uint32_t ref_lim = i <= 3 ? nodes : i <= 5 ? 0xFFFFFFFFu : (1u << 18);
        // ------------------------------------------ level set-up
        uint32_t expected = 1;
        if (i > 0) {
            // expanding parents of level i-1: word prefix, list, values
            const uint32_t pl = i - 1, pn = nodes >> 3, pw = ewords(pl);
            uint32_t* Ep = st.ebits(pl);
            uint16_t* Wp = (uint16_t*)st.epre(pl);
            uint32_t base = 0;
            for (uint32_t w0 = 0; w0 < pw; w0 += NT) {
                const uint32_t w = w0 + tid;
                uint32_t bits = w < pw ? Ep[w] : 0u;
                if (pn < 32) bits &= (1u << pn) - 1u;
                uint32_t tot;
                const uint32_t pre = block_excl_sum<NT>((uint32_t)__popc(bits), &tot, sh.red);
                if (w < pw) {
                    Wp[w] = (uint16_t)(base + pre);
                    if (pn < 32) Ep[w] = bits;
                }
                base += tot;
            }
            expected = 8 * base;
            __syncthreads();
            for (uint32_t q = tid; q < pn; q += NT) {
                const uint32_t bits = Ep[q >> 5];
                const bool ex = (bits >> (q & 31)) & 1u;
                if (ex) {
                    const uint32_t r = Wp[q >> 5] + (uint32_t)__popc(bits & ((1u << (q & 31)) - 1u));
                    st.set_list(r, q, st.value_at(pl, q));
                } else if (i <= 3) {
                    const uint32_t v = st.full[fbase(pl) + q];
                    V* d = st.full + fbase(i) + 8 * q;
#pragma unroll
                    for (int c = 0; c < 8; ++c) d[c] = (V)v;
                }
            }
        }
        if (i < t && i <= 5) {
            uint32_t* Ei = st.ebits(i);
            for (uint32_t w = tid; w < ewords(i); w += NT) Ei[w] = 0;
        }
        __syncthreads();
        // ------------------------------------------ passes over the segment
        const uint32_t mx = 0x09249249u & (nodes - 1u), my = mx << 1, mz = mx << 2;
        const uint32_t s0 = i ? sh.h.sym_end[i - 1] : 0u, s1 = sh.h.sym_end[i];
        uint32_t carry = 0, k_done = 0;
        bool bad = false;
        uint32_t snext = 0;
        if (s0 + tid < s1) {
            const uint32_t j = s0 + tid;
            snext = (nib[j >> 1] >> (4 * (j & 1))) & 15u;
        }
        for (uint32_t c = s0; c < s1; c += NT) {
            const uint32_t j = c + tid;
            const bool valid = j < s1;
            const uint32_t s = snext;
            if (j + NT < s1) {
                const uint32_t jn = j + NT;
                snext = (nib[jn >> 1] >> (4 * (jn & 1))) & 15u;
            }
            // classification for both entry states
            const uint64_t m_valid = __ballot(valid);
            const uint64_t m_cand = __ballot(valid && (s & 7u) == kDelta);
            const uint64_t m_adv = __ballot(valid && (s & 7u) == kAdv);
            uint64_t ops0, ops1;
            uint32_t x0, x1;
            if (m_cand == 0) {
                ops0 = m_valid;
                x0 = 0;
                const uint64_t m_end = m_valid & ~__ballot(valid && (s & 8u));
                if (m_end) {
                    const uint32_t f = (uint32_t)__builtin_ctzll(m_end);
                    const uint64_t upto = f >= 63 ? ~0ull : ((2ull << f) - 1ull);
                    ops1 = m_valid & ~upto;
                    x1 = 0;
                } else {
                    ops1 = 0;
                    x1 = 1;
                }
            } else {
                const uint32_t f = valid ? (((s & 7u) == kDelta ? 1u : 0u) | (((s >> 3) & 1u) << 1)) : 2u;
                uint32_t incl = f;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const uint32_t o = __shfl_up(incl, d, 64);
                    if (lane >= (uint32_t)d) incl = fn_then(o, incl);
                }
                uint32_t excl = __shfl_up(incl, 1, 64);
                if (lane == 0) excl = 2u;
                ops0 = __ballot(valid && !(excl & 1u));
                ops1 = __ballot(valid && !((excl >> 1) & 1u));
                const uint32_t tot = __shfl(incl, 63, 64);
                x0 = tot & 1u;
                x1 = (tot >> 1) & 1u;
            }
            if (lane == 0) {
                sh.pub[pbuf][wave] = (uint32_t)__popcll(ops0) | ((uint32_t)__popcll(ops1) << 7) |
                                     ((uint32_t)__popcll(ops0 & m_adv) << 14) |
                                     ((uint32_t)__popcll(ops1 & m_adv) << 21) | (x0 << 28) | (x1 << 29);
            }
            __syncthreads();
            // fold the waves' summaries: entry state, op base and ADV base of this wave; pass totals
            uint32_t e = carry, kb = k_done, ab = adv_done, my_e = 0, my_kb = 0, my_ab = 0;
#pragma unroll
            for (uint32_t w = 0; w < NW; ++w) {
                if (w == wave) {
                    my_e = e;
                    my_kb = kb;
                    my_ab = ab;
                }
                const uint32_t p = sh.pub[pbuf][w];
                kb += e ? ((p >> 7) & 127u) : (p & 127u);
                ab += e ? ((p >> 21) & 127u) : ((p >> 14) & 127u);
                e = e ? ((p >> 29) & 1u) : ((p >> 28) & 1u);
            }
            const uint32_t k0 = k_done;
            carry = e;
            k_done = kb;
            adv_done = ab;
            pbuf ^= 1u;
            const uint64_t my_ops = my_e ? ops1 : ops0;
            const bool is_op = (my_ops >> lane) & 1u;
            uint32_t myidx = 0, myval = 0;
            bool is_ref = false;
            if (is_op) {
                const uint32_t k = my_kb + mbcnt(my_ops);
                const uint32_t a = my_ab + mbcnt(my_ops & m_adv);
                const uint32_t op = s & 7u, stop = s >> 3;
                if (k >= expected) {
                    bad = true;
                } else {
                    const uint32_t r = k >> 3;
                    const uint32_t pn = i ? st.list(r) : 0u;
                    const uint32_t p = i ? ((pn << 3) | (k & 7u)) : 0u;
                    uint32_t v = FIN;
                    switch (op) {
                    case kParent:
                        if (i == 0) bad = true;
                        else v = refin(st.pval(r));
                        break;
                    case kNX:
                    case kNY:
                    case kNZ: {
                        const uint32_t am = op == kNX ? mx : op == kNY ? my : mz;
                        if (!(p & am)) {
                            bad = true;
                            break;
                        }
                        const uint32_t tn = ((((p & am) - 1u) & am) | (p & ~am));
                        const uint32_t tq = tn >> 3;
                        if (!st.ebit(i - 1, tq)) {
                            v = refin(st.value_at(i - 1, tq));  // implied target: its parent's value, final
                        } else {
                            const uint32_t kt = 8 * st.rank(i - 1, tq) + (tn & 7u);
                            const uint32_t ti = slot_index(i, tn, kt);
                            if (kt < k0) {
                                v = st.get(i, ti);  // decoded in an earlier pass: final
                            } else {
                                v = ti;  // same pass: resolved below
                                is_ref = true;
                            }
                        }
                        break;
                    }
                    case kAdv:
                        if (a >= pc) bad = true;
                        else v = FIN | a;
                        break;
                    case kLast:
                        if (a == 0) bad = true;
                        else v = FIN | (a - 1u);
                        break;
                    case kDelta: {
                        uint32_t d = 0, jj = j + 1, en = 8;
                        while (en & 8u) {
                            if (jj >= s1) {
                                bad = true;
                                break;
                            }
                            en = (nib[jj >> 1] >> (4 * (jj & 1))) & 15u;
                            d = d >= (1u << 29) ? 0xFFFFFFFFu : ((d << 3) | (en & 7u));
                            ++jj;
                        }
                        if (d == 0 || d > a) bad = true;
                        else v = FIN | (a - d);
                        break;
                    }
                    default:
                        bad = true;
                    }
                    myidx = slot_index(i, p, k);
                    myval = v;
                    // written even after an error, so that a later lookup never meets an unset slot
                    st.set(i, myidx, (is_ref && bad) ? FIN : v);
                    if (i < t && !stop) atomicOr(st.ebits(i) + (p >> 5), 1u << (p & 31));
                }
            }
            __syncthreads();
            // references within the pass: chase to a final value
            if (is_ref && !bad) {
                uint32_t v = myval, it = 0;
                while (!(v & FIN)) {
                    // a reference names an operation of this pass (compact levels: rank below k_done)
                    if ((v & IDX) >= (i <= 3 || i == 6 ? ref_lim : k_done) || ++it > NT) {
                        bad = true;
                        break;
                    }
                    v = st.get(i, v & IDX);
                }
                if (!bad) st.set(i, myidx, v);
                else st.set(i, myidx, FIN);
            }
        }
        if (bad) atomicOr(&sh.err, 1u);
        if (k_done != expected || carry != 0) {
            if (tid == 0) sh.err = 1u;
        }
        __syncthreads();
        if (sh.err) return;
    }
    if (t == sh.h.L && adv_done != pc && tid == 0) sh.err = 1u;
    __syncthreads();
}

// ------------------------------------------------------------------ output
__device__ __forceinline__ void store_pair(uint8_t* out, uint32_t lb, uint64_t e, uint64_t l0, uint64_t l1, bool vec) {
    if (lb == 4) {
        uint32_t* o = (uint32_t*)out + e;
        if (vec) *(uint2*)o = make_uint2((uint32_t)l0, (uint32_t)l1);
        else {
            o[0] = (uint32_t)l0;
            o[1] = (uint32_t)l1;
        }
    } else {
        uint64_t* o = (uint64_t*)out + e;
        if (vec) *(uint4*)o = make_uint4((uint32_t)l0, (uint32_t)(l0 >> 32), (uint32_t)l1, (uint32_t)(l1 >> 32));
        else {
            o[0] = l0;
            o[1] = l1;
        }
    }
}

template <int NT>
__device__ void zero_output(const Params& P, const TaskHdr& h) {
    const uint32_t t = h.t;
    const uint64_t n = 1ull << (3 * t);
    uint8_t* out = P.out + h.out_off * P.label_bytes;
    const uint64_t bytes = n * P.label_bytes;
    if (((uintptr_t)out & 15u) == 0 && (bytes & 15u) == 0) {
        for (uint64_t u = threadIdx.x; u < bytes / 16; u += NT) ((uint4*)out)[u] = make_uint4(0, 0, 0, 0);
    } else {
        for (uint64_t u = threadIdx.x; u < bytes / 4; u += NT) ((uint32_t*)out)[u] = 0u;
    }
}

// Labels of level t (all slots final) as an S^3 x-fastest cube.  Levels
// 0..3 voxel by voxel; levels 4..6 by 2x2x2 blocks under each node q of
// level t-1: q's value when it does not expand, else its 8 children's slots.
template <int NT, typename V, bool BIG>
__device__ void write_output(const Params& P, Shared& sh, const Store<V, BIG>& st) {
    const TaskHdr& h = sh.h;
    const uint32_t t = h.t, S = 1u << t, lb = P.label_bytes;
    const uint32_t IDXV = (uint32_t)Slot<V>::kIdx;
    uint8_t* out = P.out + h.out_off * lb;
    if (t <= 3) {
        const uint32_t n = S * S * S;
        for (uint32_t v = threadIdx.x; v < n; v += NT) {
            const uint32_t x = v & (S - 1), y = (v >> t) & (S - 1), z = v >> (2 * t);
            const uint32_t m = spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
            const uint64_t l = pal_read(P, h, sh.U, st.full[fbase(t) + m] & IDXV);
            if (lb == 4) ((uint32_t*)out)[v] = (uint32_t)l;
            else ((uint64_t*)out)[v] = l;
        }
        return;
    }
    const uint32_t hb = t - 1, H = 1u << hb;  // parents per axis
    const uint32_t n = H * H * H;
    const bool vec = ((uintptr_t)out & (2 * lb - 1)) == 0;
    for (uint32_t u = threadIdx.x; u < n; u += NT) {
        const uint32_t qx = u & (H - 1), qy = (u >> hb) & (H - 1), qz = u >> (2 * hb);
        const uint32_t q = spread3(qx) | (spread3(qy) << 1) | (spread3(qz) << 2);
        const uint64_t e0 = ((uint64_t)(2 * qz) * S + 2 * qy) * S + 2 * qx;
        uint64_t lab[8];
        if (st.ebit(t - 1, q)) {
            if (t <= 5) {
                const uint32_t r = st.rank(t - 1, q);
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    lab[c] = pal_read(P, h, sh.U, st.get(t, 8 * r + c) & IDXV);
            } else {
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const uint64_t e = e0 + ((uint64_t)((c >> 2) & 1) * S + ((c >> 1) & 1)) * S + (c & 1);
                    lab[c] = pal_read(P, h, sh.U, st.out6[e * st.lb4] & 0x7FFFFFFFu);
                }
            }
        } else {
            const uint64_t l = pal_read(P, h, sh.U, st.value_at(t - 1, q) & IDXV);
#pragma unroll
            for (int c = 0; c < 8; ++c) lab[c] = l;
        }
        // child c = x | y << 1 | z << 2 of the block
#pragma unroll
        for (int zy = 0; zy < 4; ++zy) {
            const uint64_t e = e0 + ((uint64_t)(zy >> 1) * S + (zy & 1)) * S;
            store_pair(out, lb, e, lab[2 * zy], lab[2 * zy + 1], vec);
        }
    }
}

// ------------------------------------------------------------------ a task
template <int NT, typename V, bool BIG>
__device__ void run_levels(const Params& P, Shared& sh, V* compact_lds, uint8_t* scratch, const uint8_t* nib) {
    const TaskHdr& h = sh.h;
    Store<V, BIG> st;
    st.E = sh.E;
    st.wpre = sh.wpre;
    st.E5 = (uint32_t*)(scratch + kScrE5);
    st.wpre5 = (uint16_t*)(scratch + kScrWpre5);
    st.list_g = (uint16_t*)(scratch + kScrList);
    st.pval_g = (uint32_t*)(scratch + kScrPval);
    st.lb4 = P.label_bytes / 4;
    st.out6 = (uint32_t*)(P.out + h.out_off * P.label_bytes);
    if (BIG) {
        st.full = (V*)(scratch + kScrFull);
        st.c4 = (V*)(scratch + kScrComp);
        st.c5 = st.c4 + 4096;
        st.list_l = nullptr;
        st.pval_l = nullptr;
    } else {
        st.full = (V*)sh.G;
        st.c4 = compact_lds;
        st.c5 = compact_lds + h.c5base;
        st.list_l = (uint16_t*)sh.U;
        st.pval_l = (V*)(sh.U + kUBytes / 2);
    }
    // parent lists: LDS on the fast path, except for 64^3 bricks at full
    // resolution, whose level-6 parents (up to 32768) live in scratch
    st.list_in_lds = !BIG && h.t <= 5;
    decode_levels<NT, V, BIG>(P, sh, st, nib);
    if (sh.err) return;
    // palette staging for the output pass (parent lists are no longer needed)
    if (h.pal_lds) {
        const uint32_t words = (h.pc * P.label_bytes + 3) / 4;
        const uint32_t* src = (const uint32_t*)(P.vol + h.pal_off);
        for (uint32_t w = threadIdx.x; w < words; w += NT) ((uint32_t*)sh.U)[w] = src[w];
        __syncthreads();
    }
    write_output<NT, V, BIG>(P, sh, st);
}

template <int NT>
__device__ void decode_task(const Params& P, Shared& sh, uint16_t* compact_lds, uint8_t* scratch) {
    const TaskHdr& h = sh.h;
    if (h.status != kTaskOk) {
        if (h.status == kTaskCorrupt && h.write_ok) zero_output<NT>(P, h);
        return;
    }
    const uint8_t* nib;
    if (h.coder == kRaw4) {
        nib = P.vol + h.pay_off;
    } else {
        const uint4* src = (const uint4*)P.rans_tab;
        for (uint32_t w = threadIdx.x; w < kRansM / 4; w += NT) ((uint4*)sh.U)[w] = src[w];
        __syncthreads();
        rans_decode<NT>(P, sh, scratch + kScrSym);
        nib = scratch + kScrSym;
        __syncthreads();
    }
    if (!sh.err) {
        if (h.big) run_levels<NT, uint32_t, true>(P, sh, nullptr, scratch, nib);
        else run_levels<NT, uint16_t, false>(P, sh, compact_lds, scratch, nib);
    }
    __syncthreads();
    if (sh.err) {
        if (threadIdx.x == 0) sh.h.status = kTaskCorrupt;
        zero_output<NT>(P, h);
    }
}

template <int NT>
__global__ void __launch_bounds__(NT) decode_kernel(Params P) {
    extern __shared__ uint8_t dyn_smem[];
    Shared& sh = *reinterpret_cast<Shared*>(dyn_smem);
    uint16_t* compact_lds = reinterpret_cast<uint16_t*>(dyn_smem + sizeof(Shared));
    const uint32_t tid = threadIdx.x;
    uint8_t* scratch = P.scratch + (uint64_t)blockIdx.x * P.scratch_stride;
    uint32_t iter = 0;
    for (;;) {
        if (tid == 0) {
            uint32_t jt;
            if (P.queue) jt = atomicAdd(P.queue, 1u);
            else jt = iter == 0 ? P.task0 + blockIdx.x : P.n_tasks;
            sh.err = 0;
            if (jt < P.n_tasks) {
                parse_task(P, P.order ? P.order[jt] : jt, sh.h);
            } else {
                sh.h.task = 0xFFFFFFFFu;
            }
        }
        __syncthreads();
        ++iter;
        const uint32_t task = sh.h.task;
        if (task == 0xFFFFFFFFu) break;
        decode_task<NT>(P, sh, compact_lds, scratch);
        __syncthreads();
        if (tid == 0 && P.status) P.status[task] = sh.h.status;
        __syncthreads();
    }
}

// ------------------------------------------------------------ small kernels
__global__ void reset_queue_kernel(uint32_t* q) {
    if (threadIdx.x == 0) q[0] = 0;
}

// rANS decoding table of the volume: slot -> symbol | freq << 4 | (slot - cum) << 17
__global__ void rans_table_kernel(uint32_t* tab, RansFreq f) {
    const uint32_t slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= kRansM) return;
    uint32_t cum = 0, s = 0, fs = 0;
    for (uint32_t k = 0; k < 16; ++k) {
        const uint32_t fk = (f.w[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
        if (slot >= cum && slot < cum + fk) {
            s = k;
            fs = fk;
            break;
        }
        cum += fk;
    }
    tab[slot] = s | (fs << 4) | ((slot - cum) << 17);
}

// brick side exponent of a task's record (0 when the task or record is unusable)
__device__ __forceinline__ uint32_t task_t(const Params& P, uint32_t j, uint64_t* rec_bytes) {
    const uint32_t id = P.ids[j];
    *rec_bytes = 0;
    if (id >= P.n_bricks) return 0xFFu;
    const uint64_t* offs = (const uint64_t*)(P.vol + P.off_pos);
    const uint64_t a = offs[id], b = offs[id + 1];
    if (a > b || b > P.vol_bytes || (a & 7) || b - a < 8) return 0xFFu;
    *rec_bytes = b - a;
    const uint32_t L = P.vol[a + 1];
    const uint32_t lod = P.lods[j];
    if (L < 1 || L > kMaxLog2b || lod > L) return 0xFFu;
    return L - lod;
}

// task cost classes for a decreasing-cost pop order: cls = 63 - clz(cost)
__global__ void cost_class_kernel(Params P, uint32_t* cls, uint32_t* hist) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= P.n_tasks) return;
    uint64_t rec;
    const uint32_t t = task_t(P, j, &rec);
    const uint64_t cost = rec + (t <= kMaxLog2b ? ((uint64_t)1 << (3 * t)) * P.label_bytes : 0) + 1;
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

// Dense output offsets: exclusive prefix sum of the tasks' cube sizes in task
// order (a task whose record or LOD is unusable occupies nothing).  One
// work-group of 1024 threads walks the task list in chunks.
__global__ void __launch_bounds__(1024) dense_offsets_kernel(Params P, uint64_t* offs) {
    __shared__ uint64_t wsum[16];
    __shared__ uint64_t carry;
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (uint32_t c = 0; c < P.n_tasks; c += 1024) {
        const uint32_t j = c + tid;
        uint64_t sz = 0;
        if (j < P.n_tasks) {
            uint64_t rec;
            const uint32_t t = task_t(P, j, &rec);
            sz = t <= kMaxLog2b ? (1ull << (3 * t)) : 0;
        }
        uint64_t incl = sz;
        for (int d = 1; d < 64; d <<= 1) {
            const uint64_t o = __shfl_up(incl, d, 64);
            if (lane >= (uint32_t)d) incl += o;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        uint64_t base = carry;
        uint64_t tot = 0;
        for (uint32_t w = 0; w < 16; ++w) {
            base += w < wave ? wsum[w] : 0;
            tot += wsum[w];
        }
        if (j < P.n_tasks) offs[j] = base + incl - sz;
        __syncthreads();
        if (tid == 0) carry += tot;
        __syncthreads();
    }
}

// ------------------------------------------------------------ host launch
size_t shared_bytes(uint32_t cap16) { return sizeof(Shared) + 2ull * cap16; }

template <int NT>
static hipError_t launch_nt(const Params& P, uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL(decode_kernel<NT>, dim3(grid), dim3(NT), shared_bytes(P.cap16), s, P);
    return hipGetLastError();
}

hipError_t set_kernel_attrs() {
    const int maxb = (int)shared_bytes(kMaxCap16);
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void*)decode_kernel<128>, hipFuncAttributeMaxDynamicSharedMemorySize, maxb)))
        return e;
    if ((e = hipFuncSetAttribute((const void*)decode_kernel<256>, hipFuncAttributeMaxDynamicSharedMemorySize, maxb)))
        return e;
    if ((e = hipFuncSetAttribute((const void*)decode_kernel<512>, hipFuncAttributeMaxDynamicSharedMemorySize, maxb)))
        return e;
    return hipFuncSetAttribute((const void*)decode_kernel<1024>, hipFuncAttributeMaxDynamicSharedMemorySize, maxb);
}

hipError_t launch_decode(const Params& P, int wg_size, uint32_t grid, hipStream_t s) {
    switch (wg_size) {
    case 128: return launch_nt<128>(P, grid, s);
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

hipError_t launch_rans_table(uint32_t* tab, const RansFreq& f, hipStream_t s) {
    hipLaunchKernelGGL(rans_table_kernel, dim3(kRansM / 256), dim3(256), 0, s, tab, f);
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

hipError_t launch_dense_offsets(const Params& P, uint64_t* offs, hipStream_t s) {
    hipLaunchKernelGGL(dense_offsets_kernel, dim3(1), dim3(1024), 0, s, P, offs);
    return hipGetLastError();
}

}  // namespace csgv
