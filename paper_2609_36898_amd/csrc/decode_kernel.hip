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
//   levels 0..4   full grids (4681 nodes).  When a level starts, the children
//                 of every parent that does not expand take the parent's
//                 value, and the children of expanding parents are marked
//                 "not yet decoded";
//   level 5       explicit nodes only, indexed by operation rank k (the k-th
//                 operation of a level is the k-th explicit node in Morton
//                 order); an implied node is its level-4 parent's value, an
//                 explicit one is found through the rank of its parent:
//                 prefix popcount of the level-4 expansion bitmap;
//   level 6       (64^3 bricks at full resolution) explicit nodes are kept at
//                 their voxel position in the task's own output range, which
//                 the output pass then overwrites in place with labels.
// A slot holds either a final palette index (top bit set) or a reference to
// a same-level slot whose value it copies (a neighbour operation whose target
// is decoded in the same pass).  Fast path: 16-bit slots, levels 0..5 in LDS;
// a 32^3 cube at full resolution with more level-5 nodes than the LDS share
// holds keeps its 16-bit level-5 slots in the work-group's scratch instead.
// Big path (palettes above 2^15 entries, or a 64^3 cube whose level 5 does not
// fit): 32-bit slots in a per-work-group global scratch area.
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
// rANS-coded records are first decoded into 4-bit symbols (in LDS for a cube
// of side <= 16 when they fit, else in the work-group's scratch): every 64-lane
// group of the interleaved coder is one wavefront, and the lanes that
// renormalise in a round find their word offsets with a ballot and a masked
// bit count.  The decoding table stays in LDS across tasks until a level-5
// decode reuses its space.
//
// Levels 0..2 (at most 73 nodes) are decoded by wavefront 0 alone, with wave
// barriers; meanwhile lane 0 of the last wavefront parses the work-group's
// next task (claimed when the current one started) into a second header.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "csgv_format.h"
#include "decode_kernel.h"

namespace csgv {

// ------------------------------------------------------------------ layout
// full grids of levels 0..4 at these slot offsets (8-aligned for 16-byte fills)
__device__ __forceinline__ uint32_t fbase(uint32_t i) {
    return i == 0 ? 0u : i == 1 ? 8u : i == 2 ? 16u : i == 3 ? 80u : 592u;
}
// expansion bitmaps of levels 0..4 at these word offsets
__device__ __forceinline__ uint32_t ebase(uint32_t i) {
    return i == 0 ? 0u : i == 1 ? 1u : i == 2 ? 2u : i == 3 ? 4u : 20u;
}
__host__ __device__ constexpr uint32_t ewords(uint32_t i) { return i <= 1 ? 1u : i == 2 ? 2u : (1u << (3 * i - 5)); }

// header words of a record: w0, palette count, sym_end[0..L], up to 4 group word counts
constexpr uint32_t kHdrWords = 2 + 7 + 4;

struct TaskHdr {
    uint32_t hw[kHdrWords];  // the record's first words (parse_task)
    uint32_t task, status, write_ok, coder, L, t, log2W, pc, big, c5g, pal_lds, nsym;
    uint32_t sym_end[7];
    uint32_t gw[4], gstart[4];
    uint64_t out_off, pal_off, pay_off, states_off;
};

struct Shared {
    TaskHdr h;   // the task being decoded
    TaskHdr hn;  // the work-group's next task, parsed ahead
    uint32_t err;
    uint32_t tab_ok;                     // the rANS table is in LDS from an earlier task
    uint32_t prog[4];                    // per rANS lane group: symbols out so far (release/acquire)
    uint32_t nexp;                       // expanding nodes of the parent level of the next level
    uint32_t adv;                        // PALETTE_ADV operations decoded so far (handed between phases)
    uint32_t pub[2][kMaxWaves][4];       // per pass and wave: run summary (f, n, a)
    uint32_t E[kEWords];                 // expansion bitmaps of levels 0..4
    uint16_t wpre[kEWords];              // exclusive popcount prefix of each bitmap word
    alignas(16) uint16_t G[kFullSlots];  // full grids of levels 0..4 (fast path)
    alignas(16) uint8_t U[kUBytes];      // parent list of the level being decoded | staged palette
};
static_assert(sizeof(Shared) % 16 == 0, "the slot area follows Shared 16-byte aligned");
static_assert(sizeof(TaskHdr) % 4 == 0 && sizeof(TaskHdr) / 4 <= 128, "a header is copied one word per thread");
static_assert(offsetof(Shared, U) == offsetof(Shared, G) + sizeof(Shared::G) &&
                  offsetof(Shared, U) + sizeof(Shared::U) == sizeof(Shared),
              "grids, parent list and slot area form one range (rANS staging)");

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

// Barrier of the threads that decode a level: the work-group, or (NT = 64)
// wavefront 0 alone, whose LDS accesses complete in order.
template <int NT>
__device__ __forceinline__ void lsync() {
    if (NT == 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// 2-state transfer function of one symbol, or of a run of symbols:
// bit e = state after the run when it was entered in state e
// (state 0: the next symbol is an operation; state 1: it is a delta entry).
__host__ __device__ constexpr uint32_t fn_then_ref(uint32_t first, uint32_t second) {
    return ((second >> (first & 1)) & 1) | (((second >> ((first >> 1) & 1)) & 1) << 1);
}
// all 16 compositions, 2 bits each at bit 2 * (4 * first + second)
__host__ __device__ constexpr uint32_t fn_then_table() {
    uint32_t t = 0;
    for (uint32_t a = 0; a < 4; ++a)
        for (uint32_t b = 0; b < 4; ++b) t |= fn_then_ref(a, b) << (2 * (4 * a + b));
    return t;
}
constexpr uint32_t kFnThen = fn_then_table();
__device__ __forceinline__ uint32_t fn_then(uint32_t first, uint32_t second) {
    return (kFnThen >> (2u * (4u * first + second))) & 3u;
}

// DPP moves (GFX9 controls).  A lane whose source lane does not exist, or
// whose row is masked off, keeps `old`.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ uint32_t dpp(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWS, 0xF, false);
}
constexpr int kDppRowShr = 0x110;   // + n: lane l takes lane l - n of its row of 16
constexpr int kDppWaveShl1 = 0x130;  // lane l takes lane l + 1
constexpr int kDppWaveShr1 = 0x138;  // lane l takes lane l - 1
constexpr int kDppBcast15 = 0x142;   // rows 1, 3 take lane 15 of the row before
constexpr int kDppBcast31 = 0x143;   // rows 2, 3 take lane 31
constexpr uint32_t kFnId = 2u;       // transfer function that keeps the state

// inclusive sum over the wavefront (lane 0 first)
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x) {
    x += dpp<kDppRowShr + 1>(0u, x);
    x += dpp<kDppRowShr + 2>(0u, x);
    x += dpp<kDppRowShr + 4>(0u, x);
    x += dpp<kDppRowShr + 8>(0u, x);
    x += dpp<kDppBcast15, 0xA>(0u, x);
    x += dpp<kDppBcast31, 0xC>(0u, x);
    return x;
}

// -------------------------------------------------------------- palette
// Palette entry idx: staged in LDS (PAL_LDS) or read from the record.  LT is
// the label type (u32 or u64); a global read is bounded by the palette count.
template <typename LT, bool PAL_LDS>
__device__ __forceinline__ LT pal_get(const LT* pal, uint32_t idx, uint32_t pc) {
    if (PAL_LDS) return pal[idx];
    return idx < pc ? pal[idx] : (LT)0;
}

// -------------------------------------------------------------- task parse
__device__ __forceinline__ uint32_t ld32(const uint8_t* p) { return *(const uint32_t*)p; }

// Validate task j and its record with the same checks, in the same order, as
// the CPU decoder; fills the header (thread 0 only).
__device__ __forceinline__ void parse_task(const Params& P, uint32_t task, TaskHdr& h) {
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
    const uint64_t extent = b - a;
    // the record's first kHdrWords words (more than any header holds) are loaded
    // at once, at offsets clamped into the record; the checks below use a word
    // only after placing it inside the header
    {
        const uint64_t last = (extent & ~3ull) - 4u;
#pragma unroll
        for (uint32_t k = 0; k < kHdrWords; ++k) h.hw[k] = ld32(rec + (4u * k < last ? 4u * k : last));
    }
    const uint32_t w0 = h.hw[0];
    const uint32_t coder = w0 & 0xFF, L = (w0 >> 8) & 0xFF, lb = (w0 >> 16) & 0xFF, log2W = w0 >> 24;
    const uint32_t pc = h.hw[1];
    // (a record larger than every brick the container was parsed with cannot
    // occur for the parsed bytes; it is refused because scratch is sized by them)
    if (L < 1 || L > kMaxLog2b || L > P.max_log2b) { h.status = kTaskCorrupt; return; }
    if (lod > L) { h.status = kTaskInvalid; return; }
    const uint32_t t = L - lod;
    const uint64_t S = 1ull << t, n_out = out_units(S * S * S, P.pal_bits);
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
        const uint32_t e = h.hw[2 + i];
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
            const uint32_t c = h.hw[3 + L + g];
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
    // explicit nodes of level 5: at most one per symbol of its segment
    const uint32_t need5 = t >= 5 ? h.sym_end[5] - h.sym_end[4] : 0u;
    // a 32^3 cube at full resolution whose level 5 outgrows the LDS slot area
    // keeps levels 0..4 in LDS and only its level-5 slots in scratch (c5g)
    h.big = pc > 32768u || (need5 > P.cap16 && t != 5);
    h.c5g = !h.big && need5 > P.cap16;
    h.pal_lds = (uint64_t)pc * lb <= kUBytes;
    // cache-paletted output: a palette beyond 2^I entries, or a 64^3 cube, has no packed form
    if (P.pal_bits && (t == 6 || (uint64_t)pc > (1ull << P.pal_bits))) {
        h.status = kTaskInvalid;
        h.write_ok = 0;
    }
}


// The work-group's next task: claimed by lane 0 of its last wavefront (jt, in
// that lane's register) when a task starts, and parsed into sh.hn by the same
// lane while that wavefront has nothing else to do (levels 0..2 are decoded by
// wavefront 0 alone), else at the end of the task.
struct Ahead {
    uint32_t jt;
    bool done;
};

__device__ __forceinline__ void parse_ahead(const Params& P, TaskHdr& hn, uint32_t jt) {
    if (jt < P.n_tasks) parse_task(P, P.order ? P.order[jt] : jt, hn);
    else hn.task = 0xFFFFFFFFu;
}

// ----------------------------------------------------------------- rANS
// Decode the first h.nsym symbols of the record into 4-bit symbols at nib[]
// (low nibble first).  Wavefront w handles lane groups w, w + NW, ...  A
// group's words sit in a 192-word register window; the third 64-word block is
// fetched as soon as the window moves, one window move before it is needed.
template <int NT>
__device__ __forceinline__ void rans_decode(const Params& P, Shared& sh, const uint32_t* tab, uint8_t* nib) {
    const TaskHdr& h = sh.h;
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    const uint32_t W = 1u << h.log2W, G = (W + 63) / 64, lanes = W < 64 ? W : 64;
    const uint32_t nsym = h.nsym;
    const uint16_t* words = (const uint16_t*)(P.vol + h.pay_off);
    const uint32_t* states = (const uint32_t*)(P.vol + h.states_off);
    for (uint32_t g = wave; g < G; g += NT / 64) {
        const bool active = lane < lanes;
        const uint32_t gl = 64 * g + lane;
        const uint32_t gcount = h.gw[g], gbase = h.gstart[g];
        uint32_t x = active ? states[gl] : 0u;
        uint32_t wbase = 0;
        uint32_t win0 = lane < gcount ? words[gbase + lane] : 0u;
        uint32_t win1 = 64 + lane < gcount ? words[gbase + 64 + lane] : 0u;
        uint32_t win2 = 128 + lane < gcount ? words[gbase + 128 + lane] : 0u;
        uint32_t gpos = 0, pend = 0;
        bool bad = false;
        // the loop-carried state and window start from loads: let them land here,
        // or every round would wait for all outstanding memory operations
        __builtin_amdgcn_s_waitcnt(0);
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
            const uint32_t rel = widx - wbase;  // < 128: at most 64 words per round, gpos - wbase < 64
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
                win1 = win2;
                const uint32_t p = wbase + 128 + lane;
                win2 = p < gcount ? words[gbase + p] : 0u;
            }
        }
        if (__ballot(bad) && lane == 0) atomicOr(&sh.err, 1u);
    }
}

// Copy the record's rANS words into LDS at `wl` (no barrier) and return this
// thread's state for its wavefront's first lane group.
template <int NT>
__device__ __forceinline__ uint32_t rans_stage_words(const Params& P, const TaskHdr& h, uint16_t* wl) {
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const uint32_t W = 1u << h.log2W, G = (W + 63) / 64, lanes = W < 64 ? W : 64;
    const uint32_t tw = h.gstart[G - 1] + h.gw[G - 1];
    const uint16_t* const wg = (const uint16_t*)(P.vol + h.pay_off);
    const uint32_t* states = (const uint32_t*)(P.vol + h.states_off);
    const uint32_t x0 = wave < G && lane < lanes ? states[64 * wave + lane] : 0u;
    for (uint32_t q = tid; q < tw / 2u; q += NT) ((uint32_t*)wl)[q] = ((const uint32_t*)wg)[q];
    if ((tw & 1u) && tid == 0) wl[tw - 1u] = wg[tw - 1u];
    return x0;
}

// The rounds of the decode from words staged in LDS at `wl` (after a barrier),
// symbols written to LDS at `nl`: a lane that renormalises reads its word from
// LDS, and no round waits on a global store.  Wavefront w decodes lane groups
// w, w + NW, ...  With `mark`, lane 0 publishes in sh.prog[g], with release
// order, that group g's symbols below index `mark` are out as soon as they are
// (its next round would start at or past `mark`), and ~0 when the group is done.
template <int NT>
__device__ __forceinline__ void rans_rounds(const Params& P, Shared& sh, const uint32_t* tab, const uint16_t* wl,
                                            uint8_t* nl, uint32_t x0, uint32_t mark) {
    const TaskHdr& h = sh.h;
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    const uint32_t W = 1u << h.log2W, G = (W + 63) / 64, lanes = W < 64 ? W : 64;
    const uint32_t nsym = h.nsym;
    const uint32_t* states = (const uint32_t*)(P.vol + h.states_off);
    for (uint32_t g = wave; g < G; g += NT / 64) {
        const bool active = lane < lanes;
        const uint32_t gcount = h.gw[g], gbase = h.gstart[g];
        uint32_t x = g == wave ? x0 : active ? states[64 * g + lane] : 0u;
        uint32_t gpos = 0, pend = 0;
        const uint32_t gcm1 = gcount ? gcount - 1u : 0u;  // word reads stay inside the group
        bool bad = false, marked = mark == 0;
        __builtin_amdgcn_s_waitcnt(0);
        // a round without branches: every lane looks its state up and reads a
        // word; a lane past the symbols keeps its state
        for (uint32_t r0 = 64 * g; r0 < nsym; r0 += W) {
            const uint32_t j = r0 + lane;
            const bool act = active && j < nsym;
            const uint32_t e = tab[x & (kRansM - 1)];
            const uint32_t s = e & 15u;
            const uint32_t xd = ((e >> 4) & 0x1FFFu) * (x >> kRansBits) + (e >> 17);
            const bool need = act && xd < kRansL;
            const uint64_t m = __ballot(need);
            const uint32_t widx = gpos + mbcnt(m);
            const uint32_t wv = wl[gbase + min(widx, gcm1)];
            bad = bad || (need && widx >= gcount);
            x = need ? ((xd << 16) | wv) : act ? xd : x;
            gpos += (uint32_t)__popcll(m);
            // two consecutive symbols per byte
            if (W >= 2) {
                const uint32_t hi = dpp<0xB1>(0u, s);  // quad_perm [1,0,3,2]: the pair partner
                if (act && !(lane & 1)) nl[j >> 1] = (uint8_t)(s | (j + 1 < nsym ? hi << 4 : 0u));
            } else if (lane == 0) {
                if (!(j & 1)) {
                    pend = s;
                    if (j + 1 == nsym) nl[j >> 1] = (uint8_t)pend;
                } else {
                    nl[j >> 1] = (uint8_t)(pend | (s << 4));
                }
            }
            if (!marked && r0 + W >= mark) {
                marked = true;
                if (lane == 0) __hip_atomic_store(&sh.prog[g], mark, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        if (__ballot(bad) && lane == 0) atomicOr(&sh.err, 1u);
        if (mark && lane == 0) __hip_atomic_store(&sh.prog[g], 0xFFFFFFFFu, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

// The decode with the record's words staged in LDS (`stage`, the level grids
// and slot area, idle until the levels start) and the symbols in LDS at `nl`;
// with `nib` set, the symbols then reach it in one coalesced copy.  The caller
// checks that words and symbols fit.
template <int NT>
__device__ __forceinline__ void rans_decode_lds(const Params& P, Shared& sh, const uint32_t* tab, uint8_t* stage,
                                                uint8_t* nl, uint8_t* nib) {
    const uint32_t x0 = rans_stage_words<NT>(P, sh.h, (uint16_t*)stage);
    __syncthreads();
    rans_rounds<NT>(P, sh, tab, (const uint16_t*)stage, nl, x0, 0u);
    if (nib) {
        __syncthreads();
        const uint32_t nw = ((sh.h.nsym + 1u) / 2u + 3u) / 4u;
        for (uint32_t q = threadIdx.x; q < nw; q += NT) ((uint32_t*)nib)[q] = ((const uint32_t*)nl)[q];
    }
}

// ------------------------------------------------------------ level store
template <typename V>
struct Slot {
    static constexpr V kFinal = (V)(V(1) << (sizeof(V) * 8 - 1));
    static constexpr V kIdx = (V)(kFinal - 1);
    static constexpr V kNotYet = kIdx;  // explicit node whose operation is not decoded yet (full levels)
};

// Where the levels of one task live.  V: slot type (u16 fast path, u32 big
// path).  Full grids of levels 0..4 and the compact level 5 are LDS (fast) or
// scratch (big); level-6 slots are u32 at the voxel position in the output.
template <typename V>
struct Store {
    V* full;          // levels 0..4 at fbase(i)
    V* c5;            // level-5 explicit nodes by operation rank
    uint32_t* out6;   // level-6 slot of voxel v: out6[v * lb4]
    uint32_t lb4;     // label_bytes / 4
    uint32_t* E;      // bitmaps of levels 0..4 (LDS)
    uint16_t* wpre;
    uint32_t* E5;     // bitmap of level 5 (scratch; 64^3 bricks at full resolution)
    uint16_t* wpre5;
    uint16_t* list_l;  // parents of the level being decoded, LDS (levels 1..5 on the fast path)
    uint16_t* list_g;  // the same in scratch (level 6, big path)
    uint32_t* pval_g;  // values of level-6 parents (scratch)

    // expansion bit / rank among the expanding nodes of a level: levels 0..4 in LDS ...
    __device__ __forceinline__ bool ebit(uint32_t lvl, uint32_t q) const {
        return (E[ebase(lvl) + (q >> 5)] >> (q & 31)) & 1u;
    }
    __device__ __forceinline__ uint32_t rank(uint32_t lvl, uint32_t q) const {
        const uint32_t w = E[ebase(lvl) + (q >> 5)];
        return wpre[ebase(lvl) + (q >> 5)] + (uint32_t)__popc(w & ((1u << (q & 31)) - 1u));
    }
    // ... and level 5 in scratch
    __device__ __forceinline__ bool ebit5(uint32_t q) const { return (E5[q >> 5] >> (q & 31)) & 1u; }
    __device__ __forceinline__ uint32_t rank5(uint32_t q) const {
        return wpre5[q >> 5] + (uint32_t)__popc(E5[q >> 5] & ((1u << (q & 31)) - 1u));
    }
    // value of a level-5 node (levels 0..5 final)
    __device__ __forceinline__ uint32_t value5(uint32_t node) const {
        const uint32_t q = node >> 3;
        if (ebit(4, q)) return c5[8 * rank(4, q) + (node & 7)];
        return full[fbase(4) + q];
    }
};

// voxel index (z*64 + y)*64 + x of a level-6 Morton index
__device__ __forceinline__ uint32_t vox6(uint32_t p) {
    return (compact3(p >> 2) << 12) | (compact3(p >> 1) << 6) | compact3(p);
}

// ------------------------------------------------------------ level set-up
// Expanding parents of level i (the nodes of level pl = i - 1 whose bit is set
// in its bitmap), in two steps.  level_prefix (wavefront 0): exclusive
// popcount prefix of the bitmap's words, each lane summing a run of
// consecutive words, and the number of expanding parents in sh.nexp.
// level_fill (all threads of the level): the list of their node indices by
// rank and, for a full level i, the children's initial slots; the bitmap of
// level i is cleared when level i has children.
template <typename V, bool PL5>
__device__ __forceinline__ void level_prefix(Shared& sh, const Store<V>& st, uint32_t pl) {
    const uint32_t lane = lane_id(), pn = 1u << (3 * pl), pw = ewords(pl);
    const uint32_t mask = pn < 32 ? (1u << pn) - 1u : 0xFFFFFFFFu;
    const uint32_t* const Ep = PL5 ? st.E5 : st.E + ebase(pl);
    uint16_t* const Wp = PL5 ? st.wpre5 : st.wpre + ebase(pl);
    const uint32_t per = (pw + 63u) / 64u, w0 = lane * per;
    uint32_t sum = 0;
    for (uint32_t q = 0; q < per; ++q)
        if (w0 + q < pw) sum += (uint32_t)__popc(Ep[w0 + q] & mask);
    const uint32_t incl = wave_incl_sum(sum);
    uint32_t run = incl - sum;
    for (uint32_t q = 0; q < per; ++q)
        if (w0 + q < pw) {
            Wp[w0 + q] = (uint16_t)run;
            run += (uint32_t)__popc(Ep[w0 + q] & mask);
        }
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    if (lane == 0) sh.nexp = total;
}

template <int NT, typename V, bool BIG, bool LIST_LDS, bool PL5>
__device__ __forceinline__ void level_fill(Shared& sh, const Store<V>& st, uint32_t i, uint32_t t) {
    const uint32_t tid = threadIdx.x & (NT - 1);  // (NT = 64: the calling wavefront's lane)
    const uint32_t pl = i - 1, pn = 1u << (3 * pl);
    const uint32_t* const Ep = PL5 ? st.E5 : st.E + ebase(pl);
    const uint16_t* const Wp = PL5 ? st.wpre5 : st.wpre + ebase(pl);
    constexpr V NOTYET = Slot<V>::kNotYet;
    for (uint32_t q = tid; q < pn; q += NT) {
        const uint32_t bits = Ep[q >> 5] & (pn < 32 ? (1u << pn) - 1u : 0xFFFFFFFFu);
        const bool ex = (bits >> (q & 31)) & 1u;
        if (ex) {
            const uint32_t r = Wp[q >> 5] + (uint32_t)__popc(bits & ((1u << (q & 31)) - 1u));
            if (LIST_LDS) {
                st.list_l[r] = (uint16_t)q;
            } else {
                st.list_g[r] = (uint16_t)q;
                if (PL5) st.pval_g[r] = st.value5(q);
            }
        }
        if (!PL5 && i <= 4) {
            const V v = ex ? NOTYET : st.full[fbase(pl) + q];
            V* d = st.full + fbase(i) + 8 * q;
#pragma unroll
            for (int c = 0; c < 8; ++c) d[c] = v;
        }
    }
    if (i < t) {
        if (i <= 4) {
            for (uint32_t w = tid; w < ewords(i); w += NT) st.E[ebase(i) + w] = 0;
        } else {
            for (uint32_t w = tid; w < ewords(5); w += NT) st.E5[w] = 0;
        }
    }
    lsync<NT>();
}

// ------------------------------------------------------------ level passes
// 2-state automaton summary of a run of symbols for both entry states: f (bit
// e = exit state when entered in state e), and per entry state e the number of
// operations | the number of PALETTE_ADV operations << 16 (p0, p1).  A pass
// holds at most 8 symbols per thread, so both counts stay below 2^16.
struct RunSum {
    uint32_t f, p0, p1;
};
constexpr uint32_t kHalf = 0xFFFFu;

// the run `y` after the run `x`
__device__ __forceinline__ RunSum run_then(const RunSum& x, const RunSum& y) {
    RunSum r;
    r.f = fn_then(x.f, y.f);
    r.p0 = x.p0 + ((x.f & 1u) ? y.p1 : y.p0);
    r.p1 = x.p1 + ((x.f & 2u) ? y.p1 : y.p0);
    return r;
}

template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ RunSum dpp_run(const RunSum& x) {
    return RunSum{dpp<CTRL, ROWS>(kFnId, x.f), dpp<CTRL, ROWS>(0u, x.p0), dpp<CTRL, ROWS>(0u, x.p1)};
}

// bit 4q set where nibble q of lo3 (nibbles of 3 bits) equals c (c given in every nibble)
__device__ __forceinline__ uint32_t nib_eq(uint32_t lo3, uint32_t c) {
    const uint32_t t = lo3 ^ c;
    return ~(t | (t >> 1) | (t >> 2)) & 0x11111111u;
}

// inclusive scan of run summaries over the wavefront (lane 0 first)
__device__ __forceinline__ RunSum wave_scan_run(RunSum x) {
    x = run_then(dpp_run<kDppRowShr + 1>(x), x);
    x = run_then(dpp_run<kDppRowShr + 2>(x), x);
    x = run_then(dpp_run<kDppRowShr + 4>(x), x);
    x = run_then(dpp_run<kDppRowShr + 8>(x), x);
    x = run_then(dpp_run<kDppBcast15, 0xA>(x), x);
    x = run_then(dpp_run<kDppBcast31, 0xC>(x), x);
    return x;
}

// KIND 0: full level (i <= 4), 1: compact level 5, 2: level 6 in the output.
//
// A pass gives every thread R consecutive symbols (R = 1, 2, 4 or 8 per level:
// the fewest that still fill one pass, so small levels do not serialise).
// Each thread summarises its R symbols for both automaton entry states; a
// wavefront scan and a scan of the waves' totals give each thread its entry
// state, its first operation rank and its first palette (ADV) rank; then each
// thread decodes its own operations in order.  References to nodes decoded in
// the same pass are resolved after it.
template <int NT, int KIND, typename V, bool BIG, bool LIST_LDS>
__device__ __forceinline__ void level_passes(const Params& P, Shared& sh, const Store<V>& st, const uint8_t* nib, uint32_t i,
                             uint32_t expected, uint32_t& adv_done, uint32_t& pbuf) {
    constexpr uint32_t NW = NT / 64;
    const uint32_t tid = threadIdx.x & (NT - 1), lane = lane_id(), wave = tid >> 6;
    const uint32_t t = sh.h.t, pc = sh.h.pc;
    const uint32_t nodes = 1u << (3 * i);
    // final flag of this level's slots (level 6 slots are always u32)
    constexpr uint32_t FIN = KIND == 2 ? 0x80000000u : (uint32_t)Slot<V>::kFinal;
    constexpr uint32_t IDX = FIN - 1u;
    constexpr uint32_t VIDX = (uint32_t)Slot<V>::kIdx;
    V* const full_i = st.full + (KIND == 0 ? fbase(i) : 0u);
    const V* const full_p = st.full + (i ? fbase(i <= 5 ? i - 1 : 4) : 0u);
    // expansion bits of this level (needed when t > i): LDS for full levels, scratch for level 5
    uint32_t* const Ei_l = KIND == 0 && i < t ? st.E + ebase(i) : nullptr;
    uint32_t* const Ei_g = KIND == 1 && i < t ? st.E5 : nullptr;
    const uint32_t mx = 0x09249249u & (nodes - 1u), my = mx << 1, mz = mx << 2;
    const uint32_t s0 = i ? sh.h.sym_end[i - 1] : 0u, s1 = sh.h.sym_end[i];
    const uint32_t* const nib32 = (const uint32_t*)nib;
    const uint32_t n_sym = s1 - s0;
    const uint32_t lr = n_sym <= NT ? 0u : n_sym <= 2u * NT ? 1u : n_sym <= 4u * NT ? 2u : 3u;  // log2 R
    const uint32_t g_first = s0 >> lr, g_last = n_sym ? (s1 - 1u) >> lr : 0u;
    const uint32_t n_groups = n_sym ? g_last - g_first + 1u : 0u;
    const uint32_t w_last = n_sym ? (s1 - 1u) >> 3 : 0u;  // last word holding a symbol of the level
    // slot of the operation of rank k whose node is p
    auto slot_of = [&](uint32_t k, uint32_t p) -> uint32_t { return KIND == 0 ? p : KIND == 1 ? k : vox6(p); };
    auto parent_of = [&](uint32_t k) -> uint32_t {
        return i ? (LIST_LDS ? (uint32_t)st.list_l[k >> 3] : (uint32_t)st.list_g[k >> 3]) : 0u;
    };
    auto read_slot = [&](uint32_t x) -> uint32_t {
        return KIND == 0 ? (uint32_t)full_i[x] : KIND == 1 ? (uint32_t)st.c5[x] : st.out6[(uint64_t)x * st.lb4];
    };
    auto write_slot = [&](uint32_t x, uint32_t v) {
        if (KIND == 0) full_i[x] = (V)v;
        else if (KIND == 1) st.c5[x] = (V)v;
        else st.out6[(uint64_t)x * st.lb4] = v;
    };
    uint32_t carry = 0, k_done = 0;
    bool bad = false;
    // each thread reads the two words holding its group of R symbols and what
    // follows it (delta entries), one pass ahead, at clamped indices: no branch
    // around the loads, so nothing waits for them before their use
    uint32_t nlo = 0, nhi = 0;
    if (n_groups) {
        const uint32_t w = ((g_first + tid) << lr) >> 3;
        nlo = nib32[min(w, w_last)];
        nhi = nib32[min(w + 1u, w_last)];
    }
    for (uint32_t pg = 0; pg < n_groups; pg += NT) {
        const uint32_t g = g_first + pg + tid, j0 = g << lr, pb = pbuf;
        // symbols j0, j0 + 1, ... from bit 0 on (16 - (j0 & 7) of them)
        const uint64_t win = ((((uint64_t)nhi) << 32) | nlo) >> (4u * (j0 & 7u));
        const uint32_t word = (uint32_t)win, avail = 16u - (j0 & 7u);
        {
            const uint32_t w = ((g + NT) << lr) >> 3;
            nlo = nib32[min(w, w_last)];
            nhi = nib32[min(w + 1u, w_last)];
        }
        // Masks over the thread's symbols, bit 4q for symbol j0 + q ("nibble
        // masks"): V4 the symbols of this group that belong to the level
        uint32_t V4 = 0;
        if (g <= g_last) {
            const uint32_t lo = s0 > j0 ? s0 - j0 : 0u, hi = min(s1 - j0, 1u << lr);
            V4 = (hi >= 8u ? 0xFFFFFFFFu : (1u << (4u * hi)) - 1u) & ~((1u << (4u * lo)) - 1u) & 0x11111111u;
        }
        const uint32_t lo3 = word & 0x77777777u, C4 = (word >> 3) & 0x11111111u;
        // the automaton state before each symbol for entry state 0 (S0) and 1 (S1):
        // state 1 = inside a delta chain (the symbol is a delta entry)
        uint32_t S0 = 0, S1 = 0;
        // a wave holding no symbol of the level skips its summary, scan and decode
        // (it still takes part in the barriers and the waves' scan)
        const bool wave_on = g_first + pg + 64u * wave <= g_last;
        RunSum incl{kFnId, 0u, 0u}, excl{kFnId, 0u, 0u};
        if (wave_on) {
            // a symbol outside the level keeps the state: DELTA code off, continuation on
            const uint32_t Dv = nib_eq(lo3, 0x66666666u) & V4, Cv = C4 | (~V4 & 0x11111111u);
            uint32_t e0 = 0, e1 = 1;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint32_t d = (Dv >> (4 * q)) & 1u, c = (Cv >> (4 * q)) & 1u;
                S0 |= e0 << (4 * q);
                S1 |= e1 << (4 * q);
                e0 = e0 ? c : d;
                e1 = e1 ? c : d;
            }
            const uint32_t A4 = nib_eq(lo3, 0x44444444u), O0 = V4 & ~S0, O1 = V4 & ~S1;
            const RunSum x{e0 | (e1 << 1), (uint32_t)__popc(O0) | ((uint32_t)__popc(O0 & A4) << 16),
                           (uint32_t)__popc(O1) | ((uint32_t)__popc(O1 & A4) << 16)};
            incl = wave_scan_run(x);
            excl = dpp_run<kDppWaveShr1>(incl);
        }
        // this wave's entry state and packed operation / ADV bases for both entry
        // states (wf, wp0, wp1), and the pass totals (tf, tp0, tp1): one wavefront
        // has them from its own scan
        uint32_t wf = kFnId, wp0 = 0, wp1 = 0, tf, tp0, tp1;
        if (NW == 1) {
            tf = (uint32_t)__builtin_amdgcn_readlane((int)incl.f, 63);
            tp0 = (uint32_t)__builtin_amdgcn_readlane((int)incl.p0, 63);
            tp1 = (uint32_t)__builtin_amdgcn_readlane((int)incl.p1, 63);
        } else {
            if (lane == 63) {
                uint32_t* pub = sh.pub[pb][wave];
                pub[0] = incl.f;
                pub[1] = incl.p0;
                pub[2] = incl.p1;
            }
            lsync<NT>();
            // the waves' totals, scanned over the first NW lanes (one row of 16)
            RunSum wt{kFnId, 0u, 0u};
            if (lane < NW) wt = RunSum{sh.pub[pb][lane][0], sh.pub[pb][lane][1], sh.pub[pb][lane][2]};
            wt = run_then(dpp_run<kDppRowShr + 1>(wt), wt);
            wt = run_then(dpp_run<kDppRowShr + 2>(wt), wt);
            wt = run_then(dpp_run<kDppRowShr + 4>(wt), wt);
            wt = run_then(dpp_run<kDppRowShr + 8>(wt), wt);
            const RunSum we = dpp_run<kDppRowShr + 1>(wt);
            wf = (uint32_t)__builtin_amdgcn_readlane((int)we.f, (int)wave);
            wp0 = (uint32_t)__builtin_amdgcn_readlane((int)we.p0, (int)wave);
            wp1 = (uint32_t)__builtin_amdgcn_readlane((int)we.p1, (int)wave);
            tf = (uint32_t)__builtin_amdgcn_readlane((int)wt.f, (int)(NW - 1));
            tp0 = (uint32_t)__builtin_amdgcn_readlane((int)wt.p0, (int)(NW - 1));
            tp1 = (uint32_t)__builtin_amdgcn_readlane((int)wt.p1, (int)(NW - 1));
        }
        const uint32_t my_e = (wf >> carry) & 1u;
        const uint32_t wp = carry ? wp1 : wp0, tp = carry ? tp1 : tp0;
        const uint32_t my_kb = k_done + (wp & kHalf);
        const uint32_t my_ab = adv_done + (wp >> 16);
        const uint32_t k0 = k_done;
        k_done += tp & kHalf;
        adv_done += tp >> 16;
        carry = (tf >> carry) & 1u;
        pbuf ^= 1u;
        const uint32_t ls = (excl.f >> my_e) & 1u;
        // this thread's first operation rank and first ADV rank
        const uint32_t lp = my_e ? excl.p1 : excl.p0;
        const uint32_t k_first = my_kb + (lp & kHalf);
        const uint32_t a_first = my_ab + (lp >> 16);
        uint32_t opm = 0, refm = 0;
        if (wave_on) {
            // classify the thread's symbols from its entry state (nibble masks):
            // operations, and among them ADVs, palette (ADV, LAST, DELTA, invalid code:
            // bit 2 of the code), parent and neighbour operations, and stop bits; each
            // kind is then decoded in a loop of its own, so a wavefront runs one kind's
            // code at a time
            opm = V4 & ~(ls ? S1 : S0);
            const uint32_t advm = opm & nib_eq(lo3, 0x44444444u);
            uint32_t palm = opm & (word >> 2) & 0x11111111u;
            uint32_t parm = opm & nib_eq(lo3, 0u);
            uint32_t nbm = opm & ~palm & ~parm;
            uint32_t stopm = opm & C4;
            // operations past the level's node count are an error and write nothing
            if (k_first + (uint32_t)__popc(opm) > expected) {
                bad = true;
                uint32_t keep = expected > k_first ? expected - k_first : 0u, km = 0;
                for (uint32_t m = opm; m && keep; m &= m - 1u, --keep) km |= m & (0u - m);
                palm &= km;
                parm &= km;
                nbm &= km;
                stopm |= ~km;
            }
            // rank of the operation at bit position b = 4q, its ADV rank, and its node
            auto k_at = [&](uint32_t b) -> uint32_t { return k_first + (uint32_t)__popc(opm & ((1u << b) - 1u)); };
            auto a_at = [&](uint32_t b) -> uint32_t { return a_first + (uint32_t)__popc(advm & ((1u << b) - 1u)); };
            auto node_of = [&](uint32_t kq) -> uint32_t { return i ? ((parent_of(kq) << 3) | (kq & 7u)) : 0u; };
            // palette: ADV -> a, LAST -> a - 1, DELTA -> a - delta, the entries following in the window
            for (uint32_t m = palm; m; m &= m - 1u) {
                const uint32_t b = (uint32_t)__builtin_ctz(m), q = b >> 2, kq = k_at(b), aq = a_at(b);
                const uint32_t op = (word >> b) & 7u;
                uint32_t v = FIN;
                bool err = false;
                if (op == kAdv) {
                    if (aq >= pc) err = true;
                    else v = FIN | aq;
                } else if (op == kLast) {
                    if (aq == 0) err = true;
                    else v = FIN | (aq - 1u);
                } else if (op == kDelta) {
                    uint32_t d = 0, mm = q + 1u, en = 8;
                    while (en & 8u) {
                        const uint32_t jj = j0 + mm;
                        if (jj >= s1) {
                            err = true;
                            break;
                        }
                        en = mm < avail ? (uint32_t)(win >> (4 * mm)) & 15u : (nib[jj >> 1] >> (4 * (jj & 1))) & 15u;
                        d = d >= (1u << 29) ? 0xFFFFFFFFu : ((d << 3) | (en & 7u));
                        ++mm;
                    }
                    if (!err) {
                        if (d == 0 || d > aq) err = true;
                        else v = FIN | (aq - d);
                    }
                } else {
                    err = true;
                }
                if (err) {
                    bad = true;
                    v = FIN;
                }
                // written even after an error, so that a later lookup never meets an unset slot
                write_slot(slot_of(kq, KIND == 1 ? 0u : node_of(kq)), v);
            }
            // parent copies
            for (uint32_t m = parm; m; m &= m - 1u) {
                const uint32_t kq = k_at((uint32_t)__builtin_ctz(m));
                const uint32_t pn = parent_of(kq);
                uint32_t v = FIN;
                if (i == 0) bad = true;
                else if (KIND == 2) v = (st.pval_g[kq >> 3] & VIDX) | FIN;
                else v = full_p[pn];
                write_slot(slot_of(kq, i ? ((pn << 3) | (kq & 7u)) : 0u), v);
            }
            // neighbour copies: an implied target holds its parent's value, an explicit one of
            // an earlier pass its final value, one of this pass becomes a reference
            for (uint32_t m = nbm; m; m &= m - 1u) {
                const uint32_t b = (uint32_t)__builtin_ctz(m), kq = k_at(b);
                const uint32_t op = (word >> b) & 7u;
                const uint32_t p = node_of(kq);
                const uint32_t am = mx << ((op - 1u) & 3u);  // NX, NY, NZ: the x, y or z bits
                uint32_t v = FIN;
                if (KIND == 1) {
                    // level 5 without branches: the target's implied value (its level-4
                    // parent's) and its explicit slot are both read, then selected; a
                    // node at coordinate 0 (no neighbour) reads in-range garbage
                    const uint32_t pa = p & am;
                    const uint32_t tn = ((pa - 1u) & am) | (p & ~am), tq = tn >> 3;
                    const uint32_t ew = st.E[ebase(4) + (tq >> 5)];
                    const uint32_t kt = 8u * (st.wpre[ebase(4) + (tq >> 5)] +
                                              (uint32_t)__popc(ew & ((1u << (tq & 31)) - 1u))) + (tn & 7u);
                    const uint32_t implied = full_p[tq], got = st.c5[kt < k0 ? kt : 0u];
                    v = !pa ? FIN : !((ew >> (tq & 31)) & 1u) ? implied : kt < k0 ? got : kt;
                    bad = bad || !pa;
                    refm |= (v & FIN) ? 0u : (1u << b);
                } else if (!(p & am)) {
                    bad = true;
                } else {
                    const uint32_t tn = (((p & am) - 1u) & am) | (p & ~am);
                    if (KIND == 0) {
                        v = full_i[tn];
                        if (v == (uint32_t)Slot<V>::kNotYet) v = tn;
                    } else {
                        const uint32_t tq = tn >> 3;
                        if (KIND == 1 ? !st.ebit(4, tq) : !st.ebit5(tq)) {
                            v = KIND == 1 ? (uint32_t)full_p[tq] : ((st.value5(tq) & VIDX) | FIN);
                        } else {
                            const uint32_t kt = 8 * (KIND == 1 ? st.rank(4, tq) : st.rank5(tq)) + (tn & 7u);
                            const uint32_t ti = KIND == 1 ? kt : vox6(tn);
                            v = kt < k0 ? read_slot(ti) : ti;
                        }
                    }
                    refm |= (v & FIN) ? 0u : (1u << b);
                }
                write_slot(slot_of(kq, p), v);
            }
            // expansion bits of this level's operations without a stop bit
            if (Ei_l || Ei_g) {
                for (uint32_t m = opm & ~stopm; m; m &= m - 1u) {
                    const uint32_t p = node_of(k_at((uint32_t)__builtin_ctz(m)));
                    if (Ei_l) atomicOr(Ei_l + (p >> 5), 1u << (p & 31));
                    if (Ei_g) atomicOr(Ei_g + (p >> 5), 1u << (p & 31));
                }
            }
        }
        lsync<NT>();
        // references within the pass: chase to a final value (targets precede
        // their sources, so every chain ends within the pass's operations)
        for (uint32_t m = refm; m; m &= m - 1u) {
            const uint32_t b = (uint32_t)__builtin_ctz(m);
            const uint32_t kq = k_first + (uint32_t)__popc(opm & ((1u << b) - 1u));
            const uint32_t pq = i ? ((parent_of(kq) << 3) | (kq & 7u)) : 0u;
            const uint32_t me = slot_of(kq, pq);
            const uint32_t lim = KIND == 0 ? nodes : KIND == 1 ? k_done : (1u << 18);
            uint32_t v = read_slot(me), it = 0;
            while (!(v & FIN)) {
                if ((v & IDX) >= lim || ++it > 8 * NT) {
                    bad = true;
                    v = FIN;
                    break;
                }
                v = read_slot(v & IDX);
            }
            write_slot(me, v);
        }
    }
    if (bad) atomicOr(&sh.err, 1u);
    if ((k_done != expected || carry != 0) && tid == 0) sh.err = 1u;
}

// Levels 0..min(t, last) (last = 2: at most 73 nodes; 3: 585) decoded by the
// calling wavefront alone, with wave barriers; then the parent prefix of the
// next level when the cube has one, and the ADV count in sh.adv.
template <typename V, bool BIG, bool LIST_LDS>
__device__ __forceinline__ void small_levels(const Params& P, Shared& sh, const Store<V>& st, const uint8_t* nib,
                                             uint32_t last) {
    const uint32_t t = sh.h.t, tw = t < last ? t : last, lane = lane_id();
    uint32_t adv_done = 0, pbuf = 0;
    for (uint32_t i = 0; i <= tw; ++i) {
        uint32_t expected = 1;
        if (i == 0) {
            // Level 0 is one node whose only valid operation is PALETTE_ADV (entry
            // 0), with or without a stop bit: take that case directly; anything
            // else goes through the general pass, which reports the error.
            const uint32_t s0 = nib[0] & 15u;
            if (sh.h.sym_end[0] == 1u && (s0 & 7u) == kAdv && sh.h.pc > 0u) {
                if (lane == 0) {
                    st.full[fbase(0)] = (V)Slot<V>::kFinal;
                    if (t > 0) st.E[ebase(0)] = (s0 & 8u) ? 0u : 1u;
                }
                adv_done = 1;
                lsync<64>();
                continue;
            }
            if (t > 0 && lane == 0) st.E[ebase(0)] = 0;
            lsync<64>();
        } else {
            level_prefix<V, false>(sh, st, i - 1);
            lsync<64>();
            expected = 8 * sh.nexp;
            level_fill<64, V, BIG, LIST_LDS, false>(sh, st, i, t);
        }
        level_passes<64, 0, V, BIG, LIST_LDS>(P, sh, st, nib, i, expected, adv_done, pbuf);
        lsync<64>();
        if (sh.err) break;
    }
    if (!sh.err && t > tw) level_prefix<V, false>(sh, st, tw);
    if (lane == 0) sh.adv = adv_done;
}

// Decode levels 0..t; on return all slots of level t are final unless sh.err.
// Levels 0..2 are decoded by one wavefront (wavefront 0 here; with `small_upto`
// >= 0, levels 0..min(t, small_upto) were decoded during the rANS decode), the
// other wavefronts wait at the work-group barrier that follows.  From then on,
// all threads decode; wavefront 0 computes the next level's parent prefix after
// a level's last pass, before the barrier that ends it.
template <int NT, typename V, bool BIG, bool LIST_LDS>
__device__ __forceinline__ void decode_levels(const Params& P, Shared& sh, const Store<V>& st, const uint8_t* nib,
                                              Ahead& ah, int small_upto) {
    const uint32_t t = sh.h.t, wave = threadIdx.x >> 6;
    const uint32_t last = small_upto < 0 ? 2u : (uint32_t)small_upto;
    const uint32_t tw = t < last ? t : last;  // last level of the single wavefront
    if (small_upto < 0) {
        if (wave == 0) {
            small_levels<V, BIG, LIST_LDS>(P, sh, st, nib, 2u);
        } else if (threadIdx.x == NT - 64 && !ah.done) {
            parse_ahead(P, sh.hn, ah.jt);
            ah.done = true;
        }
        __syncthreads();
    }
    if (sh.err) return;
    uint32_t adv_done = sh.adv, pbuf = 0;
    for (uint32_t i = tw + 1; i <= t; ++i) {
        const uint32_t expected = 8 * sh.nexp;
        if (i <= 5) level_fill<NT, V, BIG, LIST_LDS, false>(sh, st, i, t);
        else level_fill<NT, V, BIG, false, true>(sh, st, i, t);
        if (i <= 4) level_passes<NT, 0, V, BIG, LIST_LDS>(P, sh, st, nib, i, expected, adv_done, pbuf);
        else if (i == 5) level_passes<NT, 1, V, BIG, LIST_LDS>(P, sh, st, nib, i, expected, adv_done, pbuf);
        else level_passes<NT, 2, V, BIG, false>(P, sh, st, nib, i, expected, adv_done, pbuf);
        // the level's bitmap is final after its last pass: the next level's parent prefix
        if (i < t && wave == 0) {
            if (i == 5) level_prefix<V, true>(sh, st, i);
            else level_prefix<V, false>(sh, st, i);
        }
        __syncthreads();
        if (sh.err) return;
    }
    if (t == sh.h.L && adv_done != sh.h.pc && threadIdx.x == 0) sh.err = 1u;
    __syncthreads();
}

// ------------------------------------------------------------------ output
// Decoded labels are written once and not read again by the kernel: vector
// stores carry the non-temporal hint, so they do not displace the records and
// symbols other work-groups still read from L2.
typedef uint32_t u32x4 __attribute__((vector_size(16)));
__device__ __forceinline__ void st16_nt(void* p, uint4 v) {
    const u32x4 w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, (u32x4*)p);
}

template <typename LT>
__device__ __forceinline__ void store4(LT* o, LT a, LT b, LT c, LT d, bool vec) {
    if (sizeof(LT) == 4) {
        if (vec) st16_nt(o, make_uint4((uint32_t)a, (uint32_t)b, (uint32_t)c, (uint32_t)d));
        else {
            o[0] = a;
            o[1] = b;
            o[2] = c;
            o[3] = d;
        }
    } else {
        if (vec) {
            st16_nt((uint4*)o, make_uint4((uint32_t)a, (uint32_t)((uint64_t)a >> 32), (uint32_t)b, (uint32_t)((uint64_t)b >> 32)));
            st16_nt((uint4*)o + 1, make_uint4((uint32_t)c, (uint32_t)((uint64_t)c >> 32), (uint32_t)d, (uint32_t)((uint64_t)d >> 32)));
        } else {
            o[0] = a;
            o[1] = b;
            o[2] = c;
            o[3] = d;
        }
    }
}

template <int NT>
__device__ __forceinline__ void zero_output(const Params& P, const TaskHdr& h) {
    const uint32_t t = h.t;
    const uint64_t unit = P.pal_bits ? 4u : P.label_bytes;
    uint8_t* out = P.out + h.out_off * unit;
    const uint64_t bytes = out_units(1ull << (3 * t), P.pal_bits) * unit;
    if (((uintptr_t)out & 15u) == 0 && (bytes & 15u) == 0) {
        for (uint64_t u = threadIdx.x; u < bytes / 16; u += NT) ((uint4*)out)[u] = make_uint4(0, 0, 0, 0);
    } else {
        for (uint64_t u = threadIdx.x; u < bytes / 4; u += NT) ((uint32_t*)out)[u] = 0u;
    }
}

// Labels of level t (all slots final) as an S^3 x-fastest cube.  Full levels
// voxel by voxel (4 per thread); levels 5 and 6 by pairs of 2x2x2 blocks
// along x under two level-(t-1) nodes: a node that does not expand gives its
// value to its 8 children, an expanding one has 8 explicit children.
template <int NT, typename V, typename LT, bool PAL_LDS>
__device__ __forceinline__ void write_labels(const Params& P, Shared& sh, const Store<V>& st) {
    const TaskHdr& h = sh.h;
    const uint32_t t = h.t, S = 1u << t, pc = h.pc;
    constexpr uint32_t VIDX = (uint32_t)Slot<V>::kIdx;
    LT* out = (LT*)(P.out + h.out_off * sizeof(LT));
    const LT* pal = PAL_LDS ? (const LT*)sh.U : (const LT*)(P.vol + h.pal_off);
    const bool vec = ((uintptr_t)out & (4 * sizeof(LT) - 1)) == 0;
    if (t <= 4) {
        const V* g = st.full + fbase(t);
        if (S < 4) {
            const uint32_t n = S * S * S;
            for (uint32_t v = threadIdx.x; v < n; v += NT) {
                const uint32_t x = v & (S - 1), y = (v >> t) & (S - 1), z = v >> (2 * t);
                const LT l = pal_get<LT, PAL_LDS>(pal, g[spread3(x) | (spread3(y) << 1) | (spread3(z) << 2)] & VIDX, pc);
                __builtin_nontemporal_store(l, out + v);
            }
            return;
        }
        const uint32_t units = (S * S * S) >> 2;
        for (uint32_t u = threadIdx.x; u < units; u += NT) {
            const uint32_t lin = u << 2;
            const uint32_t x = lin & (S - 1), y = (lin >> t) & (S - 1), z = lin >> (2 * t);
            const uint32_t m = spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
            store4<LT>(out + lin, pal_get<LT, PAL_LDS>(pal, g[m] & VIDX, pc), pal_get<LT, PAL_LDS>(pal, g[m + 1] & VIDX, pc),
                       pal_get<LT, PAL_LDS>(pal, g[m + 8] & VIDX, pc), pal_get<LT, PAL_LDS>(pal, g[m + 9] & VIDX, pc), vec);
        }
        return;
    }
    const uint32_t hb = t - 1, H = 1u << hb;  // parents per axis
    const uint32_t units = (H >> 1) * H * H;   // pairs of parents along x
    for (uint32_t u = threadIdx.x; u < units; u += NT) {
        const uint32_t px = u & ((H >> 1) - 1), qy = (u >> (hb - 1)) & (H - 1), qz = u >> (2 * hb - 1);
        const uint64_t e0 = ((uint64_t)(2 * qz) * S + 2 * qy) * S + 4 * px;
        // palette indices of the 8 children of each of the two nodes (child c = x | y << 1 | z << 2)
        uint32_t ix[2][8];
        const uint32_t q0 = spread3(2 * px) | (spread3(qy) << 1) | (spread3(qz) << 2);
#pragma unroll
        for (int hx = 0; hx < 2; ++hx) {
            const uint32_t q = q0 | (uint32_t)hx;  // the x neighbour differs in bit 0
            if (t == 5) {
                if (st.ebit(4, q)) {
                    const V* c = st.c5 + 8 * st.rank(4, q);
#pragma unroll
                    for (int ch = 0; ch < 8; ++ch) ix[hx][ch] = c[ch] & VIDX;
                } else {
                    const uint32_t v = st.full[fbase(4) + q] & VIDX;
#pragma unroll
                    for (int ch = 0; ch < 8; ++ch) ix[hx][ch] = v;
                }
            } else if (st.ebit5(q)) {
                const uint32_t* o6 = st.out6 + (e0 + 2 * hx) * st.lb4;
#pragma unroll
                for (int ch = 0; ch < 8; ++ch)
                    ix[hx][ch] = o6[((((ch >> 2) & 1) * S + ((ch >> 1) & 1)) * S + (ch & 1)) * st.lb4] & 0x7FFFFFFFu;
            } else {
                const uint32_t v = st.value5(q) & VIDX;
#pragma unroll
                for (int ch = 0; ch < 8; ++ch) ix[hx][ch] = v;
            }
        }
#pragma unroll
        for (int zy = 0; zy < 4; ++zy) {
            store4<LT>(out + e0 + ((uint64_t)(zy >> 1) * S + (zy & 1)) * S,
                       pal_get<LT, PAL_LDS>(pal, ix[0][2 * zy], pc), pal_get<LT, PAL_LDS>(pal, ix[0][2 * zy + 1], pc),
                       pal_get<LT, PAL_LDS>(pal, ix[1][2 * zy], pc), pal_get<LT, PAL_LDS>(pal, ix[1][2 * zy + 1], pc), vec);
        }
    }
}

// Cache-paletted output: the cube's palette indices, I bits each, floor(32/I)
// to a 32-bit word (voxel k, x fastest, in word k / e at bit (k mod e) * I).
// One thread per word; level 5 reaches a voxel's slot through its level-4
// parent, looked up once per pair of voxels along x.
template <int NT, typename V>
__device__ __forceinline__ void write_indices(const Params& P, Shared& sh, const Store<V>& st) {
    const TaskHdr& h = sh.h;
    const uint32_t t = h.t, S = 1u << t, bits = P.pal_bits, e = 32u / bits;
    constexpr uint32_t VIDX = (uint32_t)Slot<V>::kIdx;
    const uint32_t n = S * S * S, words = (n + e - 1u) / e;
    uint32_t* const out = (uint32_t*)P.out + h.out_off;
    for (uint32_t w = threadIdx.x; w < words; w += NT) {
        uint32_t acc = 0, last_q = 0xFFFFFFFFu, base = 0;
        bool expands = false;
        for (uint32_t q = 0; q < e; ++q) {
            const uint32_t v = w * e + q;
            if (v >= n) break;
            const uint32_t x = v & (S - 1u), y = (v >> t) & (S - 1u), z = v >> (2 * t);
            const uint32_t m = spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
            uint32_t idx;
            if (t <= 4) {
                idx = st.full[fbase(t) + m] & VIDX;
            } else {
                const uint32_t pq = m >> 3;
                if (pq != last_q) {
                    last_q = pq;
                    expands = st.ebit(4, pq);
                    base = expands ? 8u * st.rank(4, pq) : (uint32_t)st.full[fbase(4) + pq];
                }
                idx = (expands ? (uint32_t)st.c5[base + (m & 7u)] : base) & VIDX;
            }
            acc |= idx << (q * bits);
        }
        __builtin_nontemporal_store(acc, out + w);
    }
}

template <int NT, typename V>
__device__ __forceinline__ void write_output(const Params& P, Shared& sh, const Store<V>& st) {
    if (P.pal_bits) {
        write_indices<NT, V>(P, sh, st);
    } else if (P.label_bytes == 4) {
        if (sh.h.pal_lds && sh.h.t > 3) write_labels<NT, V, uint32_t, true>(P, sh, st);
        else write_labels<NT, V, uint32_t, false>(P, sh, st);
    } else {
        if (sh.h.pal_lds && sh.h.t > 3) write_labels<NT, V, uint64_t, true>(P, sh, st);
        else write_labels<NT, V, uint64_t, false>(P, sh, st);
    }
}

// ------------------------------------------------------------------ a task
template <typename V, bool BIG, bool C5G>
__device__ __forceinline__ Store<V> make_store(const Params& P, Shared& sh, uint16_t* slots_lds, uint8_t* scratch) {
    const TaskHdr& h = sh.h;
    Store<V> st;
    st.E = sh.E;
    st.wpre = sh.wpre;
    st.E5 = (uint32_t*)(scratch + kScrE5);
    st.wpre5 = (uint16_t*)(scratch + kScrWpre5);
    st.list_l = (uint16_t*)sh.U;
    st.list_g = (uint16_t*)(scratch + kScrList);
    st.pval_g = (uint32_t*)(scratch + kScrPval);
    st.lb4 = P.label_bytes / 4;
    st.out6 = (uint32_t*)(P.out + h.out_off * P.label_bytes);
    if (BIG) {
        st.full = (V*)(scratch + kScrFull);
        st.c5 = (V*)(scratch + kScrComp);
    } else {
        st.full = (V*)sh.G;
        st.c5 = C5G ? (V*)(scratch + kScrComp) : (V*)slots_lds;
    }
    return st;
}

template <int NT, typename V, bool BIG, bool C5G>
__device__ __forceinline__ void run_levels(const Params& P, Shared& sh, uint16_t* slots_lds, uint8_t* scratch, const uint8_t* nib,
                                           Ahead& ah, int small_upto) {
    const TaskHdr& h = sh.h;
    const Store<V> st = make_store<V, BIG, C5G>(P, sh, slots_lds, scratch);
    if (!BIG && h.t <= 5) decode_levels<NT, V, BIG, true>(P, sh, st, nib, ah, small_upto);
    else decode_levels<NT, V, BIG, false>(P, sh, st, nib, ah, small_upto);
    if (sh.err) return;
    // palette staging for the output pass (the parent list is no longer needed);
    // a cube of side <= 8 reads its few labels straight from the record
    if (h.pal_lds && !P.pal_bits && h.t > 3) {
        const uint32_t words = (h.pc * P.label_bytes + 3) / 4;
        const uint32_t* src = (const uint32_t*)(P.vol + h.pal_off);
        for (uint32_t w = threadIdx.x; w < words; w += NT) ((uint32_t*)sh.U)[w] = src[w];
        __syncthreads();
    }
    write_output<NT, V>(P, sh, st);
}

template <int NT>
__device__ __forceinline__ void decode_task(const Params& P, Shared& sh, uint16_t* slots_lds, uint8_t* scratch,
                                            Ahead& ah) {
    const TaskHdr& h = sh.h;
    if (h.status != kTaskOk) {
        if (h.status == kTaskCorrupt && h.write_ok) zero_output<NT>(P, h);
        return;
    }
    // The symbols (4 bits each) are read by the level passes as aligned 32-bit
    // words: from the work-group's scratch, or for a cube of side <= 16 (levels
    // 0..4, whose parent lists take at most 1 KiB) from the rest of the parent
    // list area when they fit there.
    constexpr uint32_t kListMax4 = 1024;
    const bool sym_lds = h.t <= 4 && (h.nsym + 1u) / 2u + 4u <= kUBytes - kListMax4;
    uint8_t* const nib = sym_lds ? sh.U + kListMax4 : scratch + kScrSym;
    bool tab_used = false;
    int small_upto = -1;  // last level decoded during the rANS decode
    if (h.coder == kRaw4) {
        const uint32_t bytes = (h.nsym + 1u) / 2u, words = bytes / 4u;
        const uint32_t* src = (const uint32_t*)(P.vol + h.pay_off);
        for (uint32_t w = threadIdx.x; w < words; w += NT) ((uint32_t*)nib)[w] = src[w];
        for (uint32_t b = 4u * words + threadIdx.x; b < bytes; b += NT) nib[b] = P.vol[h.pay_off + b];
        __syncthreads();
    } else {
        // the rANS table sits in the last 16 KiB of the slot area until level 5
        // of a fast-path task overwrites it (later tasks find it there until
        // then); the grids, parent list and the rest of the slot area before it
        // can stage the record's words and the decoded symbols
        uint8_t* const stage = (uint8_t*)sh.G;
        const uint32_t stage_bytes = (uint32_t)(sizeof(sh.G) + sizeof(sh.U)) + 2u * P.cap16 - 4u * kRansM;
        uint32_t* tab = (uint32_t*)(stage + stage_bytes);
        tab_used = true;
        if (!sh.tab_ok) {
            const uint4* src = (const uint4*)P.rans_tab;
            for (uint32_t w = threadIdx.x; w < kRansM / 4; w += NT) ((uint4*)tab)[w] = src[w];
            __syncthreads();
        }
        const uint32_t G = ((1u << h.log2W) + 63u) / 64u, tw = h.gstart[G - 1] + h.gw[G - 1];
        const uint32_t words_bytes = (2u * tw + 15u) & ~15u;
        const uint32_t sym_bytes = ((h.nsym + 1u) / 2u + 3u) / 4u * 4u;
        // symbols bound for the parent list area: the staged words must end before it
        const uint32_t u_at = (uint32_t)(offsetof(Shared, U) - offsetof(Shared, G));
        const uint32_t nl_at = u_at + kListMax4;
        // Overlap, for a fast-path cube with a level 3 whose lane groups leave a
        // wavefront free: words staged after the grids of levels 0..3, symbols in
        // the parent-list area when they are read there, else at the end of the
        // stage (clear of the level 1..3 parent lists).  Wavefronts
        // 0..G-1 decode the lane groups, wavefront G decodes levels 0..2 (0..3 for
        // a cube with a level 5, whose rounds last long enough) as soon as every
        // group is past their symbols, and the last wavefront, when it is not G,
        // parses the next task.
        constexpr uint32_t kLoGrid = 1280;  // bytes of the level 0..3 grids (1184), rounded up
        const uint32_t G1 = ((1u << h.log2W) + 63u) / 64u;
        // (two or more lanes: a round writes whole bytes of symbol pairs)
        const bool overlap = G1 < NT / 64 && h.log2W >= 1u && !h.big && h.t >= 3 && h.t <= 5 &&
                             kLoGrid + words_bytes <= u_at && (sym_lds || sym_bytes + u_at + 160u <= stage_bytes);
        if (overlap) {
            const uint32_t wave = threadIdx.x >> 6;
            uint16_t* const wl = (uint16_t*)(stage + kLoGrid);
            uint8_t* const nl = sym_lds ? nib : stage + ((stage_bytes - sym_bytes) & ~15u);
            if (threadIdx.x < 4) sh.prog[threadIdx.x] = 0;
            const uint32_t x0 = rans_stage_words<NT>(P, h, wl);
            __syncthreads();
            const uint32_t last = h.t >= 5 ? 3u : 2u;
            const uint32_t need = h.sym_end[last];
            if (wave < G1) {
                rans_rounds<NT>(P, sh, tab, wl, nl, x0, need ? need : 1u);
            } else if (wave == G1) {
                // bounded: every group publishes ~0 when its rounds end
                for (uint32_t g = 0; g < G1; ++g)
                    while (__hip_atomic_load(&sh.prog[g], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < need)
                        __builtin_amdgcn_s_sleep(1);
                small_levels<uint16_t, false, true>(P, sh, make_store<uint16_t, false, false>(P, sh, slots_lds, scratch), nl, last);
            } else if (threadIdx.x == NT - 64 && !ah.done) {
                parse_ahead(P, sh.hn, ah.jt);
                ah.done = true;
            }
            __syncthreads();
            if (!sym_lds) {
                const uint32_t nw = ((h.nsym + 1u) / 2u + 3u) / 4u;
                for (uint32_t q = threadIdx.x; q < nw; q += NT) ((uint32_t*)nib)[q] = ((const uint32_t*)nl)[q];
            }
            small_upto = (int)last;
        } else if (sym_lds && words_bytes <= nl_at) rans_decode_lds<NT>(P, sh, tab, stage, nib, nullptr);
        else if (!sym_lds && words_bytes + sym_bytes <= stage_bytes)
            rans_decode_lds<NT>(P, sh, tab, stage, stage + words_bytes, nib);
        else rans_decode<NT>(P, sh, tab, nib);
        __syncthreads();
    }
    // level 5 of a fast-path task overwrites the table
    const bool tab_lost = !h.big && !h.c5g && h.t >= 5;
    if (!sh.err) {
        if (h.big) run_levels<NT, uint32_t, true, false>(P, sh, slots_lds, scratch, nib, ah, small_upto);
        else if (h.c5g) run_levels<NT, uint16_t, false, true>(P, sh, slots_lds, scratch, nib, ah, small_upto);
        else run_levels<NT, uint16_t, false, false>(P, sh, slots_lds, scratch, nib, ah, small_upto);
    }
    __syncthreads();
    if (sh.err) {
        if (threadIdx.x == 0) sh.h.status = kTaskCorrupt;
        zero_output<NT>(P, h);
    }
    // (read again only after the task loop's next barriers)
    if (threadIdx.x == 0) sh.tab_ok = tab_lost ? 0u : tab_used ? 1u : sh.tab_ok;
}

// at least 4 waves per SIMD: 128 VGPRs per lane at most
template <int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) decode_kernel(Params P) {
    extern __shared__ uint8_t dyn_smem[];
    Shared& sh = *reinterpret_cast<Shared*>(dyn_smem);
    uint16_t* slots_lds = reinterpret_cast<uint16_t*>(dyn_smem + sizeof(Shared));
    const uint32_t tid = threadIdx.x;
    uint8_t* scratch = P.scratch + (uint64_t)blockIdx.x * P.scratch_stride;
    // lane 0 of the last wavefront claims and parses the next task while the
    // current one is decoded (the atomic's and the header loads' latency hide
    // behind the decode)
    constexpr uint32_t PT = NT - 64;
    Ahead ah{0u, true};
    if (tid == PT) {
        const uint32_t j0 = P.queue ? atomicAdd(P.queue, 1u) : P.task0 + blockIdx.x;
        parse_ahead(P, sh.hn, j0);
        ah.jt = j0 < P.n_tasks ? j0 : P.n_tasks;
    }
    if (tid == 0) sh.tab_ok = 0;
    for (;;) {
        __syncthreads();  // sh.hn is parsed, the last task's status written
        if (tid < sizeof(TaskHdr) / 4) ((uint32_t*)&sh.h)[tid] = ((const uint32_t*)&sh.hn)[tid];
        if (tid == 0) sh.err = 0;
        __syncthreads();
        const uint32_t task = sh.h.task;
        if (task == 0xFFFFFFFFu) break;
        if (tid == PT) {
            ah.jt = P.queue && ah.jt < P.n_tasks ? atomicAdd(P.queue, 1u) : P.n_tasks;
            ah.done = false;
        }
        decode_task<NT>(P, sh, slots_lds, scratch, ah);
        if (tid == PT && !ah.done) {
            parse_ahead(P, sh.hn, ah.jt);
            ah.done = true;
        }
        if (tid == 0 && P.status) P.status[task] = sh.h.status;
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

// Lanes of one wavefront grouped by class: for every distinct class c among
// the lanes with c < 64, f(c, mask of the lanes holding it) runs once, with
// the lowest such lane as the leader.  One atomic per (wavefront, class)
// instead of one per task keeps the cost sort free of same-address contention.
template <typename F>
__device__ __forceinline__ void for_each_class(uint32_t c, F f) {
    uint64_t left = __ballot(c < 64u);
    while (left) {
        const uint32_t lead = (uint32_t)__builtin_ctzll(left);
        const uint32_t cc = (uint32_t)__builtin_amdgcn_readlane((int)c, (int)lead);
        const uint64_t m = __ballot(c == cc);
        f(cc, m, lead);
        left &= ~m;
    }
}

// Task cost classes for a decreasing-cost pop order: the class of a task is
// floor(log2(record bytes + output bytes + 1)); also the class histogram.  256 threads per block.
__global__ void __launch_bounds__(256) cost_class_kernel(Params P, uint32_t* cls, uint32_t* hist) {
    __shared__ uint32_t cnt[64];
    const uint32_t tid = threadIdx.x, j = blockIdx.x * 256 + tid, lane = lane_id();
    if (tid < 64) cnt[tid] = 0;
    __syncthreads();
    uint32_t c = 64;
    if (j < P.n_tasks) {
        uint64_t rec;
        const uint32_t t = task_t(P, j, &rec);
        const uint64_t unit = P.pal_bits ? 4u : P.label_bytes;
        const uint64_t cost = rec + (t <= kMaxLog2b ? out_units((uint64_t)1 << (3 * t), P.pal_bits) * unit : 0) + 1;
        c = 63u - (uint32_t)__clzll(cost);
        cls[j] = c;
    }
    for_each_class(c, [&](uint32_t cc, uint64_t m, uint32_t lead) {
        if (lane == lead) atomicAdd(&cnt[cc], (uint32_t)__popcll(m));
    });
    __syncthreads();
    if (tid < 64 && cnt[tid]) atomicAdd(&hist[tid], cnt[tid]);
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

// Scatter task indices to their class's range of the order: a block reserves
// one range per class it holds, and ranks its lanes within it by wavefront
// and lane.  256 threads per block.
__global__ void __launch_bounds__(256) cost_scatter_kernel(uint32_t n, const uint32_t* cls, uint32_t* cursor, uint32_t* order) {
    __shared__ uint32_t cnt[4][64];
    __shared__ uint32_t base[64];
    const uint32_t tid = threadIdx.x, j = blockIdx.x * 256 + tid, lane = lane_id(), wave = tid >> 6;
    cnt[wave][lane] = 0;
    __syncthreads();
    const uint32_t c = j < n ? cls[j] : 64u;
    uint32_t rank = 0;
    for_each_class(c, [&](uint32_t cc, uint64_t m, uint32_t lead) {
        if (c == cc) rank = mbcnt(m);
        if (lane == lead) cnt[wave][cc] = (uint32_t)__popcll(m);
    });
    __syncthreads();
    if (tid < 64) {
        const uint32_t tot = cnt[0][tid] + cnt[1][tid] + cnt[2][tid] + cnt[3][tid];
        base[tid] = tot ? atomicAdd(&cursor[tid], tot) : 0u;
    }
    __syncthreads();
    if (j < n) {
        uint32_t pos = base[c] + rank;
        for (uint32_t w = 0; w < wave; ++w) pos += cnt[w][c];
        order[pos] = j;
    }
}

__global__ void zero_u32_kernel(uint32_t* p, uint32_t n) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) p[j] = 0;
}

// Dense output offsets: exclusive prefix sum of the tasks' cube sizes (labels,
// or words of packed indices) in task order (a task whose record or LOD is
// unusable occupies nothing).  One
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
            sz = t <= kMaxLog2b ? out_units(1ull << (3 * t), P.pal_bits) : 0;
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
size_t shared_bytes(uint32_t cap16) { return sizeof(Shared) + 2ull * (cap16 < kMinCap16 ? kMinCap16 : cap16); }

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

template <int NT>
static int resident_nt(uint32_t cap16) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, decode_kernel<NT>, NT, shared_bytes(cap16)) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

int max_resident_per_cu(int wg_size, uint32_t cap16) {
    switch (wg_size) {
    case 128: return resident_nt<128>(cap16);
    case 256: return resident_nt<256>(cap16);
    case 512: return resident_nt<512>(cap16);
    case 1024: return resident_nt<1024>(cap16);
    default: return 1;
    }
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
