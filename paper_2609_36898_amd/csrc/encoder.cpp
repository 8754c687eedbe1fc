// Host-side CSGV encoder (the preprocessing step: the paper compresses on the
// CPU, in parallel over bricks -- Methods > "Compressed segmentation volumes").
//
// Per brick: the finest level is the brick in Morton order; every coarser
// node is the mode of its 8 children (ties to the smaller label) and is
// flagged constant when its whole footprint holds one label.  Nodes are then
// visited coarse to fine in Morton order; a node is explicit when it is the
// root or its parent is explicit and not constant.  Each explicit node emits
// one operation -- the first applicable of PARENT, NX, NY, NZ, LAST, DELTA
// (unlimited delta, 4-bit entries, most significant group first), ADV --
// followed by the stop bit (= constant footprint; 0 on the finest level)
// (Results > "CSGV"; supplementary operation list).  The symbol streams of all
// bricks give one 16-symbol frequency table; each brick is stored with the
// plain 4-bit coder or interleaved rANS, whichever is smaller.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "../../include/csgv.h"
#include "csgv_format.h"

using namespace csgv;

namespace {

struct Spread {
    uint32_t t[64];
    Spread() {
        for (uint32_t v = 0; v < 64; ++v) {
            uint32_t r = 0;
            for (int k = 0; k < 6; ++k) r |= ((v >> k) & 1u) << (3 * k);
            t[v] = r;
        }
    }
};
const Spread kSpread;

// mode of 8 labels, ties to the smaller label
inline uint64_t mode_of8(const uint64_t* c) {
    uint64_t v[8];
    memcpy(v, c, sizeof(v));
    std::sort(v, v + 8);
    uint64_t best = v[0];
    int best_n = 0, run = 0;
    for (int i = 0; i < 8; ++i) {
        run = (i > 0 && v[i] == v[i - 1]) ? run + 1 : 1;
        if (run > best_n) { best_n = run; best = v[i]; }  // strictly greater keeps the smaller label on ties
    }
    return best;
}

// label -> latest palette position, cleared in O(1) with a generation stamp
struct PosTable {
    std::vector<uint64_t> key;
    std::vector<uint32_t> val, gen;
    uint32_t mask = 0, cur = 0;
    void reset(size_t n) {
        size_t cap = 64;
        while (cap < 2 * n) cap <<= 1;
        if (key.size() < cap) {
            key.assign(cap, 0);
            val.assign(cap, 0);
            gen.assign(cap, 0);
            cur = 0;
        }
        mask = (uint32_t)(key.size() - 1);
        if (++cur == 0) {
            std::fill(gen.begin(), gen.end(), 0);
            cur = 1;
        }
    }
    uint32_t slot(uint64_t k) const {
        uint32_t i = (uint32_t)((k * 0xD6E8FEB86659FD93ull) >> 40) & mask;
        while (gen[i] == cur && key[i] != k) i = (i + 1) & mask;
        return i;
    }
    bool find(uint64_t k, uint32_t* v) const {
        uint32_t i = slot(k);
        if (gen[i] != cur) return false;
        *v = val[i];
        return true;
    }
    void put(uint64_t k, uint32_t v) {
        uint32_t i = slot(k);
        gen[i] = cur;
        key[i] = k;
        val[i] = v;
    }
};

struct BrickCode {
    std::vector<uint8_t> sym;
    std::vector<uint64_t> pal;
    uint32_t sym_end[kMaxLog2b + 1] = {};
    uint32_t L = 0;
    // chosen record
    std::vector<uint8_t> rec;
};

struct Worker {
    std::vector<uint64_t> lev[kMaxLog2b + 1];
    std::vector<uint8_t> cst[kMaxLog2b + 1];
    std::vector<uint8_t> open_prev, open_cur;
    PosTable pos;
};

constexpr uint32_t kLegacyDelta = 16;  // longest palette back reference with op_mask bit 6

void encode_brick(const uint8_t* vox, uint32_t lb, uint32_t L, uint32_t op_mask, uint32_t nmode, Worker& w,
                  BrickCode& out) {
    const uint32_t b = 1u << L;
    for (uint32_t i = 0; i <= L; ++i) {
        const size_t n = size_t(1) << (3 * i);
        w.lev[i].resize(n);
        w.cst[i].resize(n);
    }
    // finest level in Morton order
    uint64_t* G = w.lev[L].data();
    for (uint32_t z = 0; z < b; ++z)
        for (uint32_t y = 0; y < b; ++y) {
            const uint32_t myz = (kSpread.t[y] << 1) | (kSpread.t[z] << 2);
            const size_t row = ((size_t)z * b + y) * b;
            for (uint32_t x = 0; x < b; ++x) {
                uint64_t v;
                if (lb == 8) memcpy(&v, vox + 8 * (row + x), 8);
                else {
                    uint32_t v32;
                    memcpy(&v32, vox + 4 * (row + x), 4);
                    v = v32;
                }
                G[kSpread.t[x] | myz] = v;
            }
        }
    std::fill(w.cst[L].begin(), w.cst[L].end(), 1);
    for (uint32_t i = L; i >= 1; --i) {
        const size_t np = size_t(1) << (3 * (i - 1));
        const uint64_t* c = w.lev[i].data();
        const uint8_t* cc = w.cst[i].data();
        uint64_t* p = w.lev[i - 1].data();
        uint8_t* pc = w.cst[i - 1].data();
        for (size_t q = 0; q < np; ++q) {
            const uint64_t* ch = c + 8 * q;
            bool same = true;
            for (int j = 1; j < 8 && same; ++j) same = ch[j] == ch[0];
            bool all_const = same;
            for (int j = 0; j < 8 && all_const; ++j) all_const = cc[8 * q + j] != 0;
            pc[q] = all_const ? 1 : 0;
            p[q] = same ? ch[0] : mode_of8(ch);
        }
    }
    // traversal
    out.L = L;
    out.sym.clear();
    out.pal.clear();
    w.pos.reset(total_nodes(L));
    w.open_prev.assign(1, 1);
    for (uint32_t i = 0; i <= L; ++i) {
        const uint32_t n = 1u << (3 * i);
        const uint32_t mx = 0x09249249u & (n - 1u), my = mx << 1, mz = mx << 2;
        const uint64_t* cur = w.lev[i].data();
        const uint64_t* par = i ? w.lev[i - 1].data() : nullptr;
        const uint8_t* cst = w.cst[i].data();
        w.open_cur.assign(n, 0);
        for (uint32_t m = 0; m < n; ++m) {
            if (i > 0 && !w.open_prev[m >> 3]) continue;
            const uint64_t v = cur[m];
            uint32_t op = kBadOp, delta = 0;
            if ((op_mask & 1u) && i > 0 && par[m >> 3] == v) op = kParent;
            // neighbour copies; in neighbour mode 1 only from another sibling
            // group, i.e. when the axis coordinate is even (its lowest bit is
            // bit 0 / 1 / 2 of m)
            if (op == kBadOp && (op_mask & 2u) && (m & mx) && !(nmode && (m & 1u)) &&
                cur[(((m & mx) - 1u) & mx) | (m & ~mx)] == v)
                op = kNX;
            if (op == kBadOp && (op_mask & 4u) && (m & my) && !(nmode && (m & 2u)) &&
                cur[(((m & my) - 1u) & my) | (m & ~my)] == v)
                op = kNY;
            if (op == kBadOp && (op_mask & 8u) && (m & mz) && !(nmode && (m & 4u)) &&
                cur[(((m & mz) - 1u) & mz) | (m & ~mz)] == v)
                op = kNZ;
            if (op == kBadOp && (op_mask & 16u) && !out.pal.empty() && out.pal.back() == v) op = kLast;
            if (op == kBadOp && (op_mask & 32u)) {
                uint32_t p;
                // bit 6: back references of at most kLegacyDelta entries, as in the original
                // format; a label further back is appended again (a palette duplicate)
                if (w.pos.find(v, &p) && (!(op_mask & 64u) || out.pal.size() - p <= kLegacyDelta)) {
                    op = kDelta;
                    delta = (uint32_t)out.pal.size() - p;
                }
            }
            if (op == kBadOp) {
                op = kAdv;
                w.pos.put(v, (uint32_t)out.pal.size());
                out.pal.push_back(v);
            }
            const uint32_t stop = i < L ? cst[m] : 0u;
            out.sym.push_back((uint8_t)(op | (stop << 3)));
            if (op == kDelta) {
                int groups = 1;
                while (groups < 11 && (delta >> (3 * groups)) != 0) ++groups;
                for (int g = groups - 1; g >= 0; --g)
                    out.sym.push_back((uint8_t)(((delta >> (3 * g)) & 7u) | (g > 0 ? 8u : 0u)));
            }
            w.open_cur[m] = stop ? 0 : 1;
        }
        out.sym_end[i] = (uint32_t)out.sym.size();
        std::swap(w.open_prev, w.open_cur);
    }
}

// normalised table (sum 4096): floor(count * 4096 / total), at least 1 for
// used symbols; shortfall to the most frequent symbol (lowest on ties); any
// excess taken one by one from the largest entry above 1 (lowest on ties)
void normalise(const uint64_t cnt[16], uint16_t f[16]) {
    uint64_t tot = 0;
    for (int s = 0; s < 16; ++s) tot += cnt[s];
    if (!tot) {
        memset(f, 0, 32);
        return;
    }
    int64_t sum = 0;
    for (int s = 0; s < 16; ++s) {
        uint64_t v = cnt[s] ? std::max<uint64_t>(1, cnt[s] * kRansM / tot) : 0;
        f[s] = (uint16_t)v;
        sum += (int64_t)v;
    }
    if (sum < (int64_t)kRansM) {
        int best = 0;
        for (int s = 1; s < 16; ++s)
            if (cnt[s] > cnt[best]) best = s;
        f[best] = (uint16_t)(f[best] + (kRansM - sum));
    }
    while (sum > (int64_t)kRansM) {
        int best = -1;
        for (int s = 0; s < 16; ++s)
            if (f[s] > 1 && (best < 0 || f[s] > f[best])) best = s;
        --f[best];
        --sum;
    }
}

inline void put32(std::vector<uint8_t>& v, size_t at, uint32_t x) { memcpy(&v[at], &x, 4); }

// record with the plain 4-bit coder (rans=false) or interleaved rANS
void build_record(const BrickCode& bc, uint32_t lb, bool rans, uint32_t lane_syms, const uint16_t* freq,
                  const uint32_t* cum, std::vector<uint8_t>& rec) {
    const uint32_t L = bc.L, nsym = (uint32_t)bc.sym.size(), pc = (uint32_t)bc.pal.size();
    uint32_t log2W = 0;
    if (rans) {
        uint32_t W = 1;
        while (W < 256 && (uint64_t)W * 2 * lane_syms <= nsym) W *= 2;
        while ((1u << log2W) < W) ++log2W;
    }
    const uint32_t W = 1u << log2W, G = (W + 63) / 64;
    const size_t hdr = record_header_bytes(L, rans ? kRans : kRaw4, log2W);
    const size_t al = lb == 8 ? 8 : 4;
    const size_t pal_off = (hdr + al - 1) / al * al;
    const size_t pay_off = pal_off + (size_t)pc * lb;
    std::vector<uint32_t> state;
    std::vector<std::vector<uint16_t>> stacks;
    size_t pay = 0;
    if (!rans) {
        pay = (nsym + 1) / 2;
    } else {
        state.assign(W, kRansL);
        stacks.assign(G, {});
        for (uint32_t j = nsym; j-- > 0;) {
            const uint32_t l = j & (W - 1), g = l >> 6, s = bc.sym[j], f = freq[s];
            uint32_t x = state[l];
            if ((uint64_t)x >= ((uint64_t)f << 20)) {
                stacks[g].push_back((uint16_t)(x & 0xFFFFu));
                x >>= 16;
            }
            state[l] = ((x / f) << kRansBits) + (x % f) + cum[s];
        }
        for (auto& s : stacks) pay += 2 * s.size();
    }
    const size_t total = (pay_off + pay + 7) / 8 * 8;
    rec.assign(total, 0);
    rec[0] = (uint8_t)(rans ? kRans : kRaw4);
    rec[1] = (uint8_t)L;
    rec[2] = (uint8_t)lb;
    rec[3] = (uint8_t)log2W;
    put32(rec, 4, pc);
    for (uint32_t i = 0; i <= L; ++i) put32(rec, 8 + 4 * i, bc.sym_end[i]);
    if (rans) {
        size_t o = 8 + 4 * (L + 1);
        for (uint32_t g = 0; g < G; ++g) put32(rec, o + 4 * g, (uint32_t)stacks[g].size());
        o += 4 * G;
        for (uint32_t l = 0; l < W; ++l) put32(rec, o + 4 * l, state[l]);
    }
    for (uint32_t k = 0; k < pc; ++k) {
        if (lb == 8) memcpy(&rec[pal_off + 8 * (size_t)k], &bc.pal[k], 8);
        else {
            uint32_t v = (uint32_t)bc.pal[k];
            memcpy(&rec[pal_off + 4 * (size_t)k], &v, 4);
        }
    }
    if (!rans) {
        for (uint32_t j = 0; j < nsym; ++j) rec[pay_off + j / 2] |= (uint8_t)(bc.sym[j] << (4 * (j & 1)));
    } else {
        size_t o = pay_off;
        for (uint32_t g = 0; g < G; ++g)
            for (size_t k = stacks[g].size(); k-- > 0;) {
                memcpy(&rec[o], &stacks[g][k], 2);
                o += 2;
            }
    }
}

template <class F>
void parallel_for(uint32_t n, int threads, F&& fn) {
    if (threads <= 1 || n < 2) {
        for (uint32_t i = 0; i < n; ++i) fn(i, 0);
        return;
    }
    std::atomic<uint32_t> next{0};
    std::vector<std::thread> pool;
    for (int t = 0; t < threads; ++t)
        pool.emplace_back([&, t] {
            for (;;) {
                uint32_t i = next.fetch_add(1);
                if (i >= n) break;
                fn(i, t);
            }
        });
    for (auto& th : pool) th.join();
}

}  // namespace

// Streaming encoder: bricks are symbolised as they are added (the raw voxels
// can be dropped right after), the volume's frequency table and the records
// are produced once at the end.
struct csgv_encoder {
    uint32_t label_bytes = 4, default_log2b = 5, op_mask = 63, neighbor_mode = 0, coder_policy = 0, lane_syms = 64;
    uint32_t dims[3] = {0, 0, 0}, grid[3] = {0, 0, 0};
    bool has_grid = false, with_dir = false;
    int threads = 1;
    std::vector<BrickCode> bc;
    std::vector<uint32_t> origins;  // 3 per brick when with_dir
    std::vector<uint8_t> log2b;
};

extern "C" {

csgv_status csgv_encoder_create(uint32_t label_bytes, const uint32_t dims[3], uint32_t default_log2b,
                                const uint32_t grid[3], int with_directory, uint32_t op_mask, uint32_t neighbor_mode,
                                uint32_t coder_policy, uint32_t lane_syms, int n_threads, csgv_encoder** out) {
    if (!out) return CSGV_EINVAL;
    if (label_bytes != 4 && label_bytes != 8) return CSGV_EINVAL;
    if (coder_policy > 2) return CSGV_EINVAL;
    csgv_encoder* e = new csgv_encoder();
    e->label_bytes = label_bytes;
    e->default_log2b = default_log2b;
    e->op_mask = op_mask;
    e->neighbor_mode = neighbor_mode;
    e->coder_policy = coder_policy;
    e->lane_syms = lane_syms < 1 ? 1 : lane_syms;
    for (int a = 0; a < 3; ++a) {
        e->dims[a] = dims ? dims[a] : 0;
        e->grid[a] = grid ? grid[a] : 0;
    }
    e->with_dir = with_directory != 0;
    e->threads = n_threads > 0 ? n_threads : (int)std::max(1u, std::thread::hardware_concurrency());
    *out = e;
    return CSGV_OK;
}

csgv_status csgv_encoder_add(csgv_encoder* e, const void* h_voxels, const uint8_t* h_log2b, uint32_t n_bricks,
                             const uint32_t* h_origins) {
    if (!e || (n_bricks && (!h_voxels || !h_log2b))) return CSGV_EINVAL;
    if (e->with_dir && n_bricks && !h_origins) return CSGV_EINVAL;
    std::vector<size_t> vox_off(n_bricks + 1, 0);
    for (uint32_t k = 0; k < n_bricks; ++k) {
        if (h_log2b[k] < 1 || h_log2b[k] > kMaxLog2b) return CSGV_EINVAL;
        vox_off[k + 1] = vox_off[k] + (size_t(1) << (3 * h_log2b[k]));
    }
    const size_t base = e->bc.size();
    e->bc.resize(base + n_bricks);
    std::vector<Worker> workers(e->threads);
    const uint8_t* vox = (const uint8_t*)h_voxels;
    const uint32_t lb = e->label_bytes;
    parallel_for(n_bricks, e->threads, [&](uint32_t k, int t) {
        encode_brick(vox + vox_off[k] * lb, lb, h_log2b[k], e->op_mask, e->neighbor_mode, workers[t], e->bc[base + k]);
    });
    e->log2b.insert(e->log2b.end(), h_log2b, h_log2b + n_bricks);
    if (e->with_dir) e->origins.insert(e->origins.end(), h_origins, h_origins + 3ull * n_bricks);
    return CSGV_OK;
}

csgv_status csgv_encoder_finish(csgv_encoder* e, void** h_out, uint64_t* out_bytes) {
    if (!e || !h_out || !out_bytes) return CSGV_EINVAL;
    const uint32_t n_bricks = (uint32_t)e->bc.size();
    const uint32_t label_bytes = e->label_bytes, lane_syms = e->lane_syms, coder_policy = e->coder_policy;
    std::vector<BrickCode>& bc = e->bc;
    uint64_t cnt[16] = {0};
    for (auto& c : bc)
        for (uint8_t s : c.sym) ++cnt[s];
    uint16_t freq[16];
    normalise(cnt, freq);
    uint32_t cum[17];
    cum[0] = 0;
    for (int s = 0; s < 16; ++s) cum[s + 1] = cum[s] + freq[s];
    parallel_for(n_bricks, e->threads, [&](uint32_t k, int) {
        std::vector<uint8_t> raw, rans;
        if (coder_policy != 2) build_record(bc[k], label_bytes, false, lane_syms, freq, cum, raw);
        if (coder_policy != 1) build_record(bc[k], label_bytes, true, lane_syms, freq, cum, rans);
        if (coder_policy == 1) bc[k].rec.swap(raw);
        else if (coder_policy == 2) bc[k].rec.swap(rans);
        else if (rans.size() < raw.size()) bc[k].rec.swap(rans);
        else bc[k].rec.swap(raw);
        std::vector<uint8_t>().swap(bc[k].sym);
        std::vector<uint64_t>().swap(bc[k].pal);
    });
    const bool dir = e->with_dir;
    const uint64_t off_pos = kHeaderBytes;
    const uint64_t dir_pos = dir ? (off_pos + 8ull * (n_bricks + 1) + 7) / 8 * 8 : 0;
    uint64_t rec0 = dir ? dir_pos + 16ull * n_bricks : off_pos + 8ull * (n_bricks + 1);
    rec0 = (rec0 + 7) / 8 * 8;
    uint64_t total = rec0;
    for (auto& c : bc) total += c.rec.size();
    uint8_t* buf = (uint8_t*)calloc(total ? total : 1, 1);
    if (!buf) return CSGV_ENOMEM;
    auto w32 = [&](uint64_t at, uint32_t v) { memcpy(buf + at, &v, 4); };
    auto w64 = [&](uint64_t at, uint64_t v) { memcpy(buf + at, &v, 8); };
    w32(0, kMagic);
    w32(4, kVersion);
    for (int a = 0; a < 3; ++a) {
        w32(kHdrDims + 4 * a, e->dims[a]);
        w32(kHdrGrid + 4 * a, e->grid[a]);
    }
    w32(kHdrLog2b, e->default_log2b);
    w32(kHdrLabelBytes, label_bytes);
    w32(kHdrOpMask, e->op_mask);
    w32(kHdrNBricks, n_bricks);
    memcpy(buf + kHdrFreq, freq, 32);
    w64(kHdrOffsetsPos, off_pos);
    w64(kHdrDirPos, dir_pos);
    w64(kHdrTotal, total);
    w32(kHdrNeighborMode, e->neighbor_mode);
    uint64_t pos = rec0;
    for (uint32_t k = 0; k < n_bricks; ++k) {
        w64(off_pos + 8ull * k, pos);
        if (dir) {
            for (int a = 0; a < 3; ++a) w32(dir_pos + 16ull * k + 4 * a, e->origins[3ull * k + a]);
            w32(dir_pos + 16ull * k + 12, e->log2b[k]);
        }
        pos += bc[k].rec.size();
    }
    w64(off_pos + 8ull * n_bricks, pos);
    parallel_for(n_bricks, e->threads, [&](uint32_t k, int) {
        uint64_t at;
        memcpy(&at, buf + off_pos + 8ull * k, 8);
        memcpy(buf + at, bc[k].rec.data(), bc[k].rec.size());
        std::vector<uint8_t>().swap(bc[k].rec);
    });
    bc.clear();
    *h_out = buf;
    *out_bytes = total;
    return CSGV_OK;
}

void csgv_encoder_destroy(csgv_encoder* e) { delete e; }

csgv_status csgv_encode_bricks(const void* h_voxels, const uint8_t* h_log2b, uint32_t n_bricks, uint32_t label_bytes,
                               const uint32_t dims[3], uint32_t default_log2b, const uint32_t grid[3],
                               const uint32_t* h_origins, uint32_t op_mask, uint32_t neighbor_mode,
                               uint32_t coder_policy, uint32_t lane_syms, int n_threads, void** h_out,
                               uint64_t* out_bytes) {
    if (!h_out || !out_bytes || (n_bricks && (!h_voxels || !h_log2b))) return CSGV_EINVAL;
    csgv_encoder* e = nullptr;
    csgv_status st = csgv_encoder_create(label_bytes, dims, default_log2b, grid, h_origins != nullptr, op_mask,
                                         neighbor_mode, coder_policy, lane_syms, n_threads, &e);
    if (st != CSGV_OK) return st;
    st = csgv_encoder_add(e, h_voxels, h_log2b, n_bricks, h_origins);
    if (st == CSGV_OK) st = csgv_encoder_finish(e, h_out, out_bytes);
    csgv_encoder_destroy(e);
    return st;
}

}  // extern "C"
