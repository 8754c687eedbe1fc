/*
 * CSGV brick codec -- plain CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call this file:
 * only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code, header, table or constant with the
 * GPU decoder.  Every routine favours being checkable by eye against the
 * paper over speed: labels are widened to u64, level grids are plain arrays,
 * and the stream is read one symbol at a time.
 *
 * What it implements (paper: Results > "CSGV"; Methods > "Compressed
 * segmentation volumes"; supplementary caption of the operation ablation):
 *   - downsample():  the multi-resolution rule: a coarser voxel takes the
 *     mode of its 2^3 children (Methods > "Volcanite rendering": a mipmap that
 *     accumulates the mode instead of the average), ties to the smallest
 *     label (a reading: the paper names no tie rule).
 *   - encode:  each brick becomes a stream of one operation per explicit node,
 *     coarse to fine, with a stop bit marking all-constant children
 *     (Results > "CSGV").  Operations: PALETTE_ADV (read the next palette
 *     label), PARENT, NEIGHBOR_X/Y/Z, PALETTE_LAST (delta = 1),
 *     PALETTE_DELTA with the unlimited delta chain of 4-bit entries
 *     delta <- (delta << 3) | (entry & 7), continuation in the entry's top bit
 *     (Methods > "Compressed segmentation volumes").
 *   - decode:  the sequential reference decoder, with the error verdicts the
 *     GPU decoder must reproduce.
 *   - rANS:  the secondary entropy coder (Results > "CSGV": "secondary ANS
 *     frequency coding"; Methods > "GPU rendering pipeline": plain 4-bit or
 *     range-ANS encoders), as static 16-symbol rANS (Duda 2013/2015) with
 *     W interleaved lanes (Giesen 2014).
 *
 * The paper gives the encoding only in outline, so the byte layout and the
 * reading of every point it leaves open (node order, mode ties, stop bits,
 * symbol codes, rANS parameters, error verdicts) are this codec's own; the
 * comment above each routine states the rule it follows.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------ constants */
#define OR_MAGIC 0x56475343u /* 'CSGV' little-endian */
#define OR_VERSION 1u
#define OR_HDR_BYTES 128u

enum { OP_PARENT = 0, OP_NX = 1, OP_NY = 2, OP_NZ = 3, OP_ADV = 4, OP_LAST = 5, OP_DELTA = 6, OP_BAD = 7 };
/* op-mask bits for the encoder; PALETTE_ADV is always on */
enum { M_PARENT = 1, M_NX = 2, M_NY = 4, M_NZ = 8, M_LAST = 16, M_DELTA = 32 };
enum { ST_OK = 0, ST_INVALID = 1, ST_CORRUPT = 2 };
enum { CODER_RAW4 = 0, CODER_RANS = 1 };

#define RANS_BITS 12
#define RANS_M (1u << RANS_BITS)
#define RANS_L (1u << 16)

/* ------------------------------------------------------- little helpers */
static uint32_t rd32(const uint8_t* p) { return (uint32_t)p[0] | (uint32_t)p[1] << 8 | (uint32_t)p[2] << 16 | (uint32_t)p[3] << 24; }
static uint64_t rd64(const uint8_t* p) { return (uint64_t)rd32(p) | (uint64_t)rd32(p + 4) << 32; }
static uint16_t rd16(const uint8_t* p) { return (uint16_t)(p[0] | p[1] << 8); }
static void wr32(uint8_t* p, uint32_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); p[2] = (uint8_t)(v >> 16); p[3] = (uint8_t)(v >> 24); }
static void wr64(uint8_t* p, uint64_t v) { wr32(p, (uint32_t)v); wr32(p + 4, (uint32_t)(v >> 32)); }
static void wr16(uint8_t* p, uint16_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); }

static uint64_t get_label(const void* base, int lb, size_t i) {
    return lb == 8 ? ((const uint64_t*)base)[i] : (uint64_t)((const uint32_t*)base)[i];
}
static void put_label(void* base, int lb, size_t i, uint64_t v) {
    if (lb == 8) ((uint64_t*)base)[i] = v;
    else ((uint32_t*)base)[i] = (uint32_t)v;
}

/* Morton (Z-order) index of (x,y,z) at a level with `bits` bits per axis:
 * bit k of x goes to bit 3k, of y to 3k+1, of z to 3k+2. */
static uint32_t morton(uint32_t x, uint32_t y, uint32_t z, int bits) {
    uint32_t m = 0;
    for (int k = 0; k < bits; k++)
        m |= ((x >> k) & 1u) << (3 * k) | ((y >> k) & 1u) << (3 * k + 1) | ((z >> k) & 1u) << (3 * k + 2);
    return m;
}
static void demorton(uint32_t m, int bits, uint32_t* x, uint32_t* y, uint32_t* z) {
    *x = *y = *z = 0;
    for (int k = 0; k < bits; k++) {
        *x |= ((m >> (3 * k)) & 1u) << k;
        *y |= ((m >> (3 * k + 1)) & 1u) << k;
        *z |= ((m >> (3 * k + 2)) & 1u) << k;
    }
}

/* total nodes of levels 0..L: 1 + 8 + ... + 8^L */
static uint64_t total_nodes(int L) {
    uint64_t t = 0;
    for (int i = 0; i <= L; i++) t += (uint64_t)1 << (3 * i);
    return t;
}

/* ----------------------------------------------------- the mode pyramid */
/* Mode of 8 labels; among labels tied for the highest count the smallest wins. */
static uint64_t mode8(const uint64_t v[8]) {
    uint64_t best = 0;
    int best_count = 0;
    for (int a = 0; a < 8; a++) {
        int c = 0;
        for (int b = 0; b < 8; b++) c += v[b] == v[a];
        if (c > best_count || (c == best_count && v[a] < best)) { best = v[a]; best_count = c; }
    }
    return best;
}

/*
 * Plain definition of LOD k: G_L = the brick, G_{i-1}[q] = mode of the 2^3
 * children of q in G_i; the result is G_{L-k}, linear x-fastest, side b>>k.
 * brick: b^3 labels (x fastest), b = 1 << log2b.
 */
int oracle_downsample(const void* brick, int lb, int log2b, int lod, void* out) {
    if (log2b < 0 || log2b > 10 || lod < 0 || lod > log2b || (lb != 4 && lb != 8)) return -1;
    size_t b = (size_t)1 << log2b;
    uint64_t* cur = (uint64_t*)malloc(sizeof(uint64_t) * b * b * b);
    for (size_t i = 0; i < b * b * b; i++) cur[i] = get_label(brick, lb, i);
    size_t s = b;
    for (int k = 0; k < lod; k++) {
        size_t h = s / 2;
        uint64_t* nxt = (uint64_t*)malloc(sizeof(uint64_t) * (h * h * h > 0 ? h * h * h : 1));
        for (size_t z = 0; z < h; z++)
            for (size_t y = 0; y < h; y++)
                for (size_t x = 0; x < h; x++) {
                    uint64_t v[8];
                    for (int d = 0; d < 8; d++) {
                        size_t cx = 2 * x + (d & 1), cy = 2 * y + ((d >> 1) & 1), cz = 2 * z + ((d >> 2) & 1);
                        v[d] = cur[(cz * s + cy) * s + cx];
                    }
                    nxt[(z * h + y) * h + x] = mode8(v);
                }
        free(cur);
        cur = nxt;
        s = h;
    }
    for (size_t i = 0; i < s * s * s; i++) put_label(out, lb, i, cur[i]);
    free(cur);
    return 0;
}

/* ------------------------------------------------------- delta entries */
/*
 * delta >= 1 as 4-bit entries, most significant 3-bit group first, each
 * entry = (group) | (8 if another entry follows); minimal length.
 * Returns the entry count.
 */
int oracle_delta_entries(uint32_t delta, uint8_t* out) {
    int groups = 1;
    while (groups < 11 && (delta >> (3 * groups)) != 0) groups++;
    for (int g = 0; g < groups; g++) {
        uint32_t v = (delta >> (3 * (groups - 1 - g))) & 7u;
        out[g] = (uint8_t)(v | (g + 1 < groups ? 8u : 0u));
    }
    return groups;
}

/* delta accumulation with the saturating cap used by both decoders */
static uint64_t delta_step(uint64_t delta, uint32_t entry) {
    uint64_t d = (delta << 3) | (entry & 7u);
    return d > 0xFFFFFFFFull ? 0xFFFFFFFFull : d;
}

/* --------------------------------------------------------------- rANS */
/*
 * Per-volume table: normalised symbol counts, sum 4096.  freq[s] =
 * max(1, count*4096/total) for symbols that occur, 0 otherwise; a positive
 * remainder goes to the most frequent symbol (lowest symbol on ties); an
 * excess is removed one at a time from the symbol with the largest freq > 1
 * (lowest symbol on ties).
 */
void oracle_make_freq(const uint64_t counts[16], uint16_t freq[16]) {
    uint64_t total = 0;
    for (int s = 0; s < 16; s++) total += counts[s];
    if (total == 0) { memset(freq, 0, 32); return; }
    int64_t sum = 0;
    for (int s = 0; s < 16; s++) {
        uint64_t f = counts[s] ? counts[s] * RANS_M / total : 0;
        if (counts[s] && f == 0) f = 1;
        freq[s] = (uint16_t)f;
        sum += (int64_t)f;
    }
    if (sum < (int64_t)RANS_M) {
        int best = 0;
        for (int s = 1; s < 16; s++) if (counts[s] > counts[best]) best = s;
        freq[best] = (uint16_t)(freq[best] + (RANS_M - sum));
    }
    while (sum > (int64_t)RANS_M) {
        int best = -1;
        for (int s = 0; s < 16; s++) if (freq[s] > 1 && (best < 0 || freq[s] > freq[best])) best = s;
        freq[best]--;
        sum--;
    }
}

/*
 * Interleaved rANS.  Symbol j belongs to lane j mod W; lanes form groups of
 * 64 (lane l in group l/64) and every group owns one stream of u16 words.
 * Decoding symbol j on lane l: slot = x & 4095; s = the symbol whose
 * cumulative range holds slot; x = freq[s]*(x >> 12) + slot - cum[s];
 * if x < 2^16, x = (x << 16) | next word of the lane's group.  Symbols are
 * decoded in index order, so within a round the lanes of a group read their
 * words in lane order.  The encoder below is the exact inverse.
 */
static void cum_of(const uint16_t freq[16], uint32_t cum[17]) {
    cum[0] = 0;
    for (int s = 0; s < 16; s++) cum[s + 1] = cum[s] + freq[s];
}

/* returns total words written (sum over groups); words laid out group by group */
uint32_t oracle_rans_encode(const uint8_t* sym, uint32_t n, const uint16_t freq[16], int log2W, uint32_t* states,
                            uint32_t* group_words, uint16_t* words, uint32_t words_cap) {
    uint32_t W = 1u << log2W, G = (W + 63) / 64, cum[17];
    cum_of(freq, cum);
    uint32_t* x = (uint32_t*)malloc(sizeof(uint32_t) * W);
    for (uint32_t l = 0; l < W; l++) x[l] = RANS_L;
    /* per-group stacks, emitted in reverse symbol order */
    uint16_t** stk = (uint16_t**)malloc(sizeof(uint16_t*) * G);
    uint32_t* sn = (uint32_t*)calloc(G, sizeof(uint32_t));
    for (uint32_t g = 0; g < G; g++) stk[g] = (uint16_t*)malloc(sizeof(uint16_t) * (n + 1));
    for (uint32_t jj = n; jj-- > 0;) {
        uint32_t l = jj & (W - 1), g = l / 64, s = sym[jj], f = freq[s];
        if ((uint64_t)x[l] >= ((uint64_t)f << 20)) { stk[g][sn[g]++] = (uint16_t)(x[l] & 0xFFFF); x[l] >>= 16; }
        x[l] = ((x[l] / f) << RANS_BITS) + (x[l] % f) + cum[s];
    }
    uint32_t pos = 0;
    for (uint32_t g = 0; g < G; g++) {
        group_words[g] = sn[g];
        for (uint32_t k = 0; k < sn[g]; k++)
            if (pos < words_cap) words[pos++] = stk[g][sn[g] - 1 - k];
            else pos++;
        free(stk[g]);
    }
    for (uint32_t l = 0; l < W; l++) states[l] = x[l];
    free(stk); free(sn); free(x);
    return pos;
}

/* decodes n symbols; returns 0, or -1 when a group runs out of words */
int oracle_rans_decode(uint8_t* sym, uint32_t n, const uint16_t freq[16], int log2W, const uint32_t* states_in,
                       const uint32_t* group_words, const uint16_t* words) {
    uint32_t W = 1u << log2W, G = (W + 63) / 64, cum[17];
    cum_of(freq, cum);
    uint32_t* x = (uint32_t*)malloc(sizeof(uint32_t) * W);
    uint32_t* start = (uint32_t*)malloc(sizeof(uint32_t) * G);
    uint32_t* used = (uint32_t*)calloc(G, sizeof(uint32_t));
    memcpy(x, states_in, sizeof(uint32_t) * W);
    uint32_t acc = 0;
    for (uint32_t g = 0; g < G; g++) { start[g] = acc; acc += group_words[g]; }
    int rc = 0;
    for (uint32_t j = 0; j < n; j++) {
        uint32_t l = j & (W - 1), g = l / 64;
        uint32_t slot = x[l] & (RANS_M - 1), s = 0;
        while (!(slot < cum[s + 1])) s++; /* first s with slot < cum[s+1]; freq sums to 4096 */
        x[l] = (uint32_t)freq[s] * (x[l] >> RANS_BITS) + slot - cum[s];
        if (x[l] < RANS_L) {
            if (used[g] >= group_words[g]) { rc = -1; break; }
            x[l] = (x[l] << 16) | words[start[g] + used[g]++];
        }
        sym[j] = (uint8_t)s;
    }
    free(x); free(start); free(used);
    return rc;
}

/* --------------------------------------------------------- brick encode */
typedef struct {
    uint8_t* sym;       /* symbols (one per byte) */
    uint32_t nsym, cap;
    uint32_t sym_end[7];
    uint64_t* pal;
    uint32_t pc, pal_cap;
    int log2b;
} brick_stream;

static void push_sym(brick_stream* bs, uint8_t s) {
    if (bs->nsym == bs->cap) {
        bs->cap = bs->cap ? 2 * bs->cap : 1024;
        bs->sym = (uint8_t*)realloc(bs->sym, bs->cap);
    }
    bs->sym[bs->nsym++] = s;
}

/* open-addressing map label -> most recent palette position */
typedef struct { uint64_t* key; uint32_t* val; uint8_t* used; uint32_t mask; } pos_map;

static void map_init(pos_map* m, uint64_t n) {
    uint32_t cap = 16;
    while (cap < 2 * n) cap <<= 1;
    m->mask = cap - 1;
    m->key = (uint64_t*)malloc(sizeof(uint64_t) * cap);
    m->val = (uint32_t*)malloc(sizeof(uint32_t) * cap);
    m->used = (uint8_t*)calloc(cap, 1);
}
static void map_free(pos_map* m) { free(m->key); free(m->val); free(m->used); }
static uint32_t map_slot(const pos_map* m, uint64_t k) {
    uint64_t h = k * 0x9E3779B97F4A7C15ull;
    uint32_t i = (uint32_t)(h >> 32) & m->mask;
    while (m->used[i] && m->key[i] != k) i = (i + 1) & m->mask;
    return i;
}
static int map_get(const pos_map* m, uint64_t k, uint32_t* v) {
    uint32_t i = map_slot(m, k);
    if (!m->used[i]) return 0;
    *v = m->val[i];
    return 1;
}
static void map_put(pos_map* m, uint64_t k, uint32_t v) {
    uint32_t i = map_slot(m, k);
    m->used[i] = 1; m->key[i] = k; m->val[i] = v;
}

/*
 * Encode one brick (b^3 labels, x fastest) into symbols + palette.
 * Levels 0..L coarse to fine, nodes of a level in Morton order.  A node is
 * explicit when it is the root or its parent is explicit and not stopped.
 * An explicit node's operation is the first applicable of
 * PARENT, NX, NY, NZ, LAST, DELTA, ADV (restricted to op_mask), i.e. copy
 * from another node when possible, otherwise from the palette.  Its stop bit
 * is 1 when its whole footprint is one label (always 0 at the finest level).
 * neighbor_mode 1 offers NX/NY/NZ only when the neighbour lies in another
 * sibling group (the node's coordinate on that axis is even).
 */
static void encode_brick(const void* brick, int lb, int L, int op_mask, int neighbor_mode, brick_stream* bs) {
    memset(bs, 0, sizeof(*bs));
    bs->log2b = L;
    /* G[i] and C[i] in Morton order per level */
    uint64_t* G[7];
    uint8_t* C[7];
    for (int i = 0; i <= L; i++) {
        size_t n = (size_t)1 << (3 * i);
        G[i] = (uint64_t*)malloc(sizeof(uint64_t) * n);
        C[i] = (uint8_t*)malloc(n);
    }
    uint32_t b = 1u << L;
    for (uint32_t z = 0; z < b; z++)
        for (uint32_t y = 0; y < b; y++)
            for (uint32_t x = 0; x < b; x++) {
                uint32_t m = morton(x, y, z, L);
                G[L][m] = get_label(brick, lb, ((size_t)z * b + y) * b + x);
                C[L][m] = 1;
            }
    for (int i = L; i >= 1; i--) {
        size_t np = (size_t)1 << (3 * (i - 1));
        for (size_t q = 0; q < np; q++) {
            uint64_t v[8];
            int allc = 1;
            for (int j = 0; j < 8; j++) {
                v[j] = G[i][8 * q + j];
                allc &= C[i][8 * q + j] && v[j] == v[0];
            }
            G[i - 1][q] = mode8(v);
            C[i - 1][q] = (uint8_t)allc;
        }
    }
    pos_map pm;
    map_init(&pm, total_nodes(L));
    bs->pal_cap = 64;
    bs->pal = (uint64_t*)malloc(sizeof(uint64_t) * bs->pal_cap);
    uint8_t* expand_prev = NULL;
    for (int i = 0; i <= L; i++) {
        size_t n = (size_t)1 << (3 * i);
        uint8_t* expand = (uint8_t*)calloc(n, 1);
        for (size_t m = 0; m < n; m++) {
            if (i > 0 && !expand_prev[m >> 3]) continue; /* implied: takes the parent's label */
            uint64_t v = G[i][m];
            uint32_t x, y, z;
            demorton((uint32_t)m, i, &x, &y, &z);
            int op = -1;
            uint32_t delta = 0;
            if (op < 0 && (op_mask & M_PARENT) && i > 0 && G[i - 1][m >> 3] == v) op = OP_PARENT;
            if (op < 0 && (op_mask & M_NX) && x > 0 && (!neighbor_mode || !(x & 1)) && G[i][morton(x - 1, y, z, i)] == v) op = OP_NX;
            if (op < 0 && (op_mask & M_NY) && y > 0 && (!neighbor_mode || !(y & 1)) && G[i][morton(x, y - 1, z, i)] == v) op = OP_NY;
            if (op < 0 && (op_mask & M_NZ) && z > 0 && (!neighbor_mode || !(z & 1)) && G[i][morton(x, y, z - 1, i)] == v) op = OP_NZ;
            if (op < 0 && (op_mask & M_LAST) && bs->pc > 0 && bs->pal[bs->pc - 1] == v) op = OP_LAST;
            if (op < 0 && (op_mask & M_DELTA)) {
                uint32_t p;
                if (map_get(&pm, v, &p)) { op = OP_DELTA; delta = bs->pc - p; }
            }
            if (op < 0) {
                op = OP_ADV;
                if (bs->pc == bs->pal_cap) {
                    bs->pal_cap *= 2;
                    bs->pal = (uint64_t*)realloc(bs->pal, sizeof(uint64_t) * bs->pal_cap);
                }
                map_put(&pm, v, bs->pc);
                bs->pal[bs->pc++] = v;
            }
            int stop = i < L ? C[i][m] : 0;
            push_sym(bs, (uint8_t)(op | (stop << 3)));
            if (op == OP_DELTA) {
                uint8_t e[11];
                int ne = oracle_delta_entries(delta, e);
                for (int k = 0; k < ne; k++) push_sym(bs, e[k]);
            }
            expand[m] = (uint8_t)!stop;
        }
        bs->sym_end[i] = bs->nsym;
        free(expand_prev);
        expand_prev = expand;
    }
    free(expand_prev);
    map_free(&pm);
    for (int i = 0; i <= L; i++) { free(G[i]); free(C[i]); }
}

/* ------------------------------------------------------- record layout */
/*
 * Brick record (little-endian, starts 8-aligned):
 *   u8 coder (0 RAW4, 1 RANS), u8 log2b, u8 label_bytes, u8 log2W (0 for RAW4)
 *   u32 palette_count
 *   u32 sym_end[log2b+1]        symbols consumed after each level
 *   RANS only: u32 group_words[G] (G = ceil(W/64)), u32 state[W]
 *   palette (label_bytes each; 8-aligned when label_bytes == 8)
 *   payload: RAW4 = 2 symbols per byte, low nibble first;
 *            RANS = u16 words, group 0's stream then group 1's ...
 *   zero padding to a multiple of 8 bytes.
 */
static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

static size_t record_header_bytes(int L, int coder, int log2W) {
    size_t h = 8 + 4 * (size_t)(L + 1);
    if (coder == CODER_RANS) {
        uint32_t W = 1u << log2W;
        h += 4 * (size_t)((W + 63) / 64) + 4 * (size_t)W;
    }
    return h;
}

/* writes the record into out (if non-NULL); returns its size */
static size_t write_record(const brick_stream* bs, int lb, int coder, int lane_syms, const uint16_t freq[16], uint8_t* out) {
    int L = bs->log2b;
    int log2W = 0;
    if (coder == CODER_RANS) {
        uint32_t W = 1;
        while (W < 256 && (uint64_t)W * 2 * (uint64_t)lane_syms <= bs->nsym) W *= 2;
        while ((1u << log2W) < W) log2W++;
    }
    size_t hdr = record_header_bytes(L, coder, log2W);
    size_t pal_off = align_up(hdr, lb == 8 ? 8 : 4);
    size_t pay_off = pal_off + (size_t)bs->pc * lb;
    size_t pay_bytes;
    uint32_t W = 1u << log2W, G = (W + 63) / 64;
    uint32_t* states = NULL;
    uint32_t* gw = NULL;
    uint16_t* words = NULL;
    uint32_t nwords = 0;
    if (coder == CODER_RAW4) {
        pay_bytes = (bs->nsym + 1) / 2;
    } else {
        states = (uint32_t*)malloc(sizeof(uint32_t) * W);
        gw = (uint32_t*)malloc(sizeof(uint32_t) * G);
        uint32_t cap = bs->nsym + 64 * G + 16;
        words = (uint16_t*)malloc(sizeof(uint16_t) * cap);
        nwords = oracle_rans_encode(bs->sym, bs->nsym, freq, log2W, states, gw, words, cap);
        pay_bytes = 2 * (size_t)nwords;
    }
    size_t total = align_up(pay_off + pay_bytes, 8);
    if (out) {
        memset(out, 0, total);
        out[0] = (uint8_t)coder; out[1] = (uint8_t)L; out[2] = (uint8_t)lb; out[3] = (uint8_t)log2W;
        wr32(out + 4, bs->pc);
        for (int i = 0; i <= L; i++) wr32(out + 8 + 4 * i, bs->sym_end[i]);
        if (coder == CODER_RANS) {
            size_t o = 8 + 4 * (size_t)(L + 1);
            for (uint32_t g = 0; g < G; g++) wr32(out + o + 4 * g, gw[g]);
            o += 4 * G;
            for (uint32_t l = 0; l < W; l++) wr32(out + o + 4 * l, states[l]);
        }
        for (uint32_t k = 0; k < bs->pc; k++) {
            if (lb == 8) wr64(out + pal_off + 8 * (size_t)k, bs->pal[k]);
            else wr32(out + pal_off + 4 * (size_t)k, (uint32_t)bs->pal[k]);
        }
        if (coder == CODER_RAW4) {
            for (uint32_t j = 0; j < bs->nsym; j++) out[pay_off + j / 2] |= (uint8_t)(bs->sym[j] << (4 * (j & 1)));
        } else {
            for (uint32_t k = 0; k < nwords; k++) wr16(out + pay_off + 2 * (size_t)k, words[k]);
        }
    }
    free(states); free(gw); free(words);
    return total;
}

/* --------------------------------------------------------- volume encode */
/*
 * Volume container (little-endian):
 *   0  u32 magic 'CSGV'      4  u32 version (1)
 *   8  u32 dims[3]           20 u32 log2b (default brick size)
 *   24 u32 label_bytes       28 u32 op_mask
 *   32 u32 n_bricks          36 u32 grid[3] (brick grid, 0 when irregular)
 *   48 u16 freq[16]          80 u64 offsets_pos
 *   88 u64 dir_pos (0: none) 96 u64 total_bytes
 *   104 u32 neighbor_mode    108..127 zero
 *   offsets: (n_bricks + 1) u64 byte offsets of each record from the
 *            container start, the last one = end of the final record
 *   directory (optional): n_bricks x {u32 x, y, z origin, u32 log2b}
 *   records, each 8-aligned.
 *
 * voxels: all bricks concatenated, brick k holding (1 << log2b[k])^3 labels
 * x fastest.  coder_policy: 0 smaller of RAW4/RANS (RAW4 on ties), 1 RAW4,
 * 2 RANS.  lane_syms: target symbols per rANS lane (W = largest power of two
 * <= 256 with W * lane_syms <= symbols, at least 1).
 */
int oracle_encode_volume(const void* voxels, const uint8_t* log2b, uint32_t n_bricks, int lb, const uint32_t dims[3],
                         int default_log2b, const uint32_t grid[3], const uint32_t* origins, int op_mask,
                         int neighbor_mode, int coder_policy, int lane_syms, int nthreads, uint8_t** out_buf,
                         uint64_t* out_bytes) {
    if (lb != 4 && lb != 8) return -1;
    if (lane_syms < 1) lane_syms = 1;
    brick_stream* bs = (brick_stream*)calloc(n_bricks ? n_bricks : 1, sizeof(brick_stream));
    size_t* vox_off = (size_t*)malloc(sizeof(size_t) * (n_bricks + 1));
    vox_off[0] = 0;
    for (uint32_t k = 0; k < n_bricks; k++) {
        if (log2b[k] < 1 || log2b[k] > 6) { free(bs); free(vox_off); return -1; }
        vox_off[k + 1] = vox_off[k] + ((size_t)1 << (3 * log2b[k]));
    }
    (void)nthreads;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads > 0 ? nthreads : 1)
    for (long k = 0; k < (long)n_bricks; k++)
        encode_brick((const uint8_t*)voxels + vox_off[k] * (size_t)lb, lb, log2b[k], op_mask, neighbor_mode, &bs[k]);
    uint64_t counts[16] = {0};
    for (uint32_t k = 0; k < n_bricks; k++)
        for (uint32_t j = 0; j < bs[k].nsym; j++) counts[bs[k].sym[j]]++;
    uint16_t freq[16];
    oracle_make_freq(counts, freq);
    int* coder = (int*)malloc(sizeof(int) * (n_bricks ? n_bricks : 1));
    size_t* rsize = (size_t*)malloc(sizeof(size_t) * (n_bricks ? n_bricks : 1));
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads > 0 ? nthreads : 1)
    for (long k = 0; k < (long)n_bricks; k++) {
        size_t raw = write_record(&bs[k], lb, CODER_RAW4, lane_syms, freq, NULL);
        size_t rans = coder_policy == 1 ? 0 : write_record(&bs[k], lb, CODER_RANS, lane_syms, freq, NULL);
        int c = coder_policy == 1 ? CODER_RAW4 : coder_policy == 2 ? CODER_RANS : (rans < raw ? CODER_RANS : CODER_RAW4);
        coder[k] = c;
        rsize[k] = c == CODER_RANS ? rans : raw;
    }
    size_t off_pos = OR_HDR_BYTES;
    size_t dir_pos = origins ? align_up(off_pos + 8 * ((size_t)n_bricks + 1), 8) : 0;
    size_t rec0 = align_up(origins ? dir_pos + 16 * (size_t)n_bricks : off_pos + 8 * ((size_t)n_bricks + 1), 8);
    size_t total = rec0;
    for (uint32_t k = 0; k < n_bricks; k++) total += rsize[k];
    uint8_t* buf = (uint8_t*)calloc(total, 1);
    wr32(buf + 0, OR_MAGIC); wr32(buf + 4, OR_VERSION);
    for (int a = 0; a < 3; a++) { wr32(buf + 8 + 4 * a, dims[a]); wr32(buf + 36 + 4 * a, grid ? grid[a] : 0); }
    wr32(buf + 20, (uint32_t)default_log2b); wr32(buf + 24, (uint32_t)lb); wr32(buf + 28, (uint32_t)op_mask);
    wr32(buf + 32, n_bricks);
    for (int s = 0; s < 16; s++) wr16(buf + 48 + 2 * s, freq[s]);
    wr64(buf + 80, off_pos); wr64(buf + 88, dir_pos); wr64(buf + 96, total);
    wr32(buf + 104, (uint32_t)neighbor_mode);
    size_t pos = rec0;
    for (uint32_t k = 0; k < n_bricks; k++) {
        wr64(buf + off_pos + 8 * (size_t)k, pos);
        if (origins) {
            for (int a = 0; a < 3; a++) wr32(buf + dir_pos + 16 * (size_t)k + 4 * a, origins[3 * k + a]);
            wr32(buf + dir_pos + 16 * (size_t)k + 12, log2b[k]);
        }
        pos += rsize[k];
    }
    wr64(buf + off_pos + 8 * (size_t)n_bricks, pos);
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads > 0 ? nthreads : 1)
    for (long k = 0; k < (long)n_bricks; k++)
        write_record(&bs[k], lb, coder[k], lane_syms, freq, buf + rd64(buf + off_pos + 8 * (size_t)k));
    for (uint32_t k = 0; k < n_bricks; k++) { free(bs[k].sym); free(bs[k].pal); }
    free(bs); free(vox_off); free(coder); free(rsize);
    *out_buf = buf;
    *out_bytes = total;
    return 0;
}

void oracle_free(void* p) { free(p); }

/* --------------------------------------------------------------- decode */
typedef struct {
    const uint8_t* rec;
    uint64_t extent;
    int coder, L, lb, log2W;
    uint32_t pc;
    uint32_t sym_end[7];
    const uint8_t* pal;
    const uint8_t* payload;
    uint64_t payload_bytes;
    const uint8_t* gw;     /* RANS group word counts */
    const uint8_t* states; /* RANS states */
} rec_view;

/*
 * Parse the record of brick `id` (steps common to decoding and inspection).
 * Returns ST_OK, or the verdict with *write_ok telling whether the task's
 * output range may be zero-filled.  Checks, in order:
 *   brick id < n_bricks                               else INVALID
 *   record offsets ordered, in the buffer, 8-aligned, >= 8 bytes   else CORRUPT (no write)
 *   log2b in [1, 6]                                    else CORRUPT (no write)
 *   lod <= log2b                                       else INVALID
 *   output range fits (labels, or 32-bit words of       else INVALID
 *   per_word packed indices when per_word > 0)
 *   -- later failures are CORRUPT with the output zero-filled --
 *   label width = the volume's, coder in {RAW4, RANS}, RAW4 has log2W 0,
 *   RANS has log2W <= 8; header and palette fit the record; sym_end is
 *   non-decreasing and sym_end[L] <= 8 * (number of nodes of levels 0..L);
 *   RAW4: sym_end[L] <= 2 * payload bytes; RANS: all group words fit and the
 *   volume's frequency table sums to 4096.
 */
static int parse_record(const uint8_t* c, uint64_t bytes, uint32_t id, int lod, uint64_t out_off, uint64_t out_cap,
                        uint32_t per_word, rec_view* r, int* write_ok) {
    *write_ok = 0;
    uint32_t n_bricks = rd32(c + 32);
    uint64_t off_pos = rd64(c + 80);
    if (id >= n_bricks) return ST_INVALID;
    uint64_t a = rd64(c + off_pos + 8 * (uint64_t)id), b = rd64(c + off_pos + 8 * (uint64_t)id + 8);
    if (a > b || b > bytes || (a & 7) || b - a < 8) return ST_CORRUPT;
    r->rec = c + a;
    r->extent = b - a;
    r->coder = r->rec[0]; r->L = r->rec[1]; r->lb = r->rec[2]; r->log2W = r->rec[3];
    r->pc = rd32(r->rec + 4);
    if (r->L < 1 || r->L > 6) return ST_CORRUPT;
    if (lod < 0 || lod > r->L) return ST_INVALID;
    uint64_t S = (uint64_t)1 << (r->L - lod), n_out = S * S * S;
    if (per_word) n_out = (n_out + per_word - 1) / per_word; /* packed indices: 32-bit words */
    if (out_off > out_cap || n_out > out_cap - out_off) return ST_INVALID;
    *write_ok = 1;
    if (r->lb != (int)rd32(c + 24) || r->coder > 1 || (r->coder == CODER_RAW4 && r->log2W != 0) ||
        (r->coder == CODER_RANS && r->log2W > 8))
        return ST_CORRUPT;
    uint64_t hdr = record_header_bytes(r->L, r->coder, r->log2W);
    if (hdr > r->extent) return ST_CORRUPT;
    uint64_t pal_off = align_up(hdr, r->lb == 8 ? 8 : 4);
    if (pal_off > r->extent || (uint64_t)r->pc * (uint64_t)r->lb > r->extent - pal_off) return ST_CORRUPT;
    r->pal = r->rec + pal_off;
    r->payload = r->pal + (uint64_t)r->pc * r->lb;
    r->payload_bytes = r->extent - (pal_off + (uint64_t)r->pc * r->lb);
    for (int i = 0; i <= r->L; i++) r->sym_end[i] = rd32(r->rec + 8 + 4 * i);
    for (int i = 1; i <= r->L; i++)
        if (r->sym_end[i] < r->sym_end[i - 1]) return ST_CORRUPT;
    if ((uint64_t)r->sym_end[r->L] > 8 * total_nodes(r->L)) return ST_CORRUPT;
    if (r->coder == CODER_RAW4) {
        if ((uint64_t)r->sym_end[r->L] > 2 * r->payload_bytes) return ST_CORRUPT;
    } else {
        uint32_t W = 1u << r->log2W, G = (W + 63) / 64;
        r->gw = r->rec + 8 + 4 * (r->L + 1);
        r->states = r->gw + 4 * G;
        uint64_t tw = 0;
        for (uint32_t g = 0; g < G; g++) tw += rd32(r->gw + 4 * g);
        if (2 * tw > r->payload_bytes) return ST_CORRUPT;
        uint32_t fs = 0;
        for (int s = 0; s < 16; s++) fs += rd16(c + 48 + 2 * s);
        if (fs != RANS_M) return ST_CORRUPT;
    }
    return ST_OK;
}

/* the first n symbols of the record's stream; 0 or -1 (RANS words exhausted) */
static int read_symbols(const uint8_t* c, const rec_view* r, uint32_t n, uint8_t* sym) {
    if (r->coder == CODER_RAW4) {
        for (uint32_t j = 0; j < n; j++) sym[j] = (uint8_t)((r->payload[j / 2] >> (4 * (j & 1))) & 15);
        return 0;
    }
    uint32_t W = 1u << r->log2W, G = (W + 63) / 64;
    uint16_t freq[16];
    for (int s = 0; s < 16; s++) freq[s] = rd16(c + 48 + 2 * s);
    uint32_t* gw = (uint32_t*)malloc(sizeof(uint32_t) * G);
    uint32_t* st = (uint32_t*)malloc(sizeof(uint32_t) * W);
    uint64_t tw = 0;
    for (uint32_t g = 0; g < G; g++) { gw[g] = rd32(r->gw + 4 * g); tw += gw[g]; }
    for (uint32_t l = 0; l < W; l++) st[l] = rd32(r->states + 4 * l);
    uint16_t* words = (uint16_t*)malloc(sizeof(uint16_t) * (tw ? tw : 1));
    for (uint64_t k = 0; k < tw; k++) words[k] = rd16(r->payload + 2 * k);
    int rc = oracle_rans_decode(sym, n, freq, r->log2W, st, gw, words);
    free(gw); free(st); free(words);
    return rc;
}

/*
 * Cache-paletted output (Methods > Memory management > Cache paletting): n
 * palette indices of `bits` bits each (1..31) packed floor(32 / bits) to a
 * 32-bit word, index k in word k / e at bit (k % e) * bits (e = entries per
 * word), the unused high bits of every word zero.  Writes ceil(n / e) words.
 */
void oracle_pack_indices(const uint32_t* idx, uint64_t n, int bits, uint32_t* out) {
    uint64_t e = (uint64_t)(32 / bits), words = (n + e - 1) / e;
    for (uint64_t w = 0; w < words; w++) out[w] = 0;
    for (uint64_t k = 0; k < n; k++) out[k / e] |= idx[k] << ((k % e) * (uint64_t)bits);
}

/*
 * Decode brick `id` at LOD `lod` into out at element offset out_off:
 * S^3 labels (x fastest, S = b>>lod) when bits = 0, else the S^3 palette
 * indices packed by oracle_pack_indices into 32-bit words at word offset
 * out_off.  Level t = L - lod is reconstructed; levels 0..t are read in
 * order and nodes within a level in Morton order.  A node whose parent is
 * implied or stopped is implied and takes its parent's palette index; any
 * other node consumes one symbol s: op = s & 7, stop = s >> 3 (the stop bit
 * of level t is not needed).  PARENT copies the parent; NX/NY/NZ copy the
 * node at x-1 / y-1 / z-1 of the same level; ADV takes index n and n += 1;
 * LAST takes n-1; DELTA reads its entry chain into delta and takes n-delta,
 * where n counts the ADV operations so far.  A voxel's label is the palette
 * entry at its index.
 * CORRUPT verdicts: PARENT at level 0, a neighbour outside the brick,
 * ADV with n >= palette_count, LAST with n = 0, delta = 0 or > n, op 7,
 * a level whose symbols do not end exactly at sym_end[level] (including a
 * delta chain running past it), RANS words exhausted, and at t = L an ADV
 * count different from palette_count.  With bits > 0 a task that passes the
 * record checks is INVALID (output untouched) when t = 6 or the record's
 * palette has more than 2^bits entries.
 */
static int decode_one(const uint8_t* c, uint64_t bytes, uint32_t id, int lod, uint64_t out_off, uint64_t out_cap, void* out,
                      int lb_vol, int bits) {
    rec_view r;
    int write_ok;
    memset(&r, 0, sizeof(r));
    uint32_t per_word = bits ? (uint32_t)(32 / bits) : 0;
    int st = parse_record(c, bytes, id, lod, out_off, out_cap, per_word, &r, &write_ok);
    int L = r.L, t = L - lod;
    uint64_t S = write_ok ? (uint64_t)1 << t : 0, n_out = S * S * S;
    uint64_t n_units = per_word ? (n_out + per_word - 1) / per_word : n_out;
    uint64_t* G[7] = {0};
    uint8_t* expand[7] = {0};
    uint8_t* sym = NULL;
    if (st == ST_OK && bits && (t == 6 || (uint64_t)r.pc > ((uint64_t)1 << bits))) return ST_INVALID;
    if (st != ST_OK) goto done;
    {
        uint32_t nsym = r.sym_end[t];
        sym = (uint8_t*)malloc(nsym ? nsym : 1);
        if (read_symbols(c, &r, nsym, sym) != 0) { st = ST_CORRUPT; goto done; }
        uint32_t pos = 0, n = 0;
        for (int i = 0; i <= t && st == ST_OK; i++) {
            size_t nn = (size_t)1 << (3 * i);
            G[i] = (uint64_t*)calloc(nn, sizeof(uint64_t));
            expand[i] = (uint8_t*)calloc(nn, 1);
            for (size_t m = 0; m < nn && st == ST_OK; m++) {
                if (i > 0 && !expand[i - 1][m >> 3]) { G[i][m] = G[i - 1][m >> 3]; continue; }
                if (pos >= r.sym_end[i]) { st = ST_CORRUPT; break; }
                uint32_t s = sym[pos++], op = s & 7, stop = (s >> 3) & 1;
                uint32_t x, y, z;
                demorton((uint32_t)m, i, &x, &y, &z);
                uint64_t v = 0;
                switch (op) {
                case OP_PARENT:
                    if (i == 0) st = ST_CORRUPT;
                    else v = G[i - 1][m >> 3];
                    break;
                case OP_NX:
                    if (x == 0) st = ST_CORRUPT;
                    else v = G[i][morton(x - 1, y, z, i)];
                    break;
                case OP_NY:
                    if (y == 0) st = ST_CORRUPT;
                    else v = G[i][morton(x, y - 1, z, i)];
                    break;
                case OP_NZ:
                    if (z == 0) st = ST_CORRUPT;
                    else v = G[i][morton(x, y, z - 1, i)];
                    break;
                case OP_ADV:
                    if (n >= r.pc) st = ST_CORRUPT;
                    else v = n++;
                    break;
                case OP_LAST:
                    if (n == 0) st = ST_CORRUPT;
                    else v = n - 1;
                    break;
                case OP_DELTA: {
                    uint64_t delta = 0;
                    uint32_t e;
                    do {
                        if (pos >= r.sym_end[i]) { st = ST_CORRUPT; break; }
                        e = sym[pos++];
                        delta = delta_step(delta, e);
                    } while (e & 8);
                    if (st == ST_OK && (delta == 0 || delta > n)) st = ST_CORRUPT;
                    if (st == ST_OK) v = n - (uint32_t)delta;
                    break;
                }
                default:
                    st = ST_CORRUPT;
                }
                G[i][m] = v;
                expand[i][m] = (uint8_t)!stop;
            }
            if (st == ST_OK && pos != r.sym_end[i]) st = ST_CORRUPT;
        }
        if (st == ST_OK && t == L && n != r.pc) st = ST_CORRUPT;
        if (st == ST_OK && !bits) {
            for (uint64_t zz = 0; zz < S; zz++)
                for (uint64_t yy = 0; yy < S; yy++)
                    for (uint64_t xx = 0; xx < S; xx++)
                        put_label(out, lb_vol, out_off + (zz * S + yy) * S + xx,
                                  get_label(r.pal, r.lb, G[t][morton((uint32_t)xx, (uint32_t)yy, (uint32_t)zz, t)]));
        } else if (st == ST_OK) {
            uint32_t* idx = (uint32_t*)malloc(sizeof(uint32_t) * n_out);
            for (uint64_t zz = 0; zz < S; zz++)
                for (uint64_t yy = 0; yy < S; yy++)
                    for (uint64_t xx = 0; xx < S; xx++)
                        idx[(zz * S + yy) * S + xx] =
                            (uint32_t)G[t][morton((uint32_t)xx, (uint32_t)yy, (uint32_t)zz, t)];
            oracle_pack_indices(idx, n_out, bits, (uint32_t*)out + out_off);
            free(idx);
        }
    }
done:
    if (st == ST_CORRUPT && write_ok)
        for (uint64_t k = 0; k < n_units; k++) {
            if (bits) ((uint32_t*)out)[out_off + k] = 0;
            else put_label(out, lb_vol, out_off + k, 0);
        }
    for (int i = 0; i < 7; i++) { free(G[i]); free(expand[i]); }
    free(sym);
    return st;
}

/*
 * Decode a task list: task j decodes brick ids[j] at lods[j] into
 * out[out_offsets[j] ...] (element offsets, labels of the volume's width).
 * status[j] gets 0 (ok), 1 (invalid task: output untouched) or 2 (corrupt
 * record: output zero-filled when its range is valid).  Returns 0, or -1
 * when the container header itself is unusable.
 */
static int decode_list(const uint8_t* c, uint64_t bytes, const uint32_t* ids, const uint8_t* lods,
                       const uint64_t* out_offsets, uint32_t n, void* out, uint64_t out_cap, uint32_t* status,
                       int bits, int nthreads) {
    if (bytes < OR_HDR_BYTES || rd32(c) != OR_MAGIC || rd32(c + 4) != OR_VERSION) return -1;
    int lb = (int)rd32(c + 24);
    if (lb != 4 && lb != 8) return -1;
    uint64_t nb = rd32(c + 32), off_pos = rd64(c + 80);
    if (off_pos > bytes || 8 * (nb + 1) > bytes - off_pos) return -1;
    (void)nthreads;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
    for (long j = 0; j < (long)n; j++)
        status[j] = (uint32_t)decode_one(c, bytes, ids[j], lods[j], out_offsets[j], out_cap, out, lb, bits);
    return 0;
}

int oracle_decode_tasks(const uint8_t* c, uint64_t bytes, const uint32_t* ids, const uint8_t* lods,
                        const uint64_t* out_offsets, uint32_t n, void* out, uint64_t out_cap, uint32_t* status,
                        int nthreads) {
    return decode_list(c, bytes, ids, lods, out_offsets, n, out, out_cap, status, 0, nthreads);
}

/*
 * The same task list decoded to cache-paletted form: out is 32-bit words,
 * out_offsets and out_cap count words, task j writes its packed indices
 * (oracle_pack_indices with `bits`, 1..31) at word out_offsets[j].
 * Returns 0, or -1 for an unusable header or bits outside 1..31.
 */
int oracle_decode_tasks_paletted(const uint8_t* c, uint64_t bytes, const uint32_t* ids, const uint8_t* lods,
                                 const uint64_t* out_offsets, uint32_t n, uint32_t* out, uint64_t out_cap,
                                 uint32_t* status, int bits, int nthreads) {
    if (bits < 1 || bits > 31) return -1;
    return decode_list(c, bytes, ids, lods, out_offsets, n, out, out_cap, status, bits, nthreads);
}

/* ------------------------------------------------------------ inspection */
/*
 * Palette of one record (for tests): copies up to cap entries of the
 * volume's label width into out; returns the palette count, or -1.
 */
int64_t oracle_record_palette(const uint8_t* c, uint64_t bytes, uint32_t id, uint64_t* out, uint32_t cap) {
    rec_view r;
    int write_ok;
    memset(&r, 0, sizeof(r));
    if (bytes < OR_HDR_BYTES || parse_record(c, bytes, id, 0, 0, UINT64_MAX, 0, &r, &write_ok) != ST_OK) return -1;
    for (uint32_t k = 0; k < r.pc && k < cap; k++) out[k] = get_label(r.pal, r.lb, k);
    return (int64_t)r.pc;
}

/*
 * Symbol stream and palette of one record (for tests).  Fills sym (cap
 * entries), sym_end (7), and returns the symbol count (sym_end[L]), or -1.
 */
int64_t oracle_record_symbols(const uint8_t* c, uint64_t bytes, uint32_t id, uint8_t* sym, uint32_t cap,
                              uint32_t* sym_end, uint32_t* info) {
    rec_view r;
    int write_ok;
    memset(&r, 0, sizeof(r));
    if (parse_record(c, bytes, id, 0, 0, UINT64_MAX, 0, &r, &write_ok) != ST_OK) return -1;
    if (r.sym_end[r.L] > cap) return -1;
    if (read_symbols(c, &r, r.sym_end[r.L], sym) != 0) return -1;
    for (int i = 0; i <= r.L; i++) sym_end[i] = r.sym_end[i];
    info[0] = (uint32_t)r.coder; info[1] = (uint32_t)r.L; info[2] = (uint32_t)r.lb; info[3] = (uint32_t)r.log2W;
    info[4] = r.pc; info[5] = (uint32_t)r.extent;
    return r.sym_end[r.L];
}
