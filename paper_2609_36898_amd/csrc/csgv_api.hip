// C ABI of the decoder: argument checks, scratch, the plain and persistent
// launch forms, and batched plans (cost-sorted queue, captured HIP graph).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/csgv.h"
#include "csgv_format.h"
#include "decode_kernel.h"

using namespace csgv;

namespace {

thread_local std::string g_last_error;

csgv_status fail(csgv_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(CSGV_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

uint32_t rd32(const uint8_t* p) {
    uint32_t v;
    memcpy(&v, p, 4);
    return v;
}
uint64_t rd64(const uint8_t* p) {
    uint64_t v;
    memcpy(&v, p, 8);
    return v;
}

std::once_flag g_attr_once;
hipError_t g_attr_err = hipSuccess;

hipError_t ensure_attrs() {
    std::call_once(g_attr_once, [] { g_attr_err = set_kernel_attrs(); });
    return g_attr_err;
}

int device_cus() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
    return n;
}

int device_lds_per_cu() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 160 * 1024;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess || n <= 0)
        return 160 * 1024;
    return n;
}

bool valid_wg(int wg) { return wg == 128 || wg == 256 || wg == 512 || wg == 1024; }

// resident work-groups per CU for a shape (HIP occupancy: registers, LDS, waves)
int resident_per_cu(int wg, uint32_t cap16) {
    const int by_lds = device_lds_per_cu() / (int)shared_bytes(cap16);
    return std::max(1, std::min(by_lds, max_resident_per_cu(wg, std::max<uint32_t>(cap16, kMinCap16))));
}

RansFreq pack_freq(const csgv_volume_info* vol, bool* ok) {
    RansFreq f;
    uint32_t sum = 0;
    for (int s = 0; s < 16; ++s) sum += vol->rans_freq[s];
    *ok = sum == kRansM;
    for (int k = 0; k < 8; ++k) f.w[k] = (uint32_t)vol->rans_freq[2 * k] | ((uint32_t)vol->rans_freq[2 * k + 1] << 16);
    return f;
}

Params make_params(const csgv_volume_info* vol, const void* d_container, const uint32_t* ids, const uint8_t* lods,
                   const uint64_t* offs, uint32_t n, void* out, uint64_t cap, uint32_t* status) {
    Params P;
    memset(&P, 0, sizeof(P));
    P.vol = (const uint8_t*)d_container;
    P.vol_bytes = vol->total_bytes;
    P.off_pos = vol->offsets_pos;
    P.n_bricks = vol->n_bricks;
    P.label_bytes = vol->label_bytes;
    bool ok;
    (void)pack_freq(vol, &ok);
    P.freq_ok = ok;
    P.max_log2b = vol->max_log2b ? std::min<uint32_t>(vol->max_log2b, kMaxLog2b) : kMaxLog2b;
    P.ids = ids;
    P.lods = lods;
    P.out_offs = offs;
    P.n_tasks = n;
    P.out = (uint8_t*)out;
    P.out_cap = cap;
    P.status = status;
    P.scratch_stride = scratch_per_wg(P.max_log2b);
    P.cap16 = kDefaultCap16;
    return P;
}

csgv_status check_task_args(const csgv_volume_info* vol, const void* d_container, const uint32_t* ids,
                            const uint8_t* lods, uint32_t n, void* out) {
    if (!vol) return fail(CSGV_EINVAL, "volume info is NULL");
    if (vol->label_bytes != 4 && vol->label_bytes != 8) return fail(CSGV_EINVAL, "label_bytes must be 4 or 8");
    if (vol->offsets_pos < kHeaderBytes || vol->offsets_pos + 8ull * ((uint64_t)vol->n_bricks + 1) > vol->total_bytes)
        return fail(CSGV_EINVAL, "offset table outside the container");
    if (n == 0) return CSGV_OK;
    if (!d_container || !ids || !lods || !out) return fail(CSGV_EINVAL, "NULL device pointer");
    return CSGV_OK;
}

csgv_status check_opts(const csgv_decode_opts* o) {
    if (!o) return CSGV_OK;
    if (o->wg_size != 0 && !valid_wg(o->wg_size)) return fail(CSGV_EINVAL, "wg_size %d (128, 256, 512 or 1024)", o->wg_size);
    if (o->lds_slots < 0 || (uint32_t)o->lds_slots > kMaxCap16)
        return fail(CSGV_EINVAL, "lds_slots %d (0, or %u..%u)", o->lds_slots, kMinCap16, kMaxCap16);
    if (o->lds_slots > 0 && (uint32_t)o->lds_slots < kMinCap16)
        return fail(CSGV_EINVAL, "lds_slots %d below %u (the slot area also holds the rANS table)", o->lds_slots,
                    kMinCap16);
    if (o->bricks_per_wave < 0) return fail(CSGV_EINVAL, "bricks_per_wave %d", o->bricks_per_wave);
    if (o->wgs_per_cu < -1) return fail(CSGV_EINVAL, "wgs_per_cu %d", o->wgs_per_cu);
    if (o->palette_bits < -1 || o->palette_bits > 31) return fail(CSGV_EINVAL, "palette_bits %d (0..31)", o->palette_bits);
    return CSGV_OK;
}

// device memory of one launch sequence (a plan's, or a one-shot call's)
struct Bufs {
    uint8_t* scratch = nullptr;
    uint32_t* queue = nullptr;
    uint32_t* hist = nullptr;   // 128
    uint32_t* cls = nullptr;    // max_tasks
    uint32_t* order = nullptr;  // max_tasks
    uint32_t* rans_tab = nullptr;
    uint64_t* dense = nullptr;  // max_tasks
    bool table_built = false;   // rans_tab already holds the volume's table
};

uint64_t aux_bytes(uint32_t max_tasks) {
    return 256 + 4 * 128 + 8ull * max_tasks + 4ull * kRansM + 8ull * max_tasks + 256;
}

void carve(uint8_t* base, uint64_t scratch_bytes, uint32_t max_tasks, Bufs* b) {
    b->scratch = base;
    uint8_t* a = base + scratch_bytes;
    b->queue = (uint32_t*)a;
    b->hist = (uint32_t*)(a + 256);
    b->cls = b->hist + 128;
    b->order = b->cls + max_tasks;
    b->rans_tab = b->order + max_tasks;
    uint8_t* d = (uint8_t*)(b->rans_tab + kRansM);
    d = (uint8_t*)(((uintptr_t)d + 255) & ~(uintptr_t)255);
    b->dense = (uint64_t*)d;
}

// everything a persistent launch enqueues, in order
hipError_t enqueue_persistent(Params P, const Bufs& b, const csgv_volume_info* vol, int wg, uint32_t grid, bool sort,
                              hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    P.scratch = b.scratch;
    P.queue = b.queue;
    P.rans_tab = b.rans_tab;
    hipError_t e = launch_reset(P.queue, s);
    if (e != hipSuccess) return e;
    bool ok;
    const RansFreq f = pack_freq(vol, &ok);
    if (ok && !b.table_built && (e = launch_rans_table(b.rans_tab, f, s)) != hipSuccess) return e;
    if (!P.out_offs) {
        P.dense_offs = b.dense;
        if ((e = launch_dense_offsets(P, b.dense, s)) != hipSuccess) return e;
    }
    // with no more tasks than work-groups every task starts at once: order is moot
    if (sort && P.n_tasks > grid) {
        if ((e = launch_sort(P, b.cls, b.hist, b.order, s)) != hipSuccess) return e;
        P.order = b.order;
    }
    if (ev0 && (e = hipEventRecord(ev0, s)) != hipSuccess) return e;
    if ((e = launch_decode(P, wg, grid, s)) != hipSuccess) return e;
    if (ev1 && (e = hipEventRecord(ev1, s)) != hipSuccess) return e;
    return hipSuccess;
}

}  // namespace

// ------------------------------------------------------------------ C ABI
extern "C" {

const char* csgv_last_error(void) { return g_last_error.c_str(); }

csgv_status csgv_volume_parse(const void* h_container, uint64_t bytes, csgv_volume_info* out) {
    if (!h_container || !out) return fail(CSGV_EINVAL, "NULL argument");
    if (bytes < kHeaderBytes) return fail(CSGV_EINVAL, "container shorter than its header");
    const uint8_t* h = (const uint8_t*)h_container;
    if (rd32(h) != kMagic) return fail(CSGV_EINVAL, "bad magic");
    if (rd32(h + 4) != kVersion) return fail(CSGV_EINVAL, "unsupported version %u", rd32(h + 4));
    csgv_volume_info v;
    memset(&v, 0, sizeof(v));
    for (int a = 0; a < 3; ++a) {
        v.dims[a] = rd32(h + kHdrDims + 4 * a);
        v.grid[a] = rd32(h + kHdrGrid + 4 * a);
    }
    v.log2b = rd32(h + kHdrLog2b);
    v.label_bytes = rd32(h + kHdrLabelBytes);
    v.op_mask = rd32(h + kHdrOpMask);
    v.n_bricks = rd32(h + kHdrNBricks);
    memcpy(v.rans_freq, h + kHdrFreq, 32);
    v.offsets_pos = rd64(h + kHdrOffsetsPos);
    v.dir_pos = rd64(h + kHdrDirPos);
    v.total_bytes = rd64(h + kHdrTotal);
    v.neighbor_mode = rd32(h + kHdrNeighborMode);
    if (v.label_bytes != 4 && v.label_bytes != 8) return fail(CSGV_EINVAL, "label_bytes %u", v.label_bytes);
    if (v.total_bytes > bytes)
        return fail(CSGV_EINVAL, "header claims %llu bytes, only %llu given", (unsigned long long)v.total_bytes,
                    (unsigned long long)bytes);
    if (v.offsets_pos < kHeaderBytes || v.offsets_pos > v.total_bytes ||
        8ull * ((uint64_t)v.n_bricks + 1) > v.total_bytes - v.offsets_pos)
        return fail(CSGV_EINVAL, "offset table outside the container");
    // largest brick side any record claims (sizes the decoder's scratch)
    // and the largest palette (|P|max of cache paletting)
    uint32_t mx = 0, mp = 0;
    for (uint64_t k = 0; k < v.n_bricks; ++k) {
        const uint64_t a = rd64(h + v.offsets_pos + 8 * k), b = rd64(h + v.offsets_pos + 8 * k + 8);
        if (a > b || b > v.total_bytes || b - a < 8) continue;
        const uint32_t L = h[a + 1];
        if (L >= 1 && L <= kMaxLog2b) mx = std::max(mx, L);
        mp = std::max(mp, rd32(h + a + 4));
    }
    v.max_log2b = mx ? mx : 1;
    v.max_palette = mp;
    *out = v;
    return CSGV_OK;
}

}  // extern "C"

namespace {

// Enqueue one call of csgv_decode_bricks on buffers b (scratch of `grid`
// work-groups in persistent mode, of one in plain mode).
csgv_status decode_on(hipStream_t stream, const csgv_volume_info* vol, Params P, const csgv_decode_opts* opts,
                      int mode, int wg, uint32_t grid, const Bufs& b) {
    hipError_t e = hipSuccess;
    if (mode == CSGV_MODE_PERSISTENT) {
        const bool sort = opts ? opts->sort_tasks != 0 : true;
        e = enqueue_persistent(P, b, vol, wg, grid, sort, stream, nullptr, nullptr);
    } else {
        P.scratch = b.scratch;
        P.rans_tab = b.rans_tab;
        bool ok;
        const RansFreq f = pack_freq(vol, &ok);
        if (ok) e = launch_rans_table(b.rans_tab, f, stream);
        if (e == hipSuccess && !P.out_offs) {
            P.dense_offs = b.dense;
            e = launch_dense_offsets(P, b.dense, stream);
        }
        for (uint32_t j = 0; j < P.n_tasks && e == hipSuccess; ++j) {
            P.task0 = j;
            e = launch_decode(P, wg, 1, stream);
        }
    }
    if (e != hipSuccess) return fail(CSGV_EHIP, "decode launch: %s", hipGetErrorString(e));
    return CSGV_OK;
}

// checks shared by both one-shot entry points; fills P, the mode and the shape
csgv_status prepare_call(const csgv_volume_info* vol, const void* d_container, const uint32_t* d_brick_ids,
                         const uint8_t* d_lods, const uint64_t* d_out_offsets, uint32_t n, void* d_out,
                         uint64_t out_capacity, uint32_t* d_status, const csgv_decode_opts* opts, Params* P, int* mode,
                         int* wg, int* per_cu) {
    csgv_status st = check_task_args(vol, d_container, d_brick_ids, d_lods, n, d_out);
    if (st != CSGV_OK || n == 0) return st;  // n = 0 enqueues nothing
    if ((st = check_opts(opts)) != CSGV_OK) return st;
    HIP_TRY(ensure_attrs());
    *mode = opts ? opts->mode : CSGV_MODE_PLAIN;
    if (*mode != CSGV_MODE_PLAIN && *mode != CSGV_MODE_PERSISTENT) return fail(CSGV_EINVAL, "unknown mode %d", *mode);
    *P = make_params(vol, d_container, d_brick_ids, d_lods, d_out_offsets, n, d_out, out_capacity, d_status);
    if (opts && opts->lds_slots > 0) P->cap16 = std::max<uint32_t>((uint32_t)opts->lds_slots, kMinCap16) & ~7u;
    if (opts && opts->palette_bits > 0) P->pal_bits = (uint32_t)opts->palette_bits;
    *wg = opts && opts->wg_size ? opts->wg_size : 256;
    *per_cu = opts && opts->wgs_per_cu > 0 ? opts->wgs_per_cu : resident_per_cu(*wg, P->cap16);
    return CSGV_OK;
}

}  // namespace

extern "C" {

csgv_status csgv_decode_bricks(hipStream_t stream, const csgv_volume_info* vol, const void* d_container,
                               const uint32_t* d_brick_ids, const uint8_t* d_lods, const uint64_t* d_out_offsets,
                               uint32_t n, void* d_out, uint64_t out_capacity, uint32_t* d_status,
                               const csgv_decode_opts* opts) {
    Params P;
    int mode, wg, per_cu;
    csgv_status st = prepare_call(vol, d_container, d_brick_ids, d_lods, d_out_offsets, n, d_out, out_capacity,
                                  d_status, opts, &P, &mode, &wg, &per_cu);
    if (st != CSGV_OK || n == 0) return st;
    uint32_t grid = 1;
    if (mode == CSGV_MODE_PERSISTENT) grid = (uint32_t)std::min<uint64_t>((uint64_t)device_cus() * per_cu, n);
    const uint64_t sb = P.scratch_stride * grid;
    void* mem = nullptr;
    HIP_TRY(hipMallocAsync(&mem, sb + aux_bytes(n), stream));
    Bufs b;
    carve((uint8_t*)mem, sb, n, &b);
    st = decode_on(stream, vol, P, opts, mode, wg, grid, b);
    hipError_t e2 = hipFreeAsync(mem, stream);
    if (st != CSGV_OK) return st;
    if (e2 != hipSuccess) return fail(CSGV_EHIP, "hipFreeAsync: %s", hipGetErrorString(e2));
    return CSGV_OK;
}

csgv_status csgv_check_status(const uint32_t* d_status, uint32_t n, hipStream_t stream) {
    if (n == 0) return CSGV_OK;
    if (!d_status) return fail(CSGV_EINVAL, "NULL status");
    std::vector<uint32_t> h(n);
    HIP_TRY(hipMemcpyAsync(h.data(), d_status, 4ull * n, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    for (uint32_t j = 0; j < n; ++j)
        if (h[j]) return fail(CSGV_ECORRUPT, "task %u status %u", j, h[j]);
    return CSGV_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ plans
struct csgv_plan {
    csgv_volume_info vol;
    uint32_t max_tasks = 0;
    csgv_decode_opts opts;
    uint32_t grid = 0;
    uint64_t scratch_bytes = 0;
    uint8_t* mem = nullptr;
    Bufs b;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t exec = nullptr;
    bool use_graph = true;
    bool timing = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool ev_valid = false;
    // arguments the cached graph was captured with
    struct Key {
        const void* c;
        const void* ids;
        const void* lods;
        const void* offs;
        uint32_t n;
        void* out;
        uint64_t cap;
        void* status;
        int wg, grid, sort, cap16, pal_bits;
        bool operator==(const Key& o) const { return memcmp(this, &o, sizeof(Key)) == 0; }
    } key;
    bool have_key = false;
};

namespace {

uint32_t plan_grid(const csgv_plan* p, uint32_t n) {
    return std::min<uint32_t>(p->grid, std::max<uint32_t>(n, 1));
}

csgv_status plan_enqueue(csgv_plan* p, hipStream_t s, const Params& P0, bool with_events) {
    Params P = P0;
    P.cap16 = std::max<uint32_t>((uint32_t)p->opts.lds_slots, kMinCap16) & ~7u;
    P.pal_bits = p->opts.palette_bits > 0 ? (uint32_t)p->opts.palette_bits : 0u;
    hipError_t e = enqueue_persistent(P, p->b, &p->vol, p->opts.wg_size, plan_grid(p, P.n_tasks),
                                      p->opts.sort_tasks != 0, s, with_events ? p->ev0 : nullptr,
                                      with_events ? p->ev1 : nullptr);
    if (e != hipSuccess) return fail(CSGV_EHIP, "plan launch: %s", hipGetErrorString(e));
    return CSGV_OK;
}

// (re)size the plan's grid and scratch for its current shape
csgv_status plan_alloc(csgv_plan* p) {
    const int per_cu = p->opts.wgs_per_cu > 0 ? p->opts.wgs_per_cu : resident_per_cu(p->opts.wg_size, p->opts.lds_slots);
    const uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)device_cus() * per_cu, p->max_tasks);
    const uint32_t lmax = p->vol.max_log2b ? std::min<uint32_t>(p->vol.max_log2b, kMaxLog2b) : kMaxLog2b;
    const uint64_t sb = scratch_per_wg(lmax) * grid;
    if (p->mem && grid <= p->grid && sb <= p->scratch_bytes) {
        p->grid = grid;
        return CSGV_OK;
    }
    if (p->mem) {
        (void)hipDeviceSynchronize();
        (void)hipFree(p->mem);
        p->mem = nullptr;
    }
    hipError_t e = hipMalloc(&p->mem, sb + aux_bytes(p->max_tasks));
    if (e != hipSuccess) return fail(CSGV_ENOMEM, "plan scratch (%llu bytes): %s", (unsigned long long)sb,
                                     hipGetErrorString(e));
    carve(p->mem, sb, p->max_tasks, &p->b);
    p->grid = grid;
    p->scratch_bytes = sb;
    // the volume's rANS table, built once for every launch of the plan
    bool ok;
    const RansFreq f = pack_freq(&p->vol, &ok);
    if (ok) {
        if ((e = launch_rans_table(p->b.rans_tab, f, nullptr)) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess)
            return fail(CSGV_EHIP, "rANS table: %s", hipGetErrorString(e));
    }
    p->b.table_built = true;
    return CSGV_OK;
}

}  // namespace

extern "C" {

csgv_status csgv_plan_create(const csgv_volume_info* vol, uint32_t max_tasks, const csgv_decode_opts* opts,
                             csgv_plan** out) {
    if (!vol || !out) return fail(CSGV_EINVAL, "NULL argument");
    if (max_tasks == 0) return fail(CSGV_EINVAL, "max_tasks must be positive");
    csgv_status st = check_opts(opts);
    if (st != CSGV_OK) return st;
    HIP_TRY(ensure_attrs());
    csgv_plan* p = new csgv_plan();
    p->vol = *vol;
    p->max_tasks = max_tasks;
    p->opts.mode = CSGV_MODE_PERSISTENT;
    p->opts.wg_size = opts && opts->wg_size ? opts->wg_size : 256;
    p->opts.wgs_per_cu = opts && opts->wgs_per_cu > 0 ? opts->wgs_per_cu : 0;
    p->opts.sort_tasks = opts && opts->sort_tasks >= 0 ? opts->sort_tasks : 1;
    p->opts.bricks_per_wave = opts && opts->bricks_per_wave > 0 ? opts->bricks_per_wave : 1;
    p->opts.lds_slots = opts && opts->lds_slots > 0 ? opts->lds_slots : (int)kDefaultCap16;
    p->opts.palette_bits = opts && opts->palette_bits > 0 ? opts->palette_bits : 0;
    if ((st = plan_alloc(p)) != CSGV_OK) {
        delete p;
        return st;
    }
    if (hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&p->ev0) != hipSuccess || hipEventCreate(&p->ev1) != hipSuccess) {
        csgv_plan_destroy(p);
        return fail(CSGV_EHIP, "plan stream/events");
    }
    *out = p;
    return CSGV_OK;
}

csgv_status csgv_plan_set_graph(csgv_plan* p, int enable) {
    if (!p) return fail(CSGV_EINVAL, "NULL plan");
    p->use_graph = enable != 0;
    return CSGV_OK;
}

csgv_status csgv_plan_set_timing(csgv_plan* p, int enable) {
    if (!p) return fail(CSGV_EINVAL, "NULL plan");
    p->timing = enable != 0;
    return CSGV_OK;
}

csgv_status csgv_plan_set_opts(csgv_plan* p, const csgv_decode_opts* o) {
    if (!p || !o) return fail(CSGV_EINVAL, "NULL argument");
    csgv_status st = check_opts(o);
    if (st != CSGV_OK) return st;
    csgv_decode_opts n = p->opts;
    if (o->wg_size) n.wg_size = o->wg_size;
    if (o->wgs_per_cu >= 0) n.wgs_per_cu = o->wgs_per_cu;
    if (o->sort_tasks >= 0) n.sort_tasks = o->sort_tasks ? 1 : 0;
    if (o->bricks_per_wave > 0) n.bricks_per_wave = o->bricks_per_wave;
    if (o->lds_slots > 0) n.lds_slots = o->lds_slots;
    if (o->palette_bits >= 0) n.palette_bits = o->palette_bits;
    const csgv_decode_opts old = p->opts;
    p->opts = n;
    if ((st = plan_alloc(p)) != CSGV_OK) {
        p->opts = old;
        return st;
    }
    p->have_key = false;
    return CSGV_OK;
}

csgv_status csgv_plan_launch(csgv_plan* p, hipStream_t stream, const void* d_container, const uint32_t* d_brick_ids,
                             const uint8_t* d_lods, const uint64_t* d_out_offsets, uint32_t n, void* d_out,
                             uint64_t out_capacity, uint32_t* d_status) {
    if (!p) return fail(CSGV_EINVAL, "NULL plan");
    csgv_status st = check_task_args(&p->vol, d_container, d_brick_ids, d_lods, n, d_out);
    if (st != CSGV_OK) return st;
    if (n == 0) return CSGV_OK;
    if (n > p->max_tasks) return fail(CSGV_EINVAL, "n = %u exceeds the plan's max_tasks = %u", n, p->max_tasks);
    Params P = make_params(&p->vol, d_container, d_brick_ids, d_lods, d_out_offsets, n, d_out, out_capacity, d_status);
    if (p->timing || !p->use_graph) {
        st = plan_enqueue(p, stream, P, p->timing);
        p->ev_valid = st == CSGV_OK && p->timing;
        return st;
    }
    csgv_plan::Key k;
    memset(&k, 0, sizeof(k));
    k.c = d_container; k.ids = d_brick_ids; k.lods = d_lods; k.offs = d_out_offsets; k.n = n; k.out = d_out;
    k.cap = out_capacity; k.status = d_status; k.wg = p->opts.wg_size; k.grid = (int)p->grid;
    k.sort = p->opts.sort_tasks; k.cap16 = p->opts.lds_slots; k.pal_bits = p->opts.palette_bits;
    if (!p->have_key || !(k == p->key) || !p->exec) {
        if (p->exec) {
            (void)hipGraphExecDestroy(p->exec);
            p->exec = nullptr;
        }
        HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
        st = plan_enqueue(p, p->cap_stream, P, false);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
        if (st != CSGV_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return fail(CSGV_EHIP, "end capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail(CSGV_EHIP, "graph instantiate: %s", hipGetErrorString(e));
        p->key = k;
        p->have_key = true;
    }
    HIP_TRY(hipGraphLaunch(p->exec, stream));
    p->ev_valid = false;
    return CSGV_OK;
}

csgv_status csgv_plan_get_opts(const csgv_plan* p, csgv_decode_opts* out) {
    if (!p || !out) return fail(CSGV_EINVAL, "NULL argument");
    *out = p->opts;
    if (out->wgs_per_cu == 0) out->wgs_per_cu = (int)(p->grid / std::max(1, device_cus()));
    return CSGV_OK;
}

csgv_status csgv_plan_last_kernel_ms(csgv_plan* p, float* ms) {
    if (!p || !ms) return fail(CSGV_EINVAL, "NULL argument");
    if (!p->ev_valid) return fail(CSGV_EINVAL, "no timed launch recorded (enable timing first)");
    HIP_TRY(hipEventSynchronize(p->ev1));
    HIP_TRY(hipEventElapsedTime(ms, p->ev0, p->ev1));
    return CSGV_OK;
}

void csgv_plan_destroy(csgv_plan* p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    if (p->mem) (void)hipFree(p->mem);
    delete p;
}

void csgv_free_host(void* p) { free(p); }

}  // extern "C"

// ------------------------------------------------------------------ autotuner
namespace {

std::string tune_key(const csgv_plan* p, const std::vector<uint8_t>& lods, uint32_t n) {
    int dev = 0;
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch = arch.substr(0, colon);
    }
    uint32_t hist[8] = {0};
    for (uint8_t l : lods) ++hist[l < 7 ? l : 7];
    char buf[512];
    snprintf(buf, sizeof(buf), "%s|cus=%d|lb=%u|L=%u|bricks=%u|bytes=%llu|n=%u|lods=%u,%u,%u,%u,%u,%u,%u,%u|I=%d",
             arch.c_str(), device_cus(), p->vol.label_bytes, p->vol.max_log2b, p->vol.n_bricks,
             (unsigned long long)p->vol.total_bytes, n, hist[0], hist[1], hist[2], hist[3], hist[4], hist[5],
             hist[6], hist[7], p->opts.palette_bits);
    return buf;
}

bool tune_lookup(const char* path, const std::string& key, csgv_decode_opts* o) {
    if (!path) return false;
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    while (fgets(line, sizeof(line), f)) {
        char* tab = strchr(line, '\t');
        if (!tab) continue;
        *tab = 0;
        int wg, lds, wpc;
        if (key == line && sscanf(tab + 1, "%d %d %d", &wg, &lds, &wpc) == 3) {
            o->wg_size = wg;
            o->lds_slots = lds;
            o->wgs_per_cu = wpc;
            found = true;  // the last matching line wins
        }
    }
    fclose(f);
    return found;
}

void tune_store(const char* path, const std::string& key, const csgv_decode_opts& o) {
    if (!path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s\t%d %d %d\n", key.c_str(), o.wg_size, o.lds_slots, o.wgs_per_cu);
    fclose(f);
}

}  // namespace

extern "C" csgv_status csgv_plan_autotune(csgv_plan* p, hipStream_t stream, const void* d_container,
                                          const uint32_t* d_brick_ids, const uint8_t* d_lods,
                                          const uint64_t* d_out_offsets, uint32_t n, void* d_out,
                                          uint64_t out_capacity, uint32_t* d_status, const char* cache_path,
                                          csgv_tune_report* report) {
    if (!p) return fail(CSGV_EINVAL, "NULL plan");
    csgv_status st = check_task_args(&p->vol, d_container, d_brick_ids, d_lods, n, d_out);
    if (st != CSGV_OK) return st;
    if (n == 0 || n > p->max_tasks) return fail(CSGV_EINVAL, "n = %u (plan max_tasks %u)", n, p->max_tasks);
    std::vector<uint8_t> lods(n);
    HIP_TRY(hipMemcpyAsync(lods.data(), d_lods, n, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    const std::string key = tune_key(p, lods, n);
    csgv_tune_report rep;
    memset(&rep, 0, sizeof(rep));
    csgv_decode_opts cached = p->opts;
    if (tune_lookup(cache_path, key, &cached)) {
        if ((st = csgv_plan_set_opts(p, &cached)) != CSGV_OK) return st;
        rep.from_cache = 1;
        rep.chosen = p->opts;
        if (report) *report = rep;
        return CSGV_OK;
    }
    const bool had_timing = p->timing;
    p->timing = true;
    const csgv_decode_opts start = p->opts;
    auto time_shape = [&](const csgv_decode_opts& o, float* best) -> csgv_status {
        csgv_status s2 = csgv_plan_set_opts(p, &o);
        if (s2 != CSGV_OK) return s2;
        *best = 1e30f;
        for (int rep_i = 0; rep_i < 4; ++rep_i) {
            s2 = csgv_plan_launch(p, stream, d_container, d_brick_ids, d_lods, d_out_offsets, n, d_out, out_capacity,
                                  d_status);
            if (s2 != CSGV_OK) return s2;
            float ms = 0;
            if ((s2 = csgv_plan_last_kernel_ms(p, &ms)) != CSGV_OK) return s2;
            if (rep_i > 0) *best = std::min(*best, ms);  // the first launch of a shape warms caches
        }
        return CSGV_OK;
    };
    static const int kWg[] = {128, 256, 512};
    static const int kLds[] = {8192, 10240, 16384, 24576};
    float best_ms = 1e30f;
    csgv_decode_opts best = start;
    int tried = 0;
    for (int wg : kWg)
        for (int lds : kLds) {
            csgv_decode_opts o = start;
            o.wg_size = wg;
            o.lds_slots = lds;
            o.wgs_per_cu = 0;
            float ms;
            st = time_shape(o, &ms);
            if (st != CSGV_OK) {
                p->timing = had_timing;
                return st;
            }
            ++tried;
            if (wg == 256 && lds == (int)kDefaultCap16) rep.default_ms = ms;
            if (ms < best_ms) {
                best_ms = ms;
                best = o;
            }
        }
    p->timing = had_timing;
    if ((st = csgv_plan_set_opts(p, &best)) != CSGV_OK) return st;
    tune_store(cache_path, key, best);
    rep.tried = tried;
    rep.best_ms = best_ms;
    rep.chosen = p->opts;
    if (report) *report = rep;
    return CSGV_OK;
}

// ------------------------------------------------- decode without allocating
// Scratch of csgv_decode_bricks_noalloc: one array per GPU the library runs
// on, held until the process ends.  Host code uses it only through the device
// address hipGetSymbolAddress returns on each device (the array's name is a
// host-side stand-in there).
static __device__ __align__(256) uint8_t scratch[CSGV_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
uint8_t* g_noalloc_base[kMaxDevices] = {};

// device address of this GPU's array, looked up once per device
csgv_status noalloc_base(uint8_t** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(CSGV_EINVAL, "device %d beyond the supported %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_base[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_noalloc_base[dev] = (uint8_t*)p;
    }
    *out = g_noalloc_base[dev];
    return CSGV_OK;
}

}  // namespace

extern "C" {

csgv_status csgv_decode_bricks_noalloc(hipStream_t stream, const csgv_volume_info* vol, const void* d_container,
                                       const uint32_t* d_brick_ids, const uint8_t* d_lods,
                                       const uint64_t* d_out_offsets, uint32_t n, void* d_out, uint64_t out_capacity,
                                       uint32_t* d_status, const csgv_decode_opts* opts) {
    Params P;
    int mode, wg, per_cu;
    csgv_status st = prepare_call(vol, d_container, d_brick_ids, d_lods, d_out_offsets, n, d_out, out_capacity,
                                  d_status, opts, &P, &mode, &wg, &per_cu);
    if (st != CSGV_OK || n == 0) return st;
    if (n > CSGV_NOALLOC_MAX_TASKS)
        return fail(CSGV_EINVAL, "n = %u exceeds the %u tasks of the fixed scratch", n, (uint32_t)CSGV_NOALLOC_MAX_TASKS);
    // per-task arrays for CSGV_NOALLOC_MAX_TASKS after the work-groups' scratch
    const uint64_t aux = aux_bytes(CSGV_NOALLOC_MAX_TASKS);
    const uint64_t sb = (CSGV_NOALLOC_SCRATCH_BYTES - aux) / 256 * 256;
    const uint64_t fit = sb / P.scratch_stride;
    if (fit == 0)
        return fail(CSGV_EINVAL, "records of brick side 2^%u need %llu scratch bytes per work-group, more than the "
                    "fixed scratch holds", P.max_log2b, (unsigned long long)P.scratch_stride);
    uint32_t grid = 1;
    if (mode == CSGV_MODE_PERSISTENT)
        grid = (uint32_t)std::min<uint64_t>(std::min<uint64_t>((uint64_t)device_cus() * per_cu, n), fit);
    uint8_t* base = nullptr;
    if ((st = noalloc_base(&base)) != CSGV_OK) return st;
    Bufs b;
    carve(base, sb, CSGV_NOALLOC_MAX_TASKS, &b);
    return decode_on(stream, vol, P, opts, mode, wg, grid, b);
}

}  // extern "C"
