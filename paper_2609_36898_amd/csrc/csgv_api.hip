// C ABI of the decoder: argument checks, scratch, the plain and persistent
// launch forms, and batched plans (cost-sorted queue, captured HIP graph,
// autotuned launch shape).
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

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
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

Params make_params(const csgv_volume_info* vol, const void* d_container, const uint32_t* ids, const uint8_t* lods,
                   const uint64_t* offs, uint32_t n, void* out, uint64_t cap, uint32_t* status) {
    Params P;
    memset(&P, 0, sizeof(P));
    P.vol = (const uint8_t*)d_container;
    P.vol_bytes = vol->total_bytes;
    P.off_pos = vol->offsets_pos;
    P.n_bricks = vol->n_bricks;
    P.label_bytes = vol->label_bytes;
    uint32_t sum = 0;
    for (int s = 0; s < 16; ++s) sum += vol->rans_freq[s];
    P.freq_ok = sum == kRansM;
    for (int k = 0; k < 8; ++k) P.freq[k] = (uint32_t)vol->rans_freq[2 * k] | ((uint32_t)vol->rans_freq[2 * k + 1] << 16);
    P.ids = ids;
    P.lods = lods;
    P.out_offs = offs;
    P.n_tasks = n;
    P.out = (uint8_t*)out;
    P.out_cap = cap;
    P.status = status;
    P.scratch_stride = kScratchPerWG;
    return P;
}

csgv_status check_task_args(const csgv_volume_info* vol, const void* d_container, const uint32_t* ids,
                            const uint8_t* lods, const uint64_t* offs, uint32_t n, void* out) {
    if (!vol) return fail(CSGV_EINVAL, "volume info is NULL");
    if (vol->label_bytes != 4 && vol->label_bytes != 8) return fail(CSGV_EINVAL, "label_bytes must be 4 or 8");
    if (vol->offsets_pos < kHeaderBytes || vol->offsets_pos + 8ull * ((uint64_t)vol->n_bricks + 1) > vol->total_bytes)
        return fail(CSGV_EINVAL, "offset table outside the container");
    if (n == 0) return CSGV_OK;
    if (!d_container || !ids || !lods || !offs || !out) return fail(CSGV_EINVAL, "NULL device pointer");
    return CSGV_OK;
}

int pick_wg(int requested, int dflt) {
    if (requested == 256 || requested == 512 || requested == 1024) return requested;
    return dflt;
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
    if (v.offsets_pos < kHeaderBytes || v.offsets_pos + 8ull * ((uint64_t)v.n_bricks + 1) > v.total_bytes)
        return fail(CSGV_EINVAL, "offset table outside the container");
    *out = v;
    return CSGV_OK;
}

csgv_status csgv_decode_bricks(hipStream_t stream, const csgv_volume_info* vol, const void* d_container,
                               const uint32_t* d_brick_ids, const uint8_t* d_lods, const uint64_t* d_out_offsets,
                               uint32_t n, void* d_out, uint64_t out_capacity, uint32_t* d_status,
                               const csgv_decode_opts* opts) {
    csgv_status st = check_task_args(vol, d_container, d_brick_ids, d_lods, d_out_offsets, n, d_out);
    if (st != CSGV_OK || n == 0) return st;
    HIP_TRY(ensure_attrs());
    const int mode = opts ? opts->mode : CSGV_MODE_PLAIN;
    if (mode != CSGV_MODE_PLAIN && mode != CSGV_MODE_PERSISTENT) return fail(CSGV_EINVAL, "unknown mode %d", mode);
    Params P = make_params(vol, d_container, d_brick_ids, d_lods, d_out_offsets, n, d_out, out_capacity, d_status);
    if (mode == CSGV_MODE_PLAIN) {
        const int wg = pick_wg(opts ? opts->wg_size : 0, 1024);
        void* scratch = nullptr;
        HIP_TRY(hipMallocAsync(&scratch, kScratchPerWG, stream));
        P.scratch = (uint8_t*)scratch;
        for (uint32_t j = 0; j < n; ++j) {
            P.task0 = j;
            hipError_t e = launch_decode(P, wg, 1, stream);
            if (e != hipSuccess) {
                (void)hipFreeAsync(scratch, stream);
                return fail(CSGV_EHIP, "decode launch: %s", hipGetErrorString(e));
            }
        }
        HIP_TRY(hipFreeAsync(scratch, stream));
        return CSGV_OK;
    }
    // one-shot persistent launch
    const int wg = pick_wg(opts ? opts->wg_size : 0, 512);
    const int per_cu = opts && opts->wgs_per_cu > 0 ? opts->wgs_per_cu : 1;
    uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)device_cus() * per_cu, n);
    const bool sort = opts ? opts->sort_tasks != 0 : true;
    const uint64_t aux = 256 + (sort ? 8ull * n + 4 * 128 : 0);
    void* mem = nullptr;
    HIP_TRY(hipMallocAsync(&mem, kScratchPerWG * grid + aux, stream));
    uint8_t* base = (uint8_t*)mem;
    P.scratch = base;
    uint8_t* a = base + kScratchPerWG * grid;
    P.queue = (uint32_t*)a;
    hipError_t e = launch_reset(P.queue, stream);
    if (e == hipSuccess && sort) {
        uint32_t* hist = (uint32_t*)(a + 256);
        uint32_t* cls = hist + 128;
        uint32_t* order = cls + n;
        e = launch_sort(P, cls, hist, order, stream);
        P.order = order;
    }
    if (e == hipSuccess) e = launch_decode(P, wg, grid, stream);
    hipError_t e2 = hipFreeAsync(mem, stream);
    if (e != hipSuccess) return fail(CSGV_EHIP, "decode launch: %s", hipGetErrorString(e));
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
    uint8_t* mem = nullptr;  // scratch | queue | hist | cls | order
    uint8_t* scratch = nullptr;
    uint32_t* queue = nullptr;
    uint32_t* hist = nullptr;
    uint32_t* cls = nullptr;
    uint32_t* order = nullptr;
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
        int wg, grid, sort;
        bool operator==(const Key& o) const { return memcmp(this, &o, sizeof(Key)) == 0; }
    } key;
    bool have_key = false;
};

namespace {

csgv_status enqueue_plan(csgv_plan* p, hipStream_t s, const Params& P0, bool with_events) {
    Params P = P0;
    P.scratch = p->scratch;
    P.queue = p->queue;
    HIP_TRY(launch_reset(p->queue, s));
    if (p->opts.sort_tasks) {
        HIP_TRY(launch_sort(P, p->cls, p->hist, p->order, s));
        P.order = p->order;
    }
    const uint32_t grid = std::min<uint32_t>(p->grid, std::max<uint32_t>(P.n_tasks, 1));
    if (with_events) HIP_TRY(hipEventRecord(p->ev0, s));
    HIP_TRY(launch_decode(P, p->opts.wg_size, grid, s));
    if (with_events) HIP_TRY(hipEventRecord(p->ev1, s));
    return CSGV_OK;
}

}  // namespace

extern "C" {

csgv_status csgv_plan_create(const csgv_volume_info* vol, uint32_t max_tasks, const csgv_decode_opts* opts,
                             csgv_plan** out) {
    if (!vol || !out) return fail(CSGV_EINVAL, "NULL argument");
    if (max_tasks == 0) return fail(CSGV_EINVAL, "max_tasks must be positive");
    HIP_TRY(ensure_attrs());
    csgv_plan* p = new csgv_plan();
    p->vol = *vol;
    p->max_tasks = max_tasks;
    p->opts.mode = CSGV_MODE_PERSISTENT;
    p->opts.wg_size = pick_wg(opts ? opts->wg_size : 0, 512);
    p->opts.wgs_per_cu = opts && opts->wgs_per_cu > 0 ? opts->wgs_per_cu : 1;
    p->opts.sort_tasks = opts && opts->sort_tasks >= 0 ? opts->sort_tasks : 1;
    p->grid = (uint32_t)std::min<uint64_t>((uint64_t)device_cus() * p->opts.wgs_per_cu, max_tasks);
    const uint64_t aux = 256 + 4 * 128 + 8ull * max_tasks;
    hipError_t e = hipMalloc(&p->mem, kScratchPerWG * p->grid + aux);
    if (e != hipSuccess) {
        delete p;
        return fail(CSGV_ENOMEM, "plan scratch: %s", hipGetErrorString(e));
    }
    p->scratch = p->mem;
    uint8_t* a = p->mem + kScratchPerWG * p->grid;
    p->queue = (uint32_t*)a;
    p->hist = (uint32_t*)(a + 256);
    p->cls = p->hist + 128;
    p->order = p->cls + max_tasks;
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

csgv_status csgv_plan_set_shape(csgv_plan* p, int wg_size, int sort_tasks) {
    if (!p) return fail(CSGV_EINVAL, "NULL plan");
    if (wg_size != 256 && wg_size != 512 && wg_size != 1024) return fail(CSGV_EINVAL, "wg_size %d", wg_size);
    p->opts.wg_size = wg_size;
    p->opts.sort_tasks = sort_tasks ? 1 : 0;
    return CSGV_OK;
}

csgv_status csgv_plan_launch(csgv_plan* p, hipStream_t stream, const void* d_container, const uint32_t* d_brick_ids,
                             const uint8_t* d_lods, const uint64_t* d_out_offsets, uint32_t n, void* d_out,
                             uint64_t out_capacity, uint32_t* d_status) {
    if (!p) return fail(CSGV_EINVAL, "NULL plan");
    csgv_status st = check_task_args(&p->vol, d_container, d_brick_ids, d_lods, d_out_offsets, n, d_out);
    if (st != CSGV_OK) return st;
    if (n == 0) return CSGV_OK;
    if (n > p->max_tasks) return fail(CSGV_EINVAL, "n = %u exceeds the plan's max_tasks = %u", n, p->max_tasks);
    Params P = make_params(&p->vol, d_container, d_brick_ids, d_lods, d_out_offsets, n, d_out, out_capacity, d_status);
    if (p->timing || !p->use_graph) {
        st = enqueue_plan(p, stream, P, p->timing);
        p->ev_valid = st == CSGV_OK && p->timing;
        return st;
    }
    csgv_plan::Key k;
    memset(&k, 0, sizeof(k));
    k.c = d_container; k.ids = d_brick_ids; k.lods = d_lods; k.offs = d_out_offsets; k.n = n; k.out = d_out;
    k.cap = out_capacity; k.status = d_status; k.wg = p->opts.wg_size; k.grid = (int)p->grid; k.sort = p->opts.sort_tasks;
    if (!p->have_key || !(k == p->key) || !p->exec) {
        if (p->exec) {
            (void)hipGraphExecDestroy(p->exec);
            p->exec = nullptr;
        }
        HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
        st = enqueue_plan(p, p->cap_stream, P, false);
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
