// Served decode: the host scheduler of serve_core.h driving batched decode
// plans on several HIP streams, and its C ABI.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <deque>
#include <string>
#include <thread>
#include <vector>

#include "../../include/csgv.h"
#include "serve_core.h"

namespace {

// One decode plan per stream; a batch's task arrays travel through pinned
// staging buffers (stream-ordered copies), and an event marks its end.
struct GpuBackend {
    struct Lane {
        hipStream_t stream = nullptr;
        csgv_plan* plan = nullptr;
        hipEvent_t done = nullptr;
        // one pinned staging block per batch: offsets | ids | LODs (one copy to the device)
        uint8_t* h_tasks = nullptr;
        uint8_t* d_tasks = nullptr;
        uint32_t* h_status = nullptr;
        uint32_t* d_status = nullptr;
        uint32_t n = 0;
        bool busy = false;
    };
    std::vector<Lane> lanes;
    const void* container = nullptr;
    void* cache = nullptr;
    uint64_t cache_elems = 0;
    hipError_t err = hipSuccess;
    csgv_status plan_err = CSGV_OK;
    uint64_t failed_tasks = 0;
    std::vector<uint64_t> rec_off;  // host copy of the container's record offsets
    uint64_t record_bytes = 0;
    double kernel_ms = 0;

    int streams() const { return (int)lanes.size(); }
    bool busy(int s) { return lanes[s].busy; }
    bool poll(int s) {
        Lane& l = lanes[s];
        if (!l.busy) return false;
        const hipError_t e = hipEventQuery(l.done);
        if (e == hipErrorNotReady) return false;
        if (e != hipSuccess && err == hipSuccess) err = e;
        for (uint32_t j = 0; j < l.n; ++j) failed_tasks += l.h_status[j] != 0;
        float ms = 0;
        if (csgv_plan_last_kernel_ms(l.plan, &ms) == CSGV_OK) kernel_ms += ms;
        l.busy = false;
        return true;
    }
    void launch(int s, const uint32_t* ids, const uint8_t* lods, const uint64_t* offs, uint32_t n) {
        Lane& l = lanes[s];
        memcpy(l.h_tasks, offs, 8ull * n);
        memcpy(l.h_tasks + 8ull * n, ids, 4ull * n);
        memcpy(l.h_tasks + 12ull * n, lods, n);
        for (uint32_t j = 0; j < n; ++j) record_bytes += rec_off[ids[j] + 1] - rec_off[ids[j]];
        l.n = n;
        l.busy = true;
        hipError_t e = hipMemcpyAsync(l.d_tasks, l.h_tasks, 13ull * n, hipMemcpyHostToDevice, l.stream);
        if (e == hipSuccess) {
            const csgv_status st = csgv_plan_launch(l.plan, l.stream, container, (const uint32_t*)(l.d_tasks + 8ull * n),
                                                    l.d_tasks + 12ull * n, (const uint64_t*)l.d_tasks, n, cache,
                                                    cache_elems, l.d_status);
            if (st != CSGV_OK && plan_err == CSGV_OK) plan_err = st;
        }
        if (e == hipSuccess) e = hipMemcpyAsync(l.h_status, l.d_status, 4ull * n, hipMemcpyDeviceToHost, l.stream);
        if (e == hipSuccess) e = hipEventRecord(l.done, l.stream);
        if (e != hipSuccess && err == hipSuccess) err = e;
    }
};

thread_local std::string g_serve_error;

}  // namespace

struct csgv_server {
    GpuBackend be;
    csgv::Scheduler<GpuBackend>* sched = nullptr;
    std::chrono::steady_clock::time_point t0;
    std::deque<csgv::ServeDone> done;  // completions not yet drained
};

namespace {

csgv_status serve_fail(csgv_status s, const char* msg) {
    g_serve_error = msg;
    return s;
}

csgv_status backend_status(csgv_server* s) {
    if (s->be.err != hipSuccess) return serve_fail(CSGV_EHIP, hipGetErrorString(s->be.err));
    if (s->be.plan_err != CSGV_OK) return serve_fail(s->be.plan_err, csgv_last_error());
    return CSGV_OK;
}

void destroy_lanes(GpuBackend& be) {
    for (auto& l : be.lanes) {
        if (l.stream) (void)hipStreamSynchronize(l.stream);
        if (l.plan) csgv_plan_destroy(l.plan);
        if (l.done) (void)hipEventDestroy(l.done);
        if (l.stream) (void)hipStreamDestroy(l.stream);
        if (l.h_tasks) (void)hipHostFree(l.h_tasks);
        if (l.h_status) (void)hipHostFree(l.h_status);
        if (l.d_tasks) (void)hipFree(l.d_tasks);
        if (l.d_status) (void)hipFree(l.d_status);
    }
    be.lanes.clear();
}

}  // namespace

extern "C" {

csgv_status csgv_server_create(const csgv_volume_info* vol, const void* d_container, const uint8_t* h_brick_log2b,
                               void* d_cache, uint64_t cache_elements, const csgv_server_config* cfg,
                               csgv_server** out) {
    if (!vol || !d_container || !d_cache || !out || cache_elements == 0) return serve_fail(CSGV_EINVAL, "NULL argument");
    const int n_streams = cfg && cfg->n_streams > 0 ? cfg->n_streams : 2;
    const uint32_t max_batch = cfg && cfg->max_batch > 0 ? cfg->max_batch : 4096;
    if (n_streams > 16) return serve_fail(CSGV_EINVAL, "at most 16 streams");
    std::vector<uint8_t> l2(vol->n_bricks, (uint8_t)vol->log2b);
    if (h_brick_log2b) memcpy(l2.data(), h_brick_log2b, vol->n_bricks);
    for (uint8_t v : l2)
        if (v < 1 || v > 6) return serve_fail(CSGV_EINVAL, "brick side exponent outside 1..6");
    if (cfg && cfg->shape.palette_bits > 0)
        return serve_fail(CSGV_EINVAL, "the brick cache holds labels (palette_bits must be 0)");
    csgv_server* s = new csgv_server();
    s->be.container = d_container;
    s->be.cache = d_cache;
    s->be.cache_elems = cache_elements;
    csgv_decode_opts o;
    memset(&o, 0, sizeof(o));
    if (cfg) o = cfg->shape;
    else o.sort_tasks = -1;
    o.mode = CSGV_MODE_PERSISTENT;
    s->be.lanes.resize(n_streams);
    for (auto& l : s->be.lanes) {
        if (hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&l.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void**)&l.h_tasks, 13ull * max_batch, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&l.h_status, 4ull * max_batch, hipHostMallocDefault) != hipSuccess ||
            hipMalloc((void**)&l.d_tasks, 13ull * max_batch) != hipSuccess ||
            hipMalloc((void**)&l.d_status, 4ull * max_batch) != hipSuccess) {
            destroy_lanes(s->be);
            delete s;
            return serve_fail(CSGV_ENOMEM, "server stream resources");
        }
        const csgv_status st = csgv_plan_create(vol, max_batch, &o, &l.plan);
        if (st != CSGV_OK) {
            destroy_lanes(s->be);
            delete s;
            return serve_fail(st, csgv_last_error());
        }
        (void)csgv_plan_set_graph(l.plan, 0);  // batches differ in size: direct launches
        (void)csgv_plan_set_timing(l.plan, 1);
    }
    // record offsets (the parsed volume guarantees they lie inside the container)
    s->be.rec_off.resize((size_t)vol->n_bricks + 1);
    if (hipMemcpy(s->be.rec_off.data(), (const uint8_t*)d_container + vol->offsets_pos, 8ull * (vol->n_bricks + 1),
                  hipMemcpyDeviceToHost) != hipSuccess) {
        destroy_lanes(s->be);
        delete s;
        return serve_fail(CSGV_EHIP, "reading the record offsets");
    }
    s->sched = new csgv::Scheduler<GpuBackend>(s->be, cache_elements, l2.data(), vol->n_bricks, max_batch,
                                               cfg && cfg->keep_pinned);
    s->t0 = std::chrono::steady_clock::now();
    *out = s;
    return CSGV_OK;
}

double csgv_server_clock(const csgv_server* s) {
    return s ? std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count() : 0.0;
}

csgv_status csgv_server_submit(csgv_server* s, const uint32_t* h_ids, const uint8_t* h_lods, uint32_t n,
                               double t_arrival, uint64_t* req) {
    if (!s || (n && (!h_ids || !h_lods)) || !req) return serve_fail(CSGV_EINVAL, "NULL argument");
    if (!s->sched->submit(h_ids, h_lods, n, t_arrival, req))
        return serve_fail(CSGV_EINVAL, "a pair names no brick, or a LOD beyond the brick side");
    return CSGV_OK;
}

csgv_status csgv_server_step(csgv_server* s, int* busy) {
    if (!s) return serve_fail(CSGV_EINVAL, "NULL server");
    const bool b = s->sched->step(csgv_server_clock(s));
    if (busy) *busy = b ? 1 : 0;
    return backend_status(s);
}

csgv_status csgv_server_drain(csgv_server* s, csgv_request_done* out, uint32_t cap, uint32_t* n_out) {
    if (!s || !n_out || (cap && !out)) return serve_fail(CSGV_EINVAL, "NULL argument");
    static_assert(sizeof(csgv_request_done) == sizeof(csgv::ServeDone), "layouts agree");
    for (const csgv::ServeDone& d : s->sched->drain()) s->done.push_back(d);
    uint32_t n = 0;
    while (n < cap && !s->done.empty()) {
        memcpy(&out[n++], &s->done.front(), sizeof(csgv::ServeDone));
        s->done.pop_front();
    }
    *n_out = n;
    return CSGV_OK;
}

csgv_status csgv_server_release(csgv_server* s, uint64_t req) {
    if (!s) return serve_fail(CSGV_EINVAL, "NULL server");
    if (!s->sched->release(req)) return serve_fail(CSGV_EINVAL, "request not held");
    return CSGV_OK;
}

csgv_status csgv_server_where(csgv_server* s, uint32_t id, uint8_t lod, uint64_t* elem_offset) {
    if (!s || !elem_offset) return serve_fail(CSGV_EINVAL, "NULL argument");
    if (!s->sched->where(id, lod, elem_offset)) return serve_fail(CSGV_EINVAL, "pair not resident");
    return CSGV_OK;
}

csgv_status csgv_server_run(csgv_server* s, const uint32_t* h_ids, const uint8_t* h_lods, const uint64_t* h_req_start,
                            uint32_t n_req, const double* h_arrival, csgv_request_done* out) {
    if (!s || !h_req_start || (n_req && (!h_arrival || !out))) return serve_fail(CSGV_EINVAL, "NULL argument");
    for (uint32_t r = 0; r < n_req; ++r) {
        if (h_req_start[r + 1] < h_req_start[r]) return serve_fail(CSGV_EINVAL, "request starts not ordered");
        if (r && h_arrival[r] < h_arrival[r - 1]) return serve_fail(CSGV_EINVAL, "arrivals not ordered");
    }
    const double base = csgv_server_clock(s);
    std::vector<uint64_t> ids(n_req);
    uint32_t next = 0, done = 0;
    uint64_t first = 0;
    while (done < n_req) {
        // requests are handed to the scheduler as they arrive
        const double now = csgv_server_clock(s);
        for (; next < n_req && base + h_arrival[next] <= now; ++next) {
            const uint64_t a = h_req_start[next], b = h_req_start[next + 1];
            if (!s->sched->submit(h_ids + a, h_lods + a, (uint32_t)(b - a), base + h_arrival[next], &ids[next]))
                return serve_fail(CSGV_EINVAL, "a pair names no brick, or a LOD beyond the brick side");
            if (next == 0) first = ids[0];
        }
        s->sched->step(csgv_server_clock(s));
        const csgv_status st = backend_status(s);
        if (st != CSGV_OK) return st;
        for (const csgv::ServeDone& d : s->sched->drain()) {
            const uint64_t r = d.req - first;
            if (next > 0 && d.req >= first && r < n_req) {
                memcpy(&out[r], &d, sizeof(d));
                out[r].t_arrival -= base;
                out[r].t_admit -= base;
                out[r].t_done -= base;
                ++done;
            } else {
                s->done.push_back(d);  // a request submitted outside this run
            }
        }
        // idle until the next arrival when nothing is waiting, queued or in flight
        if (s->sched->in_flight() == 0 && next < n_req && s->sched->next_arrival() < 0) {
            const double na = base + h_arrival[next], t = csgv_server_clock(s);
            if (na > t + 2e-4) std::this_thread::sleep_for(std::chrono::duration<double>(na - t - 1e-4));
        }
    }
    return CSGV_OK;
}

csgv_status csgv_server_get_stats(csgv_server* s, csgv_server_stats* out) {
    if (!s || !out) return serve_fail(CSGV_EINVAL, "NULL argument");
    const csgv::ServeStats& t = s->sched->stats();
    out->requests_done = t.requests_done;
    out->pairs_requested = t.pairs_requested;
    out->hits = t.hits;
    out->joined = t.joined;
    out->decoded = t.decoded;
    out->evictions = t.evictions;
    out->resets = t.resets;
    out->batches = t.batches;
    out->decoded_elements = t.decoded_elements;
    out->requested_elements = t.requested_elements;
    out->cache_top = t.top;
    out->resident = t.resident;
    out->pinned = t.pinned;
    out->failed_tasks = s->be.failed_tasks;
    out->splits = t.splits;
    out->record_bytes = s->be.record_bytes;
    out->kernel_ms = s->be.kernel_ms;
    out->max_batch_seen = t.max_batch_seen;
    return CSGV_OK;
}

const char* csgv_server_last_error(void) { return g_serve_error.c_str(); }

void csgv_server_destroy(csgv_server* s) {
    if (!s) return;
    destroy_lanes(s->be);
    delete s->sched;
    delete s;
}

}  // extern "C"
