// Served decode: the host scheduler of serve_core.h driving batched decode
// plans on several HIP streams, and its C ABI.  The cache may be split into
// brick shards (ShardSet), each with its own streams and plans, served by one
// host thread each in csgv_server_run.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <deque>
#include <memory>
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
    std::string plan_msg;  // the plan's error message (read on the thread that launched)
    uint64_t failed_tasks = 0;
    const uint64_t* rec_off = nullptr;  // host copy of the container's record offsets
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
            if (st != CSGV_OK && plan_err == CSGV_OK) {
                plan_err = st;
                plan_msg = csgv_last_error();
            }
        }
        if (e == hipSuccess) e = hipMemcpyAsync(l.h_status, l.d_status, 4ull * n, hipMemcpyDeviceToHost, l.stream);
        if (e == hipSuccess) e = hipEventRecord(l.done, l.stream);
        if (e != hipSuccess && err == hipSuccess) err = e;
    }
};

thread_local std::string g_serve_error;

}  // namespace

struct csgv_server {
    std::vector<std::unique_ptr<GpuBackend>> be;  // one per shard
    std::vector<uint64_t> rec_off;                 // the container's record offsets (host copy)
    csgv::ShardSet<GpuBackend>* sched = nullptr;
    std::chrono::steady_clock::time_point t0;
    std::deque<csgv::ServeDone> done;  // completions not yet drained
};

namespace {

csgv_status serve_fail(csgv_status s, const char* msg) {
    g_serve_error = msg;
    return s;
}

bool backend_ok(const GpuBackend& b) { return b.err == hipSuccess && b.plan_err == CSGV_OK; }

csgv_status backend_status(csgv_server* s) {
    for (auto& b : s->be) {
        if (b->err != hipSuccess) return serve_fail(CSGV_EHIP, hipGetErrorString(b->err));
        if (b->plan_err != CSGV_OK) return serve_fail(b->plan_err, b->plan_msg.c_str());
    }
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

void destroy_server(csgv_server* s) {
    for (auto& b : s->be) destroy_lanes(*b);
    delete s->sched;
    delete s;
}

}  // namespace

extern "C" {

csgv_status csgv_server_create(const csgv_volume_info* vol, const void* d_container, const uint8_t* h_brick_log2b,
                               void* d_cache, uint64_t cache_elements, const csgv_server_config* cfg,
                               csgv_server** out) {
    if (!vol || !d_container || !d_cache || !out || cache_elements == 0) return serve_fail(CSGV_EINVAL, "NULL argument");
    const int n_streams = cfg && cfg->n_streams > 0 ? cfg->n_streams : 2;
    const uint32_t max_batch = cfg && cfg->max_batch > 0 ? cfg->max_batch : 4096;
    const uint32_t n_shards = cfg && cfg->n_shards > 0 ? (uint32_t)cfg->n_shards : 1u;
    if (n_streams > 16) return serve_fail(CSGV_EINVAL, "at most 16 streams");
    if (n_shards > 16) return serve_fail(CSGV_EINVAL, "at most 16 shards");
    // equal shard ranges, 64-element aligned
    const uint64_t share = n_shards == 1 ? cache_elements : (cache_elements / n_shards) & ~uint64_t(63);
    if (share == 0) return serve_fail(CSGV_EINVAL, "cache too small for the shard count");
    std::vector<uint8_t> l2(vol->n_bricks, (uint8_t)vol->log2b);
    if (h_brick_log2b) memcpy(l2.data(), h_brick_log2b, vol->n_bricks);
    for (uint8_t v : l2)
        if (v < 1 || v > 6) return serve_fail(CSGV_EINVAL, "brick side exponent outside 1..6");
    if (cfg && cfg->shape.palette_bits > 0)
        return serve_fail(CSGV_EINVAL, "the brick cache holds labels (palette_bits must be 0)");
    csgv_server* s = new csgv_server();
    // record offsets (the parsed volume guarantees they lie inside the container)
    s->rec_off.resize((size_t)vol->n_bricks + 1);
    if (hipMemcpy(s->rec_off.data(), (const uint8_t*)d_container + vol->offsets_pos, 8ull * (vol->n_bricks + 1),
                  hipMemcpyDeviceToHost) != hipSuccess) {
        destroy_server(s);
        return serve_fail(CSGV_EHIP, "reading the record offsets");
    }
    csgv_decode_opts o;
    memset(&o, 0, sizeof(o));
    if (cfg) o = cfg->shape;
    else o.sort_tasks = -1;
    o.mode = CSGV_MODE_PERSISTENT;
    std::vector<GpuBackend*> bes;
    std::vector<uint64_t> base, cap;
    for (uint32_t w = 0; w < n_shards; ++w) {
        s->be.emplace_back(new GpuBackend());
        GpuBackend& be = *s->be.back();
        be.container = d_container;
        be.cache = (uint8_t*)d_cache + (uint64_t)w * share * vol->label_bytes;
        be.cache_elems = share;
        be.rec_off = s->rec_off.data();
        be.lanes.resize(n_streams);
        for (auto& l : be.lanes) {
            if (hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&l.done, hipEventDisableTiming) != hipSuccess ||
                hipHostMalloc((void**)&l.h_tasks, 13ull * max_batch, hipHostMallocDefault) != hipSuccess ||
                hipHostMalloc((void**)&l.h_status, 4ull * max_batch, hipHostMallocDefault) != hipSuccess ||
                hipMalloc((void**)&l.d_tasks, 13ull * max_batch) != hipSuccess ||
                hipMalloc((void**)&l.d_status, 4ull * max_batch) != hipSuccess) {
                destroy_server(s);
                return serve_fail(CSGV_ENOMEM, "server stream resources");
            }
            const csgv_status st = csgv_plan_create(vol, max_batch, &o, &l.plan);
            if (st != CSGV_OK) {
                const std::string msg = csgv_last_error();
                destroy_server(s);
                return serve_fail(st, msg.c_str());
            }
            (void)csgv_plan_set_graph(l.plan, 0);  // batches differ in size: direct launches
            (void)csgv_plan_set_timing(l.plan, 1);
        }
        bes.push_back(&be);
        base.push_back((uint64_t)w * share);
        cap.push_back(share);
    }
    s->sched = new csgv::ShardSet<GpuBackend>(bes, base, cap, l2.data(), vol->n_bricks, max_batch,
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
    if (n_req && (!h_ids || !h_lods) && h_req_start[n_req] > h_req_start[0]) return serve_fail(CSGV_EINVAL, "NULL pairs");
    if (n_req && !s->sched->valid(h_ids + h_req_start[0], h_lods + h_req_start[0], h_req_start[n_req] - h_req_start[0]))
        return serve_fail(CSGV_EINVAL, "a pair names no brick, or a LOD beyond the brick side");
    static_assert(sizeof(csgv_request_done) == sizeof(csgv::ServeDone), "layouts agree");
    const bool ok = s->sched->run(
        h_ids, h_lods, h_req_start, n_req, h_arrival, csgv_server_clock(s), [s] { return csgv_server_clock(s); },
        [s](uint32_t w) { return backend_ok(*s->be[w]); }, reinterpret_cast<csgv::ServeDone*>(out));
    for (const csgv::ServeDone& d : s->sched->take_early()) s->done.push_back(d);
    if (!ok) {
        const csgv_status st = backend_status(s);
        return st != CSGV_OK ? st : serve_fail(CSGV_EHIP, "served run stopped");
    }
    return CSGV_OK;
}

csgv_status csgv_server_get_stats(csgv_server* s, csgv_server_stats* out) {
    if (!s || !out) return serve_fail(CSGV_EINVAL, "NULL argument");
    const csgv::ServeStats t = s->sched->stats();
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
    out->failed_tasks = 0;
    out->record_bytes = 0;
    out->kernel_ms = 0;
    for (auto& b : s->be) {
        out->failed_tasks += b->failed_tasks;
        out->record_bytes += b->record_bytes;
        out->kernel_ms += b->kernel_ms;
    }
    out->splits = t.splits;
    out->max_batch_seen = t.max_batch_seen;
    return CSGV_OK;
}

const char* csgv_server_last_error(void) { return g_serve_error.c_str(); }

void csgv_server_destroy(csgv_server* s) {
    if (s) destroy_server(s);
}

}  // extern "C"
