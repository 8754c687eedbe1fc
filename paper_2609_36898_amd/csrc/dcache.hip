// Device-resident brick cache stages: request, provision and assign run on the
// GPU, so a batch of (brick, LOD) requests turns into decode tasks with no host
// round trip (Methods > GPU rendering pipeline, the request / provision /
// assign stages ahead of decompression; Methods > Memory management, per-LOD
// free stacks and a cache top pointer).
//
// State in device memory (one allocation):
//   slot_of[id * 8 + lod]  element offset of a resident pair, kEmpty, or kPending
//                          while the request kernel that claimed it runs
//   stack[c][k], count[c]  free stacks of released slots per size class
//                          c = log2(side) - lod (a slot holds 8^c elements);
//                          with one brick side this is the paper's per-LOD stack
//   top                    elements handed out at the cache top so far
//
// Request kernel, one thread per request:
//   1. validate the pair against the brick's record header (side exponent);
//   2. claim the pair: CAS kEmpty -> kPending.  The winner provisions a slot:
//      pop its class's free stack, else advance the cache top atomically; when
//      neither has room the claim is undone (pair stays absent, state FULL);
//   3. assign: the winner publishes the slot and becomes a decode task; every
//      other request of the pair is a hit (slot already set) or joins the
//      winner and takes its slot in the resolve kernel that follows.
// Requests that are not decode tasks get brick id 0xFFFFFFFF, which the decoder
// rejects before touching the output, so the decode launch takes the request
// arrays as they are, with the request count the host already knows.
//
// Free-stack pops run only in the request kernel and pushes only in the free
// kernel, so neither kernel sees both.  Both are aggregated per wavefront and
// size class: one atomic per (wavefront, class) instead of one per request.
// A pop of m entries subtracts m from the count and takes the min(m, old)
// entries below the old count; the shortfall is added back.  The first short
// pop happens only once every entry is taken, and since nothing is pushed
// meanwhile no later pop sees a positive count, so the entries taken are
// distinct.  Pushes mirror this against the stack's capacity.  The cache top
// only grows: a wavefront adds the sum of its requests' slot sizes at once and
// keeps the prefix of them that ends within the capacity.  Nothing is given
// back, so ranges never overlap; a wavefront that overflows leaves the top
// past the capacity, and from then on (until a reset) only the free stacks
// provide slots -- the paper resets a cache that has filled up.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "csgv.h"
#include "csgv_format.h"

namespace csgv {
namespace {

constexpr uint64_t kEmpty = ~0ull;
constexpr uint64_t kPending = ~0ull - 1;
constexpr uint32_t kClasses = kMaxLog2b + 1;
constexpr uint32_t kNoTask = 0xFFFFFFFFu;

struct DcState {
    unsigned long long* slot_of;  // n_bricks * 8
    unsigned long long* stack;    // kClasses * stack_cap
    int* count;                   // kClasses
    unsigned long long* top;      // 1
    uint32_t n_bricks;
    uint32_t stack_cap;
    uint64_t cache_elems;
    const uint8_t* vol;
    uint64_t vol_bytes;
    uint64_t off_pos;
};

thread_local std::string g_dc_error;

csgv_status dc_fail(csgv_status s, const std::string& m) {
    g_dc_error = m;
    return s;
}

// side exponent of brick id's record, or 0xFF when the record is unusable
__device__ uint32_t record_log2b(const DcState& S, uint32_t id) {
    const uint64_t* offs = (const uint64_t*)(S.vol + S.off_pos);
    const uint64_t a = offs[id], b = offs[id + 1];
    if (a > b || b > S.vol_bytes || (a & 7) || b - a < 8) return 0xFFu;
    const uint32_t L = S.vol[a + 1];
    return (L >= 1 && L <= kMaxLog2b) ? L : 0xFFu;
}

__global__ void dc_fill_kernel(unsigned long long* p, uint64_t n, unsigned long long v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void dc_zero_counters_kernel(int* count, unsigned long long* top) {
    if (threadIdx.x < kClasses) count[threadIdx.x] = 0;
    if (threadIdx.x == 0) *top = 0;
}

__device__ __forceinline__ uint64_t lanes_below(uint32_t lane) { return lane ? (~0ull >> (64 - lane)) : 0ull; }

__global__ void __launch_bounds__(256) dc_request_kernel(DcState S, const uint32_t* ids, const uint8_t* lods,
                                                         uint32_t n, uint32_t* task_ids, uint64_t* slot,
                                                         uint32_t* state) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x, lane = __lane_id();
    unsigned long long* key = nullptr;
    uint32_t c = 0;
    bool want = false;  // this request claimed an absent pair and provisions it
    if (i < n) {
        const uint32_t id = ids[i], lod = lods[i];
        task_ids[i] = kNoTask;
        slot[i] = kEmpty;
        const uint32_t L = id < S.n_bricks ? record_log2b(S, id) : 0xFFu;
        if (L == 0xFFu || lod > L) {
            state[i] = CSGV_DC_INVALID;
        } else {
            key = S.slot_of + (uint64_t)id * 8 + lod;
            const unsigned long long old = atomicCAS(key, kEmpty, kPending);
            if (old == kPending) {  // another request of this launch provisions the pair
                state[i] = CSGV_DC_JOINED;
            } else if (old != kEmpty) {  // resident
                slot[i] = old;
                state[i] = CSGV_DC_HIT;
            } else {
                want = true;
                c = L - lod;
            }
        }
    }
    // pops, one atomic per (wavefront, class); every lane runs this loop
    unsigned long long off = kEmpty;
    for (uint64_t left = __ballot(want); left;) {
        const uint32_t lead = (uint32_t)__builtin_ctzll(left);
        const uint32_t cc = (uint32_t)__shfl((int)c, (int)lead);
        const bool mine = want && c == cc;
        const uint64_t m = __ballot(mine);
        const int cnt = __popcll(m);
        int k = 0;
        if (lane == lead) k = atomicSub(&S.count[cc], cnt);
        k = __shfl(k, (int)lead);
        const int avail = k > 0 ? min(k, cnt) : 0;
        if (lane == lead && avail < cnt) atomicAdd(&S.count[cc], cnt - avail);
        if (mine) {
            const int rank = __popcll(m & lanes_below(lane));
            if (rank < avail) off = S.stack[(uint64_t)cc * S.stack_cap + (uint32_t)(k - 1 - rank)];
        }
        left &= ~m;
    }
    // the rest from the cache top: the wavefront's inclusive prefix of slot sizes
    const bool need = want && off == kEmpty;
    const unsigned long long units = need ? 1ull << (3 * c) : 0ull;
    unsigned long long pre = units;
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long v = __shfl_up(pre, (unsigned)d);
        if (lane >= (uint32_t)d) pre += v;
    }
    const unsigned long long total = __shfl(pre, 63);
    if (total) {
        unsigned long long t = 0;
        if (lane == 0) t = atomicAdd(S.top, total);
        t = __shfl(t, 0);
        const unsigned long long room = t < S.cache_elems ? S.cache_elems - t : 0ull;
        if (need && pre <= room) off = t + pre - units;
    }
    if (!want) return;
    if (off == kEmpty) {
        atomicExch(key, kEmpty);
        state[i] = CSGV_DC_FULL;
        return;
    }
    atomicExch(key, off);
    task_ids[i] = ids[i];
    slot[i] = off;
    state[i] = CSGV_DC_NEW;
}

// Joined requests take their winner's slot, or FULL when the winner found no
// room.  A FULL request whose pair another request of the launch placed after
// all (a later claim may fit where a wavefront's prefix did not) becomes a hit,
// so after the call a pair is FULL in every request naming it or in none.
__global__ void __launch_bounds__(256) dc_resolve_kernel(DcState S, const uint32_t* ids, const uint8_t* lods,
                                                         uint32_t n, uint64_t* slot, uint32_t* state) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const uint32_t st = state[i];
    if (st != CSGV_DC_JOINED && st != CSGV_DC_FULL) return;
    const unsigned long long v = S.slot_of[(uint64_t)ids[i] * 8 + lods[i]];
    if (v == kEmpty || v == kPending) {
        if (st == CSGV_DC_JOINED) state[i] = CSGV_DC_FULL;
    } else {
        slot[i] = v;
        if (st == CSGV_DC_FULL) state[i] = CSGV_DC_HIT;
    }
}

__global__ void __launch_bounds__(256) dc_free_kernel(DcState S, const uint32_t* ids, const uint8_t* lods,
                                                      uint32_t n) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x, lane = __lane_id();
    unsigned long long old = kEmpty;
    uint32_t c = 0;
    bool have = false;  // this request released a resident pair
    if (i < n) {
        const uint32_t id = ids[i], lod = lods[i];
        if (id < S.n_bricks && lod <= kMaxLog2b) {
            old = atomicExch(S.slot_of + (uint64_t)id * 8 + lod, kEmpty);
            if (old != kEmpty && old != kPending) {
                const uint32_t L = record_log2b(S, id);
                have = L != 0xFFu && lod <= L;  // always so for a pair the request kernel placed
                c = L - lod;
            }
        }
    }
    // pushes, one atomic per (wavefront, class); a full stack drops the slot until a reset
    for (uint64_t left = __ballot(have); left;) {
        const uint32_t lead = (uint32_t)__builtin_ctzll(left);
        const uint32_t cc = (uint32_t)__shfl((int)c, (int)lead);
        const bool mine = have && c == cc;
        const uint64_t m = __ballot(mine);
        const int cnt = __popcll(m);
        int k = 0;
        if (lane == lead) k = atomicAdd(&S.count[cc], cnt);
        k = __shfl(k, (int)lead);
        const int room = k < (int)S.stack_cap ? min((int)S.stack_cap - k, cnt) : 0;
        if (lane == lead && room < cnt) atomicSub(&S.count[cc], cnt - room);
        if (mine) {
            const int rank = __popcll(m & lanes_below(lane));
            if (rank < room) S.stack[(uint64_t)cc * S.stack_cap + (uint32_t)(k + rank)] = old;
        }
        left &= ~m;
    }
}

}  // namespace
}  // namespace csgv

using namespace csgv;

struct csgv_dcache {
    DcState S;
    void* mem = nullptr;
    int device = 0;
};

extern "C" {

const char* csgv_dcache_last_error(void) { return g_dc_error.c_str(); }

csgv_status csgv_dcache_reset(csgv_dcache* c, hipStream_t stream) {
    if (!c) return dc_fail(CSGV_EINVAL, "csgv_dcache_reset: null cache");
    const uint64_t n = (uint64_t)c->S.n_bricks * 8;
    hipLaunchKernelGGL(dc_fill_kernel, dim3((uint32_t)std::min<uint64_t>((n + 255) / 256, 4096)), dim3(256), 0, stream,
                       c->S.slot_of, n, kEmpty);
    hipLaunchKernelGGL(dc_zero_counters_kernel, dim3(1), dim3(64), 0, stream, c->S.count, c->S.top);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return dc_fail(CSGV_EHIP, std::string("csgv_dcache_reset: ") + hipGetErrorString(e));
    return CSGV_OK;
}

csgv_status csgv_dcache_create(const csgv_volume_info* vol, const void* d_container, uint64_t cache_elements,
                               uint32_t stack_cap, hipStream_t stream, csgv_dcache** out) {
    if (!vol || !d_container || !out) return dc_fail(CSGV_EINVAL, "csgv_dcache_create: null argument");
    *out = nullptr;
    if (vol->n_bricks == 0 || cache_elements == 0)
        return dc_fail(CSGV_EINVAL, "csgv_dcache_create: empty volume or cache");
    if (stack_cap == 0) stack_cap = 1u << 20;
    if (stack_cap > (1u << 30)) return dc_fail(CSGV_EINVAL, "csgv_dcache_create: stack_cap above 2^30");
    const uint64_t n_keys = (uint64_t)vol->n_bricks * 8;
    const uint64_t bytes = 8 * n_keys + 8ull * kClasses * stack_cap + 8 + 4 * kClasses + 256;
    csgv_dcache* c = new csgv_dcache();
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipMalloc(&c->mem, bytes);
    if (e != hipSuccess) {
        delete c;
        return dc_fail(e == hipErrorOutOfMemory ? CSGV_ENOMEM : CSGV_EHIP,
                       std::string("csgv_dcache_create: ") + hipGetErrorString(e));
    }
    uint8_t* p = (uint8_t*)c->mem;
    c->S.slot_of = (unsigned long long*)p;
    c->S.stack = (unsigned long long*)(p + 8 * n_keys);
    c->S.top = (unsigned long long*)(p + 8 * n_keys + 8ull * kClasses * stack_cap);
    c->S.count = (int*)(p + 8 * n_keys + 8ull * kClasses * stack_cap + 8);
    c->S.n_bricks = vol->n_bricks;
    c->S.stack_cap = stack_cap;
    c->S.cache_elems = cache_elements;
    c->S.vol = (const uint8_t*)d_container;
    c->S.vol_bytes = vol->total_bytes;
    c->S.off_pos = vol->offsets_pos;
    const csgv_status s = csgv_dcache_reset(c, stream);
    if (s != CSGV_OK) {
        (void)hipFree(c->mem);
        delete c;
        return s;
    }
    *out = c;
    return CSGV_OK;
}

void csgv_dcache_destroy(csgv_dcache* c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    (void)hipFree(c->mem);
    delete c;
}

csgv_status csgv_dcache_request(csgv_dcache* c, hipStream_t stream, const uint32_t* d_ids, const uint8_t* d_lods,
                                uint32_t n, uint32_t* d_task_ids, uint64_t* d_slot, uint32_t* d_state) {
    if (!c) return dc_fail(CSGV_EINVAL, "csgv_dcache_request: null cache");
    if (n == 0) return CSGV_OK;
    if (!d_ids || !d_lods || !d_task_ids || !d_slot || !d_state)
        return dc_fail(CSGV_EINVAL, "csgv_dcache_request: null array");
    const dim3 grid((n + 255) / 256);
    hipLaunchKernelGGL(dc_request_kernel, grid, dim3(256), 0, stream, c->S, d_ids, d_lods, n, d_task_ids, d_slot,
                       d_state);
    hipLaunchKernelGGL(dc_resolve_kernel, grid, dim3(256), 0, stream, c->S, d_ids, d_lods, n, d_slot, d_state);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return dc_fail(CSGV_EHIP, std::string("csgv_dcache_request: ") + hipGetErrorString(e));
    return CSGV_OK;
}

csgv_status csgv_dcache_free(csgv_dcache* c, hipStream_t stream, const uint32_t* d_ids, const uint8_t* d_lods,
                             uint32_t n) {
    if (!c) return dc_fail(CSGV_EINVAL, "csgv_dcache_free: null cache");
    if (n == 0) return CSGV_OK;
    if (!d_ids || !d_lods) return dc_fail(CSGV_EINVAL, "csgv_dcache_free: null array");
    hipLaunchKernelGGL(dc_free_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, c->S, d_ids, d_lods, n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return dc_fail(CSGV_EHIP, std::string("csgv_dcache_free: ") + hipGetErrorString(e));
    return CSGV_OK;
}

csgv_status csgv_dcache_query(csgv_dcache* c, hipStream_t stream, uint64_t* h_top, int32_t* h_counts) {
    if (!c || !h_top || !h_counts) return dc_fail(CSGV_EINVAL, "csgv_dcache_query: null argument");
    hipError_t e = hipMemcpyAsync(h_top, c->S.top, 8, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h_counts, c->S.count, 4 * kClasses, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return dc_fail(CSGV_EHIP, std::string("csgv_dcache_query: ") + hipGetErrorString(e));
    return CSGV_OK;
}

}  // extern "C"
