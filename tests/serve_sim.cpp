// Host-only harness for the serving scheduler (paper_2609_36898_amd/csrc/serve_core.h):
// a simulated backend whose batches finish after a fixed number of polls, and
// which records, per cache element range, which (id, LOD) pair was decoded
// there.  It checks that decoded slots never overlap another live slot, that
// every completed request still finds each of its pairs in the slot it was
// decoded into, and that requests are admitted in arrival order.  The cache
// may be split into brick shards (ShardSet), one simulated backend each,
// stepped in turn on a simulated clock or served by one thread per shard on
// the real clock (ShardSet::run).
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../paper_2609_36898_amd/csrc/serve_core.h"

namespace {

struct SimBackend {
    int n = 2, delay = 3;
    std::vector<int> left;
    std::vector<std::vector<uint64_t>> keys;     // pairs of the batch in flight per stream
    std::vector<std::vector<uint64_t>> offs;
    std::map<uint64_t, std::pair<uint64_t, uint64_t>> live;  // slot start -> (end, key)
    std::map<uint64_t, uint64_t> owner;          // key -> slot start (last decode)
    const std::vector<uint8_t>* l2 = nullptr;  // side exponents of the whole volume's bricks
    uint64_t base = 0, cap = 0;                // this backend's cache range
    std::string err;

    int streams() const { return n; }
    bool busy(int s) { return left[s] > 0; }
    bool poll(int s) {
        if (left[s] <= 0) return false;
        return --left[s] == 0;
    }
    void launch(int s, const uint32_t* ids, const uint8_t* lods, const uint64_t* o, uint32_t m) {
        if (left[s] > 0 && err.empty()) err = "launch on a busy stream";
        left[s] = delay;
        for (uint32_t j = 0; j < m; ++j) {
            const uint64_t key = ((uint64_t)ids[j] << 8) | lods[j];
            const uint32_t cls = (*l2)[ids[j]] - lods[j];
            const uint64_t size = uint64_t(1) << (3 * cls), a = base + o[j], b = a + size;
            if (b > base + cap && err.empty()) err = "slot beyond the cache range";
            // drop whatever older slot this range replaces, then check overlap with the rest
            auto it = live.lower_bound(a);
            if (it != live.begin()) --it;
            while (it != live.end() && it->first < b) {
                if (it->second.first > a) {
                    const uint64_t k2 = it->second.second;
                    if (owner.count(k2) && owner[k2] == it->first) owner.erase(k2);
                    it = live.erase(it);
                } else {
                    ++it;
                }
            }
            live[a] = {b, key};
            owner[key] = a;
        }
    }
};

}  // namespace

extern "C" int sim_run(const uint8_t* l2p, uint32_t n_bricks, uint64_t cache_elems, int streams, uint32_t max_batch,
                       int keep_pinned, int delay, int shards, int threaded, const uint32_t* ids, const uint8_t* lods,
                       const uint64_t* starts, uint32_t n_req, const double* arrival, double dt, double* t_admit,
                       double* t_done, int32_t* status, uint32_t* n_decoded, uint32_t* n_pairs, uint64_t* stats,
                       char* errbuf, int errcap) {
    std::vector<uint8_t> l2(l2p, l2p + n_bricks);
    const uint32_t T = shards > 0 ? (uint32_t)shards : 1u;
    const uint64_t share = T == 1 ? cache_elems : (cache_elems / T) & ~uint64_t(63);
    std::vector<std::unique_ptr<SimBackend>> bes;
    std::vector<SimBackend*> bp;
    std::vector<uint64_t> base, cap;
    for (uint32_t w = 0; w < T; ++w) {
        bes.emplace_back(new SimBackend());
        SimBackend& be = *bes.back();
        be.n = streams;
        be.delay = delay;
        be.left.assign(streams, 0);
        be.l2 = &l2;
        be.base = w * share;
        be.cap = share;
        bp.push_back(&be);
        base.push_back(w * share);
        cap.push_back(share);
    }
    csgv::ShardSet<SimBackend> sch(bp, base, cap, l2.data(), n_bricks, max_batch, keep_pinned != 0);
    std::string err;
    auto backend_err = [&]() -> std::string {
        for (auto& b : bes)
            if (!b->err.empty()) return b->err;
        return std::string();
    };
    auto record = [&](const csgv::ServeDone& d, uint32_t r) {
        t_admit[r] = d.t_admit;
        t_done[r] = d.t_done;
        status[r] = d.status;
        n_decoded[r] = d.n_decoded;
        n_pairs[r] = d.n_pairs;
    };
    if (threaded) {
        // one thread per shard on the real clock; slots and statuses are checked afterwards
        std::vector<csgv::ServeDone> out(n_req);
        const auto c0 = std::chrono::steady_clock::now();
        auto clock = [c0] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - c0).count(); };
        if (!sch.valid(ids, lods, starts[n_req])) err = "invalid pair in the trace";
        else if (!sch.run(ids, lods, starts, n_req, arrival, clock(), clock, [](uint32_t) { return true; }, out.data()))
            err = "run stopped";
        for (uint32_t r = 0; r < n_req && err.empty(); ++r) {
            if (out[r].req != out[0].req + r) err = "record " + std::to_string(r) + " names another request";
            record(out[r], r);
        }
        if (err.empty()) err = backend_err();
        if (err.empty() && keep_pinned)
            for (uint32_t r = 0; r < n_req; ++r)
                if (status[r] == 0) sch.release(out[r].req);
        sch.step(clock());
    } else {
        std::vector<uint64_t> rid(n_req);
        for (uint32_t r = 0; r < n_req; ++r)
            if (!sch.submit(ids + starts[r], lods + starts[r], (uint32_t)(starts[r + 1] - starts[r]), arrival[r], &rid[r]))
                err = "submit refused request " + std::to_string(r);
        double now = 0;
        uint32_t done = 0;
        uint64_t steps = 0;
        while (err.empty() && done < n_req) {
            sch.step(now);
            err = backend_err();
            for (const csgv::ServeDone& d : sch.drain()) {
                const uint32_t r = (uint32_t)(d.req - rid[0]);
                record(d, r);
                ++done;
                if (d.status == 0) {
                    // every pair of the request sits where it was decoded
                    for (uint64_t j = starts[r]; j < starts[r + 1]; ++j) {
                        uint64_t off;
                        const uint64_t key = ((uint64_t)ids[j] << 8) | lods[j];
                        SimBackend& be = *bes[ids[j] % T];
                        if (!sch.where(ids[j], lods[j], &off)) {
                            err = "completed request " + std::to_string(r) + " has a pair that is not resident";
                            break;
                        }
                        if (!be.owner.count(key) || be.owner[key] != off) {
                            err = "completed request " + std::to_string(r) + " has a pair whose slot was reused";
                            break;
                        }
                    }
                    if (keep_pinned) sch.release(d.req);
                }
            }
            now += dt;
            if (++steps > 50000000ull) err = "no progress";
        }
        sch.step(now);  // releases the pairs of the last completions
    }
    // requests were submitted in arrival order: admission times must not decrease
    for (uint32_t r = 1; r < n_req && err.empty(); ++r)
        if (t_admit[r] < t_admit[r - 1]) err = "admission out of arrival order at request " + std::to_string(r);
    const csgv::ServeStats s = sch.stats();
    const uint64_t v[14] = {s.requests_done, s.pairs_requested, s.hits, s.decoded, s.evictions, s.resets,
                            s.batches, s.decoded_elements, s.requested_elements, s.top, s.pinned, s.max_batch_seen,
                            s.joined, s.splits};
    memcpy(stats, v, sizeof(v));
    if (!err.empty()) {
        snprintf(errbuf, errcap, "%s", err.c_str());
        return 1;
    }
    return 0;
}
