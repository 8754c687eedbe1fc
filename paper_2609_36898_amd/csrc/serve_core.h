// Serving core: the request / provision / assign stages in front of the
// decode stage (Methods > "GPU rendering pipeline"; Methods > "Memory
// management" for per-LOD cache regions and the reset-on-full
// defragmentation), on the host, independent of how a batch is decoded.
//
// A request is a set of (brick id, LOD) pairs that must all be resident in
// the brick cache.  The cache is one element range split into slots whose
// size is the pair's cube, side = brick side >> LOD (a brick shrinks 8x per
// LOD); a slot, once carved from the top of the cache, keeps its size class
// (class c holds 8^c elements).  Residency is keyed by
// (id, LOD); entries are pinned while a request that needs them is pending,
// and unpinned resident entries form a per-class LRU list that provisioning
// evicts from.  Requests are admitted strictly in arrival order when every
// pair is resident, in flight, or can be given a slot (free list of its
// class, cache top, or the least recently used unpinned entry of its class);
// a request that cannot be admitted waits, and a full cache with nothing
// pinned is reset.  Admitted misses queue as decode tasks; whenever a
// backend stream is free, up to max_batch queued tasks are launched on it
// (continuous batching: requests admitted while earlier batches run get
// their own batches on the other streams).  A request completes when the
// last of its pairs becomes resident; its pairs stay pinned until the next
// step (or, with keep_pinned, until released), so the caller can read them.
//
// Backend interface (used as a template parameter):
//   int  streams() const;                       number of streams
//   bool busy(int s);                           a batch is in flight on s
//   bool poll(int s);                           true once s's batch has finished
//   void launch(int s, const uint32_t* ids, const uint8_t* lods, const uint64_t* offs, uint32_t n);
#pragma once
#include <stdint.h>

#include <algorithm>
#include <deque>
#include <list>
#include <unordered_map>
#include <vector>

namespace csgv {

struct ServeDone {
    uint64_t req;
    double t_arrival, t_admit, t_done;
    uint32_t n_pairs, n_decoded;  // distinct pairs; pairs this request had decoded
    int32_t status;               // 0 ok; -1 rejected (larger than the cache)
};

struct ServeStats {
    // pairs_requested = hits (resident) + joined (queued or in flight for another request) + decoded
    uint64_t requests_done = 0, pairs_requested = 0, hits = 0, joined = 0, decoded = 0, evictions = 0, resets = 0,
             batches = 0;
    uint64_t decoded_elements = 0, requested_elements = 0, top = 0, resident = 0, pinned = 0;
    uint32_t max_batch_seen = 0;
};

template <class Backend>
class Scheduler {
public:
    static constexpr uint32_t kClasses = 7;  // cube sides 1 .. 64

    // brick_log2b: side exponent of every brick (1..6)
    Scheduler(Backend& be, uint64_t cache_elems, const uint8_t* brick_log2b, uint32_t n_bricks, uint32_t max_batch,
              bool keep_pinned)
        : be_(be), cap_(cache_elems), max_batch_(max_batch ? max_batch : 1), keep_pinned_(keep_pinned) {
        l2_.assign(brick_log2b, brick_log2b + n_bricks);
        for (uint32_t c = 0; c < kClasses; ++c) cls_elems_.push_back(uint64_t(1) << (3 * c));
        free_.resize(kClasses);
        lru_.resize(kClasses);
        batches_.resize(be_.streams());
    }

    // a request arrives; pairs may repeat (counted once).  Returns false (and
    // queues nothing) when a pair names no brick or a LOD beyond its side.
    bool submit(const uint32_t* ids, const uint8_t* lods, uint32_t n, double t_arrival, uint64_t* req) {
        for (uint32_t j = 0; j < n; ++j)
            if (ids[j] >= l2_.size() || lods[j] > l2_[ids[j]]) return false;
        Req r;
        r.id = next_req_++;
        r.t_arr = t_arrival;
        r.keys.reserve(n);
        for (uint32_t j = 0; j < n; ++j) r.keys.push_back(key_of(ids[j], lods[j]));
        std::sort(r.keys.begin(), r.keys.end());
        r.keys.erase(std::unique(r.keys.begin(), r.keys.end()), r.keys.end());
        *req = r.id;
        waiting_.push_back(r.id);
        reqs_.emplace(r.id, std::move(r));
        return true;
    }

    // one scheduling step at time `now`: retire finished batches, admit waiting
    // requests in order, launch queued tasks on free streams.  Returns true
    // while anything is waiting, queued or in flight.
    bool step(double now) {
        // pairs of requests completed in the previous step: the caller has seen them
        for (uint64_t k : to_unpin_) unpin(k);
        to_unpin_.clear();
        for (int s = 0; s < (int)batches_.size(); ++s)
            if (!batches_[s].empty() && be_.poll(s)) retire(s, now);
        while (!waiting_.empty()) {
            Req& r = reqs_.at(waiting_.front());
            if (r.t_arr > now) break;
            if (!admit(r, now)) {
                if (can_reset()) {
                    reset();
                    if (admit(r, now)) {
                        waiting_.pop_front();
                        continue;
                    }
                    reject(r, now);  // larger than the whole cache
                    waiting_.pop_front();
                    continue;
                }
                break;
            }
            waiting_.pop_front();
        }
        for (int s = 0; s < (int)batches_.size() && !queued_.empty(); ++s)
            if (batches_[s].empty() && !be_.busy(s)) launch(s);
        return !waiting_.empty() || !queued_.empty() || in_flight() > 0;
    }

    // completed requests since the last call
    std::vector<ServeDone> drain() {
        std::vector<ServeDone> d;
        d.swap(done_);
        return d;
    }

    // unpin the pairs of a request completed while keep_pinned was set
    bool release(uint64_t req) {
        auto it = held_.find(req);
        if (it == held_.end()) return false;
        for (uint64_t k : it->second) unpin(k);
        held_.erase(it);
        return true;
    }

    // element offset of a resident pair (false if not resident)
    bool where(uint32_t id, uint8_t lod, uint64_t* off) const {
        auto it = map_.find(key_of(id, lod));
        if (it == map_.end() || it->second.state != kResident) return false;
        *off = it->second.off;
        return true;
    }

    double next_arrival() const {
        return waiting_.empty() ? -1.0 : reqs_.at(waiting_.front()).t_arr;
    }
    uint32_t in_flight() const {
        uint32_t n = 0;
        for (auto& b : batches_) n += b.empty() ? 0 : 1;
        return n;
    }
    const ServeStats& stats() {
        st_.top = top_;
        st_.resident = map_.size();
        uint64_t p = 0;
        for (auto& kv : map_) p += kv.second.pins ? 1 : 0;
        st_.pinned = p;
        return st_;
    }

private:
    enum { kQueued = 0, kFlight = 1, kResident = 2 };
    struct Entry {
        uint64_t off = 0;
        uint32_t cls = 0, pins = 0;
        int state = kQueued;
        std::vector<uint64_t> waiters;  // requests waiting for this pair
        std::list<uint64_t>::iterator lru;
        bool in_lru = false;
    };
    struct Req {
        uint64_t id = 0;
        double t_arr = 0, t_adm = 0;
        std::vector<uint64_t> keys;
        uint32_t pending = 0, n_decoded = 0;
    };
    static uint64_t key_of(uint32_t id, uint8_t lod) { return ((uint64_t)id << 8) | lod; }
    uint32_t class_of(uint64_t k) const { return l2_[(uint32_t)(k >> 8)] - (uint32_t)(k & 0xFF); }

    bool alloc(uint32_t cls, uint64_t* off) {
        if (!free_[cls].empty()) {
            *off = free_[cls].back();
            free_[cls].pop_back();
            return true;
        }
        if (cls_elems_[cls] <= cap_ - top_) {
            *off = top_;
            top_ += cls_elems_[cls];
            return true;
        }
        if (!lru_[cls].empty()) {  // least recently used unpinned resident pair of this class
            const uint64_t victim = lru_[cls].back();
            lru_[cls].pop_back();
            auto it = map_.find(victim);
            *off = it->second.off;
            map_.erase(it);
            ++st_.evictions;
            return true;
        }
        return false;
    }

    void pin(uint64_t k, Entry& e) {
        (void)k;
        if (e.in_lru) {
            lru_[e.cls].erase(e.lru);
            e.in_lru = false;
        }
        ++e.pins;
    }
    void unpin(uint64_t k) {
        auto it = map_.find(k);
        if (it == map_.end()) return;
        Entry& e = it->second;
        if (e.pins && --e.pins == 0 && e.state == kResident) {
            lru_[e.cls].push_front(k);
            e.lru = lru_[e.cls].begin();
            e.in_lru = true;
        }
    }

    bool admit(Req& r, double now) {
        std::vector<uint64_t> pinned, created;
        for (uint64_t k : r.keys) {
            auto it = map_.find(k);
            if (it != map_.end()) {
                pin(k, it->second);
                pinned.push_back(k);
                continue;
            }
            const uint32_t cls = class_of(k);
            uint64_t off;
            if (!alloc(cls, &off)) {
                rollback(pinned, created);
                return false;
            }
            Entry e;
            e.off = off;
            e.cls = cls;
            e.pins = 1;
            e.state = kQueued;
            map_.emplace(k, std::move(e));
            created.push_back(k);
            pinned.push_back(k);
        }
        r.t_adm = now;
        r.pending = 0;
        for (uint64_t k : r.keys) {
            Entry& e = map_.at(k);
            if (e.state != kResident) {
                e.waiters.push_back(r.id);
                ++r.pending;
            } else {
                ++st_.hits;
            }
        }
        st_.joined += r.pending - created.size();
        for (uint64_t k : created) queued_.push_back(k);
        r.n_decoded = (uint32_t)created.size();
        st_.pairs_requested += r.keys.size();
        for (uint64_t k : r.keys) st_.requested_elements += cls_elems_[class_of(k)];
        if (r.pending == 0) finish(r, now);
        return true;
    }

    void rollback(const std::vector<uint64_t>& pinned, const std::vector<uint64_t>& created) {
        for (uint64_t k : created) {
            auto it = map_.find(k);
            free_[it->second.cls].push_back(it->second.off);
            map_.erase(it);
        }
        for (uint64_t k : pinned) {
            if (std::find(created.begin(), created.end(), k) != created.end()) continue;
            unpin(k);
        }
    }

    void reject(Req& r, double now) {
        ServeDone d{r.id, r.t_arr, now, now, (uint32_t)r.keys.size(), 0, -1};
        done_.push_back(d);
        reqs_.erase(r.id);
    }

    bool can_reset() const {
        if (!queued_.empty() || in_flight() > 0 || !held_.empty() || !to_unpin_.empty()) return false;
        for (auto& kv : map_)
            if (kv.second.pins) return false;
        return true;
    }
    void reset() {
        map_.clear();
        for (auto& f : free_) f.clear();
        for (auto& l : lru_) l.clear();
        top_ = 0;
        ++st_.resets;
    }

    void launch(int s) {
        std::vector<uint64_t>& b = batches_[s];
        ids_.clear();
        lods_.clear();
        offs_.clear();
        while (!queued_.empty() && b.size() < max_batch_) {
            const uint64_t k = queued_.front();
            queued_.pop_front();
            Entry& e = map_.at(k);
            e.state = kFlight;
            b.push_back(k);
            ids_.push_back((uint32_t)(k >> 8));
            lods_.push_back((uint8_t)(k & 0xFF));
            offs_.push_back(e.off);
            st_.decoded_elements += cls_elems_[e.cls];
        }
        st_.decoded += b.size();
        ++st_.batches;
        st_.max_batch_seen = std::max<uint32_t>(st_.max_batch_seen, (uint32_t)b.size());
        be_.launch(s, ids_.data(), lods_.data(), offs_.data(), (uint32_t)b.size());
    }

    void retire(int s, double now) {
        for (uint64_t k : batches_[s]) {
            Entry& e = map_.at(k);
            e.state = kResident;
            std::vector<uint64_t> w;
            w.swap(e.waiters);
            for (uint64_t rid : w) {
                Req& r = reqs_.at(rid);
                if (--r.pending == 0) finish(r, now);
            }
        }
        batches_[s].clear();
    }

    void finish(Req& r, double now) {
        ServeDone d{r.id, r.t_arr, r.t_adm, now, (uint32_t)r.keys.size(), r.n_decoded, 0};
        done_.push_back(d);
        ++st_.requests_done;
        if (keep_pinned_) held_.emplace(r.id, r.keys);
        else to_unpin_.insert(to_unpin_.end(), r.keys.begin(), r.keys.end());
        reqs_.erase(r.id);
    }

    Backend& be_;
    uint64_t cap_, top_ = 0;
    uint32_t max_batch_;
    bool keep_pinned_;
    std::vector<uint8_t> l2_;
    std::vector<uint64_t> cls_elems_;
    std::vector<std::vector<uint64_t>> free_;
    std::vector<std::list<uint64_t>> lru_;
    std::unordered_map<uint64_t, Entry> map_;
    std::unordered_map<uint64_t, Req> reqs_;
    std::unordered_map<uint64_t, std::vector<uint64_t>> held_;
    std::deque<uint64_t> waiting_;  // request ids in arrival order
    std::deque<uint64_t> queued_;   // pairs waiting for a batch
    std::vector<uint64_t> to_unpin_;  // pairs of requests completed in the last step
    std::vector<std::vector<uint64_t>> batches_;
    std::vector<ServeDone> done_;
    std::vector<uint32_t> ids_;
    std::vector<uint8_t> lods_;
    std::vector<uint64_t> offs_;
    uint64_t next_req_ = 0;
    ServeStats st_;
};

}  // namespace csgv
