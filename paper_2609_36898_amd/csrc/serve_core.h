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
// pair is resident, in flight, or can be given a slot: the free list of its
// class, the cache top, the least recently used unpinned entry of its class,
// or a slot of a larger class (free, else its least recently used entry)
// split into slots of this class.  A request that cannot be admitted waits,
// and a full cache with nothing pinned is reset.  Admitted misses queue as decode tasks; whenever a
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
#include <atomic>
#include <chrono>
#include <deque>
#include <memory>
#include <thread>
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
             batches = 0, splits = 0;
    uint64_t decoded_elements = 0, requested_elements = 0, top = 0, resident = 0, pinned = 0;
    uint32_t max_batch_seen = 0;
};

template <class Backend>
class Scheduler {
public:
    static constexpr uint32_t kClasses = 7;  // cube sides 1 .. 64

    // brick_log2b: side exponent of every brick (1..6).  Batches name brick
    // i * id_stride + id_offset for the scheduler's brick i (a shard of a
    // larger volume, see ShardSet).
    Scheduler(Backend& be, uint64_t cache_elems, const uint8_t* brick_log2b, uint32_t n_bricks, uint32_t max_batch,
              bool keep_pinned, uint32_t id_stride = 1, uint32_t id_offset = 0)
        : be_(be), cap_(cache_elems), max_batch_(max_batch ? max_batch : 1), keep_pinned_(keep_pinned),
          id_stride_(id_stride), id_offset_(id_offset) {
        l2_.assign(brick_log2b, brick_log2b + n_bricks);
        slot_.assign((size_t)n_bricks * 8, 0u);
        stamp_.assign((size_t)n_bricks * 8, 0u);
        for (uint32_t c = 0; c < kClasses; ++c) cls_elems_.push_back(uint64_t(1) << (3 * c));
        free_.resize(kClasses);
        head_.assign(kClasses, kNil);
        tail_.assign(kClasses, kNil);
        batches_.resize(be_.streams());
    }

    // a request arrives; pairs may repeat (counted once).  Returns false (and
    // queues nothing) when a pair names no brick or a LOD beyond its side.
    bool submit(const uint32_t* ids, const uint8_t* lods, uint32_t n, double t_arrival, uint64_t* req) {
        for (uint32_t j = 0; j < n; ++j)
            if (ids[j] >= l2_.size() || lods[j] > l2_[ids[j]]) return false;
        if (++stamp_now_ == 0) {  // wrapped: forget every stamp
            std::fill(stamp_.begin(), stamp_.end(), 0u);
            stamp_now_ = 1;
        }
        Req r;
        r.id = next_req_++;
        r.t_arr = t_arrival;
        r.keys.reserve(n);
        for (uint32_t j = 0; j < n; ++j) {
            const uint64_t k = key_of(ids[j], lods[j]);
            if (stamp_[k] != stamp_now_) {
                stamp_[k] = stamp_now_;
                r.keys.push_back(k);
            }
        }
        *req = r.id;
        if (reqs_.empty()) req_base_ = r.id;
        reqs_.push_back(std::move(r));
        waiting_.push_back(*req);
        return true;
    }

    // one scheduling step at time `now`: retire finished batches, admit waiting
    // requests in order, launch queued tasks on free streams.  Returns true
    // while anything is waiting, queued or in flight.
    bool step(double now) {
        // pairs of requests completed in the previous step: the caller has seen them
        prefetch_keys(to_unpin_);
        for (uint64_t k : to_unpin_) unpin(k);
        to_unpin_.clear();
        for (int s = 0; s < (int)batches_.size(); ++s)
            if (!batches_[s].empty() && be_.poll(s)) retire(s, now);
        while (!waiting_.empty()) {
            Req& r = req(waiting_.front());
            if (r.t_arr > now) break;
            if (!admit(r, now)) {
                if (can_reset()) {
                    reset();
                    if (!admit(r, now)) reject(r, now);  // larger than the whole cache
                    waiting_.pop_front();
                    continue;
                }
                break;
            }
            waiting_.pop_front();
            // a full batch goes out at once when a stream is free, so the device
            // works while a long admission run continues
            if (queued_.size() >= max_batch_) launch_full(now);
        }
        for (int s = 0; s < (int)batches_.size() && !queued_.empty(); ++s)
            if (batches_[s].empty() && !be_.busy(s)) launch(s);
        drop_finished();
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
        if (id >= l2_.size() || lod > 7) return false;
        const uint32_t e = slot_[key_of(id, lod)];
        if (!e || ent_[e - 1].state != kResident) return false;
        *off = ent_[e - 1].off;
        return true;
    }

    double next_arrival() const { return waiting_.empty() ? -1.0 : reqs_[waiting_.front() - req_base_].t_arr; }
    uint32_t in_flight() const {
        uint32_t n = 0;
        for (auto& b : batches_) n += b.empty() ? 0 : 1;
        return n;
    }
    const ServeStats& stats() {
        st_.top = top_;
        st_.resident = n_live_;
        st_.pinned = n_pinned_;
        return st_;
    }

private:
    enum { kQueued = 0, kFlight = 1, kResident = 2 };
    static constexpr uint32_t kNil = 0xFFFFFFFFu;
    // a cache entry (pair resident, queued or in flight); slot_[key] = index + 1
    struct Entry {
        uint64_t off = 0, key = 0;
        uint32_t pins = 0, prev = kNil, next = kNil;  // LRU links while unpinned and resident
        uint8_t cls = 0, state = kQueued;
        bool in_lru = false, live = false;
        std::vector<uint64_t> waiters;  // requests waiting for this pair
    };
    struct Req {
        uint64_t id = 0;
        double t_arr = 0, t_adm = 0;
        std::vector<uint64_t> keys;
        uint32_t pending = 0, n_decoded = 0;
        bool finished = false;
    };
    static uint64_t key_of(uint32_t id, uint8_t lod) { return (uint64_t)id * 8 + lod; }
    uint32_t class_of(uint64_t k) const { return l2_[k >> 3] - (uint32_t)(k & 7); }
    Req& req(uint64_t id) { return reqs_[id - req_base_]; }
    Entry* find(uint64_t k) { return slot_[k] ? &ent_[slot_[k] - 1] : nullptr; }

    uint32_t create(uint64_t k, uint64_t off, uint32_t cls) {
        uint32_t i;
        if (!ent_free_.empty()) {
            i = ent_free_.back();
            ent_free_.pop_back();
        } else {
            i = (uint32_t)ent_.size();
            ent_.emplace_back();
        }
        Entry& e = ent_[i];
        e.off = off;
        e.key = k;
        e.cls = (uint8_t)cls;
        e.pins = 1;
        e.state = kQueued;
        e.in_lru = false;
        e.live = true;
        e.waiters.clear();
        slot_[k] = i + 1;
        ++n_live_;
        ++n_pinned_;
        return i;
    }
    void erase(uint32_t i) {
        Entry& e = ent_[i];
        slot_[e.key] = 0;
        e.live = false;
        e.waiters.clear();
        ent_free_.push_back(i);
        --n_live_;
    }

    // per-class LRU list, most recent at the head
    void lru_push(uint32_t i) {
        Entry& e = ent_[i];
        e.prev = kNil;
        e.next = head_[e.cls];
        if (e.next != kNil) ent_[e.next].prev = i;
        else tail_[e.cls] = i;
        head_[e.cls] = i;
        e.in_lru = true;
    }
    void lru_remove(uint32_t i) {
        Entry& e = ent_[i];
        if (e.prev != kNil) ent_[e.prev].next = e.next;
        else head_[e.cls] = e.next;
        if (e.next != kNil) ent_[e.next].prev = e.prev;
        else tail_[e.cls] = e.prev;
        e.prev = e.next = kNil;
        e.in_lru = false;
    }

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
        if (tail_[cls] != kNil) {  // least recently used unpinned resident pair of this class
            *off = evict_lru(cls);
            return true;
        }
        // split a slot of the nearest larger class: a free one first, else its LRU entry
        for (int pass = 0; pass < 2; ++pass) {
            for (uint32_t c = cls + 1; c < kClasses; ++c) {
                uint64_t big;
                if (pass == 0 && !free_[c].empty()) {
                    big = free_[c].back();
                    free_[c].pop_back();
                } else if (pass == 1 && tail_[c] != kNil) {
                    big = evict_lru(c);
                } else {
                    continue;
                }
                const uint64_t n = cls_elems_[c] / cls_elems_[cls];
                for (uint64_t q = n - 1; q >= 1; --q) free_[cls].push_back(big + q * cls_elems_[cls]);
                *off = big;
                ++st_.splits;
                return true;
            }
        }
        return false;
    }

    uint64_t evict_lru(uint32_t cls) {
        const uint32_t v = tail_[cls];
        lru_remove(v);
        const uint64_t off = ent_[v].off;
        erase(v);
        ++st_.evictions;
        return off;
    }

    void pin(Entry& e, uint32_t i) {
        if (e.in_lru) lru_remove(i);
        if (e.pins++ == 0) ++n_pinned_;
    }
    void unpin(uint64_t k) {
        const uint32_t s = slot_[k];
        if (!s) return;
        Entry& e = ent_[s - 1];
        if (e.pins && --e.pins == 0) {
            --n_pinned_;
            if (e.state == kResident) lru_push(s - 1);
        }
    }

    // the table slots, then the entries, of a run of keys: issued together so
    // that the walks that follow find them in cache
    void prefetch_keys(const std::vector<uint64_t>& keys) {
        for (uint64_t k : keys) __builtin_prefetch(&slot_[k]);
        for (uint64_t k : keys)
            if (const uint32_t s = slot_[k]) __builtin_prefetch(&ent_[s - 1]);
    }

    bool admit(Req& r, double now) {
        created_.clear();
        prefetch_keys(r.keys);
        for (size_t j = 0; j < r.keys.size(); ++j) {
            const uint64_t k = r.keys[j];
            if (const uint32_t s = slot_[k]) {
                pin(ent_[s - 1], s - 1);
                continue;
            }
            const uint32_t cls = class_of(k);
            uint64_t off;
            if (!alloc(cls, &off)) {
                rollback(r, j);
                return false;
            }
            create(k, off, cls);
            created_.push_back(k);
        }
        r.t_adm = now;
        r.pending = 0;
        for (uint64_t k : r.keys) {
            Entry& e = ent_[slot_[k] - 1];
            if (e.state != kResident) {
                e.waiters.push_back(r.id);
                ++r.pending;
            } else {
                ++st_.hits;
            }
            st_.requested_elements += cls_elems_[e.cls];
        }
        st_.joined += r.pending - created_.size();
        for (uint64_t k : created_) queued_.push_back(k);
        r.n_decoded = (uint32_t)created_.size();
        st_.pairs_requested += r.keys.size();
        if (r.pending == 0) finish(r, now);
        return true;
    }

    // undo the first n_done keys of a failed admission: entries created by it
    // give their slots back (and are gone), the others are unpinned
    void rollback(Req& r, size_t n_done) {
        for (uint64_t k : created_) {
            const uint32_t s = slot_[k];
            free_[ent_[s - 1].cls].push_back(ent_[s - 1].off);
            --n_pinned_;
            erase(s - 1);
        }
        for (size_t j = 0; j < n_done; ++j)
            if (slot_[r.keys[j]]) unpin(r.keys[j]);
        created_.clear();
    }

    void reject(Req& r, double now) {
        ServeDone d{r.id, r.t_arr, now, now, (uint32_t)r.keys.size(), 0, -1};
        done_.push_back(d);
        r.finished = true;
        r.keys = std::vector<uint64_t>();
    }

    bool can_reset() const {
        return queued_.empty() && in_flight() == 0 && held_.empty() && to_unpin_.empty() && n_pinned_ == 0;
    }
    void reset() {
        for (uint32_t i = 0; i < (uint32_t)ent_.size(); ++i)
            if (ent_[i].live) erase(i);
        for (auto& f : free_) f.clear();
        std::fill(head_.begin(), head_.end(), kNil);
        std::fill(tail_.begin(), tail_.end(), kNil);
        top_ = 0;
        ++st_.resets;
    }

    // launch full batches on the streams that are (or have just become) free
    void launch_full(double now) {
        for (int s = 0; s < (int)batches_.size() && queued_.size() >= max_batch_; ++s) {
            if (!batches_[s].empty() && be_.poll(s)) retire(s, now);
            if (batches_[s].empty() && !be_.busy(s)) launch(s);
        }
    }

    void launch(int s) {
        std::vector<uint64_t>& b = batches_[s];
        ids_.clear();
        lods_.clear();
        offs_.clear();
        while (!queued_.empty() && b.size() < max_batch_) {
            const uint64_t k = queued_.front();
            queued_.pop_front();
            Entry& e = ent_[slot_[k] - 1];
            e.state = kFlight;
            b.push_back(k);
            ids_.push_back((uint32_t)(k >> 3) * id_stride_ + id_offset_);
            lods_.push_back((uint8_t)(k & 7));
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
            Entry& e = ent_[slot_[k] - 1];
            e.state = kResident;
            waiters_tmp_.swap(e.waiters);
            for (uint64_t rid : waiters_tmp_) {
                Req& r = req(rid);
                if (--r.pending == 0) finish(r, now);
            }
            waiters_tmp_.clear();
            // a pair whose requests all completed earlier (rollback) is unpinned and resident now
            if (e.pins == 0 && !e.in_lru) lru_push(slot_[k] - 1);
        }
        batches_[s].clear();
    }

    void finish(Req& r, double now) {
        ServeDone d{r.id, r.t_arr, r.t_adm, now, (uint32_t)r.keys.size(), r.n_decoded, 0};
        done_.push_back(d);
        ++st_.requests_done;
        if (keep_pinned_) held_.emplace(r.id, std::move(r.keys));
        else to_unpin_.insert(to_unpin_.end(), r.keys.begin(), r.keys.end());
        r.keys = std::vector<uint64_t>();
        r.finished = true;
    }

    void drop_finished() {
        while (!reqs_.empty() && reqs_.front().finished) {
            reqs_.pop_front();
            ++req_base_;
        }
    }

    Backend& be_;
    uint64_t cap_, top_ = 0;
    uint32_t max_batch_;
    bool keep_pinned_;
    uint32_t id_stride_, id_offset_;
    std::vector<uint8_t> l2_;
    std::vector<uint32_t> slot_;   // (id * 8 + LOD) -> entry index + 1, 0 when absent
    std::vector<uint32_t> stamp_;  // duplicate pairs within one submitted request
    uint32_t stamp_now_ = 0;
    std::vector<Entry> ent_;
    std::vector<uint32_t> ent_free_;
    uint64_t n_live_ = 0, n_pinned_ = 0;  // live entries; entries with pins > 0
    std::vector<uint64_t> cls_elems_;
    std::vector<std::vector<uint64_t>> free_;
    std::vector<uint32_t> head_, tail_;  // per-class LRU list ends
    std::deque<Req> reqs_;               // requests by id, from req_base_ on
    uint64_t req_base_ = 0;
    std::unordered_map<uint64_t, std::vector<uint64_t>> held_;
    std::deque<uint64_t> waiting_;  // request ids in arrival order
    std::deque<uint64_t> queued_;   // pairs waiting for a batch
    std::vector<uint64_t> to_unpin_;  // pairs of requests completed in the last step
    std::vector<std::vector<uint64_t>> batches_;
    std::vector<ServeDone> done_;
    std::vector<uint32_t> ids_;
    std::vector<uint8_t> lods_;
    std::vector<uint64_t> offs_;
    std::vector<uint64_t> created_, waiters_tmp_;
    uint64_t next_req_ = 0;
    ServeStats st_;
};

// Brick-sharded serving: the cache is partitioned by brick id.  Brick b
// belongs to shard b mod T, which knows it as brick b / T; every shard is a
// Scheduler over its own contiguous range of the cache and its own backend
// (streams), so T host threads can serve a trace side by side without
// sharing any scheduling state.  Every request is submitted to every shard
// with the pairs that shard owns (possibly none), so request ids agree across
// shards.  A request completes when its last part does: its admission and
// completion times are the latest over its parts, its pair counts the sums,
// and it is rejected when a part is.  Admission is in arrival order within a
// shard; across shards a later request can be admitted by one shard while an
// earlier one still waits in another.  Shards keep a completed part pinned
// until the whole request has completed (then until the next step, or with
// keep_pinned until release).  With T = 1 this is the Scheduler.
template <class Backend>
class ShardSet {
public:
    // be[w]: backend of shard w, whose batches carry offsets relative to base[w];
    // cap[w]: elements of shard w's range
    ShardSet(const std::vector<Backend*>& be, const std::vector<uint64_t>& base, const std::vector<uint64_t>& cap,
             const uint8_t* brick_log2b, uint32_t n_bricks, uint32_t max_batch, bool keep_pinned)
        : T_((uint32_t)be.size()), keep_(keep_pinned), base_(base), l2_(brick_log2b, brick_log2b + n_bricks),
          part_(be.size()) {
        for (uint32_t w = 0; w < T_; ++w) {
            const uint32_t nl = n_bricks / T_ + (w < n_bricks % T_ ? 1u : 0u);
            std::vector<uint8_t> l2(nl);
            for (uint32_t i = 0; i < nl; ++i) l2[i] = brick_log2b[(uint64_t)i * T_ + w];
            // several shards: parts stay held until the shard set releases them
            sh_.emplace_back(
                new Scheduler<Backend>(*be[w], cap[w], l2.data(), nl, max_batch, keep_pinned || T_ > 1, T_, w));
        }
    }

    uint32_t shards() const { return T_; }

    // false when a pair names no brick or a LOD beyond its side
    bool valid(const uint32_t* ids, const uint8_t* lods, uint64_t n) const {
        for (uint64_t j = 0; j < n; ++j)
            if (ids[j] >= l2_.size() || lods[j] > l2_[ids[j]]) return false;
        return true;
    }

    bool submit(const uint32_t* ids, const uint8_t* lods, uint32_t n, double t_arrival, uint64_t* req) {
        if (!valid(ids, lods, n)) return false;
        if (T_ == 1) return sh_[0]->submit(ids, lods, n, t_arrival, req);
        for (auto& p : part_) {
            p.ids.clear();
            p.lods.clear();
        }
        for (uint32_t j = 0; j < n; ++j) {
            Part& p = part_[ids[j] % T_];
            p.ids.push_back(ids[j] / T_);
            p.lods.push_back(lods[j]);
        }
        for (uint32_t w = 0; w < T_; ++w)
            sh_[w]->submit(part_[w].ids.data(), part_[w].lods.data(), (uint32_t)part_[w].ids.size(), t_arrival, req);
        Acc& a = acc_[*req];
        a.left = T_;
        a.d = ServeDone{*req, t_arrival, t_arrival, t_arrival, 0, 0, 0};
        return true;
    }

    bool step(double now) {
        // parts of requests completed (or rejected) since the last step
        for (uint64_t r : release_next_)
            for (auto& s : sh_) s->release(r);
        release_next_.clear();
        bool busy = false;
        for (auto& s : sh_) busy |= s->step(now);
        return busy;
    }

    std::vector<ServeDone> drain() {
        if (T_ == 1) return sh_[0]->drain();
        std::vector<ServeDone> out;
        for (auto& s : sh_)
            for (const ServeDone& d : s->drain()) merge(d, out);
        return out;
    }

    bool release(uint64_t req) {
        bool any = false;
        for (auto& s : sh_) any |= s->release(req);
        return any;
    }

    // element offset of a resident pair in the whole cache
    bool where(uint32_t id, uint8_t lod, uint64_t* off) const {
        if (id >= l2_.size()) return false;
        const uint32_t w = id % T_;
        if (!sh_[w]->where(id / T_, lod, off)) return false;
        *off += base_[w];
        return true;
    }

    ServeStats stats() {
        ServeStats t;
        for (auto& s : sh_) {
            const ServeStats& u = s->stats();
            t.requests_done += u.requests_done;
            t.pairs_requested += u.pairs_requested;
            t.hits += u.hits;
            t.joined += u.joined;
            t.decoded += u.decoded;
            t.evictions += u.evictions;
            t.resets += u.resets;
            t.batches += u.batches;
            t.splits += u.splits;
            t.decoded_elements += u.decoded_elements;
            t.requested_elements += u.requested_elements;
            t.top += u.top;
            t.resident += u.resident;
            t.pinned += u.pinned;
            t.max_batch_seen = std::max(t.max_batch_seen, u.max_batch_seen);
        }
        // a request counts once, when all its parts completed without a rejection
        if (T_ > 1) t.requests_done = done_ok_;
        return t;
    }

    // Serve a whole trace, one host thread per shard: request r holds pairs
    // [starts[r], starts[r + 1]) and arrives at t0 + arrival[r] on clock()
    // (nondecreasing); out[r] receives its record, times relative to t0.
    // ok(w) is asked after every step of shard w (a backend error) and stops
    // the run when false.  Completions of requests submitted before the run
    // stay queued for drain().  The pairs must be valid.
    template <class Clock, class Ok>
    bool run(const uint32_t* ids, const uint8_t* lods, const uint64_t* starts, uint32_t n_req, const double* arrival,
             double t0, Clock clock, Ok ok, ServeDone* out) {
        std::vector<std::vector<ServeDone>> parts(T_), early(T_);
        std::vector<std::vector<uint64_t>> late(T_);  // parts completed in a shard's last step
        std::atomic<bool> stop{false};
        // The trace is split once: thread c buckets the pairs of its contiguous
        // range of requests by shard (local brick ids, per-request counts); after
        // all threads have, shard w concatenates its buckets in request order.
        struct Bucket {
            std::vector<uint32_t> ids, count;  // count: pairs of each request of the range
            std::vector<uint8_t> lods;
        };
        std::vector<std::vector<Bucket>> bucket(T_, std::vector<Bucket>(T_));
        std::atomic<uint32_t> split_done{0};
        auto split = [&](uint32_t c) {
            const uint32_t r_lo = (uint32_t)((uint64_t)n_req * c / T_), r_hi = (uint32_t)((uint64_t)n_req * (c + 1) / T_);
            std::vector<Bucket>& b = bucket[c];
            for (auto& x : b) x.count.assign(r_hi - r_lo, 0u);
            for (uint32_t r = r_lo; r < r_hi; ++r)
                for (uint64_t j = starts[r]; j < starts[r + 1]; ++j) {
                    Bucket& x = b[ids[j] % T_];
                    x.ids.push_back(ids[j] / T_);
                    x.lods.push_back(lods[j]);
                    ++x.count[r - r_lo];
                }
            split_done.fetch_add(1);
        };
        auto serve = [&](uint32_t w) {
            Scheduler<Backend>& s = *sh_[w];
            // this shard's pairs of every request, as local brick ids
            std::vector<uint32_t> li;
            std::vector<uint8_t> ll;
            std::vector<uint64_t> ls;
            const uint32_t* pi = ids;
            const uint8_t* pl = lods;
            const uint64_t* ps = starts;
            if (T_ > 1) {
                split(w);
                // every thread is running (one per shard), so this wait ends
                while (split_done.load() < T_) std::this_thread::yield();
                size_t total = 0;
                for (uint32_t c = 0; c < T_; ++c) total += bucket[c][w].ids.size();
                li.reserve(total);
                ll.reserve(total);
                ls.assign(n_req + 1, 0);
                uint32_t r = 0;
                for (uint32_t c = 0; c < T_; ++c) {
                    const Bucket& x = bucket[c][w];
                    li.insert(li.end(), x.ids.begin(), x.ids.end());
                    ll.insert(ll.end(), x.lods.begin(), x.lods.end());
                    for (uint32_t q = 0; q < (uint32_t)x.count.size(); ++q, ++r) ls[r + 1] = ls[r] + x.count[q];
                }
                pi = li.data();
                pl = ll.data();
                ps = ls.data();
            }
            std::vector<ServeDone>& mine = parts[w];
            mine.resize(n_req);
            std::vector<uint64_t> rel;  // this shard's parts of this run to release at its next step
            uint32_t next = 0, done = 0;
            uint64_t first = 0, rid = 0;
            while (done < n_req && !stop.load(std::memory_order_relaxed)) {
                // (the caller reads no cache contents during a run, so without
                // keep_pinned a part need not wait for its request's other parts)
                for (uint64_t r : rel) s.release(r);
                rel.clear();
                // requests are handed to the scheduler as they arrive
                const double now = clock();
                for (; next < n_req && t0 + arrival[next] <= now; ++next) {
                    s.submit(pi + ps[next], pl + ps[next], (uint32_t)(ps[next + 1] - ps[next]), t0 + arrival[next],
                             &rid);
                    if (next == 0) first = rid;
                }
                s.step(clock());
                if (!ok(w)) {
                    stop.store(true);
                    break;
                }
                for (const ServeDone& d : s.drain()) {
                    if (next > 0 && d.req >= first && d.req - first < n_req) {
                        mine[d.req - first] = d;
                        ++done;
                        if (T_ > 1 && !keep_) rel.push_back(d.req);
                    } else {
                        early[w].push_back(d);  // a request submitted before this run
                    }
                }
                // idle until the next arrival when nothing is waiting, queued or in flight
                if (s.in_flight() == 0 && next < n_req && s.next_arrival() < 0) {
                    const double na = t0 + arrival[next], t = clock();
                    if (na > t + 2e-4) std::this_thread::sleep_for(std::chrono::duration<double>(na - t - 1e-4));
                }
            }
            late[w].swap(rel);
        };
        if (T_ == 1) {
            serve(0);
        } else {
            std::vector<std::thread> th;
            for (uint32_t w = 0; w < T_; ++w) th.emplace_back(serve, w);
            for (auto& t : th) t.join();
        }
        for (auto& l : late) release_next_.insert(release_next_.end(), l.begin(), l.end());
        if (stop.load()) return false;
        for (uint32_t r = 0; r < n_req; ++r) {
            ServeDone d = parts[0][r];
            for (uint32_t w = 1; w < T_; ++w) fold(d, parts[w][r]);
            if (T_ > 1 && d.status == 0) ++done_ok_;
            if (T_ > 1 && keep_ && d.status != 0) release_next_.push_back(d.req);  // parts held by a rejected request
            d.t_arrival -= t0;
            d.t_admit -= t0;
            d.t_done -= t0;
            out[r] = d;
        }
        for (uint32_t w = 0; w < T_; ++w)
            for (const ServeDone& d : early[w]) {
                if (T_ == 1) early_done_.push_back(d);
                else merge(d, early_done_);
            }
        return true;
    }

    // completions of requests submitted before a run, found during it
    std::vector<ServeDone> take_early() {
        std::vector<ServeDone> d;
        d.swap(early_done_);
        return d;
    }

private:
    struct Part {
        std::vector<uint32_t> ids;
        std::vector<uint8_t> lods;
    };
    struct Acc {
        uint32_t left = 0;
        ServeDone d;
    };
    // part b of a request folded into its record a
    static void fold(ServeDone& a, const ServeDone& b) {
        a.t_admit = std::max(a.t_admit, b.t_admit);
        a.t_done = std::max(a.t_done, b.t_done);
        a.n_pairs += b.n_pairs;
        a.n_decoded += b.n_decoded;
        a.status = std::min(a.status, b.status);
    }
    void merge(const ServeDone& d, std::vector<ServeDone>& out) {
        auto it = acc_.find(d.req);
        if (it == acc_.end()) return;
        fold(it->second.d, d);
        if (--it->second.left == 0) {
            const ServeDone& w = it->second.d;
            out.push_back(w);
            done_ok_ += w.status == 0 ? 1u : 0u;
            // unpinned at the next step, unless the caller releases it
            if (!keep_ || w.status != 0) release_next_.push_back(w.req);
            acc_.erase(it);
        }
    }

    uint32_t T_;
    bool keep_;
    std::vector<uint64_t> base_;
    std::vector<uint8_t> l2_;
    std::vector<std::unique_ptr<Scheduler<Backend>>> sh_;
    std::vector<Part> part_;
    std::unordered_map<uint64_t, Acc> acc_;
    std::vector<ServeDone> early_done_;
    std::vector<uint64_t> release_next_;
    uint64_t done_ok_ = 0;
};

}  // namespace csgv
