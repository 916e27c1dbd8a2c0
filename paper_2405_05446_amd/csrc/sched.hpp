// Host-side scheduling core of the render server: a first-fit device-memory
// arena, a cache of idle request slots, and the admission and completion
// rules for requests.  Plain C++ with no HIP dependency, so that it is unit
// tested on the host; the server drives it from its scheduler thread.
//
// Model.  Every in-flight request owns one slot: a contiguous range of the
// arena holding all of its transient state (projected splats, pair lists,
// gradient image, multigrid hierarchy, solution).  The arena is the memory
// budget.  A request is admitted when it has arrived, a stream is free and a
// slot can be had; waiting requests are served in arrival order (no request
// overtakes an earlier one, so none starves).  Idle slots are kept per shape
// (W, H, pair capacity) and handed to the next request of that shape, so the
// device addresses a request runs at recur and its launch sequence can be
// replayed from a cached graph; idle slots are given back to the arena,
// oldest first, when a request of another shape needs the room.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <functional>
#include <iterator>
#include <map>
#include <vector>

namespace gdgs {
namespace sched {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over offsets [0, size) with coalescing of free ranges.
class Arena {
   public:
    explicit Arena(size_t bytes) : size_(bytes & ~(kAlign - 1)) {
        if (size_) free_[0] = size_;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = align_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t o = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[o + bytes] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            *off = o;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align_up(bytes ? bytes : 1);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t largest_free() const {
        size_t m = 0;
        for (const auto& kv : free_) m = std::max(m, kv.second);
        return m;
    }
    // Free ranges sorted, disjoint, never adjacent, and summing to size - used.
    bool consistent() const {
        size_t sum = 0, end = 0;
        bool first = true;
        for (const auto& kv : free_) {
            if (kv.second == 0 || kv.first % kAlign || kv.second % kAlign) return false;
            if (!first && kv.first <= end) return false;  // overlapping or adjacent
            if (kv.first + kv.second > size_) return false;
            end = kv.first + kv.second;
            sum += kv.second;
            first = false;
        }
        return sum + used_ == size_;
    }

   private:
    size_t size_, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length
};

struct SlotKey {
    int32_t W = 0, H = 0;
    int64_t cap = 0;
    bool operator==(const SlotKey& o) const { return W == o.W && H == o.H && cap == o.cap; }
};

struct Slot {
    size_t off = 0, bytes = 0;
    SlotKey key;
};

class SlotPool {
   public:
    explicit SlotPool(size_t budget) : arena_(budget) {}
    // An idle slot of this key (the most recently released), else fresh arena
    // memory, giving idle slots of other keys back (oldest first) while the
    // arena cannot serve the request.
    bool acquire(const SlotKey& key, size_t bytes, Slot* out) {
        for (auto it = idle_.rbegin(); it != idle_.rend(); ++it) {
            if (it->key == key && it->bytes >= bytes) {
                *out = *it;
                idle_.erase(std::next(it).base());
                return true;
            }
        }
        size_t off = 0;
        while (!arena_.alloc(bytes, &off)) {
            if (idle_.empty()) return false;
            arena_.release(idle_.front().off, idle_.front().bytes);
            idle_.pop_front();
        }
        *out = Slot{off, align_up(bytes ? bytes : 1), key};
        return true;
    }
    void release(const Slot& s) { idle_.push_back(s); }
    void discard(const Slot& s) { arena_.release(s.off, s.bytes); }
    // Whether `bytes` could be served if every idle slot were given back.
    bool could_fit(size_t bytes) const { return align_up(bytes) <= arena_.size(); }
    size_t idle_count() const { return idle_.size(); }
    const Arena& arena() const { return arena_; }

   private:
    Arena arena_;
    std::deque<Slot> idle_;  // front = released longest ago
};

enum class Phase { Waiting, Running, Done };
enum class Next { Complete, Resume, Retry };

struct Request {
    int64_t id = 0;
    uint64_t tag = 0;
    int32_t W = 0, H = 0;
    int64_t arrival_ns = 0;
    int64_t admit_ns = -1;   // first admission
    Phase phase = Phase::Waiting;
    bool cancelled = false;
    int stream = -1;
    Slot slot;
    int64_t cap = 0;         // pair capacity of the slot
    int run_cycles = 0;      // V-cycle budget of the current run
    int cycles = 0;          // cycles done so far (largest over channels)
    int attempts = 0;        // admissions (more than one after a capacity retry)
    int runs = 0;            // runs in the current attempt (first run + resumes)
    int64_t num_pairs = 0;
    bool converged = false;
};

// Per-resolution learning: the pair capacity from the largest pair count seen
// (plus a quarter), and the first-run cycle budget from the most cycles a
// finished request of that size needed.  Later runs of a request resume the
// solve two cycles at a time, so the budget affects only speed, never the
// result.
struct ResInfo {
    int64_t cap = 0;
    int budget = 0;
    bool learned = false;
};

class Core {
   public:
    struct Config {
        size_t budget = 0;       // arena bytes
        int streams = 1;         // concurrent requests
        int max_cycles = 20;     // per-request V-cycle limit
        int resume_cycles = 2;   // cycles per resumed run
        int64_t initial_cap = 0; // pair capacity before anything is learned
        int64_t max_cap = 0xFFFFFFF0ll;
        std::function<size_t(int32_t W, int32_t H, int64_t cap)> slot_bytes;
    };

    explicit Core(const Config& c) : cfg_(c), pool_(c.budget), stream_busy_(c.streams, 0) {}

    // false: the request could never fit the budget (rejected).
    bool submit(int64_t id, uint64_t tag, int32_t W, int32_t H, int64_t arrival_ns) {
        const int64_t cap = res(W, H).cap;
        if (!pool_.could_fit(cfg_.slot_bytes(W, H, cap))) return false;
        Request& r = reqs_[id];
        r.id = id;
        r.tag = tag;
        r.W = W;
        r.H = H;
        r.arrival_ns = arrival_ns;
        waiting_.insert(std::make_pair(std::make_pair(arrival_ns, id), id));
        return true;
    }

    // The next request to start at time `now`, or null.  Strict arrival
    // order: the oldest arrived request waits for memory rather than being
    // overtaken.
    Request* admit(int64_t now) {
        if (waiting_.empty()) return nullptr;
        auto it = waiting_.begin();
        if (it->first.first > now) return nullptr;
        int s = -1;
        for (int k = 0; k < cfg_.streams; ++k)
            if (!stream_busy_[k]) {
                s = k;
                break;
            }
        if (s < 0) return nullptr;
        Request& r = reqs_.at(it->second);
        ResInfo& ri = res(r.W, r.H);
        if (r.cap < ri.cap) r.cap = ri.cap;
        const SlotKey key{r.W, r.H, r.cap};
        const size_t bytes = cfg_.slot_bytes(r.W, r.H, r.cap);
        if (!pool_.could_fit(bytes)) {
            // grown past the whole budget by a capacity retry: can never run
            waiting_.erase(it);
            r.phase = Phase::Done;
            rejected_.push_back(r.id);
            return nullptr;
        }
        Slot slot;
        if (!pool_.acquire(key, bytes, &slot)) return nullptr;  // wait for memory
        waiting_.erase(it);
        stream_busy_[s] = 1;
        ++running_;
        r.phase = Phase::Running;
        r.stream = s;
        r.slot = slot;
        r.cycles = 0;
        r.runs = 1;
        r.converged = false;
        ++r.attempts;
        if (r.admit_ns < 0) r.admit_ns = now;
        r.run_cycles = std::max(1, std::min(cfg_.max_cycles, ri.budget));
        return &r;
    }

    // Earliest arrival among waiting requests (INT64_MAX if none).
    int64_t next_arrival() const {
        return waiting_.empty() ? INT64_MAX : waiting_.begin()->first.first;
    }

    // A run of r ended with these device statistics.  Complete: r is done and
    // its slot and stream are free; Resume: run r again on the same slot and
    // stream for r->run_cycles more cycles; Retry: the pair list overflowed, r
    // waits again at the head of the queue with a larger capacity.
    Next finish_run(Request* r, bool overflow, int64_t num_pairs, bool converged, int cycles) {
        r->num_pairs = num_pairs;
        ResInfo& ri = res(r->W, r->H);
        if (overflow && !r->cancelled) {
            const int64_t want = std::min(cfg_.max_cap, num_pairs + num_pairs / 4 + 1024);
            ri.cap = std::max(ri.cap, round_cap(want));
            r->cap = ri.cap;
            pool_.discard(r->slot);   // a slot of the old capacity is of no further use
            free_stream(r);
            r->phase = Phase::Waiting;
            // keeps its arrival time, so it is first in line again
            waiting_.insert(std::make_pair(std::make_pair(r->arrival_ns, r->id), r->id));
            return Next::Retry;
        }
        r->cycles = cycles;
        r->converged = converged;
        if (!r->cancelled && !converged && cycles < cfg_.max_cycles) {
            r->run_cycles = std::min(cfg_.resume_cycles, cfg_.max_cycles - cycles);
            ++r->runs;
            return Next::Resume;
        }
        // learn from a finished request
        const int64_t grown = round_cap(num_pairs + num_pairs / 4 + 1024);
        if (!r->cancelled && grown > ri.cap && grown <= cfg_.max_cap) ri.cap = grown;
        if (!r->cancelled && converged) {
            // the first finished request of a size sets the budget, later ones
            // only raise it: few distinct budgets, so few distinct graphs
            ri.budget = ri.learned ? std::max(ri.budget, cycles) : std::max(1, cycles);
            ri.learned = true;
        }
        pool_.release(r->slot);
        free_stream(r);
        r->phase = Phase::Done;
        return Next::Complete;
    }

    // A running request gives up its stream but keeps its slot (and counts as
    // running) until finish_run: its remaining device work is carried
    // elsewhere (the server's batched solve rounds).
    void detach_stream(Request* r) {
        if (r->stream >= 0) stream_busy_[r->stream] = 0;
        r->stream = -1;
    }

    // Waiting: removed now (true).  Running: flagged, ends after its current
    // run (false).  Unknown or done: false.
    bool cancel(int64_t id) {
        auto it = reqs_.find(id);
        if (it == reqs_.end() || it->second.phase == Phase::Done) return false;
        Request& r = it->second;
        r.cancelled = true;
        if (r.phase == Phase::Running) return false;
        waiting_.erase(std::make_pair(r.arrival_ns, r.id));
        r.phase = Phase::Done;
        return true;
    }

    // Drop a finished request's record.
    void forget(int64_t id) { reqs_.erase(id); }
    Request* find(int64_t id) {
        auto it = reqs_.find(id);
        return it == reqs_.end() ? nullptr : &it->second;
    }
    // Requests rejected at admission (grown past the budget); drained by the caller.
    std::vector<int64_t> take_rejected() {
        std::vector<int64_t> v;
        v.swap(rejected_);
        return v;
    }

    size_t waiting() const { return waiting_.size(); }
    int running() const { return running_; }
    const SlotPool& pool() const { return pool_; }
    ResInfo& res(int32_t W, int32_t H) {
        ResInfo& ri = res_[std::make_pair(W, H)];
        if (ri.cap == 0) {
            ri.cap = std::min(cfg_.max_cap, round_cap(cfg_.initial_cap));
            ri.budget = cfg_.max_cycles;
        }
        return ri;
    }

    static int64_t round_cap(int64_t p) {
        const int64_t q = 1 << 16;
        return ((std::max<int64_t>(p, 1) + q - 1) / q) * q;
    }

   private:
    void free_stream(Request* r) {
        if (r->stream >= 0) stream_busy_[r->stream] = 0;
        r->stream = -1;
        --running_;
    }

    Config cfg_;
    SlotPool pool_;
    std::vector<char> stream_busy_;
    int running_ = 0;
    std::map<int64_t, Request> reqs_;
    std::map<std::pair<int64_t, int64_t>, int64_t> waiting_;  // (arrival, id) -> id
    std::map<std::pair<int32_t, int32_t>, ResInfo> res_;
    std::vector<int64_t> rejected_;
};

}  // namespace sched
}  // namespace gdgs
