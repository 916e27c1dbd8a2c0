// Host-only tests of the render server's scheduling core (arena, idle-slot
// cache, admission and completion rules).  Built with g++ and run by
// tests/test_sched_host.py; prints one line per check group and exits non-zero
// on the first failure.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "sched.hpp"

using namespace gdgs::sched;

#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                                 \
        }                                                                 \
    } while (0)

// Arena against a brute-force byte map: random alloc/free never overlaps,
// stays aligned and inside the arena, and freeing everything coalesces back
// into one range.
static void arena_random() {
    std::mt19937_64 rng(1);
    const size_t N = 1 << 20;
    Arena a(N);
    std::vector<char> owner(N / kAlign, 0);
    std::vector<std::pair<size_t, size_t>> live;
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || rng() % 3) {
            const size_t want = 1 + rng() % 40000;
            size_t off;
            if (a.alloc(want, &off)) {
                const size_t b = align_up(want);
                CHECK(off % kAlign == 0 && off + b <= N);
                for (size_t k = off / kAlign; k < (off + b) / kAlign; ++k) {
                    CHECK(!owner[k]);
                    owner[k] = 1;
                }
                live.push_back({off, want});
            } else {
                CHECK(a.largest_free() < align_up(want));
            }
        } else {
            const size_t i = rng() % live.size();
            const auto [off, want] = live[i];
            a.release(off, want);
            for (size_t k = off / kAlign; k < (off + align_up(want)) / kAlign; ++k) owner[k] = 0;
            live[i] = live.back();
            live.pop_back();
        }
        CHECK(a.consistent());
    }
    for (auto [off, want] : live) a.release(off, want);
    CHECK(a.used() == 0 && a.largest_free() == N && a.consistent());
    CHECK(a.peak() <= N);
    std::printf("arena: random alloc/free consistent, peak %zu of %zu\n", a.peak(), N);
}

// Idle slots are reused per key (same offset), and given back oldest first
// when another key needs the room.
static void slot_pool() {
    SlotPool p(10 * kAlign * 100);
    const SlotKey a{64, 64, 1000}, b{128, 128, 4000};
    Slot s1, s2, s3;
    CHECK(p.acquire(a, 300 * kAlign, &s1));
    CHECK(p.acquire(a, 300 * kAlign, &s2));
    p.release(s1);
    p.release(s2);
    CHECK(p.idle_count() == 2);
    CHECK(p.acquire(a, 300 * kAlign, &s3) && s3.off == s2.off);  // most recent first
    p.release(s3);
    // b needs 700 units: only 400 free, so both idle a-slots go back
    Slot sb;
    CHECK(p.acquire(b, 700 * kAlign, &sb));
    CHECK(p.idle_count() == 1 || p.idle_count() == 0);
    CHECK(!p.could_fit(1001 * kAlign));
    p.discard(sb);
    std::printf("slot pool: reuse and eviction ok\n");
}

static Core::Config cfg(size_t budget, int streams) {
    Core::Config c;
    c.budget = budget;
    c.streams = streams;
    c.max_cycles = 10;
    c.resume_cycles = 2;
    c.initial_cap = 1 << 16;
    c.slot_bytes = [](int32_t W, int32_t H, int64_t cap) {
        return (size_t)W * H * 16 + (size_t)cap * 8;
    };
    return c;
}

// Arrival order, stream limit, no start before arrival.
static void admission_order() {
    Core c(cfg(size_t(1) << 30, 2));
    CHECK(c.submit(1, 0, 64, 64, 300));
    CHECK(c.submit(2, 0, 64, 64, 100));
    CHECK(c.submit(3, 0, 64, 64, 200));
    CHECK(c.admit(50) == nullptr);            // nothing has arrived
    Request* r = c.admit(150);
    CHECK(r && r->id == 2 && r->admit_ns == 150);
    CHECK(c.admit(150) == nullptr);           // 3 and 1 not arrived yet
    Request* r3 = c.admit(1000);
    CHECK(r3 && r3->id == 3);
    CHECK(c.admit(1000) == nullptr);          // both streams busy
    CHECK(r->stream != r3->stream);
    const int freed = r->stream;
    CHECK(c.finish_run(r, false, 1000, true, 5) == Next::Complete);
    CHECK(r->stream == -1);
    Request* r1 = c.admit(1000);
    CHECK(r1 && r1->id == 1 && r1->stream == freed);
    CHECK(r1->run_cycles == 5);               // learned from request 2 (same size)
    std::printf("admission: arrival order, stream limit ok\n");
}

// The head of the queue waits for memory and is not overtaken.
static void memory_blocking() {
    // slot bytes: 256x256 -> 1 MiB + cap*8
    Core::Config k = cfg((5u << 20) / 2, 4);   // room for one 1.5 MiB slot only
    k.initial_cap = 1 << 16;
    Core c(k);
    CHECK(c.submit(1, 0, 256, 256, 0));       // ~1.5 MiB
    CHECK(c.submit(2, 0, 256, 256, 1));
    CHECK(c.submit(3, 0, 16, 16, 2));         // small, but behind 2
    Request* a = c.admit(10);
    CHECK(a && a->id == 1);
    CHECK(c.admit(10) == nullptr);            // 2 does not fit next to 1: 3 waits too
    CHECK(c.waiting() == 2);
    CHECK(c.finish_run(a, false, 10, true, 3) == Next::Complete);
    Request* b = c.admit(10);
    CHECK(b && b->id == 2 && b->slot.off == a->slot.off);  // idle slot reused
    CHECK(!c.submit(9, 0, 1024, 1024, 0));    // 16 MiB never fits: rejected
    std::printf("admission: memory-blocked head waits, reject oversize ok\n");
}

// Overflow -> retry at the head with a larger capacity; unconverged -> resume
// in steps of 2 up to max_cycles; cancel.
static void completion_rules() {
    Core c(cfg(size_t(1) << 30, 1));
    CHECK(c.submit(1, 7, 64, 64, 0));
    CHECK(c.submit(2, 8, 64, 64, 5));
    Request* r = c.admit(10);
    CHECK(r->id == 1 && r->cap == (1 << 16) && r->run_cycles == 10);
    CHECK(c.finish_run(r, true, 200000, false, 0) == Next::Retry);
    CHECK(c.running() == 0 && c.waiting() == 2);
    Request* again = c.admit(11);
    CHECK(again && again->id == 1 && again->attempts == 2);
    CHECK(again->cap >= 200000 && again->cap % (1 << 16) == 0);
    CHECK(c.finish_run(again, false, 200000, false, 4) == Next::Resume);
    CHECK(again->run_cycles == 2 && again->runs == 2);
    CHECK(c.finish_run(again, false, 200000, false, 6) == Next::Resume);
    CHECK(c.finish_run(again, false, 200000, false, 8) == Next::Resume);
    CHECK(c.finish_run(again, false, 200000, false, 10) == Next::Complete);  // limit
    CHECK(!again->converged && again->cycles == 10);
    Request* r2 = c.admit(12);
    CHECK(r2 && r2->id == 2 && r2->cap >= 200000);  // capacity learned for 64x64
    // cancel while running: completes after this run, no resume
    CHECK(!c.cancel(2));
    CHECK(c.finish_run(r2, false, 100, false, 1) == Next::Complete && r2->cancelled);
    // cancel while waiting
    CHECK(c.submit(3, 0, 64, 64, 100));
    CHECK(c.cancel(3) && c.waiting() == 0);
    CHECK(c.admit(1000) == nullptr);
    std::printf("completion: retry, resume, limit, cancel ok\n");
}

// A request that gives up its stream (its solve continues in the batched
// rounds) keeps its slot and counts as running; the stream takes the next
// request at once.
static void detached_streams() {
    Core c(cfg(size_t(1) << 30, 1));
    CHECK(c.submit(1, 0, 64, 64, 0));
    CHECK(c.submit(2, 0, 64, 64, 1));
    Request* a = c.admit(10);
    CHECK(a && a->id == 1 && c.admit(10) == nullptr);   // the one stream is busy
    const size_t used = c.pool().arena().used();
    c.detach_stream(a);
    CHECK(a->stream == -1 && c.running() == 1);
    Request* b = c.admit(10);
    CHECK(b && b->id == 2 && b->stream == 0 && c.running() == 2);
    CHECK(b->slot.off != a->slot.off && c.pool().arena().used() > used);  // both slots held
    CHECK(c.finish_run(a, false, 10, true, 7) == Next::Complete);
    CHECK(c.running() == 1 && c.pool().idle_count() == 1);
    c.forget(1);
    CHECK(c.finish_run(b, false, 10, true, 7) == Next::Complete);
    CHECK(c.running() == 0 && c.admit(20) == nullptr);
    std::printf("detached streams: slot kept, stream reused ok\n");
}

// Simulated serving: random sizes and arrivals through a fake executor with
// random durations.  Every request completes exactly once, memory in use
// never exceeds the budget, at most `streams` run at once, and starts follow
// arrival order.
static void simulated_serving() {
    std::mt19937_64 rng(7);
    const int streams = 3;
    Core c(cfg(64u << 20, streams));
    const int sizes[4][2] = {{256, 256}, {512, 512}, {800, 800}, {1920, 1080}};
    const int N = 400;
    std::vector<int64_t> arrival(N);
    int64_t t = 0;
    for (int i = 0; i < N; ++i) {
        t += rng() % 1000;
        arrival[i] = t;
        const int* s = sizes[rng() % 4];
        CHECK(c.submit(i + 1, i, s[0], s[1], t));
    }
    struct Run { int64_t end; Request* r; };
    std::vector<Run> runs;
    std::set<int64_t> done;
    std::vector<int64_t> start_order;
    int64_t now = 0;
    while ((int)done.size() < N) {
        while (Request* r = c.admit(now)) {
            if (r->runs == 1 && r->attempts == 1) start_order.push_back(r->id);
            runs.push_back({now + 1 + (int64_t)(rng() % 5000), r});
        }
        CHECK((int)runs.size() <= streams && c.running() == (int)runs.size());
        CHECK(c.pool().arena().used() <= c.pool().arena().size());
        CHECK(c.pool().arena().consistent());
        if (runs.empty()) {
            now = std::max(now + 1, c.next_arrival());
            continue;
        }
        auto it = std::min_element(runs.begin(), runs.end(),
                                   [](const Run& a, const Run& b) { return a.end < b.end; });
        now = it->end;
        Request* r = it->r;
        runs.erase(it);
        const int64_t pairs = (int64_t)r->W * r->H / 8 + (int64_t)(rng() % 20000);
        const bool ovf = pairs > r->cap;
        // the fake solve converges after its 6th cycle and stops there
        const int cyc = std::min(6, r->cycles + r->run_cycles);
        const bool conv = cyc >= 6;
        const Next nx = c.finish_run(r, ovf, pairs, conv, cyc);
        if (nx == Next::Resume) runs.push_back({now + 1 + (int64_t)(rng() % 500), r});
        if (nx == Next::Complete) {
            CHECK(done.insert(r->id).second);
            CHECK(r->converged && r->cycles == 6 && r->num_pairs <= r->cap);
            c.forget(r->id);
        }
    }
    for (size_t i = 1; i < start_order.size(); ++i)
        CHECK(arrival[start_order[i] - 1] >= arrival[start_order[i - 1] - 1]);
    CHECK(c.waiting() == 0 && c.running() == 0);
    std::printf("simulation: %d requests, each once, budget and order kept (peak %zu of %zu)\n",
                N, c.pool().arena().peak(), c.pool().arena().size());
}

int main() {
    arena_random();
    slot_pool();
    admission_order();
    memory_blocking();
    completion_rules();
    detached_streams();
    simulated_serving();
    std::printf("ALL OK\n");
    return 0;
}
