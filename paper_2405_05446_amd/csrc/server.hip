// Render server: one resident scene, many concurrent views of mixed sizes.
//
// Two ways of running the Poisson solves (gdgs_server_params.flags):
//  * batched (GDGS_SERVER_BATCHED): a request's stream carries its projection,
//    binning, compositing and the solve's set-up only; then the request joins
//    the batch table of in-flight solves and gives its stream back.  One solver
//    stream runs rounds -- one V-cycle of every solve in the table, each kernel
//    a persistent grid whose workgroups take tile tasks of all of them -- and
//    a solve that has converged is reported through a completion ring in
//    pinned host memory.  Its slot returns to the pool once no round that can
//    still touch it is in flight.
//  * per request (flags 0), described below.
//
// A native scheduler thread owns the device side.  It admits requests through
// the scheduling core (arrival order, free stream, memory budget), enqueues
// each request's frame on the request's own stream -- the projection with
// the request's camera, a copy of its boundary ring into its slot, then the
// binning and compositing as one cached graph per slot and size, the Poisson
// solve as another, a copy of the result to the caller's buffer and of the
// statistics to pinned host memory -- and records an event.  When the event has fired it
// reads the statistics: a pair overflow sends the request back to the queue
// with a larger capacity, an unconverged solve is resumed two V-cycles at a
// time (GDGS_MG_RESUME: bit for bit the same as one longer solve), and a
// finished request is moved to the completion queue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "graph.hpp"
#include "internal.hpp"
#include "sched.hpp"

namespace gdgs {
namespace {

int64_t steady_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// Copies the one-pixel ring of a [3][H][W] image (the only part of the
// boundary the solve reads).
__global__ void k_copy_ring(const float* __restrict__ src, float* __restrict__ dst, int W, int H) {
    const int nring = 2 * W + 2 * (H - 2);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * nring) return;
    const int c = i / nring, k = i % nring;
    int y, x;
    if (k < W) {
        y = 0;
        x = k;
    } else if (k < 2 * W) {
        y = H - 1;
        x = k - W;
    } else {
        const int q = k - 2 * W;
        y = 1 + (q >> 1);
        x = (q & 1) ? W - 1 : 0;
    }
    const size_t o = (size_t)c * H * W + (size_t)y * W + x;
    dst[o] = src[o];
}

// A request's slot: the render workspace, then the solution, the boundary
// copy and the statistics.
struct SlotLayout {
    RenderWs rw;
    float* u;
    float* boundary;
    gdgs_stats* stats;
};

size_t slot_layout(int64_t K, int W, int H, int64_t cap, const MgPlan& plan, char* base,
                   SlotLayout* out) {
    const size_t rbytes = render_layout(K, W, H, cap, plan, base, out ? &out->rw : nullptr);
    Carver c(base ? base + rbytes : nullptr);
    float* u = c.take<float>((size_t)3 * W * H);
    float* b = c.take<float>((size_t)3 * W * H);
    gdgs_stats* st = c.take<gdgs_stats>(1);
    if (out) {
        out->u = u;
        out->boundary = b;
        out->stats = st;
    }
    return rbytes + c.off + 256;
}

struct Payload {
    gdgs_camera cam;
    const float* boundary;
    float* u;
    const float* u_init;  // starting image of a warm-started solve, or null
};

}  // namespace
}  // namespace gdgs

struct gdgs_server {
    int dev = 0;
    uint64_t uid = 0;
    gdgs_scene scene{};
    gdgs_mg_params mg{};
    char* arena = nullptr;
    size_t arena_bytes = 0;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<int64_t> running;      // request id per stream, -1 if idle
    gdgs_stats* host_stats = nullptr;  // pinned, one per stream
    gdgs::sched::Core* core = nullptr;
    std::unordered_map<int64_t, gdgs::Payload> payload;
    std::map<std::tuple<int, int, int, int>, gdgs::MgPlan> plans;  // (W, H, cycles, flags)
    std::deque<gdgs_completion> done;
    // batched solves (flags & GDGS_SERVER_BATCHED)
    bool batched = false;
    hipStream_t solver = nullptr;
    void* btab = nullptr;                 // device table of in-flight solves
    gdgs::BatchRing* ring = nullptr;      // completion ring (pinned host memory)
    long long ring_read = 0;
    int64_t ent_req[gdgs::kBatchMax];     // request of each entry, -1 = free
    int ent_state[gdgs::kBatchMax];       // 0 free, 1 in the rounds, 2 leaving
    int ent_depth[gdgs::kBatchMax];
    int64_t ent_retire_at[gdgs::kBatchMax];  // rounds that must have completed first
    std::deque<int64_t> joinq;            // set-up done, waiting for an entry
    std::deque<std::pair<int64_t, hipEvent_t>> rounds;  // in flight: (sequence, event)
    std::vector<hipEvent_t> free_round_events;
    int64_t rounds_enq = 0, rounds_done = 0;
    std::mutex mu;
    std::condition_variable wake;       // scheduler: new work or stop
    std::condition_variable done_cv;    // pollers: a completion
    std::thread thread;
    bool stop = false;
    int64_t next_id = 1;
    int64_t submitted = 0, completed = 0;
    gdgs_status fatal = GDGS_OK;

    // Plans are cached per size, cycle budget and flags (mg_plan also sets
    // kernel attributes, which is not free).
    const gdgs::MgPlan* plan(int W, int H, int cycles, int flags) {
        const auto key = std::make_tuple(W, H, cycles, flags);
        auto it = plans.find(key);
        if (it != plans.end()) return &it->second;
        gdgs_mg_params q = mg;
        q.max_cycles = cycles;
        q.flags = flags | (mg.flags & GDGS_MG_NEUMANN);  // the server's boundary condition
        gdgs::MgPlan p;
        if (gdgs::mg_plan(W, H, &q, &p) != GDGS_OK) return nullptr;
        return &plans.emplace(key, p).first->second;
    }
    size_t slot_bytes(int W, int H, int64_t cap) {
        const gdgs::MgPlan* p = plan(W, H, mg.max_cycles, 0);
        if (!p) return SIZE_MAX / 2;
        return gdgs::slot_layout(scene.K, W, H, cap, *p, nullptr, nullptr);
    }

    void complete(const gdgs::sched::Request& r, int32_t status) {
        gdgs_completion c{};
        c.id = r.id;
        c.tag = r.tag;
        c.status = status;
        c.converged = r.converged ? 1 : 0;
        c.cycles = r.cycles;
        c.attempts = r.attempts;
        c.num_pairs = r.num_pairs;
        c.arrival_ns = r.arrival_ns;
        c.admit_ns = r.admit_ns;
        c.done_ns = gdgs::steady_ns();
        done.push_back(c);
        ++completed;
        payload.erase(r.id);
        done_cv.notify_all();
    }

    // the plan of a batched solve: the whole cycle limit (no resumed runs)
    const gdgs::MgPlan* batch_plan(const gdgs::Payload& p, int W, int H) {
        return plan(W, H, mg.max_cycles, p.u_init ? GDGS_MG_WARM_START : 0);
    }

    // First run of an admission (new request or capacity re-run).
    gdgs_status enqueue_first(gdgs::sched::Request* r) {
        using namespace gdgs;
        const Payload& p = payload.at(r->id);
        const int W = r->W, H = r->H, s = r->stream;
        hipStream_t st = streams[s];
        const MgPlan* plan = batched
                                 ? batch_plan(p, W, H)
                                 : this->plan(W, H, r->run_cycles,
                                              p.u_init ? GDGS_MG_WARM_START : 0);
        if (!plan) return GDGS_ERR_INVALID_ARGUMENT;
        char* base = arena + r->slot.off;
        SlotLayout L;
        slot_layout(scene.K, W, H, r->cap, *plan, base, &L);
        const int64_t K = scene.K;
        if (K > 0) {
            const gdgs_status e = launch_project(scene, p.cam, L.rw.proj, st);
            if (e != GDGS_OK) return e;
        }
        const float* bnd = nullptr;
        if (p.boundary) {
            const int nring = 3 * (2 * W + 2 * (H - 2));
            hipLaunchKernelGGL(k_copy_ring, dim3((nring + 255) / 256), dim3(256), 0, st,
                               p.boundary, L.boundary, W, H);
            GDGS_LAUNCH_CHECK();
            bnd = L.boundary;
        }
        BinWs b;
        bin_ws_layout(K, r->cap, num_tiles(W, H), L.rw.bin_ws, &b);
        const gdgs_scene sc = scene;
        const int64_t cap = r->cap;
        KeyBuilder kb;
        kb.tag("server").add(uid).add(base).add(W).add(H).add(cap).add(K).add(sc.opacity)
            .add(sc.value).add(bnd);
        add_plan(kb, *plan);
        KeyBuilder kr = kb;
        kr.tag("bin+raster");
        gdgs_status e = with_graph(kr, st, [&](hipStream_t q) -> gdgs_status {
            gdgs_status t = launch_bin_sort(L.rw.proj, K, W, H, L.rw.bins, b, q);
            if (t != GDGS_OK) return t;
            return launch_raster(L.rw.proj, sc.opacity, sc.value, K, L.rw.bins, W, H, L.rw.grad,
                                 L.rw.raster_ws, q);
        });
        if (e != GDGS_OK) return e;
        if (batched) {
            // the solve runs in the caller's image itself: set-up here, the
            // V-cycles in the batched rounds once this stream's work is done
            if (p.u_init && p.u_init != p.u)
                GDGS_HIP_TRY(hipMemcpyAsync(p.u, p.u_init, sizeof(float) * 3 * (size_t)W * H,
                                            hipMemcpyDeviceToDevice, st));
            e = launch_render_stats(L.rw.bins.num_pairs, cap, L.stats, st);
            if (e != GDGS_OK) return e;
            e = launch_poisson_setup(L.rw.grad, bnd, W, H, *plan, p.u, L.stats,
                                     L.rw.poisson_ws, st);
            if (e != GDGS_OK) return e;
            GDGS_HIP_TRY(hipMemcpyAsync(&host_stats[r->stream], L.stats, sizeof(gdgs_stats),
                                        hipMemcpyDeviceToHost, st));
            GDGS_HIP_TRY(hipEventRecord(events[r->stream], st));
            return GDGS_OK;
        }
        // warm start: the slot's image starts as the caller's (the solve sets
        // the ring from the boundary and keeps the interior)
        if (p.u_init)
            GDGS_HIP_TRY(hipMemcpyAsync(L.u, p.u_init, sizeof(float) * 3 * (size_t)W * H,
                                        hipMemcpyDeviceToDevice, st));
        // requests already overlap one another: the solve stays on the
        // request's stream as one graph
        e = launch_poisson(L.rw.grad, nullptr, bnd, W, H, *plan, L.u, L.stats, L.rw.poisson_ws,
                           st, &kb, false);
        if (e != GDGS_OK) return e;
        e = launch_render_stats(L.rw.bins.num_pairs, cap, L.stats, st);
        if (e != GDGS_OK) return e;
        return finish_enqueue(r, L, p, st);
    }

    // A resumed run: more V-cycles of the same solve in the same slot.
    gdgs_status enqueue_resume(gdgs::sched::Request* r) {
        using namespace gdgs;
        const Payload& p = payload.at(r->id);
        const int W = r->W, H = r->H;
        hipStream_t st = streams[r->stream];
        const MgPlan* plan = this->plan(W, H, r->run_cycles, GDGS_MG_RESUME);
        if (!plan) return GDGS_ERR_INVALID_ARGUMENT;
        char* base = arena + r->slot.off;
        SlotLayout L;
        slot_layout(scene.K, W, H, r->cap, *plan, base, &L);
        const float* bnd = p.boundary ? L.boundary : nullptr;
        KeyBuilder kb;
        kb.tag("server-resume").add(uid).add(base).add(W).add(H).add(r->cap).add(scene.K)
            .add(bnd);
        add_plan(kb, *plan);
        const gdgs_status e = launch_poisson(L.rw.grad, nullptr, bnd, W, H, *plan, L.u,
                                             L.stats, L.rw.poisson_ws, st, &kb, false);
        if (e != GDGS_OK) return e;
        return finish_enqueue(r, L, p, st);
    }

    gdgs_status finish_enqueue(gdgs::sched::Request* r, const gdgs::SlotLayout& L,
                               const gdgs::Payload& p, hipStream_t st) {
        const size_t ubytes = sizeof(float) * 3 * (size_t)r->W * r->H;
        GDGS_HIP_TRY(hipMemcpyAsync(p.u, L.u, ubytes, hipMemcpyDeviceToDevice, st));
        GDGS_HIP_TRY(hipMemcpyAsync(&host_stats[r->stream], L.stats, sizeof(gdgs_stats),
                                    hipMemcpyDeviceToHost, st));
        GDGS_HIP_TRY(hipEventRecord(events[r->stream], st));
        return GDGS_OK;
    }

    void fail(gdgs::sched::Request* r, gdgs_status e) {
        // the request's device work may be partial: report it and retire the
        // slot as if finished (its memory stays valid for later requests)
        if (fatal == GDGS_OK) fatal = e;
        running[r->stream] = -1;
        r->cancelled = true;  // retire without resuming or learning from it
        core->finish_run(r, false, r->num_pairs, true, r->cycles);
        complete(*r, e);
        core->forget(r->id);
    }

    // ---- batched solves
    // The request's set-up has run and its pair list fitted: enter the table.
    gdgs_status activate(int e, gdgs::sched::Request* r) {
        using namespace gdgs;
        const Payload& p = payload.at(r->id);
        const MgPlan* pl = batch_plan(p, r->W, r->H);
        if (!pl) return GDGS_ERR_INVALID_ARGUMENT;
        SlotLayout L;
        slot_layout(scene.K, r->W, r->H, r->cap, *pl, arena + r->slot.off, &L);
        const gdgs_status st = batch_activate(btab, e, r->id, L.rw.grad, r->W, r->H, *pl, p.u,
                                              L.stats, L.rw.poisson_ws, solver);
        if (st != GDGS_OK) return st;
        ent_req[e] = r->id;
        ent_state[e] = 1;
        ent_depth[e] = batch_depth(*pl);
        return GDGS_OK;
    }

    // Entry e stops taking part in rounds; rounds enqueued before this may
    // still read its slot, so the slot is freed once they have completed.
    gdgs_status retire(int e) {
        const gdgs_status st = gdgs::batch_deactivate(btab, e, solver);
        ent_state[e] = 2;
        ent_retire_at[e] = rounds_enq;
        return st;
    }

    // One pass of the batched side; true if anything changed.
    bool batch_step() {
        using gdgs::sched::Next;
        bool progress = false;
        // completed rounds
        while (!rounds.empty() && hipEventQuery(rounds.front().second) != hipErrorNotReady) {
            (void)hipGetLastError();
            rounds_done = rounds.front().first + 1;
            free_round_events.push_back(rounds.front().second);
            rounds.pop_front();
            progress = true;
        }
        // completion records: the solve is final in the caller's image
        const long long head = __atomic_load_n(&ring->head, __ATOMIC_ACQUIRE);
        while (ring_read < head) {
            const gdgs::BatchRec rec = ring->rec[ring_read % gdgs::kRingCap];
            ++ring_read;
            progress = true;
            int e = -1;
            for (int k = 0; k < gdgs::kBatchMax; ++k)
                if (ent_state[k] == 1 && ent_req[k] == rec.id) e = k;
            if (e < 0) continue;  // left the table already (cancelled)
            gdgs::sched::Request* r = core->find(rec.id);
            r->cycles = rec.cycles;
            r->converged = rec.converged != 0;
            if (retire(e) != GDGS_OK && fatal == GDGS_OK) fatal = GDGS_ERR_HIP;
            complete(*r, r->cancelled ? GDGS_ERR_CANCELLED : GDGS_OK);
        }
        // cancelled requests leave the table
        for (int k = 0; k < gdgs::kBatchMax; ++k) {
            if (ent_state[k] != 1) continue;
            gdgs::sched::Request* r = core->find(ent_req[k]);
            if (!r || !r->cancelled) continue;
            if (retire(k) != GDGS_OK && fatal == GDGS_OK) fatal = GDGS_ERR_HIP;
            complete(*r, GDGS_ERR_CANCELLED);
            progress = true;
        }
        // slots of retired entries go back to the pool
        for (int k = 0; k < gdgs::kBatchMax; ++k) {
            if (ent_state[k] != 2 || ent_retire_at[k] > rounds_done) continue;
            if (gdgs::sched::Request* r = core->find(ent_req[k])) {
                (void)core->finish_run(r, false, r->num_pairs, r->converged, r->cycles);
                core->forget(r->id);
            }
            ent_state[k] = 0;
            ent_req[k] = -1;
            progress = true;
        }
        // new members
        while (!joinq.empty()) {
            int e = -1;
            for (int k = 0; k < gdgs::kBatchMax && e < 0; ++k)
                if (ent_state[k] == 0) e = k;
            if (e < 0) break;
            const int64_t id = joinq.front();
            joinq.pop_front();
            progress = true;
            gdgs::sched::Request* r = core->find(id);
            if (r->cancelled) {
                complete(*r, GDGS_ERR_CANCELLED);
                (void)core->finish_run(r, false, r->num_pairs, false, 0);
                core->forget(id);
                continue;
            }
            const gdgs_status st = activate(e, r);
            if (st != GDGS_OK) {
                if (fatal == GDGS_OK) fatal = st;
                complete(*r, st);
                (void)core->finish_run(r, false, r->num_pairs, false, 0);
                core->forget(id);
            }
        }
        // the next round (two in flight keep the solver stream busy)
        int depth = -1;
        for (int k = 0; k < gdgs::kBatchMax; ++k)
            if (ent_state[k] == 1) depth = std::max(depth, ent_depth[k]);
        if (depth >= 0 && rounds.size() < 2) {
            hipEvent_t ev = nullptr;
            if (!free_round_events.empty()) {
                ev = free_round_events.back();
                free_round_events.pop_back();
            } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                ev = nullptr;
            }
            gdgs_status st = ev ? GDGS_OK : GDGS_ERR_HIP;
            if (st == GDGS_OK)
                st = gdgs::launch_batch_round(btab, ring, depth, mg.pre_sweeps, mg.post_sweeps,
                                              solver);
            if (st == GDGS_OK && hipEventRecord(ev, solver) != hipSuccess) st = GDGS_ERR_HIP;
            if (st != GDGS_OK) {
                // the device side cannot go on: finish every member with the error
                if (fatal == GDGS_OK) fatal = st;
                for (int k = 0; k < gdgs::kBatchMax; ++k) {
                    if (ent_state[k] != 1) continue;
                    gdgs::sched::Request* r = core->find(ent_req[k]);
                    complete(*r, st);
                    ent_state[k] = 2;
                    ent_retire_at[k] = rounds_enq;
                }
                if (ev) free_round_events.push_back(ev);
            } else {
                rounds.emplace_back(rounds_enq++, ev);
            }
            progress = true;
        }
        return progress;
    }

    bool batch_busy() const {
        if (!rounds.empty() || !joinq.empty()) return true;
        for (int k = 0; k < gdgs::kBatchMax; ++k)
            if (ent_state[k] != 0) return true;
        return false;
    }

    void loop() {
        using gdgs::sched::Next;
        (void)hipSetDevice(dev);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            bool progress = false;
            for (size_t s = 0; s < streams.size(); ++s) {
                const int64_t id = running[s];
                if (id < 0) continue;
                const hipError_t q = hipEventQuery(events[s]);
                if (q == hipErrorNotReady) continue;
                progress = true;
                gdgs::sched::Request* r = core->find(id);
                if (q != hipSuccess) {
                    (void)hipGetLastError();
                    fail(r, GDGS_ERR_HIP);
                    continue;
                }
                const gdgs_stats& hs = host_stats[s];
                if (batched) {
                    // front half done: re-run on overflow, else join the batch
                    if (hs.overflow != 0 && !r->cancelled) {
                        GDGS_LOG(2, "server: request %lld needs %lld pairs; run again with a "
                                    "larger capacity", (long long)id, (long long)hs.num_pairs);
                        (void)core->finish_run(r, true, hs.num_pairs, false, 0);
                        running[s] = -1;
                        continue;
                    }
                    r->num_pairs = hs.num_pairs;
                    core->detach_stream(r);
                    running[s] = -1;
                    joinq.push_back(id);
                    continue;
                }
                const int cyc = std::max(hs.cycles[0], std::max(hs.cycles[1], hs.cycles[2]));
                if (hs.overflow != 0)
                    GDGS_LOG(2, "server: request %lld needs %lld pairs; run again with a "
                                "larger capacity", (long long)id, (long long)hs.num_pairs);
                const Next nx = core->finish_run(r, hs.overflow != 0, hs.num_pairs,
                                                 hs.converged != 0, cyc);
                if (nx == Next::Resume) {
                    const gdgs_status e = enqueue_resume(r);
                    if (e != GDGS_OK) fail(r, e);
                } else {
                    running[s] = -1;
                    if (nx == Next::Complete) {
                        complete(*r, r->cancelled ? GDGS_ERR_CANCELLED : GDGS_OK);
                        core->forget(id);
                    }
                }
            }
            for (int64_t id : core->take_rejected()) {
                gdgs::sched::Request* r = core->find(id);
                complete(*r, GDGS_ERR_BUDGET);
                core->forget(id);
                progress = true;
            }
            while (gdgs::sched::Request* r = core->admit(gdgs::steady_ns())) {
                progress = true;
                running[r->stream] = r->id;
                const gdgs_status e = enqueue_first(r);
                if (e != GDGS_OK) fail(r, e);
            }
            if (batched && batch_step()) progress = true;
            if (stop && core->waiting() == 0 && core->running() == 0 && !(batched && batch_busy()))
                break;
            if (progress) continue;
            if (core->running() > 0 || (batched && batch_busy())) {
                // device work in flight: poll its events again shortly
                lk.unlock();
                std::this_thread::yield();
                lk.lock();
            } else {
                const int64_t t = core->next_arrival();
                if (t == INT64_MAX)
                    wake.wait(lk);
                else
                    wake.wait_for(lk, std::chrono::nanoseconds(std::max<int64_t>(0, t - gdgs::steady_ns())));
            }
        }
    }
};

using namespace gdgs;

namespace {

#define SREQ(cond, ...)                       \
    do {                                      \
        if (!(cond)) {                        \
            set_error(__VA_ARGS__);           \
            return GDGS_ERR_INVALID_ARGUMENT; \
        }                                     \
    } while (0)

bool al4(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

}  // namespace

extern "C" {

int64_t gdgs_now_ns(void) { return steady_ns(); }

gdgs_status gdgs_server_create(const gdgs_scene* scene, const gdgs_server_params* params,
                               gdgs_server** out) {
    GDGS_TRACE("gdgs_server_create");
    clear_error();
    SREQ(scene && params && out, "scene, params or out is null");
    const int64_t K = scene->K;
    SREQ(K >= 0 && K < (int64_t)0xFFFFFFFFll, "K = %lld out of range", (long long)K);
    if (K > 0)
        SREQ(scene->mean && scene->log_scale && scene->quat && scene->opacity && scene->value &&
                 al4(scene->mean) && al4(scene->log_scale) && al4(scene->quat) &&
                 al4(scene->opacity) && al4(scene->value),
             "scene arrays must be non-null and 4-byte aligned");
    SREQ(params->streams >= 1 && params->streams <= 16, "streams = %d, must be 1..16",
         params->streams);
    SREQ(params->hbm_budget >= (1 << 20), "hbm_budget must be at least 1 MiB");
    SREQ((params->mg.flags & ~GDGS_MG_NEUMANN) == 0,
         "server solver flags must be 0 or GDGS_MG_NEUMANN");
    SREQ((params->flags & ~GDGS_SERVER_BATCHED) == 0, "unknown server flags 0x%x",
         params->flags);
    SREQ(!((params->flags & GDGS_SERVER_BATCHED) && (params->mg.flags & GDGS_MG_NEUMANN)),
         "batched solves take the Dirichlet problem only");
    MgPlan probe;
    if (mg_plan(64, 64, &params->mg, &probe) != GDGS_OK) return GDGS_ERR_INVALID_ARGUMENT;

    static std::atomic<uint64_t> uids{1};
    gdgs_server* s = new gdgs_server();
    s->uid = uids.fetch_add(1);
    s->scene = *scene;
    s->mg = params->mg;
    s->arena_bytes = (size_t)params->hbm_budget & ~(size_t)255;
    s->batched = (params->flags & GDGS_SERVER_BATCHED) != 0;
    for (int k = 0; k < kBatchMax; ++k) {
        s->ent_req[k] = -1;
        s->ent_state[k] = 0;
        s->ent_depth[k] = 0;
        s->ent_retire_at[k] = 0;
    }
    auto cleanup = [&](hipError_t e, const char* what) {
        set_error("%s: %s", what, hipGetErrorString(e));
        for (auto ev : s->events) (void)hipEventDestroy(ev);
        for (auto st : s->streams) (void)hipStreamDestroy(st);
        if (s->solver) (void)hipStreamDestroy(s->solver);
        if (s->host_stats) (void)hipHostFree(s->host_stats);
        if (s->ring) (void)hipHostFree(s->ring);
        if (s->btab) (void)hipFree(s->btab);
        if (s->arena) (void)hipFree(s->arena);
        delete s;
        return GDGS_ERR_HIP;
    };
    hipError_t e = hipGetDevice(&s->dev);
    if (e != hipSuccess) return cleanup(e, "hipGetDevice");
    e = hipMalloc(reinterpret_cast<void**>(&s->arena), s->arena_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        s->arena = nullptr;
        const gdgs_status r = cleanup(e, "allocating the memory budget");
        return r == GDGS_ERR_HIP ? GDGS_ERR_BUDGET : r;
    }
    e = hipHostMalloc(reinterpret_cast<void**>(&s->host_stats),
                      sizeof(gdgs_stats) * params->streams, hipHostMallocDefault);
    if (e != hipSuccess) {
        s->host_stats = nullptr;
        return cleanup(e, "hipHostMalloc");
    }
    for (int k = 0; k < params->streams; ++k) {
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) return cleanup(e, "hipStreamCreate");
        s->streams.push_back(st);
        hipEvent_t ev = nullptr;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return cleanup(e, "hipEventCreate");
        s->events.push_back(ev);
    }
    if (s->batched) {
        e = hipStreamCreateWithFlags(&s->solver, hipStreamNonBlocking);
        if (e != hipSuccess) return cleanup(e, "hipStreamCreate (solver)");
        e = hipMalloc(&s->btab, batch_table_bytes());
        if (e != hipSuccess) {
            s->btab = nullptr;
            return cleanup(e, "allocating the batch table");
        }
        e = hipHostMalloc(reinterpret_cast<void**>(&s->ring), sizeof(BatchRing),
                          hipHostMallocDefault);
        if (e != hipSuccess) {
            s->ring = nullptr;
            return cleanup(e, "hipHostMalloc (completion ring)");
        }
        std::memset(s->ring, 0, sizeof(BatchRing));
        if (batch_clear(s->btab, s->solver) != GDGS_OK)
            return cleanup(hipErrorLaunchFailure, "clearing the batch table");
    }
    s->running.assign(params->streams, -1);
    sched::Core::Config cfg;
    cfg.budget = s->arena_bytes;
    cfg.streams = params->streams;
    cfg.max_cycles = params->mg.max_cycles;
    cfg.resume_cycles = 2;
    cfg.initial_cap = std::max<int64_t>(1 << 16, 4 * K);
    cfg.slot_bytes = [s](int32_t W, int32_t H, int64_t cap) { return s->slot_bytes(W, H, cap); };
    s->core = new sched::Core(cfg);
    s->thread = std::thread([s] { s->loop(); });
    *out = s;
    GDGS_LOG(2, "server created: %zu-byte budget, %d front-half stream(s), %s solves",
             (size_t)s->arena_bytes, params->streams, s->batched ? "batched" : "per-request");
    return GDGS_OK;
}

gdgs_status gdgs_server_submit(gdgs_server* srv, const gdgs_request* req, int64_t* id) {
    GDGS_TRACE("gdgs_server_submit");
    clear_error();
    SREQ(srv && req && id, "server, request or id is null");
    const gdgs_camera& cam = req->cam;
    SREQ(cam.W >= 3 && cam.H >= 3 && cam.W / 16 < 65535 && cam.H / 16 < 65535,
         "image size %dx%d out of range", cam.W, cam.H);
    SREQ(cam.fx > 0 && cam.fy > 0, "focal lengths must be positive");
    SREQ(req->u && al4(req->u), "u is null or not 4-byte aligned");
    SREQ(!req->boundary || al4(req->boundary), "boundary is not 4-byte aligned");
    SREQ(!(req->boundary && (srv->mg.flags & GDGS_MG_NEUMANN)),
         "the Neumann problem takes no boundary data");
    SREQ(!req->u_init || al4(req->u_init), "u_init is not 4-byte aligned");
    std::lock_guard<std::mutex> g(srv->mu);
    SREQ(!srv->stop, "server is shutting down");
    if (srv->batched) {
        const MgPlan* pl = srv->plan(cam.W, cam.H, srv->mg.max_cycles, 0);
        SREQ(pl && batch_supported(*pl), "a %dx%d view cannot be solved batched", cam.W, cam.H);
    }
    const int64_t rid = srv->next_id++;
    const int64_t t = req->arrival_ns > 0 ? req->arrival_ns : steady_ns();
    if (!srv->core->submit(rid, req->tag, cam.W, cam.H, t)) {
        set_error("a %dx%d request needs more than the %zu-byte budget", cam.W, cam.H,
                  srv->arena_bytes);
        return GDGS_ERR_BUDGET;
    }
    srv->payload[rid] = Payload{cam, req->boundary, req->u, req->u_init};
    ++srv->submitted;
    *id = rid;
    srv->wake.notify_all();
    return GDGS_OK;
}

gdgs_status gdgs_server_poll(gdgs_server* srv, gdgs_completion* out, int32_t max, int32_t wait_us,
                             int32_t* n) {
    GDGS_TRACE("gdgs_server_poll");
    clear_error();
    SREQ(srv && n && (max == 0 || out) && max >= 0, "bad poll arguments");
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->done.empty() && wait_us > 0)
        srv->done_cv.wait_for(lk, std::chrono::microseconds(wait_us),
                              [&] { return !srv->done.empty(); });
    int32_t k = 0;
    while (k < max && !srv->done.empty()) {
        out[k++] = srv->done.front();
        srv->done.pop_front();
    }
    *n = k;
    return GDGS_OK;
}

gdgs_status gdgs_server_cancel(gdgs_server* srv, int64_t id) {
    GDGS_TRACE("gdgs_server_cancel");
    clear_error();
    SREQ(srv, "server is null");
    std::lock_guard<std::mutex> g(srv->mu);
    sched::Request* r = srv->core->find(id);
    SREQ(r && r->phase != sched::Phase::Done && !r->cancelled && srv->payload.count(id),
         "request %lld is unknown, finished or already cancelled", (long long)id);
    if (srv->core->cancel(id)) {
        srv->complete(*r, GDGS_ERR_CANCELLED);
        srv->core->forget(id);
    }
    srv->wake.notify_all();
    return GDGS_OK;
}

gdgs_status gdgs_server_query(gdgs_server* srv, gdgs_server_state* out) {
    GDGS_TRACE("gdgs_server_query");
    clear_error();
    SREQ(srv && out, "server or out is null");
    std::lock_guard<std::mutex> g(srv->mu);
    const sched::Arena& a = srv->core->pool().arena();
    out->budget_bytes = (int64_t)a.size();
    out->used_bytes = (int64_t)a.used();
    out->peak_bytes = (int64_t)a.peak();
    out->submitted = srv->submitted;
    out->completed = srv->completed;
    out->waiting = (int32_t)srv->core->waiting();
    out->running = srv->core->running();
    out->idle_slots = (int32_t)srv->core->pool().idle_count();
    out->streams = (int32_t)srv->streams.size();
    if (srv->fatal != GDGS_OK) {
        set_error("a request failed on the device (%d)", (int)srv->fatal);
        return srv->fatal;
    }
    return GDGS_OK;
}

gdgs_status gdgs_server_destroy(gdgs_server* srv) {
    GDGS_TRACE("gdgs_server_destroy");
    clear_error();
    if (!srv) return GDGS_OK;
    GDGS_LOG(2, "server destroyed");
    {
        std::lock_guard<std::mutex> g(srv->mu);
        srv->stop = true;
        std::vector<int64_t> ids;
        for (const auto& kv : srv->payload) ids.push_back(kv.first);
        for (int64_t id : ids) {
            sched::Request* r = srv->core->find(id);
            if (r && srv->core->cancel(id)) {
                srv->complete(*r, GDGS_ERR_CANCELLED);
                srv->core->forget(id);
            }
        }
        srv->wake.notify_all();
    }
    if (srv->thread.joinable()) srv->thread.join();
    gdgs_status st = GDGS_OK;
    for (auto s : srv->streams)
        if (hipStreamSynchronize(s) != hipSuccess) st = GDGS_ERR_HIP;
    if (srv->solver && hipStreamSynchronize(srv->solver) != hipSuccess) st = GDGS_ERR_HIP;
    for (auto ev : srv->events) (void)hipEventDestroy(ev);
    for (auto& r : srv->rounds) (void)hipEventDestroy(r.second);
    for (auto ev : srv->free_round_events) (void)hipEventDestroy(ev);
    for (auto s : srv->streams) (void)hipStreamDestroy(s);
    if (srv->solver) (void)hipStreamDestroy(srv->solver);
    if (srv->ring) (void)hipHostFree(srv->ring);
    if (srv->btab) (void)hipFree(srv->btab);
    if (srv->host_stats) (void)hipHostFree(srv->host_stats);
    if (srv->arena) (void)hipFree(srv->arena);
    delete srv->core;
    delete srv;
    if (st != GDGS_OK) set_error("a server stream failed while draining");
    return st;
}

}  // extern "C"
