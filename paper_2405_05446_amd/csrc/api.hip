// extern "C" entry points of libgdgs (declared in include/gdgs.h): argument
// validation on the host, workspace carving, and enqueueing of the HIP
// kernels of the individual steps on the caller's stream.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "graph.hpp"
#include "internal.hpp"

namespace gdgs {

namespace {
thread_local char g_err[512] = "";
}

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    GDGS_LOG(1, "%s", g_err);
}

int log_level() {
    static const int v = [] {
        const char* e = std::getenv("GDGS_LOG");
        if (!e || !*e) return 0;
        const int l = std::atoi(e);
        return l < 0 ? 0 : (l > 3 ? 3 : l);
    }();
    return v;
}

void log_msg(int level, const char* fmt, ...) {
    static const char* const names[4] = {"", "error", "info", "debug"};
    char line[640];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(line, sizeof(line), fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "gdgs[%s] %s\n", names[level < 0 ? 0 : (level > 3 ? 3 : level)], line);
}

void clear_error() { g_err[0] = '\0'; }

KernelTimer* kernel_timers() {
    static KernelTimer t[kMaxTimers];
    return t;
}

bool timer_events(const char* name, hipEvent_t* start, hipEvent_t* stop) {
    KernelTimer* ts = kernel_timers();
    for (int k = 0; k < kMaxTimers; ++k) {
        KernelTimer& t = ts[k];
        if (t.n <= 0 || std::strncmp(t.name, name, sizeof(t.name)) != 0) continue;
        const int i = t.next++;
        if (i >= t.n) return false;
        *start = t.starts[i];
        *stop = t.stops[i];
        return true;
    }
    return false;
}

int timer_repeats(const char* name) {
    const KernelTimer* ts = kernel_timers();
    for (int k = 0; k < kMaxTimers; ++k)
        if (ts[k].n > 0 && std::strncmp(ts[k].name, name, sizeof(ts[k].name)) == 0)
            return ts[k].repeats;
    return 1;
}

namespace {
struct GraphCache {
    std::mutex mu;
    std::list<std::pair<std::string, hipGraphExec_t>> lru;
    static constexpr size_t kMax = 128;

    hipGraphExec_t find(const std::string& k) {
        std::lock_guard<std::mutex> g(mu);
        for (auto it = lru.begin(); it != lru.end(); ++it) {
            if (it->first == k) {
                lru.splice(lru.begin(), lru, it);
                return lru.front().second;
            }
        }
        return nullptr;
    }
    void put(const std::string& k, hipGraphExec_t e) {
        std::lock_guard<std::mutex> g(mu);
        lru.emplace_front(k, e);
        while (lru.size() > kMax) {
            (void)hipGraphExecDestroy(lru.back().second);
            lru.pop_back();
        }
    }
    void clear() {
        std::lock_guard<std::mutex> g(mu);
        for (auto& kv : lru) (void)hipGraphExecDestroy(kv.second);
        lru.clear();
    }
};

GraphCache& graph_cache_impl() {
    static GraphCache* c = new GraphCache();  // never destroyed: outlives static teardown
    return *c;
}

}  // namespace

hipGraphExec_t graph_find(const std::string& key) { return graph_cache_impl().find(key); }
void graph_put(const std::string& key, hipGraphExec_t exec) { graph_cache_impl().put(key, exec); }

int& graphs_flag() {
    static int v = [] {
        const char* e = std::getenv("GDGS_GRAPHS");
        return (e && e[0] == '0') ? 0 : 1;
    }();
    return v;
}

int& channel_streams_flag() {
    static int v = 1;
    return v;
}

hipStream_t capture_stream(int dev) {
    thread_local std::map<int, hipStream_t> streams;
    auto it = streams.find(dev);
    if (it != streams.end()) return it->second;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    streams[dev] = s;
    return s;
}


bool channel_streams(hipStream_t st, ChannelStreams* out) {
    static const bool enabled = [] {
        const char* e = std::getenv("GDGS_CHANNEL_STREAMS");
        return !(e && e[0] == '0');
    }();
    if (!enabled) return false;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    thread_local std::map<std::pair<int, hipStream_t>, ChannelStreams> table;
    const auto k = std::make_pair(dev, st);
    auto it = table.find(k);
    if (it != table.end()) {
        *out = it->second;
        return true;
    }
    ChannelStreams c{};
    bool ok = true;
    for (int i = 0; i < 2 && ok; ++i)
        ok = hipStreamCreateWithFlags(&c.aux[i], hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&c.fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < 2 && ok; ++i)
        ok = hipEventCreateWithFlags(&c.join[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        return false;
    }
    table.emplace(k, c);
    *out = c;
    return true;
}

bool timer_active(const char* name) {
    const KernelTimer* ts = kernel_timers();
    for (int k = 0; k < kMaxTimers; ++k)
        if (ts[k].n > 0 && std::strncmp(ts[k].name, name, sizeof(ts[k].name)) == 0) return true;
    return false;
}

void reset_timers() {
    for (int k = 0; k < kMaxTimers; ++k) kernel_timers()[k].next = 0;
}

namespace {

bool aligned4(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

#define REQUIRE(cond, ...)                   \
    do {                                     \
        if (!(cond)) {                       \
            set_error(__VA_ARGS__);          \
            return GDGS_ERR_INVALID_ARGUMENT; \
        }                                    \
    } while (0)

#define REQUIRE_PTR(p)                                                          \
    REQUIRE((p) != nullptr && aligned4(p), "%s is null or not 4-byte aligned", #p)

gdgs_status check_size(int32_t W, int32_t H) {
    REQUIRE(W >= 3 && H >= 3, "image size %dx%d: both sides must be >= 3", W, H);
    REQUIRE((int64_t)tiles_x(W) < 65536 && (int64_t)tiles_y(H) < 65536,
            "image size %dx%d too large for 16-bit tile indices", W, H);
    return GDGS_OK;
}

gdgs_status check_proj(const gdgs_proj* p) {
    REQUIRE(p != nullptr, "proj is null");
    REQUIRE_PTR(p->mean2d);
    REQUIRE_PTR(p->conic);
    REQUIRE_PTR(p->depth);
    REQUIRE_PTR(p->rect);
    REQUIRE_PTR(p->count);
    return GDGS_OK;
}

gdgs_status check_bins(const gdgs_bins* b, int64_t K) {
    REQUIRE(b != nullptr, "bins is null");
    REQUIRE(b->capacity >= 1 && b->capacity < (int64_t)0xFFFFFFFFll,
            "pair capacity %lld must be in [1, 2^32 - 1)", (long long)b->capacity);
    REQUIRE_PTR(b->tile_of_pair);
    REQUIRE_PTR(b->splat_of_pair);
    REQUIRE_PTR(b->ranges);
    REQUIRE(b->num_pairs != nullptr && (reinterpret_cast<uintptr_t>(b->num_pairs) & 7u) == 0,
            "bins.num_pairs is null or not 8-byte aligned");
    if (K > 0) REQUIRE_PTR(b->order);
    return GDGS_OK;
}

gdgs_status check_ws(void* ws, size_t have, size_t need) {
    if (need > have || (need > 0 && ws == nullptr)) {
        set_error("workspace of %zu bytes is smaller than the %zu bytes required", have, need);
        return GDGS_ERR_WORKSPACE;
    }
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) {
        set_error("workspace must be 256-byte aligned");
        return GDGS_ERR_WORKSPACE;
    }
    return GDGS_OK;
}

#define TRY(expr)                          \
    do {                                   \
        gdgs_status s_ = (expr);           \
        if (s_ != GDGS_OK) return s_;      \
    } while (0)

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace


size_t render_layout(int64_t K, int W, int H, int64_t cap, const MgPlan& plan, void* ws,
                     RenderWs* out) {
    Carver c(ws);
    RenderWs r{};
    const int64_t Kp = K > 0 ? K : 1;
    r.proj.mean2d = c.take<float>(2 * Kp);
    r.proj.conic = c.take<float>(3 * Kp);
    r.proj.depth = c.take<float>(Kp);
    r.proj.rect = c.take<uint32_t>(2 * Kp);
    r.proj.count = c.take<uint32_t>(Kp);
    r.bins.capacity = cap;
    r.bins.tile_of_pair = c.take<uint32_t>(cap);
    r.bins.splat_of_pair = c.take<uint32_t>(cap);
    r.bins.order = c.take<uint32_t>(Kp);
    r.bins.ranges = c.take<uint32_t>(2 * (size_t)tiles_x(W) * tiles_y(H));
    r.bins.num_pairs = c.take<int64_t>(1);
    r.bins.tile_order = c.take<uint32_t>((size_t)tiles_x(W) * tiles_y(H));
    r.grad = c.take<float>((size_t)6 * W * H);
    r.bin_ws = c.take<char>(bin_ws_layout(K, cap, num_tiles(W, H), nullptr, nullptr));
    r.raster_ws = c.take<char>(raster_ws_bytes(K));
    r.poisson_ws = c.take<char>(poisson_ws_bytes(plan, W, H));
    if (out) *out = r;
    return c.off + 256;
}

namespace {
__global__ void k_render_stats(const int64_t* num_pairs, int64_t cap, gdgs_stats* stats) {
    if (threadIdx.x == 0) {
        const int64_t p = *num_pairs;
        stats->num_pairs = p;
        stats->overflow = p > cap ? 1 : 0;
    }
}
}  // namespace

gdgs_status launch_render_stats(const int64_t* num_pairs, int64_t cap, gdgs_stats* stats,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_render_stats, dim3(1), dim3(64), 0, st, num_pairs, cap, stats);
    GDGS_LAUNCH_CHECK();
    return GDGS_OK;
}

void add_plan(KeyBuilder& kb, const MgPlan& p) {
    kb.add(p.levels).add(p.lc).add(p.pre).add(p.post).add(p.max_cycles).add(p.coarse_sweeps)
        .add(p.omega).add(p.sw).add(p.tol).add(p.warm).add(p.resume).add(p.neumann).add(p.fmg).add(p.stop_eta)
        .add(p.lds_bytes);
    for (int l = 0; l < p.levels; ++l) kb.add(p.n[l]).add(p.m[l]).add(p.pitch[l]);
}

void add_proj(KeyBuilder& kb, const gdgs_proj& p) {
    kb.add(p.mean2d).add(p.conic).add(p.depth).add(p.rect).add(p.count);
}

void add_bins(KeyBuilder& kb, const gdgs_bins& b) {
    kb.add(b.capacity).add(b.tile_of_pair).add(b.splat_of_pair).add(b.order).add(b.ranges)
        .add(b.num_pairs).add(b.tile_order);
}

}  // namespace gdgs

using namespace gdgs;

extern "C" {

const char* gdgs_status_string(gdgs_status s) {
    switch (s) {
        case GDGS_OK: return "ok";
        case GDGS_ERR_INVALID_ARGUMENT: return "invalid argument";
        case GDGS_ERR_CAPACITY: return "pair capacity exceeded";
        case GDGS_ERR_WORKSPACE: return "workspace too small";
        case GDGS_ERR_BUDGET: return "memory budget exceeded";
        case GDGS_ERR_HIP: return "HIP runtime error";
        case GDGS_ERR_UNSUPPORTED: return "unsupported";
        case GDGS_ERR_NOT_READY: return "not ready";
        case GDGS_ERR_CANCELLED: return "cancelled";
    }
    return "unknown status";
}

const char* gdgs_last_error(void) { return g_err; }

const char* gdgs_version(void) { return "gdgs 0.1 gfx950"; }

void gdgs_set_graphs(int enable) { graphs_flag() = enable ? 1 : 0; }

void gdgs_set_channel_streams(int enable) { channel_streams_flag() = enable ? 1 : 0; }

void gdgs_clear_graphs(void) { graph_cache_impl().clear(); }

gdgs_status gdgs_set_kernel_timer(const char* kernel, void** start_events, void** stop_events,
                                  int n) {
    GDGS_TRACE("gdgs_set_kernel_timer");
    clear_error();
    KernelTimer* ts = kernel_timers();
    if (kernel == nullptr) {
        for (int k = 0; k < kMaxTimers; ++k) ts[k] = KernelTimer();
        return GDGS_OK;
    }
    REQUIRE(std::strlen(kernel) < sizeof(ts[0].name), "kernel name too long");
    int slot = -1;
    for (int k = 0; k < kMaxTimers; ++k)
        if (ts[k].n > 0 && std::strncmp(ts[k].name, kernel, sizeof(ts[k].name)) == 0) slot = k;
    if (n <= 0) {
        if (slot >= 0) ts[slot] = KernelTimer();
        return GDGS_OK;
    }
    REQUIRE(start_events != nullptr && stop_events != nullptr, "event arrays are null");
    for (int k = 0; slot < 0 && k < kMaxTimers; ++k)
        if (ts[k].n <= 0) slot = k;
    REQUIRE(slot >= 0, "at most %d kernel timers", kMaxTimers);
    KernelTimer& t = ts[slot];
    t = KernelTimer();
    std::strncpy(t.name, kernel, sizeof(t.name) - 1);
    t.starts = reinterpret_cast<hipEvent_t*>(start_events);
    t.stops = reinterpret_cast<hipEvent_t*>(stop_events);
    t.n = n;
    return GDGS_OK;
}

gdgs_status gdgs_set_kernel_timer_repeats(const char* kernel, int repeats) {
    GDGS_TRACE("gdgs_set_kernel_timer_repeats");
    clear_error();
    REQUIRE(kernel != nullptr, "kernel name is null");
    REQUIRE(repeats >= 1 && repeats <= 64, "repeats %d outside [1, 64]", repeats);
    REQUIRE(std::strcmp(kernel, "mg_post_fine") == 0 || std::strcmp(kernel, "mg_post_coarse") == 0,
            "repeats apply to the multigrid post passes only (\"mg_post_fine\", "
            "\"mg_post_coarse\")");
    KernelTimer* ts = kernel_timers();
    for (int k = 0; k < kMaxTimers; ++k)
        if (ts[k].n > 0 && std::strncmp(ts[k].name, kernel, sizeof(ts[k].name)) == 0) {
            ts[k].repeats = repeats;
            return GDGS_OK;
        }
    set_error("timer \"%s\" is not armed", kernel);
    return GDGS_ERR_INVALID_ARGUMENT;
}

void gdgs_rewind_kernel_timers(void) { reset_timers(); }

int gdgs_kernel_timer_count(const char* kernel) {
    if (kernel == nullptr) return 0;
    const KernelTimer* ts = kernel_timers();
    for (int k = 0; k < kMaxTimers; ++k)
        if (ts[k].n > 0 && std::strncmp(ts[k].name, kernel, sizeof(ts[k].name)) == 0)
            return ts[k].next < ts[k].n ? ts[k].next : ts[k].n;
    return 0;
}

gdgs_status gdgs_bin_sort_workspace_size(int64_t K, int32_t W, int32_t H, int64_t pair_capacity,
                                         size_t* bytes) {
    GDGS_TRACE("gdgs_bin_sort_workspace_size");
    clear_error();
    REQUIRE(bytes != nullptr, "bytes is null");
    REQUIRE(K >= 0 && K < (int64_t)0xFFFFFFFFll, "K = %lld out of range", (long long)K);
    TRY(check_size(W, H));
    REQUIRE(pair_capacity >= 1 && pair_capacity < (int64_t)0xFFFFFFFFll,
            "pair capacity %lld out of range", (long long)pair_capacity);
    *bytes = bin_ws_layout(K, pair_capacity, num_tiles(W, H), nullptr, nullptr);
    return GDGS_OK;
}

gdgs_status gdgs_raster_workspace_size(int64_t K, size_t* bytes) {
    GDGS_TRACE("gdgs_raster_workspace_size");
    clear_error();
    REQUIRE(bytes != nullptr, "bytes is null");
    REQUIRE(K >= 0 && K < (int64_t)0xFFFFFFFFll, "K = %lld out of range", (long long)K);
    *bytes = raster_ws_bytes(K);
    return GDGS_OK;
}

gdgs_status gdgs_poisson_workspace_size(int32_t W, int32_t H, const gdgs_mg_params* mg,
                                        size_t* bytes) {
    GDGS_TRACE("gdgs_poisson_workspace_size");
    clear_error();
    REQUIRE(bytes != nullptr, "bytes is null");
    TRY(check_size(W, H));
    MgPlan plan;
    TRY(mg_plan(W, H, mg, &plan));
    *bytes = poisson_ws_bytes(plan, W, H);
    return GDGS_OK;
}

gdgs_status gdgs_workspace_size(int64_t K, int32_t W, int32_t H, int64_t pair_capacity,
                                const gdgs_mg_params* mg, size_t* bytes) {
    GDGS_TRACE("gdgs_workspace_size");
    clear_error();
    REQUIRE(bytes != nullptr, "bytes is null");
    REQUIRE(K >= 0 && K < (int64_t)0xFFFFFFFFll, "K = %lld out of range", (long long)K);
    TRY(check_size(W, H));
    REQUIRE(pair_capacity >= 1 && pair_capacity < (int64_t)0xFFFFFFFFll,
            "pair capacity %lld out of range", (long long)pair_capacity);
    MgPlan plan;
    TRY(mg_plan(W, H, mg, &plan));
    *bytes = render_layout(K, W, H, pair_capacity, plan, nullptr, nullptr);
    return GDGS_OK;
}

gdgs_status gdgs_raster_backward_workspace_size(int64_t K, int64_t pair_capacity, size_t* bytes) {
    GDGS_TRACE("gdgs_raster_backward_workspace_size");
    clear_error();
    REQUIRE(bytes != nullptr, "bytes is null");
    REQUIRE(K >= 0 && K < (int64_t)0xFFFFFFFFll, "K = %lld out of range", (long long)K);
    REQUIRE(pair_capacity >= 1 && pair_capacity < (int64_t)0xFFFFFFFFll,
            "pair capacity %lld out of range", (long long)pair_capacity);
    *bytes = raster_bwd_ws_bytes(K, pair_capacity);
    return GDGS_OK;
}

gdgs_status gdgs_project(const gdgs_scene* scene, const gdgs_camera* cam, const gdgs_proj* out,
                         void* stream) {
    GDGS_TRACE("gdgs_project");
    clear_error();
    REQUIRE(scene != nullptr && cam != nullptr, "scene or camera is null");
    REQUIRE(scene->K >= 0 && scene->K < (int64_t)0xFFFFFFFFll, "K = %lld out of range",
            (long long)scene->K);
    TRY(check_size(cam->W, cam->H));
    REQUIRE(cam->fx > 0 && cam->fy > 0, "focal lengths must be positive (fx %g, fy %g)", cam->fx,
            cam->fy);
    if (scene->K == 0) return GDGS_OK;
    REQUIRE_PTR(scene->mean);
    REQUIRE_PTR(scene->log_scale);
    REQUIRE_PTR(scene->quat);
    TRY(check_proj(out));
    return launch_project(*scene, *cam, *out, as_stream(stream));
}

gdgs_status gdgs_threshold(float* x, int64_t n, float t, uint64_t* nonzero_dev, void* stream) {
    GDGS_TRACE("gdgs_threshold");
    clear_error();
    REQUIRE(n >= 0, "n must be >= 0");
    REQUIRE(t >= 0.f, "threshold must be >= 0");
    if (n > 0) REQUIRE_PTR(x);
    if (nonzero_dev)
        REQUIRE((reinterpret_cast<uintptr_t>(nonzero_dev) & 7u) == 0,
                "nonzero_dev is not 8-byte aligned");
    return launch_threshold(x, n, t, reinterpret_cast<unsigned long long*>(nonzero_dev),
                            as_stream(stream));
}

gdgs_status gdgs_image_loss_workspace_size(int32_t W, int32_t H, size_t* bytes) {
    GDGS_TRACE("gdgs_image_loss_workspace_size");
    clear_error();
    REQUIRE(bytes != nullptr, "bytes is null");
    TRY(check_size(W, H));
    *bytes = loss_ws_bytes(W, H);
    return GDGS_OK;
}

gdgs_status gdgs_image_loss(const float* c, const float* im, int32_t W, int32_t H, double lam,
                            double beta, double* loss_dev, float* dc, void* ws, size_t ws_bytes,
                            void* stream) {
    GDGS_TRACE("gdgs_image_loss");
    clear_error();
    TRY(check_size(W, H));
    REQUIRE_PTR(c);
    REQUIRE_PTR(im);
    if (dc) REQUIRE_PTR(dc);
    REQUIRE(loss_dev != nullptr && (reinterpret_cast<uintptr_t>(loss_dev) & 7u) == 0,
            "loss_dev is null or not 8-byte aligned");
    REQUIRE(lam >= 0.0 && lam <= 1.0 && beta >= 0.0, "need 0 <= lam <= 1 and beta >= 0");
    TRY(check_ws(ws, ws_bytes, loss_ws_bytes(W, H)));
    return launch_image_loss(c, im, W, H, lam, beta, loss_dev, dc, ws, as_stream(stream));
}

gdgs_status gdgs_adam_step(float* param, const float* grad, float* m, float* v, int64_t n,
                           int32_t t, float lr, float beta1, float beta2, float eps, float lo,
                           float hi, void* stream) {
    GDGS_TRACE("gdgs_adam_step");
    clear_error();
    REQUIRE(n >= 0, "n must be >= 0");
    REQUIRE(t >= 1, "step t must be >= 1");
    REQUIRE(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f,
            "invalid Adam constants");
    if (n > 0) {
        REQUIRE_PTR(param);
        REQUIRE_PTR(grad);
        REQUIRE_PTR(m);
        REQUIRE_PTR(v);
    }
    return launch_adam(param, grad, m, v, n, t, lr, beta1, beta2, eps, lo, hi,
                       as_stream(stream));
}

gdgs_status gdgs_project_backward(const gdgs_scene* scene, const gdgs_camera* cam,
                                  const float* dmean2d, const float* dconic, float* dmean,
                                  float* dlog_scale, float* dquat, void* stream) {
    GDGS_TRACE("gdgs_project_backward");
    clear_error();
    REQUIRE(scene != nullptr && cam != nullptr, "scene or camera is null");
    const int64_t K = scene->K;
    REQUIRE(K >= 0 && K < (int64_t)0xFFFFFFFFll, "K = %lld out of range", (long long)K);
    REQUIRE(cam->fx > 0 && cam->fy > 0, "focal lengths must be positive");
    if (K == 0) return GDGS_OK;
    REQUIRE_PTR(scene->mean);
    REQUIRE_PTR(scene->log_scale);
    REQUIRE_PTR(scene->quat);
    REQUIRE_PTR(dmean2d);
    REQUIRE_PTR(dconic);
    REQUIRE_PTR(dmean);
    REQUIRE_PTR(dlog_scale);
    REQUIRE_PTR(dquat);
    return launch_project_backward(*scene, *cam, dmean2d, dconic, dmean, dlog_scale, dquat,
                                   as_stream(stream));
}

gdgs_status gdgs_project_2d(const float* mean2d, const float* conic, const float* depth,
                            int64_t K, int32_t W, int32_t H, const gdgs_proj* out, void* stream) {
    GDGS_TRACE("gdgs_project_2d");
    clear_error();
    REQUIRE(K >= 0 && K < (int64_t)0xFFFFFFFFll, "K = %lld out of range", (long long)K);
    TRY(check_size(W, H));
    if (K == 0) return GDGS_OK;
    REQUIRE_PTR(mean2d);
    REQUIRE_PTR(conic);
    REQUIRE_PTR(depth);
    TRY(check_proj(out));
    return launch_project_2d(mean2d, conic, depth, K, W, H, *out, as_stream(stream));
}

gdgs_status gdgs_bin_sort(const gdgs_proj* proj, int64_t K, int32_t W, int32_t H,
                          const gdgs_bins* bins, void* ws, size_t ws_bytes, void* stream) {
    GDGS_TRACE("gdgs_bin_sort");
    clear_error();
    REQUIRE(K >= 0 && K < (int64_t)0xFFFFFFFFll, "K = %lld out of range", (long long)K);
    TRY(check_size(W, H));
    if (K > 0) TRY(check_proj(proj));
    TRY(check_bins(bins, K));
    TRY(check_ws(ws, ws_bytes,
                 bin_ws_layout(K, bins->capacity, num_tiles(W, H), nullptr, nullptr)));
    BinWs b;
    bin_ws_layout(K, bins->capacity, num_tiles(W, H), ws, &b);
    gdgs_proj p = K > 0 ? *proj : gdgs_proj{};
    const gdgs_bins bb = *bins;
    KeyBuilder kb;
    kb.tag("bin_sort").add(K).add(W).add(H).add(ws);
    add_proj(kb, p);
    add_bins(kb, bb);
    return with_graph(kb, as_stream(stream),
                      [&](hipStream_t s) { return launch_bin_sort(p, K, W, H, bb, b, s); });
}

static gdgs_status raster_common(const gdgs_proj* proj, const float* opacity,
                                 const float* value, int64_t K, const gdgs_bins* bins, int32_t W,
                                 int32_t H, float* out, void* ws, size_t ws_bytes, void* stream,
                                 int nch, float thr = -1.f, uint64_t* nonzero = nullptr) {
    clear_error();
    if (nonzero)
        REQUIRE((reinterpret_cast<uintptr_t>(nonzero) & 7u) == 0,
                "nonzero is not 8-byte aligned");
    REQUIRE(K >= 0 && K < (int64_t)0xFFFFFFFFll, "K = %lld out of range", (long long)K);
    TRY(check_size(W, H));
    REQUIRE_PTR(out);
    if (K > 0) {
        TRY(check_proj(proj));
        REQUIRE_PTR(opacity);
        REQUIRE_PTR(value);
    }
    TRY(check_bins(bins, K));
    TRY(check_ws(ws, ws_bytes, raster_ws_bytes(K)));
    gdgs_proj p = K > 0 ? *proj : gdgs_proj{};
    const gdgs_bins bb = *bins;
    KeyBuilder kb;
    kb.tag("raster").add(nch).add(K).add(W).add(H).add(ws).add(opacity).add(value).add(out)
        .add(thr).add(nonzero);
    add_proj(kb, p);
    add_bins(kb, bb);
    return with_graph(
        kb, as_stream(stream),
        [&](hipStream_t s) {
            return launch_raster(p, opacity, value, K, bb, W, H, out, ws, s, nch, thr,
                                 reinterpret_cast<unsigned long long*>(nonzero));
        },
        {"raster"});
}

gdgs_status gdgs_raster_grad(const gdgs_proj* proj, const float* opacity, const float* value,
                             int64_t K, const gdgs_bins* bins, int32_t W, int32_t H, float* grad,
                             void* ws, size_t ws_bytes, void* stream) {
    GDGS_TRACE("gdgs_raster_grad");
    return raster_common(proj, opacity, value, K, bins, W, H, grad, ws, ws_bytes, stream, 6);
}

gdgs_status gdgs_raster_laplacian(const gdgs_proj* proj, const float* opacity, const float* lap,
                                  int64_t K, const gdgs_bins* bins, int32_t W, int32_t H,
                                  float* rho, void* ws, size_t ws_bytes, void* stream) {
    GDGS_TRACE("gdgs_raster_laplacian");
    return raster_common(proj, opacity, lap, K, bins, W, H, rho, ws, ws_bytes, stream, 3);
}

gdgs_status gdgs_raster_laplacian_threshold(const gdgs_proj* proj, const float* opacity,
                                            const float* lap, int64_t K, const gdgs_bins* bins,
                                            int32_t W, int32_t H, float threshold, float* rho,
                                            uint64_t* nonzero, void* ws, size_t ws_bytes,
                                            void* stream) {
    GDGS_TRACE("gdgs_raster_laplacian_threshold");
    if (!(threshold >= 0.f)) {
        clear_error();
        set_error("threshold %g must be >= 0", (double)threshold);
        return GDGS_ERR_INVALID_ARGUMENT;
    }
    return raster_common(proj, opacity, lap, K, bins, W, H, rho, ws, ws_bytes, stream, 3,
                         threshold, nonzero);
}

gdgs_status gdgs_raster_count(const gdgs_proj* proj, const float* opacity, const float* value,
                              int64_t K, const gdgs_bins* bins, int32_t W, int32_t H,
                              uint64_t* counts, void* ws, size_t ws_bytes, void* stream) {
    GDGS_TRACE("gdgs_raster_count");
    clear_error();
    REQUIRE(K >= 0 && K < (int64_t)0xFFFFFFFFll, "K = %lld out of range", (long long)K);
    TRY(check_size(W, H));
    REQUIRE(counts != nullptr && (reinterpret_cast<uintptr_t>(counts) & 7u) == 0,
            "counts is null or not 8-byte aligned");
    if (K > 0) {
        TRY(check_proj(proj));
        REQUIRE_PTR(opacity);
        REQUIRE_PTR(value);
    }
    TRY(check_bins(bins, K));
    TRY(check_ws(ws, ws_bytes, raster_ws_bytes(K)));
    gdgs_proj p = K > 0 ? *proj : gdgs_proj{};
    return launch_raster_count(p, opacity, value, K, *bins, W, H,
                               reinterpret_cast<unsigned long long*>(counts), ws,
                               as_stream(stream));
}

static gdgs_status poisson_common(const float* grad, const float* rho, const float* boundary,
                                  int32_t W, int32_t H, const gdgs_mg_params* mg, float* u,
                                  gdgs_stats* stats_dev, void* ws, size_t ws_bytes,
                                  void* stream) {
    TRY(check_size(W, H));
    REQUIRE_PTR(u);
    if (boundary) REQUIRE_PTR(boundary);
    if (stats_dev) REQUIRE((reinterpret_cast<uintptr_t>(stats_dev) & 7u) == 0,
                           "stats_dev not 8-byte aligned");
    MgPlan plan;
    TRY(mg_plan(W, H, mg, &plan));
    REQUIRE(!(plan.neumann && boundary), "the Neumann problem takes no boundary data");
    TRY(check_ws(ws, ws_bytes, poisson_ws_bytes(plan, W, H)));
    KeyBuilder kb;
    kb.tag("poisson").add(grad).add(rho).add(boundary).add(W).add(H).add(u).add(stats_dev).add(ws);
    add_plan(kb, plan);
    // the solve caches its own graph segments (one per colour channel)
    return launch_poisson(grad, rho, boundary, W, H, plan, u, stats_dev, ws, as_stream(stream),
                          &kb);
}

gdgs_status gdgs_poisson_solve(const float* grad, const float* boundary, int32_t W, int32_t H,
                               const gdgs_mg_params* mg, float* u, gdgs_stats* stats_dev,
                               void* ws, size_t ws_bytes, void* stream) {
    GDGS_TRACE("gdgs_poisson_solve");
    clear_error();
    REQUIRE_PTR(grad);
    return poisson_common(grad, nullptr, boundary, W, H, mg, u, stats_dev, ws, ws_bytes, stream);
}

gdgs_status gdgs_poisson_solve_rhs(const float* rho, const float* boundary, int32_t W, int32_t H,
                                   const gdgs_mg_params* mg, float* u, gdgs_stats* stats_dev,
                                   void* ws, size_t ws_bytes, void* stream) {
    GDGS_TRACE("gdgs_poisson_solve_rhs");
    clear_error();
    REQUIRE_PTR(rho);
    return poisson_common(nullptr, rho, boundary, W, H, mg, u, stats_dev, ws, ws_bytes, stream);
}

// nch 6: gradient splats (composite, divergence, solve); nch 3: Laplacian
// splats (the composite is the right-hand side).
// sparse (nch 3): the hard threshold thr >= 0 of Eq. 24 fused into the
// composite (kept values counted into *nonzero), and the solve's set-up skips
// tiles without splats.
static gdgs_status render_common(const gdgs_scene* scene, const gdgs_camera* cam,
                                 const float* boundary, const gdgs_mg_params* mg,
                                 int64_t pair_capacity, float* u, gdgs_stats* stats_dev,
                                 int sync_stats, void* ws, size_t ws_bytes, void* stream, int nch,
                                 bool sparse = false, float thr = -1.f,
                                 unsigned long long* nonzero = nullptr) {
    clear_error();
    if (sparse) {
        REQUIRE(nch == 3, "the sparse render takes Laplacian splats");
        REQUIRE(thr >= 0.f, "threshold %g must be >= 0", (double)thr);
        if (nonzero)
            REQUIRE((reinterpret_cast<uintptr_t>(nonzero) & 7u) == 0,
                    "nonzero is not 8-byte aligned");
    }
    REQUIRE(scene != nullptr && cam != nullptr, "scene or camera is null");
    const int64_t K = scene->K;
    REQUIRE(K >= 0 && K < (int64_t)0xFFFFFFFFll, "K = %lld out of range", (long long)K);
    TRY(check_size(cam->W, cam->H));
    REQUIRE(cam->fx > 0 && cam->fy > 0, "focal lengths must be positive");
    REQUIRE(pair_capacity >= 1 && pair_capacity < (int64_t)0xFFFFFFFFll,
            "pair capacity %lld out of range", (long long)pair_capacity);
    REQUIRE_PTR(u);
    REQUIRE(stats_dev != nullptr && (reinterpret_cast<uintptr_t>(stats_dev) & 7u) == 0,
            "stats_dev is null or not 8-byte aligned");
    if (boundary) REQUIRE_PTR(boundary);
    if (K > 0) {
        REQUIRE_PTR(scene->mean);
        REQUIRE_PTR(scene->log_scale);
        REQUIRE_PTR(scene->quat);
        REQUIRE_PTR(scene->opacity);
        REQUIRE_PTR(scene->value);
    }
    const int W = cam->W, H = cam->H;
    MgPlan plan;
    TRY(mg_plan(W, H, mg, &plan));
    REQUIRE(!(plan.neumann && boundary), "the Neumann problem takes no boundary data");
    TRY(check_ws(ws, ws_bytes, render_layout(K, W, H, pair_capacity, plan, nullptr, nullptr)));
    RenderWs r;
    render_layout(K, W, H, pair_capacity, plan, ws, &r);
    hipStream_t st = as_stream(stream);
    // the projection takes the camera by value and is launched directly; the
    // rest depends only on sizes and buffers and is replayed as one graph
    if (K > 0) TRY(launch_project(*scene, *cam, r.proj, st));
    BinWs b;
    bin_ws_layout(K, pair_capacity, num_tiles(W, H), r.bin_ws, &b);
    const gdgs_scene sc = *scene;
    KeyBuilder kb;
    kb.tag("render").add(nch).add(K).add(W).add(H).add(pair_capacity).add(ws).add(sc.opacity)
        .add(sc.value).add(boundary).add(u).add(stats_dev).add(sparse).add(thr).add(nonzero);
    add_plan(kb, plan);
    KeyBuilder kr = kb;
    kr.tag("bin+raster");
    TRY(with_graph(
        kr, st,
        [&](hipStream_t s) -> gdgs_status {
            TRY(launch_bin_sort(r.proj, K, W, H, r.bins, b, s));
            return launch_raster(r.proj, sc.opacity, sc.value, K, r.bins, W, H, r.grad,
                                 r.raster_ws, s, nch, sparse ? thr : -1.f,
                                 sparse ? nonzero : nullptr);
        },
        {"raster"}));
    // the Laplacian composite (first three planes of the gradient buffer) is rho
    TRY(launch_poisson(nch == 6 ? r.grad : nullptr, nch == 6 ? nullptr : r.grad, boundary, W, H,
                       plan, u, stats_dev, r.poisson_ws, st, &kb, true,
                       sparse ? r.bins.ranges : nullptr));
    TRY(launch_render_stats(r.bins.num_pairs, pair_capacity, stats_dev, st));
    if (sync_stats) {
        GDGS_HIP_TRY(hipStreamSynchronize(st));
        gdgs_stats h;
        GDGS_HIP_TRY(hipMemcpy(&h, stats_dev, sizeof(h), hipMemcpyDeviceToHost));
        if (h.overflow) {
            set_error("render needed %lld pairs, capacity is %lld", (long long)h.num_pairs,
                      (long long)pair_capacity);
            return GDGS_ERR_CAPACITY;
        }
    }
    return GDGS_OK;
}

gdgs_status gdgs_render(const gdgs_scene* scene, const gdgs_camera* cam, const float* boundary,
                        const gdgs_mg_params* mg, int64_t pair_capacity, float* u,
                        gdgs_stats* stats_dev, int sync_stats, void* ws, size_t ws_bytes,
                        void* stream) {
    GDGS_TRACE("gdgs_render");
    return render_common(scene, cam, boundary, mg, pair_capacity, u, stats_dev, sync_stats, ws,
                         ws_bytes, stream, 6);
}

gdgs_status gdgs_render_laplacian(const gdgs_scene* scene, const gdgs_camera* cam,
                                  const float* boundary, const gdgs_mg_params* mg,
                                  int64_t pair_capacity, float* u, gdgs_stats* stats_dev,
                                  int sync_stats, void* ws, size_t ws_bytes, void* stream) {
    GDGS_TRACE("gdgs_render_laplacian");
    return render_common(scene, cam, boundary, mg, pair_capacity, u, stats_dev, sync_stats, ws,
                         ws_bytes, stream, 3);
}

gdgs_status gdgs_render_laplacian_sparse(const gdgs_scene* scene, const gdgs_camera* cam,
                                         const float* boundary, const gdgs_mg_params* mg,
                                         int64_t pair_capacity, float threshold, float* u,
                                         gdgs_stats* stats_dev, uint64_t* nonzero,
                                         int sync_stats, void* ws, size_t ws_bytes,
                                         void* stream) {
    GDGS_TRACE("gdgs_render_laplacian_sparse");
    return render_common(scene, cam, boundary, mg, pair_capacity, u, stats_dev, sync_stats, ws,
                         ws_bytes, stream, 3, true, threshold,
                         reinterpret_cast<unsigned long long*>(nonzero));
}

gdgs_status gdgs_div_adjoint(const float* lam, int32_t W, int32_t H, float* dgrad, void* stream) {
    GDGS_TRACE("gdgs_div_adjoint");
    clear_error();
    TRY(check_size(W, H));
    REQUIRE_PTR(lam);
    REQUIRE_PTR(dgrad);
    return launch_div_adjoint(lam, W, H, dgrad, as_stream(stream));
}

gdgs_status gdgs_div_adjoint_neumann(const float* lam, int32_t W, int32_t H, float* dgrad,
                                     void* stream) {
    GDGS_TRACE("gdgs_div_adjoint_neumann");
    clear_error();
    TRY(check_size(W, H));
    REQUIRE_PTR(lam);
    REQUIRE_PTR(dgrad);
    return launch_div_adjoint(lam, W, H, dgrad, as_stream(stream), true);
}

gdgs_status gdgs_raster_grad_backward(const gdgs_proj* proj, const float* opacity,
                                      const float* value, int64_t K, const gdgs_bins* bins,
                                      int32_t W, int32_t H, const float* grad, const float* dgrad,
                                      float* dmean2d, float* dconic, float* dopacity,
                                      float* dvalue, void* ws, size_t ws_bytes, void* stream) {
    GDGS_TRACE("gdgs_raster_grad_backward");
    clear_error();
    REQUIRE(K >= 0 && K < (int64_t)0xFFFFFFFFll, "K = %lld out of range", (long long)K);
    TRY(check_size(W, H));
    if (K == 0) return GDGS_OK;
    TRY(check_proj(proj));
    TRY(check_bins(bins, K));
    REQUIRE_PTR(opacity);
    REQUIRE_PTR(value);
    REQUIRE_PTR(grad);
    REQUIRE_PTR(dgrad);
    REQUIRE_PTR(dmean2d);
    REQUIRE_PTR(dconic);
    REQUIRE_PTR(dopacity);
    REQUIRE_PTR(dvalue);
    TRY(check_ws(ws, ws_bytes, raster_bwd_ws_bytes(K, bins->capacity)));
    return launch_raster_backward(*proj, opacity, value, K, *bins, W, H, grad, dgrad, dmean2d,
                                  dconic, dopacity, dvalue, ws, as_stream(stream));
}

}  // extern "C"
