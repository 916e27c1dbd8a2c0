// Internal declarations shared by the HIP translation units of libgdgs.
// Not part of the public C ABI (include/gdgs.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/gdgs.h"
#include "trace.hpp"

namespace gdgs {

// Support cut-off of a splat: G = exp(-E) only where E <= ln(1e5).
constexpr double kEcutD = 11.512925464970229;
constexpr float kEcut = 11.512925464970229f;
// Splats at camera depth <= kZnear are culled.
constexpr double kZnear = 0.2;
// Screen tile edge (pixels) used to bin the compositing work.
constexpr int kTile = 16;
// A pixel stops accumulating once its transmittance is below this.
constexpr float kTmin = 1e-7f;
// Multigrid: at most this many grids, each channel's coarse grids that fit
// together in kLdsBudget bytes of LDS are solved inside one workgroup.
constexpr int kMaxLevels = 8;
constexpr int kLdsBudget = 150 * 1024;

// Workgroups are dealt to the 8 XCDs (each with its own L2) round-robin by
// linear block id.  xcd_remap turns linear id b of nb into a logical index so
// that every XCD receives one contiguous range: neighbouring tiles (shared
// halos, shared splat records) then meet in the same L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int fq = nb / kXcds, r = nb % kXcds, x = b % kXcds, k = b / kXcds;
    return x < r ? x * (fq + 1) + k : r * (fq + 1) + (x - r) * fq + k;
}

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
void clear_error();

#define GDGS_HIP_TRY(expr)                                                        \
    do {                                                                          \
        hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess) {                                                   \
            ::gdgs::set_error("%s failed: %s", #expr, hipGetErrorString(e_));      \
            return GDGS_ERR_HIP;                                                  \
        }                                                                         \
    } while (0)

#define GDGS_LAUNCH_CHECK()                                                       \
    do {                                                                          \
        hipError_t e_ = hipGetLastError();                                        \
        if (e_ != hipSuccess) {                                                   \
            ::gdgs::set_error("kernel launch failed at %s:%d: %s", __FILE__,       \
                              __LINE__, hipGetErrorString(e_));                   \
            return GDGS_ERR_HIP;                                                  \
        }                                                                         \
    } while (0)

// ---------------------------------------------------------------- workspace
// Bump allocator over a caller-provided workspace; every carve is 256-byte
// aligned.  With base == nullptr it only measures.
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base(static_cast<char*>(b)) {}
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

inline int tiles_x(int W) { return (W + kTile - 1) / kTile; }
inline int tiles_y(int H) { return (H + kTile - 1) / kTile; }
inline int64_t num_tiles(int W, int H) { return (int64_t)tiles_x(W) * tiles_y(H); }

// ---------------------------------------------------------------- sort
// Sizes of the radix-sort launch for n (or a device-side n up to cap) keys.
int sort_grid(int64_t cap);

// Workspace of the binning step.
struct BinWs {
    uint32_t* dkey[2];   // depth-sort ping-pong keys [K]
    uint32_t* dval[2];   // depth-sort ping-pong values [K]
    uint32_t* drect[2][2]; // rectangle words riding with the depth sort [word][ping-pong][K]
    uint32_t* pkey[2];   // pair ping-pong keys [cap]
    uint32_t* pval[2];   // pair ping-pong values [cap]
    uint32_t* hist;      // [256][G]
    uint32_t* digit_tot; // [256]
    uint32_t* bsum;      // [nb] block sums of tile counts
    uint32_t* tile_bh;   // [ceil(T/256)][33] per-block key counts of the tile order
};
size_t bin_ws_layout(int64_t K, int64_t cap, int64_t T, void* ws, BinWs* out);

gdgs_status launch_bin_sort(const gdgs_proj& proj, int64_t K, int W, int H, const gdgs_bins& bins,
                            const BinWs& ws, hipStream_t st);

// ---------------------------------------------------------------- project
gdgs_status launch_project(const gdgs_scene& s, const gdgs_camera& cam, const gdgs_proj& out,
                           hipStream_t st);
gdgs_status launch_project_backward(const gdgs_scene& s, const gdgs_camera& cam,
                                    const float* dmean2d, const float* dconic, float* gmean,
                                    float* glog, float* gquat, hipStream_t st);
size_t loss_ws_bytes(int W, int H);
gdgs_status launch_threshold(float* x, int64_t n, float t, unsigned long long* nz,
                             hipStream_t st);
gdgs_status launch_image_loss(const float* c, const float* im, int W, int H, double lam,
                              double beta, double* out, float* dc, void* ws, hipStream_t st);
gdgs_status launch_adam(float* p, const float* g, float* m, float* v, int64_t n, int t, float lr,
                        float b1, float b2, float eps, float lo, float hi, hipStream_t st);
gdgs_status launch_project_2d(const float* mean2d, const float* conic, const float* depth,
                              int64_t K, int W, int H, const gdgs_proj& out, hipStream_t st);

// ---------------------------------------------------------------- raster
// 64-byte per-splat record in depth-rank order: (mx, my, ox, oy),
// (a, 2b, c, alpha), (v0..v3), (v4, v5, 0, 0).
size_t raster_ws_bytes(int64_t K);
// nch: value rows and output channels (6 image gradients, or 3 Laplacians)
// thr >= 0 (nch 3 only): the hard threshold of Eq. 24 fused into the store,
// kept non-zero values counted into *nonzero (zeroed first; may be null)
gdgs_status launch_raster(const gdgs_proj& proj, const float* opacity, const float* value,
                          int64_t K, const gdgs_bins& bins, int W, int H, float* grad,
                          void* ws, hipStream_t st, int nch = 6, float thr = -1.f,
                          unsigned long long* nonzero = nullptr);
gdgs_status launch_raster_count(const gdgs_proj& proj, const float* opacity, const float* value,
                                int64_t K, const gdgs_bins& bins, int W, int H,
                                unsigned long long* counts, void* ws, hipStream_t st);
size_t raster_bwd_ws_bytes(int64_t K, int64_t cap);
gdgs_status launch_raster_backward(const gdgs_proj& proj, const float* opacity,
                                   const float* value, int64_t K, const gdgs_bins& bins, int W,
                                   int H, const float* grad, const float* dgrad, float* dmean2d,
                                   float* dconic, float* dopacity, float* dvalue, void* ws,
                                   hipStream_t st);

// ---------------------------------------------------------------- poisson
struct MgPlan {
    int levels = 0;       // grids including the finest
    int lc = 0;           // first grid handled inside one workgroup
    int n[kMaxLevels];    // interior rows per level
    int m[kMaxLevels];    // interior columns per level
    int pitch[kMaxLevels];
    double dy[kMaxLevels];  // distance of the high-side boundary beyond the last row (grid units)
    double dx[kMaxLevels];  // same for the last column
    size_t lds_bytes = 0; // dynamic LDS of the in-workgroup V-cycle
    int pre = 2, post = 2, max_cycles = 20, coarse_sweeps = 0;
    float omega = 1.0f;   // SOR factor on the coarsest grid
    float sw = 1.0f;      // over-relaxation weight of the red-black smoothing sweeps
    double tol = 1e-6;
    bool warm = false;    // start from the caller's u instead of zero
    bool resume = false;  // continue the previous solve (setup skipped)
    bool neumann = false; // no flux across the image border, zero-mean gauge
    bool fmg = false;     // full-multigrid start (first cycle of a fresh solve)
    bool stop_eta = false; // stop on the normwise backward error instead of the correction
};
gdgs_status mg_plan(int W, int H, const gdgs_mg_params* mg, MgPlan* plan);
size_t poisson_ws_bytes(const MgPlan& plan, int W, int H);
// grad != nullptr: divergence of grad; else rho is the right-hand side.
class KeyBuilder;
// key: graph-cache key of the whole call (extended per segment); may be null.
// channel_parallel: run each colour channel's V-cycles on its own helper
// stream (lowest latency for one solve); false runs all channels in each
// launch on `st`, the whole solve replayed as one graph (least host work,
// for callers that already overlap many solves).
// tile_ranges ([2][T] tile pair ranges of the composite that produced rho, or
// null): the Dirichlet set-up of a given rho skips reading tiles that no splat
// touches (their composite is exactly zero).
gdgs_status launch_poisson(const float* grad, const float* rho, const float* boundary, int W,
                           int H, const MgPlan& plan, float* u, gdgs_stats* stats, void* ws,
                           hipStream_t st, const KeyBuilder* key = nullptr,
                           bool channel_parallel = true,
                           const uint32_t* tile_ranges = nullptr);
gdgs_status launch_div_adjoint(const float* lam, int W, int H, float* dgrad, hipStream_t st,
                               bool neumann = false);

// ---------------------------------------------------------------- batched solves
// Up to kBatchMax Dirichlet solves advance together, one V-cycle of every
// active solve per round (see poisson.hip).  Completions are written to a
// ring in host memory (pinned, allocated by the caller).
constexpr int kBatchMax = 64;
constexpr int kRingCap = 256;
struct BatchRec {
    long long id;
    int cycles;
    int converged;
    double eta;
    double rel_res;
};
struct BatchRing {
    long long head;   // records written so far; record k is rec[k % kRingCap]
    long long pad[7];
    BatchRec rec[kRingCap];
};
size_t batch_table_bytes();
// true if the batched kernels can run this plan (Dirichlet, no FMG or resume,
// small tiles on every global coarse grid)
bool batch_supported(const MgPlan& p);
int batch_depth(const MgPlan& p);  // global coarse grids below the finest
gdgs_status batch_clear(void* table, hipStream_t st);
// the solve's set-up (divergence, right-hand-side norms, flags) in its workspace
gdgs_status launch_poisson_setup(const float* grad, const float* boundary, int W, int H,
                                 const MgPlan& p, float* u, gdgs_stats* stats, void* ws,
                                 hipStream_t st);
gdgs_status batch_activate(void* table, int e, int64_t id, const float* grad, int W, int H,
                           const MgPlan& p, float* u, gdgs_stats* stats, void* ws,
                           hipStream_t st);
gdgs_status batch_deactivate(void* table, int e, hipStream_t st);
// one V-cycle of every active solve whose global coarse grids are <= depth
gdgs_status launch_batch_round(void* table, BatchRing* ring, int depth, int pre, int post,
                               hipStream_t st);

// ---------------------------------------------------------------- whole frame
// Everything one render carves out of its workspace.
struct RenderWs {
    gdgs_proj proj;
    gdgs_bins bins;
    float* grad;
    void* bin_ws;
    void* raster_ws;
    void* poisson_ws;
};
// Bytes of the render workspace (ws may be null: size only).
size_t render_layout(int64_t K, int W, int H, int64_t cap, const MgPlan& plan, void* ws,
                     RenderWs* out);
// stats->num_pairs and stats->overflow from the binning's pair count.
gdgs_status launch_render_stats(const int64_t* num_pairs, int64_t cap, gdgs_stats* stats,
                                hipStream_t st);

// ---------------------------------------------------------------- timing hook
// Optional per-launch event timing of one named kernel (set through the C ABI).
struct KernelTimer {
    char name[32] = {0};
    hipEvent_t* starts = nullptr;
    hipEvent_t* stops = nullptr;
    int n = 0;
    int next = 0;
    int repeats = 1;  // launches between one pair (idempotent kernels only)
};
constexpr int kMaxTimers = 4;
KernelTimer* kernel_timers();  // [kMaxTimers]
// Event pair (start, stop) to bracket this launch of `name` with, or false.
bool timer_events(const char* name, hipEvent_t* start, hipEvent_t* stop);
// How many times a timed launch of `name` is issued between its events (1
// unless set by gdgs_set_kernel_timer_repeats).
int timer_repeats(const char* name);
// Timed launches count from pair 0 again (called at every ABI entry).
void reset_timers();

// Fill a u32 array with a value (graph-capture friendly, no memset nodes).
gdgs_status launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t st);

}  // namespace gdgs
