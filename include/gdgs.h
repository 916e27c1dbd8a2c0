/*
 * gdgs.h -- C ABI of the gradient-domain Gaussian splatting render + Poisson
 * hot path (GDGS, arXiv 2405.05446) for AMD Instinct MI355X (gfx950).
 *
 * The method (Sec. 2.2 and Algorithm 1 of the paper): splats carrying image
 * gradients are projected to the image plane (Eq. 19), composited front to back
 * into a gradient image (Eq. 20), and the image is recovered by solving the 2D
 * Poisson equation on the divergence of that gradient image (Eq. 21).
 *
 * Conventions (the paper leaves them open):
 *   - camera: OpenCV axes, x_c = R x + t, pinhole (fx x/z + cx, fy y/z + cy);
 *     pixel (i, j) has centre (j + 0.5, i + 0.5);
 *   - a splat's Gaussian is exp(-d^T Sigma2D^{-1} d) (no factor 1/2, Eq. 9),
 *     taken as exactly 0 where the exponent exceeds ln(1e5);
 *   - splats with camera depth <= 0.2, a zero quaternion or a singular 2D
 *     covariance are culled;
 *   - six gradient channels, index 2*c + d: colour c, d = 0 derivative along
 *     image columns (x), d = 1 along image rows (y);
 *   - gradients are forward differences, the divergence is the backward
 *     difference, the Laplacian the 5-point stencil with unit spacing;
 *   - the Poisson problem is solved on the (H-2) x (W-2) interior pixels with
 *     Dirichlet values on the one-pixel outer ring.
 *
 * Memory and ownership:
 *   - every array argument is a DEVICE pointer to caller-owned memory, FP32
 *     (or u32 / i64 where stated), planar structure-of-arrays layout, 4-byte
 *     aligned; "[a][b]" is row-major with b fastest;
 *   - the library never allocates device memory: scratch comes from a
 *     caller-provided workspace of the size the *_workspace_size calls report;
 *   - host structs (camera, parameters) are read during the call only.
 *
 * Streams: every call enqueues work on `stream` (a hipStream_t; NULL = the
 * default stream) and returns without waiting, unless stated otherwise.
 *
 * Errors: calls return a gdgs_status.  Argument checks happen on the host
 * before anything is enqueued; gdgs_last_error() then describes the failure
 * (thread-local).  Conditions found on the device (pair-capacity overflow,
 * non-convergence) are reported in a device-side gdgs_stats the caller reads
 * after synchronising the stream; they are not call failures.
 *
 * Environment (read once per process):
 *   - GDGS_GRAPHS=0: launch directly instead of replaying cached HIP graphs
 *     (gdgs_set_graphs);
 *   - GDGS_CHANNEL_STREAMS=0: run every multigrid launch over the three
 *     channels on the caller's stream (gdgs_set_channel_streams);
 *   - GDGS_LOG=0..3: host log lines on stderr, prefixed "gdgs[<level>] ":
 *     0 none (default), 1 every error the library records (the text of
 *     gdgs_last_error), 2 also graph captures and server events, 3 also every
 *     entry-point call and multigrid plan.
 * Every entry point also opens a roctx range named after it (visible with
 * rocprofv3 --marker-trace); a range spans the host's enqueue of the call.
 */
#ifndef GDGS_H
#define GDGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gdgs_status {
    GDGS_OK = 0,
    GDGS_ERR_INVALID_ARGUMENT = 1, /* bad size, null or misaligned pointer, bad parameter */
    GDGS_ERR_CAPACITY = 2,         /* pair list larger than the caller's capacity */
    GDGS_ERR_WORKSPACE = 3,        /* workspace missing or smaller than required */
    GDGS_ERR_BUDGET = 4,           /* serving: request does not fit the memory budget */
    GDGS_ERR_HIP = 5,              /* a HIP runtime call failed */
    GDGS_ERR_UNSUPPORTED = 6,      /* valid request this build does not handle */
    GDGS_ERR_NOT_READY = 7,        /* serving: nothing finished yet */
    GDGS_ERR_CANCELLED = 8         /* serving: the request was cancelled */
} gdgs_status;

/* Splat scene, K splats (Sec. 1.2: Sigma = R S S^T R^T).  Device pointers. */
typedef struct gdgs_scene {
    const float* mean;      /* [3][K] world position */
    const float* log_scale; /* [3][K] log of the per-axis scale (S = diag(exp)) */
    const float* quat;      /* [4][K] rotation quaternion (w, x, y, z), normalised by the kernel */
    const float* opacity;   /* [K] alpha in (0, 1) */
    const float* value;     /* [6][K] gradient values carried by each splat */
    int64_t K;
} gdgs_scene;

/* Pinhole camera (host struct). R is row-major world-to-camera rotation. */
typedef struct gdgs_camera {
    int32_t W, H;           /* image size in pixels, each >= 3 */
    double fx, fy, cx, cy;  /* focal lengths (> 0) and principal point, pixels */
    double R[9];
    double t[3];
} gdgs_camera;

/* Projected splats (Eq. 19), [.][K] device arrays written by gdgs_project or
 * gdgs_project_2d.  The mean is stored relative to the pixel origin of the
 * splat's tile rectangle, (16 * tx0, 16 * ty0), which keeps FP32 offsets small
 * at any image size. */
typedef struct gdgs_proj {
    float* mean2d;    /* [2][K] image-plane mean minus (16 tx0, 16 ty0) */
    float* conic;     /* [3][K] (a, b, c) of Sigma2D^{-1}: E = a dx^2 + 2 b dx dy + c dy^2 */
    float* depth;     /* [K] camera-space depth (the compositing order key) */
    uint32_t* rect;   /* [2][K] tile rectangle: rect[0] = tx0 | tx1 << 16, rect[1] = ty0 | ty1 << 16 (half-open) */
    uint32_t* count;  /* [K] number of tiles in the rectangle, 0 if culled or off-screen */
} gdgs_proj;

/* Tile bins: the (tile, splat) pairs sorted by (tile, FP32 depth, splat
 * index) and each tile's range.  Device arrays, caller-owned. */
typedef struct gdgs_bins {
    int64_t capacity;     /* length of tile_of_pair / splat_of_pair */
    uint32_t* tile_of_pair; /* [capacity] sorted tile id (ty * ceil(W/16) + tx) */
    uint32_t* splat_of_pair; /* [capacity] splat index of each sorted pair */
    uint32_t* order;      /* [K] splat index of depth rank s (stable: ties by index; culled last) */
    uint32_t* ranges;     /* [2][T] start and end (half-open) of each tile, T = ceil(W/16) ceil(H/16) */
    int64_t* num_pairs;   /* [1] total pairs P; pairs beyond capacity are dropped */
    uint32_t* tile_order; /* [T] or NULL: the tiles, those with the most pairs first (by
                           * floor(log2(pairs)), ties by tile id; empty tiles last).  Only
                           * the order in which the compositing kernels take the tiles;
                           * NULL takes them by tile id.  Images do not depend on it. */
} gdgs_bins;

/* Multigrid parameters (host struct) for the Poisson solve (Eq. 21).
 * A channel stops after the first V-cycle whose correction is small relative
 * to the solution, ||u_k - u_{k-1}||_inf <= tol ||u_k||_inf (interior pixels);
 * with the cycle's contraction factor rho (about 0.02 with the default
 * smoothing weight at 1080p, 0.06 with plain Gauss-Seidel) the remaining error
 * is then about rho / (1 - rho) of that correction. */
#define GDGS_MG_WARM_START 1  /* flags: start from the caller's u (interior) instead of zero */
/* flags: continue the previous solve in the same workspace.  Setup is skipped:
 * the right-hand side, its norms, each channel's convergence flag and its
 * cycle count (stats cycles[] keep counting) carry over, and channels that
 * had already converged are left as they are.  Requires the same W, H, grid
 * parameters, u, stats and workspace as the call it continues, with nothing
 * written to them since.  Calls totalling n cycles give bit for bit the
 * result of one call with max_cycles = n. */
#define GDGS_MG_RESUME 2
/* flags: the paper's Neumann condition (Sec. 2.1 "Poisson Equation" and Sec. 2.2 "Poisson Equation", Eq. 21)
 * instead of Dirichlet data on the image ring.  Every one of the H x W pixels
 * is an unknown and no flux crosses the image border: the Laplacian at a
 * pixel sums only its neighbours inside the image, and with gradients the
 * divergence drops the differences that would cross the border (gx in the
 * last column, gy in the last row).  The problem is singular: rho is replaced
 * by rho - mean(rho) per channel and u is returned with zero mean per
 * channel.  boundary must be NULL.  The finest grid lives in the workspace
 * (padded), so the workspace is larger than for the Dirichlet problem;
 * GDGS_MG_WARM_START reads the caller's u as the starting image, and
 * GDGS_MG_RESUME continues from the workspace.  stats: b = mean(rho) - rho
 * over all pixels, and the residual norms are over all pixels.  The server
 * takes it in its parameters; the reverse chain uses the same solve and
 * gdgs_div_adjoint_neumann. */
#define GDGS_MG_NEUMANN 4
/* flags: a full-multigrid start (nested iteration) instead of a first V-cycle
 * from the initial image: the residual of the initial image is restricted to
 * every grid, the coarse grids' problems are solved from the coarsest up, each
 * grid starting from the interpolated solution of the one below and getting
 * one V-cycle, and the interpolated result corrects the finest grid.  Counts
 * as the first cycle (stats cycles[]); later cycles are ordinary V-cycles and
 * the stopping test is the same.  Ignored with GDGS_MG_RESUME and when every
 * grid fits in one workgroup's LDS. */
#define GDGS_MG_FMG 8
/* flags: stop a channel on the normwise backward error instead of the
 * relative correction: after the first V-cycle with
 * eta = ||b - A w||_inf / (8 ||w||_inf + ||b||_inf) <= tol (evaluated in FP64
 * from FP32 iterates).  A backward-error bound, not a bound on the error of w:
 * for the 5-point operator a small smooth residual can still leave an error
 * of order (grid size)^2 times the residual, so the default rule (relative
 * correction) is the safer one; this flag exists to measure the trade-off. */
#define GDGS_MG_STOP_ETA 16
typedef struct gdgs_mg_params {
    int32_t levels;        /* grids including the finest, >= 1; 0 = as many as the size allows, at most 8 */
    int32_t pre_sweeps;    /* red-black Gauss-Seidel sweeps before restriction, 1..2 */
    int32_t post_sweeps;   /* sweeps after prolongation, 1..2 */
    int32_t max_cycles;    /* V-cycle limit, 1..64 */
    int32_t coarse_sweeps; /* SOR sweeps on the coarsest grid; 0 = automatic */
    int32_t flags;         /* GDGS_MG_WARM_START, GDGS_MG_RESUME, GDGS_MG_NEUMANN, GDGS_MG_FMG,
                              GDGS_MG_STOP_ETA (or-ed) or 0 */
    double tol;            /* relative-correction tolerance (see above); 0 runs max_cycles */
    double smooth_weight;  /* over-relaxation weight w of every red-black smoothing sweep:
                              u <- u + w (Gauss-Seidel value - u); 1 = plain Gauss-Seidel,
                              0 = the default, 1.15; otherwise in [0.5, 1.5] */
} gdgs_mg_params;

/* Device-side statistics written by the solve and the render (b and w are
 * the right-hand side and unknowns of A w = b, A = minus the interior
 * 5-point Laplacian). */
typedef struct gdgs_stats {
    int32_t cycles[3];     /* V-cycles run per colour channel */
    int32_t converged;     /* 1 if every channel met tol */
    double eta[3];         /* ||b - A w||_inf / (8 ||w||_inf + ||b||_inf) after the last cycle */
    double rel_res[3];     /* ||b - A w||_2 / ||b||_2 after the last cycle */
    double b_norm[3];      /* ||b||_2 per channel */
    double delta[3];       /* relative correction of the last cycle (the stopping quantity) */
    int64_t num_pairs;     /* render: (tile, splat) pairs needed */
    int32_t overflow;      /* render: 1 if num_pairs exceeded the pair capacity */
    int32_t reserved;
} gdgs_stats;

/* ------------------------------------------------------------------ */
/* Status and errors.                                                  */
const char* gdgs_status_string(gdgs_status s);
/* Thread-local description of the last failure on this thread ("" if none). */
const char* gdgs_last_error(void);
/* Version string of the library build. */
const char* gdgs_version(void);
/* Host-only switch (default on; environment GDGS_GRAPHS=0 turns it off):
 * gdgs_render and the Poisson calls capture their launch sequence once per
 * argument set into a HIP graph and replay it, which removes per-kernel host
 * launch cost.  Calls on a stream that is itself being captured always
 * launch directly.  gdgs_clear_graphs() destroys the cached graphs. */
void gdgs_set_graphs(int enable);
void gdgs_clear_graphs(void);
/* Host-only switch (default on): the Poisson calls run each colour channel's
 * V-cycles on a helper stream of its own, bound to the caller's stream, so
 * that the three channels overlap.  Off, every multigrid launch covers all
 * three channels on the caller's stream (one kernel at a time: the timing
 * of a single launch is then that of the kernel alone).  Results are the
 * same bit for bit either way. */
void gdgs_set_channel_streams(int enable);
/* Host-only profiling hook (up to 4 names at once).  After arming, the i-th
 * launch of the named kernel (i < n, counted over all later calls until the
 * next gdgs_rewind_kernel_timers or re-arming) is bracketed by
 * hipEventRecord(start_events[i]) and hipEventRecord(stop_events[i]) on the
 * stream it runs on; later launches are not timed.  Calls that would launch
 * a timed kernel bypass the graph cache for that kernel (events recorded as
 * graph nodes do not reliably bracket their neighbour), so timed figures are
 * those of direct launches.  Names: "raster" (the compositing kernel),
 * "mg_pre_fine" and "mg_post_fine" (the finest-grid multigrid passes, once
 * per V-cycle).  The events (hipEvent_t) belong to the caller and must
 * outlive the timer.  n <= 0 clears that name, kernel NULL clears all. */
gdgs_status gdgs_set_kernel_timer(const char* kernel, void** start_events, void** stop_events,
                                  int n);
/* Host-only profiling hook: each timed launch of an armed multigrid post
 * pass ("mg_post_fine" or "mg_post_coarse") is issued `repeats` (1..64) times
 * in a row between its two events, so that the event overhead is spread over
 * the repeats.  A post pass reads the second buffer, the right-hand side and
 * the coarse correction and writes the iterate and its norm records, none of
 * which it reads, so the repeats leave every result unchanged.  Re-arming the
 * name resets it to 1.  GDGS_ERR_INVALID_ARGUMENT for another name, a name
 * not armed, or repeats out of range. */
gdgs_status gdgs_set_kernel_timer_repeats(const char* kernel, int repeats);
/* Start every armed timer at pair 0 again. */
void gdgs_rewind_kernel_timers(void);
/* Number of launches of `kernel` bracketed since arming or the last rewind
 * (at most its n); 0 for a name that is not armed. */
int gdgs_kernel_timer_count(const char* kernel);

/* ------------------------------------------------------------------ */
/* Workspace sizes (bytes, host-only calls, nothing is enqueued).      */
gdgs_status gdgs_bin_sort_workspace_size(int64_t K, int32_t W, int32_t H, int64_t pair_capacity,
                                         size_t* bytes);
gdgs_status gdgs_raster_workspace_size(int64_t K, size_t* bytes);
gdgs_status gdgs_poisson_workspace_size(int32_t W, int32_t H, const gdgs_mg_params* mg,
                                        size_t* bytes);
/* Everything gdgs_render needs, including its projected splats and bins. */
gdgs_status gdgs_workspace_size(int64_t K, int32_t W, int32_t H, int64_t pair_capacity,
                                const gdgs_mg_params* mg, size_t* bytes);

/* ------------------------------------------------------------------ */
/* Step 1, projection (Sec. 1.2 Eq. 10; Sec. 2.2 "Projection", Eq. 19).
 * Per splat: q -> R, Sigma = R diag(exp(2 l)) R^T, x_c = cam.R x + cam.t,
 * J = d(pinhole)/d(x_c) at the mean, Sigma2D = J cam.R Sigma cam.R^T J^T,
 * conic = Sigma2D^{-1}, depth = z_c, and the tile rectangle of the support
 * box {columns j : |j + 0.5 - mu_x| <= sqrt(ln(1e5) Sigma2D_xx)} (rows alike),
 * clamped to the image.  Arithmetic in FP64, results stored in FP32.
 * K = 0 is allowed (nothing is enqueued). */
gdgs_status gdgs_project(const gdgs_scene* scene, const gdgs_camera* cam, const gdgs_proj* out,
                         void* stream);

/* Step 1 for splats already in image space (used by the differentiable
 * path): mean2d[2][K] absolute image coordinates, conic[3][K] and depth[K]
 * given; fills out->mean2d (tile-relative), out->conic (copied), out->depth
 * (copied), out->rect and out->count exactly as gdgs_project does. */
gdgs_status gdgs_project_2d(const float* mean2d, const float* conic, const float* depth,
                            int64_t K, int32_t W, int32_t H, const gdgs_proj* out, void* stream);

/* ------------------------------------------------------------------ */
/* Step 2, tile binning and ordering (the front-to-back order of Eq. 11 /
 * Eq. 20, "sorted from the view direction").  Stable radix sort of the splats
 * by FP32 depth (culled last), one (tile, rank) pair per tile of each splat's
 * rectangle, stable radix sort of the pairs by tile, tile ranges.  The pair
 * order equals a lexicographic sort by (tile, FP32 depth bits, splat index).
 * If bins->tile_order is not NULL it receives the heaviest-first tile order.
 * Writes bins->num_pairs = P on the device; only the first min(P, capacity)
 * pairs are kept and later steps use those (check P after the stream syncs).
 * Workspace: gdgs_bin_sort_workspace_size(K, W, H, bins->capacity). */
gdgs_status gdgs_bin_sort(const gdgs_proj* proj, int64_t K, int32_t W, int32_t H,
                          const gdgs_bins* bins, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ */
/* Step 3, gradient compositing (Eq. 11 applied to the projected field,
 * Eq. 20): for every pixel p and channel m,
 *   grad[m][p] = sum_k value[m][k] a_k T_{k-1},  a_k = opacity[k] G_k(p),
 *   T_0 = 1, T_k = T_{k-1} (1 - a_k),
 * over the tile's pairs in bin order.  A pixel stops accumulating once its
 * T falls below 1e-7 (the dropped weight is below 1e-7).  Output grad[6][H][W]
 * is fully written.  Workspace: gdgs_raster_workspace_size(K). */
gdgs_status gdgs_raster_grad(const gdgs_proj* proj, const float* opacity, const float* value,
                             int64_t K, const gdgs_bins* bins, int32_t W, int32_t H, float* grad,
                             void* ws, size_t ws_bytes, void* stream);

/* Step 3 of the Laplacian-splat form (Sec. 2.2 "Projection" and Eq. 20 with
 * splats that carry the Laplacian of each colour channel instead of its
 * gradient): the same compositing with three values per splat,
 *   rho[c][p] = sum_k lap[c][k] a_k T_{k-1},  c = 0, 1, 2,
 * whose result is the right-hand side of the Poisson equation (Eq. 21)
 * directly, with no divergence step (gdgs_poisson_solve_rhs).  lap is [3][K];
 * rho[3][H][W] is fully written.  Workspace: gdgs_raster_workspace_size(K). */
gdgs_status gdgs_raster_laplacian(const gdgs_proj* proj, const float* opacity, const float* lap,
                                  int64_t K, const gdgs_bins* bins, int32_t W, int32_t H,
                                  float* rho, void* ws, size_t ws_bytes, void* stream);

/* Sparse compositing (Sec. 2.2 "Projection": the projected Laplacian field of
 * Eq. 20 is sparse; Sec. 3.1: the hard threshold T of Eq. 24 gives the sparse
 * representation): the three-channel composite of gdgs_raster_laplacian with
 * T applied to every value before it is stored (kept when |x| >= threshold,
 * ties kept, the comparison in FP32), fused into the compositing kernel, so no
 * separate pass over rho is made.  threshold >= 0 (0 keeps every value).
 * nonzero (device uint64, may be NULL) receives the number of values of
 * rho[3][H][W] that are non-zero after the threshold (zeroed by the call).
 * Tiles that no splat touches are written as zeros.  Errors as
 * gdgs_raster_laplacian, plus GDGS_ERR_INVALID_ARGUMENT for threshold < 0. */
gdgs_status gdgs_raster_laplacian_threshold(const gdgs_proj* proj, const float* opacity,
                                            const float* lap, int64_t K, const gdgs_bins* bins,
                                            int32_t W, int32_t H, float threshold, float* rho,
                                            uint64_t* nonzero, void* ws, size_t ws_bytes,
                                            void* stream);

/* Profiling companion of gdgs_raster_grad: the same traversal without an
 * image; counts[0] (device, uint64) receives the number of (pixel, splat)
 * contributions the composite makes (terms of the sum of Eq. 20 with a non-zero
 * opacity), counts[1] is zeroed.  Same workspace as gdgs_raster_grad. */
gdgs_status gdgs_raster_count(const gdgs_proj* proj, const float* opacity, const float* value,
                              int64_t K, const gdgs_bins* bins, int32_t W, int32_t H,
                              uint64_t* counts, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ */
/* Step 4, Poisson reconstruction (Sec. 2.1 Eq. 13-16; Sec. 2.2 Eq. 21) with
 * Dirichlet data.  rho = backward-difference divergence of grad[6][H][W] on
 * interior pixels, then multigrid V-cycles (red-black Gauss-Seidel smoothing,
 * full-weighting restriction, bilinear prolongation, SOR on the coarsest
 * grid) for L u = rho on the interior, u = boundary on the ring.
 * boundary[3][H][W] (only its ring is read) may be NULL for a zero ring.
 * Output u[3][H][W] is fully written (ring = boundary ring).  stats_dev
 * (device pointer, may be NULL) receives cycles, eta, rel_res, delta.
 * Workspace: gdgs_poisson_workspace_size(W, H, mg). */
gdgs_status gdgs_poisson_solve(const float* grad, const float* boundary, int32_t W, int32_t H,
                               const gdgs_mg_params* mg, float* u, gdgs_stats* stats_dev,
                               void* ws, size_t ws_bytes, void* stream);

/* Same solve with the right-hand side rho[3][H][W] given directly (interior
 * read): used for the adjoint solve of the backward pass and for Laplacian
 * splats. */
gdgs_status gdgs_poisson_solve_rhs(const float* rho, const float* boundary, int32_t W, int32_t H,
                                   const gdgs_mg_params* mg, float* u, gdgs_stats* stats_dev,
                                   void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve of
 * gdgs_poisson_solve (same arguments, same kernels, same results) with its
 * scratch in a fixed device array of the library instead of a caller
 * workspace.  The array holds GDGS_STATIC_SCRATCH_BYTES (80 MiB) on every GPU
 * the library runs on, from the first call on that GPU until the process
 * ends: enough for the Dirichlet problem up to 1920 x 1080 (72.5 MiB) and the
 * Neumann problem up to about 1.7 Mpixels.  A size that needs more returns
 * GDGS_ERR_WORKSPACE with a message (gdgs_poisson_workspace_size gives the
 * need).  This call allocates nothing: no hipMalloc, no stream, event or graph
 * is created; its kernels are launched directly on `stream`, every channel in
 * each launch.  The solve initialises the part of the array it reads (a
 * previous call's contents are overwritten), except under GDGS_MG_RESUME,
 * which continues whatever solve the array holds on this GPU.  All calls on one
 * GPU share that GPU's array: calls whose work overlaps on the device (other
 * streams, other threads) race and must be serialised by the caller.  Errors as
 * gdgs_poisson_solve, plus GDGS_ERR_HIP if the array's address cannot be
 * found. */
#define GDGS_STATIC_SCRATCH_BYTES (80ull << 20)
gdgs_status gdgs_poisson_solve_static(const float* grad, const float* boundary, int32_t W,
                                      int32_t H, const gdgs_mg_params* mg, float* u,
                                      gdgs_stats* stats_dev, void* stream);

/* ------------------------------------------------------------------ */
/* Steps 1-4 on one stream with no host synchronisation: project, bin and
 * sort, composite, solve.  u[3][H][W] is the recovered image.  If sync_stats
 * is non-zero the call waits for the stream and returns GDGS_ERR_CAPACITY when
 * the pairs exceeded pair_capacity (stats hold the needed count).
 * Workspace: gdgs_workspace_size(scene->K, W, H, pair_capacity, mg). */
gdgs_status gdgs_render(const gdgs_scene* scene, const gdgs_camera* cam, const float* boundary,
                        const gdgs_mg_params* mg, int64_t pair_capacity, float* u,
                        gdgs_stats* stats_dev, int sync_stats, void* ws, size_t ws_bytes,
                        void* stream);

/* gdgs_render for Laplacian splats (Sec. 2.2): scene->value is [3][K] (the
 * Laplacian of each colour channel carried by the splat); steps 1, 2, the
 * three-channel composite of gdgs_raster_laplacian and the Poisson solve with
 * that composite as rho.  Same workspace, statistics and errors as
 * gdgs_render. */
gdgs_status gdgs_render_laplacian(const gdgs_scene* scene, const gdgs_camera* cam,
                                  const float* boundary, const gdgs_mg_params* mg,
                                  int64_t pair_capacity, float* u, gdgs_stats* stats_dev,
                                  int sync_stats, void* ws, size_t ws_bytes, void* stream);

/* The sparse form of gdgs_render_laplacian (Sec. 2.2, Eq. 20 and 21, with the
 * threshold of Eq. 24, Sec. 3.1): compositing with the threshold fused (see
 * gdgs_raster_laplacian_threshold; nonzero may be NULL), and the solve's
 * set-up reads rho only in tiles that some splat touches (the others are
 * exact zeros).  Same arguments, workspace (gdgs_workspace_size) and errors
 * as gdgs_render_laplacian, plus threshold >= 0.  The result equals
 * gdgs_raster_laplacian_threshold followed by gdgs_poisson_solve_rhs. */
gdgs_status gdgs_render_laplacian_sparse(const gdgs_scene* scene, const gdgs_camera* cam,
                                         const float* boundary, const gdgs_mg_params* mg,
                                         int64_t pair_capacity, float threshold, float* u,
                                         gdgs_stats* stats_dev, uint64_t* nonzero,
                                         int sync_stats, void* ws, size_t ws_bytes,
                                         void* stream);

/* ------------------------------------------------------------------ */
/* Backward pass (gradients of a loss on u through the Poisson solve and the
 * compositing; the particle-parameter gradients of Sec. 1.1, Eq. 5-7). */

/* Reverse mode of gdgs_project (Sec. 1.2 Eq. 10 / Sec. 2.2 Eq. 19, the
 * particle-parameter gradients of Sec. 1.1): from dL/dmean2d[2][K] and
 * dL/dconic[3][K] (with respect to the image-plane mean and the conic
 * (a, b, c) as gdgs_project writes them) to dL/dmean[3][K] (world),
 * dL/dlog_scale[3][K] and dL/dquat[4][K] (the raw quaternion, through its
 * normalisation).  The chain: conic -> Sigma2D -> (J W, Sigma) -> camera-space
 * mean and (R, S) -> quaternion and log-scales; FP64 inside, FP32 stored.
 * Culled splats (zero quaternion, z_c <= 0.2, det <= 0) get zeros.  The
 * outputs are fully written; the depth gets no gradient (it only orders). */
gdgs_status gdgs_project_backward(const gdgs_scene* scene, const gdgs_camera* cam,
                                  const float* dmean2d, const float* dconic, float* dmean,
                                  float* dlog_scale, float* dquat, void* stream);

/* Image loss of an optimisation step (Sec. 2.3, Eq. 22, the loss Algorithm 1
 * evaluates each iteration) between the rendered image c[3][H][W] and the
 * observed im[3][H][W]:
 *   L = (1 - lam) mean|c - im| + beta mean|grad c - grad im| + lam (1 - mean SSIM),
 * forward differences along columns and rows; SSIM per channel over an
 * 11 x 11 Gaussian window (sigma 1.5, normalised, zero padding), C1 = 1e-4,
 * C2 = 9e-4.  loss_dev (device, 4 doubles) receives L and its three terms;
 * dc[3][H][W] (may be NULL) receives dL/dc.  Workspace:
 * gdgs_image_loss_workspace_size(W, H). */
gdgs_status gdgs_image_loss_workspace_size(int32_t W, int32_t H, size_t* bytes);
gdgs_status gdgs_image_loss(const float* c, const float* im, int32_t W, int32_t H, double lam,
                            double beta, double* loss_dev, float* dc, void* ws, size_t ws_bytes,
                            void* stream);

/* Hard threshold of Sec. 3.1 (Eq. 24), in place on x[n] (device):
 * x = x if |x| >= t else 0 (t >= 0), the sparse representation of a
 * Laplacian field before the Poisson solve.  nonzero_dev (device uint64, may
 * be NULL) receives the number of non-zero values left. */
gdgs_status gdgs_threshold(float* x, int64_t n, float t, uint64_t* nonzero_dev, void* stream);

/* One Adam update (Kingma and Ba) of n parameters at step t >= 1:
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * param -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), then clamped
 * to [lo, hi] if lo < hi.  All arrays device, in place. */
gdgs_status gdgs_adam_step(float* param, const float* grad, float* m, float* v, int64_t n,
                           int32_t t, float lr, float beta1, float beta2, float eps, float lo,
                           float hi, void* stream);

/* Transpose of the divergence: dgrad[6][H][W] from lam[3][H][W] (interior
 * read, taken as 0 elsewhere): dgx = lam[i][j] - lam[i][j+1],
 * dgy = lam[i][j] - lam[i+1][j]. */
gdgs_status gdgs_div_adjoint(const float* lam, int32_t W, int32_t H, float* dgrad, void* stream);

/* Transpose of the Neumann divergence (the reverse step of GDGS_MG_NEUMANN,
 * Sec. 2.1 and Sec. 2.2): dgrad[6][H][W] from lam[3][H][W] (every pixel):
 * dgx[i][j] = lam[i][j] - lam[i][j+1] for j < W-1 and 0 in the last column,
 * dgy[i][j] = lam[i][j] - lam[i+1][j] for i < H-1 and 0 in the last row.
 * Device arrays, caller-owned; enqueued on stream; size errors are returned. */
gdgs_status gdgs_div_adjoint_neumann(const float* lam, int32_t W, int32_t H, float* dgrad,
                                     void* stream);

/* Reverse compositing.  Given the forward inputs, the forward output grad
 * and dL/dgrad, writes dL/d(mean2d)[2][K], dL/d(conic)[3][K],
 * dL/d(opacity)[K], dL/d(value)[6][K] (fully written; zero for splats that
 * touch no pixel).  Per-pixel transmittance is recomputed, not stored.
 * The per-splat sums are deterministic (no atomics).
 * Workspace: gdgs_raster_backward_workspace_size(K, bins->capacity). */
gdgs_status gdgs_raster_backward_workspace_size(int64_t K, int64_t pair_capacity, size_t* bytes);
gdgs_status gdgs_raster_grad_backward(const gdgs_proj* proj, const float* opacity,
                                      const float* value, int64_t K, const gdgs_bins* bins,
                                      int32_t W, int32_t H, const float* grad, const float* dgrad,
                                      float* dmean2d, float* dconic, float* dopacity,
                                      float* dvalue, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ */
/* Serving: continuous batching of render + Poisson requests (one GPU).
 * The paper's method produces one view per camera pose (Algorithm 1 takes
 * the poses as input; Sec. 2.2 renders each view by projection, compositing
 * and the Poisson solve of Eq. 21).  A server keeps one scene resident and
 * runs many such views, of mixed image sizes, concurrently:
 *   - a native scheduler thread admits requests in arrival order whenever
 *     one of `streams` HIP streams is free and the request's transient state
 *     fits the memory budget (one device allocation of hbm_budget bytes,
 *     made at creation; nothing is allocated afterwards);
 *   - each request runs the same kernels as gdgs_render on its own stream,
 *     so its result is bit for bit the one it would have alone: the Poisson
 *     solve is resumed (GDGS_MG_RESUME) until it converges or mg.max_cycles
 *     is reached, and a pair-capacity overflow re-runs the request with a
 *     larger capacity;
 *   - finished requests are reported through gdgs_server_poll.
 * Device buffers named in a request (boundary, u) must stay valid and
 * untouched until its completion has been polled; the scene's arrays must
 * outlive the server.  All calls are thread-safe. */
typedef struct gdgs_server gdgs_server;

/* Server flag: batched solves.  A request's stream carries its projection,
 * binning, compositing and the solve's set-up; the request then joins a
 * device table of up to 64 in-flight solves and gives its stream back.  A
 * separate solver stream runs rounds, each one V-cycle of every solve in the
 * table: every kernel of a round is a persistent grid whose workgroups take
 * the tasks of all the solves (finest-grid strips, coarse-grid tiles, in-LDS
 * coarse V-cycles, end-of-cycle bookkeeping) from the table.  Each task runs
 * the same code as the per-request kernels, so results are bit for bit those
 * of gdgs_render alone.  A solve that has converged (or reached
 * mg.max_cycles) leaves the table and is reported through a completion ring
 * in pinned host memory.  The solve runs in the request's u directly.
 * Dirichlet problem only (mg.flags 0); streams + 1 HIP streams are used. */
#define GDGS_SERVER_BATCHED 1

typedef struct gdgs_server_params {
    int64_t hbm_budget;   /* bytes of device memory for in-flight requests */
    int32_t streams;      /* requests whose front half (projection .. set-up, or the
                             whole render without GDGS_SERVER_BATCHED) runs at once,
                             1..16 (1 and no flags = plain FIFO) */
    int32_t flags;        /* 0 or GDGS_SERVER_BATCHED */
    gdgs_mg_params mg;    /* solver parameters of every request; flags 0 or
                             GDGS_MG_NEUMANN (then requests take no boundary) */
} gdgs_server_params;

typedef struct gdgs_request {
    gdgs_camera cam;        /* image size and pose */
    const float* boundary;  /* device [3][H][W], ring read; NULL = zero ring */
    float* u;               /* device [3][H][W], receives the reconstruction */
    uint64_t tag;           /* caller's value, returned in the completion */
    int64_t arrival_ns;     /* gdgs_now_ns() time before which the request is not
                               started; 0 = on submission */
    const float* u_init;    /* device [3][H][W] or NULL: the solve starts from this
                               image's interior instead of zero (GDGS_MG_WARM_START),
                               e.g. the previous view of a moving camera, which needs
                               fewer V-cycles; read when the request starts (and again
                               on a capacity re-run), so it must stay unchanged until
                               the completion arrives.  May be the request's own u. */
} gdgs_request;

typedef struct gdgs_completion {
    int64_t id;          /* from gdgs_server_submit */
    uint64_t tag;
    int32_t status;      /* GDGS_OK, GDGS_ERR_CANCELLED, GDGS_ERR_BUDGET or GDGS_ERR_HIP */
    int32_t converged;   /* every channel met mg.tol */
    int32_t cycles;      /* V-cycles of the slowest channel */
    int32_t attempts;    /* admissions (2 or more after a capacity re-run) */
    int64_t num_pairs;   /* (tile, splat) pairs of the view */
    int64_t arrival_ns;  /* scheduled (or submission) time */
    int64_t admit_ns;    /* first start */
    int64_t done_ns;     /* completion seen by the scheduler */
} gdgs_completion;

typedef struct gdgs_server_state {
    int64_t budget_bytes, used_bytes, peak_bytes; /* arena size, in use (incl. idle slots), peak */
    int64_t submitted, completed;
    int32_t waiting, running, idle_slots, streams;
} gdgs_server_state;

/* Steady-clock nanoseconds, the time base of arrival and completion times. */
int64_t gdgs_now_ns(void);
/* Creates the server on the current device (allocates the budget, the
 * streams and the scheduler thread).  scene: device arrays, kept by pointer. */
gdgs_status gdgs_server_create(const gdgs_scene* scene, const gdgs_server_params* params,
                               gdgs_server** out);
/* Queues a request; *id identifies it.  GDGS_ERR_BUDGET if its state can
 * never fit the budget, GDGS_ERR_INVALID_ARGUMENT for a bad camera or
 * buffer. */
gdgs_status gdgs_server_submit(gdgs_server* srv, const gdgs_request* req, int64_t* id);
/* Moves up to `max` completions into out[0..*n), oldest first, waiting up to
 * wait_us microseconds for the first one (0 = do not wait). */
gdgs_status gdgs_server_poll(gdgs_server* srv, gdgs_completion* out, int32_t max,
                             int32_t wait_us, int32_t* n);
/* A waiting request completes at once with GDGS_ERR_CANCELLED; a running one
 * completes so after its current run.  GDGS_ERR_INVALID_ARGUMENT for an
 * unknown or finished id. */
gdgs_status gdgs_server_cancel(gdgs_server* srv, int64_t id);
gdgs_status gdgs_server_query(gdgs_server* srv, gdgs_server_state* out);
/* Cancels every request (running ones stop after their current run), waits
 * for the device work, frees everything.  Completions not yet polled are
 * dropped. */
gdgs_status gdgs_server_destroy(gdgs_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* GDGS_H */
