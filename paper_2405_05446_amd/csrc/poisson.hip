// Poisson reconstruction of the image from the composited gradients (GDGS
// Sec. 2.1, Eq. 13-16, and Sec. 2.2 "Poisson Equation", Eq. 21; the paper names
// multigrid as a linear-complexity solver).  Discretisation: backward-
// difference divergence of forward-difference gradients, 5-point Laplacian with
// unit spacing, unknowns on the interior pixels, Dirichlet values on the ring.
//
// Multigrid: vertex-centred grids, coarse point I <-> fine point 2I, n_c =
// floor(n/2) interior points per axis (for even n the coarse boundary sits one
// fine cell beyond the fine one).  Each grid keeps the distance delta (in its
// own spacing) from its last interior row/column to the true boundary: 1 on the
// finest grid, (1 + delta)/2 after an odd count, delta/2 after an even one.
// Where delta < 1 the Dirichlet condition is imposed through a linearly
// extrapolated ghost value u_ghost = u (1 - 1/delta), i.e. the diagonal of the
// last row/column grows by 1/delta - 1 (for delta = 1/2 this is exactly the
// Galerkin coarse operator of the 1D problem), and prolongation onto a fine
// point between the last coarse point and the boundary uses the matching
// linear weight 1 - 1/(2 delta).  V(pre, post) cycles: red-black Gauss-Seidel
// (pre sweeps red then black), full-weighting restriction of the residual
// (coarse right-hand side = 4 x full weighting, the unit-spacing scaling of a
// grid twice as coarse), bilinear prolongation, SOR on the coarsest grid.
// Post sweeps: red then black too for the Dirichlet problem (in the reverse
// order they would end on red and the next cycle's first red half-sweep
// would change nothing; the V(2,2) contraction is about 0.06 per cycle this
// way against 0.13); black then red for the Neumann problem, which needed
// fewer cycles that way on rendered frames (10.6 against 12.2 at 1080p).
//
// Kernels:
//  * finest grid (k_fine_pre, k_fine_post): register strips.  A block of four
//    waves holds 48 rows x 128 columns of the grid in VGPRs (12 rows per wave,
//    two adjacent columns per lane); column neighbours come from DPP lane
//    shifts, the rows above and below a wave are exchanged through LDS after
//    every half-sweep.  The pre pass does its sweeps, writes the smoothed
//    iterate to the second buffer, evaluates the residual in FP64 registers
//    and writes its full-weighting restriction; the post pass adds the
//    bilinear interpolation of the coarse correction, smooths and takes the
//    residual, iterate and correction norms of the cycle (one partial per
//    block).  Smoothing is FP32; residuals on this grid are FP64, because near
//    convergence the FP32 cancellation noise of f - (sum of neighbours - 4u)
//    would otherwise be fed to the coarse grids as spurious corrections;
//  * coarse grids too large for one workgroup (k_mg_pre, k_mg_post): 32 x 16
//    tiles loaded once with a halo of 2*sweeps+2 into LDS, all sweeps in LDS
//    (temporal blocking: the valid region shrinks by one cell per half-sweep),
//    so each pass reads u and f once and writes u (and the coarse right-hand
//    side) once;
//  * the coarse grids that fit in LDS together are run as a whole V-cycle by
//    a single workgroup per channel (k_mg_lds: no launches per coarse level);
//  * a finalize kernel per cycle (k_cycle_finalize) combines the partials of
//    each channel and applies the stopping rule: the cycle's largest change
//    of u against the largest |u| (or, under GDGS_MG_STOP_ETA, the normwise
//    backward error of the residual); a finished channel raises a device flag
//    and every later kernel of that channel returns at once, so no host
//    synchronisation is needed.
#include <cstring>
#include <functional>

#include "graph.hpp"
#include "internal.hpp"

namespace gdgs {
namespace {

// Tiles of the grid kernels: 64 x 32 where the grid is large; 32 x 16 on
// grids too small to fill the chip with 64 x 32 tiles, whose kernels are
// bound by the latency of one block's chain of phases rather than by
// bandwidth (a smaller tile shortens that chain).
constexpr int kTX = 64, kTY = 32;
constexpr int kTXs = 32, kTYs = 16;
constexpr int kTXf = 32, kTYf = 32;   // finest grid
constexpr int kNTf = 256, kNTs = 256; // threads per block: finest grid, small tiles
constexpr int kSmallTileBelow = 4096; // blocks of 64 x 32 under which small tiles are used
constexpr int kLdsTopCells = 4096;    // largest grid solved inside one workgroup
// Default over-relaxation of the red-black smoothing sweeps.  Over-relaxing
// red-black Gauss-Seidel improves its smoothing of the 5-point Laplacian
// (Yavneh, SIAM J. Sci. Comput. 17, 1996); with two pre- and two post-sweeps,
// 1.15 takes the Dirichlet V-cycle's contraction from about 0.06 to about
// 0.02 (an FP64 emulation of this cycle at 62^2 .. 1078 x 1918; 1.1 and 1.2
// lie between), so the 1e-6 relative-correction stop comes one cycle sooner
// (5 instead of 6 at 1080p).  The Neumann cycle gains little (10.3 -> 10).
constexpr float kSmoothW = 1.15f;
constexpr int kDivTX = 64;
constexpr int kDivTY = 4;     // threads per block = kDivTX * kDivTY
constexpr int kDivRows = 16;  // rows per block of the divergence kernel
constexpr int kLdsThreads = 1024;
constexpr int kCounters = 72; // [0] setup, [1 + cycle] cycle finalize, [kLaunch0 + c] below
constexpr int kLaunch0 = 68;   // per-channel count of cycle-finalize launches in this call

struct LevelDev {
    float* u;        // [3][n+2][pitch] iterate at the start and end of a cycle
    float* ub;       // second buffer of the same shape: the pre-smoothing pass
                     // reads u and writes ub, the post pass reads ub and writes
                     // u, so no workgroup reads cells another one is updating
    const float* f;  // right-hand side, same layout
    float* fw;       // writable alias of f (coarse levels)
    int n, m, pitch;
    long long cs;    // channel stride (floats)
    float ey, ex;    // extra diagonal on the last interior row / column (1/delta - 1)
    float wy, wx;    // prolongation weight onto a fine point beyond the last row / column
    float sw;        // over-relaxation weight of the smoothing sweeps (1: Gauss-Seidel)
    // Neumann, finest grid: per channel, the mean that the FP32 right-hand side
    // keeps after centring (below its rounding); subtracted from every FP64
    // residual so that the residual has zero sum, as the singular coarse
    // problems need.  Null otherwise.
    const double* fofs;
};

// Neumann boundary terms, the same on every grid (kernels take them under
// their compile-time switch NM; the Dirichlet problem has none).  A pixel on
// the border has one neighbour fewer: the diagonal drops by one per missing
// neighbour.  Coarse point I sits on fine point 2I, so the first fine point
// (and the last one when the count n is odd) lies outside the coarse points
// and takes the nearest one's value (prolongation weight 1); restriction is
// the transpose of that prolongation, i.e. the residual of such a point counts
// twice in full weighting, which keeps the sum of the coarse right-hand side
// equal to the sum of the fine residual.
constexpr float kNmDiag = -1.f;  // extra diagonal on a first or last row / column
constexpr float kNmW = 1.f;      // prolongation weight onto a fine point outside the coarse points
__device__ __forceinline__ float nm_scale(int g, int n) {
    return (g == 1 || (g == n && (n & 1))) ? 2.f : 1.f;
}

// First colour of a post-smoothing sweep (0 red, 1 black): NM, the Neumann
// problem (see the file comment).
template <bool NM>
constexpr int kPost0 = NM ? 1 : 0;

// Diagonal of the (possibly boundary-modified) 5-point operator at (gi, gj).
__device__ __forceinline__ float diag_at(int gi, int gj, int n, int m, float ey, float ex,
                                         float ey0, float ex0) {
    float d = 4.f;
    if (gi == 1) d += ey0;
    if (gj == 1) d += ex0;
    if (gi == n) d += ey;
    if (gj == m) d += ex;
    return d;
}

// Gauss-Seidel value (sum of the four neighbours - f) / diagonal.
__device__ __forceinline__ float gs_value(float a, float b, float c, float e, float f, float d) {
    const float x = ((a + b) + (c + e)) - f;
    return d == 4.f ? 0.25f * x : x / d;
}

// Residual f - (neighbours - d u) in FP64 registers (see the file comment).
__device__ __forceinline__ double res_value(float a, float b, float c, float e, float u, float f,
                                            float d) {
    const double nb = ((double)a + (double)b) + ((double)c + (double)e);
    return (double)f - (nb - (double)d * (double)u);
}

struct LdsPlan {
    int lc, L;
    int lw;                // levels lw .. L-1 are run by one wave (lw == L: none)
    int n[kMaxLevels], m[kMaxLevels];
    int M[kMaxLevels];     // row pitch of grid l in LDS (see lds_pitch)
    float ey[kMaxLevels], ex[kMaxLevels], wy[kMaxLevels], wx[kMaxLevels];
    const double* fofs;    // offset of the finest grid's residual (see LevelDev), or null
    int off[kMaxLevels];   // float offset of u_l in LDS; f_l follows u_l
    int roff[kMaxLevels];  // float offset of the residual of level l (l < L-1)
    uint32_t mg_m[kMaxLevels], mg_h[kMaxLevels];  // division magics for m and (m+1)/2
    int zero0, zero1;      // float range cleared at entry: coarse grids and residuals
    int trash;             // float offset of 64 cells that take the stores of unused slots
    int pre, post, csweeps;
    float omega;           // SOR factor of the coarsest grid's sweeps
    float sw;              // over-relaxation weight of the other grids' sweeps
    LevelDev top;          // global arrays of level lc
};

__device__ __forceinline__ double wave_max_d(double x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x = fmax(x, __shfl_xor(x, d, 64));
    return x;
}
__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

// Block-wide (max, max, sum) of three doubles; result valid in thread 0.
__device__ void block_reduce3(double& a, double& b, double& s, double* sh /*[3*nwaves]*/) {
    const int lane = __lane_id(), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    a = wave_max_d(a);
    b = wave_max_d(b);
    s = wave_sum_d(s);
    if (lane == 0) {
        sh[3 * w] = a;
        sh[3 * w + 1] = b;
        sh[3 * w + 2] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < nw; ++i) {
            a = fmax(a, sh[3 * i]);
            b = fmax(b, sh[3 * i + 1]);
            s += sh[3 * i + 2];
        }
    }
    __syncthreads();
}

// After the last cycle of a call (on the caller's stream, behind every
// channel's work): whether all three channels met the tolerance.
__global__ void k_publish_converged(const int* __restrict__ done, gdgs_stats* __restrict__ stats) {
    if (threadIdx.x == 0) stats->converged = done[0] && done[1] && done[2];
}

// ---------------------------------------------------------------- setup
// rho (from the gradients or given), the level-0 right-hand side f0, the
// initial u0 (ring = boundary, interior 0 unless warm), and per-block
// max|b|, sum b^2 with b = -rho + ring neighbours.
// ranges (rho given, or null): the [2][T] tile pair ranges of the composite
// that produced rho; a tile without pairs holds exact zeros and is not read.
__global__ __launch_bounds__(kDivTX* kDivTY) void k_div_init(
    const float* __restrict__ grad, const float* __restrict__ rho_in,
    const float* __restrict__ boundary, int H, int W, float* __restrict__ f0,
    float* __restrict__ u0, double* __restrict__ bpart, int* __restrict__ counters, int warm,
    const uint32_t* __restrict__ ranges = nullptr) {
    __shared__ double sh[3 * 4];
    const int c = blockIdx.z;
    if (blockIdx.x == 0 && blockIdx.y == 0 && c == 0 && threadIdx.x < kCounters)
        counters[threadIdx.x] = 0;
    const int j = blockIdx.x * kDivTX + (threadIdx.x % kDivTX);
    const size_t HW = (size_t)H * W;
    double bmax = 0.0, bdum = 0.0, bss = 0.0;
    constexpr int R = kDivRows / kDivTY;
    // all of a thread's loads first (addresses clamped into the image; values
    // of cells off the image or on the ring are not used), then the stores
    float ld[R][4];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = blockIdx.y * kDivRows + k * kDivTY + (threadIdx.x / kDivTX);
        const int ic = min(max(i, 1), H - 1), jc = min(max(j, 1), W - 1);
        const size_t p = (size_t)ic * W + jc;
        if (grad) {
            const float* gx = grad + (size_t)(2 * c) * HW;
            const float* gy = grad + (size_t)(2 * c + 1) * HW;
            ld[k][0] = gx[p];
            ld[k][1] = gx[p - 1];
            ld[k][2] = gy[p];
            ld[k][3] = gy[p - W];
        } else if (ranges) {
            const int ntx = (W + kTile - 1) / kTile, T = ntx * ((H + kTile - 1) / kTile);
            const int tile = (ic / kTile) * ntx + jc / kTile;
            ld[k][0] = ranges[tile] != ranges[T + tile] ? rho_in[(size_t)c * HW + p] : 0.f;
            ld[k][1] = ld[k][2] = ld[k][3] = 0.f;
        } else {
            ld[k][0] = rho_in[(size_t)c * HW + p];
            ld[k][1] = ld[k][2] = ld[k][3] = 0.f;
        }
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = blockIdx.y * kDivRows + k * kDivTY + (threadIdx.x / kDivTX);
        if (i >= H || j >= W) continue;
        const size_t o = (size_t)c * HW + (size_t)i * W + j;
        const bool ring = (i == 0) || (i == H - 1) || (j == 0) || (j == W - 1);
        if (ring) {
            u0[o] = boundary ? boundary[o] : 0.f;
            if (f0) f0[o] = 0.f;
        } else {
            const float rho =
                grad ? (ld[k][0] - ld[k][1]) + (ld[k][2] - ld[k][3]) : ld[k][0];
            if (f0) f0[o] = rho;
            if (!warm) u0[o] = 0.f;
            double b = -(double)rho;
            if (boundary) {
                const float* g = boundary + (size_t)c * HW;
                if (i == 1) b += g[(size_t)j];
                if (i == H - 2) b += g[(size_t)(H - 1) * W + j];
                if (j == 1) b += g[(size_t)i * W];
                if (j == W - 2) b += g[(size_t)i * W + W - 1];
            }
            bmax = fmax(bmax, fabs(b));
            bss += b * b;
        }
    }
    block_reduce3(bmax, bdum, bss, sh);
    if (threadIdx.x == 0) {
        const int nblk = gridDim.x * gridDim.y;
        const int blk = blockIdx.y * gridDim.x + blockIdx.x;
        bpart[((size_t)c * nblk + blk) * 2] = bmax;
        bpart[((size_t)c * nblk + blk) * 2 + 1] = bss;
    }
}

// One block per channel.
__global__ __launch_bounds__(256) void k_setup_finalize(const double* __restrict__ bpart, int nblk,
                                                        double* __restrict__ bnorm,
                                                        int* __restrict__ done,
                                                        int* __restrict__ counters,
                                                        gdgs_stats* __restrict__ stats,
                                                        int warm) {
    __shared__ double sh[3 * 4];
    const int c = blockIdx.x;
    double mx = 0.0, dum = 0.0, ss = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
        mx = fmax(mx, bpart[((size_t)c * nblk + b) * 2]);
        ss += bpart[((size_t)c * nblk + b) * 2 + 1];
    }
    block_reduce3(mx, dum, ss, sh);
    if (threadIdx.x == 0) {
        bnorm[2 * c] = mx;
        bnorm[2 * c + 1] = sqrt(ss);
        // zero right-hand side and zero initial interior: already exact
        const int d = (mx == 0.0) && !warm;
        done[c] = d;
        stats->cycles[c] = 0;
        stats->eta[c] = d ? 0.0 : 1.0;
        stats->rel_res[c] = d ? 0.0 : 1.0;
        stats->delta[c] = d ? 0.0 : 1.0;
        stats->b_norm[c] = sqrt(ss);
    }
}

// ---------------------------------------------------------------- Neumann set-up and gauge
// The Neumann problem keeps its finest grid in padded workspace arrays: pixel
// (i, j) at (i + 1, j + 1), a zero ring around the H x W pixels.  The kernels
// below cover the padded grid with the block shape of k_div_init.

// Sum of a block's doubles into thread 0 (any block size that is a multiple of 64).
__device__ double block_sum(double v, double* sh /*[3 * nwaves]*/) {
    double a = 0.0, b = 0.0;
    block_reduce3(a, b, v, sh);
    return v;
}

// rho on every pixel (the backward-difference divergence of the forward
// differences inside the image, or given), f0 = rho, u0 = 0 or the caller's
// image, zero rings in u0, u0b and f0; per-block sum of rho.
__global__ __launch_bounds__(kDivTX* kDivTY) void k_nm_init(
    const float* __restrict__ grad, const float* __restrict__ rho_in,
    const float* __restrict__ uprev, int H, int W, int pitch, float* __restrict__ f0,
    float* __restrict__ u0, float* __restrict__ u0b, double* __restrict__ bpart,
    int* __restrict__ counters) {
    __shared__ double sh[3 * 4];
    const int c = blockIdx.z;
    if (blockIdx.x == 0 && blockIdx.y == 0 && c == 0 && threadIdx.x < kCounters)
        counters[threadIdx.x] = 0;
    const int pj = blockIdx.x * kDivTX + (threadIdx.x % kDivTX);
    const size_t HW = (size_t)H * W, cs = (size_t)(H + 2) * pitch;
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < kDivRows / kDivTY; ++k) {
        const int pi = blockIdx.y * kDivRows + k * kDivTY + (threadIdx.x / kDivTX);
        if (pi >= H + 2 || pj >= W + 2) continue;
        const size_t po = (size_t)c * cs + (size_t)pi * pitch + pj;
        const int i = pi - 1, j = pj - 1;
        if (i < 0 || i >= H || j < 0 || j >= W) {
            f0[po] = 0.f;
            u0[po] = 0.f;
            u0b[po] = 0.f;
            continue;
        }
        const size_t p = (size_t)i * W + j;
        float rho;
        if (grad) {
            const float* gx = grad + (size_t)(2 * c) * HW;
            const float* gy = grad + (size_t)(2 * c + 1) * HW;
            const float ax = j < W - 1 ? gx[p] : 0.f, bx = j > 0 ? gx[p - 1] : 0.f;
            const float ay = i < H - 1 ? gy[p] : 0.f, by = i > 0 ? gy[p - W] : 0.f;
            rho = (ax - bx) + (ay - by);
        } else {
            rho = rho_in[(size_t)c * HW + p];
        }
        f0[po] = rho;
        u0[po] = uprev ? uprev[(size_t)c * HW + p] : 0.f;
        sum += (double)rho;
    }
    sum = block_sum(sum, sh);
    if (threadIdx.x == 0) {
        const int nblk = gridDim.x * gridDim.y;
        bpart[((size_t)c * nblk + blockIdx.y * gridDim.x + blockIdx.x) * 2] = sum;
    }
}

// One block per channel: out[c] = scale * (sum of the per-block values, which
// are stride doubles apart).
__global__ __launch_bounds__(256) void k_nm_mean(const double* __restrict__ bpart, int nblk,
                                                 int stride, double scale,
                                                 double* __restrict__ out) {
    __shared__ double sh[3 * 4];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x)
        s += bpart[((size_t)c * nblk + b) * stride];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[c] = s * scale;
}

// f0 <- f0 - mean (the compatible part of rho, to FP32 rounding); per-block
// max|b| and sum b^2 of b = mean - rho (the form k_setup_finalize reduces), and
// the per-block sum of the centred FP32 values (spart).
__global__ __launch_bounds__(kDivTX* kDivTY) void k_nm_center(float* __restrict__ f0, int H,
                                                              int W, int pitch,
                                                              const double* __restrict__ mean,
                                                              double* __restrict__ bpart,
                                                              double* __restrict__ spart) {
    __shared__ double sh[3 * 4];
    const int c = blockIdx.z;
    const int pj = blockIdx.x * kDivTX + (threadIdx.x % kDivTX);
    const size_t cs = (size_t)(H + 2) * pitch;
    const float mu = (float)mean[c];
    double bmax = 0.0, bdum = 0.0, bss = 0.0;
#pragma unroll
    for (int k = 0; k < kDivRows / kDivTY; ++k) {
        const int pi = blockIdx.y * kDivRows + k * kDivTY + (threadIdx.x / kDivTX);
        if (pi < 1 || pi > H || pj < 1 || pj > W) continue;
        float* f = f0 + (size_t)c * cs + (size_t)pi * pitch + pj;
        const float v = *f - mu;
        *f = v;
        bmax = fmax(bmax, fabs((double)v));
        bss += (double)v * (double)v;
        bdum += (double)v;
    }
    double x0 = 0.0;
    block_reduce3(bmax, x0, bss, sh);
    bdum = block_sum(bdum, sh);
    if (threadIdx.x == 0) {
        const int nblk = gridDim.x * gridDim.y;
        const int blk = blockIdx.y * gridDim.x + blockIdx.x;
        bpart[((size_t)c * nblk + blk) * 2] = bmax;
        bpart[((size_t)c * nblk + blk) * 2 + 1] = bss;
        spart[(size_t)c * nblk + blk] = bdum;
    }
}

// Per-block sum of the solution over the pixels.
__global__ __launch_bounds__(kDivTX* kDivTY) void k_nm_usum(const float* __restrict__ u0, int H,
                                                            int W, int pitch,
                                                            double* __restrict__ bpart) {
    __shared__ double sh[3 * 4];
    const int c = blockIdx.z;
    const int pj = blockIdx.x * kDivTX + (threadIdx.x % kDivTX);
    const size_t cs = (size_t)(H + 2) * pitch;
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < kDivRows / kDivTY; ++k) {
        const int pi = blockIdx.y * kDivRows + k * kDivTY + (threadIdx.x / kDivTX);
        if (pi < 1 || pi > H || pj < 1 || pj > W) continue;
        sum += (double)u0[(size_t)c * cs + (size_t)pi * pitch + pj];
    }
    sum = block_sum(sum, sh);
    if (threadIdx.x == 0) {
        const int nblk = gridDim.x * gridDim.y;
        bpart[((size_t)c * nblk + blockIdx.y * gridDim.x + blockIdx.x) * 2] = sum;
    }
}

// The caller's image: the pixels of the padded solution minus its mean.
__global__ __launch_bounds__(kDivTX* kDivTY) void k_nm_out(const float* __restrict__ u0, int H,
                                                           int W, int pitch,
                                                           const double* __restrict__ mean,
                                                           float* __restrict__ u) {
    const int c = blockIdx.z;
    const int j = blockIdx.x * kDivTX + (threadIdx.x % kDivTX);
    const size_t cs = (size_t)(H + 2) * pitch, HW = (size_t)H * W;
    const float mu = (float)mean[c];
#pragma unroll
    for (int k = 0; k < kDivRows / kDivTY; ++k) {
        const int i = blockIdx.y * kDivRows + k * kDivTY + (threadIdx.x / kDivTX);
        if (i >= H || j >= W) continue;
        u[(size_t)c * HW + (size_t)i * W + j] =
            u0[(size_t)c * cs + (size_t)(i + 1) * pitch + j + 1] - mu;
    }
}

// Start of a resumed solve: only the per-call finalize counters restart.
__global__ void k_resume(int* __restrict__ counters) {
    if (threadIdx.x < kCounters) counters[threadIdx.x] = 0;
}

// ---------------------------------------------------------------- smoothing
// Red-black Gauss-Seidel half-sweeps on an LDS region RX x RY whose cell (0,0)
// is grid point (gi0, gj0); only interior grid points (1..n, 1..m) change.
// Thread t owns LDS row 1 + t / TPR and every TPR-th point of one colour in
// it, KR points per colour.  A half-sweep loads the neighbours of all of a
// thread's points before it stores any (points of one colour read only the
// other colour); a slot off the row reads cell (1, 1) and stores to the
// thread's trash cell, so no access is conditional.
template <int RX, int RY, int NT, bool NM>
__device__ __forceinline__ void smooth_rows(float* __restrict__ su, const float* __restrict__ sf,
                                            float* trash, int gi0, int gj0, const LevelDev& L,
                                            int color0, int sweeps) {
    const int n = L.n, m = L.m;
    constexpr int NR = RY - 2;
    constexpr int TPR = NT / NR;
    constexpr int KR = ((RX - 1) / 2 + TPR - 1) / TPR;
    const int t = threadIdx.x;
    const int r = 1 + t / TPR, sgm = t % TPR;
    const int gi = gi0 + r;
    const bool row_ok = (t < NR * TPR) && gi >= 1 && gi <= n;
    const int qlo = max(1, 1 - gj0), qhi = min(RX - 2, m - gj0);
    const int qm = m - gj0, q1 = 1 - gj0;  // local columns of the last / first interior column
    float drow = 4.f + (gi == n ? L.ey : 0.f);
    if (NM && gi == 1) drow += kNmDiag;
    const float cw = 1.f - L.sw;  // u <- (1 - w) u + w (Gauss-Seidel value)
    int ro[2][KR];
    float* wo[2][KR];
    float rd[2][KR];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int q0 = qlo + ((c + gi + gj0 + qlo) & 1) + 2 * sgm;
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int q = q0 + 2 * TPR * k;
            const bool ok = row_ok && q <= qhi;
            ro[c][k] = ok ? r * RX + q : RX + 1;
            wo[c][k] = ok ? su + r * RX + q : trash;
            float dq = q == qm ? drow + L.ex : drow;
            if (NM && q == q1) dq += kNmDiag;
            rd[c][k] = L.sw / dq;
        }
    }
    auto half = [&](const int* o, float* const* w, const float* d) {
        float v[KR];
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int q = o[k];
            v[k] = fmaf(cw, su[q],
                        (((su[q - RX] + su[q + RX]) + (su[q - 1] + su[q + 1])) - sf[q]) * d[k]);
        }
#pragma unroll
        for (int k = 0; k < KR; ++k) *w[k] = v[k];
        __syncthreads();
    };
    for (int s = 0; s < sweeps; ++s) {
        if (color0 == 0) {
            half(ro[0], wo[0], rd[0]);
            half(ro[1], wo[1], rd[1]);
        } else {
            half(ro[1], wo[1], rd[1]);
            half(ro[0], wo[0], rd[0]);
        }
    }
}

// A thread's share of an RY x RX region of a grid (cell (0,0) = grid point
// (gi0, gj0)), held in registers: every global load is issued before the
// first one is waited for, then stored to LDS (zero outside the grid).
template <int RX, int RY, int NT>
struct RegionRegs {
    static constexpr int NI = (RY * RX + NT - 1) / NT;
    float a[NI], b[NI];
    // a <- x, b <- y (y may be null: b unused)
    __device__ __forceinline__ void load(const LevelDev& L, const float* x, const float* y, int c,
                                         int gi0, int gj0) {
        const int N = L.n + 2, M = L.m + 2;
        const float* xc = x ? x + (size_t)c * L.cs : nullptr;
        const float* yc = y ? y + (size_t)c * L.cs : nullptr;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int idx = threadIdx.x + k * NT;
            const int r = idx / RX, q = idx - r * RX;
            const int gi = gi0 + r, gj = gj0 + q;
            const bool in =
                idx < RY * RX && (unsigned)gi < (unsigned)N && (unsigned)gj < (unsigned)M;
            const size_t o = (size_t)gi * L.pitch + gj;
            a[k] = (in && xc) ? xc[o] : 0.f;
            b[k] = (in && yc) ? yc[o] : 0.f;
        }
    }
    __device__ __forceinline__ void store(float* sa, float* sb) const {
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int idx = threadIdx.x + k * NT;
            if (idx < RY * RX) {
                sa[idx] = a[k];
                if (sb) sb[idx] = b[k];
            }
        }
    }
};

// Logical (tile x, tile y, channel) of this block under the XCD remap; the
// launch covers channels c0 .. c0 + gridDim.z - 1.
struct TileId {
    int tx, ty, c;
    __device__ TileId(int tx_, int ty_, int c_) : tx(tx_), ty(ty_), c(c_) {}
    __device__ explicit TileId(int c0) {
        const int gx = gridDim.x, gy = gridDim.y;
        const int nb = gx * gy * gridDim.z;
        const int b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
        const int L = xcd_remap(b, nb);
        const int cz = L / (gx * gy);
        const int rem = L - cz * gx * gy;
        c = c0 + cz;
        ty = rem / gx;
        tx = rem - ty * gx;
    }
};

// Thread t of an NT-thread block owns the tile cells t, t + NT, ...

// Pre-smoothing + residual + restriction to the next grid.  FINE (the finest
// grid only): record the largest change of u and evaluate the residual in
// FP64; coarser grids carry small corrections and stay in FP32.  A finished
// channel returns at once on the finest grid; on coarser grids, whose blocks
// are few and latency-bound, the done flag is read together with the tile.
template <int NU, bool FINE, int TX, int TY, int NT, bool NM>
__device__ __forceinline__ void mg_pre_tile(const LevelDev& L, const LevelDev& C, int zero_guess,
                                            const int* __restrict__ done,
                                            double* __restrict__ part, const TileId id, int gx,
                                            int gy) {
    constexpr int HALO = 2 * NU + 2;
    constexpr int CPT = TX * TY / NT;
    constexpr int RX = TX + 2 * HALO, RY = TY + 2 * HALO;
    __shared__ float su[RY * RX];
    __shared__ float sf[RY * RX];
    __shared__ float s_trash[NT];
    __shared__ double sh[3 * (NT / 64)];
    const int c = id.c;
    if (FINE && done[c]) return;
    const int dn = FINE ? 0 : done[c];
    const int gi0 = id.ty * TY - HALO, gj0 = id.tx * TX - HALO;
    {
        RegionRegs<RX, RY, NT> reg;
        reg.load(L, zero_guess ? nullptr : L.u, L.f, c, gi0, gj0);
        if (dn) return;
        reg.store(su, sf);
    }
    __syncthreads();
    float before[CPT];
    if (FINE) {
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int idx = threadIdx.x + NT * k;
            before[k] = su[(HALO + idx / TX) * RX + HALO + idx % TX];
        }
        __syncthreads();  // every snapshot is taken before any cell changes
    }
    smooth_rows<RX, RY, NT, NM>(su, sf, s_trash + threadIdx.x, gi0, gj0, L, 0, NU);
    const int N = L.n + 2, M = L.m + 2;
    float* u = L.ub + (size_t)c * L.cs;
    double dmax = 0.0;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        const int idx = threadIdx.x + NT * k;
        const int r = HALO + idx / TX, q = HALO + idx % TX;
        const int gi = gi0 + r, gj = gj0 + q;
        if (gi < N && gj < M) {
            const float v = su[r * RX + q];
            u[(size_t)gi * L.pitch + gj] = v;
            if (FINE && gi >= 1 && gi <= L.n && gj >= 1 && gj <= L.m)
                dmax = fmax(dmax, fabs((double)v - (double)before[k]));
        }
    }
    // residual on rows/cols [HALO-1, HALO+T-1], zero off the interior; thread t
    // owns every TPR-th cell of one row (all loads before the stores: each
    // cell's residual overwrites only its own f)
    {
        constexpr int ZR = TY + 1, ZC = TX + 1;
        constexpr int TPR = NT / ZR;
        constexpr int KZ = (ZC + TPR - 1) / TPR;
        const int t = threadIdx.x;
        const int r = HALO - 1 + t / TPR;
        const int gi = gi0 + r;
        const bool row_in = t < ZR * TPR && gi >= 1 && gi <= L.n;
        float drow = 4.f + (gi == L.n ? L.ey : 0.f);
        if (NM && gi == 1) drow += kNmDiag;
        const float srow = NM ? nm_scale(gi, L.n) : 1.f;
        float rv[KZ];
        float* dst[KZ];
#pragma unroll
        for (int k = 0; k < KZ; ++k) {
            const int q = HALO - 1 + t % TPR + TPR * k;
            const int gj = gj0 + q;
            const bool live = t < ZR * TPR && q < HALO - 1 + ZC;
            const bool in = live && row_in && gj >= 1 && gj <= L.m;
            const int o = live ? r * RX + q : RX + 1;
            float d = gj == L.m ? drow + L.ex : drow;
            if (NM && gj == 1) d += kNmDiag;
            float v;
            if (FINE)
                v = (float)res_value(su[o - RX], su[o + RX], su[o - 1], su[o + 1], su[o], sf[o],
                                     d);
            else
                v = sf[o] - (((su[o - RX] + su[o + RX]) + (su[o - 1] + su[o + 1])) - d * su[o]);
            rv[k] = in ? (NM ? v * (srow * nm_scale(gj, L.m)) : v) : 0.f;
            dst[k] = live ? sf + o : s_trash + t;
        }
#pragma unroll
        for (int k = 0; k < KZ; ++k) *dst[k] = rv[k];
    }
    __syncthreads();
    const int I0 = id.ty * (TY / 2), J0 = id.tx * (TX / 2);
    float* fc = C.fw + (size_t)c * C.cs;
    for (int idx = threadIdx.x; idx < (TY / 2) * (TX / 2); idx += blockDim.x) {
        const int I = I0 + idx / (TX / 2), J = J0 + idx % (TX / 2);
        if (I >= 1 && I <= C.n && J >= 1 && J <= C.m) {
            const int o = (2 * I - gi0) * RX + (2 * J - gj0);
            const float v = 4.f * sf[o] + 2.f * (sf[o - 1] + sf[o + 1] + sf[o - RX] + sf[o + RX]) +
                            (sf[o - RX - 1] + sf[o - RX + 1] + sf[o + RX - 1] + sf[o + RX + 1]);
            fc[(size_t)I * C.pitch + J] = 0.25f * v;
        }
    }
    if (FINE) {
        double d1 = 0.0, d2 = 0.0;
        block_reduce3(dmax, d1, d2, sh);
        if (threadIdx.x == 0) {
            const int nblk = gx * gy;
            part[((size_t)c * nblk + id.ty * gx + id.tx) * 5 + 3] = dmax;
        }
    }
}

template <int NU, bool FINE, int TX, int TY, int NT, bool NM>
__global__ __launch_bounds__(NT) void k_mg_pre(LevelDev L, LevelDev C, int zero_guess,
                                                const int* __restrict__ done,
                                                double* __restrict__ part, int c0) {
    mg_pre_tile<NU, FINE, TX, TY, NT, NM>(L, C, zero_guess, done, part, TileId(c0), gridDim.x,
                                          gridDim.y);
}

// Prolongation + correction + post-smoothing.  FINE (the finest grid only):
// also the residual and correction norms of the cycle.  The done flag is
// handled as in k_mg_pre.
template <int NU, bool FINE, int TX, int TY, int NT, bool NM>
__device__ __forceinline__ void mg_post_tile(const LevelDev& L, const LevelDev& C,
                                             const int* __restrict__ done,
                                             double* __restrict__ part, const TileId id, int gx,
                                             int gy) {
    constexpr bool NORM = FINE;
    constexpr int HALO = 2 * NU + 2;
    constexpr int CPT = TX * TY / NT;
    constexpr int RX = TX + 2 * HALO, RY = TY + 2 * HALO;
    constexpr int CX = RX / 2 + 2, CY = RY / 2 + 2;  // staged coarse tile
    __shared__ float su[RY * RX];
    __shared__ float sf[RY * RX];
    __shared__ float se[CY * CX];
    __shared__ float s_trash[NT];
    __shared__ double sh[3 * (NT / 64)];
    const int c = id.c;
    if (FINE && done[c]) return;
    const int dn = FINE ? 0 : done[c];
    const int gi0 = id.ty * TY - HALO, gj0 = id.tx * TX - HALO;
    // coarse rows (gi0 >> 1) .. ((gi0 + RY - 1) >> 1) + 1, columns alike
    const int ci0 = gi0 >> 1, cj0 = gj0 >> 1;
    {
        RegionRegs<RX, RY, NT> reg;
        reg.load(L, L.ub, L.f, c, gi0, gj0);
        const float* e = C.u + (size_t)c * C.cs;
        const int NC = C.n + 2, MC = C.m + 2;
        constexpr int NE = (CY * CX + NT - 1) / NT;
        float ve[NE];
#pragma unroll
        for (int k = 0; k < NE; ++k) {
            const int idx = threadIdx.x + k * NT;
            const int a = idx / CX, b = idx - a * CX;
            const int I = ci0 + a, J = cj0 + b;
            ve[k] = (idx < CY * CX && (unsigned)I < (unsigned)NC && (unsigned)J < (unsigned)MC)
                        ? e[(size_t)I * C.pitch + J]
                        : 0.f;
        }
        if (dn) return;
        reg.store(su, sf);
#pragma unroll
        for (int k = 0; k < NE; ++k) {
            const int idx = threadIdx.x + k * NT;
            if (idx < CY * CX) se[idx] = ve[k];
        }
    }
    __syncthreads();
    float before[CPT];
    if (NORM) {
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int idx = threadIdx.x + NT * k;
            before[k] = su[(HALO + idx / TX) * RX + HALO + idx % TX];
        }
        __syncthreads();  // every snapshot is taken before any cell changes
    }
    // bilinear prolongation of the correction onto the interior points of the
    // region (all of a thread's loads before its stores: each point changes
    // only itself)
    {
        constexpr int NI = (RY * RX + NT - 1) / NT;
        float v[NI];
        float* dst[NI];
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int i0 = threadIdx.x + k * NT;
            const bool live = i0 < RY * RX;
            const int idx = live ? i0 : 0;
            const int r = idx / RX, q = idx - r * RX;
            const int gi = gi0 + r, gj = gj0 + q;
            const bool in = gi >= 1 && gi <= L.n && gj >= 1 && gj <= L.m;
            const int oi = gi & 1, oj = gj & 1;
            const int I0 = gi >> 1, J0 = gj >> 1;
            const float* p = se + (I0 - ci0) * CX + (J0 - cj0);
            float w = p[0];
            const float pa = p[CX], pb = p[1], pc = p[CX + 1];
            if (oi) w += pa;
            if (oj) w += pb;
            if (oi & oj) w += pc;
            const float fy = oi ? ((NM && I0 == 0) ? kNmW : (I0 == C.n ? C.wy : 0.5f)) : 1.f;
            const float fx = oj ? ((NM && J0 == 0) ? kNmW : (J0 == C.m ? C.wx : 0.5f)) : 1.f;
            v[k] = su[idx] + fy * fx * w;
            dst[k] = (live && in) ? su + idx : s_trash + threadIdx.x;
        }
#pragma unroll
        for (int k = 0; k < NI; ++k) *dst[k] = v[k];
    }
    __syncthreads();
    smooth_rows<RX, RY, NT, NM>(su, sf, s_trash + threadIdx.x, gi0, gj0, L, kPost0<NM>, NU);
    float* u = L.u + (size_t)c * L.cs;
    const int N = L.n + 2, M = L.m + 2;
    double rmax = 0.0, umax = 0.0, rss = 0.0, dmax = 0.0;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        const int idx = threadIdx.x + NT * k;
        const int r = HALO + idx / TX, q = HALO + idx % TX;
        const int gi = gi0 + r, gj = gj0 + q;
        const int o = r * RX + q;
        // ring cells too: they keep the boundary (or zero) values in both buffers
        if (gi < N && gj < M) u[(size_t)gi * L.pitch + gj] = su[o];
        if (gi >= 1 && gi <= L.n && gj >= 1 && gj <= L.m) {
            const float uv = su[o];
            if (NORM) {
                dmax = fmax(dmax, fabs((double)uv - (double)before[k]));
                const double rv = res_value(su[o - RX], su[o + RX], su[o - 1], su[o + 1], uv,
                                            sf[o], diag_at(gi, gj, L.n, L.m, L.ey, L.ex,
                                                           NM ? kNmDiag : 0.f, NM ? kNmDiag : 0.f));
                rmax = fmax(rmax, fabs(rv));
                umax = fmax(umax, fabs((double)uv));
                rss += rv * rv;
            }
        }
    }
    if (NORM) {
        block_reduce3(rmax, umax, rss, sh);
        double d1 = 0.0, d2 = 0.0;
        block_reduce3(dmax, d1, d2, sh);
        if (threadIdx.x == 0) {
            const int nblk = gx * gy;
            const int blk = id.ty * gx + id.tx;
            double* p = part + ((size_t)c * nblk + blk) * 5;
            p[0] = rmax;
            p[1] = umax;
            p[2] = rss;
            p[4] = dmax;
        }
    }
}

template <int NU, bool FINE, int TX, int TY, int NT, bool NM>
__global__ __launch_bounds__(NT) void k_mg_post(LevelDev L, LevelDev C,
                                                 const int* __restrict__ done,
                                                 double* __restrict__ part, int c0) {
    mg_post_tile<NU, FINE, TX, TY, NT, NM>(L, C, done, part, TileId(c0), gridDim.x, gridDim.y);
}

// ---------------------------------------------------------------- finest grid in register strips
// On the finest grid a block owns a region of kSR rows x kSW columns, held in
// registers: kSNW waves stacked vertically, kSWR rows each, two adjacent
// columns per lane (even column in e, odd column in o).  The neighbour
// columns of the lanes on either side come through DPP lane shifts; the rows
// just above and below a wave's own (ghost rows) are refreshed from the
// neighbouring waves through LDS after every half-sweep (one barrier).  The
// region's outer ghost rows and edge columns are not refreshed, so the
// block's output is the region minus a halo of kSH cells (2 x 2 half-sweeps
// shrink the valid region by 4, the residual and the restriction stencil by
// one each).  The region origin is even in both directions, so a lane's even
// column is coarse column (origin / 2 + lane) and a row's parity is that of
// its index in the region (kSWR is even).  Blocks whose region and ghost rows
// lie inside the interior (most of them) take a path without any boundary
// test: every point is updated and the diagonal is 4.
constexpr int kSWR = 12, kSNW = 4, kSW = 128, kSH = 6;
constexpr int kSR = kSWR * kSNW;
constexpr int kSTX = kSW - 2 * kSH, kSTY = kSR - 2 * kSH;  // output tile 116 x 36

int strip_tiles_x(int m) { return (m + 2 + kSTX - 1) / kSTX; }
int strip_tiles(int n, int m) { return strip_tiles_x(m) * ((n + 2 + kSTY - 1) / kSTY); }

// lane l receives lane l-1's v (lane 0: 0) / lane l+1's v (lane 63: 0)
__device__ __forceinline__ float from_left(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float from_right(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}

// This wave's place: channel, tile, region origin, first region row (r0) and
// the grid column of its lane's even column.
struct Strip {
    int c, tile, gi0, gj0, r0, je, lane, w;
    // strip `tile` of channel c (tiles_x strips per row of strips)
    __device__ Strip(int c_, int tile_, int tiles_x) {
        c = c_;
        tile = tile_;
        const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
        gi0 = ty * kSTY - kSH;
        gj0 = tx * kSTX - kSH;
        w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        lane = threadIdx.x & 63;
        r0 = w * kSWR;
        je = gj0 + 2 * lane;
    }
    __device__ Strip(int c0, int tiles_x) {
        const int nbx = gridDim.x, nb = nbx * gridDim.y;
        const int Lb = xcd_remap(blockIdx.x + nbx * blockIdx.y, nb);
        c = c0 + Lb / nbx;
        tile = Lb % nbx;
        const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
        gi0 = ty * kSTY - kSH;
        gj0 = tx * kSTX - kSH;
        w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: scalar row math
        lane = threadIdx.x & 63;
        r0 = w * kSWR;
        je = gj0 + 2 * lane;
    }
    // the region and its outer ghost rows hold interior points only, and the
    // region holds no first or last interior row or column (whose diagonal and
    // transfer weights may differ)
    __device__ bool interior(const LevelDev& L) const {
        return gi0 - 1 >= 1 && gi0 + kSR <= L.n && gj0 >= 2 && gj0 + kSW <= L.m;
    }
    __device__ int slot(int ntiles) const { return c * ntiles + tile; }
};

// Region rows r0 - 1 + q, q = 0 .. Q-1, of x (channel c) into e/o; zero
// outside the array (addresses clamped into it: every load unconditional).
template <bool INT, int Q>
__device__ __forceinline__ void strip_load(const LevelDev& L, const float* x, const Strip& S,
                                           float (&e)[Q], float (&o)[Q], int q_off) {
    const float* xc = x + (size_t)S.c * L.cs;
    const int jo = S.je + 1;
    if (INT) {
        const float* pe = xc + (size_t)(S.gi0 + S.r0 - q_off) * L.pitch + S.je;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            e[q] = pe[(size_t)q * L.pitch];
            o[q] = pe[(size_t)q * L.pitch + 1];
        }
        return;
    }
    const bool ce = S.je >= 0 && S.je <= L.m + 1, co = jo >= 0 && jo <= L.m + 1;
    const int je_c = min(max(S.je, 0), L.m + 1), jo_c = min(max(jo, 0), L.m + 1);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int gi = S.gi0 + S.r0 + q - q_off;
        const bool rok = gi >= 0 && gi <= L.n + 1;
        const int ro = min(max(gi, 0), L.n + 1) * L.pitch;
        const float ve = xc[ro + je_c], vo = xc[ro + jo_c];
        e[q] = (rok && ce) ? ve : 0.f;
        o[q] = (rok && co) ? vo : 0.f;
    }
}

// Exchange of ghost rows: this wave's first and last own rows (e/o index 1
// and kSWR) go out, the neighbours' come into index 0 and kSWR + 1.  buf
// alternates between calls so one barrier per exchange suffices.
__device__ __forceinline__ void strip_exchange(float (&e)[kSWR + 2], float (&o)[kSWR + 2],
                                               float2 (*sx)[kSNW][2][64], int buf,
                                               const Strip& S) {
    sx[buf][S.w][0][S.lane] = make_float2(e[1], o[1]);
    sx[buf][S.w][1][S.lane] = make_float2(e[kSWR], o[kSWR]);
    __syncthreads();
    if (S.w > 0) {
        const float2 t = sx[buf][S.w - 1][1][S.lane];
        e[0] = t.x;
        o[0] = t.y;
    }
    if (S.w < kSNW - 1) {
        const float2 t = sx[buf][S.w + 1][0][S.lane];
        e[kSWR + 1] = t.x;
        o[kSWR + 1] = t.y;
    }
}

// Diagonal of the lane's even (e) and odd (o) column on a middle and on the
// last (l) interior row, with their reciprocals, for boundary blocks.  NM:
// the Neumann problem, whose first row has one neighbour fewer as well (the
// finest grid has n >= 3 rows, so no row is both first and last); otherwise
// the first row is a middle row, known at compile time.
template <bool NM>
struct StripDiag {
    float de, dd, dl_e, dl_o;
    float rde, rdo, rdl_e, rdl_o, rdf_e, rdf_o;  // smoothing weight / diagonal
    float cw, q4;                               // 1 - weight, weight / 4
    int n;
    bool ine, ino;
    __device__ StripDiag(const LevelDev& L, const Strip& S) {
        const int jo = S.je + 1;
        n = L.n;
        ine = S.je >= 1 && S.je <= L.m;
        ino = jo >= 1 && jo <= L.m;
        de = 4.f + (S.je == L.m ? L.ex : 0.f);
        dd = 4.f + (jo == L.m ? L.ex : 0.f);
        if (NM) {
            if (S.je == 1) de += kNmDiag;
            if (jo == 1) dd += kNmDiag;
        }
        dl_e = de + L.ey;
        dl_o = dd + L.ey;
        const float w = L.sw;
        cw = 1.f - w;
        q4 = 0.25f * w;
        rde = w / de;
        rdo = w / dd;
        rdl_e = w / dl_e;
        rdl_o = w / dl_o;
        rdf_e = NM ? w / (de + kNmDiag) : 0.f;
        rdf_o = NM ? w / (dd + kNmDiag) : 0.f;
    }
    __device__ float diag_e(int gi) const {
        return (NM && gi == 1) ? de + kNmDiag : (gi == n ? dl_e : de);
    }
    __device__ float diag_o(int gi) const {
        return (NM && gi == 1) ? dd + kNmDiag : (gi == n ? dl_o : dd);
    }
    __device__ float rdiag_e(int gi) const {
        return (NM && gi == 1) ? rdf_e : (gi == n ? rdl_e : rde);
    }
    __device__ float rdiag_o(int gi) const {
        return (NM && gi == 1) ? rdf_o : (gi == n ? rdl_o : rdo);
    }
};

// Red-black half-sweep of colour col (0 red: i + j even) over the wave's own
// rows; in a row exactly one of e, o has the colour.  Over-relaxed: a point
// takes (1 - w) u + w (Gauss-Seidel value).
template <bool INT, bool NM>
__device__ __forceinline__ void strip_half(float (&e)[kSWR + 2], float (&o)[kSWR + 2],
                                           const float (&fe)[kSWR], const float (&fo)[kSWR],
                                           int col, const Strip& S, const LevelDev& L,
                                           const StripDiag<NM>& D) {
#pragma unroll
    for (int q = 1; q <= kSWR; ++q) {
        const int gi = S.gi0 + S.r0 + q - 1;  // parity that of q - 1
        const bool upd = INT || (gi >= 1 && gi <= L.n);
        if (((q - 1 + col) & 1) == 0) {  // even column has the colour
            const float x = ((e[q - 1] + e[q + 1]) + (from_left(o[q]) + o[q])) - fe[q - 1];
            if (INT) {
                e[q] = fmaf(D.cw, e[q], x * D.q4);
            } else {
                const float v = fmaf(D.cw, e[q], x * D.rdiag_e(gi));
                e[q] = (upd && D.ine) ? v : e[q];
            }
        } else {
            const float x = ((o[q - 1] + o[q + 1]) + (e[q] + from_right(e[q]))) - fo[q - 1];
            if (INT) {
                o[q] = fmaf(D.cw, o[q], x * D.q4);
            } else {
                const float v = fmaf(D.cw, o[q], x * D.rdiag_o(gi));
                o[q] = (upd && D.ino) ? v : o[q];
            }
        }
    }
}

// FP64 residuals of the even- and odd-column points of own row q (grid row gi).
template <bool INT, bool NM>
__device__ __forceinline__ void strip_residual(const float (&e)[kSWR + 2],
                                               const float (&o)[kSWR + 2], float fe_q, float fo_q,
                                               int q, int gi, const StripDiag<NM>& D, double ofs,
                                               double& re, double& ro) {
    re = res_value(e[q - 1], e[q + 1], from_left(o[q]), o[q], e[q], fe_q,
                   INT ? 4.f : D.diag_e(gi)) - ofs;
    ro = res_value(o[q - 1], o[q + 1], e[q], from_right(e[q]), o[q], fo_q,
                   INT ? 4.f : D.diag_o(gi)) - ofs;
}

template <int NU, bool INT, bool NM>
__device__ __forceinline__ void fine_pre_body(const LevelDev& L, const LevelDev& C,
                                              double* __restrict__ part, int ntiles,
                                              const Strip& S, float2 (*sx)[kSNW][2][64]) {
    const double ofs = NM ? L.fofs[S.c] : 0.0;
    float e[kSWR + 2], o[kSWR + 2], fe[kSWR], fo[kSWR], be[kSWR], bo[kSWR];
    strip_load<INT, kSWR + 2>(L, L.u, S, e, o, 1);
    strip_load<INT, kSWR>(L, L.f, S, fe, fo, 0);
#pragma unroll
    for (int q = 0; q < kSWR; ++q) {
        be[q] = e[q + 1];
        bo[q] = o[q + 1];
    }
    const StripDiag<NM> D(L, S);
    int buf = 0;
#pragma unroll
    for (int s = 0; s < NU; ++s) {
        strip_half<INT, NM>(e, o, fe, fo, 0, S, L, D);
        strip_exchange(e, o, sx, buf, S);
        buf ^= 1;
        strip_half<INT, NM>(e, o, fe, fo, 1, S, L, D);
        strip_exchange(e, o, sx, buf, S);
        buf ^= 1;
    }
    // output rows: region rows [kSH, kSR - kSH); lanes [kSH/2, 64 - kSH/2).
    // (The largest change is taken in FP32: |a - b| of two FP32 values is
    // within one rounding of the exact difference.)
    const bool lane_out = S.lane >= kSH / 2 && S.lane < 64 - kSH / 2;
    const int jo = S.je + 1;
    float* ub = L.ub + (size_t)S.c * L.cs;
    float dmaxf = 0.f;
#pragma unroll
    for (int q = 1; q <= kSWR; ++q) {
        const int R = S.r0 + q - 1, gi = S.gi0 + R;
        if (R < kSH || R >= kSR - kSH || (!INT && gi > L.n + 1)) continue;
        const bool rin = INT || (gi >= 1 && gi <= L.n);
        const bool ie = lane_out && rin && (INT || D.ine), io = lane_out && rin && (INT || D.ino);
        dmaxf = fmaxf(dmaxf, ie ? fabsf(e[q] - be[q - 1]) : 0.f);
        dmaxf = fmaxf(dmaxf, io ? fabsf(o[q] - bo[q - 1]) : 0.f);
        if (!lane_out) continue;
        const size_t ro = (size_t)gi * L.pitch;
        if (INT || S.je <= L.m + 1) ub[ro + S.je] = e[q];
        if (INT || jo <= L.m + 1) ub[ro + jo] = o[q];
    }
    // residual (FP64 registers, stored FP32 over f) on the own rows; zero off
    // the interior
#pragma unroll
    for (int q = 1; q <= kSWR; ++q) {
        const int gi = S.gi0 + S.r0 + q - 1;
        const bool rin = INT || (gi >= 1 && gi <= L.n);
        double re, rv;
        strip_residual<INT, NM>(e, o, fe[q - 1], fo[q - 1], q, gi, D, ofs, re, rv);
        if (INT) {
            fe[q - 1] = (float)re;
            fo[q - 1] = (float)rv;
        } else {
            const float sr = NM ? nm_scale(gi, L.n) : 1.f;
            const float se = NM ? sr * nm_scale(S.je, L.m) : 1.f;
            const float so = NM ? sr * nm_scale(S.je + 1, L.m) : 1.f;
            fe[q - 1] = (rin && D.ine) ? (float)re * se : 0.f;
            fo[q - 1] = (rin && D.ino) ? (float)rv * so : 0.f;
        }
    }
    // the residual row just above the wave (the last row of the wave above)
    float ge = 0.f, go = 0.f;
    sx[buf][S.w][1][S.lane] = make_float2(fe[kSWR - 1], fo[kSWR - 1]);
    __syncthreads();
    if (S.w > 0) {
        const float2 t = sx[buf][S.w - 1][1][S.lane];
        ge = t.x;
        go = t.y;
    }
    // full weighting at the even points of the output tile: own rows q - 1
    // even (region row even), neighbours above (q - 2, or the ghost) and below
    float* fc = C.fw + (size_t)S.c * C.cs;
    const int J = S.je >> 1;
#pragma unroll
    for (int q = 1; q <= kSWR; q += 2) {
        const int R = S.r0 + q - 1;
        const int I = (S.gi0 + R) >> 1;
        const float ue = q >= 2 ? fe[q - 2] : ge, uo = q >= 2 ? fo[q - 2] : go;
        const float ce = fe[q - 1], co = fo[q - 1];
        const float bwe = fe[q], bwo = fo[q];  // q < kSWR: the row below is own
        const float v = 4.f * ce + 2.f * (from_left(co) + co + ue + bwe) +
                        (from_left(uo) + uo + from_left(bwo) + bwo);
        if (R < kSH || R >= kSR - kSH || !lane_out) continue;
        if (INT || (I >= 1 && I <= C.n && J >= 1 && J <= C.m))
            fc[(size_t)I * C.pitch + J] = 0.25f * v;
    }
    // one partial per block: the waves' maxima combined through LDS
    __shared__ double red[kSNW];
    const double dmax = wave_max_d((double)dmaxf);
    if (S.lane == 0) red[S.w] = dmax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
#pragma unroll
        for (int k = 1; k < kSNW; ++k) m = fmax(m, red[k]);
        part[(size_t)S.slot(ntiles) * 5 + 3] = m;
    }
}

// Finest-grid pre-smoothing + FP64 residual + restriction (see k_mg_pre).
// NM: the Neumann problem (residual offset).
template <int NU, bool NM>
__global__ __launch_bounds__(64 * kSNW) void k_fine_pre(LevelDev L, LevelDev C,
                                                         const int* __restrict__ done,
                                                         double* __restrict__ part, int c0,
                                                         int ntiles, int tiles_x) {
    __shared__ float2 sx[2][kSNW][2][64];
    const Strip S(c0, tiles_x);
    if (done[S.c]) return;  // uniform over the block
    if (S.interior(L))
        fine_pre_body<NU, true, NM>(L, C, part, ntiles, S, sx);
    else
        fine_pre_body<NU, false, NM>(L, C, part, ntiles, S, sx);
}

template <int NU, bool INT, bool NM>
__device__ __forceinline__ void fine_post_body(const LevelDev& L, const LevelDev& C,
                                               double* __restrict__ part, int ntiles,
                                               const Strip& S, float2 (*sx)[kSNW][2][64]) {
    const double ofs = NM ? L.fofs[S.c] : 0.0;
    constexpr int KC = kSWR / 2 + 1;  // coarse rows under the wave's own rows
    float e[kSWR + 2], o[kSWR + 2], fe[kSWR], fo[kSWR], E[KC], be[kSWR], bo[kSWR];
    strip_load<INT, kSWR + 2>(L, L.ub, S, e, o, 1);
    strip_load<INT, kSWR>(L, L.f, S, fe, fo, 0);
#pragma unroll
    for (int q = 0; q < kSWR; ++q) {
        be[q] = e[q + 1];
        bo[q] = o[q + 1];
    }
    const int ci0 = (S.gi0 + S.r0) >> 1, J0 = S.je >> 1;
    {
        const float* ec = C.u + (size_t)S.c * C.cs;
        const bool cj = J0 >= 0 && J0 <= C.m + 1;
        const int Jc = min(max(J0, 0), C.m + 1);
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const int I = ci0 + k;
            const float v = ec[(size_t)min(max(I, 0), C.n + 1) * C.pitch + Jc];
            E[k] = (cj && I >= 0 && I <= C.n + 1) ? v : 0.f;
        }
    }
    const StripDiag<NM> D(L, S);
    // bilinear prolongation onto the own rows: e has oj = 0, o has oj = 1
    // (coarse columns J0 and J0 + 1)
    const float fxo = (NM && J0 == 0) ? kNmW : (J0 == C.m ? C.wx : 0.5f);
#pragma unroll
    for (int q = 1; q <= kSWR; ++q) {
        const int gi = S.gi0 + S.r0 + q - 1;
        const bool rin = INT || (gi >= 1 && gi <= L.n);
        const int k = (q - 1) >> 1;
        const bool oi = (q - 1) & 1;
        const float fy =
            oi ? ((NM && (ci0 + k) == 0) ? kNmW : ((ci0 + k) == C.n ? C.wy : 0.5f)) : 1.f;
        const float p0 = E[k], pa = oi ? E[k + 1] : 0.f;
        const float q0 = from_right(p0), qa = from_right(pa);
        float we = p0;
        if (oi) we += pa;
        float wo = p0;
        if (oi) wo += pa;
        wo += q0;
        if (oi) wo += qa;
        const float ve = e[q] + fy * 1.f * we, vo = o[q] + fy * fxo * wo;
        e[q] = (rin && (INT || D.ine)) ? ve : e[q];
        o[q] = (rin && (INT || D.ino)) ? vo : o[q];
    }
    int buf = 0;
    strip_exchange(e, o, sx, buf, S);  // ghosts carry the correction too
    buf ^= 1;
#pragma unroll
    for (int s = 0; s < NU; ++s) {
        strip_half<INT, NM>(e, o, fe, fo, kPost0<NM>, S, L, D);
        strip_exchange(e, o, sx, buf, S);
        buf ^= 1;
        strip_half<INT, NM>(e, o, fe, fo, 1 - kPost0<NM>, S, L, D);
        strip_exchange(e, o, sx, buf, S);
        buf ^= 1;
    }
    // store the output rows; norms over their interior points (the largest
    // change and |u| in FP32: exact or within one rounding)
    const bool lane_out = S.lane >= kSH / 2 && S.lane < 64 - kSH / 2;
    const int jo = S.je + 1;
    float* u = L.u + (size_t)S.c * L.cs;
    double rmax = 0.0, rss = 0.0;
    float dmaxf = 0.f, umaxf = 0.f;
#pragma unroll
    for (int q = 1; q <= kSWR; ++q) {
        const int R = S.r0 + q - 1, gi = S.gi0 + R;
        if (R < kSH || R >= kSR - kSH || (!INT && gi > L.n + 1)) continue;
        const bool rin = INT || (gi >= 1 && gi <= L.n);
        double re, rv;
        strip_residual<INT, NM>(e, o, fe[q - 1], fo[q - 1], q, gi, D, ofs, re, rv);
        const bool ie = lane_out && rin && (INT || D.ine), io = lane_out && rin && (INT || D.ino);
        dmaxf = fmaxf(dmaxf, ie ? fabsf(e[q] - be[q - 1]) : 0.f);
        dmaxf = fmaxf(dmaxf, io ? fabsf(o[q] - bo[q - 1]) : 0.f);
        umaxf = fmaxf(umaxf, ie ? fabsf(e[q]) : 0.f);
        umaxf = fmaxf(umaxf, io ? fabsf(o[q]) : 0.f);
        rmax = fmax(rmax, ie ? fabs(re) : 0.0);
        rmax = fmax(rmax, io ? fabs(rv) : 0.0);
        rss += ie ? re * re : 0.0;
        rss += io ? rv * rv : 0.0;
        if (!lane_out) continue;
        const size_t ro = (size_t)gi * L.pitch;
        if (INT || S.je <= L.m + 1) u[ro + S.je] = e[q];
        if (INT || jo <= L.m + 1) u[ro + jo] = o[q];
    }
    rmax = wave_max_d(rmax);
    const double umax = wave_max_d((double)umaxf);
    rss = wave_sum_d(rss);
    const double dmax = wave_max_d((double)dmaxf);
    // one partial per block: the waves' values combined through LDS (the sum
    // in wave order, so the result is deterministic)
    __shared__ double red[kSNW][4];
    if (S.lane == 0) {
        red[S.w][0] = rmax;
        red[S.w][1] = umax;
        red[S.w][2] = rss;
        red[S.w][3] = dmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = red[0][0], b = red[0][1], q = red[0][2], d = red[0][3];
#pragma unroll
        for (int k = 1; k < kSNW; ++k) {
            a = fmax(a, red[k][0]);
            b = fmax(b, red[k][1]);
            q += red[k][2];
            d = fmax(d, red[k][3]);
        }
        double* p = part + (size_t)S.slot(ntiles) * 5;
        p[0] = a;
        p[1] = b;
        p[2] = q;
        p[4] = d;
    }
}

// Finest-grid prolongation + correction + post-smoothing + norms (see k_mg_post).
template <int NU, bool NM>
__global__ __launch_bounds__(64 * kSNW) void k_fine_post(LevelDev L, LevelDev C,
                                                          const int* __restrict__ done,
                                                          double* __restrict__ part, int c0,
                                                          int ntiles, int tiles_x) {
    __shared__ float2 sx[2][kSNW][2][64];
    const Strip S(c0, tiles_x);
    if (done[S.c]) return;  // uniform over the block
    if (S.interior(L))
        fine_post_body<NU, true, NM>(L, C, part, ntiles, S, sx);
    else
        fine_post_body<NU, false, NM>(L, C, part, ntiles, S, sx);
}

// ---------------------------------------------------------------- coarse V-cycle in LDS
// Thread layout for a grid of n interior rows: tpr threads share a row,
// rows 1 + t / tpr, stepping by rpp rows per pass.
struct RowMap {
    int tpr, rpp, r0, sg;
    bool active;
    __device__ RowMap(int rows) {
        const int nt = blockDim.x, t = threadIdx.x;
        tpr = rows > 0 ? max(1, nt / rows) : nt;
        rpp = nt / tpr;
        r0 = t / tpr;
        sg = t % tpr;
        active = t < rpp * tpr;
    }
};

// q / d for q d < 2^32 with mg = floor(2^32 / d) + 1 (d >= 2), exact.
__device__ __forceinline__ int udiv(int q, int d, uint32_t mg) {
    const int h = (int)__umulhi((uint32_t)q, mg);
    return d == 1 ? q : h;
}

// One wave's LDS operations are performed in order; this only keeps the
// compiler from moving LDS accesses across the point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The group of threads running a coarse-grid operation: the whole workgroup
// (NT = blockDim.x, __syncthreads between steps) or wave 0 alone.
template <int NT>
__device__ __forceinline__ void group_sync() {
    if (NT == 64)
        wave_sync();
    else
        __syncthreads();
}

struct LdsGrid {
    float* U;
    float* F;
    int n, m, M, h;    // interior size, row pitch, cells of one colour per row
    uint32_t mg_m, mg_h;
    float ey, ex;
};

__device__ __forceinline__ LdsGrid lds_grid(const LdsPlan& P, float* lds, int l) {
    LdsGrid g;
    g.n = P.n[l];
    g.m = P.m[l];
    g.M = P.M[l];
    g.h = (g.m + 1) >> 1;
    g.U = lds + P.off[l];
    g.F = g.U + (g.n + 2) * g.M;
    g.mg_m = P.mg_m[l];
    g.mg_h = P.mg_h[l];
    g.ey = P.ey[l];
    g.ex = P.ex[l];
    return g;
}

// Slot q of colour c: row 1 + q / h, the (q % h)-th point of that colour in
// the row (red: i + j even).  Slots past the grid read cell (1, 1) and store
// to the thread's trash cell, so that no load or store is conditional and a
// thread issues the loads of all its slots before it waits for them.
struct Slot {
    int r;      // LDS offset read
    float* w;   // LDS address written
    float rd;   // 1 / diagonal
};

template <bool NM>
__device__ __forceinline__ Slot colour_slot(const LdsGrid& g, int c, int q, float* trash) {
    const int r = udiv(q, g.h, g.mg_h);
    const int i = 1 + r, j = 1 + ((c + i + 1) & 1) + 2 * (q - r * g.h);
    float d = 4.f;
    if (NM && i == 1) d += kNmDiag;
    if (NM && j == 1) d += kNmDiag;
    if (i == g.n) d += g.ey;
    if (j == g.m) d += g.ex;
    const bool ok = i <= g.n && j <= g.m;
    Slot s;
    s.r = ok ? i * g.M + j : g.M + 1;
    s.w = ok ? g.U + s.r : trash;
    s.rd = 1.f / d;
    return s;
}

// Red-black Gauss-Seidel (SOR = false) or SOR with omega, sweeps x (colour
// c0, then the other).  Points of one colour read only the other colour.
// The first NT * KPT slots of each colour are held in registers; slots beyond
// (only a large coarsest grid has them) are walked one at a time.
template <int NT, int KPT, bool SOR, bool NM>
__device__ void lds_smooth_k(const LdsGrid& g, int c0, int sweeps, float omega, int t,
                             float* trash) {
    Slot sl[2][KPT];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int k = 0; k < KPT; ++k) sl[c][k] = colour_slot<NM>(g, c, t + NT * k, trash);
    const int slots = g.n * g.h, M = g.M;
    const float* U = g.U;
    const float* F = g.F;
    auto value = [&](int q, float rd) -> float {
        const float x = ((U[q - M] + U[q + M]) + (U[q - 1] + U[q + 1])) - F[q];
        const float gs = x * rd;
        return SOR ? U[q] + omega * (gs - U[q]) : gs;
    };
    auto half = [&](const Slot* sc, int c) {
        float v[KPT];
#pragma unroll
        for (int k = 0; k < KPT; ++k) v[k] = value(sc[k].r, sc[k].rd);
#pragma unroll
        for (int k = 0; k < KPT; ++k) *sc[k].w = v[k];
        for (int q = t + NT * KPT; q < slots; q += NT) {
            const Slot s = colour_slot<NM>(g, c, q, trash);
            *s.w = value(s.r, s.rd);
        }
        group_sync<NT>();
    };
    for (int s = 0; s < sweeps; ++s) {
        if (c0 == 0) {
            half(sl[0], 0);
            half(sl[1], 1);
        } else {
            half(sl[1], 1);
            half(sl[0], 0);
        }
    }
}

template <int NT, bool NM>
__device__ void lds_smooth(const LdsGrid& g, int c0, int sweeps, float omega, int t,
                           float* trash) {
    const int per = (g.n * g.h + NT - 1) / NT;  // slots of a colour per thread
    if (omega != 1.f) {
        if (per > 2)
            lds_smooth_k<NT, 4, true, NM>(g, c0, sweeps, omega, t, trash);
        else if (per > 1)
            lds_smooth_k<NT, 2, true, NM>(g, c0, sweeps, omega, t, trash);
        else
            lds_smooth_k<NT, 1, true, NM>(g, c0, sweeps, omega, t, trash);
    } else {
        if (per > 2)
            lds_smooth_k<NT, 4, false, NM>(g, c0, sweeps, omega, t, trash);
        else if (per > 1)
            lds_smooth_k<NT, 2, false, NM>(g, c0, sweeps, omega, t, trash);
        else
            lds_smooth_k<NT, 1, false, NM>(g, c0, sweeps, omega, t, trash);
    }
}

// Interior point q of grid g (row-major over the n x m interior), clamped to
// the last point past the end.
__device__ __forceinline__ void interior_point(const LdsGrid& g, int q, int& i, int& j) {
    const int r = udiv(q, g.m, g.mg_m);
    i = 1 + r;
    j = 1 + q - r * g.m;
}

// R = F - A U on the interior (evaluated in FP64, stored FP32); the ring of R
// stays zero from the kernel's entry.  B points per thread and pass.
template <int NT, int B, bool NM>
__device__ void lds_residual(const LdsGrid& g, float* R, int t, float* trash, double ofs) {
    const int cells = g.n * g.m, M = g.M;
    const float* U = g.U;
    for (int q0 = 0; q0 < cells; q0 += B * NT) {
        float v[B];
        float* dst[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int q = q0 + t + b * NT;
            int i, j;
            interior_point(g, q < cells ? q : cells - 1, i, j);
            const int o = i * M + j;
            const float d =
                diag_at(i, j, g.n, g.m, g.ey, g.ex, NM ? kNmDiag : 0.f, NM ? kNmDiag : 0.f);
            const float r =
                (float)(res_value(U[o - M], U[o + M], U[o - 1], U[o + 1], U[o], g.F[o], d) - ofs);
            v[b] = NM ? r * (nm_scale(i, g.n) * nm_scale(j, g.m)) : r;
            dst[b] = q < cells ? R + o : trash;
        }
#pragma unroll
        for (int b = 0; b < B; ++b) *dst[b] = v[b];
    }
    group_sync<NT>();
}

// Full-weighting restriction of R (grid g) to the right-hand side of grid cg
// (times 4: the unit-spacing scaling of the coarse operator).
template <int NT, int B>
__device__ void lds_restrict(const LdsGrid& g, const float* R, const LdsGrid& cg, int t,
                             float* trash) {
    const int cells = cg.n * cg.m, M = g.M;
    for (int q0 = 0; q0 < cells; q0 += B * NT) {
        float v[B];
        float* dst[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int q = q0 + t + b * NT;
            int I, J;
            interior_point(cg, q < cells ? q : cells - 1, I, J);
            const int o = 2 * I * M + 2 * J;
            v[b] = 0.25f * (4.f * R[o] + 2.f * (R[o - 1] + R[o + 1] + R[o - M] + R[o + M]) +
                            (R[o - M - 1] + R[o - M + 1] + R[o + M - 1] + R[o + M + 1]));
            dst[b] = q < cells ? cg.F + I * cg.M + J : trash;
        }
#pragma unroll
        for (int b = 0; b < B; ++b) *dst[b] = v[b];
    }
    group_sync<NT>();
}

// Bilinear prolongation of the coarse correction onto the interior of g;
// wy / wx weight fine points between the last coarse point and the boundary
// (Neumann: also those before the first coarse point, weight kNmW).
template <int NT, int B, bool NM>
__device__ void lds_prolong(const LdsGrid& g, const LdsGrid& cg, float wy, float wx, int t,
                            float* trash) {
    const int cells = g.n * g.m, Mc = cg.M;
    const float* Uc = cg.U;
    for (int q0 = 0; q0 < cells; q0 += B * NT) {
        float v[B];
        float* dst[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int q = q0 + t + b * NT;
            int i, j;
            interior_point(g, q < cells ? q : cells - 1, i, j);
            const int o = i * g.M + j;
            const bool oi = i & 1, oj = j & 1;
            const int I0 = i >> 1, J0 = j >> 1;
            const float fy = oi ? ((NM && I0 == 0) ? kNmW : (I0 == cg.n ? wy : 0.5f)) : 1.f;
            const float fx = oj ? ((NM && J0 == 0) ? kNmW : (J0 == cg.m ? wx : 0.5f)) : 1.f;
            const float* p = Uc + I0 * Mc + J0;  // rows I0 + 1 <= nc + 1: in the grid
            float w = p[0];
            const float a = p[Mc], c = p[1], e = p[Mc + 1];
            if (oi) w += a;
            if (oj) w += c;
            if (oi && oj) w += e;
            v[b] = g.U[o] + fy * fx * w;
            dst[b] = q < cells ? g.U + o : trash;
        }
#pragma unroll
        for (int b = 0; b < B; ++b) *dst[b] = v[b];
    }
    group_sync<NT>();
}

// Levels lw .. L-1 of the V-cycle below a grid already restricted, run by
// wave 0 alone: these grids hold at most 64 x 4 points of a colour.
template <bool NM>
__device__ void lds_wave_tail(const LdsPlan& P, float* lds, int lane, float* trash) {
    const int L = P.L;
    for (int l = P.lw; l < L - 1; ++l) {
        const LdsGrid g = lds_grid(P, lds, l);
        lds_smooth<64, NM>(g, 0, P.pre, P.sw, lane, trash);
        lds_residual<64, 8, NM>(g, lds + P.roff[l], lane, trash, 0.0);
        lds_restrict<64, 4>(g, lds + P.roff[l], lds_grid(P, lds, l + 1), lane, trash);
    }
    lds_smooth<64, NM>(lds_grid(P, lds, L - 1), 0, P.csweeps, P.omega, lane, trash);
    for (int l = L - 2; l >= P.lw; --l) {
        const LdsGrid g = lds_grid(P, lds, l);
        lds_prolong<64, 8, NM>(g, lds_grid(P, lds, l + 1), P.wy[l + 1], P.wx[l + 1], lane, trash);
        lds_smooth<64, NM>(g, kPost0<NM>, P.post, P.sw, lane, trash);
    }
}

template <bool NM>
__device__ __forceinline__ void mg_lds_task(const LdsPlan& P, const int* __restrict__ done,
                                            double* __restrict__ part, int c, float* lds,
                                            double* sh) {
    const int lc = P.lc, L = P.L, t = threadIdx.x;
    // load the top level (the done flag is read together with its first
    // chunk); clear the coarser grids and the residuals (their rings stay zero
    // for the whole cycle)
    {
        constexpr int KL = 4;  // points per thread and chunk, loaded before stored
        const int n = P.n[lc], m = P.m[lc], M = P.M[lc];  // pitch M >= m + 2: padding is zero
        const int cells = (n + 2) * M;
        float* U = lds + P.off[lc];
        float* F = U + cells;
        const float* gu = P.top.u + (size_t)c * P.top.cs;
        const float* gf = P.top.f + (size_t)c * P.top.cs;
        const int dn = done[c];
        for (int q0 = 0; q0 < cells; q0 += KL * kLdsThreads) {
            float vu[KL], vf[KL];
            int at[KL];
#pragma unroll
            for (int k = 0; k < KL; ++k) {
                const int q = q0 + t + k * kLdsThreads;
                const int i = q / M, j = q - i * M;
                const bool live = q < cells;
                const bool row = live && j <= m + 1;  // not a padding cell
                const bool in = live && i >= 1 && i <= n && j >= 1 && j <= m;
                const size_t o = (size_t)i * P.top.pitch + j;
                vu[k] = (lc == 0 && row) ? gu[o] : 0.f;
                vf[k] = in ? gf[o] : 0.f;
                at[k] = live ? q : -1;
            }
            if (dn) return;  // uniform over the block
#pragma unroll
            for (int k = 0; k < KL; ++k)
                if (at[k] >= 0) {
                    U[at[k]] = vu[k];
                    F[at[k]] = vf[k];
                }
        }
        if (dn) return;
        for (int i = P.zero0 + t; i < P.zero1; i += kLdsThreads) lds[i] = 0.f;
        __syncthreads();
    }
    float* trash = lds + P.trash + (t & 63);
    const int lb = P.lw < L - 1 ? P.lw : L - 1;  // first level below the workgroup's levels
    for (int l = lc; l < lb; ++l) {
        const LdsGrid g = lds_grid(P, lds, l);
        lds_smooth<kLdsThreads, NM>(g, 0, P.pre, P.sw, t, trash);
        lds_residual<kLdsThreads, 2, NM>(g, lds + P.roff[l], t, trash,
                                     (NM && l == 0) ? P.fofs[c] : 0.0);
        lds_restrict<kLdsThreads, 1>(g, lds + P.roff[l], lds_grid(P, lds, l + 1), t, trash);
    }
    if (P.lw < L) {
        if (t < 64) lds_wave_tail<NM>(P, lds, t, trash);
        __syncthreads();
    } else {
        lds_smooth<kLdsThreads, NM>(lds_grid(P, lds, L - 1), 0, P.csweeps, P.omega, t, trash);
    }
    for (int l = lb - 1; l >= lc; --l) {
        const LdsGrid g = lds_grid(P, lds, l);
        lds_prolong<kLdsThreads, 2, NM>(g, lds_grid(P, lds, l + 1), P.wy[l + 1], P.wx[l + 1], t,
                                        trash);
        lds_smooth<kLdsThreads, NM>(g, kPost0<NM>, P.post, P.sw, t, trash);
    }
    // write back the top level (its ring too: zero for coarse grids, the
    // unchanged Dirichlet data for the finest)
    {
        const int n = P.n[lc], m = P.m[lc], M = P.M[lc];
        const float* U = lds + P.off[lc];
        const float* F = U + (n + 2) * M;
        float* gu = P.top.u + (size_t)c * P.top.cs;
        double rmax = 0.0, umax = 0.0, rss = 0.0, dmax = 0.0;
        const RowMap rm(n + 2);
        if (rm.active) {
            for (int i = rm.r0; i <= n + 1; i += rm.rpp) {
                for (int j = rm.sg; j <= m + 1; j += rm.tpr) {
                    const int idx = i * M + j;
                    const size_t go = (size_t)i * P.top.pitch + j;
                    const bool in = i >= 1 && i <= n && j >= 1 && j <= m;
                    if (lc == 0 && in) {
                        dmax = fmax(dmax, fabs((double)U[idx] - (double)gu[go]));
                        const double rv =
                            res_value(U[idx - M], U[idx + M], U[idx - 1], U[idx + 1], U[idx],
                                      F[idx], diag_at(i, j, n, m, P.ey[0], P.ex[0],
                                                      NM ? kNmDiag : 0.f, NM ? kNmDiag : 0.f)) -
                            ((NM && lc == 0) ? P.fofs[c] : 0.0);
                        rmax = fmax(rmax, fabs(rv));
                        umax = fmax(umax, fabs((double)U[idx]));
                        rss += rv * rv;
                    }
                    gu[go] = U[idx];
                }
            }
        }
        if (lc == 0) {
            block_reduce3(rmax, umax, rss, sh);
            double d1 = 0.0, d2 = 0.0;
            block_reduce3(dmax, d1, d2, sh);
            if (threadIdx.x == 0) {
                part[(size_t)c * 5] = rmax;
                part[(size_t)c * 5 + 1] = umax;
                part[(size_t)c * 5 + 2] = rss;
                part[(size_t)c * 5 + 3] = dmax;
                part[(size_t)c * 5 + 4] = 0.0;
            }
        }
    }
}

template <bool NM>
__global__ __launch_bounds__(kLdsThreads) void k_mg_lds(LdsPlan P, const int* __restrict__ done,
                                                        double* __restrict__ part, int c0) {
    extern __shared__ float lds[];
    __shared__ double sh[3 * (kLdsThreads / 64)];
    mg_lds_task<NM>(P, done, part, c0 + blockIdx.x, lds, sh);
}

// End-of-cycle bookkeeping, one block per channel still running: reduce the
// per-block partials, write the statistics, raise the channel's flag when the
// relative correction is <= tol.  (Only these blocks synchronise through
// memory: a device-scope fence per block of a large grid would write back
// the L2 of its die each time.)
constexpr int kFinThreads = 256;
__device__ __forceinline__ void finalize_task(const double* __restrict__ part, int nblk,
                                              const double* __restrict__ bnorm,
                                              int* __restrict__ done,
                                              gdgs_stats* __restrict__ stats, double tol, int c,
                                              int stop_eta, double* sh) {
    // every load of the task is issued before any is waited for: the flag,
    // the norms of b, the cycle count and the block partials (one memory
    // latency instead of three in a row)
    const int dn = done[c];
    const double bn_inf = bnorm[2 * c], bn_2 = bnorm[2 * c + 1];
    const int cyc = stats->cycles[c];
    double rmax = 0.0, umax = 0.0, rss = 0.0, dpre = 0.0, dpost = 0.0;
    // two blocks' partials per thread and round, loaded before use
    constexpr int nt = kFinThreads;
    for (int b0 = threadIdx.x; b0 < nblk; b0 += 2 * nt) {
        double v[2][5];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int b = b0 + k * nt;
            const double* p = part + ((size_t)c * nblk + (b < nblk ? b : 0)) * 5;
#pragma unroll
            for (int q = 0; q < 5; ++q) v[k][q] = p[q];
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            if (b0 + k * nt >= nblk) break;
            rmax = fmax(rmax, v[k][0]);
            umax = fmax(umax, v[k][1]);
            rss += v[k][2];
            dpre = fmax(dpre, v[k][3]);
            dpost = fmax(dpost, v[k][4]);
        }
    }
    if (dn) return;  // uniform: finished before this cycle
    block_reduce3(rmax, umax, rss, sh);
    double d0 = 0.0;
    block_reduce3(dpre, dpost, d0, sh);
    if (threadIdx.x == 0) {
        // |u_k - u_{k-1}| <= (change in pre-smoothing) + (change in the post pass)
        const double dcyc = dpre + dpost;
        const double rel = umax > 0.0 ? dcyc / umax : (dcyc > 0.0 ? 1.0 : 0.0);
        const double den = 8.0 * umax + bn_inf;
        const double eta = den > 0.0 ? rmax / den : 0.0;
        stats->eta[c] = eta;
        stats->rel_res[c] = bn_2 > 0.0 ? sqrt(rss) / bn_2 : 0.0;
        stats->delta[c] = rel;
        stats->cycles[c] = cyc + 1;  // zeroed by setup; accumulates over resumed calls
        if ((stop_eta ? eta : rel) <= tol) done[c] = 1;
    }
}

__global__ __launch_bounds__(kFinThreads) void k_cycle_finalize(const double* __restrict__ part,
                                                               int nblk,
                                                               const double* __restrict__ bnorm,
                                                               int* __restrict__ done,
                                                               gdgs_stats* __restrict__ stats,
                                                               double tol, int c0,
                                                               int stop_eta) {
    __shared__ double sh[3 * (kFinThreads / 64)];
    finalize_task(part, nblk, bnorm, done, stats, tol, c0 + blockIdx.x, stop_eta, sh);
}

// ---------------------------------------------------------------- divergence adjoint
__global__ void k_div_adjoint(const float* __restrict__ lam, int H, int W,
                              float* __restrict__ dgrad) {
    const int j = blockIdx.x * kDivTX + (threadIdx.x % kDivTX);
    const int i = blockIdx.y * kDivTY + (threadIdx.x / kDivTX);
    const int c = blockIdx.z;
    if (i >= H || j >= W) return;
    const size_t HW = (size_t)H * W;
    const float* L = lam + (size_t)c * HW;
    auto li = [&](int a, int b) -> float {
        return (a >= 1 && a <= H - 2 && b >= 1 && b <= W - 2) ? L[(size_t)a * W + b] : 0.f;
    };
    const float l0 = li(i, j);
    dgrad[(size_t)(2 * c) * HW + (size_t)i * W + j] = l0 - li(i, j + 1);
    dgrad[(size_t)(2 * c + 1) * HW + (size_t)i * W + j] = l0 - li(i + 1, j);
}

// Transpose of the Neumann divergence (every pixel; the differences that
// would cross the border get 0).
__global__ void k_div_adjoint_nm(const float* __restrict__ lam, int H, int W,
                                 float* __restrict__ dgrad) {
    const int j = blockIdx.x * kDivTX + (threadIdx.x % kDivTX);
    const int i = blockIdx.y * kDivTY + (threadIdx.x / kDivTX);
    const int c = blockIdx.z;
    if (i >= H || j >= W) return;
    const size_t HW = (size_t)H * W, p = (size_t)i * W + j;
    const float* L = lam + (size_t)c * HW;
    const float l0 = L[p];
    dgrad[(size_t)(2 * c) * HW + p] = j < W - 1 ? l0 - L[p + 1] : 0.f;
    dgrad[(size_t)(2 * c + 1) * HW + p] = i < H - 1 ? l0 - L[p + W] : 0.f;
}

// Row pitch of a grid of m interior columns in LDS: m + 2 rounded up to even.
// The half-sweeps read every other cell of a row; with an odd pitch the rows
// of one colour line up on the same banks more often (a model of the reads
// over the grids held in LDS: about 35% fewer bank conflicts).
int lds_pitch(int m) { return (m + 3) & ~1; }

int lds_budget() {
    static int cached = -1;
    if (cached < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                hipSuccess || v <= 0)
            v = 64 * 1024;
        (void)hipGetLastError();
        v -= 2048;  // static LDS of the kernel
        cached = v < kLdsBudget ? v : kLdsBudget;
    }
    return cached;
}

bool small_tiles(const LevelDev& L) {
    const int nb = ((L.m + 2 + kTX - 1) / kTX) * ((L.n + 2 + kTY - 1) / kTY) * 3;
    return nb < kSmallTileBelow;
}

template <int NU, bool NM>
gdgs_status launch_pre(const LevelDev& L, const LevelDev& C, bool zero, bool delta,
                       const int* done, double* part, int c0, int nch, hipStream_t st,
                       bool may_time = true) {
    hipEvent_t ev0, ev1;
    const bool timed = delta && may_time && timer_events("mg_pre_fine", &ev0, &ev1);
    if (timed) GDGS_HIP_TRY(hipEventRecord(ev0, st));
    const int z = zero ? 1 : 0;
    if (delta) {
        const int nt = strip_tiles(L.n, L.m);
        hipLaunchKernelGGL((k_fine_pre<NU, NM>), dim3(nt, nch), dim3(64 * kSNW), 0, st, L, C,
                           done, part, c0, nt, strip_tiles_x(L.m));
    } else if (small_tiles(L)) {
        dim3 grid((L.m + 2 + kTXs - 1) / kTXs, (L.n + 2 + kTYs - 1) / kTYs, nch);
        hipLaunchKernelGGL((k_mg_pre<NU, false, kTXs, kTYs, kNTs, NM>), grid, dim3(kNTs), 0, st, L, C, z,
                           done, part, c0);
    } else {
        dim3 grid((L.m + 2 + kTX - 1) / kTX, (L.n + 2 + kTY - 1) / kTY, nch);
        hipLaunchKernelGGL((k_mg_pre<NU, false, kTX, kTY, 256, NM>), grid, dim3(256), 0, st, L, C, z,
                           done, part, c0);
    }
    if (timed) GDGS_HIP_TRY(hipEventRecord(ev1, st));
    return GDGS_OK;
}

template <int NU, bool NM>
gdgs_status launch_post(const LevelDev& L, const LevelDev& C, bool fine, const int* done,
                        double* part, int c0, int nch, hipStream_t st, bool may_time = true) {
    hipEvent_t ev0, ev1;
    const char* tname = fine ? "mg_post_fine" : "mg_post_coarse";
    const bool timed = may_time && timer_events(tname, &ev0, &ev1);
    if (timed) GDGS_HIP_TRY(hipEventRecord(ev0, st));
    // a timed pass may be repeated between its events: it reads none of what
    // it writes, so every repeat leaves the same results
    const int reps = timed ? timer_repeats(tname) : 1;
    for (int r = 0; r < reps; ++r) {
        if (fine) {
            const int nt = strip_tiles(L.n, L.m);
            hipLaunchKernelGGL((k_fine_post<NU, NM>), dim3(nt, nch), dim3(64 * kSNW), 0, st, L,
                               C, done, part, c0, nt, strip_tiles_x(L.m));
        } else if (small_tiles(L)) {
            dim3 grid((L.m + 2 + kTXs - 1) / kTXs, (L.n + 2 + kTYs - 1) / kTYs, nch);
            hipLaunchKernelGGL((k_mg_post<NU, false, kTXs, kTYs, kNTs, NM>), grid, dim3(kNTs), 0,
                               st, L, C, done, part, c0);
        } else {
            dim3 grid((L.m + 2 + kTX - 1) / kTX, (L.n + 2 + kTY - 1) / kTY, nch);
            hipLaunchKernelGGL((k_mg_post<NU, false, kTX, kTY, 256, NM>), grid, dim3(256), 0, st,
                               L, C, done, part, c0);
        }
    }
    if (timed) GDGS_HIP_TRY(hipEventRecord(ev1, st));
    return GDGS_OK;
}

int pitch_of(int cols) { return (cols + 31) / 32 * 32; }

}  // namespace

gdgs_status mg_plan(int W, int H, const gdgs_mg_params* mg, MgPlan* plan) {
    MgPlan p;
    gdgs_mg_params d{0, 2, 2, 20, 0, 0, 1e-6, 0.0};
    const gdgs_mg_params& q = mg ? *mg : d;
    if (q.levels < 0 || q.levels > kMaxLevels || q.pre_sweeps < 1 || q.pre_sweeps > 2 ||
        q.post_sweeps < 1 || q.post_sweeps > 2 || q.max_cycles < 1 || q.max_cycles > 64 ||
        q.coarse_sweeps < 0 || q.coarse_sweeps > 4096 || !(q.tol >= 0.0) ||
        !(q.smooth_weight == 0.0 || (q.smooth_weight >= 0.5 && q.smooth_weight <= 1.5))) {
        set_error("invalid multigrid parameters (levels %d, sweeps %d/%d, cycles %d, tol %g, "
                  "smoothing weight %g)",
                  q.levels, q.pre_sweeps, q.post_sweeps, q.max_cycles, q.tol, q.smooth_weight);
        return GDGS_ERR_INVALID_ARGUMENT;
    }
    if ((q.flags & ~(GDGS_MG_WARM_START | GDGS_MG_RESUME | GDGS_MG_NEUMANN | GDGS_MG_FMG |
                     GDGS_MG_STOP_ETA)) != 0) {
        set_error("unknown multigrid flags 0x%x", q.flags);
        return GDGS_ERR_INVALID_ARGUMENT;
    }
    p.warm = (q.flags & GDGS_MG_WARM_START) != 0;
    p.resume = (q.flags & GDGS_MG_RESUME) != 0;
    p.neumann = (q.flags & GDGS_MG_NEUMANN) != 0;
    p.fmg = (q.flags & GDGS_MG_FMG) != 0 && !p.resume;
    p.stop_eta = (q.flags & GDGS_MG_STOP_ETA) != 0;
    p.pre = q.pre_sweeps;
    p.post = q.post_sweeps;
    p.max_cycles = q.max_cycles;
    p.tol = q.tol;
    p.sw = q.smooth_weight > 0.0 ? (float)q.smooth_weight : kSmoothW;
    // Dirichlet: the interior pixels, in the caller's image; Neumann: every
    // pixel, in a padded array of the workspace (zero ring)
    p.n[0] = p.neumann ? H : H - 2;
    p.m[0] = p.neumann ? W : W - 2;
    p.pitch[0] = p.neumann ? pitch_of(W + 2) : W;
    p.dy[0] = 1.0;
    p.dx[0] = 1.0;
    int L = 1;
    const int want = q.levels == 0 ? kMaxLevels : q.levels;
    // (Neumann: no 1 x 1 grid, whose only point has no neighbour and only the
    // constant mode)
    while (L < want && p.n[L - 1] / 2 >= 1 && p.m[L - 1] / 2 >= 1 &&
           !(p.neumann && p.n[L - 1] / 2 == 1 && p.m[L - 1] / 2 == 1)) {
        p.n[L] = p.n[L - 1] / 2;
        p.m[L] = p.m[L - 1] / 2;
        p.dy[L] = 0.5 * (p.n[L - 1] + p.dy[L - 1]) - p.n[L];
        p.dx[L] = 0.5 * (p.m[L - 1] + p.dx[L - 1]) - p.m[L];
        p.pitch[L] = pitch_of(p.m[L] + 2);
        ++L;
    }
    p.levels = L;
    // coarse grids that fit in one workgroup's LDS: u and f of every grid
    // from lc down, plus the residual of every grid but the coarsest
    const size_t budget = (size_t)lds_budget();
    size_t bytes = 0;
    int lc = L;
    while (lc > 0) {
        const size_t cells = (size_t)(p.n[lc - 1] + 2) * (p.m[lc - 1] + 2);
        const size_t add = sizeof(float) * (size_t)(p.n[lc - 1] + 2) * lds_pitch(p.m[lc - 1]) *
                           (lc - 1 < L - 1 ? 3 : 2);
        if (bytes + add > budget) break;
        // a larger top grid would leave the chip idle while one workgroup per
        // channel smooths it; the tiled kernels take it instead
        if (lc - 1 < L - 1 && cells > (size_t)kLdsTopCells) break;
        bytes += add;
        --lc;
    }
    bytes += 64 * sizeof(float);  // trash cells
    if (lc == L || bytes > budget) {
        set_error("coarsest grid %dx%d does not fit in LDS; use more multigrid levels",
                  p.n[L - 1], p.m[L - 1]);
        return GDGS_ERR_UNSUPPORTED;
    }
    p.lc = lc;
    p.lds_bytes = bytes;
    if (bytes > 64 * 1024 &&
        hipFuncSetAttribute(p.neumann ? (const void*)k_mg_lds<true> : (const void*)k_mg_lds<false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) {
        (void)hipGetLastError();
        set_error("cannot reserve %zu bytes of LDS for the coarse-grid solve", bytes);
        return GDGS_ERR_HIP;
    }
    const int nc = p.n[L - 1], mcc = p.m[L - 1];
    // Jacobi's spectral radius on the coarsest grid.  Neumann: its largest
    // eigenvalue below the constant mode's 1, that of the slowest non-constant
    // mode, which is constant along the shorter side
    const double rj = p.neumann ? 0.5 * (1.0 + cos(M_PI / (nc > mcc ? nc : mcc)))
                                : 0.5 * (cos(M_PI / (nc + 1)) + cos(M_PI / (mcc + 1)));
    p.omega = (float)(2.0 / (1.0 + sqrt(1.0 - rj * rj)));
    if (q.coarse_sweeps > 0) {
        p.coarse_sweeps = q.coarse_sweeps;
    } else {
        // SOR sweeps for a 1e-2 error reduction, (omega - 1)^k <= 1e-2: the
        // coarsest correction only has to be small against the V-cycle's own
        // contraction (about 0.02).  (At 1080p this gives 8; an FP64
        // emulation of the cycle keeps 5 cycles with 6 or more sweeps and
        // needs 9 with 4.)
        const double rho = p.omega - 1.0;
        int k = rho > 0.0 ? (int)ceil(log(1e-2) / log(rho)) : 4;
        if (k < 4) k = 4;
        if (k > 4096) k = 4096;
        p.coarse_sweeps = k;
    }
    GDGS_LOG(3, "multigrid plan %dx%d: %d grids (the last %d in one workgroup), V(%d,%d), "
                "smoothing weight %g, %d coarsest sweeps, tol %g, flags%s%s%s%s%s", W, H,
             p.levels, p.levels - p.lc, p.pre, p.post, (double)p.sw, p.coarse_sweeps, p.tol, p.warm ? " warm" : "",
             p.resume ? " resume" : "", p.neumann ? " neumann" : "", p.fmg ? " fmg" : "",
             p.stop_eta ? " eta" : "");
    *plan = p;
    return GDGS_OK;
}

namespace {
uint32_t div_magic(int d) { return d >= 2 ? (uint32_t)((1ull << 32) / (uint64_t)d + 1) : 0u; }

// LDS layout of the coarse V-cycle: u_l, f_l for l = lc .. L-1, then the
// residuals of lc .. L-2, then 64 trash cells; levels whose colour classes
// fit 4 points per lane of one wave are run by wave 0 alone.
LdsPlan lds_plan(const MgPlan& p, const LevelDev* lev) {
    LdsPlan lp{};
    lp.lc = p.lc;
    lp.L = p.levels;
    int off = 0;
    for (int l = 0; l < p.levels; ++l) {
        lp.n[l] = p.n[l];
        lp.m[l] = p.m[l];
        lp.M[l] = lds_pitch(p.m[l]);
        lp.ey[l] = lev[l].ey;
        lp.ex[l] = lev[l].ex;
        lp.wy[l] = lev[l].wy;
        lp.wx[l] = lev[l].wx;

        lp.mg_m[l] = div_magic(p.m[l]);
        lp.mg_h[l] = div_magic((p.m[l] + 1) / 2);
        if (l >= p.lc) {
            lp.off[l] = off;
            off += 2 * (p.n[l] + 2) * lp.M[l];
        }
    }
    lp.zero0 = p.lc + 1 < p.levels ? lp.off[p.lc + 1] : off;
    for (int l = p.lc; l < p.levels - 1; ++l) {
        lp.roff[l] = off;
        off += (p.n[l] + 2) * lp.M[l];
    }
    if (p.lc == p.levels - 1) lp.zero0 = off;
    lp.zero1 = off;
    lp.trash = off;
    lp.lw = p.levels;
    for (int l = p.levels - 1; l > p.lc; --l) {
        if (p.n[l] * ((p.m[l] + 1) / 2) > 64 * 4) break;
        lp.lw = l;
    }
    return lp;
}

struct PoissonWs {
    float* f0;
    float* u0b;  // second buffer of the finest grid
    float* u0;   // Neumann: the finest grid's iterate (padded); Dirichlet: null (the caller's u)
    double* mean;  // Neumann: mean of rho [0..2], of the solution [3..5], residual offset [6..8]
    double* spart; // Neumann: per-block sums of the centred right-hand side
    float* u[kMaxLevels];
    float* ub[kMaxLevels];
    float* f[kMaxLevels];
    double* part;
    double* bpart;
    double* bnorm;
    int* done;
    int* counters;
    gdgs_stats* stats;
};

int norm_blocks(const MgPlan& p) {
    if (p.lc == 0) return 1;
    return strip_tiles(p.n[0], p.m[0]);
}

int div_blocks(int W, int H) {
    return ((W + kDivTX - 1) / kDivTX) * ((H + kDivRows - 1) / kDivRows);
}

// blocks of the set-up kernels: the image, or the padded Neumann grid
int setup_blocks(const MgPlan& p, int W, int H) {
    return p.neumann ? div_blocks(W + 2, H + 2) : div_blocks(W, H);
}

size_t poisson_layout(const MgPlan& p, int W, int H, void* ws, PoissonWs* out) {
    Carver c(ws);
    PoissonWs w{};
    const size_t fine = p.neumann ? (size_t)3 * (H + 2) * p.pitch[0] : (size_t)3 * H * W;
    w.f0 = c.take<float>(fine);
    w.u0b = c.take<float>(fine);
    w.u0 = p.neumann ? c.take<float>(fine) : nullptr;
    for (int l = 1; l < p.levels; ++l) {
        const size_t cells = (size_t)(p.n[l] + 2) * p.pitch[l];
        w.u[l] = c.take<float>(3 * cells);
        w.ub[l] = c.take<float>(3 * cells);
        w.f[l] = c.take<float>(3 * cells);
    }
    w.part = c.take<double>((size_t)3 * 5 * norm_blocks(p));
    w.bpart = c.take<double>((size_t)3 * 2 * setup_blocks(p, W, H));
    w.bnorm = c.take<double>(6);
    w.mean = c.take<double>(9);
    w.spart = c.take<double>((size_t)3 * setup_blocks(p, W, H));
    w.done = c.take<int>(4);
    w.counters = c.take<int>(kCounters);
    w.stats = c.take<gdgs_stats>(1);
    if (out) *out = w;
    return c.off + 256;
}
}  // namespace

size_t poisson_ws_bytes(const MgPlan& plan, int W, int H) {
    return poisson_layout(plan, W, H, nullptr, nullptr);
}

namespace {
// The grids of one solve: level 0 is the caller's image (Dirichlet) or the
// padded workspace array (Neumann), coarser levels live in the workspace.
void build_levels(const MgPlan& p, const PoissonWs& w, float* u, const float* grad,
                  const float* rho, LevelDev* lev) {
    const bool nm = p.neumann;
    lev[0].u = nm ? w.u0 : u;
    lev[0].ub = w.u0b;
    lev[0].f = (grad || nm) ? w.f0 : rho;
    lev[0].fw = nullptr;
    lev[0].n = p.n[0];
    lev[0].m = p.m[0];
    lev[0].pitch = p.pitch[0];
    lev[0].cs = (long long)(p.n[0] + 2) * p.pitch[0];
    lev[0].ey = lev[0].ex = 0.f;
    lev[0].wy = lev[0].wx = 0.5f;
    for (int l = 1; l < p.levels; ++l) {
        lev[l].u = w.u[l];
        lev[l].ub = w.ub[l];
        lev[l].f = w.f[l];
        lev[l].fw = w.f[l];
        lev[l].n = p.n[l];
        lev[l].m = p.m[l];
        lev[l].pitch = p.pitch[l];
        lev[l].cs = (long long)(p.n[l] + 2) * p.pitch[l];
        lev[l].ey = (float)(1.0 / p.dy[l] - 1.0);
        lev[l].ex = (float)(1.0 / p.dx[l] - 1.0);
        lev[l].wy = (float)(1.0 - 0.5 / p.dy[l]);
        lev[l].wx = (float)(1.0 - 0.5 / p.dx[l]);
    }
    for (int l = 0; l < p.levels; ++l) {
        LevelDev& v = lev[l];
        v.sw = p.sw;
        v.fofs = (nm && l == 0) ? w.mean + 6 : nullptr;
        if (nm) {
            // Neumann: the last row / column has one neighbour fewer and the
            // fine point beyond the last coarse point takes its value (the
            // first-edge terms are the kernels' constants kNmDiag, kNmW)
            v.ey = v.ex = kNmDiag;
            v.wy = v.wx = kNmW;
        }
    }
}

LdsPlan full_lds_plan(const MgPlan& p, const LevelDev* lev) {
    LdsPlan lp = lds_plan(p, lev);
    lp.fofs = lev[0].fofs;
    lp.pre = p.pre;
    lp.post = p.post;
    lp.csweeps = p.coarse_sweeps;
    lp.omega = p.omega;
    lp.sw = p.sw;
    lp.top = lev[p.lc];
    return lp;
}
}  // namespace

gdgs_status launch_poisson(const float* grad, const float* rho, const float* boundary, int W,
                           int H, const MgPlan& p, float* u, gdgs_stats* stats, void* ws,
                           hipStream_t st, const KeyBuilder* key, bool channel_parallel,
                           const uint32_t* tile_ranges) {
    PoissonWs w;
    poisson_layout(p, W, H, ws, &w);
    gdgs_stats* sd = stats ? stats : w.stats;
    const bool nm = p.neumann;
    LevelDev lev[kMaxLevels];
    build_levels(p, w, u, grad, rho, lev);
    const int nblk_div = setup_blocks(p, W, H);
    const dim3 grid_pad((W + 2 + kDivTX - 1) / kDivTX, (H + 2 + kDivRows - 1) / kDivRows, 3);
    auto setup = [&](hipStream_t s) -> gdgs_status {
        if (p.resume) {
            hipLaunchKernelGGL(k_resume, dim3(1), dim3(128), 0, s, w.counters);
            GDGS_LAUNCH_CHECK();
            return GDGS_OK;
        }
        if (nm) {
            hipLaunchKernelGGL(k_nm_init, grid_pad, dim3(kDivTX * kDivTY), 0, s, grad,
                               grad ? nullptr : rho, p.warm ? u : nullptr, H, W, p.pitch[0], w.f0,
                               w.u0, w.u0b, w.bpart, w.counters);
            hipLaunchKernelGGL(k_nm_mean, dim3(3), dim3(256), 0, s, w.bpart, nblk_div, 2,
                               1.0 / ((double)H * W), w.mean);
            hipLaunchKernelGGL(k_nm_center, grid_pad, dim3(kDivTX * kDivTY), 0, s, w.f0, H, W,
                               p.pitch[0], w.mean, w.bpart, w.spart);
            hipLaunchKernelGGL(k_nm_mean, dim3(3), dim3(256), 0, s, w.spart, nblk_div, 1,
                               1.0 / ((double)H * W), w.mean + 6);
            hipLaunchKernelGGL(k_setup_finalize, dim3(3), dim3(256), 0, s, w.bpart, nblk_div,
                               w.bnorm, w.done, w.counters, sd, p.warm ? 1 : 0);
            GDGS_LAUNCH_CHECK();
            return GDGS_OK;
        }
        hipLaunchKernelGGL(k_div_init,
                           dim3((W + kDivTX - 1) / kDivTX, (H + kDivRows - 1) / kDivRows, 3),
                           dim3(kDivTX * kDivTY), 0, s, grad, grad ? nullptr : rho, boundary, H,
                           W, grad ? w.f0 : nullptr, u, w.bpart, w.counters, p.warm ? 1 : 0,
                           grad ? nullptr : tile_ranges);
        hipLaunchKernelGGL(k_setup_finalize, dim3(3), dim3(256), 0, s, w.bpart, nblk_div,
                           w.bnorm, w.done, w.counters, sd, p.warm ? 1 : 0);
        GDGS_LAUNCH_CHECK();
        return GDGS_OK;
    };

    const LdsPlan lp = full_lds_plan(p, lev);
    const int nblk = norm_blocks(p);
    // channels c0 .. c0 + nch - 1 of one grid pass.  pre_nu: nu sweeps (0: the
    // residual of the current iterate restricted, nothing smoothed), from zero
    // (zero) or from grid l's iterate
    auto pre_nu = [&](int l, int nu, bool zero, int c0, int nch, hipStream_t s) {
        const LevelDev &a = lev[l], &b = lev[l + 1];
        const int*  dn = w.done;
        double* pt = w.part;
        if (nu == 0)  // only in the full-multigrid start, which is never timed
            nm ? launch_pre<0, true>(a, b, zero, l == 0, dn, pt, c0, nch, s, false)
               : launch_pre<0, false>(a, b, zero, l == 0, dn, pt, c0, nch, s, false);
        else if (nu == 1)
            nm ? launch_pre<1, true>(a, b, zero, l == 0, dn, pt, c0, nch, s)
               : launch_pre<1, false>(a, b, zero, l == 0, dn, pt, c0, nch, s);
        else
            nm ? launch_pre<2, true>(a, b, zero, l == 0, dn, pt, c0, nch, s)
               : launch_pre<2, false>(a, b, zero, l == 0, dn, pt, c0, nch, s);
    };
    // a V-cycle's pre pass: coarse grids hold corrections that start at zero
    auto pre = [&](int l, int c0, int nch, hipStream_t s) { pre_nu(l, p.pre, l > 0, c0, nch, s); };
    auto post_t = [&](int l, int c0, int nch, hipStream_t s, bool may_time) {
        const LevelDev &a = lev[l], &b = lev[l + 1];
        if (p.post == 1)
            nm ? launch_post<1, true>(a, b, l == 0, w.done, w.part, c0, nch, s, may_time)
               : launch_post<1, false>(a, b, l == 0, w.done, w.part, c0, nch, s, may_time);
        else
            nm ? launch_post<2, true>(a, b, l == 0, w.done, w.part, c0, nch, s, may_time)
               : launch_post<2, false>(a, b, l == 0, w.done, w.part, c0, nch, s, may_time);
    };
    auto post = [&](int l, int c0, int nch, hipStream_t s) { post_t(l, c0, nch, s, true); };
    // the in-workgroup V-cycle over the grids held in LDS
    auto lds_cycle = [&](int c0, int nch, hipStream_t s) {
        if (nm)
            hipLaunchKernelGGL((k_mg_lds<true>), dim3(nch), dim3(kLdsThreads), p.lds_bytes, s, lp,
                               w.done, w.part, c0);
        else
            hipLaunchKernelGGL((k_mg_lds<false>), dim3(nch), dim3(kLdsThreads), p.lds_bytes, s, lp,
                               w.done, w.part, c0);
    };
    // everything of a cycle between the finest pre and post passes
    auto body = [&](int c0, int nch, hipStream_t s) -> gdgs_status {
        for (int l = 1; l < p.lc; ++l) pre(l, c0, nch, s);
        lds_cycle(c0, nch, s);
        for (int l = p.lc - 1; l >= 1; --l) post(l, c0, nch, s);
        GDGS_LAUNCH_CHECK();
        return GDGS_OK;
    };
    auto finalize = [&](int c0, int nch, hipStream_t s) -> gdgs_status {
        hipLaunchKernelGGL(k_cycle_finalize, dim3(nch), dim3(kFinThreads), 0, s, w.part, nblk,
                           w.bnorm, w.done, sd, p.tol, c0, p.stop_eta ? 1 : 0);
        GDGS_LAUNCH_CHECK();
        return GDGS_OK;
    };
    auto cycle = [&](int c0, int nch, hipStream_t s) -> gdgs_status {
        if (p.lc > 0) pre(0, c0, nch, s);
        gdgs_status r = body(c0, nch, s);
        if (r != GDGS_OK) return r;
        if (p.lc > 0) post(0, c0, nch, s);
        return finalize(c0, nch, s);
    };
    // Full-multigrid start (nested iteration on the error equation): the
    // residual of the initial image is restricted down to the first grid held
    // in LDS (pre passes without sweeps leave every coarse iterate zero, and
    // the finest grid's second buffer equal to its iterate); that grid gets one
    // in-LDS V-cycle from zero; then each coarser global grid, from the one
    // above the LDS grids up to grid 1, is set to the interpolation of the
    // grid below (a post pass onto its zero buffer) and gets one V-cycle of
    // its own; the last interpolation corrects the finest grid (its post pass,
    // which also takes the norms), and the cycle is finalized like any other.
    auto fmg_cycle = [&](int c0, int nch, hipStream_t s) -> gdgs_status {
        for (int l = 0; l < p.lc; ++l) pre_nu(l, 0, l > 0, c0, nch, s);
        lds_cycle(c0, nch, s);
        for (int l = p.lc - 1; l >= 1; --l) {
            post(l, c0, nch, s);                  // interpolation onto grid l
            pre_nu(l, p.pre, false, c0, nch, s);  // its V-cycle, from that iterate
            for (int k = l + 1; k < p.lc; ++k) pre(k, c0, nch, s);
            lds_cycle(c0, nch, s);
            for (int k = p.lc - 1; k >= l; --k) post(k, c0, nch, s);
        }
        post_t(0, c0, nch, s, false);
        GDGS_LAUNCH_CHECK();
        return finalize(c0, nch, s);
    };
    const bool use_fmg = p.fmg && p.lc > 0;
    auto first_or = [&](int cyc, int c0, int nch, hipStream_t s) -> gdgs_status {
        return (cyc == 0 && use_fmg) ? fmg_cycle(c0, nch, s) : cycle(c0, nch, s);
    };

    gdgs_status r = GDGS_OK;
    if (key) {
        KeyBuilder ks = *key;
        ks.tag("setup");
        r = with_graph(ks, st, setup);
    } else {
        r = setup(st);
    }
    if (r != GDGS_OK) return r;

    auto run_cycles = [&]() -> gdgs_status {
        // The three colour channels are independent systems: each runs its
        // V-cycles on its own stream, so one channel's bandwidth-bound finest
        // passes overlap another's latency-bound coarse grids.
        const bool timed =
            p.lc > 0 && (timer_active("mg_pre_fine") || timer_active("mg_post_fine") ||
                         timer_active("mg_post_coarse"));
        // a timed coarse post pass launches directly between its events
        const bool coarse_timed = timer_active("mg_post_coarse");
        ChannelStreams cs;
        if (!channel_parallel || !channel_streams_flag() || !channel_streams(st, &cs)) {
            // all channels in each launch, on the caller's stream
            if (!timed) {
                auto all = [&](hipStream_t s) -> gdgs_status {
                    gdgs_status t = GDGS_OK;
                    for (int cyc = 0; cyc < p.max_cycles && t == GDGS_OK; ++cyc)
                        t = first_or(cyc, 0, 3, s);
                    return t;
                };
                if (!key) return all(st);
                KeyBuilder ka = *key;
                ka.tag("cycles3");
                return with_graph(ka, st, all);
            }
            for (int cyc = 0; cyc < p.max_cycles && r == GDGS_OK; ++cyc) {
                if (cyc == 0 && use_fmg) {  // the start is not timed
                    r = fmg_cycle(0, 3, st);
                    continue;
                }
                pre(0, 0, 3, st);
                auto mid = [&](hipStream_t s) { return body(0, 3, s); };
                if (key && !coarse_timed) {
                    KeyBuilder kb = *key;
                    kb.tag("body3");
                    r = with_graph(kb, st, mid);
                } else {
                    r = mid(st);
                }
                if (r != GDGS_OK) break;
                post(0, 0, 3, st);
                r = finalize(0, 3, st);
            }
            return r;
        }
        hipStream_t sc[3] = {st, cs.aux[0], cs.aux[1]};
        GDGS_HIP_TRY(hipEventRecord(cs.fork, st));
        for (int k = 0; k < 2; ++k) GDGS_HIP_TRY(hipStreamWaitEvent(cs.aux[k], cs.fork, 0));
        // Cycles are launched in rounds over the channels, so that all three
        // streams have work queued early.  (Measured alternatives: one graph per
        // channel for all cycles, staggered channel starts, one graph with three
        // branches: none faster; overlapped kernels of different channels slow
        // each other down, so about two run at a time on average.)
        auto run = [&](const char* tag, int c, const std::function<gdgs_status(hipStream_t)>& f) {
            if (!key || coarse_timed) return f(sc[c]);
            KeyBuilder kc = *key;
            kc.tag(tag).add(c);
            return with_graph(kc, sc[c], f);
        };
        for (int cyc = 0; cyc < p.max_cycles && r == GDGS_OK; ++cyc) {
            for (int c = 0; c < 3 && r == GDGS_OK; ++c) {
                if (cyc == 0 && use_fmg) {
                    r = run("fmg", c, [&](hipStream_t s) { return fmg_cycle(c, 1, s); });
                    continue;
                }
                if (!timed) {
                    r = run("cycle", c, [&](hipStream_t s) { return cycle(c, 1, s); });
                    continue;
                }
                // timed finest passes launch directly between their events; the
                // rest of the cycle is replayed from a cached graph
                pre(0, c, 1, sc[c]);
                r = run("body", c, [&](hipStream_t s) { return body(c, 1, s); });
                if (r != GDGS_OK) break;
                post(0, c, 1, sc[c]);
                r = finalize(c, 1, sc[c]);
            }
        }
        // join (also after a failure, so the caller's stream never runs ahead)
        for (int k = 0; k < 2; ++k) {
            GDGS_HIP_TRY(hipEventRecord(cs.join[k], cs.aux[k]));
            GDGS_HIP_TRY(hipStreamWaitEvent(st, cs.join[k], 0));
        }
        return r;
    };
    r = run_cycles();
    if (r != GDGS_OK) return r;
    if (nm) {
        // zero-mean gauge, written to the caller's image
        auto gauge = [&](hipStream_t s) -> gdgs_status {
            hipLaunchKernelGGL(k_nm_usum, grid_pad, dim3(kDivTX * kDivTY), 0, s, w.u0, H, W,
                               p.pitch[0], w.bpart);
            hipLaunchKernelGGL(k_nm_mean, dim3(3), dim3(256), 0, s, w.bpart, nblk_div, 2,
                               1.0 / ((double)H * W), w.mean + 3);
            hipLaunchKernelGGL(k_nm_out,
                               dim3((W + kDivTX - 1) / kDivTX, (H + kDivRows - 1) / kDivRows, 3),
                               dim3(kDivTX * kDivTY), 0, s, w.u0, H, W, p.pitch[0], w.mean + 3, u);
            GDGS_LAUNCH_CHECK();
            return GDGS_OK;
        };
        if (key) {
            KeyBuilder kg = *key;
            kg.tag("gauge");
            r = with_graph(kg, st, gauge);
        } else {
            r = gauge(st);
        }
        if (r != GDGS_OK) return r;
    }
    hipLaunchKernelGGL(k_publish_converged, dim3(1), dim3(64), 0, st, w.done, sd);
    GDGS_LAUNCH_CHECK();
    return GDGS_OK;
}

gdgs_status launch_div_adjoint(const float* lam, int W, int H, float* dgrad, hipStream_t st,
                               bool neumann) {
    const dim3 grid((W + kDivTX - 1) / kDivTX, (H + kDivTY - 1) / kDivTY, 3);
    if (neumann)
        hipLaunchKernelGGL(k_div_adjoint_nm, grid, dim3(kDivTX * kDivTY), 0, st, lam, H, W, dgrad);
    else
        hipLaunchKernelGGL(k_div_adjoint, grid, dim3(kDivTX * kDivTY), 0, st, lam, H, W, dgrad);
    GDGS_LAUNCH_CHECK();
    return GDGS_OK;
}


// ---------------------------------------------------------------- batched solves
// Many Dirichlet solves advance together, one V-cycle per "round": a table of
// up to kBatchMax in-flight solves lives in device memory, and every kernel of
// a round is a persistent grid whose workgroups take the tasks of all active
// solves at one step (a finest-grid strip, a coarse-grid tile, an in-LDS
// coarse V-cycle, a channel's end-of-cycle bookkeeping) from that table, in a
// grid-stride loop.  Each task runs the same device code on the same tile as
// the per-solve kernels, so a solve's result is the same bit for bit alone, in
// any mix, and on the per-solve path.  A solve leaves the table when all its
// channels have converged (or max_cycles is reached); the round's last kernel
// then appends a record to a completion ring in host memory.
namespace {

struct BatchSolve {
    LevelDev lev[kMaxLevels];
    LdsPlan lp;
    int active;     // takes part in rounds
    int reported;   // its completion record has been written (device)
    int lc;         // first grid held in LDS
    int fine_tiles, fine_tx;  // register strips of the finest grid (per channel, per strip row)
    int gx[kMaxLevels], gy[kMaxLevels];  // 32 x 16 tiles of each global coarse grid
    int nblk;       // norm partials per channel
    int stop_eta, max_cycles;
    double tol;
    double* part;
    double* bnorm;
    int* done;
    gdgs_stats* stats;
    long long id;
};

enum : int { kBFinePre = 0, kBFinePost, kBPre, kBPost, kBLds, kBFin };
// launches of a round: finest pre and post, coarse pre and post for levels
// 1 .. kMaxLevels - 1, the in-LDS V-cycle and the finalize
constexpr int kBSteps = 2 + 2 * (kMaxLevels - 1) + 2;
__host__ __device__ constexpr int bstep(int kind, int l) {
    return kind == kBFinePre    ? 0
           : kind == kBFinePost ? 1
           : kind == kBPre      ? 1 + l
           : kind == kBPost     ? kMaxLevels + l
           : kind == kBLds      ? 2 * kMaxLevels
                                : 2 * kMaxLevels + 1;
}
static_assert(bstep(kBFin, 0) == kBSteps - 1, "step numbering");

struct BatchTable {
    long long ring_head;  // records written so far (the device's copy)
    long long pad[7];
    // per step, tasks of the entries before e (written at the start of a round)
    int pref[kBSteps][kBatchMax + 1];
    BatchSolve e[kBatchMax];
};

__device__ __forceinline__ int batch_tasks(const BatchSolve& b, int kind, int l) {
    if (!b.active) return 0;
    if (kind == kBFinePre || kind == kBFinePost) return b.lc > 0 ? 3 * b.fine_tiles : 0;
    if (kind == kBPre || kind == kBPost) return (l >= 1 && l < b.lc) ? 3 * b.gx[l] * b.gy[l] : 0;
    return 3;  // in-LDS V-cycle, finalize: one task per channel
}

// Start of a round, one wave (lane e = entry e): the task prefix of every
// step, so that each workgroup of a step reads 65 integers instead of
// scanning the table.
__global__ __launch_bounds__(64) void k_batch_plan(BatchTable* __restrict__ T) {
    static_assert(kBatchMax == 64, "one wave scans the table");
    const int e = threadIdx.x;
    const BatchSolve& b = T->e[e];
    for (int s = 0; s < kBSteps; ++s) {
        int kind, l = 0;
        if (s == 0) kind = kBFinePre;
        else if (s == 1) kind = kBFinePost;
        else if (s < 1 + kMaxLevels) { kind = kBPre; l = s - 1; }
        else if (s < 2 * kMaxLevels) { kind = kBPost; l = s - kMaxLevels; }
        else kind = s == 2 * kMaxLevels ? kBLds : kBFin;
        int v = batch_tasks(b, kind, l);
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(v, d, 64);
            if (e >= d) v += y;
        }
        T->pref[s][e + 1] = v;
        if (e == 0) T->pref[s][0] = 0;
    }
}

// The step's prefix into LDS; returns the total.
__device__ int batch_prefix(const BatchTable* __restrict__ T, int kind, int l, int* pref) {
    const int* src = T->pref[bstep(kind, l)];
    for (int i = threadIdx.x; i <= kBatchMax; i += blockDim.x) pref[i] = src[i];
    __syncthreads();
    return pref[kBatchMax];
}

// The entry holding task q: the largest e with pref[e] <= q (an entry with
// tasks, since q < total).
__device__ __forceinline__ int batch_find(const int* pref, int q) {
    int lo = 0, hi = kBatchMax;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pref[mid] <= q)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Task v of a grid-stride loop: the entry and the task's index inside it.
// Grids are multiples of the 8 XCDs, so every XCD takes a contiguous range of
// tasks (neighbouring tiles meet in one L2), as in the per-solve kernels.
struct BatchTask {
    int e, loc;
    __device__ BatchTask(const int* pref, int v, int total) {
        const int q = xcd_remap(v, total);
        e = __builtin_amdgcn_readfirstlane(batch_find(pref, q));
        loc = __builtin_amdgcn_readfirstlane(q - pref[e]);
    }
};

template <int NU, bool PRE>
__global__ __launch_bounds__(64 * kSNW) void k_batch_fine(const BatchTable* __restrict__ T) {
    __shared__ int pref[kBatchMax + 1];
    __shared__ float2 sx[2][kSNW][2][64];
    const int total = batch_prefix(T, PRE ? kBFinePre : kBFinePost, 0, pref);
    for (int v = blockIdx.x; v < total; v += gridDim.x) {
        const BatchTask k(pref, v, total);
        const BatchSolve& B = T->e[k.e];
        const int nt = B.fine_tiles;
        const int c = k.loc / nt, tile = k.loc - c * nt;
        const int* done = B.done;
        double* part = B.part;
        const int ftx = B.fine_tx;
        const LevelDev L = B.lev[0];  // copies: fields in scalar registers
        const LevelDev C = B.lev[1];
        __syncthreads();  // the previous task is done with the LDS
        if (done[c]) continue;  // uniform over the block
        const Strip S(c, tile, ftx);
        if (PRE) {
            if (S.interior(L))
                fine_pre_body<NU, true, false>(L, C, part, nt, S, sx);
            else
                fine_pre_body<NU, false, false>(L, C, part, nt, S, sx);
        } else {
            if (S.interior(L))
                fine_post_body<NU, true, false>(L, C, part, nt, S, sx);
            else
                fine_post_body<NU, false, false>(L, C, part, nt, S, sx);
        }
    }
}

template <int NU, bool PRE>
__device__ __forceinline__ void batch_mg(const BatchTable* __restrict__ T, int l) {
    __shared__ int pref[kBatchMax + 1];
    const int total = batch_prefix(T, PRE ? kBPre : kBPost, l, pref);
    for (int v = blockIdx.x; v < total; v += gridDim.x) {
        const BatchTask k(pref, v, total);
        const BatchSolve& B = T->e[k.e];
        const int gx = B.gx[l], gy = B.gy[l], per = gx * gy;
        const int c = k.loc / per, t = k.loc - c * per;
        const int ty = t / gx, tx = t - ty * gx;
        const int* done = B.done;
        double* part = B.part;
        const LevelDev L = B.lev[l];
        const LevelDev C = B.lev[l + 1];
        __syncthreads();
        if (PRE)
            mg_pre_tile<NU, false, kTXs, kTYs, kNTs, false>(L, C, 1, done, part,
                                                            TileId(tx, ty, c), gx, gy);
        else
            mg_post_tile<NU, false, kTXs, kTYs, kNTs, false>(L, C, done, part,
                                                             TileId(tx, ty, c), gx, gy);
    }
}

// Coarse-grid tiles (the pre pass at 8 waves per SIMD: its registers allow
// it without spilling; the post pass keeps its registers).
template <int NU>
__global__ __launch_bounds__(kNTs) __attribute__((amdgpu_waves_per_eu(8))) void k_batch_mg_pre(
    const BatchTable* __restrict__ T, int l) {
    batch_mg<NU, true>(T, l);
}
template <int NU>
__global__ __launch_bounds__(kNTs) void k_batch_mg_post(const BatchTable* __restrict__ T, int l) {
    batch_mg<NU, false>(T, l);
}

__global__ __launch_bounds__(kLdsThreads) void k_batch_lds(const BatchTable* __restrict__ T) {
    extern __shared__ float lds[];
    __shared__ double sh[3 * (kLdsThreads / 64)];
    __shared__ int pref[kBatchMax + 1];
    __shared__ LdsPlan sp;  // the task's plan, read from LDS by every thread
    const int total = batch_prefix(T, kBLds, 0, pref);
    for (int v = blockIdx.x; v < total; v += gridDim.x) {
        const BatchTask k(pref, v, total);
        const BatchSolve& B = T->e[k.e];
        const int* done = B.done;
        double* part = B.part;
        __syncthreads();
        {
            static_assert(sizeof(LdsPlan) % 4 == 0, "copied as 32-bit words");
            const uint32_t* src = reinterpret_cast<const uint32_t*>(&B.lp);
            uint32_t* dst = reinterpret_cast<uint32_t*>(&sp);
            for (int i = threadIdx.x; i < (int)(sizeof(LdsPlan) / 4); i += blockDim.x)
                dst[i] = src[i];
        }
        __syncthreads();
        mg_lds_task<false>(sp, done, part, k.loc, lds, sh);
    }
}

__global__ __launch_bounds__(kFinThreads) void k_batch_finalize(const BatchTable* __restrict__ T) {
    __shared__ double sh[3 * (kFinThreads / 64)];
    __shared__ int pref[kBatchMax + 1];
    const int total = batch_prefix(T, kBFin, 0, pref);
    for (int v = blockIdx.x; v < total; v += gridDim.x) {
        const BatchTask k(pref, v, total);
        const BatchSolve& B = T->e[k.e];
        const double* part = B.part;
        const double* bnorm = B.bnorm;
        int* done = B.done;
        gdgs_stats* st = B.stats;
        const int nblk = B.nblk, stop_eta = B.stop_eta;
        const double tol = B.tol;
        __syncthreads();
        finalize_task(part, nblk, bnorm, done, st, tol, k.loc, stop_eta, sh);
    }
}

// One wave, lane e = entry e: a solve whose channels have all converged (or
// that has reached max_cycles) stops taking work and gets a completion record
// in the host ring, in entry order; then the ring's head is published.
__global__ __launch_bounds__(64) void k_batch_complete(BatchTable* __restrict__ T,
                                                        BatchRing* __restrict__ ring) {
    const int e = threadIdx.x;
    BatchSolve& B = T->e[e];
    bool rep = false;
    int cyc = 0, all = 0;
    double eta = 0.0, rr = 0.0;
    if (B.active && !B.reported) {
        int* d = B.done;
        gdgs_stats* st = B.stats;
        all = d[0] && d[1] && d[2];
        cyc = max(st->cycles[0], max(st->cycles[1], st->cycles[2]));
        if (all || cyc >= B.max_cycles) {
            rep = true;
            st->converged = all;
            if (!all) d[0] = d[1] = d[2] = 1;  // no further work for it
            B.reported = 1;
            eta = fmax(st->eta[0], fmax(st->eta[1], st->eta[2]));
            rr = fmax(st->rel_res[0], fmax(st->rel_res[1], st->rel_res[2]));
        }
    }
    const unsigned long long m = __ballot(rep);
    const long long head = T->ring_head;
    if (rep) {
        const long long k = head + __popcll(m & ((1ull << e) - 1ull));
        BatchRec* r = &ring->rec[k % kRingCap];
        __hip_atomic_store(&r->id, B.id, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&r->cycles, cyc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&r->converged, all, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&r->eta, eta, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&r->rel_res, rr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");  // system scope: the records before the head
    if (e == 0 && m != 0ull) {
        const long long nh = head + __popcll(m);
        T->ring_head = nh;
        __hip_atomic_store(&ring->head, nh, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// Entry e <- v (v travels as a kernel argument, so the host keeps no staging
// buffer alive); active 0 only clears the entry's flag.
__global__ void k_batch_set(BatchTable* __restrict__ T, int e, BatchSolve v, int whole) {
    if (!whole) {
        if (threadIdx.x == 0) T->e[e].active = 0;
        return;
    }
    static_assert(sizeof(BatchSolve) % 4 == 0, "copied as 32-bit words");
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&v);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&T->e[e]);
    for (int i = threadIdx.x; i < (int)(sizeof(BatchSolve) / 4); i += blockDim.x) dst[i] = src[i];
}

__global__ void k_batch_clear(BatchTable* __restrict__ T) {
    if (threadIdx.x == 0) T->ring_head = 0;
    if (threadIdx.x < kBatchMax) {
        T->e[threadIdx.x].active = 0;
        T->e[threadIdx.x].reported = 1;
    }
}

// Persistent grid of a kernel: the workgroups resident at once on the whole
// chip (occupancy x compute units), a multiple of the 8 XCDs.
int persistent_grid(const void* fn, int threads, size_t dyn_lds) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, threads, dyn_lds) != hipSuccess ||
        cus <= 0 || per <= 0) {
        (void)hipGetLastError();
        return 8 * kXcds;
    }
    const int g = cus * per;
    return g < kXcds ? kXcds : g / kXcds * kXcds;
}

}  // namespace

size_t batch_table_bytes() { return sizeof(BatchTable); }

bool batch_supported(const MgPlan& p) {
    if (p.neumann || p.fmg || p.resume) return false;
    for (int l = 1; l < p.lc; ++l) {
        const int nb = ((p.m[l] + 2 + kTX - 1) / kTX) * ((p.n[l] + 2 + kTY - 1) / kTY) * 3;
        if (nb >= kSmallTileBelow) return false;  // the batched kernels use the small tiles
    }
    return true;
}

int batch_depth(const MgPlan& p) { return p.lc > 1 ? p.lc - 1 : 0; }

gdgs_status batch_clear(void* table, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_clear, dim3(1), dim3(kBatchMax), 0, st,
                       static_cast<BatchTable*>(table));
    GDGS_LAUNCH_CHECK();
    return GDGS_OK;
}

gdgs_status launch_poisson_setup(const float* grad, const float* boundary, int W, int H,
                                 const MgPlan& p, float* u, gdgs_stats* stats, void* ws,
                                 hipStream_t st) {
    if (!batch_supported(p)) {
        set_error("this solve cannot run batched");
        return GDGS_ERR_UNSUPPORTED;
    }
    PoissonWs w;
    poisson_layout(p, W, H, ws, &w);
    gdgs_stats* sd = stats ? stats : w.stats;
    hipLaunchKernelGGL(k_div_init, dim3((W + kDivTX - 1) / kDivTX, (H + kDivRows - 1) / kDivRows, 3),
                       dim3(kDivTX * kDivTY), 0, st, grad, nullptr, boundary, H, W, w.f0, u,
                       w.bpart, w.counters, p.warm ? 1 : 0, nullptr);
    hipLaunchKernelGGL(k_setup_finalize, dim3(3), dim3(256), 0, st, w.bpart,
                       setup_blocks(p, W, H), w.bnorm, w.done, w.counters, sd, p.warm ? 1 : 0);
    GDGS_LAUNCH_CHECK();
    return GDGS_OK;
}

gdgs_status batch_activate(void* table, int e, int64_t id, const float* grad, int W, int H,
                           const MgPlan& p, float* u, gdgs_stats* stats, void* ws,
                           hipStream_t st) {
    if (e < 0 || e >= kBatchMax || !batch_supported(p)) {
        set_error("bad batch entry %d or unsupported solve", e);
        return GDGS_ERR_INVALID_ARGUMENT;
    }
    PoissonWs w;
    poisson_layout(p, W, H, ws, &w);
    BatchSolve b;
    std::memset(&b, 0, sizeof(b));
    build_levels(p, w, u, grad, nullptr, b.lev);
    b.lp = full_lds_plan(p, b.lev);
    b.active = 1;
    b.reported = 0;
    b.lc = p.lc;
    b.fine_tiles = strip_tiles(p.n[0], p.m[0]);
    b.fine_tx = strip_tiles_x(p.m[0]);
    for (int l = 1; l < p.levels; ++l) {
        b.gx[l] = (p.m[l] + 2 + kTXs - 1) / kTXs;
        b.gy[l] = (p.n[l] + 2 + kTYs - 1) / kTYs;
    }
    b.nblk = norm_blocks(p);
    b.stop_eta = p.stop_eta ? 1 : 0;
    b.max_cycles = p.max_cycles;
    b.tol = p.tol;
    b.part = w.part;
    b.bnorm = w.bnorm;
    b.done = w.done;
    b.stats = stats ? stats : w.stats;
    b.id = (long long)id;
    hipLaunchKernelGGL(k_batch_set, dim3(1), dim3(256), 0, st, static_cast<BatchTable*>(table),
                       e, b, 1);
    GDGS_LAUNCH_CHECK();
    return GDGS_OK;
}

gdgs_status batch_deactivate(void* table, int e, hipStream_t st) {
    BatchSolve b;
    std::memset(&b, 0, sizeof(b));
    hipLaunchKernelGGL(k_batch_set, dim3(1), dim3(64), 0, st, static_cast<BatchTable*>(table),
                       e, b, 0);
    GDGS_LAUNCH_CHECK();
    return GDGS_OK;
}

namespace {
int g_fine[2][2], g_mg[2][2], g_lds, g_fin;  // persistent grid sizes (set once)
gdgs_status enqueue_batch_round(const BatchTable* T, BatchRing* ring, int depth, int pre,
                                int post, int a, int b, size_t lds_bytes, hipStream_t st);
}  // namespace

gdgs_status launch_batch_round(void* table, BatchRing* ring, int depth, int pre, int post,
                               hipStream_t st) {
    static bool sized = false;
    const size_t lds_bytes = (size_t)lds_budget();
    if (!sized) {
        if (hipFuncSetAttribute((const void*)k_batch_lds,
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds_bytes) != hipSuccess) {
            (void)hipGetLastError();
            set_error("cannot reserve %zu bytes of LDS for the batched coarse solve", lds_bytes);
            return GDGS_ERR_HIP;
        }
        g_fine[0][0] = persistent_grid((const void*)k_batch_fine<1, true>, 64 * kSNW, 0);
        g_fine[0][1] = persistent_grid((const void*)k_batch_fine<2, true>, 64 * kSNW, 0);
        g_fine[1][0] = persistent_grid((const void*)k_batch_fine<1, false>, 64 * kSNW, 0);
        g_fine[1][1] = persistent_grid((const void*)k_batch_fine<2, false>, 64 * kSNW, 0);
        g_mg[0][0] = persistent_grid((const void*)k_batch_mg_pre<1>, kNTs, 0);
        g_mg[0][1] = persistent_grid((const void*)k_batch_mg_pre<2>, kNTs, 0);
        g_mg[1][0] = persistent_grid((const void*)k_batch_mg_post<1>, kNTs, 0);
        g_mg[1][1] = persistent_grid((const void*)k_batch_mg_post<2>, kNTs, 0);
        g_lds = persistent_grid((const void*)k_batch_lds, kLdsThreads, lds_bytes);
        g_fin = persistent_grid((const void*)k_batch_finalize, kFinThreads, 0);
        sized = true;
    }
    if (depth < 0 || depth >= kMaxLevels || pre < 1 || pre > 2 || post < 1 || post > 2) {
        set_error("bad batched round (depth %d, sweeps %d/%d)", depth, pre, post);
        return GDGS_ERR_INVALID_ARGUMENT;
    }
    const BatchTable* T = static_cast<const BatchTable*>(table);
    const int a = pre - 1, b = post - 1;
    // the round's launches depend only on the table, the ring, the depth and
    // the sweeps: one cached graph per such set, replayed every round
    KeyBuilder kb;
    kb.tag("batch-round").add(table).add(ring).add(depth).add(pre).add(post);
    return with_graph(kb, st, [&](hipStream_t s) -> gdgs_status {
        return enqueue_batch_round(T, ring, depth, pre, post, a, b, lds_bytes, s);
    });
}

namespace {
gdgs_status enqueue_batch_round(const BatchTable* T, BatchRing* ring, int depth, int pre,
                                int post, int a, int b, size_t lds_bytes, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(64), 0, st, const_cast<BatchTable*>(T));
    if (pre == 1)
        hipLaunchKernelGGL((k_batch_fine<1, true>), dim3(g_fine[0][a]), dim3(64 * kSNW), 0, st, T);
    else
        hipLaunchKernelGGL((k_batch_fine<2, true>), dim3(g_fine[0][a]), dim3(64 * kSNW), 0, st, T);
    for (int l = 1; l <= depth; ++l) {
        if (pre == 1)
            hipLaunchKernelGGL((k_batch_mg_pre<1>), dim3(g_mg[0][a]), dim3(kNTs), 0, st, T, l);
        else
            hipLaunchKernelGGL((k_batch_mg_pre<2>), dim3(g_mg[0][a]), dim3(kNTs), 0, st, T, l);
    }
    hipLaunchKernelGGL(k_batch_lds, dim3(g_lds), dim3(kLdsThreads), lds_bytes, st, T);
    for (int l = depth; l >= 1; --l) {
        if (post == 1)
            hipLaunchKernelGGL((k_batch_mg_post<1>), dim3(g_mg[1][b]), dim3(kNTs), 0, st, T, l);
        else
            hipLaunchKernelGGL((k_batch_mg_post<2>), dim3(g_mg[1][b]), dim3(kNTs), 0, st, T, l);
    }
    if (post == 1)
        hipLaunchKernelGGL((k_batch_fine<1, false>), dim3(g_fine[1][b]), dim3(64 * kSNW), 0, st, T);
    else
        hipLaunchKernelGGL((k_batch_fine<2, false>), dim3(g_fine[1][b]), dim3(64 * kSNW), 0, st, T);
    hipLaunchKernelGGL(k_batch_finalize, dim3(g_fin), dim3(kFinThreads), 0, st, T);
    hipLaunchKernelGGL(k_batch_complete, dim3(1), dim3(64), 0, st, const_cast<BatchTable*>(T),
                       ring);
    GDGS_LAUNCH_CHECK();
    return GDGS_OK;
}
}  // namespace

}  // namespace gdgs
