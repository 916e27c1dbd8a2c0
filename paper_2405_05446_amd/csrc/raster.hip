// Front-to-back compositing of the projected gradient field (GDGS Sec. 1.2,
// Eq. 11, applied to the projected field in Sec. 2.2 "Projection", Eq. 20) and
// its reverse-mode derivative.
//
// Forward: a transpose kernel packs each splat into a 64-byte record (read
// with three float4 loads, coalesced by splat index); then one workgroup per
// 16x16 screen tile, one thread per pixel.  The tile's pairs (already in
// front-to-back order) are consumed in batches of 256: every thread fetches
// one record into LDS, then all threads walk the batch reading the records as
// LDS broadcasts.  A wave covers one 8 x 8 quadrant of the tile and skips,
// as a whole, every splat whose support ellipse misses it (an exact test
// with a rounding margin, so no pixel loses a contribution).  A pixel stops
// accumulating once its transmittance is below 1e-7; the tile stops when all
// its pixels have.  Splat means are stored relative to the pixel origin of
// the splat's tile rectangle; when a record enters a tile's batch its mean is
// made relative to that tile and its conic prescaled by -log2(e) (once, in
// FP64), so each pixel evaluates the exponent with six operations and one
// exp2.
//
// The same kernel composites the three Laplacian channels of the Laplacian
// splats of Sec. 2.2 (NCH = 3: records carry v0..v2, zero beyond).
//
// Backward: same traversal; each pixel recomputes a_k and T_{k-1} exactly as
// the forward did, so its running prefix sum of v w equals the forward's and
// the suffix S_k = out - prefix_k needs no division by transmittance.  For
// every (pixel, splat) the 12 partial derivatives are summed over the
// workgroup (wave shuffles + LDS) into one record per pair; a second kernel
// sums each splat's pair records in a fixed order (tile order of its
// rectangle; position found by binary search in the tile's depth-ranked
// range), so the result is deterministic.
#include "internal.hpp"

namespace gdgs {
namespace {

constexpr int kBatch = 256;

__global__ void k_inv_order(const uint32_t* __restrict__ order, int64_t K,
                            uint32_t* __restrict__ inv) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < K) {
        const uint32_t k = order[s];
        if (k < (uint64_t)K) inv[k] = (uint32_t)s;
    }
}

// Record of splat k: (mx, my, ox, oy), (a, 2b, c, alpha), (v0..v3),
// (v4, v5, ylo, yhi).  [ylo, yhi] bounds the image rows of the support with a
// small safety margin (+-inf if the FP32 conic is not positive definite).
__global__ __launch_bounds__(256) void k_build_records(gdgs_proj proj,
                                                       const float* __restrict__ opacity,
                                                       const float* __restrict__ value, int64_t K,
                                                       int nch, float4* __restrict__ rec) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    // every load is issued before the culled test (one memory latency, not two)
    const uint32_t cnt = proj.count[k];
    const uint32_t r0 = proj.rect[k], r1 = proj.rect[K + k];
    const float mx = proj.mean2d[k], my = proj.mean2d[K + k];
    const float ca = proj.conic[k], cb = proj.conic[K + k], cc = proj.conic[2 * K + k];
    const float op = opacity[k];
    float vv[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) vv[m] = m < nch ? value[(size_t)m * K + k] : 0.f;
    if (cnt == 0) return;
    const float ox = (float)(kTile * (int)(r0 & 0xFFFF)), oy = (float)(kTile * (int)(r1 & 0xFFFF));
    const float det = ca * cc - cb * cb;
    float ylo = -INFINITY, yhi = INFINITY;
    if (det > 0.f && ca > 0.f) {
        const float ry = sqrtf(kEcut * (ca / det)) * 1.0001f + 1e-3f;
        ylo = oy + my - ry;
        yhi = oy + my + ry;
    }
    float4* r = rec + 4 * (size_t)k;
    r[0] = make_float4(mx, my, ox, oy);
    r[1] = make_float4(ca, 2.f * cb, cc, op);
    // value rows past nch (the Laplacian form has three) are zero
    r[2] = make_float4(vv[0], vv[1], vv[2], vv[3]);
    r[3] = make_float4(vv[4], vv[5], ylo, yhi);
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Quadrant mask of a record from its support rows [ylo, yhi]: bits 0 and 1
// (the tile's left and right 8 x 8 quadrants of rows 0..7) if those rows are
// met, bits 2 and 3 likewise for rows 8..15.
__device__ __forceinline__ uint32_t quad_rows(float ylo, float yhi, int ty) {
    const float r0 = (float)(ty * kTile) + 0.5f;
    uint32_t m = 0;
    if (!(yhi < r0 || ylo > r0 + 7.f)) m |= 3u;
    if (!(yhi < r0 + 8.f || ylo > r0 + 15.f)) m |= 12u;
    return m;
}

// Per (tile, splat) pair, set up once when the record enters a tile's batch:
// the mean relative to the tile's pixel origin and the conic scaled by
// -log2(e), so that a pixel at tile-relative centre (x, y) in [0.5, 15.5]
// evaluates E' = -log2(e) E with two subtractions and four multiply-adds,
// G = exp2(E'), and the support test E <= E_cut is E' >= kEcutL.
// q0 = (a', 2b', c', mx), q1 = (my, alpha, 0, 0).  (A fully expanded
// quadratic in (x, y) would save two more operations but loses ~1e-3 in E
// to cancellation for sub-pixel splats.)
constexpr float kEcutL = -16.609640474436812f;  // -E_cut log2(e) = log2(1e-5)
__device__ __forceinline__ void pair_form(const float4& r0, const float4& r1, int tx, int ty,
                                          float4& q0, float4& q1) {
    const double mx = ((double)r0.z - 16.0 * tx) + (double)r0.x;  // tile-relative mean
    const double my = ((double)r0.w - 16.0 * ty) + (double)r0.y;
    const double sc = -1.4426950408889634;  // -log2(e)
    q0 = make_float4((float)(sc * r1.x), (float)(sc * r1.y), (float)(sc * r1.z), (float)mx);
    q1 = make_float4((float)my, r1.w, 0.f, 0.f);
}

__device__ __forceinline__ float pair_exponent(const float4& q0, const float4& q1, float x,
                                               float y) {
    const float dx = x - q0.w, dy = y - q1.x;
    return dx * fmaf(q0.x, dx, q0.y * dy) + q0.z * dy * dy;
}

// Quadrants of a tile (8 x 8 pixel centres; bit q: columns 8 (q & 1) ..,
// rows 8 (q >> 1) ..) that the support ellipse {E <= E_cut} meets, among
// those in m.  With the pair form below, E' = -(A dx^2 + B dx dy + C dy^2)
// and the support is A dx^2 + B dx dy + C dy^2 <= -log2(1e-5).  Unless the
// centre lies in the rectangle, the minimum of the quadratic over it lies on
// an edge; on a vertical edge dx = X it is C (dy - dy*)^2 + X^2 D / C with
// dy* = -B X / (2C) clamped to the edge and D = A C - B^2 / 4 (horizontal
// edges alike), a sum of non-negative terms.  A quadrant is dropped only if
// that minimum exceeds the threshold by a margin above the FP32 rounding of
// both this test and the per-pixel exponent, so no pixel that would blend
// the splat loses it.
__device__ __forceinline__ uint32_t support_quads(const float4& q0, const float4& q1,
                                                  uint32_t m) {
    const float A = -q0.x, B = -q0.y, C = -q0.z, mx = q0.w, my = q1.x;
    const double D = (double)A * (double)C - 0.25 * (double)B * (double)B;
    if (!(A > 0.f) || !(C > 0.f) || !(D > 0.0)) return m;
    const float rA = 1.f / A, rC = 1.f / C;
    const float Df = (float)D, DA = Df * rA, DC = Df * rC;
    const float sv = -0.5f * B * rC, sh = -0.5f * B * rA;
    // edges at pixel centres 0.5, 7.5, 8.5, 15.5: X (columns), Y (rows), the
    // clamp-free minimisers along them and the constant parts of the minima
    float X[4], Y[4], v[4], w[4], h[4], g[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float e = (float)(8 * (k >> 1)) + ((k & 1) ? 7.5f : 0.5f);
        X[k] = e - mx;
        Y[k] = e - my;
        v[k] = sv * X[k];
        w[k] = X[k] * X[k] * DC;
        h[k] = sh * Y[k];
        g[k] = Y[k] * Y[k] * DA;
    }
    constexpr float thr = -kEcutL * 1.001f + 1e-3f;
    uint32_t keep = 0;
#pragma unroll
    for (int qd = 0; qd < 4; ++qd) {
        const int i = 2 * (qd & 1), j = 2 * (qd >> 1);
        const float x0 = X[i], x1 = X[i + 1], y0 = Y[j], y1 = Y[j + 1];
        const float d0 = v[i] - fminf(fmaxf(v[i], y0), y1);
        const float d1 = v[i + 1] - fminf(fmaxf(v[i + 1], y0), y1);
        const float e0 = h[j] - fminf(fmaxf(h[j], x0), x1);
        const float e1 = h[j + 1] - fminf(fmaxf(h[j + 1], x0), x1);
        float q = fminf(fmaf(C * d0, d0, w[i]), fmaf(C * d1, d1, w[i + 1]));
        q = fminf(q, fmaf(A * e0, e0, g[j]));
        q = fminf(q, fmaf(A * e1, e1, g[j + 1]));
        if (x0 <= 0.f && x1 >= 0.f && y0 <= 0.f && y1 >= 0.f) q = 0.f;
        const float lim =
            fmaf(1e-5f, A * fmaxf(x0 * x0, x1 * x1) + C * fmaxf(y0 * y0, y1 * y1), thr);
        if (q <= lim) keep |= 1u << qd;
    }
    return m & keep;
}

// Composite one splat into a pixel (the Eq. 20 update); counts the
// contributions when asked to.
template <bool COUNT, int NCH>
__device__ __forceinline__ void blend(const float4& q0, const float4& q1, const float4& r2,
                                      const float4& r3, float x, float y, float& Tr,
                                      float (&acc)[NCH], uint32_t& ncon) {
    const float Ep = pair_exponent(q0, q1, x, y);
    if (Ep >= kEcutL && Tr >= kTmin) {
        if (COUNT && q1.y > 0.f) ++ncon;
        const float al = q1.y * __builtin_amdgcn_exp2f(Ep);
        const float w = al * Tr;
        acc[0] += r2.x * w;
        acc[1] += r2.y * w;
        acc[2] += r2.z * w;
        if constexpr (NCH == 6) {
            acc[3] += r2.w * w;
            acc[4] += r3.x * w;
            acc[5] += r3.y * w;
        }
        Tr = Tr - al * Tr;
    }
}

// COUNT: write no image; add the number of (pixel, splat) contributions of
// the block to counts[0] (profiling only).  NCH: channels written (6 image
// gradients, or 3 Laplacians).
// THR: the hard threshold of Eq. 24 (Sec. 3.1) is applied to each composited
// value before it is stored (a value is kept when |x| >= thr), and the kept
// non-zero values are counted into counts[0].
template <bool COUNT, int NCH, bool THR = false>
__global__ __launch_bounds__(256) void k_raster_fwd(const float4* __restrict__ rec,
                                                    const uint32_t* __restrict__ splat_of_pair,
                                                    const uint32_t* __restrict__ ranges,
                                                    const uint32_t* __restrict__ tile_order, int T,
                                                    int nx, int W, int H, int64_t K,
                                                    float* __restrict__ grad,
                                                    unsigned long long* __restrict__ counts,
                                                    float thr = 0.f) {
    // per batch entry: the pair's exponent form (s_r0, s_r1) and the values
    // (s_r2, s_r3); slot kBatch is inert (alpha 0), used to pad the wave lists
    __shared__ float4 s_r0[kBatch + 1], s_r1[kBatch + 1], s_r2[kBatch + 1], s_r3[kBatch + 1];
    __shared__ uint32_t s_mask[kBatch];
    __shared__ int s_list[4][kBatch + 4];
    // blocks take the tiles heaviest first (or by id): round-robin dispatch
    // over the XCDs balances the uneven tile costs better than giving each
    // XCD one band of the image
    const uint32_t tile = tile_order ? tile_order[blockIdx.x] : blockIdx.x;
    if (tile >= (uint32_t)T) return;
    const int tx = tile % nx, ty = tile / nx;
    const int t = threadIdx.x, lane = __lane_id(), wv = t >> 6;
    // wave wv: the 8 x 8 quadrant (wv & 1, wv >> 1) of the tile
    const int ox = 8 * (wv & 1) + (lane & 7), oy = 8 * (wv >> 1) + (lane >> 3);
    const int px = tx * kTile + ox, py = ty * kTile + oy;
    const bool inside = px < W && py < H;
    const float xt = (float)ox + 0.5f, yt = (float)oy + 0.5f;  // tile-relative
    const uint64_t lt = lanemask_lt();
    const uint32_t start = ranges[tile], end = ranges[T + tile];
    if (t == 0) {
        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
        s_r0[kBatch] = z;
        s_r1[kBatch] = z;
        s_r2[kBatch] = z;
        s_r3[kBatch] = z;
    }
    float Tr = inside ? 1.f : 0.f;
    float acc[NCH];
#pragma unroll
    for (int m = 0; m < NCH; ++m) acc[m] = 0.f;
    uint32_t ncon = 0;
    for (uint32_t b0 = start; b0 < end; b0 += kBatch) {
        const int n = (int)min((uint32_t)kBatch, end - b0);
        __syncthreads();
        if (t < n) {
            const uint32_t s = splat_of_pair[b0 + t];
            uint32_t m = 0;
            if (s < (uint64_t)K) {
                const float4* r = rec + 4 * (size_t)s;
                const float4 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
                float4 q0, q1;
                pair_form(r0, r1, tx, ty, q0, q1);
                s_r0[t] = q0;
                s_r1[t] = q1;
                s_r2[t] = r2;
                if (NCH > 4) s_r3[t] = r3;
                m = quad_rows(r3.z, r3.w, ty);
                if (m) m = support_quads(q0, q1, m);
            }
            s_mask[t] = m;
        }
        __syncthreads();
        // this wave's list of batch entries whose support meets its quadrant (empty
        // once all 64 pixels of the wave have stopped accumulating)
        const bool wave_live = __ballot(Tr >= kTmin) != 0ull;
        int cnt = 0;
        for (int c0 = 0; wave_live && c0 < n; c0 += 64) {
            const int e = c0 + lane;
            const bool hit = e < n && ((s_mask[e] >> wv) & 1u);
            const uint64_t m = __ballot(hit);
            if (hit) s_list[wv][cnt + __popcll(m & lt)] = e;
            cnt += __popcll(m);
        }
        const int cnt4 = (cnt + 3) & ~3;
        if (lane < cnt4 - cnt) s_list[wv][cnt + lane] = kBatch;
        __builtin_amdgcn_wave_barrier();
        for (int i = 0; i < cnt4; i += 4) {
            const int4 jj = *reinterpret_cast<const int4*>(&s_list[wv][i]);
            const float4 a0 = s_r0[jj.x], a1 = s_r0[jj.y], a2 = s_r0[jj.z], a3 = s_r0[jj.w];
            const float4 c0 = s_r1[jj.x], c1 = s_r1[jj.y], c2 = s_r1[jj.z], c3 = s_r1[jj.w];
            const float4 v0 = s_r2[jj.x], v1 = s_r2[jj.y], v2 = s_r2[jj.z], v3 = s_r2[jj.w];
            const float4 zz = make_float4(0.f, 0.f, 0.f, 0.f);
            const float4 e0 = NCH > 4 ? s_r3[jj.x] : zz, e1 = NCH > 4 ? s_r3[jj.y] : zz;
            const float4 e2 = NCH > 4 ? s_r3[jj.z] : zz, e3 = NCH > 4 ? s_r3[jj.w] : zz;
            blend<COUNT, NCH>(a0, c0, v0, e0, xt, yt, Tr, acc, ncon);
            blend<COUNT, NCH>(a1, c1, v1, e1, xt, yt, Tr, acc, ncon);
            blend<COUNT, NCH>(a2, c2, v2, e2, xt, yt, Tr, acc, ncon);
            blend<COUNT, NCH>(a3, c3, v3, e3, xt, yt, Tr, acc, ncon);
        }
        if (__syncthreads_count(Tr >= kTmin) == 0) break;
    }
    if (COUNT) {
        unsigned long long v = (unsigned long long)ncon;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
        if (lane == 0) atomicAdd(counts, v);
        return;
    }
    uint32_t kept = 0;
    if (inside) {
        const size_t HW = (size_t)H * W, p = (size_t)py * W + px;
#pragma unroll
        for (int m = 0; m < NCH; ++m) {
            const float v = THR ? (fabsf(acc[m]) >= thr ? acc[m] : 0.f) : acc[m];
            grad[m * HW + p] = v;
            kept += (THR && v != 0.f) ? 1u : 0u;
        }
    }
    if (THR && counts) {
        unsigned long long v = kept;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
        if (lane == 0 && v) atomicAdd(counts, v);
    }
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

// Partials per pair: (dmx, dmy, da, db, dc, dalpha, dv0..dv5).
constexpr int kNP = 12;
constexpr int kBatchB = 128;

__global__ __launch_bounds__(256) void k_raster_bwd(const float4* __restrict__ rec,
                                                    const uint32_t* __restrict__ splat_of_pair,
                                                    const uint32_t* __restrict__ ranges,
                                                    const uint32_t* __restrict__ tile_order, int T,
                                                    int nx, int W, int H, int64_t K,
                                                    const float* __restrict__ grad,
                                                    const float* __restrict__ dgrad,
                                                    float* __restrict__ part, int64_t cap) {
    __shared__ float4 s_r0[kBatchB], s_r1[kBatchB], s_r2[kBatchB], s_r3[kBatchB];
    __shared__ float4 s_q0[kBatchB], s_q1[kBatchB];  // the forward's exponent form
    __shared__ float s_p[4][kNP][kBatchB];
    const uint32_t tile = tile_order ? tile_order[blockIdx.x] : blockIdx.x;
    if (tile >= (uint32_t)T) return;
    const int tx = tile % nx, ty = tile / nx;
    const int t = threadIdx.x, lane = __lane_id(), wv = t >> 6;
    const int px = tx * kTile + (t & 15), py = ty * kTile + (t >> 4);
    const bool inside = px < W && py < H;
    const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
    const float xt = (float)(t & 15) + 0.5f, yt = (float)(t >> 4) + 0.5f;
    const size_t HW = (size_t)H * W, pp = (size_t)py * W + px;
    const float wy_lo = (float)(ty * kTile + 4 * wv) + 0.5f, wy_hi = wy_lo + 3.f;
    float out[6], del[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        out[m] = inside ? grad[m * HW + pp] : 0.f;
        del[m] = inside ? dgrad[m * HW + pp] : 0.f;
    }
    const uint32_t start = ranges[tile], end = ranges[T + tile];
    float Tr = inside ? 1.f : 0.f;
    float pre0 = 0.f, pre1 = 0.f, pre2 = 0.f, pre3 = 0.f, pre4 = 0.f, pre5 = 0.f;
    for (uint32_t b0 = start; b0 < end; b0 += kBatchB) {
        const int n = (int)min((uint32_t)kBatchB, end - b0);
        __syncthreads();
        if (t < n) {
            const uint32_t s = splat_of_pair[b0 + t];
            if (s < (uint64_t)K) {
                const float4* r = rec + 4 * (size_t)s;
                const float4 r0 = r[0], r1 = r[1];
                float4 q0, q1;
                pair_form(r0, r1, tx, ty, q0, q1);
                s_r0[t] = r0;
                s_r1[t] = r1;
                s_r2[t] = r[2];
                s_r3[t] = r[3];
                s_q0[t] = q0;
                s_q1[t] = q1;
            } else {  // never produced by the binning; contributes nothing
                const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
                s_r0[t] = z;
                s_r1[t] = z;
                s_r2[t] = z;
                s_r3[t] = z;
                s_q0[t] = z;
                s_q1[t] = z;
            }
        }
        __syncthreads();
        for (int j = 0; j < n; ++j) {
            const float4 r3 = s_r3[j];
            if (r3.w < wy_lo || r3.z > wy_hi) {  // wave-uniform: rows missed
                if (lane == 0) {
#pragma unroll
                    for (int q = 0; q < kNP; ++q) s_p[wv][q][j] = 0.f;
                }
                continue;
            }
            const float4 r0 = s_r0[j], r1 = s_r1[j];
            const float dx = (fpx - r0.z) - r0.x;
            const float dy = (fpy - r0.w) - r0.y;
            // a_k exactly as the forward computed it
            const float Ep = pair_exponent(s_q0[j], s_q1[j], xt, yt);
            const bool on = Ep >= kEcutL && Tr >= kTmin;
            float g[kNP];
#pragma unroll
            for (int q = 0; q < kNP; ++q) g[q] = 0.f;
            if (on) {
                const float4 r2 = s_r2[j];
                const float G = __builtin_amdgcn_exp2f(Ep);
                const float al = r1.w * G;
                const float w = al * Tr;
                const float v[6] = {r2.x, r2.y, r2.z, r2.w, r3.x, r3.y};
                pre0 += v[0] * w;
                pre1 += v[1] * w;
                pre2 += v[2] * w;
                pre3 += v[3] * w;
                pre4 += v[4] * w;
                pre5 += v[5] * w;
                const float pre[6] = {pre0, pre1, pre2, pre3, pre4, pre5};
                const float inv1m = 1.f / (1.f - al);
                float dla = 0.f;
#pragma unroll
                for (int m = 0; m < 6; ++m) {
                    dla += del[m] * (v[m] * Tr - (out[m] - pre[m]) * inv1m);
                    g[6 + m] = del[m] * w;
                }
                g[5] = dla * G;
                const float dE = -dla * r1.w * G;
                g[0] = -dE * (2.f * r1.x * dx + r1.y * dy);
                g[1] = -dE * (r1.y * dx + 2.f * r1.z * dy);
                g[2] = dE * dx * dx;
                g[3] = dE * 2.f * dx * dy;
                g[4] = dE * dy * dy;
                Tr = Tr - al * Tr;
            }
            if (__ballot(on) != 0ull) {
#pragma unroll
                for (int q = 0; q < kNP; ++q) g[q] = wave_sum(g[q]);
            }
            if (lane == 0) {
#pragma unroll
                for (int q = 0; q < kNP; ++q) s_p[wv][q][j] = g[q];
            }
        }
        __syncthreads();
        for (int idx = t; idx < n * kNP; idx += 256) {
            const int j = idx / kNP, q = idx - j * kNP;
            const float v = s_p[0][q][j] + s_p[1][q][j] + s_p[2][q][j] + s_p[3][q][j];
            if (b0 + j < cap) part[(size_t)(b0 + j) * kNP + q] = v;
        }
        if (__syncthreads_count(Tr >= kTmin) == 0) {
            // remaining pairs of this tile contribute nothing
            for (uint32_t i = b0 + n + t; i < end; i += 256)
                for (int q = 0; q < kNP; ++q) part[(size_t)i * kNP + q] = 0.f;
            break;
        }
    }
}

// Per splat: sum its pair records over the tiles of its rectangle.
__global__ __launch_bounds__(256) void k_seg_reduce(
    gdgs_proj proj, const uint32_t* __restrict__ inv, const uint32_t* __restrict__ splat_of_pair,
    const uint32_t* __restrict__ ranges, int T, int nx, int64_t K, const float* __restrict__ part,
    float* __restrict__ dmean2d, float* __restrict__ dconic, float* __restrict__ dopacity,
    float* __restrict__ dvalue) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    float acc[kNP];
#pragma unroll
    for (int q = 0; q < kNP; ++q) acc[q] = 0.f;
    if (proj.count[k] != 0) {
        const uint32_t s = inv[k];
        const uint32_t r0 = proj.rect[k], r1 = proj.rect[K + k];
        const int tx0 = r0 & 0xFFFF, tx1 = r0 >> 16, ty0 = r1 & 0xFFFF, ty1 = r1 >> 16;
        for (int ty = ty0; ty < ty1; ++ty) {
            for (int tx = tx0; tx < tx1; ++tx) {
                const int tl = ty * nx + tx;
                uint32_t lo = ranges[tl], hi = ranges[T + tl];
                // the tile's pairs are in depth-rank order: search rank s
                while (lo < hi) {
                    const uint32_t mid = lo + ((hi - lo) >> 1);
                    const uint32_t km = splat_of_pair[mid];
                    if ((km < (uint64_t)K ? inv[km] : 0xFFFFFFFFu) < s)
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                if (lo < ranges[T + tl] && splat_of_pair[lo] == (uint32_t)k) {
                    const float* p = part + (size_t)lo * kNP;
#pragma unroll
                    for (int q = 0; q < kNP; ++q) acc[q] += p[q];
                }
            }
        }
    }
    dmean2d[k] = acc[0];
    dmean2d[K + k] = acc[1];
    dconic[k] = acc[2];
    dconic[K + k] = acc[3];
    dconic[2 * K + k] = acc[4];
    dopacity[k] = acc[5];
#pragma unroll
    for (int m = 0; m < 6; ++m) dvalue[m * K + k] = acc[6 + m];
}

}  // namespace

size_t raster_ws_bytes(int64_t K) {
    Carver c(nullptr);
    c.take<float4>(4 * (size_t)(K > 0 ? K : 1));
    return c.off + 256;
}

gdgs_status launch_raster(const gdgs_proj& proj, const float* opacity, const float* value,
                          int64_t K, const gdgs_bins& bins, int W, int H, float* grad, void* ws,
                          hipStream_t st, int nch, float thr, unsigned long long* nonzero) {
    if (thr >= 0.f && nch != 3) {
        set_error("the threshold applies to the three-channel (Laplacian) composite");
        return GDGS_ERR_INVALID_ARGUMENT;
    }
    Carver c(ws);
    float4* rec = c.take<float4>(4 * (size_t)(K > 0 ? K : 1));
    const int nx = tiles_x(W), T = nx * tiles_y(H);
    if (K > 0) {
        const unsigned g = (unsigned)((K + 255) / 256);
        hipLaunchKernelGGL(k_build_records, dim3(g), dim3(256), 0, st, proj, opacity, value, K,
                           nch, rec);
    }
    hipEvent_t ev0, ev1;
    const bool timed = timer_events("raster", &ev0, &ev1);
    if (timed) GDGS_HIP_TRY(hipEventRecord(ev0, st));
    if (thr >= 0.f) {
        if (nonzero) {
            const gdgs_status z =
                launch_fill_u32(reinterpret_cast<uint32_t*>(nonzero), 2, 0u, st);
            if (z != GDGS_OK) return z;
        }
        hipLaunchKernelGGL((k_raster_fwd<false, 3, true>), dim3(T), dim3(256), 0, st, rec,
                           bins.splat_of_pair, bins.ranges, bins.tile_order, T, nx, W, H, K, grad,
                           nonzero, thr);
    } else if (nch == 3)
        hipLaunchKernelGGL((k_raster_fwd<false, 3>), dim3(T), dim3(256), 0, st, rec,
                           bins.splat_of_pair, bins.ranges, bins.tile_order, T, nx, W, H, K, grad,
                           nullptr, 0.f);
    else
        hipLaunchKernelGGL((k_raster_fwd<false, 6>), dim3(T), dim3(256), 0, st, rec,
                           bins.splat_of_pair, bins.ranges, bins.tile_order, T, nx, W, H, K, grad,
                           nullptr, 0.f);
    if (timed) GDGS_HIP_TRY(hipEventRecord(ev1, st));
    GDGS_LAUNCH_CHECK();
    return GDGS_OK;
}

gdgs_status launch_raster_count(const gdgs_proj& proj, const float* opacity, const float* value,
                                int64_t K, const gdgs_bins& bins, int W, int H,
                                unsigned long long* counts, void* ws, hipStream_t st) {
    Carver c(ws);
    float4* rec = c.take<float4>(4 * (size_t)(K > 0 ? K : 1));
    const int nx = tiles_x(W), T = nx * tiles_y(H);
    gdgs_status s = launch_fill_u32(reinterpret_cast<uint32_t*>(counts), 2, 0u, st);
    if (s != GDGS_OK) return s;
    if (K > 0) {
        const unsigned g = (unsigned)((K + 255) / 256);
        hipLaunchKernelGGL(k_build_records, dim3(g), dim3(256), 0, st, proj, opacity, value, K,
                           6, rec);
    }
    hipLaunchKernelGGL((k_raster_fwd<true, 6>), dim3(T), dim3(256), 0, st, rec,
                       bins.splat_of_pair, bins.ranges, bins.tile_order, T, nx, W, H, K, nullptr,
                       counts, 0.f);
    GDGS_LAUNCH_CHECK();
    return GDGS_OK;
}

size_t raster_bwd_ws_bytes(int64_t K, int64_t cap) {
    Carver c(nullptr);
    c.take<uint32_t>(K > 0 ? K : 1);
    c.take<float4>(4 * (size_t)(K > 0 ? K : 1));
    c.take<float>((size_t)kNP * (cap > 0 ? cap : 1));
    return c.off + 256;
}

gdgs_status launch_raster_backward(const gdgs_proj& proj, const float* opacity,
                                   const float* value, int64_t K, const gdgs_bins& bins, int W,
                                   int H, const float* grad, const float* dgrad, float* dmean2d,
                                   float* dconic, float* dopacity, float* dvalue, void* ws,
                                   hipStream_t st) {
    if (K == 0) return GDGS_OK;
    Carver c(ws);
    uint32_t* inv = c.take<uint32_t>(K);
    float4* rec = c.take<float4>(4 * (size_t)K);
    float* part = c.take<float>((size_t)kNP * (bins.capacity > 0 ? bins.capacity : 1));
    const int nx = tiles_x(W), T = nx * tiles_y(H);
    const unsigned g = (unsigned)((K + 255) / 256);
    hipLaunchKernelGGL(k_inv_order, dim3(g), dim3(256), 0, st, bins.order, K, inv);
    hipLaunchKernelGGL(k_build_records, dim3(g), dim3(256), 0, st, proj, opacity, value, K, 6,
                       rec);
    hipLaunchKernelGGL(k_raster_bwd, dim3(T), dim3(256), 0, st, rec, bins.splat_of_pair,
                       bins.ranges, bins.tile_order, T, nx, W, H, K, grad, dgrad, part,
                       bins.capacity);
    hipLaunchKernelGGL(k_seg_reduce, dim3(g), dim3(256), 0, st, proj, inv, bins.splat_of_pair,
                       bins.ranges, T, nx, K, part, dmean2d, dconic, dopacity, dvalue);
    GDGS_LAUNCH_CHECK();
    return GDGS_OK;
}

}  // namespace gdgs
