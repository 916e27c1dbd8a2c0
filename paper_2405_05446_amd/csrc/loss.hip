// Image loss of the method's optimisation (GDGS Sec. 2.3 "Loss Function",
// Eq. 22, evaluated in every iteration of Algorithm 1) and its gradient with
// respect to the rendered image, the Adam update of the parameters, and the
// hard threshold of Sec. 3.1 (Eq. 24).
//
// L = (1 - lam) mean|c - im| + beta mean|grad c - grad im| + lam (1 - mean SSIM)
// with forward differences along columns and rows, and SSIM per colour
// channel over an 11 x 11 Gaussian window (sigma 1.5, normalised, zero
// padding), C1 = 0.01^2, C2 = 0.03^2.  With m1 = G*c, m2 = G*im,
// m11 = G*c^2, m22 = G*im^2, m12 = G*(c im):
//   S = (2 m1 m2 + C1)(2 (m12 - m1 m2) + C2) / ((m1^2 + m2^2 + C1)((m11 - m1^2) + (m22 - m2^2) + C2)),
// and, the filter being self-adjoint, d mean S / dc = (G*dS/dm1 + 2 c G*dS/dm11 + im G*dS/dm12) / n.
//
// Pass 1 (one block per 32 x 32 tile of one channel): the tile with a halo of
// 5 in LDS, the five maps filtered along rows then columns in LDS, S and its
// three partials written out, per-block sums of S, |c - im| and the gradient
// differences.  Pass 2: the three partial maps filtered the same way and the
// gradient assembled.  Pass 3: the block sums reduced in a fixed order (FP64).
#include "internal.hpp"

namespace gdgs {
namespace {

constexpr int kLT = 32;               // output tile edge
constexpr int kLR = 5;                // filter radius (11 taps)
constexpr int kLE = kLT + 2 * kLR;    // tile edge with halo
constexpr int kLThreads = 256;
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;

// normalised Gaussian taps, sigma 1.5 (computed in FP64, rounded once)
struct Taps {
    float w[2 * kLR + 1];
};

Taps make_taps() {
    Taps t;
    double s = 0.0, v[2 * kLR + 1];
    for (int i = 0; i < 2 * kLR + 1; ++i) {
        const double x = i - kLR;
        v[i] = exp(-(x * x) / (2.0 * 1.5 * 1.5));
        s += v[i];
    }
    for (int i = 0; i < 2 * kLR + 1; ++i) t.w[i] = (float)(v[i] / s);
    return t;
}

__global__ void k_zero_u64(unsigned long long* p) {
    if (threadIdx.x == 0) *p = 0ull;
}

__device__ __forceinline__ double block_sum_d(double x, double* sh) {
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = x;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += sh[i];
    return s;
}

// Filter NM planes held in LDS (kLE x kLE each, zero outside the image) along
// rows into hb (kLE rows x kLT columns), then along columns into out (kLT x
// kLT) at the caller's pleasure: returns nothing, out via lambda per point.
template <int NM>
__device__ __forceinline__ void filter_rows(const float (*src)[kLE * kLE], float (*hb)[kLE * kLT],
                                           const Taps& tp) {
    for (int idx = threadIdx.x; idx < kLE * kLT; idx += kLThreads) {
        const int r = idx / kLT, q = idx - r * kLT;
        float acc[NM];
#pragma unroll
        for (int m = 0; m < NM; ++m) acc[m] = 0.f;
#pragma unroll
        for (int k = 0; k < 2 * kLR + 1; ++k) {
#pragma unroll
            for (int m = 0; m < NM; ++m) acc[m] += tp.w[k] * src[m][r * kLE + q + k];
        }
#pragma unroll
        for (int m = 0; m < NM; ++m) hb[m][r * kLT + q] = acc[m];
    }
}

template <int NM>
__device__ __forceinline__ void filter_col(const float (*hb)[kLE * kLT], int r, int q,
                                           const Taps& tp, float (&out)[NM]) {
#pragma unroll
    for (int m = 0; m < NM; ++m) out[m] = 0.f;
#pragma unroll
    for (int k = 0; k < 2 * kLR + 1; ++k) {
#pragma unroll
        for (int m = 0; m < NM; ++m) out[m] += tp.w[k] * hb[m][(r + k) * kLT + q];
    }
}

__global__ __launch_bounds__(kLThreads) void k_loss_pass1(const float* __restrict__ c,
                                                          const float* __restrict__ im, int W,
                                                          int H, Taps tp, float* __restrict__ pm,
                                                          double* __restrict__ bsum) {
    __shared__ float s_in[5][kLE * kLE];
    __shared__ float s_h[5][kLE * kLT];
    __shared__ double sh[kLThreads / 64];
    const int ch = blockIdx.z, i0 = blockIdx.y * kLT, j0 = blockIdx.x * kLT;
    const size_t HW = (size_t)H * W;
    const float* x = c + ch * HW;
    const float* y = im + ch * HW;
    for (int idx = threadIdx.x; idx < kLE * kLE; idx += kLThreads) {
        const int r = idx / kLE, q = idx - r * kLE;
        const int gi = i0 - kLR + r, gj = j0 - kLR + q;
        float a = 0.f, b = 0.f;
        if (gi >= 0 && gi < H && gj >= 0 && gj < W) {
            a = x[(size_t)gi * W + gj];
            b = y[(size_t)gi * W + gj];
        }
        s_in[0][idx] = a;
        s_in[1][idx] = b;
        s_in[2][idx] = a * a;
        s_in[3][idx] = b * b;
        s_in[4][idx] = a * b;
    }
    __syncthreads();
    filter_rows<5>(s_in, s_h, tp);
    __syncthreads();
    double sS = 0.0, sL1 = 0.0, sG = 0.0;
    for (int idx = threadIdx.x; idx < kLT * kLT; idx += kLThreads) {
        const int r = idx / kLT, q = idx - r * kLT;
        const int gi = i0 + r, gj = j0 + q;
        if (gi >= H || gj >= W) continue;
        float m[5];
        filter_col<5>(s_h, r, q, tp, m);
        const float m1 = m[0], m2 = m[1], m11 = m[2], m22 = m[3], m12 = m[4];
        const float A1 = 2.f * m1 * m2 + kC1, A2 = 2.f * (m12 - m1 * m2) + kC2;
        const float B1 = m1 * m1 + m2 * m2 + kC1;
        const float B2 = (m11 - m1 * m1) + (m22 - m2 * m2) + kC2;
        const float BB = B1 * B2, S = (A1 * A2) / BB;
        const size_t o = ch * HW + (size_t)gi * W + gj;
        pm[o] = (2.f * m2 * A2 - 2.f * m2 * A1) / BB - S * (2.f * m1 / B1 - 2.f * m1 / B2);
        pm[3 * HW + o] = -S / B2;
        pm[6 * HW + o] = 2.f * A1 / BB;
        sS += (double)S;
        const int li = kLR + r, lj = kLR + q;
        const float d = s_in[0][li * kLE + lj] - s_in[1][li * kLE + lj];
        sL1 += fabs((double)d);
        if (gj + 1 < W) {
            const float g = (s_in[0][li * kLE + lj + 1] - s_in[0][li * kLE + lj]) -
                            (s_in[1][li * kLE + lj + 1] - s_in[1][li * kLE + lj]);
            sG += fabs((double)g);
        }
        if (gi + 1 < H) {
            const float g = (s_in[0][(li + 1) * kLE + lj] - s_in[0][li * kLE + lj]) -
                            (s_in[1][(li + 1) * kLE + lj] - s_in[1][li * kLE + lj]);
            sG += fabs((double)g);
        }
    }
    sS = block_sum_d(sS, sh);
    sL1 = block_sum_d(sL1, sh);
    sG = block_sum_d(sG, sh);
    if (threadIdx.x == 0) {
        const size_t b = ((size_t)ch * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        bsum[3 * b] = sS;
        bsum[3 * b + 1] = sL1;
        bsum[3 * b + 2] = sG;
    }
}

__device__ __forceinline__ float sgn(float v) { return v > 0.f ? 1.f : (v < 0.f ? -1.f : 0.f); }

__global__ __launch_bounds__(kLThreads) void k_loss_pass2(const float* __restrict__ c,
                                                          const float* __restrict__ im, int W,
                                                          int H, Taps tp,
                                                          const float* __restrict__ pm, float lam,
                                                          float beta, float* __restrict__ dc) {
    __shared__ float s_in[3][kLE * kLE];
    __shared__ float s_h[3][kLE * kLT];
    const int ch = blockIdx.z, i0 = blockIdx.y * kLT, j0 = blockIdx.x * kLT;
    const size_t HW = (size_t)H * W;
    for (int idx = threadIdx.x; idx < kLE * kLE; idx += kLThreads) {
        const int r = idx / kLE, q = idx - r * kLE;
        const int gi = i0 - kLR + r, gj = j0 - kLR + q;
        const bool in = gi >= 0 && gi < H && gj >= 0 && gj < W;
        const size_t o = ch * HW + (size_t)(in ? gi : 0) * W + (in ? gj : 0);
#pragma unroll
        for (int m = 0; m < 3; ++m) s_in[m][idx] = in ? pm[m * 3 * HW + o] : 0.f;
    }
    __syncthreads();
    filter_rows<3>(s_in, s_h, tp);
    __syncthreads();
    const float n = (float)(3 * HW);
    const float ng = (float)(3 * ((size_t)H * (W - 1) + (size_t)(H - 1) * W));
    const float* x = c + ch * HW;
    const float* y = im + ch * HW;
    for (int idx = threadIdx.x; idx < kLT * kLT; idx += kLThreads) {
        const int r = idx / kLT, q = idx - r * kLT;
        const int gi = i0 + r, gj = j0 + q;
        if (gi >= H || gj >= W) continue;
        float f[3];
        filter_col<3>(s_h, r, q, tp, f);
        const size_t p = (size_t)gi * W + gj;
        const float xv = x[p], yv = y[p];
        // L1 term
        float g = (1.f - lam) * sgn(xv - yv) / n;
        // gradient term: this point enters the differences to its right and
        // below (with -) and from its left and above (with +)
        float dg = 0.f;
        if (gj + 1 < W) dg -= sgn((x[p + 1] - xv) - (y[p + 1] - yv));
        if (gj >= 1) dg += sgn((xv - x[p - 1]) - (yv - y[p - 1]));
        if (gi + 1 < H) dg -= sgn((x[p + W] - xv) - (y[p + W] - yv));
        if (gi >= 1) dg += sgn((xv - x[p - W]) - (yv - y[p - W]));
        g += beta * dg / ng;
        // D_SSIM = 1 - mean S
        g += lam * (-(f[0] + 2.f * xv * f[1] + yv * f[2]) / n);
        dc[ch * HW + p] = g;
    }
}

__global__ __launch_bounds__(256) void k_loss_reduce(const double* __restrict__ bsum, int nb,
                                                     double n, double ng, double lam, double beta,
                                                     double* __restrict__ out) {
    __shared__ double sh[4];
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += blockDim.x)
        for (int k = 0; k < 3; ++k) s[k] += bsum[3 * b + k];
    for (int k = 0; k < 3; ++k) s[k] = block_sum_d(s[k], sh);
    if (threadIdx.x == 0) {
        const double l1 = s[1] / n, lg = ng > 0 ? s[2] / ng : 0.0, ds = 1.0 - s[0] / n;
        out[0] = (1.0 - lam) * l1 + beta * lg + lam * ds;
        out[1] = l1;
        out[2] = lg;
        out[3] = ds;
    }
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2, float lo, float hi, int clamp) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        float x = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        if (clamp) x = fminf(fmaxf(x, lo), hi);
        p[i] = x;
    }
}

// Hard threshold T of Sec. 3.1 (Eq. 24): x if |x| >= t, else 0, in place;
// counts the values that remain non-zero.
__global__ void k_threshold(float* __restrict__ x, int64_t n, float t,
                            unsigned long long* __restrict__ nz) {
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float v = x[i];
        const float r = fabsf(v) >= t ? v : 0.f;
        x[i] = r;
        c += r != 0.f ? 1ull : 0ull;
    }
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
    if (nz && (threadIdx.x & 63) == 0 && c) atomicAdd(nz, c);
}

}  // namespace

gdgs_status launch_threshold(float* x, int64_t n, float t, unsigned long long* nz,
                             hipStream_t st) {
    if (nz) {
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, nz);
    }
    if (n > 0) {
        int64_t blocks = (n + 255) / 256;
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(k_threshold, dim3((unsigned)blocks), dim3(256), 0, st, x, n, t, nz);
    }
    GDGS_LAUNCH_CHECK();
    return GDGS_OK;
}

size_t loss_ws_bytes(int W, int H) {
    const size_t HW = (size_t)W * H;
    const size_t nb = (size_t)3 * ((W + kLT - 1) / kLT) * ((H + kLT - 1) / kLT);
    Carver c(nullptr);
    c.take<float>(9 * HW);
    c.take<double>(3 * nb);
    return c.off + 256;
}

gdgs_status launch_image_loss(const float* c, const float* im, int W, int H, double lam,
                              double beta, double* out, float* dc, void* ws, hipStream_t st) {
    const size_t HW = (size_t)W * H;
    Carver cv(ws);
    float* pm = cv.take<float>(9 * HW);
    const dim3 grid((W + kLT - 1) / kLT, (H + kLT - 1) / kLT, 3);
    double* bsum = cv.take<double>((size_t)3 * grid.x * grid.y * grid.z);
    static const Taps tp = make_taps();
    hipLaunchKernelGGL(k_loss_pass1, grid, dim3(kLThreads), 0, st, c, im, W, H, tp, pm, bsum);
    const double n = 3.0 * (double)HW;
    const double ng = 3.0 * ((double)H * (W - 1) + (double)(H - 1) * W);
    hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(256), 0, st, bsum,
                       (int)(grid.x * grid.y * grid.z), n, ng, lam, beta, out);
    if (dc)
        hipLaunchKernelGGL(k_loss_pass2, grid, dim3(kLThreads), 0, st, c, im, W, H, tp, pm,
                           (float)lam, (float)beta, dc);
    GDGS_LAUNCH_CHECK();
    return GDGS_OK;
}

gdgs_status launch_adam(float* p, const float* g, float* m, float* v, int64_t n, int t, float lr,
                        float b1, float b2, float eps, float lo, float hi, hipStream_t st) {
    if (n == 0) return GDGS_OK;
    const float c1 = (float)(1.0 - pow((double)b1, t)), c2 = (float)(1.0 - pow((double)b2, t));
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, st, p, g, m, v, n, lr, b1,
                       b2, eps, c1, c2, lo, hi, lo < hi ? 1 : 0);
    GDGS_LAUNCH_CHECK();
    return GDGS_OK;
}

}  // namespace gdgs
