// Projection of the splats to the image plane (GDGS Sec. 1.2, Eq. 10, and
// Sec. 2.2 "Projection", Eq. 19): Sigma = R S S^T R^T, Sigma2D = J W Sigma
// W^T J^T with W the world-to-camera rotation and J the Jacobian of the
// pinhole map at the splat mean.  One thread per splat, structure-of-arrays
// loads and stores (coalesced), FP64 arithmetic (the per-splat cost is tiny
// next to the memory traffic), FP32 results.  FP contraction is off so the
// rounding of every product and sum is that of the plain expression.
#include "internal.hpp"

#pragma clang fp contract(off)

namespace gdgs {
namespace {

struct CamDev {
    double fx, fy, cx, cy;
    double R[9];
    double t[3];
    int W, H;
};

// Tile rectangle and count of the support box of a splat with image mean
// (mx, my) and 2D covariance diagonal (sxx, syy); returns false if empty.
__device__ __forceinline__ bool support_rect(double mx, double my, double sxx, double syy, int W,
                                             int H, int* tx0, int* tx1, int* ty0, int* ty1) {
    const double rx = sqrt(kEcutD * sxx), ry = sqrt(kEcutD * syy);
    const double big = 4.0 * (double)(W + H) + 64.0;
    double a = mx - rx - 0.5, b = mx + rx - 0.5, c = my - ry - 0.5, d = my + ry - 0.5;
    if (!(a == a) || !(b == b) || !(c == c) || !(d == d)) return false;
    a = fmin(fmax(a, -big), big);
    b = fmin(fmax(b, -big), big);
    c = fmin(fmax(c, -big), big);
    d = fmin(fmax(d, -big), big);
    int j0 = (int)ceil(a), j1 = (int)floor(b), i0 = (int)ceil(c), i1 = (int)floor(d);
    j0 = j0 < 0 ? 0 : j0;
    i0 = i0 < 0 ? 0 : i0;
    j1 = j1 > W - 1 ? W - 1 : j1;
    i1 = i1 > H - 1 ? H - 1 : i1;
    if (j0 > j1 || i0 > i1) return false;
    *tx0 = j0 / kTile;
    *tx1 = j1 / kTile + 1;
    *ty0 = i0 / kTile;
    *ty1 = i1 / kTile + 1;
    return true;
}

__device__ __forceinline__ void write_culled(const gdgs_proj& o, int64_t K, int64_t k) {
    o.mean2d[k] = 0.f;
    o.mean2d[K + k] = 0.f;
    o.conic[k] = 0.f;
    o.conic[K + k] = 0.f;
    o.conic[2 * K + k] = 0.f;
    o.depth[k] = 0.f;
    o.rect[k] = 0u;
    o.rect[K + k] = 0u;
    o.count[k] = 0u;
}

__device__ __forceinline__ void write_splat(const gdgs_proj& o, int64_t K, int64_t k, double mx,
                                            double my, double ca, double cb, double cc,
                                            double depth, double sxx, double syy, int W, int H) {
    int tx0, tx1, ty0, ty1;
    if (!support_rect(mx, my, sxx, syy, W, H, &tx0, &tx1, &ty0, &ty1)) {
        write_culled(o, K, k);
        o.depth[k] = (float)depth;
        return;
    }
    o.mean2d[k] = (float)(mx - (double)(kTile * tx0));
    o.mean2d[K + k] = (float)(my - (double)(kTile * ty0));
    o.conic[k] = (float)ca;
    o.conic[K + k] = (float)cb;
    o.conic[2 * K + k] = (float)cc;
    o.depth[k] = (float)depth;
    o.rect[k] = (uint32_t)tx0 | ((uint32_t)tx1 << 16);
    o.rect[K + k] = (uint32_t)ty0 | ((uint32_t)ty1 << 16);
    o.count[k] = (uint32_t)((tx1 - tx0) * (ty1 - ty0));
}

__global__ __launch_bounds__(256) void k_project(const float* __restrict__ mean,
                                                 const float* __restrict__ log_scale,
                                                 const float* __restrict__ quat, int64_t K,
                                                 CamDev cam, gdgs_proj out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const double px = mean[k], py = mean[K + k], pz = mean[2 * K + k];
    double qw = quat[k], qx = quat[K + k], qy = quat[2 * K + k], qz = quat[3 * K + k];
    const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    // camera-space mean
    const double* R = cam.R;
    const double xc = R[0] * px + R[1] * py + R[2] * pz + cam.t[0];
    const double yc = R[3] * px + R[4] * py + R[5] * pz + cam.t[1];
    const double zc = R[6] * px + R[7] * py + R[8] * pz + cam.t[2];
    if (!(qn > 0.0) || !(zc > kZnear)) {
        write_culled(out, K, k);
        out.depth[k] = (float)zc;
        return;
    }
    qw /= qn;
    qx /= qn;
    qy /= qn;
    qz /= qn;
    // rotation of the splat (unit quaternion (w, x, y, z))
    const double r00 = 1 - 2 * (qy * qy + qz * qz), r01 = 2 * (qx * qy - qw * qz),
                 r02 = 2 * (qx * qz + qw * qy);
    const double r10 = 2 * (qx * qy + qw * qz), r11 = 1 - 2 * (qx * qx + qz * qz),
                 r12 = 2 * (qy * qz - qw * qx);
    const double r20 = 2 * (qx * qz - qw * qy), r21 = 2 * (qy * qz + qw * qx),
                 r22 = 1 - 2 * (qx * qx + qy * qy);
    const double s0 = exp(2.0 * (double)log_scale[k]);
    const double s1 = exp(2.0 * (double)log_scale[K + k]);
    const double s2 = exp(2.0 * (double)log_scale[2 * K + k]);
    // Sigma = Rs diag(s) Rs^T (symmetric)
    const double S00 = r00 * r00 * s0 + r01 * r01 * s1 + r02 * r02 * s2;
    const double S01 = r00 * r10 * s0 + r01 * r11 * s1 + r02 * r12 * s2;
    const double S02 = r00 * r20 * s0 + r01 * r21 * s1 + r02 * r22 * s2;
    const double S11 = r10 * r10 * s0 + r11 * r11 * s1 + r12 * r12 * s2;
    const double S12 = r10 * r20 * s0 + r11 * r21 * s1 + r12 * r22 * s2;
    const double S22 = r20 * r20 * s0 + r21 * r21 * s1 + r22 * r22 * s2;
    // T = J W (2x3); J = [[fx/z, 0, -fx x/z^2], [0, fy/z, -fy y/z^2]]
    const double iz = 1.0 / zc;
    const double j00 = cam.fx * iz, j02 = -cam.fx * xc * iz * iz;
    const double j11 = cam.fy * iz, j12 = -cam.fy * yc * iz * iz;
    const double t00 = j00 * R[0] + j02 * R[6], t01 = j00 * R[1] + j02 * R[7],
                 t02 = j00 * R[2] + j02 * R[8];
    const double t10 = j11 * R[3] + j12 * R[6], t11 = j11 * R[4] + j12 * R[7],
                 t12 = j11 * R[5] + j12 * R[8];
    // M = T Sigma, cov = M T^T
    const double m00 = t00 * S00 + t01 * S01 + t02 * S02;
    const double m01 = t00 * S01 + t01 * S11 + t02 * S12;
    const double m02 = t00 * S02 + t01 * S12 + t02 * S22;
    const double m10 = t10 * S00 + t11 * S01 + t12 * S02;
    const double m11 = t10 * S01 + t11 * S11 + t12 * S12;
    const double m12 = t10 * S02 + t11 * S12 + t12 * S22;
    const double sxx = m00 * t00 + m01 * t01 + m02 * t02;
    const double sxy = m00 * t10 + m01 * t11 + m02 * t12;
    const double syy = m10 * t10 + m11 * t11 + m12 * t12;
    const double det = sxx * syy - sxy * sxy;
    if (!(det > 0.0)) {
        write_culled(out, K, k);
        out.depth[k] = (float)zc;
        return;
    }
    const double mx = cam.fx * xc / zc + cam.cx;
    const double my = cam.fy * yc / zc + cam.cy;
    write_splat(out, K, k, mx, my, syy / det, -sxy / det, sxx / det, zc, sxx, syy, cam.W, cam.H);
}

__global__ __launch_bounds__(256) void k_project_2d(const float* __restrict__ mean2d,
                                                    const float* __restrict__ conic,
                                                    const float* __restrict__ depth, int64_t K,
                                                    int W, int H, gdgs_proj out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const double a = conic[k], b = conic[K + k], c = conic[2 * K + k];
    const double det = a * c - b * b;
    if (!(det > 0.0)) {
        write_culled(out, K, k);
        out.depth[k] = depth[k];
        return;
    }
    int tx0, tx1, ty0, ty1;
    const double mx = mean2d[k], my = mean2d[K + k];
    if (!support_rect(mx, my, c / det, a / det, W, H, &tx0, &tx1, &ty0, &ty1)) {
        write_culled(out, K, k);
        out.depth[k] = depth[k];
        return;
    }
    out.mean2d[k] = (float)(mx - (double)(kTile * tx0));
    out.mean2d[K + k] = (float)(my - (double)(kTile * ty0));
    out.conic[k] = conic[k];
    out.conic[K + k] = conic[K + k];
    out.conic[2 * K + k] = conic[2 * K + k];
    out.depth[k] = depth[k];
    out.rect[k] = (uint32_t)tx0 | ((uint32_t)tx1 << 16);
    out.rect[K + k] = (uint32_t)ty0 | ((uint32_t)ty1 << 16);
    out.count[k] = (uint32_t)((tx1 - tx0) * (ty1 - ty0));
}

// Reverse mode of k_project: gradients of a loss with respect to the world
// mean, log-scales and quaternion from its gradients with respect to the
// image-plane mean and the conic (a, b, c) (E = a dx^2 + 2 b dx dy + c dy^2).
// The chain rule is applied backwards through the forward steps: conic ->
// Sigma2D (G_S2 = -A G_A A, G_A the symmetric-matrix form of (ga, gb, gc)),
// Sigma2D = T Sigma T^T (G_T = 2 G_S2 T Sigma, G_Sigma = T^T G_S2 T), T = J W,
// the pinhole map and its Jacobian at the camera-space mean, Sigma = M M^T
// with M = R S, the rotation-matrix formula and the quaternion normalisation.
// Culled splats get zero gradients.  FP64, one thread per splat.
__global__ __launch_bounds__(256) void k_project_backward(
    const float* __restrict__ mean, const float* __restrict__ log_scale,
    const float* __restrict__ quat, int64_t K, CamDev cam, const float* __restrict__ dmean2d,
    const float* __restrict__ dconic, float* __restrict__ gmean, float* __restrict__ glog,
    float* __restrict__ gquat) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    auto zero = [&]() {
        for (int i = 0; i < 3; ++i) gmean[i * K + k] = 0.f;
        for (int i = 0; i < 3; ++i) glog[i * K + k] = 0.f;
        for (int i = 0; i < 4; ++i) gquat[i * K + k] = 0.f;
    };
    const double p[3] = {mean[k], mean[K + k], mean[2 * K + k]};
    const double q0[4] = {quat[k], quat[K + k], quat[2 * K + k], quat[3 * K + k]};
    const double qn = sqrt(q0[0] * q0[0] + q0[1] * q0[1] + q0[2] * q0[2] + q0[3] * q0[3]);
    const double* W = cam.R;
    double xc[3];
    for (int i = 0; i < 3; ++i)
        xc[i] = W[3 * i] * p[0] + W[3 * i + 1] * p[1] + W[3 * i + 2] * p[2] + cam.t[i];
    if (!(qn > 0.0) || !(xc[2] > kZnear)) {
        zero();
        return;
    }
    const double w = q0[0] / qn, x = q0[1] / qn, y = q0[2] / qn, z = q0[3] / qn;
    const double R[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                            {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                            {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
    const double sc[3] = {exp((double)log_scale[k]), exp((double)log_scale[K + k]),
                          exp((double)log_scale[2 * K + k])};
    double M[3][3], Sg[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[i][j] = R[i][j] * sc[j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            Sg[i][j] = M[i][0] * M[j][0] + M[i][1] * M[j][1] + M[i][2] * M[j][2];
    const double X = xc[0], Y = xc[1], Z = xc[2], iz = 1.0 / Z;
    const double J[2][3] = {{cam.fx * iz, 0.0, -cam.fx * X * iz * iz},
                            {0.0, cam.fy * iz, -cam.fy * Y * iz * iz}};
    double T[2][3], TS[2][3], S2[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j)
            T[i][j] = J[i][0] * W[j] + J[i][1] * W[3 + j] + J[i][2] * W[6 + j];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j)
            TS[i][j] = T[i][0] * Sg[0][j] + T[i][1] * Sg[1][j] + T[i][2] * Sg[2][j];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            S2[i][j] = TS[i][0] * T[j][0] + TS[i][1] * T[j][1] + TS[i][2] * T[j][2];
    const double det = S2[0][0] * S2[1][1] - S2[0][1] * S2[1][0];
    if (!(det > 0.0)) {
        zero();
        return;
    }
    const double A[2][2] = {{S2[1][1] / det, -S2[0][1] / det}, {-S2[1][0] / det, S2[0][0] / det}};
    const double ga = dconic[k], gb = dconic[K + k], gc = dconic[2 * K + k];
    const double GA[2][2] = {{ga, 0.5 * gb}, {0.5 * gb, gc}};
    double AG[2][2], GS2[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) AG[i][j] = A[i][0] * GA[0][j] + A[i][1] * GA[1][j];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) GS2[i][j] = -(AG[i][0] * A[0][j] + AG[i][1] * A[1][j]);
    // G_T = 2 G_S2 (T Sigma); G_Sigma = T^T G_S2 T
    double GT[2][3], GSg[3][3], GTt[2][3];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) GT[i][j] = 2.0 * (GS2[i][0] * TS[0][j] + GS2[i][1] * TS[1][j]);
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) GTt[i][j] = GS2[i][0] * T[0][j] + GS2[i][1] * T[1][j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) GSg[i][j] = T[0][i] * GTt[0][j] + T[1][i] * GTt[1][j];
    // G_J = G_T W^T
    double GJ[2][3];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j)
            GJ[i][j] = GT[i][0] * W[3 * j] + GT[i][1] * W[3 * j + 1] + GT[i][2] * W[3 * j + 2];
    const double gmx = dmean2d[k], gmy = dmean2d[K + k];
    const double fx = cam.fx, fy = cam.fy, iz2 = iz * iz, iz3 = iz2 * iz;
    const double gX = GJ[0][2] * (-fx * iz2) + gmx * (fx * iz);
    const double gY = GJ[1][2] * (-fy * iz2) + gmy * (fy * iz);
    const double gZ = GJ[0][0] * (-fx * iz2) + GJ[0][2] * (2.0 * fx * X * iz3) +
                      GJ[1][1] * (-fy * iz2) + GJ[1][2] * (2.0 * fy * Y * iz3) +
                      gmx * (-fx * X * iz2) + gmy * (-fy * Y * iz2);
    for (int i = 0; i < 3; ++i)
        gmean[i * K + k] = (float)(W[i] * gX + W[3 + i] * gY + W[6 + i] * gZ);
    // Sigma = M M^T: G_M = 2 G_Sigma M; M = R S: G_R = G_M S, G_s = diag(R^T G_M)
    double GM[3][3], GR[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            GM[i][j] = 2.0 * (GSg[i][0] * M[0][j] + GSg[i][1] * M[1][j] + GSg[i][2] * M[2][j]);
    for (int j = 0; j < 3; ++j) {
        double gs = 0.0;
        for (int i = 0; i < 3; ++i) {
            GR[i][j] = GM[i][j] * sc[j];
            gs += R[i][j] * GM[i][j];
        }
        glog[j * K + k] = (float)(gs * sc[j]);
    }
    // rotation-matrix formula -> unit quaternion -> raw quaternion
    const double gw = 2 * (-z * GR[0][1] + y * GR[0][2] + z * GR[1][0] - x * GR[1][2] -
                           y * GR[2][0] + x * GR[2][1]);
    const double gx = 2 * (y * GR[0][1] + z * GR[0][2] + y * GR[1][0] - 2 * x * GR[1][1] -
                           w * GR[1][2] + z * GR[2][0] + w * GR[2][1] - 2 * x * GR[2][2]);
    const double gy = 2 * (-2 * y * GR[0][0] + x * GR[0][1] + w * GR[0][2] + x * GR[1][0] +
                           z * GR[1][2] - w * GR[2][0] + z * GR[2][1] - 2 * y * GR[2][2]);
    const double gz = 2 * (-2 * z * GR[0][0] - w * GR[0][1] + x * GR[0][2] + w * GR[1][0] -
                           2 * z * GR[1][1] + y * GR[1][2] + x * GR[2][0] + y * GR[2][1]);
    const double dotq = w * gw + x * gx + y * gy + z * gz;
    gquat[k] = (float)((gw - w * dotq) / qn);
    gquat[K + k] = (float)((gx - x * dotq) / qn);
    gquat[2 * K + k] = (float)((gy - y * dotq) / qn);
    gquat[3 * K + k] = (float)((gz - z * dotq) / qn);
}

}  // namespace

gdgs_status launch_project(const gdgs_scene& s, const gdgs_camera& cam, const gdgs_proj& out,
                           hipStream_t st) {
    if (s.K == 0) return GDGS_OK;
    CamDev c;
    c.fx = cam.fx;
    c.fy = cam.fy;
    c.cx = cam.cx;
    c.cy = cam.cy;
    for (int i = 0; i < 9; ++i) c.R[i] = cam.R[i];
    for (int i = 0; i < 3; ++i) c.t[i] = cam.t[i];
    c.W = cam.W;
    c.H = cam.H;
    hipLaunchKernelGGL(k_project, dim3((unsigned)((s.K + 255) / 256)), dim3(256), 0, st, s.mean,
                       s.log_scale, s.quat, s.K, c, out);
    GDGS_LAUNCH_CHECK();
    return GDGS_OK;
}

gdgs_status launch_project_backward(const gdgs_scene& s, const gdgs_camera& cam,
                                    const float* dmean2d, const float* dconic, float* gmean,
                                    float* glog, float* gquat, hipStream_t st) {
    if (s.K == 0) return GDGS_OK;
    CamDev c;
    c.fx = cam.fx;
    c.fy = cam.fy;
    c.cx = cam.cx;
    c.cy = cam.cy;
    for (int i = 0; i < 9; ++i) c.R[i] = cam.R[i];
    for (int i = 0; i < 3; ++i) c.t[i] = cam.t[i];
    c.W = cam.W;
    c.H = cam.H;
    hipLaunchKernelGGL(k_project_backward, dim3((unsigned)((s.K + 255) / 256)), dim3(256), 0, st,
                       s.mean, s.log_scale, s.quat, s.K, c, dmean2d, dconic, gmean, glog, gquat);
    GDGS_LAUNCH_CHECK();
    return GDGS_OK;
}

gdgs_status launch_project_2d(const float* mean2d, const float* conic, const float* depth,
                              int64_t K, int W, int H, const gdgs_proj& out, hipStream_t st) {
    if (K == 0) return GDGS_OK;
    hipLaunchKernelGGL(k_project_2d, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, st, mean2d,
                       conic, depth, K, W, H, out);
    GDGS_LAUNCH_CHECK();
    return GDGS_OK;
}

}  // namespace gdgs
