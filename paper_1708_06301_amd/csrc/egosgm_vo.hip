// Ego-motion front end: direct stereo visual odometry on gfx950.
//
// The motion T = (R, t) between consecutive frames (M_k = R M_{k-1} + t, the
// motion the warp of Sec. 2.2 consumes) is estimated by aligning the previous
// left image to the current one through the previous disparity map: every
// pixel with a disparity is lifted to 3-D (Z = f b / d, Eq. 1), moved,
// projected and compared with the current image, and Gauss-Newton minimises
// the Huber-weighted photometric error, coarse to fine over an image pyramid
// with a fixed number of iterations per level.  The update is
// left-multiplicative, T <- exp(xi) T, xi = (rho, phi).  (The paper takes the
// motion from a feature-based odometry it cites; this front end is the
// library's own.)
//
// The pyramid is one kernel per level (images, disparities and gradients).
// Per iteration of a large level: one kernel evaluates every pixel's
// residual and Jacobian and reduces the normal equations (21 + 6 + cost +
// count terms) per block in float32; one single-block kernel sums the block
// partials in double in a fixed order, solves the 6x6 system by Cholesky and
// updates the pose.  A small level (at most 8 Ki pixels) runs all its
// iterations in one block, the pose in LDS between them.  The pose stays in
// device memory (12 doubles) from the first level to the last, so a whole
// estimate is a fixed sequence of launches with no host round trip.
#include "egosgm_internal.h"

#include <math.h>

namespace egosgm {
namespace {

constexpr int kVoBlock = 256;
constexpr int kVoPix = 4;       // pixels per thread in the normal-equation pass
constexpr int kVoTerms = 29;    // 21 (upper triangle of H) + 6 (g) + cost + count
constexpr int kVoSmallLevel = 1 << 13;   // levels of at most this many pixels run in one block

// Level 0: both images as float, and the central differences of the
// current one, (I(x+1) - I(x-1)) * 0.5, zero on the border.
__global__ __launch_bounds__(kVoBlock) void vo_level0_kernel(const uint8_t* prev, const uint8_t* cur, int w, int h,
                                                              int pitch, float* ref0, float* cur0, float* gx,
                                                              float* gy) {
    const int i = (int)(blockIdx.x * kVoBlock + threadIdx.x);
    if (i >= w * h) return;
    const int y = i / w, x = i - y * w;
    const uint8_t* c = cur + (size_t)y * pitch + x;
    ref0[i] = (float)prev[(size_t)y * pitch + x];
    cur0[i] = (float)c[0];
    gx[i] = (x > 0 && x < w - 1) ? ((float)c[1] - (float)c[-1]) * 0.5f : 0.0f;
    gy[i] = (y > 0 && y < h - 1) ? ((float)c[pitch] - (float)c[-pitch]) * 0.5f : 0.0f;
}

// Level l from level l-1 (sizes w x h of level l): images by the 2x2 mean
// ((a + b) + (c + d)) * 0.25, disparities by the sample at (2x, 2y), halved,
// and the central differences of the current image, zero on the border (its
// neighbours' means are recomputed the same way, so they equal the stored ones).
__global__ __launch_bounds__(kVoBlock) void vo_down_kernel(const float* ref_in, const float* cur_in, const float* d_in,
                                                            int w_in, float* ref, float* cur, float* d, float* gx,
                                                            float* gy, int w, int h) {
    const int i = (int)(blockIdx.x * kVoBlock + threadIdx.x);
    if (i >= w * h) return;
    const int y = i / w, x = i - y * w;
    auto mean = [&](const float* I, int xx, int yy) {
        const size_t a = (size_t)(2 * yy) * w_in + 2 * xx, c = a + w_in;
        return ((I[a] + I[a + 1]) + (I[c] + I[c + 1])) * 0.25f;
    };
    ref[i] = mean(ref_in, x, y);
    cur[i] = mean(cur_in, x, y);
    const float s = d_in[(size_t)(2 * y) * w_in + 2 * x];
    d[i] = s > 0.0f ? s * 0.5f : -1.0f;
    gx[i] = (x > 0 && x < w - 1) ? (mean(cur_in, x + 1, y) - mean(cur_in, x - 1, y)) * 0.5f : 0.0f;
    gy[i] = (y > 0 && y < h - 1) ? (mean(cur_in, x, y + 1) - mean(cur_in, x, y - 1)) * 0.5f : 0.0f;
}

struct VoLevel {
    const float *ref, *cur, *gx, *gy, *disp;
    int w, h;
    float f, cx, cy, fb;   // f_l, principal point, f_l * b
    float min_disp;        // at this level
    float huber;
};

__device__ inline float bilinear(const float* I, int w, int x0, int y0, float fx, float fy) {
    const float* r0 = I + (size_t)y0 * w + x0;
    const float* r1 = r0 + w;
    return (1.0f - fy) * ((1.0f - fx) * r0[0] + fx * r0[1]) + fy * ((1.0f - fx) * r1[0] + fx * r1[1]);
}

// Adds pixel i's terms (upper triangle of w J^T J, w J r, w r^2, 1) to acc
// when it enters the sum at the motion (R, t).
__device__ inline void add_pixel(const VoLevel& L, const float (&R)[9], const float (&t)[3], int i,
                                 float (&acc)[kVoTerms]) {
    const float d = L.disp[i];
    if (!(d >= L.min_disp)) return;
    const int y = i / L.w, x = i - y * L.w;
    // the lift, the motion and the projection in float32, in this order
    const float Z = L.fb / d;
    const float X = (((float)x - L.cx) * Z) / L.f;
    const float Y = (((float)y - L.cy) * Z) / L.f;
    const float Xp = ((R[0] * X + R[1] * Y) + R[2] * Z) + t[0];
    const float Yp = ((R[3] * X + R[4] * Y) + R[5] * Z) + t[1];
    const float Zp = ((R[6] * X + R[7] * Y) + R[8] * Z) + t[2];
    if (!(Zp > 0.0f)) return;
    const float up = (L.f * Xp) / Zp + L.cx;
    const float vp = (L.f * Yp) / Zp + L.cy;
    if (!(up >= 1.0f && up < (float)(L.w - 2) && vp >= 1.0f && vp < (float)(L.h - 2))) return;
    const float x0f = floorf(up), y0f = floorf(vp);
    const int x0 = (int)x0f, y0 = (int)y0f;
    const float fx = up - x0f, fy = vp - y0f;
    const float r = bilinear(L.cur, L.w, x0, y0, fx, fy) - L.ref[i];
    const float gx = bilinear(L.gx, L.w, x0, y0, fx, fy);
    const float gy = bilinear(L.gy, L.w, x0, y0, fx, fy);
    const float ju = gx * L.f / Zp, jv = gy * L.f / Zp;
    const float jz = -(gx * L.f * Xp + gy * L.f * Yp) / (Zp * Zp);
    const float J[6] = {ju, jv, jz, Yp * jz - Zp * jv, Zp * ju - Xp * jz, Xp * jv - Yp * ju};
    const float a = fabsf(r);
    const float wgt = a <= L.huber ? 1.0f : L.huber / a;
    int q = 0;
#pragma unroll
    for (int u = 0; u < 6; ++u) {
        const float wj = wgt * J[u];
#pragma unroll
        for (int v = u; v < 6; ++v) acc[q++] += wj * J[v];
    }
#pragma unroll
    for (int u = 0; u < 6; ++u) acc[21 + u] += wgt * J[u] * r;
    acc[27] += wgt * r * r;
    acc[28] += 1.0f;
}

// Normal equations of one level at the pose in `pose` (12 doubles, device):
// every thread takes kVoPix pixels (strided by the grid), the block sums its
// threads' terms in LDS and writes kVoTerms floats to part[block].
__global__ __launch_bounds__(kVoBlock) void vo_normal_kernel(VoLevel L, const double* pose, float* part) {
    __shared__ float red[kVoTerms][kVoBlock];
    float R[9], t[3];
#pragma unroll
    for (int k = 0; k < 9; ++k) R[k] = (float)pose[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) t[k] = (float)pose[9 + k];
    float acc[kVoTerms];
#pragma unroll
    for (int k = 0; k < kVoTerms; ++k) acc[k] = 0.0f;
    const int n = L.w * L.h;
    const int stride = (int)(gridDim.x * kVoBlock);
    for (int k = 0, i = (int)(blockIdx.x * kVoBlock + threadIdx.x); k < kVoPix && i < n; ++k, i += stride)
        add_pixel(L, R, t, i, acc);
#pragma unroll
    for (int k = 0; k < kVoTerms; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = kVoBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int k = 0; k < kVoTerms; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        }
        __syncthreads();
    }
    if ((int)threadIdx.x < kVoTerms) part[(size_t)blockIdx.x * kVoTerms + threadIdx.x] = red[threadIdx.x][0];
}

// SE(3) exponential of xi = (rho, phi) in double: Rodrigues for the rotation,
// V(phi) rho for the translation.
__device__ inline void se3_exp(const double xi[6], double Rd[9], double td[3]) {
    const double p0 = xi[3], p1 = xi[4], p2 = xi[5];
    const double a2 = p0 * p0 + p1 * p1 + p2 * p2, a = sqrt(a2);
    double A, B, C;
    if (a < 1e-8) {
        A = 1.0 - a2 / 6.0;
        B = 0.5 - a2 / 24.0;
        C = 1.0 / 6.0 - a2 / 120.0;
    } else {
        A = sin(a) / a;
        B = (1.0 - cos(a)) / a2;
        C = (a - sin(a)) / (a2 * a);
    }
    const double K[9] = {0.0, -p2, p1, p2, 0.0, -p0, -p1, p0, 0.0};
    double K2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            K2[3 * i + j] = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
    double V[9];
    for (int k = 0; k < 9; ++k) {
        const double I = (k % 4 == 0) ? 1.0 : 0.0;
        Rd[k] = I + A * K[k] + B * K2[k];
        V[k] = I + B * K[k] + C * K2[k];
    }
    for (int i = 0; i < 3; ++i) td[i] = V[3 * i] * xi[0] + V[3 * i + 1] * xi[1] + V[3 * i + 2] * xi[2];
}

// From the summed terms: either writes H (36), g (6), cost, count to `out`,
// or takes the Gauss-Newton step xi = -(H + lambda I)^-1 g, lambda =
// 1e-9 trace(H) / 6 (none below 16 pixels, or when H + lambda I is not
// positive definite), and sets pose <- exp(xi) pose.  One thread.
__device__ inline void finish_level_step(const double (&sum)[kVoTerms], double* pose, double* out) {
    double H[36], g[6];
    int q = 0;
    for (int u = 0; u < 6; ++u)
        for (int v = u; v < 6; ++v) {
            H[6 * u + v] = sum[q];
            H[6 * v + u] = sum[q];
            ++q;
        }
    for (int u = 0; u < 6; ++u) g[u] = sum[21 + u];
    const double cost = sum[27], count = sum[28];
    if (out != nullptr) {
        for (int k = 0; k < 36; ++k) out[k] = H[k];
        for (int k = 0; k < 6; ++k) out[36 + k] = g[k];
        out[42] = cost;
        out[43] = count;
        return;
    }
    if (count < 16.0) return;
    const double lam = 1e-9 * (H[0] + H[7] + H[14] + H[21] + H[28] + H[35]) / 6.0;
    for (int u = 0; u < 6; ++u) H[7 * u] += lam;
    // Cholesky H = L L^T (lower triangle in place), then L L^T xi = -g; one
    // division per column (inv[j] = 1 / L_jj), products elsewhere
    double inv[6];
    for (int j = 0; j < 6; ++j) {
        double s = H[6 * j + j];
        for (int k = 0; k < j; ++k) s -= H[6 * j + k] * H[6 * j + k];
        if (!(s > 0.0)) return;
        const double ljj = sqrt(s);
        H[6 * j + j] = ljj;
        inv[j] = 1.0 / ljj;
        for (int i = j + 1; i < 6; ++i) {
            double v = H[6 * i + j];
            for (int k = 0; k < j; ++k) v -= H[6 * i + k] * H[6 * j + k];
            H[6 * i + j] = v * inv[j];
        }
    }
    double z[6], xi[6];
    for (int i = 0; i < 6; ++i) {
        double v = -g[i];
        for (int k = 0; k < i; ++k) v -= H[6 * i + k] * z[k];
        z[i] = v * inv[i];
    }
    for (int i = 5; i >= 0; --i) {
        double v = z[i];
        for (int k = i + 1; k < 6; ++k) v -= H[6 * k + i] * xi[k];
        xi[i] = v * inv[i];
    }
    double Rd[9], td[3];
    se3_exp(xi, Rd, td);
    double R[9], t[3];
    for (int k = 0; k < 9; ++k) R[k] = pose[k];
    for (int k = 0; k < 3; ++k) t[k] = pose[9 + k];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            pose[3 * i + j] = Rd[3 * i] * R[j] + Rd[3 * i + 1] * R[3 + j] + Rd[3 * i + 2] * R[6 + j];
        pose[9 + i] = Rd[3 * i] * t[0] + Rd[3 * i + 1] * t[1] + Rd[3 * i + 2] * t[2] + td[i];
    }
}

// Sums the block partials of vo_normal_kernel in double (thread j takes
// blocks j, j + 256, ..., then a fixed tree) and finishes the step.
__global__ __launch_bounds__(kVoBlock) void vo_solve_kernel(const float* part, int n_blocks, double* pose, double* out) {
    __shared__ double red[kVoTerms][kVoBlock];
    double acc[kVoTerms];
    for (int k = 0; k < kVoTerms; ++k) acc[k] = 0.0;
    for (int b = (int)threadIdx.x; b < n_blocks; b += kVoBlock)
        for (int k = 0; k < kVoTerms; ++k) acc[k] += (double)part[(size_t)b * kVoTerms + k];
    for (int k = 0; k < kVoTerms; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = kVoBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < kVoTerms; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    double sum[kVoTerms];
    for (int k = 0; k < kVoTerms; ++k) sum[k] = red[k][0];
    finish_level_step(sum, pose, out);
}

// Every iteration of one small level in one block of kVoSmallBlock threads:
// the pose lives in LDS between iterations; per iteration each thread sums
// its pixels (stride kVoSmallBlock) in float32, each wave folds its lanes by
// an xor butterfly, and thread 0 adds the waves in double and takes the step.
constexpr int kVoSmallBlock = 1024;
__global__ __launch_bounds__(kVoSmallBlock) void vo_small_level_kernel(VoLevel L, int iters, double* pose, double* out) {
    __shared__ float wsum[kVoSmallBlock / 64][kVoTerms];
    __shared__ double pose_s[12];
    __shared__ double dsum[kVoTerms];
    const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid < 12) pose_s[tid] = pose[tid];
    __syncthreads();
    const int n = L.w * L.h;
    for (int it = 0; it < iters; ++it) {
        float R[9], t[3];
#pragma unroll
        for (int k = 0; k < 9; ++k) R[k] = (float)pose_s[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) t[k] = (float)pose_s[9 + k];
        float acc[kVoTerms];
#pragma unroll
        for (int k = 0; k < kVoTerms; ++k) acc[k] = 0.0f;
        for (int i = tid; i < n; i += kVoSmallBlock) add_pixel(L, R, t, i, acc);
#pragma unroll
        for (int k = 0; k < kVoTerms; ++k) {
            float v = acc[k];
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
            acc[k] = v;
        }
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < kVoTerms; ++k) wsum[wave][k] = acc[k];
        }
        __syncthreads();
        if (tid < kVoTerms) {   // one term per thread, the waves in order
            double v = 0.0;
            for (int w = 0; w < kVoSmallBlock / 64; ++w) v += (double)wsum[w][tid];
            dsum[tid] = v;
        }
        __syncthreads();
        if (tid == 0) {
            double sum[kVoTerms];
            for (int k = 0; k < kVoTerms; ++k) sum[k] = dsum[k];
            finish_level_step(sum, pose_s, out);
        }
        __syncthreads();
    }
    if (out == nullptr && tid < 12) pose[tid] = pose_s[tid];   // `out`: the pose is read only
}

unsigned vo_grid(int n) { return (unsigned)((n + kVoBlock - 1) / kVoBlock); }

}  // namespace

int vo_level_w(int w, int l) { return w >> l; }
int vo_level_h(int h, int l) { return h >> l; }

size_t vo_partial_blocks(int w, int h) {
    return (size_t)((w * h + kVoBlock * kVoPix - 1) / (kVoBlock * kVoPix));
}

// Workspace: for every level, five float images (reference, current,
// gradient x, gradient y, disparity; the level-0 disparity is the caller's),
// then the block partials of the largest level.
size_t vo_workspace_bytes(int w, int h, int levels) {
    size_t n = 0;
    for (int l = 0; l < levels; ++l) n += (size_t)vo_level_w(w, l) * vo_level_h(h, l) * 5;
    n += vo_partial_blocks(w, h) * kVoTerms;
    return ((n * sizeof(float)) + 255) & ~(size_t)255;
}

hipError_t launch_vo(const VoArgs& v, hipStream_t s) {
    float* base = reinterpret_cast<float*>(v.workspace);
    const float* ref[kVoMaxLevels];
    const float* cur[kVoMaxLevels];
    const float* gx[kVoMaxLevels];
    const float* gy[kVoMaxLevels];
    const float* dsp[kVoMaxLevels];
    float* mref[kVoMaxLevels];
    float* mcur[kVoMaxLevels];
    float* mgx[kVoMaxLevels];
    float* mgy[kVoMaxLevels];
    float* mdsp[kVoMaxLevels];
    float* p = base;
    for (int l = 0; l < v.levels; ++l) {
        const size_t n = (size_t)vo_level_w(v.w, l) * vo_level_h(v.h, l);
        mref[l] = p; p += n;
        mcur[l] = p; p += n;
        mgx[l] = p; p += n;
        mgy[l] = p; p += n;
        mdsp[l] = p; p += n;
        ref[l] = mref[l]; cur[l] = mcur[l]; gx[l] = mgx[l]; gy[l] = mgy[l];
        dsp[l] = l == 0 ? v.prev_disp : mdsp[l];
    }
    float* part = p;
    // pyramids
    vo_level0_kernel<<<vo_grid(v.w * v.h), kVoBlock, 0, s>>>(v.prev, v.cur, v.w, v.h, v.pitch, mref[0], mcur[0],
                                                            mgx[0], mgy[0]);
    for (int l = 1; l < v.levels; ++l) {
        const int wl = vo_level_w(v.w, l), hl = vo_level_h(v.h, l);
        vo_down_kernel<<<vo_grid(wl * hl), kVoBlock, 0, s>>>(ref[l - 1], cur[l - 1], dsp[l - 1], vo_level_w(v.w, l - 1),
                                                              mref[l], mcur[l], mdsp[l], mgx[l], mgy[l], wl, hl);
    }
    // levels coarse to fine (or the one level asked for)
    for (int l = v.levels - 1; l >= 0; --l) {
        if (v.only_level >= 0 && l != v.only_level) continue;
        const int wl = vo_level_w(v.w, l), hl = vo_level_h(v.h, l);
        const double sc = (double)(1 << l);
        VoLevel L{ref[l], cur[l], gx[l], gy[l], dsp[l], wl, hl,
                  (float)(v.f / sc), (float)((v.cx + 0.5) / sc - 0.5), (float)((v.cy + 0.5) / sc - 0.5),
                  (float)(v.f / sc * v.baseline), (float)(v.min_disp / sc), v.huber};
        const int nb = (int)vo_partial_blocks(wl, hl);
        const int iters = v.only_level >= 0 ? 1 : v.iters[l];
        double* out = v.only_level >= 0 ? v.out : nullptr;
        if (iters == 0) continue;
        if (wl * hl <= kVoSmallLevel) {
            // a small level: all its iterations in one block, one launch
            vo_small_level_kernel<<<1, kVoSmallBlock, 0, s>>>(L, iters, v.pose, out);
            continue;
        }
        for (int it = 0; it < iters; ++it) {
            vo_normal_kernel<<<(unsigned)nb, kVoBlock, 0, s>>>(L, v.pose, part);
            vo_solve_kernel<<<1, kVoBlock, 0, s>>>(part, nb, v.pose, out);
        }
    }
    return hipGetLastError();
}

}  // namespace egosgm
