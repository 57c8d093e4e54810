/*
 * egosgm_oracle.c — plain CPU oracle (see egosgm_oracle.h).
 *
 * TEST INFRASTRUCTURE ONLY: read by tests, the smoke check and the CPU
 * baseline of the benchmark; never by the product path.
 *
 * Every function follows a statement of the method written out plainly:
 *  - the 8-path semi-global matching recurrence is the textbook one of
 *    Hirschmüller (2008), which the paper cites for its matcher (Sec. 1 and
 *    Sec. 2.3, with eight paths);
 *  - the reduced search interval is [d_pred +- 3 sqrt(p_pred)] (Sec. 2.3);
 *  - the matching uncertainty counts neighbouring disparities while the
 *    running cost sum stays below S_max, r = n_l + n_r (Sec. 2.3.1, Eq. 9);
 *  - the disparity-space transform is H = Gamma T Gamma^-1 with the
 *    prediction normalised by its fourth component (Sec. 2.1, Eq. 1-4;
 *    Sec. 2.2), variance predicted as Phi^2 p + q with Phi = d'/d
 *    (Eq. 5-6), collisions keep the largest predicted disparity (Sec. 2.2.2);
 *  - the update is the scalar Kalman filter of Eq. 10-12 (Sec. 2.4).
 * Where the paper is silent the reading taken is stated at the function.
 *
 * Compiled with -O2 -ffp-contract=off -fno-fast-math so that every float32
 * expression is evaluated exactly in the order written.
 */
#include "egosgm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_CW 9           /* census window width  */
#define ORC_CH 7           /* census window height */
#define ORC_CBITS 62       /* ORC_CW*ORC_CH - 1     */
#define ORC_INF 0x3fffffff

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
static int mini(int a, int b) { return a < b ? a : b; }
static int maxi(int a, int b) { return a > b ? a : b; }

/* Number of set bits, counted one bit at a time. */
static int bitcount64(uint64_t v) {
    int n = 0;
    for (int i = 0; i < 64; ++i) n += (int)((v >> i) & 1u);
    return n;
}

/* Census (the paper only names a 3x3 matching window; the matching cost used
 * here is a 9x7 census with Hamming distance).  Offsets are visited row by row,
 * dy = -3..3 outer, dx = -4..4 inner, the centre skipped; the k-th visited
 * offset sets bit k when that neighbour (coordinates clamped into the image)
 * is darker than the centre. */
int orc_census(const uint8_t* img, int w, int h, uint64_t* out) {
    if (!img || !out || w <= 0 || h <= 0) return -1;
    for (int y = 0; y < h; ++y) {
        for (int x = 0; x < w; ++x) {
            const int c = img[y * w + x];
            uint64_t code = 0;
            int k = 0;
            for (int dy = -(ORC_CH / 2); dy <= ORC_CH / 2; ++dy) {
                for (int dx = -(ORC_CW / 2); dx <= ORC_CW / 2; ++dx) {
                    if (dx == 0 && dy == 0) continue;
                    const int v = img[clampi(y + dy, 0, h - 1) * w + clampi(x + dx, 0, w - 1)];
                    if (v < c) code |= (uint64_t)1 << k;
                    ++k;
                }
            }
            out[y * w + x] = code;
        }
    }
    return 0;
}

/* Matching cost: Hamming distance between the left code at x and the right
 * code at x-d; a right pixel left of the image costs the maximum, 62. */
int orc_cost(const uint64_t* cl, const uint64_t* cr, int w, int x, int y, int d) {
    if (x - d < 0) return ORC_CBITS;
    return bitcount64(cl[y * w + x] ^ cr[y * w + (x - d)]);
}

/* Search windows (Sec. 2.3: [d_pred +- 3 sqrt(p_pred)]; Sec. 2.4.1: pixels
 * without a usable prediction search the whole range).  The interval is made
 * integer with the centre rounded half up and the radius rounded up, both in
 * float32, the radius clamped to [r_min, r_max] and the interval clipped to
 * [0, max_disp-1].  A prediction is usable when d_pred >= 0 and p_pred >= 0
 * (NaN fails both tests); an interval that is empty after clipping falls
 * back to the full range. */
int orc_windows(const float* d_pred, const float* p_pred, int n, float k_sigma,
                int r_fixed, int r_min, int r_max, int max_disp,
                int16_t* lo, int16_t* hi, uint32_t* off) {
    if (n < 0 || max_disp < 1 || max_disp > 256 || !lo || !hi || !off) return -1;
    if (r_min < 0 || r_max < r_min) return -1;
    if (d_pred && r_fixed < 0 && !p_pred) return -1;
    off[0] = 0;
    for (int i = 0; i < n; ++i) {
        int l = 0, u = max_disp - 1;
        if (d_pred) {
            const float d = d_pred[i];
            int usable = d >= 0.0f && d <= 65536.0f;
            int r = r_fixed;
            if (usable && r_fixed < 0) {
                const float p = p_pred[i];
                if (!(p >= 0.0f)) {
                    usable = 0;
                } else {
                    const float rf = ceilf(k_sigma * sqrtf(p));
                    if (rf >= (float)r_max) r = r_max;
                    else if (rf <= (float)r_min) r = r_min;
                    else r = (int)rf;
                }
            }
            if (usable) {
                r = clampi(r, r_min, r_max);
                const int c = (int)floorf(d + 0.5f);
                const int l2 = maxi(0, c - r);
                const int u2 = mini(max_disp - 1, c + r);
                if (l2 <= u2) { l = l2; u = u2; }
            }
        }
        lo[i] = (int16_t)l;
        hi[i] = (int16_t)u;
        off[i + 1] = off[i] + (uint32_t)(u - l + 1);
    }
    return 0;
}

int orc_windows_full(int n, int max_disp, int16_t* lo, int16_t* hi, uint32_t* off) {
    return orc_windows(NULL, NULL, n, 3.0f, -1, 0, 0, max_disp, lo, hi, off);
}

int orc_cost_volume(const uint64_t* cl, const uint64_t* cr, int w, int h,
                    const int16_t* lo, const int16_t* hi, const uint32_t* off,
                    int32_t* cost) {
    if (!cl || !cr || !lo || !hi || !off || !cost) return -1;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            const int p = y * w + x;
            for (int d = lo[p]; d <= hi[p]; ++d)
                cost[off[p] + (uint32_t)(d - lo[p])] = orc_cost(cl, cr, w, x, y, d);
        }
    return 0;
}

/* The eight path directions, as the step from the predecessor to the pixel:
 * left-to-right, right-to-left, top-down, bottom-up and the four diagonals. */
int orc_direction(int dir, int* dx, int* dy) {
    static const int tab[8][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1},
                                  {1, 1}, {-1, 1}, {1, -1}, {-1, -1}};
    if (dir < 0 || dir > 7) return -1;
    *dx = tab[dir][0];
    *dy = tab[dir][1];
    return 0;
}

/* One path of semi-global matching (Hirschmüller's recurrence, cited by the
 * paper for its eight-path matcher):
 *   L(p,d) = C(p,d) + min(L(p-r,d), L(p-r,d-1)+P1, L(p-r,d+1)+P1, m+P2) - m,
 *   m = min_k L(p-r,k),
 * and L(p,d) = C(p,d) where p-r is outside the image.  With reduced windows
 * only d in W(p) is evaluated and predecessor entries outside W(p-r) count as
 * +infinity (m is taken over W(p-r)); with full windows this is the textbook
 * recurrence.  Pixels are visited row by row, rows ordered along dy and
 * columns along dx, so every predecessor is finished before it is used. */
int orc_path(const int32_t* cost, int w, int h, const int16_t* lo, const int16_t* hi,
             const uint32_t* off, int p1, int p2, int dir, int32_t* L) {
    int dx, dy;
    if (!cost || !lo || !hi || !off || !L || w <= 0 || h <= 0) return -1;
    if (p1 < 0 || p2 < p1) return -1;
    if (orc_direction(dir, &dx, &dy)) return -1;
    for (int iy = 0; iy < h; ++iy) {
        const int y = dy >= 0 ? iy : h - 1 - iy;
        for (int ix = 0; ix < w; ++ix) {
            const int x = dx >= 0 ? ix : w - 1 - ix;
            const int p = y * w + x;
            const int px = x - dx, py = y - dy;
            const int32_t* c = cost + off[p];
            int32_t* out = L + off[p];
            if (px < 0 || px >= w || py < 0 || py >= h) {
                for (int d = lo[p]; d <= hi[p]; ++d) out[d - lo[p]] = c[d - lo[p]];
                continue;
            }
            const int q = py * w + px;
            const int32_t* prev = L + off[q];
            int m = ORC_INF;
            for (int k = lo[q]; k <= hi[q]; ++k) m = mini(m, prev[k - lo[q]]);
            for (int d = lo[p]; d <= hi[p]; ++d) {
                int best = m + p2;
                if (d >= lo[q] && d <= hi[q]) best = mini(best, prev[d - lo[q]]);
                if (d - 1 >= lo[q] && d - 1 <= hi[q]) best = mini(best, prev[d - 1 - lo[q]] + p1);
                if (d + 1 >= lo[q] && d + 1 <= hi[q]) best = mini(best, prev[d + 1 - lo[q]] + p1);
                const int v = c[d - lo[p]] + best - m;
                if (v < 0 || v > ORC_CBITS + p2) return -3;
                out[d - lo[p]] = v;
            }
        }
    }
    return 0;
}

/* Winner-takes-all, subpixel and uncertainty for one pixel.
 *  - d* is the smallest d of the window attaining the minimum of S.
 *  - Subpixel (not part of the paper): a parabola through S(d*-1), S(d*),
 *    S(d*+1) when both neighbours are inside the window and the curvature
 *    a - 2b + c is positive; otherwise d* itself.
 *  - Uncertainty (Sec. 2.3.1, Eq. 9): walking away from d* on each side,
 *    the differences S(d*-+j) - S(d*) are summed and a neighbour is counted
 *    while the running sum stays below S_max; the walk stops at the window
 *    edge.  r = n_l + n_r. */
int orc_pixel_epilogue(const int32_t* S, int lo, int hi, int s_max,
                       int* d_star, double* d_sub, int* n_l, int* n_r) {
    if (!S || hi < lo) return -1;
    int best = lo;
    for (int d = lo + 1; d <= hi; ++d)
        if (S[d - lo] < S[best - lo]) best = d;
    *d_star = best;
    double sub = (double)best;
    if (best > lo && best < hi) {
        const int a = S[best - 1 - lo], b = S[best - lo], c = S[best + 1 - lo];
        const int den = a - 2 * b + c;
        if (den > 0) sub = (double)best + (double)(a - c) / (2.0 * (double)den);
    }
    *d_sub = sub;
    int acc = 0, nl = 0;
    for (int j = 1; best - j >= lo; ++j) {
        acc += S[best - j - lo] - S[best - lo];
        if (acc >= s_max) break;
        ++nl;
    }
    acc = 0;
    int nr = 0;
    for (int j = 1; best + j <= hi; ++j) {
        acc += S[best + j - lo] - S[best - lo];
        if (acc >= s_max) break;
        ++nr;
    }
    *n_l = nl;
    *n_r = nr;
    return 0;
}

/* Right disparity map from the left aggregated volume (the single-volume
 * right map of Hirschmüller's method): right pixel x' collects S(x'+d, d)
 * over every left pixel x'+d of the row whose window holds d; the smallest d
 * attaining the minimum wins; no candidate leaves the pixel invalid (-1). */
int orc_right_map(const int32_t* S, int w, int h, int max_disp, const int16_t* lo,
                  const int16_t* hi, const uint32_t* off, int16_t* disp_right) {
    if (!S || !lo || !hi || !off || !disp_right) return -1;
    for (int y = 0; y < h; ++y)
        for (int xr = 0; xr < w; ++xr) {
            int best_d = -1, best_s = ORC_INF;
            for (int d = 0; d < max_disp; ++d) {
                const int x = xr + d;
                if (x >= w) break;
                const int p = y * w + x;
                if (d < lo[p] || d > hi[p]) continue;
                const int s = S[off[p] + (uint32_t)(d - lo[p])];
                if (s < best_s) { best_s = s; best_d = d; }
            }
            disp_right[y * w + xr] = (int16_t)best_d;
        }
    return 0;
}

/* Left-right consistency check (Sec. 2.4.1): a left match d at x is kept
 * when x-d is inside the image, the right map there is valid and differs
 * from d by at most lr_tol.  Rejected pixels become invalid: -1 in the
 * integer map, -1.0 in the subpixel map and variance 0 (both nullable). */
int orc_lr_check(const int16_t* disp_right, int w, int h, int lr_tol, int16_t* disp_wta,
                 double* disp_sub, double* var_meas) {
    if (!disp_right || !disp_wta || lr_tol < 0) return -1;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            const int p = y * w + x;
            const int d = disp_wta[p];
            int ok = d >= 0 && x - d >= 0;
            if (ok) {
                const int e = disp_right[y * w + (x - d)];
                ok = e >= 0 && abs(d - e) <= lr_tol;
            }
            if (!ok) {
                disp_wta[p] = -1;
                if (disp_sub) disp_sub[p] = -1.0;
                if (var_meas) var_meas[p] = 0.0;
            }
        }
    return 0;
}

int orc_sgm(const uint8_t* left, const uint8_t* right, int w, int h, int max_disp,
            const int16_t* lo_in, const int16_t* hi_in, const uint32_t* off_in,
            int p1, int p2, int s_max, int lr_tol, int n_paths,
            uint64_t* census_l, uint64_t* census_r,
            int32_t* cost_out, int32_t* paths_out, int32_t* agg_out,
            int16_t* wta_raw, int16_t* disp_wta, double* disp_sub,
            double* var_meas, int16_t* disp_right) {
    if (!left || !right || !disp_wta || w <= 0 || h <= 0) return -1;
    if (max_disp < 1 || max_disp > 256 || p1 < 0 || p2 < p1) return -1;
    if (n_paths != 4 && n_paths != 8) return -1;
    if ((lo_in == NULL) != (hi_in == NULL) || (lo_in == NULL) != (off_in == NULL)) return -1;
    const size_t n = (size_t)w * (size_t)h;
    int rc = -2;
    uint64_t* cl = malloc(n * sizeof(uint64_t));
    uint64_t* cr = malloc(n * sizeof(uint64_t));
    int16_t* lo = malloc(n * sizeof(int16_t));
    int16_t* hi = malloc(n * sizeof(int16_t));
    uint32_t* off = malloc((n + 1) * sizeof(uint32_t));
    int32_t *cost = NULL, *L = NULL, *S = NULL;
    int16_t* dr = malloc(n * sizeof(int16_t));
    if (!cl || !cr || !lo || !hi || !off || !dr) goto done;

    if (lo_in) {
        memcpy(lo, lo_in, n * sizeof(int16_t));
        memcpy(hi, hi_in, n * sizeof(int16_t));
        memcpy(off, off_in, (n + 1) * sizeof(uint32_t));
        rc = -1;
        if (off[0] != 0) goto done;
        for (size_t p = 0; p < n; ++p)
            if (lo[p] < 0 || hi[p] < lo[p] || hi[p] >= max_disp ||
                off[p + 1] - off[p] != (uint32_t)(hi[p] - lo[p] + 1))
                goto done;
        rc = -2;
    } else {
        orc_windows_full((int)n, max_disp, lo, hi, off);
    }
    const size_t total = off[n];
    cost = malloc(total * sizeof(int32_t));
    L = malloc(total * sizeof(int32_t));
    S = calloc(total, sizeof(int32_t));
    if (!cost || !L || !S) goto done;

    orc_census(left, w, h, cl);
    orc_census(right, w, h, cr);
    if (census_l) memcpy(census_l, cl, n * sizeof(uint64_t));
    if (census_r) memcpy(census_r, cr, n * sizeof(uint64_t));
    orc_cost_volume(cl, cr, w, h, lo, hi, off, cost);
    if (cost_out) memcpy(cost_out, cost, total * sizeof(int32_t));

    /* Aggregation: S(p,d) is the sum of the path costs over the directions
     * used: all eight, or the four axis-aligned ones (0-3: along and against
     * the rows and the columns) of the cheaper 4-path variant. */
    for (int dir = 0; dir < n_paths; ++dir) {
        rc = orc_path(cost, w, h, lo, hi, off, p1, p2, dir, L);
        if (rc) goto done;
        for (size_t i = 0; i < total; ++i) S[i] += L[i];
        if (paths_out) memcpy(paths_out + (size_t)dir * total, L, total * sizeof(int32_t));
    }
    rc = -3;
    for (size_t i = 0; i < total; ++i)
        if (S[i] > 65535) goto done;
    if (agg_out) memcpy(agg_out, S, total * sizeof(int32_t));

    /* Left map: WTA, subpixel, uncertainty. */
    for (size_t p = 0; p < n; ++p) {
        int ds, nl, nr;
        double sub;
        orc_pixel_epilogue(S + off[p], lo[p], hi[p], s_max, &ds, &sub, &nl, &nr);
        disp_wta[p] = (int16_t)ds;
        if (disp_sub) disp_sub[p] = sub;
        if (var_meas) var_meas[p] = (double)(nl + nr);
    }
    if (wta_raw) memcpy(wta_raw, disp_wta, n * sizeof(int16_t));

    orc_right_map(S, w, h, max_disp, lo, hi, off, dr);
    if (disp_right) memcpy(disp_right, dr, n * sizeof(int16_t));
    if (lr_tol >= 0) orc_lr_check(dr, w, h, lr_tol, disp_wta, disp_sub, var_meas);
    rc = 0;
done:
    free(cl); free(cr); free(lo); free(hi); free(off);
    free(cost); free(L); free(S); free(dr);
    return rc;
}

/* Gamma of Eq. 1 extended with the principal point (cx, cy), which the
 * paper's matrix omits (it is the case cx = cy = 0):
 *   Gamma = [[f,0,cx,0],[0,f,cy,0],[0,0,0,f b],[0,0,1,0]],
 * and its inverse written out; H = Gamma T Gamma^-1 (Eq. 4) by explicit 4x4
 * products, T = [R t; 0 0 0 1] mapping previous-frame coordinates to the
 * current frame as Eq. 2 states. */
int orc_warp_matrix(const double* R, const double* t, double f, double cx, double cy,
                    double b, double* H) {
    if (!R || !t || !H || !(f > 0.0) || !(b > 0.0)) return -1;
    const double G[4][4] = {{f, 0, cx, 0}, {0, f, cy, 0}, {0, 0, 0, f * b}, {0, 0, 1, 0}};
    const double Gi[4][4] = {{1.0 / f, 0, 0, -cx / f},
                             {0, 1.0 / f, 0, -cy / f},
                             {0, 0, 0, 1},
                             {0, 0, 1.0 / (f * b), 0}};
    const double T[4][4] = {{R[0], R[1], R[2], t[0]},
                            {R[3], R[4], R[5], t[1]},
                            {R[6], R[7], R[8], t[2]},
                            {0, 0, 0, 1}};
    double GT[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s += G[i][k] * T[k][j];
            GT[i][j] = s;
        }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s += GT[i][k] * Gi[k][j];
            H[i * 4 + j] = s;
        }
    return 0;
}

/* Disparity prediction (Sec. 2.2).  Each source pixel with d > 0 is moved by
 * omega* = H omega (Eq. 3) and normalised by its fourth component; its
 * variance is predicted as Phi^2 p + q with Phi = d'/d (Eq. 5-6).  The
 * predicted pixel is (x', y') rounded half up.  On collisions the largest d'
 * is kept (Sec. 2.2.2); the paper is silent on equal d', which keep the
 * source with the smaller pixel index.  Sources whose fourth component is
 * not positive or whose target leaves the image are dropped.
 *
 * Which source wins each target is an integer decision taken from floating
 * point, so it is taken in float32 with H rounded to float32 and this exact
 * evaluation order: omega_i = ((H_i0 x + H_i1 y) + H_i2 d) + H_i3,
 * x' = omega_0/omega_3, y' = omega_1/omega_3, d' = d/omega_3.  The values
 * written for the winner, d' = omega_2/omega_3 and p' = Phi^2 p + q, are
 * then evaluated in double with the double H.  d_key_f32 (nullable) gets the
 * float32 d' the z-buffer compared. */
int orc_warp(const float* d_prev, const float* p_prev, int w, int h,
             const double* R, const double* t, double f, double cx, double cy,
             double b, double q, double* d_pred, double* p_pred,
             int32_t* winner, float* d_key_f32) {
    if (!d_prev || !p_prev || !d_pred || !p_pred || w <= 0 || h <= 0) return -1;
    if (!(q > 0.0)) return -1;
    double Hd[16];
    if (orc_warp_matrix(R, t, f, cx, cy, b, Hd)) return -1;
    float Hf[16];
    for (int i = 0; i < 16; ++i) Hf[i] = (float)Hd[i];
    const size_t n = (size_t)w * (size_t)h;
    float* best = malloc(n * sizeof(float));
    int32_t* src = malloc(n * sizeof(int32_t));
    if (!best || !src) { free(best); free(src); return -2; }
    for (size_t i = 0; i < n; ++i) { best[i] = 0.0f; src[i] = -1; }

    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            const float d = d_prev[y * w + x];
            if (!(d > 0.0f)) continue;
            const float xf = (float)x, yf = (float)y;
            const float o0 = ((Hf[0] * xf + Hf[1] * yf) + Hf[2] * d) + Hf[3];
            const float o1 = ((Hf[4] * xf + Hf[5] * yf) + Hf[6] * d) + Hf[7];
            const float o3 = ((Hf[12] * xf + Hf[13] * yf) + Hf[14] * d) + Hf[15];
            if (!(o3 > 0.0f)) continue;
            const float xp = o0 / o3, yp = o1 / o3, dp = d / o3;
            const float vx = xp + 0.5f, vy = yp + 0.5f;
            if (!(vx >= 0.0f) || !(vx < (float)w) || !(vy >= 0.0f) || !(vy < (float)h)) continue;
            const int xi = (int)floorf(vx), yi = (int)floorf(vy);
            const size_t tgt = (size_t)yi * (size_t)w + (size_t)xi;
            /* sources are visited in increasing index, so a strict > keeps
             * the smaller index on equal d' */
            if (src[tgt] < 0 || dp > best[tgt]) { best[tgt] = dp; src[tgt] = y * w + x; }
        }

    for (size_t i = 0; i < n; ++i) {
        if (winner) winner[i] = src[i];
        if (src[i] < 0) {
            d_pred[i] = -1.0;
            p_pred[i] = 0.0;
            if (d_key_f32) d_key_f32[i] = -1.0f;
            continue;
        }
        const int sx = src[i] % w, sy = src[i] / w;
        const double d = (double)d_prev[src[i]], p = (double)p_prev[src[i]];
        const double om[4] = {Hd[0] * sx + Hd[1] * sy + Hd[2] * d + Hd[3],
                              Hd[4] * sx + Hd[5] * sy + Hd[6] * d + Hd[7],
                              Hd[8] * sx + Hd[9] * sy + Hd[10] * d + Hd[11],
                              Hd[12] * sx + Hd[13] * sy + Hd[14] * d + Hd[15]};
        const double dn = om[2] / om[3];
        const double phi = dn / d;
        d_pred[i] = dn;
        p_pred[i] = phi * phi * p + q;
        if (d_key_f32) d_key_f32[i] = best[i];
    }
    free(best);
    free(src);
    return 0;
}

/* Refinement of the predicted map (Sec. 2.2.2), in this order:
 *  1. edge rejection: the paper drops predictions near disparity
 *     discontinuities without giving a test; here a valid predicted pixel is
 *     dropped when a valid pixel of its 3x3 neighbourhood differs from it by
 *     more than edge_tol (float32 comparison; edge_tol < 0 disables it);
 *  2. horizontal zoom hole filling (Eq. 7-8): an invalid pixel whose left
 *     and right neighbours are valid with |a - b| < fill_tol (float32) gets
 *     d = (a + b)/2 and, as the paper gives no rule for the variance, the
 *     mean of the two neighbours' variances; the pass reads the map left by
 *     step 1 only, so fills do not propagate along a row;
 *  3. the same with the vertical neighbours, reading the result of step 2.
 * fill_tol <= 0 disables steps 2 and 3.  The means are exact in double and
 * rounded once to float32.  Outputs may not alias the inputs. */
int orc_refine(const float* d_in, const float* p_in, int w, int h, float edge_tol,
               float fill_tol, float* d_out, float* p_out) {
    if (!d_in || !p_in || !d_out || !p_out || w <= 0 || h <= 0) return -1;
    const size_t n = (size_t)w * (size_t)h;
    float* ed = malloc(n * sizeof(float));
    float* ep = malloc(n * sizeof(float));
    float* hd = malloc(n * sizeof(float));
    float* hp = malloc(n * sizeof(float));
    if (!ed || !ep || !hd || !hp) { free(ed); free(ep); free(hd); free(hp); return -2; }
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            const size_t i = (size_t)y * w + x;
            const float d = d_in[i];
            int keep = d >= 0.0f;
            if (keep && edge_tol >= 0.0f) {
                for (int dy = -1; dy <= 1 && keep; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        const int xx = x + dx, yy = y + dy;
                        if (xx < 0 || xx >= w || yy < 0 || yy >= h) continue;
                        const float e = d_in[(size_t)yy * w + xx];
                        if (e >= 0.0f && fabsf(d - e) > edge_tol) { keep = 0; break; }
                    }
            }
            ed[i] = keep ? d : -1.0f;
            ep[i] = keep ? p_in[i] : 0.0f;
        }
    for (size_t i = 0; i < n; ++i) { hd[i] = ed[i]; hp[i] = ep[i]; }
    if (fill_tol > 0.0f) {
        for (int y = 0; y < h; ++y)
            for (int x = 1; x + 1 < w; ++x) {
                const size_t i = (size_t)y * w + x;
                const float a = ed[i - 1], b = ed[i + 1];
                if (ed[i] < 0.0f && a >= 0.0f && b >= 0.0f && fabsf(a - b) < fill_tol) {
                    hd[i] = (float)(((double)a + (double)b) / 2.0);
                    hp[i] = (float)(((double)ep[i - 1] + (double)ep[i + 1]) / 2.0);
                }
            }
    }
    for (size_t i = 0; i < n; ++i) { d_out[i] = hd[i]; p_out[i] = hp[i]; }
    if (fill_tol > 0.0f) {
        for (int y = 1; y + 1 < h; ++y)
            for (int x = 0; x < w; ++x) {
                const size_t i = (size_t)y * w + x;
                const float a = hd[i - w], b = hd[i + w];
                if (hd[i] < 0.0f && a >= 0.0f && b >= 0.0f && fabsf(a - b) < fill_tol) {
                    d_out[i] = (float)(((double)a + (double)b) / 2.0);
                    p_out[i] = (float)(((double)hp[i - w] + (double)hp[i + w]) / 2.0);
                }
            }
    }
    free(ed); free(ep); free(hd); free(hp);
    return 0;
}

/* Pixel-wise Kalman update (Sec. 2.4, Eq. 10-12):
 *   K = p/(p + r), d = d_pred + K (z - d_pred), p = (1 - K) p_pred.
 * Validity (the paper takes no prediction as it is, Sec. 2.3.2, and rejected
 * pixels fall back to a full search, Sec. 2.4.1):
 *  - prediction usable (d_pred >= 0, p_pred > 0) and measurement valid
 *    (z >= 0, r >= 0): the update above;
 *  - measurement only: d = z, p = r (the K = 1 limit; the first frame);
 *  - prediction only: invalid (-1, 0), or (d_pred, p_pred) when
 *    keep_unmeasured is set (the K = 0 limit);
 *  - neither: invalid (-1, 0). */
int orc_kalman(const float* d_pred, const float* p_pred, const float* z,
               const float* r, int n, int keep_unmeasured,
               double* d_out, double* p_out) {
    if (!d_pred || !p_pred || !z || !r || !d_out || !p_out || n < 0) return -1;
    for (int i = 0; i < n; ++i) {
        const int pv = d_pred[i] >= 0.0f && p_pred[i] > 0.0f;
        const int mv = z[i] >= 0.0f && r[i] >= 0.0f;
        if (pv && mv) {
            const double dp = d_pred[i], pp = p_pred[i], zz = z[i], rr = r[i];
            const double K = pp / (pp + rr);
            d_out[i] = dp + K * (zz - dp);
            p_out[i] = (1.0 - K) * pp;
        } else if (mv) {
            d_out[i] = z[i];
            p_out[i] = r[i];
        } else if (pv && keep_unmeasured) {
            d_out[i] = d_pred[i];
            p_out[i] = p_pred[i];
        } else {
            d_out[i] = -1.0;
            p_out[i] = 0.0;
        }
    }
    return 0;
}

/* SAD check (Sec. 2.4.1 names it beside the left-right check as a filter of
 * outliers before a map is propagated; it gives no window or threshold).
 * For a pixel with a disparity d >= 0: the sum of |I_L(x+i, y+j) -
 * I_R(x+i-d, y+j)| over i, j in [-radius, radius], coordinates clamped into
 * the image (as the census does).  A pixel whose sum exceeds sad_max is
 * rejected like a left-right failure (-1 / -1.0 / 0), in place. */
int orc_sad_check(const uint8_t* left, const uint8_t* right, int w, int h, int radius,
                  int sad_max, int16_t* disp_wta, double* disp_sub, double* var_meas) {
    if (!left || !right || !disp_wta || w <= 0 || h <= 0 || radius < 0) return -1;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            const size_t p = (size_t)y * w + x;
            const int d = disp_wta[p];
            if (d < 0) continue;
            long sad = 0;
            for (int j = -radius; j <= radius; ++j) {
                int yy = y + j;
                yy = yy < 0 ? 0 : (yy >= h ? h - 1 : yy);
                for (int i = -radius; i <= radius; ++i) {
                    int xl = x + i, xr = x + i - d;
                    xl = xl < 0 ? 0 : (xl >= w ? w - 1 : xl);
                    xr = xr < 0 ? 0 : (xr >= w ? w - 1 : xr);
                    sad += labs((long)left[(size_t)yy * w + xl] - (long)right[(size_t)yy * w + xr]);
                }
            }
            if (sad > sad_max) {
                disp_wta[p] = -1;
                if (disp_sub) disp_sub[p] = -1.0;
                if (var_meas) var_meas[p] = 0.0;
            }
        }
    return 0;
}

/* Left-right check of a *prediction* (Sec. 2.4.1 and the processing order
 * of Fig. 4: warp, zoom filling, then this check).  The right map of frame
 * k-1 is warped like the left one (with the right camera's motion); a left
 * prediction d >= 0 is kept when the right prediction at
 * xr = x - floorf(d + 0.5f) exists (xr >= 0, value >= 0) and differs from d
 * by at most tol (float32 comparison); otherwise the pixel becomes invalid
 * (d = -1, p = 0), so it is searched over the full range.  In place. */
int orc_lr_check_prediction(float* d_pred, float* p_pred, const float* d_right, int w, int h,
                            float tol) {
    if (!d_pred || !p_pred || !d_right || w <= 0 || h <= 0) return -1;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            const size_t p = (size_t)y * w + x;
            const float d = d_pred[p];
            if (!(d >= 0.0f)) continue;
            /* d >= w points left of the image anyway; the test keeps the cast in range */
            const int xr = d < (float)w ? x - (int)floorf(d + 0.5f) : -1;
            int ok = 0;
            if (xr >= 0) {
                const float e = d_right[(size_t)y * w + xr];
                ok = e >= 0.0f && fabsf(e - d) <= tol;
            }
            if (!ok) {
                d_pred[p] = -1.0f;
                p_pred[p] = 0.0f;
            }
        }
    return 0;
}

/* Motion of the right camera of a rectified rig from the left one's: with
 * M_R = M_L - (b, 0, 0), M_L^k = R M_L^{k-1} + t gives
 * M_R^k = R M_R^{k-1} + t + R (b, 0, 0) - (b, 0, 0). */
int orc_right_motion(const double* R, const double* t, double b, double* t_right) {
    if (!R || !t || !t_right) return -1;
    for (int i = 0; i < 3; ++i) t_right[i] = t[i] + R[3 * i] * b - (i == 0 ? b : 0.0);
    return 0;
}
