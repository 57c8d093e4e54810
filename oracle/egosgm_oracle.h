/*
 * egosgm_oracle.h — plain, slow, single-threaded CPU oracle for ego-motion
 * reduced census + SGM disparity estimation (Fućek et al., "Dense Disparity
 * Estimation in Ego-motion Reduced Search Space").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this code: it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can check the GPU library against an independent
 * statement of what the method computes.  It shares no code, header, table or
 * constant with the GPU library.
 *
 * Conventions (all arrays row-major, pixel index p = y*w + x):
 *  - images: uint8, w*h, pitch = w;
 *  - census codes: uint64 per pixel, bits 0..61;
 *  - ragged volumes: pixel p owns entries off[p] .. off[p+1]-1, entry
 *    off[p] + (d - lo[p]) holds disparity d of the window [lo[p], hi[p]];
 *  - invalid disparities are -1 (int16) or -1.0 (floating point).
 * Return codes: 0 ok, -1 bad argument, -2 out of memory, -3 an internal bound
 * of the recurrence was violated (a bug in the oracle itself).
 */
#ifndef EGOSGM_ORACLE_H
#define EGOSGM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Census transform, 9 wide x 7 tall, clamped borders. */
int orc_census(const uint8_t* img, int w, int h, uint64_t* out);

/* Matching cost of left pixel (x,y) at disparity d: Hamming distance of the
 * census codes, or 62 when x-d falls left of the image. */
int orc_cost(const uint64_t* cl, const uint64_t* cr, int w, int x, int y, int d);

/* Per-pixel search windows from a predicted disparity/variance map.  d_pred
 * may be NULL (every pixel gets the full range).  off has n+1 entries. */
int orc_windows(const float* d_pred, const float* p_pred, int n, float k_sigma,
                int r_fixed, int r_min, int r_max, int max_disp,
                int16_t* lo, int16_t* hi, uint32_t* off);

/* Full-range windows: lo = 0, hi = max_disp-1, off[p] = p*max_disp. */
int orc_windows_full(int n, int max_disp, int16_t* lo, int16_t* hi, uint32_t* off);

/* Cost volume over the ragged windows. */
int orc_cost_volume(const uint64_t* cl, const uint64_t* cr, int w, int h,
                    const int16_t* lo, const int16_t* hi, const uint32_t* off,
                    int32_t* cost);

/* One SGM path (direction index 0..7, see orc_direction) over a given cost
 * volume, with out-of-window predecessor entries treated as +infinity. */
int orc_path(const int32_t* cost, int w, int h, const int16_t* lo, const int16_t* hi,
             const uint32_t* off, int p1, int p2, int dir, int32_t* L);

/* Step (dx,dy) from predecessor to pixel for direction index dir. */
int orc_direction(int dir, int* dx, int* dy);

/* Per-pixel epilogue on one aggregated-cost row S[0..hi-lo]:
 * winner-takes-all, parabola subpixel (double) and uncertainty count. */
int orc_pixel_epilogue(const int32_t* S, int lo, int hi, int s_max,
                       int* d_star, double* d_sub, int* n_l, int* n_r);

/* Right map from an aggregated ragged volume S (left-image indexed). */
int orc_right_map(const int32_t* S, int w, int h, int max_disp, const int16_t* lo,
                  const int16_t* hi, const uint32_t* off, int16_t* disp_right);

/* Left-right check in place on disp_wta (and disp_sub / var_meas). */
int orc_lr_check(const int16_t* disp_right, int w, int h, int lr_tol, int16_t* disp_wta,
                 double* disp_sub, double* var_meas);

/* Whole matcher: census, cost, n_paths (8, or 4 = directions 0-3) paths,
 * aggregation, WTA, subpixel, uncertainty, right disparity map and
 * left-right check.  lo/hi/off NULL means full range.  Every output except
 * disp_wta may be NULL; paths_out holds n_paths volumes. */
int orc_sgm(const uint8_t* left, const uint8_t* right, int w, int h, int max_disp,
            const int16_t* lo, const int16_t* hi, const uint32_t* off,
            int p1, int p2, int s_max, int lr_tol, int n_paths,
            uint64_t* census_l, uint64_t* census_r,
            int32_t* cost_out, int32_t* paths_out, int32_t* agg_out,
            int16_t* wta_raw, int16_t* disp_wta, double* disp_sub,
            double* var_meas, int16_t* disp_right);

/* H = Gamma T Gamma^-1 in double, T = [R t; 0 1] (R row-major). */
int orc_warp_matrix(const double* R, const double* t, double f, double cx, double cy,
                    double b, double* H);

/* Disparity-map warp with z-buffer.  Target pixel and z-order (largest d',
 * then smallest source index) are decided in float32 with H rounded to
 * float32; the kept disparity and variance are then evaluated in double for
 * the winning source.  winner (nullable) gets the source pixel index or -1;
 * d_key_f32 (nullable) the float32 d' that won. */
int orc_warp(const float* d_prev, const float* p_prev, int w, int h,
             const double* R, const double* t, double f, double cx, double cy,
             double b, double q, double* d_pred, double* p_pred,
             int32_t* winner, float* d_key_f32);

/* Prediction refinement: edge rejection, then horizontal and vertical
 * one-pixel hole filling (float outputs, exact means). */
int orc_refine(const float* d_in, const float* p_in, int w, int h, float edge_tol,
               float fill_tol, float* d_out, float* p_out);

/* Pixel-wise Kalman update in double. */
int orc_kalman(const float* d_pred, const float* p_pred, const float* z,
               const float* r, int n, int keep_unmeasured,
               double* d_out, double* p_out);

#ifdef __cplusplus
}
#endif
/* SAD check in place: pixels whose (2 radius + 1)^2 sum of absolute left /
 * right differences at their disparity exceeds sad_max become invalid. */
int orc_sad_check(const uint8_t* left, const uint8_t* right, int w, int h, int radius,
                  int sad_max, int16_t* disp_wta, double* disp_sub, double* var_meas);

/* Left-right check of a prediction against the warped right map (in place). */
int orc_lr_check_prediction(float* d_pred, float* p_pred, const float* d_right, int w, int h,
                            float tol);
/* Translation of the right camera's motion (same rotation). */
int orc_right_motion(const double* R, const double* t, double b, double* t_right);

#endif
