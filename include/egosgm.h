/*
 * egosgm.h — C ABI of the MI355X (gfx950) library for dense disparity
 * estimation in an ego-motion reduced search space (Fućek, Marković, Cvišić,
 * Petrović: "Dense Disparity Estimation in Ego-motion Reduced Search Space").
 *
 * The method (Sec. 2) runs, per stereo frame k:
 *   disparity prediction  D^{k|k-1}, P^{k|k-1} from D^{k-1}, P^{k-1} and the
 *                         ego-motion (Sec. 2.1-2.2)          -> warp_disparity
 *   refinement            edge rejection, zoom hole filling (Sec. 2.2.2)
 *                         -> refine_prediction (or both in predict_disparity)
 *   search windows        [d^{k|k-1} +- 3 sqrt(p^{k|k-1})] (Sec. 2.3)
 *                                                 -> sgm_windows_from_prediction
 *   stereo matching       census + 8-path SGM over those windows, matching
 *                         uncertainty (Sec. 2.3, Eq. 9), left-right check
 *                         (Sec. 2.4.1)               -> sgm_reduced / sgm_full
 *   disparity update      pixel-wise Kalman filter (Sec. 2.4, Eq. 10-12)
 *                                                             -> kalman_update
 *
 * General rules for every entry point:
 *  - Buffer arguments are DEVICE pointers (HIP device memory, e.g. the data
 *    of torch tensors on the GPU) unless the argument says "host".  The
 *    caller owns every buffer; the library never allocates, frees or keeps
 *    caller-visible memory.  Its only process-wide state is the launch
 *    tuning (egosgm_set_tuning) and the opt-in stage timing
 *    (egosgm_timing_enable); results never depend on either.
 *  - Images and maps are row-major, pixel p = y*w + x.  Images are uint8
 *    with a row pitch in bytes (pitch >= w); every map is dense (pitch = w).
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL is the
 *    null stream): it only enqueues work.  Results are ready once the
 *    stream has been synchronised.  Calls on one stream run in order.
 *  - Return value: EGOSGM_OK, or a negative egosgm_status.  Arguments are
 *    validated on the host before anything is enqueued; on an error nothing
 *    is enqueued (EDEVICE: a launch failed; earlier launches of the same call
 *    may have been enqueued).  Nothing is printed, nothing throws.
 *  - Device-side contents that cannot be checked without a copy (window
 *    bounds, offsets) are documented preconditions.
 *  - Invalid disparities are -1 in int16 maps and -1.0f in float maps; the
 *    variance of an invalid pixel is 0 and is never read.
 */
#ifndef EGOSGM_H
#define EGOSGM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EGOSGM_ABI_VERSION 5

/* Largest disparity range and the census window (9 wide, 7 tall: 62 bits). */
#define EGOSGM_MAX_DISP 256
#define EGOSGM_CENSUS_BITS 62

typedef enum egosgm_status {
    EGOSGM_OK = 0,
    EGOSGM_EINVAL = -1,      /* a pointer, size or parameter is out of range   */
    EGOSGM_EWORKSPACE = -2,  /* the workspace is NULL or smaller than required */
    EGOSGM_EDEVICE = -3,     /* a HIP launch or copy failed                    */
    EGOSGM_EUNSUPPORTED = -4 /* valid request this build does not implement    */
} egosgm_status;

/* Matcher parameters.  The paper fixes none of them (it names a 3x3
 * matching window and S_max = 10 for it, Sec. 2.3.1); the values used for
 * the street sequences are D = 128, P1 = 10, P2 = 120, S_max = 80, lr_tol = 1. */
typedef struct egosgm_sgm_params {
    int32_t max_disp; /* D: disparities 0..D-1, 1 <= D <= 256                  */
    int32_t p1;       /* penalty for a disparity change of 1, 0 <= p1 <= p2    */
    int32_t p2;       /* penalty for larger changes, p2 <= 255 - 62 = 193      */
    int32_t s_max;    /* uncertainty threshold of Eq. 9, >= 0                  */
    int32_t lr_tol;   /* left-right tolerance in pixels; < 0 disables the check */
    int32_t n_paths;  /* aggregated directions: 8 (0 means 8), or 4 for the cheaper
                         variant along and against the rows and the columns       */
    int32_t census_ready; /* 0: the call computes the census codes; 1: sgm_census
                         already wrote them (and reset the right-map keys) into
                         this workspace, e.g. on another stream, ordered before
                         this call.  Plans require 0.                             */
} egosgm_sgm_params;

/* Optional intermediate outputs for inspection (each member nullable; the
 * struct pointer itself may be NULL).  "slots" is the ragged volume: pixel p
 * owns entries offsets[p] .. offsets[p+1]-1, entry offsets[p] + (d - lo[p])
 * holds disparity d; the full range is the case offsets[p] = p*D. */
typedef struct egosgm_debug {
    uint64_t* census_left;  /* w*h census codes of the left image            */
    uint64_t* census_right; /* w*h census codes of the right image           */
    uint8_t* cost;          /* slots: matching cost C(p,d), 0..62            */
    uint8_t* paths;         /* 8 x slots: path costs L_r(p,d), direction-major */
    uint16_t* agg;          /* slots: aggregated cost S(p,d) = sum_r L_r     */
    int16_t* wta_raw;       /* w*h: winner-takes-all disparity before the LR check */
} egosgm_debug;

int egosgm_abi_version(void);
const char* egosgm_status_string(int status);

/* ------------------------------------------------------------------ census
 * 9x7 census transform (the matching cost of the matcher; the paper names
 * only its [3x3] matching window, Sec. 2.3.1).  Bit k of out[p] is set when
 * the k-th neighbour, visited row by row (dy = -3..3 outer, dx = -4..4
 * inner, centre skipped, coordinates clamped into the image), is darker than
 * the centre.  Bits 62 and 63 are zero.
 *   img: w x h uint8, row pitch `pitch` bytes.  out: w*h uint64.          */
int egosgm_census(const uint8_t* img, int w, int h, int pitch, uint64_t* out, void* stream);

/* ------------------------------------------------------------------ SGM
 * Workspace bytes for sgm_full / sgm_reduced on a w x h pair with disparity
 * range max_disp (sized for the full range; a reduced call never needs more).
 * Returns 0 for out-of-range arguments. */
size_t egosgm_sgm_workspace_bytes(int w, int h, int max_disp);

/* Full-range semi-global matching (Sec. 2.3 with no prediction: the first
 * frame and the pixels rejected in the previous frame search the whole
 * range, Sec. 2.4.1 and Sec. 3).
 *   cost  C(p,d) = popcount(cL(x,y) ^ cR(x-d,y)), or 62 where x-d < 0;
 *   paths L_r(p,d) = C + min(L_r(p-r,d), L_r(p-r,d+-1)+P1, m+P2) - m,
 *         m = min_k L_r(p-r,k), for the 8 directions r (Sec. 2.3 uses eight
 *         paths; the recurrence of Hirschmüller 2008);
 *   S(p,d) = sum_r L_r(p,d);  d* = smallest argmin_d S(p,d);
 *   disp_sub = d* + (a-c)/(2(a-2b+c)) with a,b,c = S(d*-1), S(d*), S(d*+1)
 *         when d* is inside the window and a-2b+c > 0, else d*;
 *   var_meas = n_l + n_r, the neighbours counted on each side of d* while the
 *         running sum of S(d*+-j) - S(d*) stays below s_max (Eq. 9);
 *   disp_right(x') = smallest argmin_d S(x'+d, d) over the left pixels whose
 *         window holds d, or -1;
 *   LR check: d* is kept when x-d* >= 0, disp_right(x-d*) is valid and
 *         |d* - disp_right(x-d*)| <= lr_tol; rejected pixels are written as
 *         -1 / -1.0f / 0.
 * Inputs: left, right (w x h uint8, pitch).  Outputs (w*h each): disp_wta
 * int16, disp_sub float, var_meas float, disp_right int16 (nullable).
 * workspace: device memory of at least egosgm_sgm_workspace_bytes(w,h,D). */
int sgm_full(const uint8_t* left, const uint8_t* right, int w, int h, int pitch,
             const egosgm_sgm_params* params, int16_t* disp_wta, float* disp_sub,
             float* var_meas, int16_t* disp_right, const egosgm_debug* debug,
             void* workspace, size_t workspace_bytes, void* stream);

/* The census pass of sgm_full / sgm_reduced on its own (the 9x7 census of
 * both images, Sec. 2.3.1's matching cost, and the reset of the right-map
 * keys), into `workspace` as those calls lay it out for (w, h, max_disp).
 * A following sgm_full / sgm_reduced on the same workspace with
 * census_ready = 1 skips its own census pass, so the census can run on
 * another stream while the prediction of the frame runs; the caller orders
 * the two (an event) and must not start it before the previous matcher call
 * on this workspace has finished.  EINVAL / EWORKSPACE as sgm_full. */
int sgm_census(const uint8_t* left, const uint8_t* right, int w, int h, int pitch, int max_disp,
               void* workspace, size_t workspace_bytes, void* stream);

/* Workspace bytes for sgm_windows_from_prediction on a w x h map. */
size_t egosgm_windows_workspace_bytes(int w, int h);

/* Per-pixel search windows from the predicted map (Sec. 2.3: the interval
 * [d +- 3 sqrt(p)] around the prediction; pixels without a usable prediction
 * search the whole range, Sec. 2.4.1):
 *   a prediction is usable when d_pred >= 0 (and <= 65536) and, when the
 *   radius comes from the variance, p_pred >= 0;
 *   centre c = floorf(d_pred + 0.5f); radius r = r_fixed if r_fixed >= 0,
 *   else ceilf(k_sigma * sqrtf(p_pred)), both in float32; r clamped to
 *   [r_min, r_max]; lo = max(0, c-r), hi = min(D-1, c+r); an unusable
 *   prediction or an empty interval gives [0, D-1].
 *   offsets[p] = sum of (hi-lo+1) over the pixels before p, offsets[w*h] =
 *   the total (w*h+1 entries).
 * d_pred, p_pred: w*h float (p_pred may be NULL when r_fixed >= 0).
 * lo, hi: w*h int16.  workspace: egosgm_windows_workspace_bytes(w,h). */
int sgm_windows_from_prediction(const float* d_pred, const float* p_pred, int w, int h,
                                float k_sigma, int r_fixed, int r_min, int r_max,
                                int max_disp, int16_t* lo, int16_t* hi, uint32_t* offsets,
                                void* workspace, size_t workspace_bytes, void* stream);

/* sgm_windows_from_prediction without a workspace, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, rules and results; the scan's per-chunk
 * totals live in a fixed device array of the library instead, one per GPU
 * (the current device at the call), held until the process ends.  Limit:
 * h * ceil(w / 256) <= EGOSGM_NOALLOC_WINDOW_CHUNKS (e.g. 4096 x 4096), else
 * EGOSGM_EUNSUPPORTED and nothing is enqueued.  The call allocates nothing.
 * Calls that overlap on one GPU (other streams, other threads) share that
 * array and race: order them, e.g. on one stream. */
#define EGOSGM_NOALLOC_WINDOW_CHUNKS 65536
int sgm_windows_from_prediction_noalloc(const float* d_pred, const float* p_pred, int w, int h,
                                        float k_sigma, int r_fixed, int r_min, int r_max,
                                        int max_disp, int16_t* lo, int16_t* hi,
                                        uint32_t* offsets, void* stream);

/* Reduced-range semi-global matching (Sec. 2.3): sgm_full restricted to the
 * per-pixel windows [lo[p], hi[p]]; predecessor entries outside the
 * predecessor's window count as +infinity and m is the minimum over that
 * window (with every window [0, D-1] this is exactly sgm_full).
 * lo, hi, offsets: as written by sgm_windows_from_prediction; preconditions
 * (not checked): 0 <= lo <= hi < D, offsets[0] = 0, offsets[p+1]-offsets[p] =
 * hi-lo+1.  Other arguments as sgm_full; debug volumes hold offsets[w*h]
 * entries (paths: 8 blocks of w*h*D entries, the first offsets[w*h] of each
 * filled). */
int sgm_reduced(const uint8_t* left, const uint8_t* right, int w, int h, int pitch,
                const int16_t* lo, const int16_t* hi, const uint32_t* offsets,
                const egosgm_sgm_params* params, int16_t* disp_wta, float* disp_sub,
                float* var_meas, int16_t* disp_right, const egosgm_debug* debug,
                void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------ warp
 * Disparity-space motion matrix H = Gamma T Gamma^-1 (Eq. 1 and 4) with the
 * principal point added to Gamma (the paper's Gamma is cx = cy = 0):
 * Gamma = [[f,0,cx,0],[0,f,cy,0],[0,0,0,f b],[0,0,1,0]], T = [R t; 0 1].
 * R (row-major 3x3) and t (metres) map previous-frame camera coordinates to
 * the current frame, M^k = R M^{k-1} + t as in Eq. 2 (so driving forward by
 * 1 m is t = (0,0,-1)).  Computed in double on the host and rounded once to
 * float: H (host, 16 floats, row-major).  Host only; enqueues nothing. */
int egosgm_warp_matrix(const double* R, const double* t, double f, double cx, double cy,
                       double baseline, float* H);

/* Disparity prediction (Sec. 2.2): every source pixel with d > 0 moves to
 * omega* = H (x, y, d, 1) (Eq. 3), normalised by its fourth component; its
 * variance is predicted as Phi^2 p + q with Phi = d'/d (Eq. 5-6).
 * Which source lands where, and which wins a collision, is decided in
 * float32 with H rounded to float32, in this order:
 * omega_i = ((H_i0 x + H_i1 y) + H_i2 d) + H_i3, x' = omega_0/omega_3,
 * y' = omega_1/omega_3, d' = d/omega_3; the target pixel is
 * (floorf(x'+0.5f), floorf(y'+0.5f)); sources with omega_3 <= 0 or a target
 * outside the image are dropped.  Collisions keep the largest d' (Sec. 2.2.2:
 * the nearest surface), then the smaller source pixel index; the result does
 * not depend on thread order.  The kept values, d' and (d'/d)^2 p + q, are
 * then evaluated in double with the double H and rounded once to float.
 * Targets that receive nothing are invalid (-1.0f, variance 0).
 * d_prev, p_prev: w*h float; R, t: host (see egosgm_warp_matrix); q > 0.
 * d_pred, p_pred: w*h float (must not alias d_prev / p_prev).  zbuf: w*h
 * uint64 scratch owned by the caller (contents on entry are ignored, on
 * return undefined). */
int warp_disparity(const float* d_prev, const float* p_prev, int w, int h,
                   const double* R, const double* t, double f, double cx, double cy,
                   double baseline, float q, float* d_pred, float* p_pred, uint64_t* zbuf,
                   void* stream);

/* ------------------------------------------------------------------ refine
 * Refinement of the predicted map (Sec. 2.2.2), three passes in order:
 *  1. edge rejection: the paper drops predictions near disparity
 *     discontinuities without stating a test; here a valid prediction is
 *     dropped when a valid pixel of its 3x3 neighbourhood differs from it by
 *     more than edge_tol (float32 comparison; edge_tol < 0 disables it);
 *  2. horizontal one-pixel zoom hole filling (Eq. 7-8): an invalid pixel
 *     whose left and right neighbours are valid with |a - b| < fill_tol gets
 *     d = (a + b)/2 and the mean of the neighbours' variances (the paper
 *     gives no variance rule); the pass reads the result of step 1 only;
 *  3. the same with the vertical neighbours, reading the result of step 2.
 * fill_tol <= 0 disables steps 2 and 3.  Means are correctly rounded floats.
 * d_in, p_in: w*h float (a predicted map, e.g. from warp_disparity);
 * d_out, p_out: w*h float, must not alias the inputs.  workspace,
 * workspace_bytes: unused (kept for the ABI; may be NULL, 0):
 * egosgm_refine_workspace_bytes returns 0, since the kernel keeps its
 * intermediate maps on chip. */
size_t egosgm_refine_workspace_bytes(int w, int h);
int refine_prediction(const float* d_in, const float* p_in, int w, int h, float edge_tol,
                      float fill_tol, float* d_out, float* p_out, void* workspace,
                      size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------ fused prediction
 * warp_disparity followed by refine_prediction (Sec. 2.2 and 2.2.2) in three
 * kernels instead of four: the refinement decodes the warp's z-buffer itself,
 * so the unrefined prediction never goes through memory.  d_pred / p_pred are
 * bit-identical to refine_prediction(warp_disparity(...)) with the same
 * arguments.  d_prev, p_prev: w*h float; R, t, f, cx, cy, baseline, q as
 * warp_disparity; edge_tol, fill_tol as refine_prediction; d_pred, p_pred:
 * w*h float, must not alias the inputs; zbuf: w*h uint64 scratch owned by the
 * caller (contents on entry ignored, on return undefined).  EINVAL on NULL,
 * bad sizes, aliasing, q <= 0 or not finite, or NaN tolerances. */
int predict_disparity(const float* d_prev, const float* p_prev, int w, int h, const double* R,
                      const double* t, double f, double cx, double cy, double baseline, float q,
                      float edge_tol, float fill_tol, float* d_pred, float* p_pred, uint64_t* zbuf,
                      void* stream);

/* ------------------------------------------------------------------ prediction LR check
 * Left-right check of the *prediction* (Sec. 2.4.1; Fig. 4 orders it after
 * the warp and the zoom filling): the previous right disparity map is
 * warped like the left one, with the right camera's motion (for a rectified
 * rig M_R = M_L - (b, 0, 0), so R_R = R and t_R = t + R (b, 0, 0) - (b, 0, 0),
 * then warp_disparity with the same f, cx, cy, b).  A left prediction
 * d >= 0 is kept when d_right at xr = x - floorf(d + 0.5f) is >= 0 and
 * within tol of d (float32); otherwise it becomes (-1, 0), so the pixel is
 * searched over the full range.  d_pred, p_pred: w*h float, in place;
 * d_right: w*h float (negative = none).  EINVAL on NULL, bad sizes or a
 * tol that is negative or NaN; EUNSUPPORTED when w*h >= 2^31. */
int lr_check_prediction(float* d_pred, float* p_pred, const float* d_right, int w, int h, float tol,
                        void* stream);
/* Host helper, no device work: t_right = t + R (b, 0, 0) - (b, 0, 0), the
 * right camera's translation (R_R = R); R row-major 3x3, t and t_right 3
 * doubles, caller-owned.  EINVAL on NULL. */
int egosgm_right_motion(const double* R, const double* t, double baseline, double* t_right);
/* n int16 disparities (e.g. the matcher's disp_right; -1 = none) converted
 * to float, device arrays of n elements.  EINVAL on NULL or n <= 0. */
int disparity_to_float(const int16_t* d, float* out, int n, void* stream);

/* ------------------------------------------------------------------ ego-motion
 * Ego-motion from images (step 1 of Sec. 2, the T of Sec. 2.1 that the warp
 * consumes).  The paper obtains it from a visual odometry algorithm it cites
 * and does not describe; this front end is the library's own direct stereo
 * odometry: with the previous left image I^{k-1}, its disparity map D^{k-1}
 * and the current left image I^k, it minimises the Huber-weighted
 * photometric error sum_p rho(I^k(pi(R P_p + t)) - I^{k-1}(p)) over the
 * pixels with D^{k-1}(p) >= min_disp, P_p = the pixel lifted with
 * Z = f b / d (Eq. 1) and pi the pinhole projection, by Gauss-Newton on an
 * image pyramid, coarse to fine, iters[l] iterations at level l (level 0 =
 * full size; level l halves level l-1 by 2x2 means, disparities by the
 * sample at (2x, 2y) halved; its camera is f/2^l, (c + 0.5)/2^l - 0.5).
 * Updates are left-multiplicative, T <- exp(xi) T, xi = (rho, phi), with the
 * 6x6 system (H + 1e-9 trace(H)/6 I) xi = -g solved by Cholesky in double
 * (no update on a level step with fewer than 16 pixels).  The lift, motion
 * and projection are float32 in the order
 *   Z = fb/d, X = ((x - cx) Z)/f, Y = ((y - cy) Z)/f,
 *   P'_i = ((R_i0 X + R_i1 Y) + R_i2 Z) + t_i,
 *   x' = (f X')/Z' + cx, y' = (f Y')/Z' + cy,
 * and a pixel enters the sum when Z' > 0, 1 <= x' < w_l - 2 and
 * 1 <= y' < h_l - 2; the image and its central-difference gradients are
 * sampled bilinearly there.  The result depends on nothing but the inputs
 * (fixed reduction order).
 * prev_left, cur_left: uint8 w x h, row pitch `pitch` >= w; prev_disp: w*h
 * float (<= 0: no disparity).  f, cx, cy, baseline: the level-0 camera
 * (f, baseline > 0).  pose: DEVICE, 12 doubles (R row-major, then t), the
 * motion M_k = R M_{k-1} + t: on entry the initial guess (e.g. the previous
 * frame's motion), on return (once the stream is synchronised) the estimate.
 * workspace: at least egosgm_vo_workspace_bytes(w, h, prm) bytes.
 * EINVAL on NULL, pitch < w, w < 16, h < 8, w*h >= 2^31, levels outside
 * 1..EGOSGM_VO_MAX_LEVELS, a coarsest level below 16 x 8, iters outside
 * 0..64, huber <= 0, min_disp < 0, non-finite values; EWORKSPACE when the
 * workspace is NULL or too small. */
#define EGOSGM_VO_MAX_LEVELS 6
typedef struct egosgm_vo_params {
    int levels;                       /* pyramid levels (1..6)                      */
    int iters[EGOSGM_VO_MAX_LEVELS];  /* Gauss-Newton iterations per level, finest first */
    float huber;                      /* Huber threshold, intensity units (> 0)     */
    float min_disp;                   /* smallest disparity used, level-0 pixels    */
} egosgm_vo_params;
/* Workspace bytes of estimate_motion / vo_normal_equations; 0 for invalid
 * sizes or parameters.  Host only. */
size_t egosgm_vo_workspace_bytes(int w, int h, const egosgm_vo_params* prm);
int estimate_motion(const uint8_t* prev_left, const uint8_t* cur_left, int w, int h, int pitch,
                    const float* prev_disp, double f, double cx, double cy, double baseline,
                    const egosgm_vo_params* prm, double* pose, void* workspace, size_t workspace_bytes,
                    void* stream);
/* The normal equations of one level at a given pose, for checking: builds
 * the pyramids like estimate_motion, then writes H (36 doubles, row-major,
 * symmetric), g (6), the weighted cost sum rho and the pixel count (44
 * doubles, DEVICE `out`) of level `level` at `pose` (DEVICE, 12 doubles,
 * read only).  EINVAL also when level is outside 0..levels-1 or out is
 * NULL. */
int vo_normal_equations(const uint8_t* prev_left, const uint8_t* cur_left, int w, int h, int pitch,
                        const float* prev_disp, double f, double cx, double cy, double baseline,
                        const egosgm_vo_params* prm, int level, const double* pose, double* out, void* workspace,
                        size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------ SAD check
 * Second outlier filter of Sec. 2.4.1 (the paper names it beside the
 * left-right check, without window or threshold): for every pixel with
 * disp_wta >= 0, the sum of |left(x+i, y+j) - right(x+i-d, y+j)| over
 * i, j in [-radius, radius], coordinates clamped into the image; a pixel
 * whose sum exceeds sad_max is rejected in place like a left-right failure
 * (disp_wta -1, disp_sub -1.0, var_meas 0).  Integer arithmetic.
 * left, right: uint8 images with row pitch >= w; disp_wta, disp_sub,
 * var_meas: w*h, the outputs of sgm_full / sgm_reduced.  radius 0..7,
 * sad_max >= 0; EINVAL otherwise. */
int sad_check(const uint8_t* left, const uint8_t* right, int w, int h, int pitch, int radius,
              int sad_max, int16_t* disp_wta, float* disp_sub, float* var_meas, void* stream);

/* ------------------------------------------------------------------ update
 * Pixel-wise Kalman update (Sec. 2.4, Eq. 10-12), float32 in this order:
 *   K = p/(p + r); d = d_pred + K (z - d_pred); p = (1 - K) p_pred.
 * A prediction is usable when d_pred >= 0 and p_pred > 0; a measurement is
 * valid when z >= 0 and r >= 0.  Prediction only: invalid (-1, 0) unless
 * keep_unmeasured, then (d_pred, p_pred); measurement only: (z, r) (the first
 * frame); neither: (-1, 0).
 * d_pred, p_pred, d_meas (z), r_meas (r): n floats; d_out, p_out: n floats
 * (may alias d_pred / p_pred element for element). */
int kalman_update(const float* d_pred, const float* p_pred, const float* d_meas,
                  const float* r_meas, int n, int keep_unmeasured, float* d_out, float* p_out,
                  void* stream);

/* ------------------------------------------------------------------ batches
 * Batched matching (many stereo pairs of any sizes, each with its own
 * disparity range and either the full range or ragged windows, in one launch
 * per stage), captured once into a HIP graph.  A plan owns the graph; the
 * caller owns every buffer, which must keep its address while the plan lives
 * (the graph bakes the pointers).  The windows' contents may change between
 * runs; each run computes exactly what sgm_full / sgm_reduced computes for
 * each pair alone. */
typedef struct egosgm_pair {
    const uint8_t* left;      /* w x h uint8, row pitch `pitch`                   */
    const uint8_t* right;
    int32_t w, h, pitch;
    int32_t max_disp;         /* this pair's D, 1..256                            */
    const int16_t* lo;        /* ragged windows (as sgm_reduced), or all three    */
    const int16_t* hi;        /* NULL for the full range                          */
    const uint32_t* offsets;
    int16_t* disp_wta;        /* outputs, w*h each, as sgm_full                   */
    float* disp_sub;
    float* var_meas;
    int16_t* disp_right;      /* nullable                                         */
} egosgm_pair;

typedef struct egosgm_plan egosgm_plan;

/* Workspace bytes of a plan over pairs[0..n-1] (host array); 0 if invalid. */
size_t egosgm_plan_workspace_bytes(const egosgm_pair* pairs, int n);

/* Validates the pairs, lays out the workspace (device memory of at least
 * egosgm_plan_workspace_bytes), uploads the per-pair tables (synchronously)
 * and captures census, cost, paths, selection and left-right check of all
 * pairs into one graph.  The path stage is one launch over the scanline
 * tasks of every pair (rows, then columns, then diagonals): one block per
 * 256/G tasks, or, with egosgm_tuning.batch_persistent, a persistent grid of
 * only as many blocks as fit on the device at once whose waves take runs of
 * tasks from work counters in the workspace until none is left.  params:
 * p1, p2, s_max, lr_tol shared by all pairs (max_disp is taken from each
 * pair).  Lanes per scanline (G) and the persistent choice come from the
 * tuning at creation.  *out: the new plan. */
int sgm_plan_create(const egosgm_pair* pairs, int n, const egosgm_sgm_params* params,
                    void* workspace, size_t workspace_bytes, egosgm_plan** out);
/* One launch of the captured graph on `stream`. */
int sgm_plan_run(egosgm_plan* plan, void* stream);
/* The same kernels launched one by one on `stream` (no graph), each stage
 * bracketed by the timing events when timing is enabled. */
int sgm_plan_run_eager(egosgm_plan* plan, void* stream);
/* Changes of one pair of a plan for its next runs (continuous batching over
 * camera streams, Sec. 2: each stream's frame k is matched inside the
 * windows of its own prediction, its first frame over the full range).
 * index: the pair in the plan; active: 0 skips the pair in later runs
 * (its outputs are left as they are); left/right: the pair's images, same
 * shape and pitch as at creation; lo/hi/offsets: new windows as in
 * sgm_reduced, or all three NULL for the full range. */
typedef struct egosgm_pair_update {
    int32_t index;
    int32_t active;
    const uint8_t* left;
    const uint8_t* right;
    const int16_t* lo;
    const int16_t* hi;
    const uint32_t* offsets;
} egosgm_pair_update;

/* Enqueues the changes upd[0..n-1] (host array, read before return) on
 * `stream` as a small kernel, so they apply to the plan's runs enqueued
 * after it on that stream (and are safe inside a captured graph).  The
 * pointers must stay valid until those runs end.  EINVAL: bad index,
 * NULL image, or windows given only in part (nothing is enqueued). */
int sgm_plan_update(egosgm_plan* plan, const egosgm_pair_update* upd, int n, void* stream);
/* Frees the plan (not the buffers).  NULL is accepted. */
int sgm_plan_destroy(egosgm_plan* plan);

/* ------------------------------------------------------------------ tuning
 * Launch shapes and schedules of the path kernels, process-wide (the second
 * piece of state the library keeps; set it before enqueueing work, e.g. from
 * an autotuner).  Results never depend on it.  Defaults: {64, 32, 1, 16, 0, 0}. */
typedef struct egosgm_tuning {
    int32_t full_group;      /* lanes per scanline, full-range kernel: 16, 32, 64             */
    int32_t ragged_group;    /* lanes per scanline, ragged windows through LDS: 16, 32, 64    */
    int32_t ragged_schedule; /* 0: every scanline through LDS rows (work follows the windows);
                                1: the image rows (the longest scanlines) on packed registers
                                   over all disparities, one wave each, branch-free steps;
                                   the rest through LDS rows;
                                2: every scanline as the rows of 1;
                                3: every scanline on registers over its window, one wave
                                   per scanline (window-start moves by lane permutes);
                                4, 5: grouped scanlines: 8 (4) scanlines per wave, 8 (16)
                                   lanes each; a window spanning up to 16 (32) slots is done
                                   by its group, a wider one by the whole wave; the volumes
                                   use an aligned internal layout, and the selection takes
                                   narrow windows 4 lanes per pixel (images whose volumes
                                   would pass 4 GiB at w*h*(D+35) bytes fall back to 1);
                                6, 7: the rows as in 1, the columns and diagonals as in
                                   5 (16 lanes) or 4 (8 lanes), in the same layout;
                                8: grouped scanlines (4 per wave, 16 lanes) whose state
                                   stays in registers: a narrow window as one packed pair
                                   per lane, a wide one over the full range as the
                                   full-range kernel holds it, changes of form through
                                   LDS; same layout                                          */
    int32_t batch_group;     /* lanes per scanline in batched plans (fixed when a plan is
                                created): 16, 32, 64                                           */
    int32_t wide_offsets;    /* LDS scanlines of ragged windows: 0 addresses window words and
                                path costs by 32-bit offsets wherever the image allows it
                                (w*h < 2^27 and the eight path volumes within 4 GiB); 1 uses
                                64-bit addresses everywhere, the form larger images take        */
    int32_t batch_persistent; /* batched plans (fixed when a plan is created): 0 one block per
                                256/G scanline tasks; 1 a persistent path grid                  */
} egosgm_tuning;

int egosgm_set_tuning(const egosgm_tuning* tuning);
int egosgm_get_tuning(egosgm_tuning* tuning);

/* ------------------------------------------------------------------ timing
 * Opt-in profiling aid (library state like the tuning above): while
 * enabled, each stage the library enqueues is bracketed by a pair of HIP
 * events recorded on the caller's stream.  egosgm_timing_read waits for the
 * recorded events, adds the elapsed milliseconds and launch counts per stage
 * into ms[] / count[] (n_stages entries, see egosgm_stage), and forgets them.
 * Not thread-safe with concurrent callers on several host threads. */
typedef enum egosgm_stage {
    EGOSGM_STAGE_CENSUS = 0,  /* census of a pair (one kernel)                   */
    EGOSGM_STAGE_WINDOWS = 1, /* windows: row scan + offsets (two kernels)       */
    EGOSGM_STAGE_COST = 2,    /* matching cost per search slot (one kernel)      */
    EGOSGM_STAGE_PATHS = 3,   /* 8-path aggregation (one kernel)                 */
    EGOSGM_STAGE_SELECT = 4,  /* WTA/subpixel/uncertainty/right map, LR (two kernels) */
    EGOSGM_STAGE_WARP = 5,    /* z-buffer clear, scatter, decode (three kernels) */
    EGOSGM_STAGE_KALMAN = 6,  /* Kalman update (one kernel)                      */
    EGOSGM_STAGE_REFINE = 7,  /* prediction refinement (three kernels)           */
    EGOSGM_STAGE_BATCH_CENSUS = 8,  /* batched plans, run eagerly: census        */
    EGOSGM_STAGE_BATCH_COST = 9,    /* cost                                      */
    EGOSGM_STAGE_BATCH_PATHS = 10,  /* 8-path aggregation                        */
    EGOSGM_STAGE_BATCH_SELECT = 11, /* selection and left-right check            */
    EGOSGM_STAGE_VO = 12,           /* ego-motion estimate (estimate_motion)     */
    EGOSGM_STAGE_COUNT = 13
} egosgm_stage;

int egosgm_timing_enable(int on);
int egosgm_timing_read(double* ms, int* count, int n_stages);

#ifdef __cplusplus
}
#endif
#endif /* EGOSGM_H */
