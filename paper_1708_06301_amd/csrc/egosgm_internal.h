// Internal interface between the C ABI (egosgm_api.hip) and the kernels
// (egosgm_kernels.hip).  Not installed, not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace egosgm {

constexpr int kCensusBits = 62;
constexpr int kMaxDisp = 256;
constexpr int kNumPaths = 8;

// Views of the search windows: either the full range (lo = 0, hi = D-1,
// offset = p*D) or the ragged arrays of sgm_windows_from_prediction.
// Windows are computed in chunks of kWindowChunk pixels of a row; the
// workspace holds one total per chunk.
constexpr int kWindowChunk = 256;

// Census tiles: kCensusTileW x kCensusTileH pixels per 256-thread block,
// kCensusPx pixels per thread (the plan's block counts use the same shape).
constexpr int kCensusPx = 4;
constexpr int kCensusTileW = 64 * kCensusPx;
constexpr int kCensusTileH = 4;

struct Windows {
    const int16_t* lo;       // nullptr: full range
    const int16_t* hi;
    const uint32_t* off;     // w*h+1 entries
    int max_disp;
};

struct SgmLaunch {
    const uint8_t* left;     // images (read by the batched census pass)
    const uint8_t* right;
    int pitch;
    const uint64_t* census_l;
    const uint64_t* census_r;
    int w, h;
    Windows win;
    int p1, p2, s_max, lr_tol;
    int n_paths;             // aggregated directions: 8, or 4 (directions 0-3)
    int full_group;          // lanes per scanline, full-range path kernel (16, 32, 64)
    int ragged_group;        // lanes per scanline, ragged path kernel (16, 32, 64)
    int ragged_schedule;     // 0: all scanlines via LDS, 1: rows on packed registers, 2: all packed,
                             // 3: relative registers, 4/5: grouped scanlines (8/16 lanes, quad layout)
    int wide_offsets;        // 1: LDS scanlines keep 64-bit addresses even where 32-bit offsets fit
    int quad;                // ragged windows in the frame slot layout of the grouped kernels
                             // (schedules 4-8): lanes per scanline G (frames of 2G slots unless
                             // frame_pairs), or 0
    int frame_pairs;         // 1: narrow frames of 16 slots on even bases (schedule 8);
                             // 0: frames of 2G slots on bases that are multiples of 4
    uint8_t* cost;           // matching cost per search slot
    uint32_t* key_r;         // w*h right-map keys (S << 9 | d), cleared by the census pass
    uint64_t* meta;          // w*h packed windows (offset | lo << 32 | width << 48), written by
                             // the cost pass for ragged windows, read by the path kernels
    uint64_t* frame;         // w*h frame words of the frame layout (frame offset | base << 32 |
                             // form << 48 | span << 50), written by the frame cost pass
    uint8_t* vol;            // 8 path volumes, direction-major
    size_t vol_stride;       // entries per direction block (w*h*D)
    int16_t* disp_wta;
    float* disp_sub;
    float* var_meas;
    int16_t* disp_right;     // nullable
    uint16_t* agg;           // nullable (debug)
    int16_t* wta_raw;        // nullable (debug)
    int active;              // batched launches: 0 skips the pair
};

// One descriptor change of a plan (sgm_plan_update): the pair's active flag,
// images and windows (lo == nullptr: full range).
struct PlanPatch {
    int index, active;
    const uint8_t* left;
    const uint8_t* right;
    const int16_t* lo;
    const int16_t* hi;
    const uint32_t* off;
};
constexpr int kPatchBatch = 16;
struct PlanPatches {
    PlanPatch p[kPatchBatch];
    int n;
};

// Work lists of the persistent batched path kernel.
constexpr int kBatchShards = 32;
constexpr int kBatchShardStride = 256;

// Device tables of a batched launch (all pointers into device memory),
// plus the host-side launch sizes.
struct BatchTables {
    const SgmLaunch* pairs;     // n descriptors
    const int* census_prefix;   // n+1: census tiles per pair
    const int* seg_prefix;      // n+1: 64-pixel row segments per pair (cost, select)
    const int* pix_prefix;      // n+1: pixels per pair
    const int* task_start;      // n_ranges: first global scanline task of each range
    const int* task_pair;       // n_ranges: pair of each range
    const int* task_local;      // n_ranges: first local task of each range
    const int* task_count;      // n_ranges: real tasks of each range (the rest is padding)
    int n, n_ranges, n_tasks;
    unsigned* work;             // kBatchShards work counters, kBatchShardStride bytes apart
                                // (reset by the cost pass)
    int group;                  // lanes per scanline of the path kernel (16, 32, 64)
    int persistent;             // 1: persistent path grid over work counters
    int n_paths;                // 8, or 4 (no diagonal tasks, 4 volumes summed)
    int host_census_blocks, host_seg_blocks, host_pixels;
    int host_path_blocks;       // persistent path grid: blocks resident at once (at most)
};

// Blocks of the persistent batched path kernel: as many as fit on the
// current device at once, at most one per 4 waves of tasks (0 on failure).
int batch_path_blocks(int group, int max_disp, int n_tasks);

hipError_t launch_sgm_batch(const BatchTables& t, int max_disp, hipStream_t s);
hipError_t launch_plan_patch(SgmLaunch* pairs, const PlanPatches& p, hipStream_t s);
// stage 0 census, 1 cost, 2 paths, 3 selection, 4 left-right check
hipError_t launch_batch_stage(const BatchTables& t, int max_disp, int stage, hipStream_t s);
hipError_t launch_census(const uint8_t* img, int w, int h, int pitch, uint64_t* out,
                         hipStream_t s);
hipError_t launch_census_pair(const uint8_t* left, const uint8_t* right, int w, int h,
                              int pitch, uint64_t* out_l, uint64_t* out_r, uint32_t* clear,
                              hipStream_t s);
hipError_t launch_sgm_cost(const SgmLaunch& a, hipStream_t s);
hipError_t launch_sgm_paths(const SgmLaunch& a, hipStream_t s);
hipError_t launch_sgm_select(const SgmLaunch& a, hipStream_t s);
hipError_t launch_copy_slots(const SgmLaunch& a, const uint8_t* src, uint8_t* dst, hipStream_t s);
// quad-layout volumes (stride src_stride) into the public ragged layout (stride dst_stride)
hipError_t launch_copy_quad_slots(const SgmLaunch& a, const uint8_t* src, size_t src_stride, uint8_t* dst,
                                  size_t dst_stride, int nvol, hipStream_t s);
// bytes of one quad-layout volume for w*h pixels and range D (0 if it does not fit 32-bit offsets)
size_t quad_volume_bytes(int w, int h, int D);
hipError_t launch_windows(const float* d_pred, const float* p_pred, int w, int h,
                          float k_sigma, int r_fixed, int r_min, int r_max, int max_disp,
                          int16_t* lo, int16_t* hi, uint32_t* off, uint32_t* chunk_tot,
                          hipStream_t s);
hipError_t launch_warp(const float* d_prev, const float* p_prev, int w, int h, const float* H,
                       const double* Hd, double q, float* d_pred, float* p_pred,
                       unsigned long long* zbuf, hipStream_t s);
hipError_t launch_warp_scatter(const float* d_prev, int w, int h, const float* H,
                               unsigned long long* zbuf, hipStream_t s);
hipError_t launch_refine_from_zbuf(const unsigned long long* zbuf, const float* d_prev,
                                   const float* p_prev, int w, int h, const double* Hd, double q,
                                   float edge_tol, float fill_tol, float* d_out, float* p_out,
                                   hipStream_t s);
hipError_t launch_refine(const float* d_in, const float* p_in, int w, int h, float edge_tol,
                         float fill_tol, float* d_out, float* p_out, hipStream_t s);
hipError_t launch_sad_check(const uint8_t* left, const uint8_t* right, int w, int h, int pitch,
                            int radius, int sad_max, int16_t* disp_wta, float* disp_sub,
                            float* var_meas, hipStream_t s);
hipError_t launch_lr_check_prediction(float* d_pred, float* p_pred, const float* d_right, int w,
                                      int h, float tol, hipStream_t s);
hipError_t launch_disparity_to_float(const int16_t* d, float* out, int n, hipStream_t s);
hipError_t launch_kalman(const float* d_pred, const float* p_pred, const float* z,
                         const float* r, int n, int keep, float* d_out, float* p_out,
                         hipStream_t s);

// Ego-motion front end (egosgm_vo.hip): one estimate, or the normal
// equations of one level at the pose given (only_level >= 0, written to out).
constexpr int kVoMaxLevels = 6;
struct VoArgs {
    const uint8_t* prev;      // previous left image
    const uint8_t* cur;       // current left image
    int w, h, pitch;
    const float* prev_disp;   // previous disparity map (w*h, <= 0 invalid)
    double f, cx, cy, baseline;
    int levels;
    int iters[kVoMaxLevels];  // per level, finest first
    float huber, min_disp;
    double* pose;             // 12 doubles: R row-major, t (in: guess, out: estimate)
    double* out;              // only_level >= 0: H (36), g (6), cost, count
    int only_level;
    void* workspace;
};
size_t vo_workspace_bytes(int w, int h, int levels);
hipError_t launch_vo(const VoArgs& v, hipStream_t s);

}  // namespace egosgm
