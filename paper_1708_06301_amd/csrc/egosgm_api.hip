// C ABI of libegosgm (declared in include/egosgm.h): host-side validation,
// workspace layout, the disparity-space motion matrix, and kernel launches.
#include "egosgm.h"
#include "egosgm_internal.h"

#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

using namespace egosgm;

namespace {

// ---------------------------------------------------------------- timing
struct StageEvents {
    int stage;
    hipEvent_t start, stop;
};

struct Timing {
    std::mutex mu;
    bool on = false;
    std::vector<StageEvents> pending;
    std::vector<hipEvent_t> pool;
};

Timing& timing() {
    static Timing t;
    return t;
}

hipEvent_t take_event(Timing& t) {
    if (!t.pool.empty()) {
        hipEvent_t e = t.pool.back();
        t.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets the launches made by `fn` with events when timing is enabled.
template <class F>
hipError_t timed(int stage, hipStream_t s, F&& fn) {
    Timing& t = timing();
    if (!t.on) return fn();
    std::lock_guard<std::mutex> g(t.mu);
    StageEvents ev{stage, take_event(t), take_event(t)};
    if (!ev.start || !ev.stop) return fn();
    (void)hipEventRecord(ev.start, s);
    const hipError_t e = fn();
    (void)hipEventRecord(ev.stop, s);
    t.pending.push_back(ev);
    return e;
}

// Launch-shape choices (set by egosgm_set_tuning; read at every launch).
egosgm_tuning g_tuning = {64, 64, 0};
std::mutex g_tuning_mu;

constexpr size_t kAlign = 256;
constexpr int kMaxWidth = 4064;  // the epilogue keeps 16 bytes per column of a row in LDS

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Workspace: census codes of both images, right-map keys, the cost volume
// and the eight path volumes (all sized for the full range).
struct WsLayout {
    size_t census_l, census_r, key_r, cost, vol, vol_stride, total;
};

bool ws_layout(int w, int h, int D, WsLayout& L) {
    if (w <= 0 || h <= 0 || D < 1 || D > kMaxDisp) return false;
    const size_t n = (size_t)w * (size_t)h;
    L.vol_stride = n * (size_t)D;
    L.census_l = 0;
    L.census_r = L.census_l + align_up(n * sizeof(uint64_t));
    L.key_r = L.census_r + align_up(n * sizeof(uint64_t));
    L.cost = L.key_r + align_up(n * sizeof(uint32_t));
    L.vol = L.cost + align_up(L.vol_stride);
    L.total = L.vol + align_up((size_t)kNumPaths * L.vol_stride);
    return true;
}

int check_shape(int w, int h, int D) {
    if (w <= 0 || h <= 0 || D < 1 || D > kMaxDisp) return EGOSGM_EINVAL;
    if (w > kMaxWidth) return EGOSGM_EUNSUPPORTED;
    if ((unsigned long long)w * (unsigned long long)h * (unsigned long long)D >= (1ull << 32))
        return EGOSGM_EUNSUPPORTED;  // ragged offsets are uint32
    return EGOSGM_OK;
}

int check_params(const egosgm_sgm_params* prm) {
    if (!prm) return EGOSGM_EINVAL;
    if (prm->p1 < 0 || prm->p2 < prm->p1 || prm->p2 > 255 - kCensusBits) return EGOSGM_EINVAL;
    if (prm->s_max < 0) return EGOSGM_EINVAL;
    return EGOSGM_OK;
}

int run_sgm(const uint8_t* left, const uint8_t* right, int w, int h, int pitch, const Windows& win,
            const egosgm_sgm_params* prm, int16_t* disp_wta, float* disp_sub, float* var_meas,
            int16_t* disp_right, const egosgm_debug* dbg, void* ws, size_t ws_bytes,
            hipStream_t s) {
    if (!left || !right || !disp_wta || !disp_sub || !var_meas) return EGOSGM_EINVAL;
    int rc = check_params(prm);
    if (rc) return rc;
    rc = check_shape(w, h, prm->max_disp);
    if (rc) return rc;
    if (pitch < w) return EGOSGM_EINVAL;
    WsLayout L;
    ws_layout(w, h, prm->max_disp, L);
    if (!ws || ws_bytes < L.total) return EGOSGM_EWORKSPACE;
    uint8_t* base = static_cast<uint8_t*>(ws);

    SgmLaunch a;
    a.census_l = reinterpret_cast<uint64_t*>(base + L.census_l);
    a.census_r = reinterpret_cast<uint64_t*>(base + L.census_r);
    a.w = w;
    a.h = h;
    a.win = win;
    a.p1 = prm->p1;
    a.p2 = prm->p2;
    a.s_max = prm->s_max;
    a.lr_tol = prm->lr_tol;
    {
        std::lock_guard<std::mutex> g(g_tuning_mu);
        a.full_group = g_tuning.full_group;
        a.ragged_group = g_tuning.ragged_group;
        a.ragged_schedule = g_tuning.ragged_schedule;
    }
    a.cost = base + L.cost;
    a.key_r = reinterpret_cast<uint32_t*>(base + L.key_r);
    a.vol = base + L.vol;
    a.vol_stride = L.vol_stride;
    a.disp_wta = disp_wta;
    a.disp_sub = disp_sub;
    a.var_meas = var_meas;
    a.disp_right = disp_right;
    a.agg = dbg ? dbg->agg : nullptr;
    a.wta_raw = dbg ? dbg->wta_raw : nullptr;

    const size_t n = (size_t)w * h;
    if (timed(EGOSGM_STAGE_CENSUS, s, [&] {
            return launch_census_pair(left, right, w, h, pitch, const_cast<uint64_t*>(a.census_l),
                                      const_cast<uint64_t*>(a.census_r), a.key_r, s);
        }) != hipSuccess)
        return EGOSGM_EDEVICE;
    if (timed(EGOSGM_STAGE_COST, s, [&] { return launch_sgm_cost(a, s); }) != hipSuccess)
        return EGOSGM_EDEVICE;
    if (timed(EGOSGM_STAGE_PATHS, s, [&] { return launch_sgm_paths(a, s); }) != hipSuccess)
        return EGOSGM_EDEVICE;
    if (timed(EGOSGM_STAGE_SELECT, s, [&] { return launch_sgm_select(a, s); }) != hipSuccess)
        return EGOSGM_EDEVICE;
    if (dbg) {
        if (dbg->census_left &&
            hipMemcpyAsync(dbg->census_left, a.census_l, n * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return EGOSGM_EDEVICE;
        if (dbg->census_right &&
            hipMemcpyAsync(dbg->census_right, a.census_r, n * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return EGOSGM_EDEVICE;
        if (dbg->paths &&
            hipMemcpyAsync(dbg->paths, a.vol, kNumPaths * a.vol_stride, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return EGOSGM_EDEVICE;
        if (dbg->cost && launch_copy_slots(a, a.cost, dbg->cost, s) != hipSuccess)
            return EGOSGM_EDEVICE;
    }
    return EGOSGM_OK;
}

}  // namespace

extern "C" {

int egosgm_abi_version(void) { return EGOSGM_ABI_VERSION; }

const char* egosgm_status_string(int status) {
    switch (status) {
        case EGOSGM_OK: return "ok";
        case EGOSGM_EINVAL: return "invalid argument";
        case EGOSGM_EWORKSPACE: return "workspace missing or too small";
        case EGOSGM_EDEVICE: return "HIP launch or copy failed";
        case EGOSGM_EUNSUPPORTED: return "unsupported size or option";
        default: return "unknown status";
    }
}

int egosgm_census(const uint8_t* img, int w, int h, int pitch, uint64_t* out, void* stream) {
    if (!img || !out || w <= 0 || h <= 0 || pitch < w) return EGOSGM_EINVAL;
    return launch_census(img, w, h, pitch, out, static_cast<hipStream_t>(stream)) == hipSuccess
               ? EGOSGM_OK
               : EGOSGM_EDEVICE;
}

size_t egosgm_sgm_workspace_bytes(int w, int h, int max_disp) {
    WsLayout L;
    return ws_layout(w, h, max_disp, L) ? L.total : 0;
}

int sgm_full(const uint8_t* left, const uint8_t* right, int w, int h, int pitch,
             const egosgm_sgm_params* params, int16_t* disp_wta, float* disp_sub,
             float* var_meas, int16_t* disp_right, const egosgm_debug* debug, void* workspace,
             size_t workspace_bytes, void* stream) {
    if (!params) return EGOSGM_EINVAL;
    Windows win{nullptr, nullptr, nullptr, params->max_disp};
    return run_sgm(left, right, w, h, pitch, win, params, disp_wta, disp_sub, var_meas,
                   disp_right, debug, workspace, workspace_bytes,
                   static_cast<hipStream_t>(stream));
}

int sgm_reduced(const uint8_t* left, const uint8_t* right, int w, int h, int pitch,
                const int16_t* lo, const int16_t* hi, const uint32_t* offsets,
                const egosgm_sgm_params* params, int16_t* disp_wta, float* disp_sub,
                float* var_meas, int16_t* disp_right, const egosgm_debug* debug,
                void* workspace, size_t workspace_bytes, void* stream) {
    if (!params || !lo || !hi || !offsets) return EGOSGM_EINVAL;
    Windows win{lo, hi, offsets, params->max_disp};
    return run_sgm(left, right, w, h, pitch, win, params, disp_wta, disp_sub, var_meas,
                   disp_right, debug, workspace, workspace_bytes,
                   static_cast<hipStream_t>(stream));
}

size_t egosgm_windows_workspace_bytes(int w, int h) {
    if (w <= 0 || h <= 0) return 0;
    return align_up((size_t)h * sizeof(uint32_t));
}

int sgm_windows_from_prediction(const float* d_pred, const float* p_pred, int w, int h,
                                float k_sigma, int r_fixed, int r_min, int r_max, int max_disp,
                                int16_t* lo, int16_t* hi, uint32_t* offsets, void* workspace,
                                size_t workspace_bytes, void* stream) {
    if (!d_pred || !lo || !hi || !offsets) return EGOSGM_EINVAL;
    if (r_fixed < 0 && !p_pred) return EGOSGM_EINVAL;
    if (r_min < 0 || r_max < r_min || !(k_sigma >= 0.0f)) return EGOSGM_EINVAL;
    const int rc = check_shape(w, h, max_disp);
    if (rc) return rc;
    if (!workspace || workspace_bytes < egosgm_windows_workspace_bytes(w, h))
        return EGOSGM_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    return timed(EGOSGM_STAGE_WINDOWS, s, [&] {
               return launch_windows(d_pred, p_pred, w, h, k_sigma, r_fixed, r_min, r_max,
                                     max_disp, lo, hi, offsets,
                                     static_cast<uint32_t*>(workspace), s);
           }) == hipSuccess
               ? EGOSGM_OK
               : EGOSGM_EDEVICE;
}

}  // extern "C"

namespace {

// H = Gamma T Gamma^-1 in closed form.  With A = T Gamma^-1, whose rows are
// (R_i0/f, R_i1/f, t_i/(f b), R_i2 - (R_i0 cx + R_i1 cy)/f) for i < 3 and
// (0, 0, 1/(f b), 0) for i = 3, the product Gamma A gives
//   row 0 = f A_0 + cx A_2,  row 1 = f A_1 + cy A_2,  row 2 = (0,0,1,0),
//   row 3 = A_2.
int warp_matrix_d(const double* R, const double* t, double f, double cx, double cy,
                  double baseline, double* Hd) {
    if (!R || !t || !Hd || !(f > 0.0) || !(baseline > 0.0)) return EGOSGM_EINVAL;
    if (!std::isfinite(f) || !std::isfinite(cx) || !std::isfinite(cy) || !std::isfinite(baseline))
        return EGOSGM_EINVAL;
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(R[i])) return EGOSGM_EINVAL;
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(t[i])) return EGOSGM_EINVAL;
    const double fb = f * baseline;
    double A[3][4];
    for (int i = 0; i < 3; ++i) {
        A[i][0] = R[3 * i + 0] / f;
        A[i][1] = R[3 * i + 1] / f;
        A[i][2] = t[i] / fb;
        A[i][3] = R[3 * i + 2] - (R[3 * i + 0] * cx + R[3 * i + 1] * cy) / f;
    }
    for (int j = 0; j < 4; ++j) {
        Hd[0 + j] = f * A[0][j] + cx * A[2][j];
        Hd[4 + j] = f * A[1][j] + cy * A[2][j];
        Hd[8 + j] = (j == 2) ? 1.0 : 0.0;
        Hd[12 + j] = A[2][j];
    }
    return EGOSGM_OK;
}

}  // namespace

extern "C" {

int egosgm_warp_matrix(const double* R, const double* t, double f, double cx, double cy,
                       double baseline, float* H) {
    if (!H) return EGOSGM_EINVAL;
    double Hd[16];
    const int rc = warp_matrix_d(R, t, f, cx, cy, baseline, Hd);
    if (rc) return rc;
    for (int i = 0; i < 16; ++i) H[i] = (float)Hd[i];
    return EGOSGM_OK;
}

int warp_disparity(const float* d_prev, const float* p_prev, int w, int h, const double* R,
                   const double* t, double f, double cx, double cy, double baseline, float q,
                   float* d_pred, float* p_pred, uint64_t* zbuf, void* stream) {
    if (!d_prev || !p_prev || !d_pred || !p_pred || !zbuf) return EGOSGM_EINVAL;
    if (w <= 0 || h <= 0 || (long long)w * h >= (1ll << 31)) return EGOSGM_EINVAL;
    if (!(q > 0.0f) || !std::isfinite(q)) return EGOSGM_EINVAL;
    double Hd[16];
    float H[16];
    const int rc = warp_matrix_d(R, t, f, cx, cy, baseline, Hd);
    if (rc) return rc;
    for (int i = 0; i < 16; ++i) H[i] = (float)Hd[i];
    hipStream_t s = static_cast<hipStream_t>(stream);
    return timed(EGOSGM_STAGE_WARP, s, [&] {
               return launch_warp(d_prev, p_prev, w, h, H, Hd, (double)q, d_pred, p_pred,
                                  reinterpret_cast<unsigned long long*>(zbuf), s);
           }) == hipSuccess
               ? EGOSGM_OK
               : EGOSGM_EDEVICE;
}

size_t egosgm_refine_workspace_bytes(int w, int h) {
    if (w <= 0 || h <= 0) return 0;
    return align_up((size_t)w * h * 2 * sizeof(float));
}

int refine_prediction(const float* d_in, const float* p_in, int w, int h, float edge_tol,
                      float fill_tol, float* d_out, float* p_out, void* workspace,
                      size_t workspace_bytes, void* stream) {
    if (!d_in || !p_in || !d_out || !p_out) return EGOSGM_EINVAL;
    if (w <= 0 || h <= 0 || (long long)w * h >= (1ll << 31)) return EGOSGM_EINVAL;
    if (std::isnan(edge_tol) || std::isnan(fill_tol)) return EGOSGM_EINVAL;
    if (d_out == d_in || p_out == p_in || d_out == p_in || p_out == d_in) return EGOSGM_EINVAL;
    if (!workspace || workspace_bytes < egosgm_refine_workspace_bytes(w, h)) return EGOSGM_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    return timed(EGOSGM_STAGE_REFINE, s, [&] {
               return launch_refine(d_in, p_in, w, h, edge_tol, fill_tol, d_out, p_out,
                                    static_cast<float*>(workspace), s);
           }) == hipSuccess
               ? EGOSGM_OK
               : EGOSGM_EDEVICE;
}

int kalman_update(const float* d_pred, const float* p_pred, const float* d_meas,
                  const float* r_meas, int n, int keep_unmeasured, float* d_out, float* p_out,
                  void* stream) {
    if (!d_pred || !p_pred || !d_meas || !r_meas || !d_out || !p_out || n < 0)
        return EGOSGM_EINVAL;
    if (n == 0) return EGOSGM_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    return timed(EGOSGM_STAGE_KALMAN, s, [&] {
               return launch_kalman(d_pred, p_pred, d_meas, r_meas, n, keep_unmeasured, d_out,
                                    p_out, s);
           }) == hipSuccess
               ? EGOSGM_OK
               : EGOSGM_EDEVICE;
}

int egosgm_set_tuning(const egosgm_tuning* t) {
    if (!t) return EGOSGM_EINVAL;
    auto ok = [](int g) { return g == 16 || g == 32 || g == 64; };
    if (!ok(t->full_group) || !ok(t->ragged_group) || t->ragged_schedule < 0 || t->ragged_schedule > 2)
        return EGOSGM_EINVAL;
    std::lock_guard<std::mutex> g(g_tuning_mu);
    g_tuning = *t;
    return EGOSGM_OK;
}

int egosgm_get_tuning(egosgm_tuning* t) {
    if (!t) return EGOSGM_EINVAL;
    std::lock_guard<std::mutex> g(g_tuning_mu);
    *t = g_tuning;
    return EGOSGM_OK;
}

int egosgm_timing_enable(int on) {
    Timing& t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    t.on = on != 0;
    return EGOSGM_OK;
}

int egosgm_timing_read(double* ms, int* count, int n_stages) {
    if (n_stages < 0 || (n_stages > 0 && (!ms || !count))) return EGOSGM_EINVAL;
    Timing& t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    int rc = EGOSGM_OK;
    for (const StageEvents& ev : t.pending) {
        float e = 0.0f;
        if (hipEventSynchronize(ev.stop) != hipSuccess ||
            hipEventElapsedTime(&e, ev.start, ev.stop) != hipSuccess) {
            rc = EGOSGM_EDEVICE;
        } else if (ev.stage < n_stages) {
            ms[ev.stage] += (double)e;
            count[ev.stage] += 1;
        }
        t.pool.push_back(ev.start);
        t.pool.push_back(ev.stop);
    }
    t.pending.clear();
    return rc;
}

}  // extern "C"
