// C ABI of libegosgm (declared in include/egosgm.h): host-side validation,
// workspace layout, the disparity-space motion matrix, and kernel launches.
#include "egosgm.h"
#include "egosgm_internal.h"

#include <cmath>
#include <cstring>
#include <algorithm>
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
    // no system-scope fence: the host reads only the timestamps, and a fence
    // would write back the L2 after every timed stage and inflate its time
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
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

// Scratch of sgm_windows_from_prediction_noalloc: the per-chunk totals of
// the offsets scan (one uint32 per kWindowChunk pixels of a row), in a
// file-scope device array instead of a caller workspace.  Every GPU the
// library runs on holds its own copy until the process ends.  In host code
// `scratch` only names the symbol: its device address on each GPU comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) uint32_t scratch[EGOSGM_NOALLOC_WINDOW_CHUNKS];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch_ptr[kMaxDevices] = {};

hipError_t window_scratch(uint32_t** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<uint32_t*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// Launch-shape choices (set by egosgm_set_tuning; read at every launch).
egosgm_tuning g_tuning = {64, 32, 1, 16, 0, 0};
std::mutex g_tuning_mu;

constexpr size_t kAlign = 256;
constexpr int kMaxWidth = 4064;  // the epilogue keeps 16 bytes per column of a row in LDS

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Workspace: census codes of both images, right-map keys, the cost volume
// and the eight path volumes (all sized for the full range).  A volume holds
// either the ragged layout (w*h*D bytes at most, stride vol_stride) or the
// quad layout of the grouped kernels (stride vol_stride_q; 0 when its
// offsets would not fit 32 bits, and those kernels are then not used).
struct WsLayout {
    size_t census_l, census_r, key_r, meta, frame, cost, vol, vol_stride, vol_stride_q, total;
};

bool ws_layout(int w, int h, int D, WsLayout& L) {
    if (w <= 0 || h <= 0 || D < 1 || D > kMaxDisp) return false;
    const size_t n = (size_t)w * (size_t)h;
    L.vol_stride = n * (size_t)D;
    L.vol_stride_q = quad_volume_bytes(w, h, D);
    const size_t vbytes = std::max(L.vol_stride, L.vol_stride_q);
    L.census_l = 0;
    L.census_r = L.census_l + align_up(n * sizeof(uint64_t));
    L.key_r = L.census_r + align_up(n * sizeof(uint64_t));
    L.meta = L.key_r + align_up(n * sizeof(uint32_t));
    L.frame = L.meta + align_up(n * sizeof(uint64_t));
    L.cost = L.frame + align_up(n * sizeof(uint64_t));
    L.vol = L.cost + align_up(vbytes);
    L.total = L.vol + align_up((size_t)kNumPaths * vbytes);
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
    if (prm->n_paths != 0 && prm->n_paths != 4 && prm->n_paths != 8) return EGOSGM_EINVAL;
    if (prm->census_ready != 0 && prm->census_ready != 1) return EGOSGM_EINVAL;
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
    a.left = left;
    a.right = right;
    a.pitch = pitch;
    a.census_l = reinterpret_cast<uint64_t*>(base + L.census_l);
    a.census_r = reinterpret_cast<uint64_t*>(base + L.census_r);
    a.w = w;
    a.h = h;
    a.win = win;
    a.p1 = prm->p1;
    a.p2 = prm->p2;
    a.s_max = prm->s_max;
    a.lr_tol = prm->lr_tol;
    a.n_paths = prm->n_paths == 4 ? 4 : 8;
    {
        std::lock_guard<std::mutex> g(g_tuning_mu);
        a.full_group = g_tuning.full_group;
        a.ragged_group = g_tuning.ragged_group;
        a.ragged_schedule = g_tuning.ragged_schedule;
        a.wide_offsets = g_tuning.wide_offsets;
    }
    a.cost = base + L.cost;
    a.key_r = reinterpret_cast<uint32_t*>(base + L.key_r);
    a.meta = reinterpret_cast<uint64_t*>(base + L.meta);
    a.frame = reinterpret_cast<uint64_t*>(base + L.frame);
    a.vol = base + L.vol;
    // grouped scanlines (schedules 4-8) need the frame layout; where its
    // offsets would not fit 32 bits the rows-on-registers schedule runs instead
    a.quad = 0;
    a.frame_pairs = 0;
    if (win.lo != nullptr && a.ragged_schedule >= 4) {
        if (L.vol_stride_q != 0) {
            a.quad = (a.ragged_schedule == 5 || a.ragged_schedule == 6 || a.ragged_schedule == 8) ? 16 : 8;
            a.frame_pairs = a.ragged_schedule == 8 ? 1 : 0;
        } else {
            a.ragged_schedule = 1;
        }
    }
    a.vol_stride = a.quad ? L.vol_stride_q : L.vol_stride;
    a.disp_wta = disp_wta;
    a.disp_sub = disp_sub;
    a.var_meas = var_meas;
    a.disp_right = disp_right;
    a.agg = dbg ? dbg->agg : nullptr;
    a.wta_raw = dbg ? dbg->wta_raw : nullptr;

    const size_t n = (size_t)w * h;
    if (!prm->census_ready && timed(EGOSGM_STAGE_CENSUS, s, [&] {
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
        if (a.quad) {
            if (dbg->paths && launch_copy_quad_slots(a, a.vol, a.vol_stride, dbg->paths, L.vol_stride,
                                                     a.n_paths, s) != hipSuccess)
                return EGOSGM_EDEVICE;
            if (dbg->cost && launch_copy_quad_slots(a, a.cost, 0, dbg->cost, 0, 1, s) != hipSuccess)
                return EGOSGM_EDEVICE;
        } else {
            if (dbg->paths && hipMemcpyAsync(dbg->paths, a.vol, kNumPaths * a.vol_stride,
                                             hipMemcpyDeviceToDevice, s) != hipSuccess)
                return EGOSGM_EDEVICE;
            if (dbg->cost && launch_copy_slots(a, a.cost, dbg->cost, s) != hipSuccess)
                return EGOSGM_EDEVICE;
        }
    }
    return EGOSGM_OK;
}

}  // namespace

// ---------------------------------------------------------------- plans
struct egosgm_plan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int n = 0;
    int max_disp = 0;
    BatchTables tables{};
    SgmLaunch* pairs_dev = nullptr;       // device descriptors (in the workspace)
    std::vector<egosgm_pair> shape;       // creation-time pairs (shapes, outputs)
};

namespace {

size_t pair_bytes(const egosgm_pair& p) {
    WsLayout L;
    ws_layout(p.w, p.h, p.max_disp, L);
    return L.total;
}

int check_pair(const egosgm_pair& p) {
    if (!p.left || !p.right || !p.disp_wta || !p.disp_sub || !p.var_meas) return EGOSGM_EINVAL;
    const int rc = check_shape(p.w, p.h, p.max_disp);
    if (rc) return rc;
    if (p.pitch < p.w) return EGOSGM_EINVAL;
    if ((p.lo == nullptr) != (p.hi == nullptr) || (p.lo == nullptr) != (p.offsets == nullptr))
        return EGOSGM_EINVAL;
    return EGOSGM_OK;
}

struct PlanLayout {
    size_t pairs, census_prefix, seg_prefix, pix_prefix, task_start, task_pair, task_local, task_count, work;
    size_t data, total;
    int n_ranges;
};

PlanLayout plan_layout(const egosgm_pair* pairs, int n) {
    PlanLayout P;
    P.n_ranges = 3 * n;
    size_t o = 0;
    P.pairs = o;         o += align_up((size_t)n * sizeof(SgmLaunch));
    P.census_prefix = o; o += align_up((size_t)(n + 1) * sizeof(int));
    P.seg_prefix = o;    o += align_up((size_t)(n + 1) * sizeof(int));
    P.pix_prefix = o;    o += align_up((size_t)(n + 1) * sizeof(int));
    P.task_start = o;    o += align_up((size_t)P.n_ranges * sizeof(int));
    P.task_pair = o;     o += align_up((size_t)P.n_ranges * sizeof(int));
    P.task_local = o;    o += align_up((size_t)P.n_ranges * sizeof(int));
    P.task_count = o;    o += align_up((size_t)P.n_ranges * sizeof(int));
    P.work = o;          o += align_up((size_t)kBatchShards * kBatchShardStride);
    P.data = o;
    for (int i = 0; i < n; ++i) o += pair_bytes(pairs[i]);
    P.total = o;
    return P;
}

}  // namespace

extern "C" {

size_t egosgm_plan_workspace_bytes(const egosgm_pair* pairs, int n) {
    if (!pairs || n <= 0) return 0;
    for (int i = 0; i < n; ++i)
        if (check_pair(pairs[i])) return 0;
    return plan_layout(pairs, n).total;
}

int sgm_plan_create(const egosgm_pair* pairs, int n, const egosgm_sgm_params* params,
                    void* workspace, size_t workspace_bytes, egosgm_plan** out) {
    if (!pairs || n <= 0 || !out) return EGOSGM_EINVAL;
    *out = nullptr;
    if (!params || params->census_ready) return EGOSGM_EINVAL;   // a plan computes its census itself
    egosgm_sgm_params prm = *params;
    int max_disp = 1;
    for (int i = 0; i < n; ++i) {
        const int rc = check_pair(pairs[i]);
        if (rc) return rc;
        max_disp = std::max(max_disp, pairs[i].max_disp);
    }
    prm.max_disp = max_disp;
    int rc = check_params(&prm);
    if (rc) return rc;
    const PlanLayout P = plan_layout(pairs, n);
    if (!workspace || workspace_bytes < P.total) return EGOSGM_EWORKSPACE;
    uint8_t* base = static_cast<uint8_t*>(workspace);

    std::vector<SgmLaunch> desc(n);
    std::vector<int> cen(n + 1, 0), seg(n + 1, 0), pix(n + 1, 0);
    std::vector<int> ts(P.n_ranges), tp(P.n_ranges), tl(P.n_ranges), tc(P.n_ranges);
    size_t o = P.data;
    long long tasks = 0, segs = 0, tiles = 0, pixels = 0;
    for (int i = 0; i < n; ++i) {
        const egosgm_pair& q = pairs[i];
        WsLayout L;
        ws_layout(q.w, q.h, q.max_disp, L);
        SgmLaunch& a = desc[i];
        a = SgmLaunch{};
        a.left = q.left;
        a.right = q.right;
        a.pitch = q.pitch;
        a.census_l = reinterpret_cast<uint64_t*>(base + o + L.census_l);
        a.census_r = reinterpret_cast<uint64_t*>(base + o + L.census_r);
        a.key_r = reinterpret_cast<uint32_t*>(base + o + L.key_r);
        a.meta = reinterpret_cast<uint64_t*>(base + o + L.meta);
        a.cost = base + o + L.cost;
        a.vol = base + o + L.vol;
        a.vol_stride = L.vol_stride;
        a.w = q.w;
        a.h = q.h;
        a.win = Windows{q.lo, q.hi, q.offsets, q.max_disp};
        a.p1 = prm.p1;
        a.p2 = prm.p2;
        a.s_max = prm.s_max;
        a.lr_tol = prm.lr_tol;
        a.n_paths = prm.n_paths == 4 ? 4 : 8;
        a.disp_wta = q.disp_wta;
        a.disp_sub = q.disp_sub;
        a.var_meas = q.var_meas;
        a.disp_right = q.disp_right;
        a.active = 1;
        o += L.total;
        cen[i] = (int)tiles;
        seg[i] = (int)segs;
        pix[i] = (int)pixels;
        tiles += (long long)((q.w + kCensusTileW - 1) / kCensusTileW) * ((q.h + kCensusTileH - 1) / kCensusTileH);
        segs += (long long)((q.w + 63) / 64) * q.h;
        pixels += (long long)q.w * q.h;
    }
    cen[n] = (int)tiles;
    seg[n] = (int)segs;
    pix[n] = (int)pixels;
    // scanline tasks by class: rows (2h), columns (2w), diagonals (4(w+h-1))
    int r = 0;
    for (int cls = 0; cls < 3; ++cls)
        for (int i = 0; i < n; ++i) {
            const int w = pairs[i].w, h = pairs[i].h;
            const int cnt = cls == 0 ? 2 * h : (cls == 1 ? 2 * w : (prm.n_paths == 4 ? 0 : 4 * (w + h - 1)));
            ts[r] = (int)tasks;
            tp[r] = i;
            tl[r] = cls == 0 ? 0 : (cls == 1 ? 2 * h : 2 * h + 2 * w);
            tc[r] = cnt;
            tasks += (cnt + 3) / 4 * 4;   // ranges start at multiples of 4
            ++r;
        }
    if (tasks >= (1ll << 31) || pixels >= (1ll << 31) || segs >= (1ll << 31)) return EGOSGM_EUNSUPPORTED;

    auto up = [&](size_t off, const void* src, size_t bytes) {
        return hipMemcpy(base + off, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    if (!up(P.pairs, desc.data(), n * sizeof(SgmLaunch)) ||
        !up(P.census_prefix, cen.data(), (n + 1) * sizeof(int)) ||
        !up(P.seg_prefix, seg.data(), (n + 1) * sizeof(int)) ||
        !up(P.pix_prefix, pix.data(), (n + 1) * sizeof(int)) ||
        !up(P.task_start, ts.data(), P.n_ranges * sizeof(int)) ||
        !up(P.task_pair, tp.data(), P.n_ranges * sizeof(int)) ||
        !up(P.task_local, tl.data(), P.n_ranges * sizeof(int)) ||
        !up(P.task_count, tc.data(), P.n_ranges * sizeof(int)))
        return EGOSGM_EDEVICE;

    BatchTables t;
    t.pairs = reinterpret_cast<const SgmLaunch*>(base + P.pairs);
    t.census_prefix = reinterpret_cast<const int*>(base + P.census_prefix);
    t.seg_prefix = reinterpret_cast<const int*>(base + P.seg_prefix);
    t.pix_prefix = reinterpret_cast<const int*>(base + P.pix_prefix);
    t.task_start = reinterpret_cast<const int*>(base + P.task_start);
    t.task_pair = reinterpret_cast<const int*>(base + P.task_pair);
    t.task_local = reinterpret_cast<const int*>(base + P.task_local);
    t.task_count = reinterpret_cast<const int*>(base + P.task_count);
    t.work = reinterpret_cast<unsigned*>(base + P.work);
    {
        std::lock_guard<std::mutex> g(g_tuning_mu);
        t.group = g_tuning.batch_group;
        t.persistent = g_tuning.batch_persistent;
    }
    t.n = n;
    t.n_paths = prm.n_paths == 4 ? 4 : 8;
    t.n_ranges = P.n_ranges;
    t.n_tasks = (int)tasks;
    t.host_census_blocks = (int)tiles;
    t.host_seg_blocks = (int)segs;
    t.host_pixels = (int)pixels;
    t.host_path_blocks = t.persistent ? batch_path_blocks(t.group, max_disp, t.n_tasks) : 0;
    if (t.persistent && t.host_path_blocks <= 0) return EGOSGM_EDEVICE;

    egosgm_plan* plan = new egosgm_plan;
    plan->n = n;
    plan->max_disp = max_disp;
    plan->tables = t;
    plan->pairs_dev = reinterpret_cast<SgmLaunch*>(base + P.pairs);
    plan->shape.assign(pairs, pairs + n);
    hipStream_t cs = nullptr;
    bool ok = hipStreamCreate(&cs) == hipSuccess;
    ok = ok && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        const hipError_t le = launch_sgm_batch(t, max_disp, cs);
        const hipError_t ce = hipStreamEndCapture(cs, &plan->graph);
        ok = le == hipSuccess && ce == hipSuccess && plan->graph;
    }
    ok = ok && hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0) == hipSuccess;
    if (cs) (void)hipStreamDestroy(cs);
    if (!ok) {
        sgm_plan_destroy(plan);
        return EGOSGM_EDEVICE;
    }
    *out = plan;
    return EGOSGM_OK;
}

int sgm_plan_run(egosgm_plan* plan, void* stream) {
    if (!plan || !plan->exec) return EGOSGM_EINVAL;
    return hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)) == hipSuccess
               ? EGOSGM_OK
               : EGOSGM_EDEVICE;
}

int sgm_plan_run_eager(egosgm_plan* plan, void* stream) {
    if (!plan || !plan->exec) return EGOSGM_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const BatchTables& t = plan->tables;
    return timed(EGOSGM_STAGE_BATCH_CENSUS, s, [&] { return launch_batch_stage(t, plan->max_disp, 0, s); }) == hipSuccess &&
                   timed(EGOSGM_STAGE_BATCH_COST, s, [&] { return launch_batch_stage(t, plan->max_disp, 1, s); }) == hipSuccess &&
                   timed(EGOSGM_STAGE_BATCH_PATHS, s, [&] { return launch_batch_stage(t, plan->max_disp, 2, s); }) == hipSuccess &&
                   timed(EGOSGM_STAGE_BATCH_SELECT, s, [&] { return launch_batch_stage(t, plan->max_disp, 3, s); }) == hipSuccess &&
                   timed(EGOSGM_STAGE_BATCH_SELECT, s, [&] { return launch_batch_stage(t, plan->max_disp, 4, s); }) == hipSuccess
               ? EGOSGM_OK
               : EGOSGM_EDEVICE;
}

int egosgm_right_motion(const double* R, const double* t, double baseline, double* t_right) {
    if (!R || !t || !t_right) return EGOSGM_EINVAL;
    for (int i = 0; i < 3; ++i) t_right[i] = t[i] + R[3 * i] * baseline - (i == 0 ? baseline : 0.0);
    return EGOSGM_OK;
}

int lr_check_prediction(float* d_pred, float* p_pred, const float* d_right, int w, int h, float tol,
                        void* stream) {
    if (!d_pred || !p_pred || !d_right || w <= 0 || h <= 0 || !(tol >= 0.0f)) return EGOSGM_EINVAL;
    if ((long long)w * h >= (1ll << 31)) return EGOSGM_EUNSUPPORTED;
    return launch_lr_check_prediction(d_pred, p_pred, d_right, w, h, tol,
                                      static_cast<hipStream_t>(stream)) == hipSuccess
               ? EGOSGM_OK
               : EGOSGM_EDEVICE;
}

int disparity_to_float(const int16_t* d, float* out, int n, void* stream) {
    if (!d || !out || n <= 0) return EGOSGM_EINVAL;
    return launch_disparity_to_float(d, out, n, static_cast<hipStream_t>(stream)) == hipSuccess
               ? EGOSGM_OK
               : EGOSGM_EDEVICE;
}

int sad_check(const uint8_t* left, const uint8_t* right, int w, int h, int pitch, int radius,
              int sad_max, int16_t* disp_wta, float* disp_sub, float* var_meas, void* stream) {
    if (!left || !right || !disp_wta || !disp_sub || !var_meas) return EGOSGM_EINVAL;
    if (w <= 0 || h <= 0 || pitch < w || radius < 0 || radius > 7 || sad_max < 0)
        return EGOSGM_EINVAL;
    if ((long long)w * h >= (1ll << 31)) return EGOSGM_EUNSUPPORTED;
    return launch_sad_check(left, right, w, h, pitch, radius, sad_max, disp_wta, disp_sub, var_meas,
                            static_cast<hipStream_t>(stream)) == hipSuccess
               ? EGOSGM_OK
               : EGOSGM_EDEVICE;
}

int sgm_plan_update(egosgm_plan* plan, const egosgm_pair_update* upd, int n, void* stream) {
    if (!plan || !plan->exec || n < 0 || (n > 0 && !upd)) return EGOSGM_EINVAL;
    for (int j = 0; j < n; ++j) {
        const egosgm_pair_update& u = upd[j];
        if (u.index < 0 || u.index >= plan->n || !u.left || !u.right) return EGOSGM_EINVAL;
        if ((u.lo == nullptr) != (u.hi == nullptr) || (u.lo == nullptr) != (u.offsets == nullptr))
            return EGOSGM_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int j0 = 0; j0 < n; j0 += kPatchBatch) {
        PlanPatches p{};
        p.n = std::min(kPatchBatch, n - j0);
        for (int j = 0; j < p.n; ++j) {
            const egosgm_pair_update& u = upd[j0 + j];
            p.p[j] = PlanPatch{u.index, u.active ? 1 : 0, u.left, u.right, u.lo, u.hi, u.offsets};
        }
        if (launch_plan_patch(plan->pairs_dev, p, s) != hipSuccess) return EGOSGM_EDEVICE;
    }
    return EGOSGM_OK;
}

int sgm_plan_destroy(egosgm_plan* plan) {
    if (!plan) return EGOSGM_OK;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    delete plan;
    return EGOSGM_OK;
}

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

int sgm_census(const uint8_t* left, const uint8_t* right, int w, int h, int pitch, int max_disp,
               void* workspace, size_t workspace_bytes, void* stream) {
    if (!left || !right) return EGOSGM_EINVAL;
    const int rc = check_shape(w, h, max_disp);
    if (rc) return rc;
    if (pitch < w) return EGOSGM_EINVAL;
    WsLayout L;
    ws_layout(w, h, max_disp, L);
    if (!workspace || workspace_bytes < L.total) return EGOSGM_EWORKSPACE;
    uint8_t* base = static_cast<uint8_t*>(workspace);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return timed(EGOSGM_STAGE_CENSUS, s, [&] {
               return launch_census_pair(left, right, w, h, pitch,
                                         reinterpret_cast<uint64_t*>(base + L.census_l),
                                         reinterpret_cast<uint64_t*>(base + L.census_r),
                                         reinterpret_cast<uint32_t*>(base + L.key_r), s);
           }) == hipSuccess
               ? EGOSGM_OK
               : EGOSGM_EDEVICE;
}

size_t egosgm_windows_workspace_bytes(int w, int h) {
    if (w <= 0 || h <= 0) return 0;
    const size_t chunks_per_row = ((size_t)w + kWindowChunk - 1) / kWindowChunk;
    return align_up((size_t)h * chunks_per_row * sizeof(uint32_t));
}

int sgm_windows_from_prediction_noalloc(const float* d_pred, const float* p_pred, int w, int h,
                                        float k_sigma, int r_fixed, int r_min, int r_max, int max_disp,
                                        int16_t* lo, int16_t* hi, uint32_t* offsets, void* stream) {
    if (!d_pred || !lo || !hi || !offsets) return EGOSGM_EINVAL;
    if (r_fixed < 0 && !p_pred) return EGOSGM_EINVAL;
    if (r_min < 0 || r_max < r_min || !(k_sigma >= 0.0f)) return EGOSGM_EINVAL;
    const int rc = check_shape(w, h, max_disp);
    if (rc) return rc;
    const size_t chunks = (size_t)h * (((size_t)w + kWindowChunk - 1) / kWindowChunk);
    if (chunks > (size_t)EGOSGM_NOALLOC_WINDOW_CHUNKS) return EGOSGM_EUNSUPPORTED;
    uint32_t* totals = nullptr;
    if (window_scratch(&totals) != hipSuccess) return EGOSGM_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    return timed(EGOSGM_STAGE_WINDOWS, s, [&] {
               return launch_windows(d_pred, p_pred, w, h, k_sigma, r_fixed, r_min, r_max,
                                     max_disp, lo, hi, offsets, totals, s);
           }) == hipSuccess
               ? EGOSGM_OK
               : EGOSGM_EDEVICE;
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

}  // extern "C"

namespace {

// The prediction of predict_disparity and predict_disparity_static: the
// warp's scatter into the z-buffer z, then the refinement decoding it.
// with_timing: bracket the stages with the timing events when they are on.
int run_predict(const float* d_prev, const float* p_prev, int w, int h, const double* R,
                const double* t, double f, double cx, double cy, double baseline, float q,
                float edge_tol, float fill_tol, float* d_pred, float* p_pred,
                unsigned long long* z, bool with_timing, hipStream_t s) {
    if (!d_prev || !p_prev || !d_pred || !p_pred || !z) return EGOSGM_EINVAL;
    if (w <= 0 || h <= 0 || (long long)w * h >= (1ll << 31)) return EGOSGM_EINVAL;
    if (!(q > 0.0f) || !std::isfinite(q)) return EGOSGM_EINVAL;
    if (std::isnan(edge_tol) || std::isnan(fill_tol)) return EGOSGM_EINVAL;
    if (d_pred == d_prev || d_pred == p_prev || p_pred == d_prev || p_pred == p_prev) return EGOSGM_EINVAL;
    double Hd[16];
    float H[16];
    const int rc = warp_matrix_d(R, t, f, cx, cy, baseline, Hd);
    if (rc) return rc;
    for (int i = 0; i < 16; ++i) H[i] = (float)Hd[i];
    auto scatter = [&] { return launch_warp_scatter(d_prev, w, h, H, z, s); };
    auto refine = [&] {
        return launch_refine_from_zbuf(z, d_prev, p_prev, w, h, Hd, (double)q, edge_tol, fill_tol,
                                       d_pred, p_pred, s);
    };
    if ((with_timing ? timed(EGOSGM_STAGE_WARP, s, scatter) : scatter()) != hipSuccess) return EGOSGM_EDEVICE;
    return (with_timing ? timed(EGOSGM_STAGE_REFINE, s, refine) : refine()) == hipSuccess ? EGOSGM_OK
                                                                                           : EGOSGM_EDEVICE;
}

}  // namespace

extern "C" {

int predict_disparity(const float* d_prev, const float* p_prev, int w, int h, const double* R,
                      const double* t, double f, double cx, double cy, double baseline, float q,
                      float edge_tol, float fill_tol, float* d_pred, float* p_pred, uint64_t* zbuf,
                      void* stream) {
    return run_predict(d_prev, p_prev, w, h, R, t, f, cx, cy, baseline, q, edge_tol, fill_tol, d_pred,
                       p_pred, reinterpret_cast<unsigned long long*>(zbuf), true,
                       static_cast<hipStream_t>(stream));
}

size_t egosgm_refine_workspace_bytes(int w, int h) {
    (void)w;
    (void)h;
    return 0;   // the refinement keeps its intermediate maps on chip
}

int refine_prediction(const float* d_in, const float* p_in, int w, int h, float edge_tol,
                      float fill_tol, float* d_out, float* p_out, void* workspace,
                      size_t workspace_bytes, void* stream) {
    if (!d_in || !p_in || !d_out || !p_out) return EGOSGM_EINVAL;
    if (w <= 0 || h <= 0 || (long long)w * h >= (1ll << 31)) return EGOSGM_EINVAL;
    if (std::isnan(edge_tol) || std::isnan(fill_tol)) return EGOSGM_EINVAL;
    if (d_out == d_in || p_out == p_in || d_out == p_in || p_out == d_in) return EGOSGM_EINVAL;
    (void)workspace;   // none needed (egosgm_refine_workspace_bytes is 0)
    (void)workspace_bytes;
    hipStream_t s = static_cast<hipStream_t>(stream);
    return timed(EGOSGM_STAGE_REFINE, s, [&] {
               return launch_refine(d_in, p_in, w, h, edge_tol, fill_tol, d_out, p_out, s);
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

// ------------------------------------------------------------------ ego-motion
namespace {
bool vo_params_ok(int w, int h, const egosgm_vo_params* prm) {
    if (!prm || prm->levels < 1 || prm->levels > EGOSGM_VO_MAX_LEVELS) return false;
    if (w < 16 || h < 8 || (long long)w * h >= (1ll << 31)) return false;
    if ((w >> (prm->levels - 1)) < 16 || (h >> (prm->levels - 1)) < 8) return false;
    for (int l = 0; l < prm->levels; ++l)
        if (prm->iters[l] < 0 || prm->iters[l] > 64) return false;
    return std::isfinite(prm->huber) && prm->huber > 0.0f && std::isfinite(prm->min_disp) && prm->min_disp >= 0.0f;
}

int vo_call(const uint8_t* prev_left, const uint8_t* cur_left, int w, int h, int pitch, const float* prev_disp,
            double f, double cx, double cy, double baseline, const egosgm_vo_params* prm, int level,
            double* pose, double* out, void* workspace, size_t workspace_bytes, void* stream) {
    if (!prev_left || !cur_left || !prev_disp || !pose || !vo_params_ok(w, h, prm) || pitch < w)
        return EGOSGM_EINVAL;
    if (!(std::isfinite(f) && f > 0.0 && std::isfinite(baseline) && baseline > 0.0 && std::isfinite(cx) &&
          std::isfinite(cy)))
        return EGOSGM_EINVAL;
    if (level >= prm->levels || (level >= 0 && !out)) return EGOSGM_EINVAL;
    if (!workspace || workspace_bytes < vo_workspace_bytes(w, h, prm->levels)) return EGOSGM_EWORKSPACE;
    VoArgs v{};
    v.prev = prev_left;
    v.cur = cur_left;
    v.w = w;
    v.h = h;
    v.pitch = pitch;
    v.prev_disp = prev_disp;
    v.f = f;
    v.cx = cx;
    v.cy = cy;
    v.baseline = baseline;
    v.levels = prm->levels;
    for (int l = 0; l < prm->levels; ++l) v.iters[l] = prm->iters[l];
    v.huber = prm->huber;
    v.min_disp = prm->min_disp;
    v.pose = pose;
    v.out = out;
    v.only_level = level;
    v.workspace = workspace;
    hipStream_t s = static_cast<hipStream_t>(stream);
    return timed(EGOSGM_STAGE_VO, s, [&] { return launch_vo(v, s); }) == hipSuccess ? EGOSGM_OK : EGOSGM_EDEVICE;
}
}  // namespace

size_t egosgm_vo_workspace_bytes(int w, int h, const egosgm_vo_params* prm) {
    if (!vo_params_ok(w, h, prm)) return 0;
    return vo_workspace_bytes(w, h, prm->levels);
}

int estimate_motion(const uint8_t* prev_left, const uint8_t* cur_left, int w, int h, int pitch,
                    const float* prev_disp, double f, double cx, double cy, double baseline,
                    const egosgm_vo_params* prm, double* pose, void* workspace, size_t workspace_bytes,
                    void* stream) {
    return vo_call(prev_left, cur_left, w, h, pitch, prev_disp, f, cx, cy, baseline, prm, -1, pose, nullptr,
                   workspace, workspace_bytes, stream);
}

int vo_normal_equations(const uint8_t* prev_left, const uint8_t* cur_left, int w, int h, int pitch,
                        const float* prev_disp, double f, double cx, double cy, double baseline,
                        const egosgm_vo_params* prm, int level, const double* pose, double* out, void* workspace,
                        size_t workspace_bytes, void* stream) {
    if (level < 0) return EGOSGM_EINVAL;
    return vo_call(prev_left, cur_left, w, h, pitch, prev_disp, f, cx, cy, baseline, prm, level,
                   const_cast<double*>(pose), out, workspace, workspace_bytes, stream);
}

int egosgm_set_tuning(const egosgm_tuning* t) {
    if (!t) return EGOSGM_EINVAL;
    auto ok = [](int g) { return g == 16 || g == 32 || g == 64; };
    if (!ok(t->full_group) || !ok(t->ragged_group) || !ok(t->batch_group) || t->ragged_schedule < 0 ||
        t->ragged_schedule > 8 || (t->wide_offsets != 0 && t->wide_offsets != 1) ||
        (t->batch_persistent != 0 && t->batch_persistent != 1))
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
