// HIP kernels for gfx950 (CDNA4, wave64): census, search windows, 8-path
// semi-global matching over ragged per-pixel windows, its epilogue (WTA,
// subpixel, uncertainty, right map, left-right check), the disparity-space
// warp with a z-buffer, and the pixel-wise Kalman update.
//
// Floating-point steps whose results decide integers (warp target pixel and
// z-order, window centre and radius) must round exactly as written: this file
// is compiled with contraction off (the pragma below repeats it), and with
// correctly rounded float32 division and square root.  HIP's __fsqrt_rn is
// not used on purpose: without OCML_BASIC_ROUNDED_OPERATIONS it maps to the
// approximate native square root.
#include "egosgm_internal.h"

#pragma clang fp contract(off)

namespace egosgm {
namespace {

constexpr int kBlock = 256;
constexpr int kInf = 0x3fff;

// Every buffer the kernels touch is global memory.  Accesses go through
// explicitly global pointers so that the compiler emits global (not flat)
// instructions also where a pointer comes from a descriptor read from
// memory: flat loads count against the LDS wait counter as well, and every
// LDS wait would then drain the outstanding global prefetches.
template <class T>
using gmem = __attribute__((address_space(1))) T;
template <class T>
__device__ inline gmem<T>* gptr(T* p) {
    return (gmem<T>*)p;
}

// Raw buffer over n bytes: stores at offsets >= n are discarded by the
// hardware, which masks a store without a branch.  Word 3 is the gfx9
// family's raw-buffer format word.
__device__ inline __amdgpu_buffer_rsrc_t byte_buffer(void* base, uint32_t n) {
    return __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)n, 0x00020000);
}
constexpr uint32_t kDropOffset = 0xffffffffu;

// ------------------------------------------------------------------ census
// A block computes a kCensusTileW x kCensusTileH output tile; each thread
// takes kCensusPx neighbouring pixels of one row, so a tile row of 12 bytes
// (x-4 .. x+7) per census row serves four pixels.
constexpr int kCtPx = kCensusPx;
constexpr int kCtW = kCensusTileW;
constexpr int kCtH = kCensusTileH;
constexpr int kHaloX = 4, kHaloY = 3;
static_assert(kCtW == 64 * kCtPx && kCtH * 64 == kBlock && kCtPx == 4, "census tile shape");

// One census tile of one image; clear (nullable) gets 0xffffffff per pixel
// (the right-map keys of the matcher, reset here so that no memset is needed
// in a captured graph).  Bit k of a code is [I(q_k) < I(p)] over the 9x7
// offsets row by row, centre skipped; the bits are shifted in from the
// highest k down, two words per pixel, one subtract and one funnel shift
// per bit.
__device__ __attribute__((always_inline)) inline void census_tile(const uint8_t* __restrict__ img, int w, int h, int pitch,
                                   uint64_t* __restrict__ out, uint32_t* __restrict__ clear,
                                   int tx, int ty) {
    constexpr int TW = kCtW + 2 * kHaloX, TH = kCtH + 2 * kHaloY;
    static_assert(TW % 4 == 0, "tile rows are whole words");
    __shared__ uint32_t tile[TH][TW / 4];
    uint8_t* tb = reinterpret_cast<uint8_t*>(&tile[0][0]);
    const gmem<const uint8_t>* __restrict__ gimg = gptr(img);
    const int x0 = tx * kCtW, y0 = ty * kCtH;
    // every load of the staging is issued before the first LDS write, so the
    // block waits on one memory latency, not one per pass (the index of the
    // last, partial pass is clamped and its surplus loads are not stored)
    constexpr int NF = (TW * TH + kBlock - 1) / kBlock;
    uint32_t v[NF];
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        const int i = min((int)threadIdx.x + j * kBlock, TW * TH - 1);
        const int r = i / TW, c = i - r * TW;
        const int gx = min(max(x0 + c - kHaloX, 0), w - 1);
        const int gy = min(max(y0 + r - kHaloY, 0), h - 1);
        v[j] = gimg[(size_t)gy * pitch + gx];
    }
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        const int i = (int)threadIdx.x + j * kBlock;
        if (i < TW * TH) tb[i] = (uint8_t)v[j];
    }
    __syncthreads();
    const int lx = threadIdx.x % 64, ly = threadIdx.x / 64;
    const int x = x0 + kCtPx * lx, y = y0 + ly;
    if (x >= w || y >= h) return;
    // tile column 4*lx is image column x - 4: words lx .. lx+2 of a row
    // hold x-4 .. x+7, the centre row's word lx+1 the four centres.
    const uint32_t cw = tile[ly + kHaloY][lx + 1];
    uint32_t hi[kCtPx], lo[kCtPx];
#pragma unroll
    for (int i = 0; i < kCtPx; ++i) hi[i] = lo[i] = 0u;
#pragma unroll
    for (int dy = 2 * kHaloY; dy >= 0; --dy) {
        const uint32_t rw[3] = {tile[ly + dy][lx], tile[ly + dy][lx + 1], tile[ly + dy][lx + 2]};
#pragma unroll
        for (int dx = 2 * kHaloX; dx >= 0; --dx) {
            if (dy == kHaloY && dx == kHaloX) continue;
            const int k = dy * (2 * kHaloX + 1) + dx - (dy * (2 * kHaloX + 1) + dx > kHaloY * (2 * kHaloX + 1) + kHaloX ? 1 : 0);
#pragma unroll
            for (int i = 0; i < kCtPx; ++i) {
                const int b = i + dx;
                const uint32_t n = (rw[b >> 2] >> (8 * (b & 3))) & 0xffu;
                const uint32_t c = (cw >> (8 * i)) & 0xffu;
                const uint32_t diff = n - c;   // bit 31 set iff n < c
                if (k >= 32)
                    hi[i] = __builtin_amdgcn_alignbit(hi[i], diff, 31);
                else
                    lo[i] = __builtin_amdgcn_alignbit(lo[i], diff, 31);
            }
        }
    }
    gmem<uint64_t>* o = gptr(out) + (size_t)y * w + x;
#pragma unroll
    for (int i = 0; i < kCtPx; ++i)
        if (x + i < w) {
            o[i] = (uint64_t)hi[i] << 32 | lo[i];
            if (clear) gptr(clear)[(size_t)y * w + x + i] = 0xffffffffu;
        }
}

__global__ __launch_bounds__(kBlock) void census_kernel(const uint8_t* __restrict__ img0,
                                                        const uint8_t* __restrict__ img1,
                                                        int w, int h, int pitch,
                                                        uint64_t* __restrict__ out0,
                                                        uint64_t* __restrict__ out1,
                                                        uint32_t* __restrict__ clear) {
    if (blockIdx.z == 0)
        census_tile(img0, w, h, pitch, out0, clear, blockIdx.x, blockIdx.y);
    else
        census_tile(img1, w, h, pitch, out1, nullptr, blockIdx.x, blockIdx.y);
}

// ------------------------------------------------------------------ windows
__device__ inline void window_from_prediction(float d, const float* p_pred, int p, float k_sigma,
                                              int r_fixed, int r_min, int r_max, int D,
                                              int& lo, int& hi) {
    lo = 0;
    hi = D - 1;
    bool usable = d >= 0.0f && d <= 65536.0f;
    int r = r_fixed;
    if (usable && r_fixed < 0) {
        const float pv = p_pred[p];
        if (!(pv >= 0.0f)) {
            usable = false;
        } else {
            const float rf = ceilf(k_sigma * sqrtf(pv));
            r = rf >= (float)r_max ? r_max : (rf <= (float)r_min ? r_min : (int)rf);
        }
    }
    if (usable) {
        r = min(max(r, r_min), r_max);
        const int c = (int)floorf(d + 0.5f);
        const int l2 = max(0, c - r), u2 = min(D - 1, c + r);
        if (l2 <= u2) {
            lo = l2;
            hi = u2;
        }
    }
}

// Block-wide exclusive scan of one value per thread; returns the block total.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t& excl, uint32_t* ws) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) ws[wave] = inc;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) {
        const uint32_t s = ws[i];
        if (i < wave) before += s;
        total += s;
    }
    __syncthreads();
    excl = before + inc - v;
    return total;
}

// Windows in two passes over chunks of kBlock pixels of a row (chunk c of
// row y is chunk index y*nc + c in raster order).  Pass 1: each chunk's
// windows, its offsets relative to the chunk start, and the chunk total.
// Pass 2: each chunk adds the sum of the totals of all earlier chunks.
static_assert(kWindowChunk == kBlock, "one thread per pixel of a window chunk");

__global__ __launch_bounds__(kBlock) void windows_chunk_kernel(
    const float* __restrict__ d_pred, const float* __restrict__ p_pred, int w, float k_sigma,
    int r_fixed, int r_min, int r_max, int D, int16_t* __restrict__ lo, int16_t* __restrict__ hi,
    uint32_t* __restrict__ off, uint32_t* __restrict__ chunk_tot) {
    __shared__ uint32_t ws[kBlock / 64];
    const int y = blockIdx.y, c = blockIdx.x;
    const int x = c * kBlock + (int)threadIdx.x;
    const size_t p = (size_t)y * w + x;
    uint32_t width = 0;
    if (x < w) {
        int l, u;
        window_from_prediction(gptr(d_pred)[p], p_pred, (int)p, k_sigma, r_fixed, r_min, r_max, D, l, u);
        gptr(lo)[p] = (int16_t)l;
        gptr(hi)[p] = (int16_t)u;
        width = (uint32_t)(u - l + 1);
    }
    uint32_t excl;
    const uint32_t tot = block_exclusive_scan(width, excl, ws);
    if (x < w) gptr(off)[p] = excl;
    if (threadIdx.x == 0) gptr(chunk_tot)[(size_t)y * gridDim.x + c] = tot;
}

__global__ __launch_bounds__(kBlock) void windows_base_kernel(int w, int h, uint32_t* __restrict__ off,
                                                              const uint32_t* __restrict__ chunk_tot) {
    __shared__ uint32_t ws[kBlock / 64];
    const int y = blockIdx.y, c = blockIdx.x, nc = gridDim.x;
    const int q = y * nc + c;   // this chunk's raster index
    // the totals are read eight passes at a time, all loads issued before
    // the first add (indexes clamped, the surplus dropped), so a block waits
    // on one memory latency per 8 * kBlock chunks
    constexpr int U = 8;
    uint32_t part = 0;
    for (int i0 = 0; i0 < q; i0 += U * kBlock) {
        uint32_t v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) v[j] = gptr(chunk_tot)[min(i0 + j * kBlock + (int)threadIdx.x, q - 1)];
#pragma unroll
        for (int j = 0; j < U; ++j) part += i0 + j * kBlock + (int)threadIdx.x < q ? v[j] : 0u;
    }
    uint32_t excl;
    const uint32_t base = block_exclusive_scan(part, excl, ws);
    const int x = c * kBlock + (int)threadIdx.x;
    if (x < w) gptr(off)[(size_t)y * w + x] += base;
    if (q == nc * h - 1 && threadIdx.x == 0) gptr(off)[(size_t)h * w] = base + gptr(chunk_tot)[q];
}

// ------------------------------------------------------------------ SGM common
// Window modes: ragged arrays, full range, or decided per pair at run time
// (batched launches mixing both).
constexpr int kWinRagged = 0, kWinFull = 1, kWinAny = 2;

template <int WM>
__device__ inline void window_of(const Windows& win, int p, int& lo, int& hi, uint32_t& off) {
    if (WM == kWinFull || (WM == kWinAny && win.lo == nullptr)) {
        lo = 0;
        hi = win.max_disp - 1;
        off = (uint32_t)p * (uint32_t)win.max_disp;
    } else {
        lo = gptr(win.lo)[p];
        hi = gptr(win.hi)[p];
        off = gptr(win.off)[p];
    }
}

// Packed window of one pixel for the path kernels: offset | lo << 32 |
// width << 48 (lo and width < 2^16).  The cost pass writes it for ragged
// windows, so a scanline step loads one 8-byte word; the full range is
// synthesised without a load.  Rings keep the raw word and unpack it where
// it is used, so the unpacking never waits on a load early.
__device__ inline uint64_t pack_meta(uint32_t off, int lo, int w) {
    return (uint64_t)off | ((uint64_t)(uint16_t)lo << 32) | ((uint64_t)(uint16_t)w << 48);
}
__device__ inline int meta_lo(uint64_t v) { return (int)(uint16_t)(v >> 32); }
__device__ inline int meta_w(uint64_t v) { return (int)(v >> 48); }
__device__ inline uint32_t meta_off(uint64_t v) { return (uint32_t)v; }

// Minimum over each 16-lane row, left in every lane of the row (DPP:
// quad_perm xor 1, xor 2, then row_ror 4 and 8; each stage folds into one
// v_min_i32_dpp).
__device__ inline int row_min16(int v) {
    v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0xB1, 0xF, 0xF, true));
    v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0x4E, 0xF, 0xF, true));
    v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0x124, 0xF, 0xF, true));
    v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0x128, 0xF, 0xF, true));
    return v;
}

// Minimum over a lane group of G (16, 32 or 64) lanes; every lane of the
// group must be active.  32 lanes: the two rows of a half are combined by a
// row swap.  64 lanes: rows are chained with row_bcast 15 (rows 1 and 3 take
// row 0's and row 2's minimum) and row_bcast 31 (rows 2 and 3 take row 1's),
// then the last lane is read into a scalar register.
template <int G>
__device__ inline int group_min(int v) {
    v = row_min16(v);
    if (G == 16) return v;
    if (G == 32) {
        // v_permlane16_swap on (v, v) leaves rows (0,0,2,2) in one result and
        // (1,1,3,3) in the other: their minimum is each 32-lane half's
        const auto sw = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
        return min((int)sw[0], (int)sw[1]);
    }
    v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0x142, 0xA, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0x143, 0xC, 0xF, false));
    return __builtin_amdgcn_readlane(v, 63);
}

// Orders this lane group's LDS writes before its later LDS reads.  A wave's
// LDS instructions execute in issue order, so only the compiler has to be
// stopped from moving them; no wait on outstanding global stores is needed.
__device__ inline void lds_order() { __asm__ volatile("" ::: "memory"); }

// ------------------------------------------------------------------ cost
// C(p, d) = popcount(cL(x,y) ^ cR(x-d,y)), or 62 where x-d < 0, written once
// per search slot (uint8, ragged layout).  One block per 64-pixel row
// segment stages the left codes and the right codes x0-(D-1) .. x0+63 in LDS.
constexpr int kSeg = 64;

template <int G, int WM>
__device__ inline void cost_segment(const SgmLaunch& a, int seg, int y) {
    constexpr int GPB = kBlock / G;
    static_assert(kSeg <= kBlock, "one thread per pixel of a segment");
    __shared__ uint64_t crs[kSeg + kMaxDisp];
    __shared__ uint64_t cls[kSeg];
    __shared__ int s_lo[kSeg], s_w[kSeg];
    __shared__ uint32_t s_off[kSeg];
    const int W = a.w, D = a.win.max_disp;
    const int x0 = seg * kSeg;
    const int base = x0 - (D - 1);
    const gmem<const uint64_t>* rowl = gptr(a.census_l + (size_t)y * W);
    const gmem<const uint64_t>* rowr = gptr(a.census_r + (size_t)y * W);
    gmem<uint8_t>* __restrict__ cost = gptr(a.cost);
    // windows of the segment's pixels are read once, next to the codes,
    // so the slot loop below waits on no global load
    if (WM != kWinFull && threadIdx.x < kSeg && x0 + (int)threadIdx.x < W) {
        const int p = y * W + x0 + (int)threadIdx.x;
        int lo, hi;
        uint32_t off;
        window_of<WM>(a.win, p, lo, hi, off);
        s_lo[threadIdx.x] = lo;
        s_w[threadIdx.x] = hi - lo + 1;
        s_off[threadIdx.x] = off;
        if (WM == kWinRagged || a.win.lo != nullptr) gptr(a.meta)[p] = pack_meta(off, lo, hi - lo + 1);
    }
    for (int i = threadIdx.x; i < kSeg + D - 1; i += kBlock) {
        const int xr = base + i;
        crs[i] = (xr >= 0 && xr < W) ? rowr[xr] : 0ull;
    }
    for (int i = threadIdx.x; i < kSeg; i += kBlock) cls[i] = (x0 + i < W) ? rowl[x0 + i] : 0ull;
    __syncthreads();
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    if constexpr (WM == kWinFull) {
        for (int i = grp; i < kSeg; i += GPB) {
            const int x = x0 + i;
            if (x >= W) break;
            const uint32_t off = (uint32_t)(y * W + x) * (uint32_t)D;
            const uint64_t cl = cls[i];
            for (int sl = lane; sl < D; sl += G) {
                const int c = (x - sl >= 0) ? __popcll(cl ^ crs[i + (D - 1) - sl]) : kCensusBits;
                cost[off + (uint32_t)sl] = (uint8_t)c;
            }
        }
    } else {
        // the group's pixels' windows and left codes are read from LDS
        // together (one wait), then each pixel's slots are written
        constexpr int NPX = kSeg / GPB;
        int lo[NPX], wd[NPX];
        uint32_t off[NPX];
        uint64_t cl[NPX];
#pragma unroll
        for (int j = 0; j < NPX; ++j) {
            const int i = grp + j * GPB;
            lo[j] = s_lo[i];
            wd[j] = x0 + i < W ? s_w[i] : 0;   // past the row: no slots
            off[j] = s_off[i];
            cl[j] = cls[i];
        }
#pragma unroll
        for (int j = 0; j < NPX; ++j) {
            const int i = grp + j * GPB;
            const int x = x0 + i;
            for (int sl = lane; sl < wd[j]; sl += G) {
                const int d = lo[j] + sl;
                const int c = (x - d >= 0) ? __popcll(cl[j] ^ crs[i + (D - 1) - d]) : kCensusBits;
                cost[off[j] + (uint32_t)sl] = (uint8_t)c;
            }
        }
    }
}

template <int G, int WM>
__global__ __launch_bounds__(kBlock) void cost_kernel(SgmLaunch a) {
    cost_segment<G, WM>(a, blockIdx.x, blockIdx.y);
}

// ------------------------------------------------------------------ SGM paths
// Scanline tasks, longest first: rows left-to-right and right-to-left,
// columns down and up, then the four diagonal families (W+H-1 lines each).
__device__ inline void decode_task(int t, int W, int H, int& dir, int& x, int& y, int& len) {
    if (t < 2 * H) {
        dir = t / H;
        y = t - dir * H;
        x = dir == 0 ? 0 : W - 1;
        len = W;
        return;
    }
    t -= 2 * H;
    if (t < 2 * W) {
        dir = 2 + t / W;
        x = t - (dir - 2) * W;
        y = dir == 2 ? 0 : H - 1;
        len = H;
        return;
    }
    t -= 2 * W;
    const int nd = W + H - 1;
    dir = 4 + t / nd;
    const int i = t - (dir - 4) * nd;
    switch (dir) {
        case 4:  // (1,1)
            if (i < W) { x = i; y = 0; } else { x = 0; y = i - W + 1; }
            len = min(W - x, H - y);
            break;
        case 5:  // (-1,1)
            if (i < W) { x = i; y = 0; } else { x = W - 1; y = i - W + 1; }
            len = min(x + 1, H - y);
            break;
        case 6:  // (1,-1)
            if (i < W) { x = i; y = H - 1; } else { x = 0; y = i - W; }
            len = min(W - x, y + 1);
            break;
        default:  // (-1,-1)
            if (i < W) { x = i; y = H - 1; } else { x = W - 1; y = i - W; }
            len = min(x + 1, y + 1);
            break;
    }
}

__device__ inline void dir_step(int dir, int& dx, int& dy) {
    // (1,0) (-1,0) (0,1) (0,-1) (1,1) (-1,1) (1,-1) (-1,-1)
    dx = (dir == 0 || dir == 4 || dir == 6) ? 1 : ((dir == 1 || dir == 5 || dir == 7) ? -1 : 0);
    dy = (dir == 2 || dir == 4 || dir == 5) ? 1 : ((dir == 3 || dir == 6 || dir == 7) ? -1 : 0);
}

// Costs of this lane's slots s = lane + G*k of one pixel's window, through a
// raw buffer.  The window offset differs between the lane groups of a wave,
// so it goes into the per-lane offset.  Lanes past the window read other
// pixels' bytes (or zero past the buffer's end, where the hardware drops the
// read); the LDS scanline step replaces every such slot by +infinity, so the
// offset needs no clamp.
template <int G, int K>
__device__ inline void load_costs_buf(__amdgpu_buffer_rsrc_t cbuf, uint32_t off, int lane, int (&c)[K]) {
#pragma unroll
    for (int k = 0; k < K; ++k)
        c[k] = __builtin_amdgcn_raw_buffer_load_b8(cbuf, off + (uint32_t)(lane + G * k), 0, 0);
}

// A scanline task: direction, first pixel, pixel step and length.
struct Scan {
    int dir, p0, dp, len;
};

__device__ inline Scan scan_of(int task, int W, int H) {
    int dir, x, y, len, dx, dy;
    decode_task(task, W, H, dir, x, y, len);
    dir_step(dir, dx, dy);
    return Scan{dir, y * W + x, dy * W + dx, len};
}

template <int WM>
__device__ inline uint64_t scan_meta(const SgmLaunch& a, int p) {
    if (WM == kWinFull || (WM == kWinAny && a.win.lo == nullptr))
        return pack_meta((uint32_t)p * (uint32_t)a.win.max_disp, 0, a.win.max_disp);
    return gptr(a.meta)[p];
}

// Entries of one LDS row of a scanline: absolute disparity d at index d+1,
// for D <= G*K, plus room for a whole chunk of G lanes past any window.
constexpr int lds_row(int G, int K) { return 2 * G * K + 2; }

// ---- LDS scanline (ragged windows, work proportional to the window) ----
// One lane group of G lanes walks one scanline; lane l owns slots
// s = l + G*k (k < K) of each pixel's window.  The previous pixel's path
// costs sit in a per-group LDS row (ping-pong) indexed by absolute disparity
// (entry d+1; entry 0 and the entries past D are guards).  Every entry outside the
// predecessor's window holds +infinity: a step erases the row it has just
// consumed, so the row is clean when it is written again two steps later.
// The d-1, d, d+1 lookups therefore need no bounds checks, and ragged
// windows realign by plain indexing.
// Window metadata is prefetched 2*PF steps ahead and costs PF steps ahead,
// unconditionally (clamped to the scanline's last pixel) and into ring
// slots named at compile time, so a step waits only on memory operations
// issued PF steps earlier.  A zero predecessor row over the first window
// makes the first step L = C.
// ODW: chunk 0's costs are prefetched for every pixel, the other chunks'
// only for pixels where some lane group of the wave has a window wider than
// G (a wave-uniform test on the prefetched window words), into a ring of
// their own.  Narrow windows then cost one load per step instead of K.
// Q32 (ragged windows, w*h < 2^27, so every byte offset below, including
// the overshoot past either end of a scanline, fits an int; and the eight
// path volumes within 2^32 bytes): the window word RM steps ahead is read
// through a buffer at a running byte offset clamped into the scanline (past
// its end the last pixel's word again), so the prefetch address costs an
// add, a max and a min, without 64-bit address arithmetic; and path costs are
// stored at a 32-bit offset from the common base of the eight volumes, the
// same for every lane group of the wave, so a store needs no 64-bit address.
template <int G, int K, int WM, int PF, bool ODW = false, bool Q32 = false>
__device__ inline void lds_scanline(const SgmLaunch& a, const Scan& sc, int lane,
                                    uint16_t* b0, uint16_t* b1) {
    static_assert(!Q32 || WM == kWinRagged, "byte-offset window words need ragged windows");
    constexpr int RM = 2 * PF;
    constexpr int KP = ODW ? 1 : K;   // prefetched chunks
    constexpr int ROW = lds_row(G, K);
    // The cost buffer is the same for every lane group of the wave; the path
    // volume is not (groups walk different directions), so it stays a global
    // pointer.
    gmem<uint8_t>* __restrict__ vol = gptr(a.vol + (size_t)sc.dir * a.vol_stride);
    const __amdgpu_buffer_rsrc_t cbuf = byte_buffer(a.cost, (uint32_t)a.vol_stride);
    const int p1 = a.p1, p2 = a.p2;
    const int dp = sc.dp, len = sc.len, p0 = sc.p0;
    const int p_last = p0 + (len - 1) * dp;

    uint64_t mm[RM];
    auto load_meta = [&](int j, int pix) { mm[j] = scan_meta<WM>(a, pix); };
#pragma unroll
    for (int j = 0; j < RM; ++j) load_meta(j, j < len ? p0 + j * dp : p_last);
    const __amdgpu_buffer_rsrc_t mbuf = byte_buffer(a.meta, Q32 ? (uint32_t)a.w * (uint32_t)a.h * 8u : 0u);
    const int q_lo = 8 * min(p0, p_last), q_hi = 8 * max(p0, p_last), dq = 8 * dp;
    int q_next = 8 * (p0 + RM * dp);
    gmem<uint8_t>* __restrict__ vol_all = gptr(a.vol);
    const uint32_t vrow = (uint32_t)sc.dir * (uint32_t)a.vol_stride + (uint32_t)lane;
    auto next_meta = [&](int j) {
        mm[j] = __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(mbuf, min(max(q_next, q_lo), q_hi), 0, 0));
        q_next += dq;
    };
    int cst[PF][KP];
    int wst[PF][K > KP ? K - KP : 1];   // chunks KP.. of wide pixels (ODW)
    bool wide_pf[PF];                    // ODW: the wave-uniform wide test, kept for the step
    auto load_costs = [&](int slot, uint64_t m) {
        load_costs_buf<G, KP>(cbuf, meta_off(m), lane, cst[slot]);
        const bool wd = K > KP && __builtin_amdgcn_ballot_w64(meta_w(m) > G) != 0;
        wide_pf[slot] = wd;
        if (wd) {
#pragma unroll
            for (int k = KP; k < K; ++k)
                wst[slot][k - KP] = __builtin_amdgcn_raw_buffer_load_b8(
                    cbuf, meta_off(m) + (uint32_t)(lane + G * k), 0, 0);
        }
    };
#pragma unroll
    for (int j = 0; j < PF; ++j) load_costs(j, mm[j]);

    for (int e = lane; e < ROW; e += G) {
        b0[e] = kInf;
        b1[e] = kInf;
    }
    lds_order();
    for (int e = lane; e < meta_w(mm[0]); e += G) b1[meta_lo(mm[0]) + 1 + e] = 0;   // zero predecessor
    lds_order();
    int m_q = 0;
    // the previous step's row at its window start (chunk 0 of this lane):
    // the address it was written at is the one erased one step later
    uint16_t* erase = b1 + meta_lo(mm[0]) + lane + 1;
    // Chunks k (slots lane + G*k) written by the previous step: wave-uniform
    // bits, since a chunk runs when any lane group of the wave needs it.
    uint32_t done_q = 0;
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (k == 0 || __builtin_amdgcn_ballot_w64(lane + G * k < meta_w(mm[0])) != 0) done_q |= 1u << k;
    int p = p0;

    // One step.  A running chunk reads and writes all its lanes (the rows
    // are 2*G*K+2 entries, so every index stays inside): lanes past the
    // window write +infinity, which keeps the row outside the window at
    // +infinity, and only the global store is masked.  The reads depend on
    // nothing of the previous step's minimum, so they can issue while its
    // reduction runs.
    auto step = [&](int ti, int tc, int parity) {
        const int lo_c = meta_lo(mm[ti]), w_c = meta_w(mm[ti]);
        const uint32_t off_c = meta_off(mm[ti]);
        uint16_t* cur = parity ? b1 : b0;
        uint16_t* prv = parity ? b0 : b1;
        const int m2 = m_q + p2;
        int mn = kInf;
        uint32_t done_c = 0;
        // wave-uniform; with ODW the same test on the same window word was
        // taken when this step's costs were requested
        const bool wide = K > 1 && (K > KP ? wide_pf[tc] : __builtin_amdgcn_ballot_w64(w_c > G) != 0);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int s = lane + G * k;
            if (k == 0 || (wide && __builtin_amdgcn_ballot_w64(s < w_c) != 0)) {
                done_c |= 1u << k;
                const uint16_t* q = prv + lo_c + s;   // q[0] = d-1, q[1] = d, q[2] = d+1
                const int best = min(min((int)q[1], min((int)q[0], (int)q[2]) + p1), m2);
                const int ck = k < KP ? cst[tc][k < KP ? k : 0] : wst[tc][k >= KP ? k - KP : 0];
                const int L = ck + best - m_q;
                const bool in = s < w_c;
                const int Lm = in ? L : kInf;
                cur[lo_c + s + 1] = (uint16_t)Lm;
                if (in) {
                    if constexpr (Q32)
                        vol_all[vrow + off_c + (uint32_t)(G * k)] = (uint8_t)L;
                    else
                        vol[off_c + (uint32_t)s] = (uint8_t)L;
                }
                mn = k == 0 ? Lm : min(mn, Lm);   // in-window L < kInf, so chunk 0 needs no min
            }
        }
        lds_order();
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (done_q & (1u << k)) erase[G * k] = kInf;
        done_q = done_c;
        m_q = group_min<G>(mn);
        erase = cur + lo_c + lane + 1;
    };

    int i = 0;
    for (; i + RM <= len; i += RM) {
#pragma unroll
        for (int u = 0; u < RM; ++u) {
            step(u, u % PF, u & 1);
            load_costs(u % PF, mm[(u + PF) % RM]);
            if constexpr (Q32) {
                next_meta(u);
            } else {
                load_meta(u, (i + u + RM < len) ? p + RM * dp : p_last);
                p += dp;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < RM; ++u) {
        if (i + u < len) {
            step(u, u % PF, u & 1);
            if (u + PF < RM)
                load_costs(u % PF, mm[u + PF]);
            p += dp;
        }
    }
}

// ---- packed register scanline ----
// A lane group of G lanes holds all D = 2*NP*G disparities, lane l owning
// the contiguous slots 2*NP*l .. 2*NP*l + 2*NP - 1 as NP registers of two
// 16-bit values (packed u16 arithmetic).  The d-1 / d+1 neighbours come from
// v_alignbit on a lane's own registers plus one DPP lane shift for the slot
// owned by the neighbouring lane; the group minimum m uses DPP reductions.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ inline u16x2 as_pk(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ inline uint32_t as_u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ inline uint32_t pk_min(uint32_t a, uint32_t b) {
    return as_u32(__builtin_elementwise_min(as_pk(a), as_pk(b)));
}
__device__ inline uint32_t pk_add(uint32_t a, uint32_t b) { return as_u32(as_pk(a) + as_pk(b)); }
__device__ inline uint32_t pk_sub(uint32_t a, uint32_t b) { return as_u32(as_pk(a) - as_pk(b)); }
// (hi:lo) >> 16: the upper half of lo becomes the lower half of the result.
__device__ inline uint32_t align16(uint32_t hi, uint32_t lo) { return __builtin_amdgcn_alignbit(hi, lo, 16); }
constexpr uint32_t kInfPk = 0x3fff3fffu;

// Previous lane's value within a group of G lanes (lane 0 of the group gets
// INF), and the next lane's (last lane gets INF).
template <int G>
__device__ inline uint32_t from_prev_lane(uint32_t v) {
    if (G == 16) return __builtin_amdgcn_update_dpp(kInfPk, v, 0x111, 0xF, 0xF, false);  // row_shr:1
    const uint32_t r = __builtin_amdgcn_update_dpp(kInfPk, v, 0x138, 0xF, 0xF, false);   // wave_shr:1
    return (G == 32 && (threadIdx.x & 31) == 0) ? kInfPk : r;
}
template <int G>
__device__ inline uint32_t from_next_lane(uint32_t v) {
    if (G == 16) return __builtin_amdgcn_update_dpp(kInfPk, v, 0x101, 0xF, 0xF, false);  // row_shl:1
    const uint32_t r = __builtin_amdgcn_update_dpp(kInfPk, v, 0x130, 0xF, 0xF, false);   // wave_shl:1
    return (G == 32 && (threadIdx.x & 31) == 31) ? kInfPk : r;
}

// 2*NP cost bytes of one lane, loaded in one access (full range).
template <int NP> struct CostWord;
template <> struct CostWord<1> { using T = uint16_t; };
template <> struct CostWord<2> { using T = uint32_t; };
// (clang vector types: they load and store through global pointers)
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <> struct CostWord<4> { using T = u32x2; };
template <> struct CostWord<8> { using T = u32x4; };

template <int NP>
__device__ inline void unpack_costs(const typename CostWord<NP>::T& w, uint32_t (&c)[NP]) {
    // bytes b0 b1 -> (b0 | b1 << 16)
    if constexpr (NP == 1) {
        c[0] = __builtin_amdgcn_perm(0u, (uint32_t)w, 0x0C010C00u);
    } else if constexpr (NP == 2) {
        c[0] = __builtin_amdgcn_perm(0u, w, 0x0C010C00u);
        c[1] = __builtin_amdgcn_perm(0u, w, 0x0C030C02u);
    } else {
        const uint32_t* u = reinterpret_cast<const uint32_t*>(&w);
#pragma unroll
        for (int q = 0; q < NP / 2; ++q) {
            c[2 * q] = __builtin_amdgcn_perm(0u, u[q], 0x0C010C00u);
            c[2 * q + 1] = __builtin_amdgcn_perm(0u, u[q], 0x0C030C02u);
        }
    }
}

template <int NP>
__device__ inline typename CostWord<NP>::T pack_costs(const uint32_t (&L)[NP]) {
    // low bytes of the 16-bit halves, in slot order
    if constexpr (NP == 1) {
        return (uint16_t)__builtin_amdgcn_perm(0u, L[0], 0x0C0C0200u);
    } else if constexpr (NP == 2) {
        return __builtin_amdgcn_perm(L[1], L[0], 0x06040200u);
    } else {
        typename CostWord<NP>::T w;
        uint32_t* u = reinterpret_cast<uint32_t*>(&w);
#pragma unroll
        for (int q = 0; q < NP / 2; ++q) u[q] = __builtin_amdgcn_perm(L[2 * q + 1], L[2 * q], 0x06040200u);
        return w;
    }
}

// One recurrence step on the packed registers: L <- C + min(L(d), L(d+-1) +
// P1, m + P2) - m, and the new group minimum.  Entries whose cost is the
// out-of-window marker 0x3fff stay >= 0x3fff - 255, far above any in-window
// m + P2 (<= 255 + 193), so they never win a minimum: they act as +infinity
// for the next step, and stay below 0x3fff + 193, so nothing overflows.
template <int G, int NP>
// shp / shn: the last lane shifts, carried from step to step.  At 64 lanes
// the shifted-in value of lane 0 (63) is never written, so it keeps the +inf
// the caller starts them with, and no per-step copy of +inf is needed.
__device__ inline void packed_update(uint32_t (&L)[NP], const uint32_t (&c)[NP], int& m,
                                     uint32_t p1pk, int p2, uint32_t& shp, uint32_t& shn) {
    const uint32_t mpk = (uint32_t)m * 0x10001u;
    const uint32_t m2pk = (uint32_t)(m + p2) * 0x10001u;
    uint32_t prv, nxt;
    if (G == 64) {
        prv = shp = __builtin_amdgcn_update_dpp(shp, L[NP - 1], 0x138, 0xF, 0xF, false);   // wave_shr:1
        nxt = shn = __builtin_amdgcn_update_dpp(shn, L[0], 0x130, 0xF, 0xF, false);        // wave_shl:1
    } else {
        prv = from_prev_lane<G>(L[NP - 1]);
        nxt = from_next_lane<G>(L[0]);
    }
    uint32_t Ln[NP];
#pragma unroll
    for (int r = 0; r < NP; ++r) {
        const uint32_t lm1 = align16(L[r], r > 0 ? L[r - 1] : prv);
        const uint32_t lp1 = align16(r + 1 < NP ? L[r + 1] : nxt, L[r]);
        uint32_t t = pk_add(pk_min(lm1, lp1), p1pk);
        t = pk_min(pk_min(t, L[r]), m2pk);
        Ln[r] = pk_sub(pk_add(c[r], t), mpk);
    }
    uint32_t mv = Ln[0];
#pragma unroll
    for (int r = 0; r < NP; ++r) {
        L[r] = Ln[r];
        mv = pk_min(mv, Ln[r]);
    }
    m = group_min<G>((int)min(mv & 0xffffu, mv >> 16));
}

// Full range: costs and path costs are dense (pixel p, slot d at p*D + d),
// one word of 2*NP bytes per lane.  Prefetch: the cost words of step i + PF
// are loaded while step i runs, unconditionally (past the end of the
// scanline the last pixel is loaded again) and into ring slots named at
// compile time, so no loaded register is copied before use and a step waits
// only on loads and stores issued PF steps earlier.  The zero initial state
// makes the first step L = C.
template <int G, int NP, int PF>
__device__ inline void packed_scanline_full(const SgmLaunch& a, const Scan& sc, int lane) {
    using Word = typename CostWord<NP>::T;
    constexpr uint32_t WB = sizeof(Word);
    const gmem<uint8_t>* __restrict__ cost = gptr(a.cost);
    gmem<uint8_t>* __restrict__ vol = gptr(a.vol + (size_t)sc.dir * a.vol_stride);
    const int dp = sc.dp, len = sc.len, p0 = sc.p0;
    const int p_last = p0 + (len - 1) * dp;
    const uint32_t p1pk = (uint32_t)a.p1 * 0x10001u;
    const int p2 = a.p2;
    auto at = [&](int pix) { return ((uint32_t)pix * G + lane) * WB; };

    Word ring[PF];
#pragma unroll
    for (int j = 0; j < PF; ++j)
        ring[j] = *reinterpret_cast<const gmem<Word>*>(cost + at(j < len ? p0 + j * dp : p_last));
    uint32_t L[NP];
#pragma unroll
    for (int r = 0; r < NP; ++r) L[r] = 0u;
    int m = 0;
    uint32_t shp = kInfPk, shn = kInfPk;   // lane-shift state (packed_update)
    int p = p0;
    auto step = [&](const Word& w) {
        uint32_t c[NP];
        unpack_costs<NP>(w, c);
        packed_update<G, NP>(L, c, m, p1pk, p2, shp, shn);
        *reinterpret_cast<gmem<Word>*>(vol + at(p)) = pack_costs<NP>(L);
    };
    int i = 0;
    for (; i + PF <= len; i += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            step(ring[u]);
            ring[u] = *reinterpret_cast<const gmem<Word>*>(cost + at((i + u + PF < len) ? p + PF * dp : p_last));
            p += dp;
        }
    }
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        if (i + u < len) {
            step(ring[u]);
            p += dp;
        }
    }
}

// ---- register scanline (ragged windows, one wave per scanline) ----
// Lane j holds slot j + 64*k (chunk k < K) of the previous pixel's path
// costs, counted from that pixel's window start lo_q.  Slots past a window
// hold values >= kInf: their cost is the marker kInf, every candidate of a
// minimum is >= the previous minimum, so they stay in [kInf, kInf + P2] and
// act as +infinity, as the out-of-window marker does in packed_update.
// A step whose window and predecessor window fit in one chunk takes the
// d-1, d, d+1 predecessors by lane shifts: DPP when the window start is
// unchanged, ds_bpermute by the start difference otherwise.  A step with a
// wider window goes through an LDS row indexed by absolute disparity (entry
// d+1, +infinity outside the written range, erased after use), as in
// lds_scanline.  Every branch depends on wave-uniform values only.

__device__ inline int lane_from(int v, int t) {
    const int r = __builtin_amdgcn_ds_bpermute(t << 2, v);
    return (unsigned)t < 64u ? r : kInf;
}

template <int K, int WM, int PF, int RM = 2 * PF>
__device__ inline void reg_scanline(const SgmLaunch& a, const Scan& sc, int lane, uint16_t* row) {
    static_assert(RM % PF == 0 && RM >= 2 * PF, "ring sizes");
    constexpr int ROW = lds_row(64, K);
    const __amdgpu_buffer_rsrc_t vol =
        byte_buffer(a.vol + (size_t)sc.dir * a.vol_stride, (uint32_t)a.vol_stride);
    const gmem<uint8_t>* __restrict__ cost = gptr(a.cost);
    const int p1 = a.p1, p2 = a.p2;
    const int dp = sc.dp, len = sc.len, p0 = sc.p0;
    const int p_last = p0 + (len - 1) * dp;

    // Window words are loaded RM steps ahead (vector ring mm); when the
    // costs of a pixel are requested, PF steps ahead, its word is moved to
    // scalar registers (ring s_off / s_lw), which the step then uses.
    uint64_t mm[RM];
    uint32_t s_off[PF], s_lw[PF];
    int cst[PF][K];
    auto load_meta = [&](int j, int pix) { mm[j] = scan_meta<WM>(a, pix); };
    auto load_cost = [&](int slot, int j) {
        s_off[slot] = __builtin_amdgcn_readfirstlane((uint32_t)mm[j]);
        s_lw[slot] = __builtin_amdgcn_readfirstlane((uint32_t)(mm[j] >> 32));
        const int w = (int)(s_lw[slot] >> 16);
        const gmem<uint8_t>* c = cost + s_off[slot];
#pragma unroll
        for (int k = 0; k < K; ++k) cst[slot][k] = c[min(lane + 64 * k, w - 1)];
    };
#pragma unroll
    for (int j = 0; j < RM; ++j) load_meta(j, j < len ? p0 + j * dp : p_last);
#pragma unroll
    for (int j = 0; j < PF; ++j) load_cost(j, j);

    for (int e = lane; e < ROW; e += 64) row[e] = kInf;
    lds_order();
    int lo_q = (int)(s_lw[0] & 0xffffu);
    int w_q = (int)(s_lw[0] >> 16);
    int L[K];
#pragma unroll
    for (int k = 0; k < K; ++k) L[k] = lane + 64 * k < w_q ? 0 : kInf;   // zero predecessor
    int m_q = 0;
    int p = p0;

    auto step = [&](int tc) {
        const int lo_c = (int)(s_lw[tc] & 0xffffu), w_c = (int)(s_lw[tc] >> 16);
        const uint32_t off_c = s_off[tc];
        const int m2 = m_q + p2;
        int mn;
        if (__builtin_expect((w_c <= 64) & (w_q <= 64), 1)) {
            int A, B, C;
            if (__builtin_expect(lo_c == lo_q, 1)) {
                A = __builtin_amdgcn_update_dpp(kInf, L[0], 0x138, 0xF, 0xF, false);   // wave_shr:1
                B = L[0];
                C = __builtin_amdgcn_update_dpp(kInf, L[0], 0x130, 0xF, 0xF, false);   // wave_shl:1
            } else {
                const int t = lane + (lo_c - lo_q);
                A = lane_from(L[0], t - 1);
                B = lane_from(L[0], t);
                C = lane_from(L[0], t + 1);
            }
            const bool in = lane < w_c;
            const int c = in ? cst[tc][0] : kInf;
            const int Ln = c + min(min(min(A, C) + p1, B), m2) - m_q;
            L[0] = Ln;
            __builtin_amdgcn_raw_buffer_store_b8((uint8_t)Ln, vol, in ? off_c + (uint32_t)lane : kDropOffset,
                                                 0, 0);
            mn = Ln;
        } else {
#pragma unroll
            for (int k = 0; k < K; ++k) row[lo_q + lane + 64 * k + 1] = (uint16_t)L[k];
            lds_order();
            mn = kInf;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int s = lane + 64 * k;
                const uint16_t* q = row + lo_c + s;   // q[0] = d-1, q[1] = d, q[2] = d+1
                const bool in = s < w_c;
                const int c = in ? cst[tc][k] : kInf;
                const int Ln = c + min(min(min((int)q[0], (int)q[2]) + p1, (int)q[1]), m2) - m_q;
                L[k] = Ln;
                __builtin_amdgcn_raw_buffer_store_b8((uint8_t)Ln, vol, in ? off_c + (uint32_t)s : kDropOffset,
                                                     0, 0);
                mn = min(mn, Ln);
            }
            lds_order();
#pragma unroll
            for (int k = 0; k < K; ++k) row[lo_q + lane + 64 * k + 1] = kInf;
        }
        m_q = group_min<64>(mn);
        lo_q = lo_c;
        w_q = w_c;
    };

    int i = 0;
    for (; i + RM <= len; i += RM) {
#pragma unroll
        for (int u = 0; u < RM; ++u) {
            step(u % PF);
            load_cost(u % PF, (u + PF) % RM);
            load_meta(u, (i + u + RM < len) ? p + RM * dp : p_last);
            p += dp;
        }
    }
#pragma unroll
    for (int u = 0; u < RM; ++u) {
        if (i + u < len) {
            step(u % PF);
            if (u + PF < RM) load_cost(u % PF, u + PF);
            p += dp;
        }
    }
}

// ---- windowed register scanline (ragged windows, branch-free steps) ----
// One wave per scanline; lane l holds disparities 2*NP*l .. 2*NP*l+2*NP-1
// of the whole range as packed u16 pairs (the full-range layout), so a step
// never shifts lanes when the window moves.  Slots outside the pixel's
// window take the marker cost kInf (packed_update keeps them out of every
// minimum), costs are read with buffer loads clamped into the window, and
// only in-window path costs are stored: the store offset of any other slot
// is pushed out of the buffer's range, where the hardware drops it.  Every
// step runs the same instructions, without a branch.  Window words: ring mm
// (RM steps ahead), moved to scalar registers when the costs are requested
// (PF steps ahead).
template <int NP, int WM, int PF, int RM = 2 * PF>
__device__ inline void win_scanline(const SgmLaunch& a, const Scan& sc, int lane) {
    constexpr int S = 2 * NP;
    static_assert(RM % PF == 0 && RM >= 2 * PF, "ring sizes");
    const uint32_t span = (uint32_t)a.vol_stride;
    const __amdgpu_buffer_rsrc_t vol = byte_buffer(a.vol + (size_t)sc.dir * a.vol_stride, span);
    const __amdgpu_buffer_rsrc_t cbuf = byte_buffer(a.cost, span);
    const int dp = sc.dp, len = sc.len, p0 = sc.p0;
    const int p_last = p0 + (len - 1) * dp;
    const uint32_t p1pk = (uint32_t)a.p1 * 0x10001u;
    const int p2 = a.p2;
    const uint32_t d0 = (uint32_t)(S * lane);

    uint64_t mm[RM];
    uint32_t s_off[PF], s_lw[PF];
    uint32_t cb[PF][S];
    auto load_meta = [&](int j, int pix) { mm[j] = scan_meta<WM>(a, pix); };
    auto load_cost = [&](int slot, int j) {
        s_off[slot] = __builtin_amdgcn_readfirstlane((uint32_t)mm[j]);
        s_lw[slot] = __builtin_amdgcn_readfirstlane((uint32_t)(mm[j] >> 32));
        const uint32_t lo = s_lw[slot] & 0xffffu, wm1 = (s_lw[slot] >> 16) - 1u;
#pragma unroll
        for (int t = 0; t < S; ++t)   // (unsigned) clamp: below or above the window -> inside it
            cb[slot][t] = __builtin_amdgcn_raw_buffer_load_b8(cbuf, min(d0 + t - lo, wm1), s_off[slot], 0);
    };
#pragma unroll
    for (int j = 0; j < RM; ++j) load_meta(j, j < len ? p0 + j * dp : p_last);
#pragma unroll
    for (int j = 0; j < PF; ++j) load_cost(j, j);

    uint32_t L[NP];
#pragma unroll
    for (int r = 0; r < NP; ++r) L[r] = 0u;   // zero predecessor: the first step gives L = C
    int m = 0;
    uint32_t shp = kInfPk, shn = kInfPk;   // lane-shift state (packed_update)
    int p = p0;
    auto step = [&](int tc) {
        const uint32_t lo = s_lw[tc] & 0xffffu, w = s_lw[tc] >> 16;
        const uint32_t off = s_off[tc];
        uint32_t sl[S];
        bool in[S];
#pragma unroll
        for (int t = 0; t < S; ++t) {
            sl[t] = d0 + t - lo;
            in[t] = sl[t] < w;
        }
        uint32_t c[NP];
#pragma unroll
        for (int r = 0; r < NP; ++r)   // two 16-bit halves packed by one byte permute
            c[r] = __builtin_amdgcn_perm(in[2 * r + 1] ? (uint32_t)cb[tc][2 * r + 1] : (uint32_t)kInf,
                                         in[2 * r] ? (uint32_t)cb[tc][2 * r] : (uint32_t)kInf, 0x05040100u);
        packed_update<64, NP>(L, c, m, p1pk, p2, shp, shn);
        // the window offset goes into the scalar offset; the per-lane offset
        // of a slot outside the window is pushed out of range
#pragma unroll
        for (int t = 0; t < S; ++t) {
            const uint32_t v = (t & 1) ? (L[t >> 1] >> 16) : L[t >> 1];
            __builtin_amdgcn_raw_buffer_store_b8((uint8_t)v, vol, in[t] ? sl[t] : kDropOffset, off, 0);
        }
    };

    int i = 0;
    for (; i + RM <= len; i += RM) {
#pragma unroll
        for (int u = 0; u < RM; ++u) {
            step(u % PF);
            load_cost(u % PF, (u + PF) % RM);
            load_meta(u, (i + u + RM < len) ? p + RM * dp : p_last);
            p += dp;
        }
    }
#pragma unroll
    for (int u = 0; u < RM; ++u) {
        if (i + u < len) {
            step(u % PF);
            if (u + PF < RM) load_cost(u % PF, u + PF);
            p += dp;
        }
    }
}

// ---- kernels ----
// Generic: every scanline through LDS rows (any D; ragged or full windows).
template <int G, int K, int WM, int PF>
__global__ __launch_bounds__(kBlock) void sgm_paths_lds_kernel(SgmLaunch a, int n_tasks) {
    constexpr int GPB = kBlock / G;
    __shared__ uint16_t lds[GPB][2][lds_row(G, K)];
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    const int task = blockIdx.x * GPB + grp;
    if (task >= n_tasks) return;
    const Scan sc = scan_of(task, a.w, a.h);
    lds_scanline<G, K, WM, PF>(a, sc, lane, lds[grp][0], lds[grp][1]);
}

// Ragged windows, every scanline on registers (one wave per scanline).
template <int K, int PF>
__global__ __launch_bounds__(kBlock) void sgm_paths_reg_kernel(SgmLaunch a, int n_tasks) {
    constexpr int WPB = kBlock / 64;
    __shared__ uint16_t lds[WPB][lds_row(64, K)];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
    const int task = (int)blockIdx.x * WPB + wv;
    if (task >= n_tasks) return;
    reg_scanline<K, kWinRagged, PF>(a, scan_of(task, a.w, a.h), lane, lds[wv]);
}

// Full range, D = 2*NP*G: every scanline on packed registers.
template <int G, int NP, int PF>
__global__ __launch_bounds__(kBlock) void sgm_paths_full_kernel(SgmLaunch a, int n_tasks) {
    constexpr int GPB = kBlock / G;
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    const int task = blockIdx.x * GPB + grp;
    if (task >= n_tasks) return;
    packed_scanline_full<G, NP, PF>(a, scan_of(task, a.w, a.h), lane);
}

// Ragged windows (SCHED names the ragged schedule, 0-2, so each has its own
// kernel symbol).  Blocks below n_win_blocks take the first n_win_tasks
// scanline tasks (the rows, longest first; or every task) one wave each on
// windowed packed registers (D <= 128*NP); the other blocks take the rest
// through LDS rows with GL lanes per scanline (work proportional to the
// window).
template <int SCHED, int NP, int GL, int K, int PF>
__global__ __launch_bounds__(kBlock) void sgm_paths_ragged_kernel(SgmLaunch a, int n_tasks,
                                                                   int n_win_tasks, int n_win_blocks) {
    if ((int)blockIdx.x < n_win_blocks) {
        // The long register scanlines are latency-bound, one wave each; the
        // higher issue priority lets them run at close to their own speed
        // while the LDS scanlines fill the remaining issue slots.
        __builtin_amdgcn_s_setprio(2);
        const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
        const int task = (int)blockIdx.x * (kBlock / 64) + wv;
        if (task >= n_win_tasks) return;
        win_scanline<NP, kWinRagged, PF, 4 * PF>(a, scan_of(task, a.w, a.h), lane);
    } else {
        __builtin_amdgcn_s_setprio(1);
        constexpr int GPB = kBlock / GL;
        __shared__ uint16_t lds[GPB][2][lds_row(GL, K)];
        const int grp = threadIdx.x / GL, lane = threadIdx.x % GL;
        const int task = n_win_tasks + (blockIdx.x - n_win_blocks) * GPB + grp;
        if (task >= n_tasks) return;
        // wide chunks on demand at 32 lanes (measured faster there; slower at 16 and 64)
        if (!a.wide_offsets && (uint64_t)a.w * (uint64_t)a.h < (1ull << 27) &&
            (uint64_t)kNumPaths * a.vol_stride < (1ull << 32))
            lds_scanline<GL, K, kWinRagged, PF, GL == 32, true>(a, scan_of(task, a.w, a.h), lane, lds[grp][0],
                                                                lds[grp][1]);
        else
            lds_scanline<GL, K, kWinRagged, PF, GL == 32>(a, scan_of(task, a.w, a.h), lane, lds[grp][0],
                                                          lds[grp][1]);
    }
}

// ------------------------------------------------------------------ grouped scanlines
// Frame slot layout (ragged windows on the grouped kernels, frames of F = 16
// or 32 slots).  Pixel p with window [lo, lo+w) owns the slots of
// disparities base .. base + span - 1 of each volume (costs and path costs):
//  - narrow (the window and its two neighbours, [lo-1, lo+w], fit F slots
//    from base = (lo-1) rounded down to an even number (16-slot frames of
//    schedule 8) or to a multiple of 4 (the others), base = 0 when lo = 0):
//    one frame, span = F, at byte offset q(p) = F p in a dense first region;
//  - wide (otherwise): base = lo & ~15, span = roundup16(lo + w) - base, on a
//    128-byte line in a second region (frame_off below).
// Every frame and span starts on a dword, so a lane reads and writes whole
// aligned pairs, quads of slots base + 4k, or 16-slot pieces.  Slots of
// [base, base+span) outside the window are padding: their cost byte is the
// marker 255 (a real cost is at most 62), which the path kernels turn into
// +infinity, and their path costs are never read as results.  The window
// word holds the address of slot lo, q(p) + lo - base, as in the ragged
// layout.  A volume needs at most w*h*(D+195) + 1 KB (quad_volume_bytes).
struct Frame {
    int base, span;
    bool narrow;
};
__device__ inline Frame frame_of(int lo, int w, int F, bool pairs = false) {
    const int bn = lo > 0 ? ((lo - 1) & (pairs ? ~1 : ~3)) : 0;
    if (lo - bn + w + 1 <= F) return Frame{bn, F, true};
    const int bw = lo & ~15;
    return Frame{bw, ((lo + w + 15) & ~15) - bw, false};
}
// Byte offset of pixel p's frame in a volume of n pixels: narrow frames of F
// slots (16 or 32) in a dense first region, F bytes per pixel (a frame never
// shares a line with a pixel it does not neighbour); wide spans after it,
// each on a 128-byte line boundary at the window offset plus 163 bytes per
// pixel rounded up, so two spans never overlap (consecutive ones are at least
// w + 36 apart, a span is at most w + 30) and a span of 256 slots is two
// whole lines.
__device__ inline uint32_t frame_off(bool narrow, uint32_t off, uint32_t p, uint32_t n, uint32_t F) {
    return narrow ? F * p : ((F * n + 127u) & ~127u) + ((off + 163u * p + 127u) & ~127u);
}
constexpr uint32_t kPadCost = 255;
// Costs of two slots (bytes b0 b1 of v, or b2 b3) as a packed pair, with the
// padding marker 255 raised to 255 + 0x4000: a slot carrying it stays above
// any in-window path cost + P2 (< 0x4000) and so acts as +infinity, and
// nothing overflows 16 bits (0x40ff + P2 + P1 < 0x8000).
__device__ inline uint32_t pad_inf(uint32_t c) {
    const u16x2 v = as_pk(c);
    const u16x2 one = __builtin_elementwise_sub_sat(v, u16x2{254, 254});
    return as_u32(v + (one << u16x2{14, 14}));
}

// bytes b0 b1 of v -> (b0 | b1 << 16), bytes b2 b3 -> (b2 | b3 << 16)
__device__ inline uint32_t bytes01(uint32_t v) { return __builtin_amdgcn_perm(0u, v, 0x0C010C00u); }
__device__ inline uint32_t bytes23(uint32_t v) { return __builtin_amdgcn_perm(0u, v, 0x0C030C02u); }
// low bytes of the two 16-bit halves of a and b -> a.lo, a.hi, b.lo, b.hi
__device__ inline uint32_t pack4(uint32_t a, uint32_t b) { return __builtin_amdgcn_perm(b, a, 0x06040200u); }

// Minimum over each 8-lane half of a 16-lane row, left in all its lanes.
__device__ inline int min8(int v) {
    v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0xB1, 0xF, 0xF, true));    // quad xor 1
    v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0x4E, 0xF, 0xF, true));    // quad xor 2
    v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0x141, 0xF, 0xF, true));   // row_half_mirror
    return v;
}
template <int G>
__device__ inline int small_group_min(int v) {
    if constexpr (G == 8) return min8(v);
    else return row_min16(v);
}

// Scanlines of the grouped kernel: the waves of each direction, in task
// order (rows, columns, diagonals), each taking NG = 64/G scanlines of one
// direction.  With `strided`, group g of wave j of a row or column direction
// takes scanline g*waves + j, so each wave mixes scanlines from every part
// of the image; diagonals take NG neighbouring scanlines (similar lengths).
struct GroupTasks {
    int first_dir;   // directions first_dir .. n_dirs-1 (wave_start[first_dir] = 0)
    int n_dirs;
    int strided;
    int n_scan[kNumPaths];
    int first_task[kNumPaths];
    int wave_start[kNumPaths + 1];
};

// Raw-buffer offset past any volume: loads there return zero and stores
// are dropped, for every access width (volumes stay below it).
constexpr uint32_t kDropWide = 0xffffff00u;

// Loads N dwords at byte offset `at` with the widest buffer loads.
template <int N>
__device__ inline void load_dwords(__amdgpu_buffer_rsrc_t buf, uint32_t at, uint32_t (&v)[N]) {
    if constexpr (N == 1) {
        v[0] = __builtin_amdgcn_raw_buffer_load_b32(buf, at, 0, 0);
    } else if constexpr (N == 2) {
        const u32x2 t = __builtin_amdgcn_raw_buffer_load_b64(buf, at, 0, 0);
        v[0] = t.x;
        v[1] = t.y;
    } else {
#pragma unroll
        for (int k = 0; k < N / 4; ++k) {
            const u32x4 t = __builtin_amdgcn_raw_buffer_load_b128(buf, at + 16u * k, 0, 0);
            v[4 * k] = t.x;
            v[4 * k + 1] = t.y;
            v[4 * k + 2] = t.z;
            v[4 * k + 3] = t.w;
        }
    }
}

// Grouped scanline kernel (ragged windows, frame layout with F = 2G).  A
// wave walks NG = 64/G scanlines of one direction at once, lane group g (G
// lanes) owning scanline g.  Each scanline keeps its previous pixel's path
// costs in a ping-pong pair of LDS rows indexed by absolute disparity
// (entry d + 2), as packed u16 pairs; every entry outside what the last
// step wrote is +infinity (a step erases the row it has read).
//  - A narrow pixel (window span <= F slots) is one step of its own group:
//    lane l owns slots B + 2l, B + 2l + 1 of the pixel's frame; the d-1, d,
//    d+1 predecessors are three aligned dword reads and two alignbits, and
//    padding slots carry +infinity from their cost marker, so no window
//    mask is needed.  The group minimum is a DPP reduction.
//  - A wide pixel (a longer span: at the sizes used here the pixels that
//    fall back to the full range) is done by the whole wave, lane L owning
//    the quad B + 4L .. B + 4L + 3, one wide pixel after another.  Its costs
//    were prefetched by its own group (DMAX/G bytes per lane, a dropped load
//    when narrow) and are handed to the wave through LDS.
// Every memory operation of a step is issued unconditionally (out-of-range
// offsets drop unused loads and stores), so the waits before a use leave
// the later prefetches in flight.  Window words are prefetched 2*PF steps
// ahead, costs PF steps ahead.  A zero predecessor over the first pixel's
// window makes the first step L = C.
template <int G, int DMAX, int PF>
__device__ inline void group_scanlines(const SgmLaunch& a, const GroupTasks& t, int gw) {
    constexpr int NG = 64 / G;
    constexpr int F = 2 * G;
    constexpr int ROW = DMAX + 2 * G + 8;
    constexpr int RM = 2 * PF;
    constexpr int WV = DMAX / G / 4;   // dwords of a wide pixel's costs per lane of its group
    static_assert(ROW % 4 == 0 && WV >= 1 && (WV <= 2 || WV % 4 == 0), "shapes");
    __shared__ __attribute__((aligned(16))) uint16_t rows_all[kBlock / 64][NG][2][ROW];
    __shared__ __attribute__((aligned(16))) uint32_t stage_all[kBlock / 64][DMAX / 4];
    const int lane = (int)(threadIdx.x & 63u);
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (gw >= t.wave_start[t.n_dirs]) return;
    int dir = t.first_dir;
    while (gw >= t.wave_start[dir + 1]) ++dir;
    const int wl = gw - t.wave_start[dir];
    const int nwav = t.wave_start[dir + 1] - t.wave_start[dir];
    const int g = lane / G, l = lane % G;
    const int j = (t.strided && dir < 4) ? g * nwav + wl : wl * NG + g;
    const bool has = j < t.n_scan[dir];
    Scan sc{dir, 0, 0, 0};
    if (has) sc = scan_of(t.first_task[dir] + j, a.w, a.h);
    const int len = has ? sc.len : 0;
    int nmax = 0;
#pragma unroll
    for (int k = 0; k < NG; ++k) nmax = max(nmax, __builtin_amdgcn_readlane(len, k * G));
    const int dp = sc.dp, p0 = sc.p0;
    const int p_last = len > 0 ? p0 + (len - 1) * dp : p0;

    const uint32_t cap = (uint32_t)a.vol_stride;
    const __amdgpu_buffer_rsrc_t cbuf = byte_buffer(a.cost, cap);
    const __amdgpu_buffer_rsrc_t vbuf = byte_buffer(a.vol + (size_t)dir * a.vol_stride, cap);
    const __amdgpu_buffer_rsrc_t mbuf = byte_buffer(a.meta, (uint32_t)a.w * (uint32_t)a.h * 8u);
    const uint32_t p1pk = (uint32_t)a.p1 * 0x10001u;
    const int p2 = a.p2;

    uint16_t (*rows)[2][ROW] = rows_all[wv];
    uint32_t* stage = stage_all[wv];
    uint32_t* myrow[2] = {reinterpret_cast<uint32_t*>(rows[g][0]), reinterpret_cast<uint32_t*>(rows[g][1])};

    // window words of steps 0 .. RM-1, then one RM steps ahead per step
    uint64_t mm[RM];
    const int q_lo = 8 * min(p0, p_last), q_hi = 8 * max(p0, p_last), dq = 8 * dp;
    int q_next = 8 * p0;
    auto next_meta = [&](int k) {
        mm[k] = __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(mbuf, min(max(q_next, q_lo), q_hi), 0, 0));
        q_next += dq;
    };
#pragma unroll
    for (int k = 0; k < RM; ++k) next_meta(k);

    uint32_t cst[PF];       // narrow: this lane's two cost bytes
    uint32_t wcs[PF][WV];   // wide: this lane's share of its group's pixel's costs
    auto load_costs = [&](int s, uint64_t mw, int i) {
        const int lo = meta_lo(mw), w = meta_w(mw);
        const Frame fr = frame_of(lo, w, F);
        const uint32_t o = meta_off(mw) - (uint32_t)(lo - fr.base);   // the frame's first slot
        const bool wide = i < len && !fr.narrow;
        cst[s] = __builtin_amdgcn_raw_buffer_load_b16(cbuf, o + 2u * (uint32_t)l, 0, 0);
        load_dwords<WV>(cbuf, wide ? o + 4u * WV * (uint32_t)l : kDropWide, wcs[s]);
    };
#pragma unroll
    for (int k = 0; k < PF; ++k) load_costs(k, mm[k], k);

    // every entry +infinity, then a zero predecessor over the first window
    {
        uint32_t* all = reinterpret_cast<uint32_t*>(rows_all[wv]);
        for (int e = lane; e < NG * ROW; e += 64) all[e] = kInfPk;
    }
    lds_order();
    int pmode = 0;      // what the previous step wrote: 0 nothing, 1 the narrow frame, 2 span [pb, pe)
    int pb = 0, pe = 0;
    int perase = 0;     // pmode 1: dword of this lane's pair
    if (has) {
        const int lo = meta_lo(mm[0]), w = meta_w(mm[0]);
        for (int s = l; s < w; s += G) rows[g][1][lo + s + 2] = 0;
        pmode = 2;
        pb = lo & ~3;   // the written entries' quads
        pe = (lo + w + 3) & ~3;
    }
    lds_order();
    int m = 0;

    auto step = [&](int i, int ti, int tc, int par) {
        const uint64_t mt = mm[ti];
        const int lo = meta_lo(mt), w = meta_w(mt);
        const Frame fr = frame_of(lo, w, F);
        const uint32_t o = meta_off(mt) - (uint32_t)(lo - fr.base);   // the frame's first slot
        const bool act = i < len;
        const int B = fr.base;
        const int span = fr.span;
        const bool nar = fr.narrow;
        uint32_t* prv = myrow[par ^ 1];
        uint32_t* cur = myrow[par];
        int m_new = m;
        const int qd = (B >> 1) + l;   // dword of entries B + 2l - 2, B + 2l - 1
        uint32_t Lm = 0;
        if (act && nar) {
            const uint32_t W0 = prv[qd], W1 = prv[qd + 1], W2 = prv[qd + 2];
            const uint32_t tt = pk_min(pk_min(pk_add(pk_min(align16(W1, W0), align16(W2, W1)), p1pk), W1),
                                       (uint32_t)(m + p2) * 0x10001u);
            Lm = pk_sub(pk_add(pad_inf(bytes01(cst[tc])), tt), (uint32_t)m * 0x10001u);
            cur[qd + 1] = Lm;
            m_new = small_group_min<G>((int)min(Lm & 0xffffu, Lm >> 16));
        }
        __builtin_amdgcn_raw_buffer_store_b16((uint16_t)__builtin_amdgcn_perm(0u, Lm, 0x0C0C0200u), vbuf,
                                              (act && nar) ? o + 2u * (uint32_t)l : kDropWide, 0, 0);
        // wide pixels, one after another by the whole wave
        uint64_t wb = __builtin_amdgcn_ballot_w64(act && !nar && l == 0);
        while (wb) {
            const int bit = (int)__builtin_ctzll(wb);
            wb &= wb - 1;
            const int gg = bit / G;
            // group gg hands its prefetched costs to the wave
            if (g == gg) {
#pragma unroll
                for (int v = 0; v < WV; ++v) stage[WV * l + v] = wcs[tc][v];
            }
            lds_order();
            const uint32_t cw = stage[lane < DMAX / 4 ? lane : 0];
            lds_order();
            const int lo_g = __builtin_amdgcn_readlane(lo, bit), w_g = __builtin_amdgcn_readlane(w, bit);
            const uint32_t o_g = (uint32_t)__builtin_amdgcn_readlane((int)o, bit);
            const int m_g = __builtin_amdgcn_readlane(m, bit);
            const int pm_g = __builtin_amdgcn_readlane(pmode, bit);
            const Frame fw = frame_of(lo_g, w_g, F);
            const int Bw = fw.base, Ew = fw.base + fw.span;
            const uint32_t* prg = reinterpret_cast<const uint32_t*>(rows[gg][par ^ 1]);
            uint32_t* cug = reinterpret_cast<uint32_t*>(rows[gg][par]);
            const int d = Bw + 4 * lane;
            const bool in = d < Ew;
            const int qw = in ? d >> 1 : 0;   // even: 8-byte aligned
            const u32x2 A = *reinterpret_cast<const u32x2*>(prg + qw);
            const u32x2 Bq = *reinterpret_cast<const u32x2*>(prg + qw + 2);
            const uint32_t XM = align16(Bq.x, A.y);
            const uint32_t m2 = (uint32_t)(m_g + p2) * 0x10001u, mg = (uint32_t)m_g * 0x10001u;
            const uint32_t t0 = pk_min(pk_min(pk_add(pk_min(align16(A.y, A.x), XM), p1pk), A.y), m2);
            const uint32_t t1 = pk_min(pk_min(pk_add(pk_min(XM, align16(Bq.y, Bq.x)), p1pk), Bq.x), m2);
            const uint32_t L0 = pk_sub(pk_add(pad_inf(bytes01(cw)), t0), mg);
            const uint32_t L1 = pk_sub(pk_add(pad_inf(bytes23(cw)), t1), mg);
            if (pm_g == 2) {
                // the previous step of this scanline was wide too: erase its span
                // here (every lane's reads above are issued before these writes)
                const int pb_g = __builtin_amdgcn_readlane(pb, bit), pe_g = __builtin_amdgcn_readlane(pe, bit);
                const int de = pb_g + 4 * lane;
                if (de < pe_g) {
                    uint32_t* pw = reinterpret_cast<uint32_t*>(rows[gg][par ^ 1]);
                    pw[(de >> 1) + 1] = kInfPk;
                    pw[(de >> 1) + 2] = kInfPk;
                }
            }
            if (in) {
                cug[qw + 1] = L0;
                cug[qw + 2] = L1;
            }
            __builtin_amdgcn_raw_buffer_store_b32(pack4(L0, L1), vbuf, in ? o_g + 4u * (uint32_t)lane : kDropWide,
                                                  0, 0);
            const uint32_t mm2 = pk_min(L0, L1);
            const int mw = group_min<64>(in ? (int)min(mm2 & 0xffffu, mm2 >> 16) : 0x7fffffff);
            if (g == gg) m_new = mw;
        }
        lds_order();
        // erase what the previous step wrote into the row read now (a wide
        // span already erased above when this step is wide too)
        if (pmode == 1) prv[perase] = kInfPk;
        uint64_t eb = __builtin_amdgcn_ballot_w64(pmode == 2 && !(act && !nar) && l == 0);
        while (eb) {
            const int bit = (int)__builtin_ctzll(eb);
            eb &= eb - 1;
            const int gg = bit / G;
            const int b0 = __builtin_amdgcn_readlane(pb, bit), e0 = __builtin_amdgcn_readlane(pe, bit);
            uint32_t* prg = reinterpret_cast<uint32_t*>(rows[gg][par ^ 1]);
            const int de = b0 + 4 * lane;
            if (de < e0) {
                prg[(de >> 1) + 1] = kInfPk;
                prg[(de >> 1) + 2] = kInfPk;
            }
        }
        lds_order();
        m = m_new;
        pmode = act ? (nar ? 1 : 2) : 0;
        pb = B;
        pe = B + span;
        perase = qd + 1;
    };

    int i = 0;
    for (; i + RM <= nmax; i += RM) {
#pragma unroll
        for (int u = 0; u < RM; ++u) {
            step(i + u, u, u % PF, u & 1);
            load_costs(u % PF, mm[(u + PF) % RM], i + u + PF);
            next_meta(u);
        }
    }
#pragma unroll
    for (int u = 0; u < RM; ++u) {
        if (i + u < nmax) {
            step(i + u, u, u % PF, u & 1);
            if (u + PF < RM) load_costs(u % PF, mm[u + PF], i + u + PF);
        }
    }
}

template <int G, int DMAX, int PF>
__global__ __launch_bounds__(kBlock) void sgm_paths_group_kernel(SgmLaunch a, GroupTasks t) {
    const int gw = (int)blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    // the rows (the first waves, 2*H-step... W-step chains) issue first when
    // their SIMD is shared: they set the kernel's length
    if (gw < t.wave_start[t.first_dir + 2 <= t.n_dirs && t.first_dir == 0 ? 2 : t.first_dir])
        __builtin_amdgcn_s_setprio(2);
    else
        __builtin_amdgcn_s_setprio(1);
    group_scanlines<G, DMAX, PF>(a, t, gw);
}

// Hybrid: blocks below n_row_blocks walk the image rows, one wave each on
// windowed packed registers over all disparities (branch-free steps, the
// shortest step latency for the longest scanlines, at a higher issue
// priority); the other blocks run the grouped scanlines of the columns and
// diagonals (t.first_dir = 2).
template <int G, int DMAX, int PF, int NP>
__global__ __launch_bounds__(kBlock) void sgm_paths_hybrid_kernel(SgmLaunch a, GroupTasks t, int n_row_blocks) {
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if ((int)blockIdx.x < n_row_blocks) {
        __builtin_amdgcn_s_setprio(2);
        const int task = (int)blockIdx.x * (kBlock / 64) + wv;
        if (task >= 2 * a.h) return;
        win_scanline<NP, kWinRagged, PF, 4 * PF>(a, scan_of(task, a.w, a.h), (int)(threadIdx.x & 63u));
    } else {
        __builtin_amdgcn_s_setprio(1);
        group_scanlines<G, DMAX, PF>(a, t, ((int)blockIdx.x - n_row_blocks) * (kBlock / 64) + wv);
    }
}

// Register-resident grouped scanlines (ragged windows, frame layout with
// 16-slot frames on even bases; schedule 8).  A wave walks four scanlines of
// one direction, lane group g (16 lanes, one DPP row) owning scanline g.  The
// previous pixel's path costs stay in registers, in one of two forms:
//  - narrow: one packed pair per lane, slots base + 2l, base + 2l + 1 of the
//    pixel's frame in lanes 0..7 (the window and its two neighbours lie
//    inside it, so the frame edges never need a value from outside); lanes
//    8..15 take padding costs, so their values stay above every path cost
//    + P2 and act as +infinity when a moved frame shifts them in;
//  - wide: NPW = DMAX/32 packed pairs per lane, the absolute slots
//    2*NPW*l .. 2*NPW*l + 2*NPW - 1 (the full range, as the full-range
//    kernel holds it), +infinity outside the window.
// A step is the recurrence on that form: the d-1 / d+1 neighbours are
// alignbits within a lane plus one DPP row shift across lanes, the minimum
// is a DPP row reduction.  Narrow groups update one register, wide groups
// NPW registers, all wide groups of the wave in the same pass.  A change of
// form goes through a per-group LDS row (absolute disparity, +infinity
// except during the change); a narrow frame that moves is shifted by a lane
// permute.  Costs: narrow pairs, and a wide pixel's 2*NPW bytes per lane
// (the out-of-span lanes read a run of padding markers at the end of the
// cost volume), prefetched PF steps ahead; window words 2*PF steps ahead.
// The first step uses a zero predecessor, so it gives L = C.
template <int DMAX, int PF>
__global__ __launch_bounds__(kBlock) void sgm_paths_regroup_kernel(SgmLaunch a, GroupTasks t) {
    constexpr int G = 16, NG = 4;
    constexpr int NPW = DMAX / 32;   // wide registers per lane
    constexpr int WD = NPW / 2;      // wide cost dwords per lane
    constexpr int RM = 2 * PF;
    constexpr int ROWD = DMAX / 2 + 16;   // LDS row dwords (entries 0 .. DMAX+31)
    static_assert(NPW == 2 || NPW == 4 || NPW == 8, "DMAX 64, 128 or 256");
    __shared__ __attribute__((aligned(16))) uint32_t rows_all[kBlock / 64][NG][ROWD];
    const int lane = (int)(threadIdx.x & 63u);
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int gw = (int)blockIdx.x * (kBlock / 64) + wv;
    if (gw >= t.wave_start[t.n_dirs]) return;
    int dir = t.first_dir;
    while (gw >= t.wave_start[dir + 1]) ++dir;
    const int wl = gw - t.wave_start[dir];
    const int nwav = t.wave_start[dir + 1] - t.wave_start[dir];
    const int g = lane / G, l = lane % G;
    const int j = (t.strided && dir < 4) ? g * nwav + wl : wl * NG + g;
    const bool has = j < t.n_scan[dir];
    Scan sc{dir, 0, 0, 0};
    if (has) sc = scan_of(t.first_task[dir] + j, a.w, a.h);
    const int len = has ? sc.len : 0;
    int nmax = 0;
#pragma unroll
    for (int k = 0; k < NG; ++k) nmax = max(nmax, __builtin_amdgcn_readlane(len, k * G));
    const int dp = sc.dp, p0 = sc.p0;

    const uint32_t cap = (uint32_t)a.vol_stride;
    const uint32_t pad_run = cap - 64u;   // 64 padding markers written by the cost pass
    const __amdgpu_buffer_rsrc_t cbuf = byte_buffer(a.cost, cap);
    const __amdgpu_buffer_rsrc_t vbuf = byte_buffer(a.vol + (size_t)dir * a.vol_stride, cap);
    const __amdgpu_buffer_rsrc_t mbuf = byte_buffer(a.frame, (uint32_t)a.w * (uint32_t)a.h * 8u);
    const uint32_t p1pk = (uint32_t)a.p1 * 0x10001u, p2pk = (uint32_t)a.p2 * 0x10001u;
    uint32_t* row = rows_all[wv][g];

    // window words of pixels 0 .. len-1; past the end of the scanline the
    // load is out of range and returns zero (form 0: inactive, no span), so
    // a finished or empty scanline never stores (an empty one sits on pixel 0)
    uint64_t mm[RM];
    const uint32_t dq = 8u * (uint32_t)dp;
    uint32_t q_next = 8u * (uint32_t)p0;
    auto next_meta = [&](int k, int i) {
        mm[k] = __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(mbuf, i < len ? q_next : kDropWide, 0, 0));
        q_next += dq;
    };
#pragma unroll
    for (int k = 0; k < RM; ++k) next_meta(k, k);

    uint32_t cst[PF];       // narrow: this lane's two cost bytes
    uint32_t wcs[PF][WD];   // wide: this lane's 2*NPW cost bytes
    // each pixel's frame, decoded once when its costs are requested: the
    // frame's first slot offset, and base | form << 16 (form: 0 inactive,
    // 1 narrow, 2 wide) | span << 18 | (this lane's wide slots inside the span) << 31
    uint32_t f_off[PF], f_inf[PF];
    const int d0 = 2 * NPW * l;   // this lane's first wide slot
    // mw: the pixel's frame word (frame offset | base << 32 | form << 48 | span << 50,
    // span 0 for a narrow frame)
    auto load_costs = [&](int s, uint64_t mw) {
        const uint32_t o = (uint32_t)mw, hi = (uint32_t)(mw >> 32);
        const int base = (int)(hi & 0xffffu);
        const bool in = (unsigned)(d0 - base) < (hi >> 18);
        f_off[s] = o;
        f_inf[s] = hi | ((uint32_t)in << 31);
        // a narrow frame is 16 slots, lanes 0..7; lanes 8..15 take padding markers
        cst[s] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(cbuf, l < 8 ? o + 2u * (uint32_t)l : kDropWide, 0, 0) |
                 (l < 8 ? 0u : 0xffffu);
        load_dwords<WD>(cbuf, in ? o + (uint32_t)(d0 - base) : pad_run, wcs[s]);
    };
#pragma unroll
    for (int k = 0; k < PF; ++k) load_costs(k, mm[k]);

    for (int e = l; e < ROWD; e += G) row[e] = kInfPk;
    lds_order();

    // state: the first step's predecessor is zero everywhere (L = C)
    uint32_t N = 0;
    uint32_t Wr[NPW];
#pragma unroll
    for (int k = 0; k < NPW; ++k) Wr[k] = 0;
    int m = 0;
    int mode = (int)((f_inf[0] >> 16) & 3u), Bp = (int)(f_inf[0] & 0xffffu);   // step 0: no change of form

    auto step = [&](int i, int ti, int tc) {
        const uint32_t o = f_off[tc];
        const int fbase = (int)(f_inf[tc] & 0xffffu);
        const int mc = (int)((f_inf[tc] >> 16) & 3u);
        const bool act = mc != 0;
        const bool in = f_inf[tc] >> 31;
        const bool nar = mc == 1;
        // changes of form or frame (the whole wave takes this branch only when a
        // group needs it); bitwise operators keep the test free of branches
        if (__builtin_amdgcn_ballot_w64(act & ((mode != mc) | (nar & (fbase != Bp)))) != 0) {
            const bool shift = mode == 1 && mc == 1 && fbase != Bp;
            const bool n2w = mode == 1 && mc == 2;
            const bool w2n = mode == 2 && mc == 1;
            const int src = l + (shift ? (fbase - Bp) >> 1 : 0);
            const uint32_t v = (uint32_t)__builtin_amdgcn_ds_bpermute(((lane & ~15) + (src & 15)) << 2, (int)N);
            if (shift) N = (unsigned)src < 16u ? v : kInfPk;
            if (n2w) row[(Bp >> 1) + l] = N;
            if (w2n) {
#pragma unroll
                for (int k = 0; k < NPW; ++k) row[NPW * l + k] = Wr[k];
            }
            lds_order();
            if (n2w) {
#pragma unroll
                for (int k = 0; k < NPW; ++k) Wr[k] = row[NPW * l + k];
            }
            if (w2n) N = row[(fbase >> 1) + l];
            lds_order();
            if (n2w) row[(Bp >> 1) + l] = kInfPk;
            if (w2n) {
#pragma unroll
                for (int k = 0; k < NPW; ++k) row[NPW * l + k] = kInfPk;
            }
            lds_order();
        }
        const uint32_t mp = __builtin_amdgcn_perm((uint32_t)m, (uint32_t)m, 0x05040100u);   // m in both halves
        const uint32_t m2 = pk_add(mp, p2pk);
        // the narrow update runs in every lane (one basic block with the
        // prefetches around it) and is kept where the pixel is narrow
        int m_new;
        {
            // the last slot of a narrow frame is always padding, so what the
            // group's last lane receives from above does not matter (the first
            // slot is padding too, except in a frame that starts at d = 0)
            const uint32_t prv = __builtin_amdgcn_update_dpp(kInfPk, N, 0x111, 0xF, 0xF, false);   // row_shr:1
            const uint32_t nxt = __builtin_amdgcn_mov_dpp(N, 0x101, 0xF, 0xF, true);                // row_shl:1
            const uint32_t tt = pk_min(pk_min(pk_add(pk_min(align16(N, prv), align16(nxt, N)), p1pk), N), m2);
            const uint32_t Nn = pk_sub(pk_add(pad_inf(bytes01(cst[tc])), tt), mp);
            const int mn = row_min16((int)min(Nn & 0xffffu, Nn >> 16));
            N = nar ? Nn : N;
            m_new = nar ? mn : m;
        }
        __builtin_amdgcn_raw_buffer_store_b16((uint16_t)__builtin_amdgcn_perm(0u, N, 0x0C0C0200u), vbuf,
                                              nar && l < 8 ? o + 2u * (uint32_t)l : kDropWide, 0, 0);
        if (__builtin_amdgcn_ballot_w64(mc == 2) != 0) {
            if (mc == 2) {
                const uint32_t prv = __builtin_amdgcn_update_dpp(kInfPk, Wr[NPW - 1], 0x111, 0xF, 0xF, false);
                const uint32_t nxt = __builtin_amdgcn_update_dpp(kInfPk, Wr[0], 0x101, 0xF, 0xF, false);
                // one operation over all registers at a time: no packed
                // operation waits on the one just before it
                uint32_t Ln[NPW];
#pragma unroll
                for (int k = 0; k < NPW; ++k)
                    Ln[k] = pk_min(align16(Wr[k], k > 0 ? Wr[k - 1] : prv), align16(k + 1 < NPW ? Wr[k + 1] : nxt, Wr[k]));
#pragma unroll
                for (int k = 0; k < NPW; ++k) Ln[k] = pk_add(Ln[k], p1pk);
#pragma unroll
                for (int k = 0; k < NPW; ++k) Ln[k] = pk_min(Ln[k], Wr[k]);
#pragma unroll
                for (int k = 0; k < NPW; ++k) Ln[k] = pk_min(Ln[k], m2);
#pragma unroll
                for (int k = 0; k < NPW; ++k)
                    Ln[k] = pk_sub(pk_add(pad_inf((k & 1) ? bytes23(wcs[tc][k >> 1]) : bytes01(wcs[tc][k >> 1])), Ln[k]), mp);
#pragma unroll
                for (int k = 0; k < NPW; ++k) Wr[k] = Ln[k];
                // pairwise minimum tree (independent operations between the dependent ones)
#pragma unroll
                for (int h = NPW / 2; h >= 1; h /= 2) {
#pragma unroll
                    for (int k = 0; k < h; ++k) Ln[k] = pk_min(Ln[k], Ln[k + h]);
                }
                m_new = row_min16((int)min(Ln[0] & 0xffffu, Ln[0] >> 16));
            }
            uint32_t pk[WD];
#pragma unroll
            for (int q = 0; q < WD; ++q) pk[q] = pack4(Wr[2 * q], Wr[2 * q + 1]);
            const uint32_t at = in ? o + (uint32_t)(d0 - fbase) : kDropWide;
            if constexpr (WD == 1) {
                __builtin_amdgcn_raw_buffer_store_b32(pk[0], vbuf, at, 0, 0);
            } else if constexpr (WD == 2) {
                __builtin_amdgcn_raw_buffer_store_b64(u32x2{pk[0], pk[1]}, vbuf, at, 0, 0);
            } else {
#pragma unroll
                for (int q = 0; q < WD / 4; ++q)
                    __builtin_amdgcn_raw_buffer_store_b128(u32x4{pk[4 * q], pk[4 * q + 1], pk[4 * q + 2], pk[4 * q + 3]},
                                                           vbuf, at + 16u * q, 0, 0);
            }
        }
        m = m_new;
        if (act) {
            mode = mc;
            Bp = fbase;
        }
    };

    int i = 0;
    for (; i + RM <= nmax; i += RM) {
#pragma unroll
        for (int u = 0; u < RM; ++u) {
            step(i + u, u, u % PF);
            load_costs(u % PF, mm[(u + PF) % RM]);
            next_meta(u, i + u + RM);
        }
    }
#pragma unroll
    for (int u = 0; u < RM; ++u) {
        if (i + u < nmax) {
            step(i + u, u, u % PF);
            if (u + PF < RM) load_costs(u % PF, mm[u + PF]);
        }
    }
}

// Costs in the frame layout.  One block per 64-pixel row segment: the
// segment's windows (written as window words with the frame offset), then
// all quads of its pixels' spans spread over the block's threads, one dword
// of four costs per quad: C(p, d) inside the window, the padding marker
// outside it.
__global__ __launch_bounds__(kBlock) void cost_frame_kernel(SgmLaunch a) {
    __shared__ uint64_t crs[kSeg + kMaxDisp];
    __shared__ uint64_t cls[kSeg];
    __shared__ int s_wide[kSeg + 1];   // the segment's wide pixels, then their count
    __shared__ int s_b[kSeg], s_lo[kSeg], s_w[kSeg];
    __shared__ uint32_t s_q[kSeg];
    const int W = a.w, D = a.win.max_disp;
    const uint32_t F = a.frame_pairs ? 16u : 2u * (uint32_t)a.quad;
    const int y = blockIdx.y, x0 = blockIdx.x * kSeg;
    const int base = x0 - (D - 1);
    const gmem<const uint64_t>* rowl = gptr(a.census_l + (size_t)y * W);
    const gmem<const uint64_t>* rowr = gptr(a.census_r + (size_t)y * W);
    if (threadIdx.x < 64) {
        const int i = (int)threadIdx.x, x = x0 + i;
        uint32_t nq = 0;
        if (x < W) {
            const int p = y * W + x;
            const int lo = gptr(a.win.lo)[p], hi = gptr(a.win.hi)[p];
            const uint32_t off = gptr(a.win.off)[p];
            const int w = hi - lo + 1;
            const Frame fr = frame_of(lo, w, (int)F, a.frame_pairs != 0);
            const uint32_t q = frame_off(fr.narrow, off, (uint32_t)p, (uint32_t)W * (uint32_t)a.h, F);
            // the window word's offset addresses slot lo (q + d - base for slot
            // d), as in the ragged layout, so every path kernel can read it
            gptr(a.meta)[p] = pack_meta(q + (uint32_t)(lo - fr.base), lo, w);
            gptr(a.frame)[p] = (uint64_t)q | ((uint64_t)fr.base << 32) | ((uint64_t)(fr.narrow ? 1 : 2) << 48) |
                               ((uint64_t)(fr.narrow ? 0 : fr.span) << 50);
            s_b[i] = fr.base;
            s_lo[i] = lo;
            s_w[i] = fr.narrow ? w : -w;   // negative: a wide pixel
            s_q[i] = q;
            nq = fr.narrow ? 0u : (uint32_t)(fr.span >> 2);
        } else {
            s_w[i] = 0;   // no pixel: nothing to write
        }
        const uint64_t wb = __builtin_amdgcn_ballot_w64(nq != 0u);
        if (nq != 0u) s_wide[__builtin_amdgcn_mbcnt_hi((uint32_t)(wb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)wb, 0u))] = i;
        if (i == 0) s_wide[kSeg] = __builtin_popcountll(wb);
    }
    for (int i = threadIdx.x; i < kSeg + D - 1; i += kBlock) {
        const int xr = base + i;
        crs[i] = (xr >= 0 && xr < W) ? rowr[xr] : 0ull;
    }
    for (int i = threadIdx.x; i < kSeg; i += kBlock) cls[i] = (x0 + i < W) ? rowl[x0 + i] : 0ull;
    __syncthreads();
    gmem<uint32_t>* cost = reinterpret_cast<gmem<uint32_t>*>(gptr(a.cost));
    // a run of 64 padding markers at the end of the volume, which lanes of
    // a wide pixel outside its span read as their costs
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 16)
        cost[((uint32_t)a.vol_stride - 64u) / 4u + threadIdx.x] = 0xffffffffu;
    // one quad of four costs: C(p, d) inside the window, the padding marker outside
    auto quad = [&](int i, int d, int lo, int w) {
        const int x = x0 + i;
        const uint64_t cl = cls[i];
        uint32_t word = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int dd = d + b;
            uint32_t c = kPadCost;
            if ((uint32_t)(dd - lo) < (uint32_t)w)
                c = x - dd >= 0 ? (uint32_t)__popcll(cl ^ crs[i + (D - 1) - dd]) : (uint32_t)kCensusBits;
            word |= c << (8 * b);
        }
        return word;
    };
    // narrow frames (F/4 quads each): four threads per pixel
    {
        const int i = (int)threadIdx.x >> 2, j = (int)threadIdx.x & 3;
        const int w = s_w[i];
        if (w > 0) {
            const int lo = s_lo[i], B = s_b[i];
            for (int qk = j; qk < (int)(F >> 2); qk += 4) cost[(s_q[i] >> 2) + (uint32_t)qk] = quad(i, B + 4 * qk, lo, w);
        }
    }
    // wide spans: one wave per pixel, a quad per lane
    const int n_wide = s_wide[kSeg];
    for (int v = (int)threadIdx.x >> 6; v < n_wide; v += kBlock / 64) {
        const int i = s_wide[v], lo = s_lo[i], w = -s_w[i], B = s_b[i];
        const int nq = (((lo + w + 15) & ~15) - B) >> 2;
        for (int qk = (int)threadIdx.x & 63; qk < nq; qk += 64)
            cost[(s_q[i] >> 2) + (uint32_t)qk] = quad(i, B + 4 * qk, lo, w);
    }
}

// Selection in the quad layout (same results as select_segment).  One block
// per 64-pixel row segment, wave v taking pixels 16v .. 16v+15: a pixel whose
// window span fits 16 slots is done by a group of 4 lanes (lane j owning the
// quad B + 4j, B the last slot at or below lo a whole number of quads from
// the frame's base), the wider ones four at a time by 16-lane groups (lane l
// owning the four quads B + 16l ..).  S is summed from the path volumes a dword (four slots) per
// direction and lane; the winner key (S << 9 | d) is a minimum over the
// group; the pixel's S row is staged in LDS for the parabola and the
// uncertainty walk of Eq. 9 (lane 0 of the group); each slot offers its key
// to right pixel x-d through the segment's LDS key array, flushed with one
// global atomicMin per touched right pixel.
template <int NPATH>
__global__ __launch_bounds__(kBlock) void select_quad_kernel(SgmLaunch a) {
    __shared__ uint32_t keyR[kSeg + kMaxDisp];
    __shared__ __attribute__((aligned(16))) uint16_t sS[kSeg][16];
    __shared__ __attribute__((aligned(16))) uint16_t sW[kBlock / 64][4][kMaxDisp + 8];
    __shared__ float s_sub[kSeg], s_var[kSeg];
    __shared__ int16_t s_wta[kSeg];
    const int W = a.w, D = a.win.max_disp;
    const int y = blockIdx.y, x0 = blockIdx.x * kSeg;
    const int base = x0 - (D - 1);
    const int lane = (int)(threadIdx.x & 63u);
    const int wv = (int)(threadIdx.x >> 6);
    for (int i = threadIdx.x; i < kSeg + D - 1; i += kBlock) keyR[i] = 0xffffffffu;
    const uint32_t cap = (uint32_t)a.vol_stride;
    __amdgpu_buffer_rsrc_t vb[NPATH];
#pragma unroll
    for (int r = 0; r < NPATH; ++r) vb[r] = byte_buffer(a.vol + (size_t)r * a.vol_stride, cap);
    __syncthreads();

    // S of the quad at byte offset `at`: pairs (d, d+1) and (d+2, d+3)
    auto sum_quad = [&](uint32_t at, uint32_t& s01, uint32_t& s23) {
        uint32_t v[NPATH];
#pragma unroll
        for (int r = 0; r < NPATH; ++r) v[r] = __builtin_amdgcn_raw_buffer_load_b32(vb[r], at, 0, 0);
        s01 = 0;
        s23 = 0;
#pragma unroll
        for (int r = 0; r < NPATH; ++r) {
            s01 = pk_add(s01, bytes01(v[r]));
            s23 = pk_add(s23, bytes23(v[r]));
        }
    };
    // winner key of one slot (S << 9 | d), or all ones outside the window
    // (keys are below 2^20; 0x7fffffff marks a slot outside the window)
    auto key_of = [&](uint32_t S, int d, int lo, int w) {
        return (uint32_t)(d - lo) < (uint32_t)w ? (int)((S << 9) | (uint32_t)d) : 0x7fffffff;
    };
    // parabola and walk on a staged S row (index 0 = disparity B)
    auto epilogue = [&](const uint16_t* row, int B, int lo, int w, int ds, int sb, int i) {
        const int hi = lo + w - 1;
        const int j0 = ds - B;
        float sub = (float)ds;
        if (ds > lo && ds < hi) {
            const int sa = row[j0 - 1], sc = row[j0 + 1];
            const int den = sa - 2 * sb + sc;
            if (den > 0) sub = (float)ds + (float)(sa - sc) / (float)(2 * den);
        }
        int acc = 0, n = 0;
        for (int j = 1; ds - j >= lo; ++j) {
            acc += (int)row[j0 - j] - sb;
            if (acc >= a.s_max) break;
            ++n;
        }
        acc = 0;
        for (int j = 1; ds + j <= hi; ++j) {
            acc += (int)row[j0 + j] - sb;
            if (acc >= a.s_max) break;
            ++n;
        }
        s_wta[i] = (int16_t)ds;
        s_sub[i] = sub;
        s_var[i] = (float)n;
    };
    // right-map offers of the four slots d .. d+3 of pixel i (column x)
    auto offer = [&](uint32_t s01, uint32_t s23, int d, int lo, int w, int x, int i) {
        const uint32_t S[4] = {s01 & 0xffffu, s01 >> 16, s23 & 0xffffu, s23 >> 16};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int dd = d + b;
            if ((uint32_t)(dd - lo) < (uint32_t)w && x - dd >= 0)
                atomicMin(&keyR[i + (D - 1) - dd], (S[b] << 9) | (uint32_t)dd);
        }
    };
    auto debug_agg = [&](uint32_t s01, uint32_t s23, int d, int lo, int w, int p) {
        if (!a.agg) return;
        const uint32_t off = gptr(a.win.off)[p];
        const uint32_t S[4] = {s01 & 0xffffu, s01 >> 16, s23 & 0xffffu, s23 >> 16};
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if ((uint32_t)(d + b - lo) < (uint32_t)w) gptr(a.agg)[off + (uint32_t)(d + b - lo)] = (uint16_t)S[b];
    };

    // narrow pixels: group gq of 4 lanes, pixel i = 16 wv + gq
    const int gq = lane >> 2, jq = lane & 3;
    const int i = 16 * wv + gq, x = x0 + i;
    const bool in_row = x < W;
    const int p = y * W + min(x, W - 1);
    const uint64_t mt = gptr(a.meta)[p];
    const int lo = meta_lo(mt), w = meta_w(mt);
    // B: the last slot at or below lo that is a whole number of quads from
    // the base of the pixel's frame or span (so its address is dword aligned;
    // 16-slot frames have even bases, the others multiples of 4)
    const int fb = frame_of(lo, w, a.frame_pairs ? 16 : 2 * a.quad, a.frame_pairs != 0).base;
    const int B = fb + ((lo - fb) & ~3);
    const uint32_t q = meta_off(mt) - (uint32_t)(lo - B);   // slot B
    const int span = (lo + w - B + 3) & ~3;
    const bool nar = span <= 16;
    if (in_row && nar) {
        const int d = B + 4 * jq;
        uint32_t s01 = 0xffffffffu, s23 = 0xffffffffu;
        int kb = 0x7fffffff;
        if (4 * jq < span) {
            sum_quad(q + 4u * (uint32_t)jq, s01, s23);
            kb = min(min(key_of(s01 & 0xffffu, d, lo, w), key_of(s01 >> 16, d + 1, lo, w)),
                     min(key_of(s23 & 0xffffu, d + 2, lo, w), key_of(s23 >> 16, d + 3, lo, w)));
            *reinterpret_cast<u32x2*>(&sS[i][4 * jq]) = u32x2{s01, s23};
            offer(s01, s23, d, lo, w, x, i);
            debug_agg(s01, s23, d, lo, w, p);
        }
        kb = min(kb, __builtin_amdgcn_update_dpp(0x7fffffff, kb, 0xB1, 0xF, 0xF, true));   // quad xor 1
        kb = min(kb, __builtin_amdgcn_update_dpp(0x7fffffff, kb, 0x4E, 0xF, 0xF, true));   // quad xor 2
        lds_order();
        if (jq == 0) epilogue(sS[i], B, lo, w, kb & 511, kb >> 9, i);
    }
    // wide pixels of this wave, four at a time: lane group g (16 lanes, one
    // DPP row) takes the g-th, lane l of the group the 16 slots
    // B + 16 l .. B + 16 l + 15 (four quads, one 16-byte load per direction;
    // a group without a pixel loads nothing)
    uint64_t wbits = __builtin_amdgcn_ballot_w64(in_row && !nar && jq == 0);
    const int gw16 = lane >> 4, l16 = lane & 15;
    uint16_t* row = sW[wv][gw16];
    while (wbits) {
        // the group's pixel: the gw16-th remaining wide pixel of the wave
        uint64_t m = wbits;
        for (int k2 = 0; k2 < gw16 && m; ++k2) m &= m - 1;
        const bool has = m != 0;
        const int bit = has ? (int)__builtin_ctzll(m) : 0;
        for (int k2 = 0; k2 < 4 && wbits; ++k2) wbits &= wbits - 1;
        const int lo_g = __builtin_amdgcn_ds_bpermute(bit << 2, lo), w_g = __builtin_amdgcn_ds_bpermute(bit << 2, w);
        const uint32_t q_g = (uint32_t)__builtin_amdgcn_ds_bpermute(bit << 2, (int)q);
        const int Bg = __builtin_amdgcn_ds_bpermute(bit << 2, B);
        const int ig = 16 * wv + (bit >> 2), xg = x0 + ig;
        const int Eg = Bg + ((lo_g + w_g - Bg + 3) & ~3);
        const int d0 = Bg + 16 * l16;
        const bool any = has && d0 < Eg;
        u32x4 v[NPATH];
#pragma unroll
        for (int r = 0; r < NPATH; ++r)
            v[r] = __builtin_amdgcn_raw_buffer_load_b128(vb[r], any ? q_g + 16u * (uint32_t)l16 : kDropOffset, 0, 0);
        int kb = 0x7fffffff;
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const int d = d0 + 4 * qq;
            if (any && d < Eg) {
                uint32_t s01 = 0, s23 = 0;
#pragma unroll
                for (int r = 0; r < NPATH; ++r) {
                    const uint32_t vq = qq == 0 ? v[r].x : qq == 1 ? v[r].y : qq == 2 ? v[r].z : v[r].w;
                    s01 = pk_add(s01, bytes01(vq));
                    s23 = pk_add(s23, bytes23(vq));
                }
                kb = min(kb, min(min(key_of(s01 & 0xffffu, d, lo_g, w_g), key_of(s01 >> 16, d + 1, lo_g, w_g)),
                                 min(key_of(s23 & 0xffffu, d + 2, lo_g, w_g), key_of(s23 >> 16, d + 3, lo_g, w_g))));
                *reinterpret_cast<u32x2*>(&row[16 * l16 + 4 * qq]) = u32x2{s01, s23};
                offer(s01, s23, d, lo_g, w_g, xg, ig);
                debug_agg(s01, s23, d, lo_g, w_g, y * W + xg);
            }
        }
        const int kw = row_min16(kb);
        lds_order();
        if (has && l16 == 0) epilogue(row, Bg, lo_g, w_g, kw & 511, kw >> 9, ig);
        lds_order();   // the next pixels rewrite the rows
    }
    __syncthreads();
    if (threadIdx.x < kSeg && x0 + (int)threadIdx.x < W) {
        const int ii = (int)threadIdx.x, pp = y * W + x0 + ii;
        gptr(a.disp_wta)[pp] = s_wta[ii];
        gptr(a.disp_sub)[pp] = s_sub[ii];
        gptr(a.var_meas)[pp] = s_var[ii];
        if (a.wta_raw) gptr(a.wta_raw)[pp] = s_wta[ii];
    }
    for (int ii = threadIdx.x; ii < kSeg + D - 1; ii += kBlock) {
        const int xr = base + ii;
        const uint32_t k = keyR[ii];
        if (xr >= 0 && xr < W && k != 0xffffffffu)
            __hip_atomic_fetch_min(gptr(a.key_r) + (size_t)y * W + xr, k, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Debug copy of nvol quad-layout volumes (stride src_stride) into the
// public ragged layout (entry offsets[p] + d - lo[p], stride dst_stride).
__global__ __launch_bounds__(kBlock) void copy_quad_slots_kernel(SgmLaunch a, const uint8_t* src, size_t src_stride,
                                                                 uint8_t* dst, size_t dst_stride, int nvol) {
    const int n = a.w * a.h;
    for (int p = (int)(blockIdx.x * kBlock + threadIdx.x); p < n; p += (int)(gridDim.x * kBlock)) {
        const int lo = a.win.lo[p], w = a.win.hi[p] - lo + 1;
        const uint32_t off = a.win.off[p];
        const uint32_t q = meta_off(a.meta[p]);   // slot lo
        for (int v = 0; v < nvol; ++v)
            for (int s = 0; s < w; ++s) dst[v * dst_stride + off + s] = src[v * src_stride + q + s];
    }
}

// ------------------------------------------------------------------ selection
template <int NPATH>
__device__ inline int sum_paths(const gmem<uint8_t>* const (&vols)[NPATH], uint32_t j) {
    int s = 0;
#pragma unroll
    for (int r = 0; r < NPATH; ++r) s += vols[r][j];
    return s;
}

// One block per 64-pixel row segment; a lane group of G lanes per pixel,
// lane l owning slots l + G*k.  The winner-takes-all key (S << 9 | d) is a
// group minimum (ties go to the smaller d).  Each slot also offers its key
// to right pixel x-d: first into an LDS array covering x0-(D-1) .. x0+63,
// then one global atomicMin per touched right pixel.  The pixel's S row is
// kept in LDS for the parabola and the uncertainty walk.  Results before the
// left-right check go to disp_wta / disp_sub / var_meas.
template <int G, int K, int WM, int NPATH>
__device__ inline void select_segment(const SgmLaunch& a, int seg, int y) {
    constexpr int GPB = kBlock / G;
    __shared__ uint32_t keyR[kSeg + kMaxDisp];
    __shared__ uint16_t sS_all[GPB][G * K];
    __shared__ float s_sub[kSeg], s_var[kSeg];   // results, stored coalesced at the end
    __shared__ int16_t s_wta[kSeg];
    const int W = a.w, D = a.win.max_disp;
    const int x0 = seg * kSeg;
    const int base = x0 - (D - 1);
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    uint16_t* sS = sS_all[grp];
    for (int i = threadIdx.x; i < kSeg + D - 1; i += kBlock) keyR[i] = 0xffffffffu;
    __syncthreads();
    const gmem<uint8_t>* __restrict__ vol = gptr(a.vol);
    const size_t stride = a.vol_stride;
    // one base per direction (uniform), so each load is a scalar base plus
    // the slot index, without a 64-bit address per load
    const gmem<uint8_t>* vols[NPATH];
#pragma unroll
    for (int r = 0; r < NPATH; ++r) vols[r] = vol + (size_t)r * stride;
    // Pixels are taken NB at a time: their windows, then the path costs of
    // their first PK chunks, are all requested before any is used, so a group
    // waits for two memory latencies per NB pixels instead of per pixel.
    constexpr int NPIX = kSeg / GPB;
    constexpr int NB = NPIX < 4 ? NPIX : 4;
    constexpr int PK = G == 16 ? 1 : (K < 2 ? K : 2);
    for (int t0 = 0; t0 < NPIX; t0 += NB) {
        uint64_t mt[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int x = min(x0 + grp + (t0 + b) * GPB, W - 1);   // past the row: not used
            mt[b] = scan_meta<WM>(a, y * W + x);
        }
        int c[NB][PK][NPATH];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const uint32_t o = meta_off(mt[b]);
            const int wb = meta_w(mt[b]);
#pragma unroll
            for (int k = 0; k < PK; ++k) {
                const uint32_t j = o + (uint32_t)min(lane + G * k, max(wb - 1, 0));
#pragma unroll
                for (int r = 0; r < NPATH; ++r) c[b][k][r] = vols[r][j];
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int i = grp + (t0 + b) * GPB;
            const int x = x0 + i;
            if (x >= W) continue;
            const int lo = meta_lo(mt[b]);
            const uint32_t off = meta_off(mt[b]);
            const int hi = lo + meta_w(mt[b]) - 1;
            const int w = hi - lo + 1;
            int kbest = 0x7fffffff;
            int S0 = 0;                      // this lane's S in chunk 0
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int s = lane + G * k;
                if (k > 0 && __builtin_amdgcn_ballot_w64(s < w) == 0) break;   // no group needs chunk k
                if (s < w) {
                    int S = 0;
                    if (k < PK) {
#pragma unroll
                        for (int r = 0; r < NPATH; ++r) S += c[b][k < PK ? k : 0][r];
                    } else {
                        S = sum_paths<NPATH>(vols, off + (uint32_t)s);
                    }
                    const int d = lo + s;
                    const int key = (S << 9) | d;
                    kbest = min(kbest, key);
                    sS[s] = (uint16_t)S;
                    if (k == 0) S0 = S;
                    if (a.agg) gptr(a.agg)[off + (uint32_t)s] = (uint16_t)S;
                    if (x - d >= 0) atomicMin(&keyR[i + (D - 1) - d], (uint32_t)key);
                }
            }
            lds_order();
            kbest = group_min<G>(kbest);
            const int ds = kbest & 511, sb = kbest >> 9;
            const int j0 = ds - lo;
            if (G == 16 && w <= 16) {
                // Window in one 16-lane row: the walk of Eq. 9 in parallel.  The
                // terms S - S_min are >= 0, so the running sums only grow and
                // the serial walk's count equals the number of slots whose sum
                // from the minimum outwards stays below S_max.  Q = inclusive
                // prefix sum of the terms over the row (DPP row shifts).
                const int e = lane < w ? S0 - sb : 0;
                int q = e;
                q += __builtin_amdgcn_update_dpp(0, q, 0x111, 0xF, 0xF, true);   // row_shr:1
                q += __builtin_amdgcn_update_dpp(0, q, 0x112, 0xF, 0xF, true);   // row_shr:2
                q += __builtin_amdgcn_update_dpp(0, q, 0x114, 0xF, 0xF, true);   // row_shr:4
                q += __builtin_amdgcn_update_dpp(0, q, 0x118, 0xF, 0xF, true);   // row_shr:8
                const int row0 = (int)(threadIdx.x & 63u) & ~15;
                const int qa = __builtin_amdgcn_ds_bpermute((row0 + max(j0 - 1, 0)) << 2, q);
                const int qb = __builtin_amdgcn_ds_bpermute((row0 + j0) << 2, q);
                const int sa = __builtin_amdgcn_ds_bpermute((row0 + max(j0 - 1, 0)) << 2, S0);
                const int sc = __builtin_amdgcn_ds_bpermute((row0 + min(j0 + 1, 15)) << 2, S0);
                const bool left = lane < j0 && qa - q + e < a.s_max;
                const bool right = lane > j0 && lane < w && q - qb < a.s_max;
                const uint32_t sh = (uint32_t)row0;
                const int n = __builtin_popcount((uint32_t)(__builtin_amdgcn_ballot_w64(left) >> sh) & 0xffffu) +
                              __builtin_popcount((uint32_t)(__builtin_amdgcn_ballot_w64(right) >> sh) & 0xffffu);
                if (lane == 0) {
                    float sub = (float)ds;
                    if (ds > lo && ds < hi) {
                        const int den = sa - 2 * sb + sc;
                        if (den > 0) sub = (float)ds + (float)(sa - sc) / (float)(2 * den);
                    }
                    s_wta[i] = (int16_t)ds;
                    s_sub[i] = sub;
                    s_var[i] = (float)n;
                }
            } else if (lane == 0) {
                float sub = (float)ds;
                if (ds > lo && ds < hi) {
                    const int sa = sS[j0 - 1], sc = sS[j0 + 1];
                    const int den = sa - 2 * sb + sc;
                    if (den > 0) sub = (float)ds + (float)(sa - sc) / (float)(2 * den);
                }
                int acc = 0, n = 0;
                for (int j = 1; j0 - j >= 0; ++j) {
                    acc += (int)sS[j0 - j] - sb;
                    if (acc >= a.s_max) break;
                    ++n;
                }
                acc = 0;
                for (int j = 1; j0 + j < w; ++j) {
                    acc += (int)sS[j0 + j] - sb;
                    if (acc >= a.s_max) break;
                    ++n;
                }
                s_wta[i] = (int16_t)ds;
                s_sub[i] = sub;
                s_var[i] = (float)n;
            }
            lds_order();
        }
    }
    __syncthreads();
    if (threadIdx.x < kSeg && x0 + (int)threadIdx.x < W) {
        const int i = (int)threadIdx.x, p = y * W + x0 + i;
        gptr(a.disp_wta)[p] = s_wta[i];
        gptr(a.disp_sub)[p] = s_sub[i];
        gptr(a.var_meas)[p] = s_var[i];
        if (a.wta_raw) gptr(a.wta_raw)[p] = s_wta[i];
    }
    for (int i = threadIdx.x; i < kSeg + D - 1; i += kBlock) {
        const int xr = base + i;
        const uint32_t k = keyR[i];
        if (xr >= 0 && xr < W && k != 0xffffffffu)
            __hip_atomic_fetch_min(gptr(a.key_r) + (size_t)y * W + xr, k, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <int G, int K, int WM, int NPATH>
__global__ __launch_bounds__(kBlock) void sgm_select_kernel(SgmLaunch a) {
    select_segment<G, K, WM, NPATH>(a, blockIdx.x, blockIdx.y);
}

// Right map and left-right check (in place on the selection's outputs).
__device__ inline void lr_pixel(const SgmLaunch& a, int p) {
    const gmem<uint32_t>* key_r = gptr(a.key_r);
    const uint32_t kr = key_r[p];
    if (a.disp_right) gptr(a.disp_right)[p] = kr == 0xffffffffu ? (int16_t)-1 : (int16_t)(kr & 511u);
    if (a.lr_tol < 0) return;
    const int x = p % a.w;
    const int ds = gptr(a.disp_wta)[p];
    bool ok = false;
    if (x - ds >= 0) {
        const uint32_t k2 = key_r[p - ds];
        if (k2 != 0xffffffffu) ok = abs(ds - (int)(k2 & 511u)) <= a.lr_tol;
    }
    if (!ok) {
        gptr(a.disp_wta)[p] = -1;
        gptr(a.disp_sub)[p] = -1.0f;
        gptr(a.var_meas)[p] = 0.0f;
    }
}

__global__ __launch_bounds__(kBlock) void sgm_lr_kernel(SgmLaunch a) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p < a.w * a.h) lr_pixel(a, p);
}

// Copies the first n bytes of a ragged volume, n = w*h*D for the full range
// or offsets[w*h] (read on the device) otherwise.
template <int WM>
__global__ __launch_bounds__(kBlock) void copy_slots_kernel(SgmLaunch a, const uint8_t* src,
                                                            uint8_t* dst) {
    const size_t n = WM == kWinFull ? (size_t)a.w * a.h * a.win.max_disp : (size_t)a.win.off[a.w * a.h];
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        dst[i] = src[i];
}

// ------------------------------------------------------------------ batched launches
// Many stereo pairs (any sizes, full or ragged windows, own D) in one launch
// per stage.  Each stage maps its blocks (or, for the paths, its scanline
// tasks) to (pair, local index) through prefix tables; scanline tasks are
// ordered rows, then columns, then diagonals across all pairs, so the
// longest chains start first.
__device__ inline int last_leq(const int* __restrict__ prefix, int n, int v) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ inline const SgmLaunch& pair_of(const BatchTables& t, int i) {
    return t.pairs[i];
}

__global__ __launch_bounds__(kBlock) void census_batch_kernel(BatchTables t) {
    const int i = last_leq(t.census_prefix, t.n, (int)blockIdx.x);
    const SgmLaunch a = pair_of(t, i);
    if (!a.active) return;
    const int local = (int)blockIdx.x - t.census_prefix[i];
    const int tiles_x = (a.w + kCtW - 1) / kCtW;
    const int tx = local % tiles_x, ty = local / tiles_x;
    if (blockIdx.z == 0)
        census_tile(a.left, a.w, a.h, a.pitch, const_cast<uint64_t*>(a.census_l), a.key_r, tx, ty);
    else
        census_tile(a.right, a.w, a.h, a.pitch, const_cast<uint64_t*>(a.census_r), nullptr, tx, ty);
}

__global__ __launch_bounds__(kBlock) void cost_batch_kernel(BatchTables t) {
    // the path pass that follows takes its scanline tasks from these counters
    if (blockIdx.x == 0 && threadIdx.x < (unsigned)kBatchShards)
        t.work[threadIdx.x * (kBatchShardStride / sizeof(unsigned))] = 0u;
    const int i = last_leq(t.seg_prefix, t.n, (int)blockIdx.x);
    const SgmLaunch a = pair_of(t, i);
    if (!a.active) return;
    const int local = (int)blockIdx.x - t.seg_prefix[i];
    const int segs_x = (a.w + kSeg - 1) / kSeg;
    cost_segment<16, kWinAny>(a, local % segs_x, local / segs_x);
}

// Batched scanlines, one block per 256/G tasks (the hardware dispatches
// blocks as earlier ones retire).  Task ranges start at multiples of 4
// (padded with idle tasks), so the lane groups of one wave always belong to
// the same pair and the pair's descriptor stays wave-uniform for any G.
template <int G, int K, int PF>
__global__ __launch_bounds__(kBlock) void paths_batch_kernel(BatchTables t) {
    constexpr int GPB = kBlock / G;
    __shared__ uint16_t lds[GPB][2][lds_row(G, K)];
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    const int task = (int)blockIdx.x * GPB + grp;
    if (task >= t.n_tasks) return;
    const int wave_task = __builtin_amdgcn_readfirstlane(task);
    const int r = __builtin_amdgcn_readfirstlane(last_leq(t.task_start, t.n_ranges, wave_task));
    const int i = __builtin_amdgcn_readfirstlane(t.task_pair[r]);
    const int rel = task - t.task_start[r];
    if (rel >= t.task_count[r]) return;                 // padding
    const SgmLaunch a = pair_of(t, i);
    if (!a.active) return;
    lds_scanline<G, K, kWinAny, PF, G == 32>(a, scan_of(t.task_local[r] + rel, a.w, a.h), lane, lds[grp][0],
                                              lds[grp][1]);
}

// Persistent: the grid holds only as many blocks as fit on the GPU at once
// (sized at plan creation).  The runs of 64/G scanline tasks are dealt to
// kBatchShards interleaved lists (run j to list j mod kBatchShards), each
// with its own work counter on its own 256-byte line (reset by the cost
// pass): wave v serves list v mod kBatchShards, takes its first run there
// without an atomic, then the list's next free run until none is left.
// Tasks are ordered rows, then columns, then diagonals, of every pair, so
// the longest scanlines start first and a wave that finishes early takes
// more work.  Same task layout and results as paths_batch_kernel.
template <int G, int K, int PF>
__global__ __launch_bounds__(kBlock) void paths_batch_persistent_kernel(BatchTables t) {
    constexpr int GPB = kBlock / G;
    constexpr int GPW = 64 / G;   // tasks per wave
    __shared__ uint16_t lds[GPB][2][lds_row(G, K)];
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    const int n_waves = (int)gridDim.x * (kBlock / 64);
    const int v = (int)blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int shard = v % kBatchShards;
    // waves serving this list, and this wave's static first pick in it
    const int served = n_waves / kBatchShards + (shard < n_waves % kBatchShards ? 1 : 0);
    int k = v / kBatchShards;
    unsigned* counter = t.work + shard * (kBatchShardStride / sizeof(unsigned));
    for (;;) {
        const int run = shard + kBatchShards * k;
        if (run * GPW >= t.n_tasks) break;
        const int task0 = run * GPW;
        const int task = task0 + grp % GPW;
        const int r = __builtin_amdgcn_readfirstlane(last_leq(t.task_start, t.n_ranges, task0));
        const int i = __builtin_amdgcn_readfirstlane(t.task_pair[r]);
        const int rel = task - t.task_start[r];
        const SgmLaunch a = pair_of(t, i);
        if (task < t.n_tasks && rel < t.task_count[r] && a.active)   // else padding or an inactive pair
            lds_scanline<G, K, kWinAny, PF, G == 32>(a, scan_of(t.task_local[r] + rel, a.w, a.h), lane,
                                                      lds[grp][0], lds[grp][1]);
        unsigned got = 0;
        if ((threadIdx.x & 63u) == 0u) got = atomicAdd(counter, 1u);
        k = served + (int)__builtin_amdgcn_readfirstlane(got);
    }
}

template <int K, int NPATH>
__global__ __launch_bounds__(kBlock) void select_batch_kernel(BatchTables t) {
    const int i = last_leq(t.seg_prefix, t.n, (int)blockIdx.x);
    const SgmLaunch a = pair_of(t, i);
    if (!a.active) return;
    const int local = (int)blockIdx.x - t.seg_prefix[i];
    const int segs_x = (a.w + kSeg - 1) / kSeg;
    select_segment<16, K, kWinAny, NPATH>(a, local % segs_x, local / segs_x);
}

__global__ __launch_bounds__(kBlock) void lr_batch_kernel(BatchTables t) {
    const int g = (int)blockIdx.x * kBlock + (int)threadIdx.x;
    if (g >= t.pix_prefix[t.n]) return;
    const int i = last_leq(t.pix_prefix, t.n, g);
    const SgmLaunch& a = pair_of(t, i);
    if (a.active) lr_pixel(a, g - t.pix_prefix[i]);
}

// Applies descriptor changes of a plan; one thread per change.
__global__ void plan_patch_kernel(SgmLaunch* pairs, PlanPatches p) {
    const int j = threadIdx.x;
    if (j >= p.n) return;
    const PlanPatch& c = p.p[j];
    gmem<SgmLaunch>* a = gptr(pairs + c.index);
    a->active = c.active;
    a->left = c.left;
    a->right = c.right;
    a->win.lo = c.lo;
    a->win.hi = c.hi;
    a->win.off = c.off;
}

// ------------------------------------------------------------------ SAD check
// Sum of |I_L - I_R| over a (2r+1)^2 patch at the pixel's disparity,
// coordinates clamped into the image; above sad_max the pixel is rejected
// like a left-right failure.  Integer arithmetic.
__global__ __launch_bounds__(kBlock) void sad_check_kernel(const uint8_t* __restrict__ left,
                                                           const uint8_t* __restrict__ right, int w,
                                                           int h, int pitch, int radius, int sad_max,
                                                           int16_t* disp_wta, float* disp_sub,
                                                           float* var_meas) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= w * h) return;
    const int d = gptr(disp_wta)[p];
    if (d < 0) return;
    const int x = p % w, y = p / w;
    const gmem<const uint8_t>* L = gptr(left);
    const gmem<const uint8_t>* R = gptr(right);
    int sad = 0;
    for (int j = -radius; j <= radius; ++j) {
        const size_t row = (size_t)min(max(y + j, 0), h - 1) * pitch;
        for (int i = -radius; i <= radius; ++i) {
            const int xl = min(max(x + i, 0), w - 1), xr = min(max(x + i - d, 0), w - 1);
            sad += abs((int)L[row + xl] - (int)R[row + xr]);
        }
    }
    if (sad > sad_max) {
        gptr(disp_wta)[p] = -1;
        gptr(disp_sub)[p] = -1.0f;
        gptr(var_meas)[p] = 0.0f;
    }
}

// ------------------------------------------------------------------ prediction LR check
// A left prediction d >= 0 survives when the warped right map at
// xr = x - floorf(d + 0.5f) holds e >= 0 with |e - d| <= tol (float32);
// otherwise (-1, 0).  In place.
__global__ __launch_bounds__(kBlock) void lr_check_prediction_kernel(float* d_pred, float* p_pred,
                                                                     const float* d_right, int w,
                                                                     int h, float tol) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= w * h) return;
    const float d = gptr(d_pred)[p];
    if (!(d >= 0.0f)) return;
    const int x = p % w;
    /* d >= w points left of the image anyway; the test keeps the cast in range */
    const int xr = d < (float)w ? x - (int)floorf(d + 0.5f) : -1;
    bool ok = false;
    if (xr >= 0) {
        const float e = gptr(d_right)[p - (x - xr)];
        ok = e >= 0.0f && fabsf(e - d) <= tol;
    }
    if (!ok) {
        gptr(d_pred)[p] = -1.0f;
        gptr(p_pred)[p] = 0.0f;
    }
}

__global__ __launch_bounds__(kBlock) void disparity_to_float_kernel(const int16_t* d, float* out,
                                                                    int n) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) gptr(out)[i] = (float)gptr(d)[i];
}

// ------------------------------------------------------------------ warp
struct Mat4 {
    float m[16];
};
struct Mat4d {
    double m[16];
};

__global__ __launch_bounds__(kBlock) void fill_u64_kernel(unsigned long long* z, size_t n) {
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) z[i] = ~0ull;
}

// Decision pass, float32 in the documented order: the target pixel and the
// key (~bits(d') << 32 | source index), so atomicMin keeps the largest d'
// and, on equal d', the smaller source index, independent of thread order.
__global__ __launch_bounds__(kBlock) void warp_scatter_kernel(const float* __restrict__ d_prev,
                                                              int w, int h, Mat4 H,
                                                              unsigned long long* zbuf) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= w * h) return;
    const float d = d_prev[i];
    if (!(d > 0.0f)) return;
    const float xf = (float)(i % w), yf = (float)(i / w);
    const float* m = H.m;
    const float o0 = ((m[0] * xf + m[1] * yf) + m[2] * d) + m[3];
    const float o1 = ((m[4] * xf + m[5] * yf) + m[6] * d) + m[7];
    const float o3 = ((m[12] * xf + m[13] * yf) + m[14] * d) + m[15];
    if (!(o3 > 0.0f)) return;
    const float xp = o0 / o3, yp = o1 / o3, dp = d / o3;
    const float vx = xp + 0.5f, vy = yp + 0.5f;
    if (!(vx >= 0.0f) || !(vx < (float)w) || !(vy >= 0.0f) || !(vy < (float)h)) return;
    const int xi = (int)floorf(vx), yi = (int)floorf(vy);
    const unsigned long long key =
        ((unsigned long long)(0xffffffffu - __float_as_uint(dp)) << 32) | (unsigned)i;
    atomicMin(&zbuf[(size_t)yi * w + xi], key);
}

// Value pass: the winner's d' = d/omega_3 and p' = (d'/d)^2 p + q in double
// (row 2 of H is exactly (0,0,1,0), so omega_2 = d), rounded once to float;
// a target without a winner is (-1, 0).
__device__ inline void warp_value(unsigned long long k, const float* __restrict__ d_prev,
                                  const float* __restrict__ p_prev, int w, const Mat4d& H, double q,
                                  float& d_out, float& p_out) {
    if (k == ~0ull) {
        d_out = -1.0f;
        p_out = 0.0f;
        return;
    }
    const int src = (int)(uint32_t)k;
    const double x = (double)(src % w), y = (double)(src / w);
    const double d = (double)gptr(d_prev)[src], p = (double)gptr(p_prev)[src];
    const double* m = H.m;
    const double o3 = m[12] * x + m[13] * y + m[14] * d + m[15];
    const double dn = d / o3;
    const double phi = dn / d;
    d_out = (float)dn;
    p_out = (float)(phi * phi * p + q);
}

__global__ __launch_bounds__(kBlock) void warp_decode_kernel(const unsigned long long* zbuf,
                                                             const float* __restrict__ d_prev,
                                                             const float* __restrict__ p_prev,
                                                             int w, int n, Mat4d H, double q,
                                                             float* __restrict__ d_pred,
                                                             float* __restrict__ p_pred) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    float d, p;
    warp_value(gptr(zbuf)[i], d_prev, p_prev, w, H, q, d, p);
    gptr(d_pred)[i] = d;
    gptr(p_pred)[i] = p;
}

// ------------------------------------------------------------------ refinement
// The three refinement passes in one kernel.  Edge rejection: a valid
// prediction is dropped when a valid pixel of its 3x3 neighbourhood differs
// from it by more than edge_tol (edge_tol < 0: plain copy).  One-pixel
// "zoom" hole filling along rows, then along columns: an invalid pixel
// between two valid neighbours with |a - b| < fill_tol takes their means
// ((a + b) * 0.5f is the correctly rounded mean: the sum is rounded once and
// halving is exact); each pass reads the previous pass's result.  A block
// stages its 64x4 output tile with a halo of two pixels, runs the edge test
// on the tile plus one pixel, the row fill on the tile plus one row, and the
// column fill on the tile, each from the previous pass's values in LDS.
// Pixels outside the image are staged as invalid, which the edge test skips
// as it skips invalid neighbours; the fills never read them.
constexpr int kRfW = 64, kRfH = kBlock / kRfW;

// Input of the refinement: a predicted map (d_in, p_in), or, with
// FROM_ZBUF, the warp's z-buffer decoded on the fly (warp_value), so the
// prediction itself never goes through memory.
struct RefineSrc {
    const float* d_in;
    const float* p_in;
    const unsigned long long* zbuf;   // FROM_ZBUF: winners; d_in / p_in are the previous map
    Mat4d H;
    double q;
};

template <bool FROM_ZBUF>
__global__ __launch_bounds__(kBlock) void refine_fused_kernel(RefineSrc src, int w, int h,
                                                              float edge_tol, float fill_tol,
                                                              float* __restrict__ d_out,
                                                              float* __restrict__ p_out) {
    constexpr int AW = kRfW + 4, AH = kRfH + 4;   // input, halo 2
    constexpr int EW = kRfW + 2, EH = kRfH + 2;   // after the edge test, halo 1
    __shared__ float sd[AH][AW], sp[AH][AW], ed[EH][EW], ep[EH][EW], hd[EH][kRfW], hp[EH][kRfW];
    const int x0 = blockIdx.x * kRfW, y0 = blockIdx.y * kRfH;
    const gmem<const float>* gd = gptr(src.d_in);
    const gmem<const float>* gp = gptr(src.p_in);
    for (int t = threadIdx.x; t < AW * AH; t += kBlock) {
        const int r = t / AW, c = t - r * AW;
        const int gx = x0 + c - 2, gy = y0 + r - 2;
        const bool in = gx >= 0 && gx < w && gy >= 0 && gy < h;
        float dv = -1.0f, pv = 0.0f;
        if (in) {
            const size_t i = (size_t)gy * w + gx;
            if (FROM_ZBUF) {
                warp_value(gptr(src.zbuf)[i], src.d_in, src.p_in, w, src.H, src.q, dv, pv);
            } else {
                dv = gd[i];
                pv = gp[i];
            }
        }
        sd[r][c] = dv;
        sp[r][c] = pv;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < EW * EH; t += kBlock) {
        const int r = t / EW, c = t - r * EW;
        const float d = sd[r + 1][c + 1];
        bool keep = d >= 0.0f;
        if (keep && edge_tol >= 0.0f) {
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    const float e = sd[r + dy][c + dx];
                    if (e >= 0.0f && fabsf(d - e) > edge_tol) keep = false;
                }
        }
        ed[r][c] = keep ? d : -1.0f;
        ep[r][c] = keep ? sp[r + 1][c + 1] : 0.0f;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kRfW * EH; t += kBlock) {
        const int r = t / kRfW, c = t - r * kRfW;
        const int gx = x0 + c;
        float d = ed[r][c + 1], p = ep[r][c + 1];
        if (d < 0.0f && gx >= 1 && gx + 1 < w) {
            const float a = ed[r][c], b = ed[r][c + 2];
            if (a >= 0.0f && b >= 0.0f && fabsf(a - b) < fill_tol) {
                d = (a + b) * 0.5f;
                p = (ep[r][c] + ep[r][c + 2]) * 0.5f;
            }
        }
        hd[r][c] = d;
        hp[r][c] = p;
    }
    __syncthreads();
    const int c = threadIdx.x % kRfW, r = threadIdx.x / kRfW;
    const int gx = x0 + c, gy = y0 + r;
    if (gx >= w || gy >= h) return;
    float d = hd[r + 1][c], p = hp[r + 1][c];
    if (d < 0.0f && gy >= 1 && gy + 1 < h) {
        const float a = hd[r][c], b = hd[r + 2][c];
        if (a >= 0.0f && b >= 0.0f && fabsf(a - b) < fill_tol) {
            d = (a + b) * 0.5f;
            p = (hp[r][c] + hp[r + 2][c]) * 0.5f;
        }
    }
    gptr(d_out)[(size_t)gy * w + gx] = d;
    gptr(p_out)[(size_t)gy * w + gx] = p;
}

// ------------------------------------------------------------------ Kalman
__global__ __launch_bounds__(kBlock) void kalman_kernel(const float* d_pred, const float* p_pred,
                                                        const float* z, const float* r, int n,
                                                        int keep, float* d_out, float* p_out) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float dp = d_pred[i], pp = p_pred[i], zz = z[i], rr = r[i];
    const bool pv = dp >= 0.0f && pp > 0.0f;
    const bool mv = zz >= 0.0f && rr >= 0.0f;
    float d, p;
    if (pv && mv) {
        const float K = pp / (pp + rr);
        d = dp + K * (zz - dp);
        p = (1.0f - K) * pp;
    } else if (mv) {
        d = zz;
        p = rr;
    } else if (pv && keep) {
        d = dp;
        p = pp;
    } else {
        d = -1.0f;
        p = 0.0f;
    }
    d_out[i] = d;
    p_out[i] = p;
}

inline unsigned grid_for(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_census(const uint8_t* img, int w, int h, int pitch, uint64_t* out,
                         hipStream_t s) {
    dim3 grid((w + kCtW - 1) / kCtW, (h + kCtH - 1) / kCtH, 1);
    census_kernel<<<grid, kBlock, 0, s>>>(img, img, w, h, pitch, out, out, nullptr);
    return hipGetLastError();
}

hipError_t launch_census_pair(const uint8_t* left, const uint8_t* right, int w, int h, int pitch,
                              uint64_t* out_l, uint64_t* out_r, uint32_t* clear, hipStream_t s) {
    dim3 grid((w + kCtW - 1) / kCtW, (h + kCtH - 1) / kCtH, 2);
    census_kernel<<<grid, kBlock, 0, s>>>(left, right, w, h, pitch, out_l, out_r, clear);
    return hipGetLastError();
}

size_t quad_volume_bytes(int w, int h, int D) {
    // at most 32 bytes per pixel of narrow frames, then the line-aligned wide spans
    // (below w*h*(D + 163) + 512 bytes), then 64 marker bytes; below the drop offset
    const unsigned long long n = (unsigned long long)w * (unsigned long long)h;
    const unsigned long long a = (32ull * n + 127ull) & ~127ull;
    const unsigned long long b = (a + n * (unsigned long long)(D + 163) + 512ull + 64ull + 255ull) & ~255ull;
    return b < (unsigned long long)kDropWide ? (size_t)b : 0;
}

hipError_t launch_sgm_cost(const SgmLaunch& a, hipStream_t s) {
    dim3 grid((a.w + kSeg - 1) / kSeg, a.h);
    if (a.quad)
        cost_frame_kernel<<<grid, kBlock, 0, s>>>(a);
    else if (a.win.lo == nullptr)
        cost_kernel<64, kWinFull><<<grid, kBlock, 0, s>>>(a);
    else
        cost_kernel<16, kWinRagged><<<grid, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_sgm_paths(const SgmLaunch& a, hipStream_t s) {
    const int n_tasks = 2 * a.h + 2 * a.w + (a.n_paths == 4 ? 0 : 4 * (a.w + a.h - 1));
    const int D = a.win.max_disp;
    const bool full = a.win.lo == nullptr;
    auto blocks = [&](int n, int G) { return (n + kBlock / G - 1) / (kBlock / G); };
    if (full) {
        // packed kernel where D = 2 * NP * G, LDS kernel otherwise
        const int g = a.full_group;
#define EGOSGM_FULL(GG, NN) \
    sgm_paths_full_kernel<GG, NN, 8><<<blocks(n_tasks, GG), kBlock, 0, s>>>(a, n_tasks)
#define EGOSGM_LDSF(GG, KK) \
    sgm_paths_lds_kernel<GG, KK, kWinFull, 4><<<blocks(n_tasks, GG), kBlock, 0, s>>>(a, n_tasks)
        if (D == 64) {
            if (g == 32) EGOSGM_FULL(32, 1); else EGOSGM_FULL(16, 2);
        } else if (D == 128) {
            if (g == 16) EGOSGM_FULL(16, 4); else if (g == 64) EGOSGM_FULL(64, 1); else EGOSGM_FULL(32, 2);
        } else if (D == 256) {
            if (g == 16) EGOSGM_FULL(16, 8); else if (g == 64) EGOSGM_FULL(64, 2); else EGOSGM_FULL(32, 4);
        } else if (D <= 64) {
            EGOSGM_LDSF(64, 1);
        } else if (D <= 128) {
            EGOSGM_LDSF(64, 2);
        } else {
            EGOSGM_LDSF(64, 4);
        }
#undef EGOSGM_FULL
#undef EGOSGM_LDSF
        return hipGetLastError();
    }
    // ragged: schedule 0 every scanline through LDS rows, 1 the rows on
    // windowed registers and the rest through LDS, 2 every scanline on
    // windowed registers, 3 every scanline on relative registers, 4 and 5
    // grouped scanlines (8 or 16 lanes each, quad layout).  The LDS part of
    // schedules 0-2 takes its lanes per scanline from the tuning.
    const int g = a.ragged_group;
    const int sched = a.ragged_schedule;
    if (a.quad) {
        // schedules 6, 7: the rows on windowed registers, the rest grouped;
        // 8: grouped scanlines with register-resident state (16 lanes)
        const bool hybrid = sched == 6 || sched == 7;
        const int G = a.quad, NG = 64 / G;
        GroupTasks t{};
        t.first_dir = hybrid ? 2 : 0;
        t.n_dirs = a.n_paths == 4 ? 4 : 8;
        t.strided = 1;
        const int W = a.w, H = a.h;
        const int ns[kNumPaths] = {H, H, W, W, W + H - 1, W + H - 1, W + H - 1, W + H - 1};
        int task = 0;
        for (int r = 0; r < t.first_dir; ++r) task += ns[r];
        t.wave_start[t.first_dir] = 0;
        for (int r = t.first_dir; r < t.n_dirs; ++r) {
            t.n_scan[r] = ns[r];
            t.first_task[r] = task;
            task += ns[r];
            t.wave_start[r + 1] = t.wave_start[r] + (ns[r] + NG - 1) / NG;
        }
        const unsigned nb = (unsigned)((t.wave_start[t.n_dirs] + kBlock / 64 - 1) / (kBlock / 64));
        if (sched == 8) {
            // D = 256: costs six steps ahead (162 VGPRs, three waves per SIMD)
            if (D <= 64) sgm_paths_regroup_kernel<64, 4><<<nb, kBlock, 0, s>>>(a, t);
            else if (D <= 128) sgm_paths_regroup_kernel<128, 4><<<nb, kBlock, 0, s>>>(a, t);
            else sgm_paths_regroup_kernel<256, 6><<<nb, kBlock, 0, s>>>(a, t);
            return hipGetLastError();
        }
        if (hybrid) {
            const int nrb = (2 * H + kBlock / 64 - 1) / (kBlock / 64);
#define EGOSGM_HYB(GG)                                                                                     \
    do {                                                                                                   \
        if (D <= 64) sgm_paths_hybrid_kernel<GG, 64, 4, 1><<<nb + nrb, kBlock, 0, s>>>(a, t, nrb);          \
        else if (D <= 128) sgm_paths_hybrid_kernel<GG, 128, 4, 1><<<nb + nrb, kBlock, 0, s>>>(a, t, nrb);   \
        else sgm_paths_hybrid_kernel<GG, 256, 4, 2><<<nb + nrb, kBlock, 0, s>>>(a, t, nrb);                 \
    } while (0)
            if (G == 16) EGOSGM_HYB(16); else EGOSGM_HYB(8);
#undef EGOSGM_HYB
            return hipGetLastError();
        }
#define EGOSGM_GRP(GG, PP)                                                                   \
    do {                                                                                     \
        if (D <= 64) sgm_paths_group_kernel<GG, 64, PP><<<nb, kBlock, 0, s>>>(a, t);          \
        else if (D <= 128) sgm_paths_group_kernel<GG, 128, PP><<<nb, kBlock, 0, s>>>(a, t);   \
        else sgm_paths_group_kernel<GG, 256, PP><<<nb, kBlock, 0, s>>>(a, t);                 \
    } while (0)
        if (G == 16) EGOSGM_GRP(16, 4); else EGOSGM_GRP(8, 4);
#undef EGOSGM_GRP
        return hipGetLastError();
    }
    if (sched == 3) {
        const unsigned nb = blocks(n_tasks, 64);
        if (D <= 64) sgm_paths_reg_kernel<1, 4><<<nb, kBlock, 0, s>>>(a, n_tasks);
        else if (D <= 128) sgm_paths_reg_kernel<2, 4><<<nb, kBlock, 0, s>>>(a, n_tasks);
        else sgm_paths_reg_kernel<4, 4><<<nb, kBlock, 0, s>>>(a, n_tasks);
        return hipGetLastError();
    }
    const int n_win = sched == 0 ? 0 : (sched == 1 ? 2 * a.h : n_tasks);
#define EGOSGM_RAG(NP, GL, KK)                                                                      \
    do {                                                                                            \
        const int nb_w = blocks(n_win, 64);                                                         \
        const int nb = nb_w + blocks(n_tasks - n_win, GL);                                          \
        if (sched == 0)                                                                             \
            sgm_paths_ragged_kernel<0, NP, GL, KK, 4><<<nb, kBlock, 0, s>>>(a, n_tasks, n_win, nb_w); \
        else if (sched == 1)                                                                        \
            sgm_paths_ragged_kernel<1, NP, GL, KK, 4><<<nb, kBlock, 0, s>>>(a, n_tasks, n_win, nb_w); \
        else                                                                                        \
            sgm_paths_ragged_kernel<2, NP, GL, KK, 4><<<nb, kBlock, 0, s>>>(a, n_tasks, n_win, nb_w); \
    } while (0)
    if (D <= 64) {
        if (g == 16) EGOSGM_RAG(1, 16, 4); else if (g == 64) EGOSGM_RAG(1, 64, 1); else EGOSGM_RAG(1, 32, 2);
    } else if (D <= 128) {
        if (g == 16) EGOSGM_RAG(1, 16, 8); else if (g == 32) EGOSGM_RAG(1, 32, 4); else EGOSGM_RAG(1, 64, 2);
    } else {
        if (g == 16) EGOSGM_RAG(2, 16, 16); else if (g == 32) EGOSGM_RAG(2, 32, 8); else EGOSGM_RAG(2, 64, 4);
    }
#undef EGOSGM_RAG
    return hipGetLastError();
}

hipError_t launch_sgm_select(const SgmLaunch& a, hipStream_t s) {
    const int D = a.win.max_disp;
    const bool full = a.win.lo == nullptr;
    dim3 grid((a.w + kSeg - 1) / kSeg, a.h);
#define EGOSGM_SEL(GG, KK, FF)                                            \
    do {                                                                  \
        if (a.n_paths == 4) sgm_select_kernel<GG, KK, FF, 4><<<grid, kBlock, 0, s>>>(a); \
        else sgm_select_kernel<GG, KK, FF, 8><<<grid, kBlock, 0, s>>>(a);               \
    } while (0)
    if (a.quad) {
        if (a.n_paths == 4) select_quad_kernel<4><<<grid, kBlock, 0, s>>>(a);
        else select_quad_kernel<8><<<grid, kBlock, 0, s>>>(a);
    } else if (full) {
        if (D <= 64) EGOSGM_SEL(64, 1, kWinFull);
        else if (D <= 128) EGOSGM_SEL(64, 2, kWinFull);
        else EGOSGM_SEL(64, 4, kWinFull);
    } else {
        if (D <= 16) EGOSGM_SEL(16, 1, kWinRagged);
        else if (D <= 64) EGOSGM_SEL(16, 4, kWinRagged);
        else if (D <= 128) EGOSGM_SEL(16, 8, kWinRagged);
        else EGOSGM_SEL(16, 16, kWinRagged);
    }
#undef EGOSGM_SEL
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    sgm_lr_kernel<<<grid_for((size_t)a.w * a.h), kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_copy_slots(const SgmLaunch& a, const uint8_t* src, uint8_t* dst, hipStream_t s) {
    if (a.win.lo == nullptr)
        copy_slots_kernel<kWinFull><<<1024, kBlock, 0, s>>>(a, src, dst);
    else
        copy_slots_kernel<kWinRagged><<<1024, kBlock, 0, s>>>(a, src, dst);
    return hipGetLastError();
}

hipError_t launch_copy_quad_slots(const SgmLaunch& a, const uint8_t* src, size_t src_stride, uint8_t* dst,
                                  size_t dst_stride, int nvol, hipStream_t s) {
    copy_quad_slots_kernel<<<1024, kBlock, 0, s>>>(a, src, src_stride, dst, dst_stride, nvol);
    return hipGetLastError();
}

hipError_t launch_windows(const float* d_pred, const float* p_pred, int w, int h, float k_sigma,
                          int r_fixed, int r_min, int r_max, int max_disp, int16_t* lo,
                          int16_t* hi, uint32_t* off, uint32_t* chunk_tot, hipStream_t s) {
    const dim3 grid((w + kBlock - 1) / kBlock, h);
    windows_chunk_kernel<<<grid, kBlock, 0, s>>>(d_pred, p_pred, w, k_sigma, r_fixed, r_min, r_max,
                                                 max_disp, lo, hi, off, chunk_tot);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    windows_base_kernel<<<grid, kBlock, 0, s>>>(w, h, off, chunk_tot);
    return hipGetLastError();
}

hipError_t launch_sad_check(const uint8_t* left, const uint8_t* right, int w, int h, int pitch,
                            int radius, int sad_max, int16_t* disp_wta, float* disp_sub,
                            float* var_meas, hipStream_t s) {
    sad_check_kernel<<<grid_for((size_t)w * h), kBlock, 0, s>>>(left, right, w, h, pitch, radius,
                                                                 sad_max, disp_wta, disp_sub, var_meas);
    return hipGetLastError();
}

hipError_t launch_lr_check_prediction(float* d_pred, float* p_pred, const float* d_right, int w,
                                      int h, float tol, hipStream_t s) {
    lr_check_prediction_kernel<<<grid_for((size_t)w * h), kBlock, 0, s>>>(d_pred, p_pred, d_right, w,
                                                                          h, tol);
    return hipGetLastError();
}

hipError_t launch_disparity_to_float(const int16_t* d, float* out, int n, hipStream_t s) {
    disparity_to_float_kernel<<<grid_for((size_t)n), kBlock, 0, s>>>(d, out, n);
    return hipGetLastError();
}

hipError_t launch_plan_patch(SgmLaunch* pairs, const PlanPatches& p, hipStream_t s) {
    if (p.n <= 0) return hipSuccess;
    plan_patch_kernel<<<1, kPatchBatch, 0, s>>>(pairs, p);
    return hipGetLastError();
}

int batch_path_blocks(int group, int max_disp, int n_tasks) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    hipError_t e = hipSuccess;
#define EGOSGM_OCC(GG)                                                                                  \
    do {                                                                                                \
        if (max_disp <= 64)                                                                             \
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, paths_batch_persistent_kernel<GG, 64 / GG, 4>, kBlock, 0); \
        else if (max_disp <= 128)                                                                       \
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, paths_batch_persistent_kernel<GG, 128 / GG, 4>, kBlock, 0); \
        else                                                                                            \
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, paths_batch_persistent_kernel<GG, 256 / GG, 4>, kBlock, 0); \
    } while (0)
    if (group == 16) EGOSGM_OCC(16);
    else if (group == 32) EGOSGM_OCC(32);
    else EGOSGM_OCC(64);
#undef EGOSGM_OCC
    if (e != hipSuccess || per_cu <= 0) return 0;
    const int waves = (n_tasks + 64 / group - 1) / (64 / group);
    return std::max(1, std::min(cus * per_cu, (waves + kBlock / 64 - 1) / (kBlock / 64)));
}

hipError_t launch_batch_stage(const BatchTables& t, int max_disp, int stage, hipStream_t s) {
    switch (stage) {
        case 0:
            census_batch_kernel<<<dim3(t.host_census_blocks, 1, 2), kBlock, 0, s>>>(t);
            break;
        case 1:
            cost_batch_kernel<<<t.host_seg_blocks, kBlock, 0, s>>>(t);
            break;
        case 2: {
            // persistent: host_path_blocks resident blocks; else one block per 256/G tasks
            const int g = t.group;
            const unsigned pb = t.persistent ? (unsigned)t.host_path_blocks
                                             : (unsigned)((t.n_tasks + kBlock / g - 1) / (kBlock / g));
#define EGOSGM_PB(GG)                                                                                         \
    do {                                                                                                      \
        if (t.persistent) {                                                                                   \
            if (max_disp <= 64) paths_batch_persistent_kernel<GG, 64 / GG, 4><<<pb, kBlock, 0, s>>>(t);         \
            else if (max_disp <= 128) paths_batch_persistent_kernel<GG, 128 / GG, 4><<<pb, kBlock, 0, s>>>(t);  \
            else paths_batch_persistent_kernel<GG, 256 / GG, 4><<<pb, kBlock, 0, s>>>(t);                       \
        } else {                                                                                              \
            if (max_disp <= 64) paths_batch_kernel<GG, 64 / GG, 4><<<pb, kBlock, 0, s>>>(t);                    \
            else if (max_disp <= 128) paths_batch_kernel<GG, 128 / GG, 4><<<pb, kBlock, 0, s>>>(t);             \
            else paths_batch_kernel<GG, 256 / GG, 4><<<pb, kBlock, 0, s>>>(t);                                  \
        }                                                                                                     \
    } while (0)
            if (g == 16) EGOSGM_PB(16);
            else if (g == 32) EGOSGM_PB(32);
            else EGOSGM_PB(64);
#undef EGOSGM_PB
            break;
        }
        case 3:
#define EGOSGM_SB(KK)                                                                   \
    do {                                                                                \
        if (t.n_paths == 4) select_batch_kernel<KK, 4><<<t.host_seg_blocks, kBlock, 0, s>>>(t); \
        else select_batch_kernel<KK, 8><<<t.host_seg_blocks, kBlock, 0, s>>>(t);               \
    } while (0)
            if (max_disp <= 16) EGOSGM_SB(1);
            else if (max_disp <= 64) EGOSGM_SB(4);
            else if (max_disp <= 128) EGOSGM_SB(8);
            else EGOSGM_SB(16);
#undef EGOSGM_SB
            break;
        default:
            lr_batch_kernel<<<grid_for((size_t)t.host_pixels), kBlock, 0, s>>>(t);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_sgm_batch(const BatchTables& t, int max_disp, hipStream_t s) {
    for (int stage = 0; stage < 5; ++stage) {
        const hipError_t e = launch_batch_stage(t, max_disp, stage, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_warp(const float* d_prev, const float* p_prev, int w, int h, const float* H,
                       const double* Hd, double q, float* d_pred, float* p_pred,
                       unsigned long long* zbuf, hipStream_t s) {
    const size_t n = (size_t)w * h;
    Mat4 m;
    Mat4d md;
    for (int i = 0; i < 16; ++i) {
        m.m[i] = H[i];
        md.m[i] = Hd[i];
    }
    fill_u64_kernel<<<grid_for(n), kBlock, 0, s>>>(zbuf, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    warp_scatter_kernel<<<grid_for(n), kBlock, 0, s>>>(d_prev, w, h, m, zbuf);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    warp_decode_kernel<<<grid_for(n), kBlock, 0, s>>>(zbuf, d_prev, p_prev, w, (int)n, md, q,
                                                      d_pred, p_pred);
    return hipGetLastError();
}

hipError_t launch_warp_scatter(const float* d_prev, int w, int h, const float* H,
                               unsigned long long* zbuf, hipStream_t s) {
    const size_t n = (size_t)w * h;
    Mat4 m;
    for (int i = 0; i < 16; ++i) m.m[i] = H[i];
    fill_u64_kernel<<<grid_for(n), kBlock, 0, s>>>(zbuf, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    warp_scatter_kernel<<<grid_for(n), kBlock, 0, s>>>(d_prev, w, h, m, zbuf);
    return hipGetLastError();
}

hipError_t launch_refine_from_zbuf(const unsigned long long* zbuf, const float* d_prev,
                                   const float* p_prev, int w, int h, const double* Hd, double q,
                                   float edge_tol, float fill_tol, float* d_out, float* p_out,
                                   hipStream_t s) {
    dim3 grid((w + kRfW - 1) / kRfW, (h + kRfH - 1) / kRfH);
    RefineSrc src{};
    src.d_in = d_prev;
    src.p_in = p_prev;
    src.zbuf = zbuf;
    for (int i = 0; i < 16; ++i) src.H.m[i] = Hd[i];
    src.q = q;
    refine_fused_kernel<true><<<grid, kBlock, 0, s>>>(src, w, h, edge_tol, fill_tol, d_out, p_out);
    return hipGetLastError();
}

hipError_t launch_refine(const float* d_in, const float* p_in, int w, int h, float edge_tol,
                         float fill_tol, float* d_out, float* p_out, hipStream_t s) {
    dim3 grid((w + kRfW - 1) / kRfW, (h + kRfH - 1) / kRfH);
    RefineSrc src{};
    src.d_in = d_in;
    src.p_in = p_in;
    refine_fused_kernel<false><<<grid, kBlock, 0, s>>>(src, w, h, edge_tol, fill_tol, d_out, p_out);
    return hipGetLastError();
}

hipError_t launch_kalman(const float* d_pred, const float* p_pred, const float* z, const float* r,
                         int n, int keep, float* d_out, float* p_out, hipStream_t s) {
    kalman_kernel<<<grid_for((size_t)n), kBlock, 0, s>>>(d_pred, p_pred, z, r, n, keep, d_out,
                                                         p_out);
    return hipGetLastError();
}

}  // namespace egosgm
