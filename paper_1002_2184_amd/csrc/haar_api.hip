// C ABI of libhaar: argument validation, pass planning and dispatch.
//
// Every check runs before the first HIP call.  A transform is split into
// fused passes (2D: up to 5 levels per pass, the dependency block of a tile;
// 1D: up to log2(chunk) levels per pass).  Pass k reads the region left by
// pass k-1, writes its detail bands straight into the output buffer at their
// packed-layout positions and its deepest approximation either into the
// output (last pass) or into stream-ordered scratch (hipMallocAsync).  The
// synthesis runs the same passes from the deepest to the shallowest.
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "haar.h"
#include "haar_internal.h"
#include "haar_kernels.h"

namespace haar {

static thread_local std::string g_last_error;

int set_error(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_error(hipError_t e, const char* what) {
    return set_error(HAAR_ERR_HIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

int max_levels(int64_t n) {
    if (n < 1) return -1;
    int L = 0;
    while (L < 62 && ((int64_t)1 << L) < n) ++L;
    return L;
}

bool aligned(const void* p, int a) { return ((uintptr_t)p % (uintptr_t)a) == 0; }

// Compute units of the current device (queried once per device).
int device_cus() {
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cache[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        cache[dev] = n;
    }
    return cache[dev];
}

static bool ranges_overlap(const void* a, const void* b, uint64_t bytes) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bytes && y < x + bytes;
}

// Common checks of the plain calls.  Returns HAAR_OK or an error code; sets
// *nothing = true when there is nothing to enqueue (batch == 0).
static int check_common(const void* in, const void* out, int64_t elems_per_item, int32_t levels,
                        int max_lv, int64_t batch, int32_t dtype, bool* nothing) {
    *nothing = false;
    if (dtype < 0 || dtype > 2) return set_error(HAAR_ERR_DTYPE, "dtype %d is not a haar_dtype", dtype);
    if (batch < 0) return set_error(HAAR_ERR_SHAPE, "batch %lld < 0", (long long)batch);
    const int64_t eb = elem_bytes(dtype);
    if (elems_per_item > INT64_MAX / eb / (batch > 0 ? batch : 1))
        return set_error(HAAR_ERR_SHAPE, "tensor size overflows 64-bit byte counts");
    if (levels < 0 || levels > max_lv)
        return set_error(HAAR_ERR_LEVELS, "levels %d outside [0, %d]", levels, max_lv);
    if (batch == 0) {
        *nothing = true;
        return HAAR_OK;
    }
    if (!in || !out) return set_error(HAAR_ERR_NULL, "input or output pointer is NULL");
    if (ranges_overlap(in, out, (uint64_t)(elems_per_item * batch * eb)))
        return set_error(HAAR_ERR_ALIAS, "input and output overlap (out-of-place only)");
    return HAAR_OK;
}

// ---------------------------------------------------------------------------
// 2D
// ---------------------------------------------------------------------------
struct Region2D {
    int64_t h, w;
    int levels;
};

static std::vector<Region2D> passes_2d(int64_t h, int64_t w, int L) {
    std::vector<Region2D> v;
    while (L > 0) {
        const int lp = L < kMaxPassLevels2D ? L : kMaxPassLevels2D;
        v.push_back({h, w, lp});
        h = (h + ((int64_t)1 << lp) - 1) >> lp;
        w = (w + ((int64_t)1 << lp) - 1) >> lp;
        L -= lp;
    }
    return v;
}

static void tile_grid(Pass2D& p, const Tile2D& tc) {
    p.tiles_x = (p.w + tc.tw() - 1) / tc.tw();
    p.tiles_y = (p.h + tc.th() - 1) / tc.th();
    p.full_x = p.w / tc.tw();
    p.full_y = p.h / tc.th();
    p.tiles_per_item = p.tiles_y * p.tiles_x;
    p.total_tiles = p.tiles_per_item * p.batch;
}

// Launch-wide condition of the vector path.  Region rows are read/written in
// 16-byte vectors; level-1/2 band rows and (for 1-2 level passes) the LL rows
// in vectors of B1X / B2X elements (RX = 16 / region element bytes).
// Full tiles use vector accesses, which need only element alignment of every
// pointer (sizes, pitches and band origins may be anything).
static int vec_ok_2d(const Pass2D& p, bool inverse, int ebx, int ebd, int ebl) {
    const void* region = inverse ? (const void*)p.dst : p.src;
    return aligned(region, ebx) && aligned(p.det, ebd) && aligned(p.ll, ebl) ? 1 : 0;
}

// Every row piece that a tile reads (region rows, level-1/2 band rows) covers
// whole 128-byte lines, so no cache line is read by two work-groups and the
// vector loads can be nontemporal.  Where tiles share lines (rows that start
// inside a line), ordinary loads let the second reader hit in L2.
static int own_lines_2d(const Pass2D& p, bool inverse, int ebx, int ebd, int tw) {
    auto lines = [](const void* base, int64_t pitch, int64_t bstride, int eb) {
        return aligned(base, 128) && (pitch * eb) % 128 == 0 && (bstride * eb) % 128 == 0;
    };
    const void* region = inverse ? (const void*)p.dst : p.src;
    const int64_t rp = inverse ? p.dst_pitch : p.src_pitch, rb = inverse ? p.dst_bstride : p.src_bstride;
    const bool ok = lines(region, rp, rb, ebx) && (tw * ebx) % 128 == 0 &&
                    lines(p.det, p.det_pitch, p.det_bstride, ebd) &&
                    (ceil_shift_host(p.w, 1) * ebd) % 128 == 0 && (ceil_shift_host(p.w, 2) * ebd) % 128 == 0 &&
                    ((tw / 4) * ebd) % 128 == 0;
    return ok ? 1 : 0;
}

int run_2d(const void* in, void* out, int64_t H, int64_t W, int L, int64_t batch, int dtype,
           bool inverse, hipStream_t s, int cfg_override) {
    const int eb = elem_bytes(dtype);
    const std::vector<Region2D> ps = passes_2d(H, W, L);
    const int np = (int)ps.size();
    const int cfg = cfg_override >= 0 ? cfg_override : choose_config_2d(dtype, inverse, H, W, L);

    // FP32 scratch between passes: two ping-pong buffers sized for the region
    // after the first pass (the intermediate approximations)
    void* scratch = nullptr;
    int64_t half = 0;
    if (np > 1) {
        half = (batch * ps[1].h * ps[1].w + 63) & ~(int64_t)63;
        hipError_t e = hipMallocAsync(&scratch, (size_t)(2 * half * 4), s);
        if (e != hipSuccess) return hip_error(e, "hipMallocAsync (deep-transform scratch)");
    }
    // buf(k): the region that pass k reads (analysis) or writes (synthesis), k >= 1
    auto buf = [&](int k) -> char* { return (char*)scratch + ((k & 1) ? 0 : half) * 4; };

    int rc = HAAR_OK;
    for (int step = 0; step < np && rc == HAAR_OK; ++step) {
        const int k = inverse ? np - 1 - step : step;
        const Region2D& r = ps[k];
        const bool x_f32 = k > 0;             // region in scratch
        const bool ll_f32 = k < np - 1;       // deepest LL of the pass in scratch
        const bool mixed = dtype != 0 && (x_f32 || ll_f32);
        const int ebx = x_f32 ? 4 : eb, ebl = ll_f32 ? 4 : eb;
        const int pcfg = mixed ? 0 : cfg;     // mixed-type passes use the default shape
        Pass2D p{};
        p.h = r.h;
        p.w = r.w;
        p.batch = batch;
        p.levels = r.levels;
        p.det = const_cast<void*>(inverse ? in : (const void*)out);
        p.det_pitch = W;
        p.det_bstride = H * W;
        const int64_t nh = (r.h + ((int64_t)1 << r.levels) - 1) >> r.levels;
        const int64_t nw = (r.w + ((int64_t)1 << r.levels) - 1) >> r.levels;
        void* rptr = k == 0 ? (void*)(inverse ? out : in) : (void*)buf(k);
        const int64_t rpitch = k == 0 ? W : r.w, rbs = k == 0 ? H * W : r.h * r.w;
        void* lptr = k == np - 1 ? (void*)(inverse ? in : out) : (void*)buf(k + 1);
        const int64_t lpitch = k == np - 1 ? W : nw, lbs = k == np - 1 ? H * W : nh * nw;
        if (!inverse) {
            p.src = rptr; p.src_pitch = rpitch; p.src_bstride = rbs;
        } else {
            p.dst = rptr; p.dst_pitch = rpitch; p.dst_bstride = rbs;
        }
        p.ll = lptr; p.ll_pitch = lpitch; p.ll_bstride = lbs;
        const Tile2D tc = tile_config_2d(ebx, pcfg);
        tile_grid(p, tc);
        p.remap = tc.remap;
        p.persist = tc.wg_per_cu > 0 ? (int64_t)tc.wg_per_cu * device_cus() : 0;
        p.vec_ok = vec_ok_2d(p, inverse, ebx, eb, ebl);
        p.ntl = own_lines_2d(p, inverse, ebx, eb, tc.tw());
        // An FP32 analysis whose tiles share cache lines (rows or band
        // origins inside a line) writes back through L2 with the tiles of
        // each XCD contiguous, so that neighbouring tiles' halves of a shared
        // line merge in one L2 before they reach HBM (streamed, each half is
        // a partial-line write of its own): 4096 x 4104 FP32 L4 42 -> 33 us.
        // 16-bit analyses measured slower that way (4096 x 4224 BF16 14.5 ->
        // 16.9 us) and keep streaming stores.
        p.wb = !inverse && !p.ntl && p.vec_ok && tc.wg_per_cu == 0 && eb == 4 ? 1 : 0;
        if (p.wb) p.remap = 1;
        // 16-bit passes on layouts whose tiles own whole lines pace their
        // stores (Paced in haar_device.h)
        p.pace = p.ntl && !mixed && eb == 2 && tc.wg_per_cu == 0 ? 1 : 0;
        hipError_t e = inverse ? launch_inv2d(p, dtype, pcfg, x_f32, ll_f32, s)
                               : launch_fwd2d(p, dtype, pcfg, x_f32, ll_f32, s);
        if (e != hipSuccess) rc = hip_error(e, inverse ? "inv2d launch" : "fwd2d launch");
    }
    if (scratch) {
        hipError_t e = hipFreeAsync(scratch, s);
        if (e != hipSuccess && rc == HAAR_OK) rc = hip_error(e, "hipFreeAsync");
    }
    return rc;
}

// ---------------------------------------------------------------------------
// 1D
// ---------------------------------------------------------------------------
struct Region1D {
    int64_t n;
    int levels;
};

static int log2_int(int x) {
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

static std::vector<Region1D> passes_1d(int64_t n, int L, int depth) {
    std::vector<Region1D> v;
    while (L > 0) {
        const int lp = L < depth ? L : depth;
        v.push_back({n, lp});
        n = (n + ((int64_t)1 << lp) - 1) >> lp;
        L -= lp;
    }
    return v;
}

// Launch-wide condition of the vector path: 16-byte region accesses and, per
// in-register level, detail spans of min(E >> lev, 16 / ebd) elements.
// Full chunks use vector accesses, which need only element alignment.
static int vec_ok_1d(const Pass1D& p, bool inverse, int ebx, int ebd, int ebl) {
    const void* region = inverse ? (const void*)p.dst : p.src;
    return aligned(region, ebx) && aligned(p.det, ebd) && aligned(p.ll, ebl) ? 1 : 0;
}

// One chunk pass over every item (levels <= on-chip depth), shared by the
// single-pass case and the first stage of the scratch-free deep analysis.
static Pass1D chunk_pass(const void* in, void* out, int64_t N, int lv, int64_t batch, bool inverse,
                         const Chunk1D& cc) {
    Pass1D p{};
    p.n = N;
    p.batch = batch;
    p.levels = lv;
    p.det = const_cast<void*>(inverse ? in : (const void*)out);
    p.det_bstride = N;
    p.ll = const_cast<void*>(inverse ? in : (const void*)out);
    p.ll_bstride = N;
    if (!inverse) { p.src = in; p.src_bstride = N; }
    else { p.dst = out; p.dst_bstride = N; }
    p.remap = cc.remap;
    p.chunks_per_item = (N + cc.chunk() - 1) / cc.chunk();
    p.total_chunks = p.chunks_per_item * batch;
    return p;
}

// Every chunk's region span and level-1/2 band spans cover whole 128-byte
// lines (see own_lines_2d): nontemporal loads.
static int own_lines_1d(const Pass1D& p, bool inverse, int ebx, int ebd, int64_t chunk) {
    const void* region = inverse ? (const void*)p.dst : p.src;
    const int64_t rb = inverse ? p.dst_bstride : p.src_bstride;
    const bool ok = aligned(region, 128) && (rb * ebx) % 128 == 0 && (chunk * ebx) % 128 == 0 &&
                    aligned(p.det, 128) && (p.det_bstride * ebd) % 128 == 0 &&
                    (ceil_shift_host(p.n, 1) * ebd) % 128 == 0 && (ceil_shift_host(p.n, 2) * ebd) % 128 == 0 &&
                    ((chunk / 4) * ebd) % 128 == 0;
    return ok ? 1 : 0;
}

int run_1d(const void* in, void* out, int64_t N, int L, int64_t batch, int dtype, bool inverse,
           hipStream_t s, int cfg_override) {
    const int eb = elem_bytes(dtype);
    const int cfg = cfg_override >= 0 ? cfg_override : choose_config_1d(dtype, inverse, N, L, batch);
    const Chunk1D cc = chunk_config_1d(cfg);
    const int depth = log2_int(cc.chunk());

    // Deep transforms in two stages: the analysis chunks leave their
    // level-`depth` approximations in the output prefix (FP32 storage) or in
    // a small FP32 buffer (16-bit storage), and one work-group per item
    // finishes them on chip; the synthesis walks each chunk's ancestor path
    // from a_L.
    if (L > depth && !inverse && ceil_shift_host(N, depth) <= kFinishMaxHost) {
        Pass1D p = chunk_pass(in, out, N, depth, batch, false, cc);
        const int64_t m = ceil_shift_host(N, depth);
        void* a32 = nullptr;
        if (dtype != HAAR_F32) {
            hipError_t e = hipMallocAsync(&a32, (size_t)(batch * m * 4), s);
            if (e != hipSuccess) return hip_error(e, "hipMallocAsync (level approximations)");
            p.ll = a32;
            p.ll_bstride = m;
        }
        p.vec_ok = vec_ok_1d(p, false, eb, eb, a32 ? 4 : eb);
        p.ntl = own_lines_1d(p, false, eb, eb, cc.chunk());
        hipError_t e = launch_fwd1d(p, dtype, cfg, false, a32 != nullptr, s);
        if (e == hipSuccess) e = launch_finish1d(p, dtype, depth, L, a32 != nullptr, s);
        int rc = e == hipSuccess ? HAAR_OK : hip_error(e, "fwd1d launch");
        if (a32) {
            e = hipFreeAsync(a32, s);
            if (e != hipSuccess && rc == HAAR_OK) rc = hip_error(e, "hipFreeAsync");
        }
        return rc;
    }
    if (L > depth && inverse && L - depth <= kMaxWalkHost) {
        Pass1D p = chunk_pass(in, out, N, depth, batch, true, cc);
        p.levels_total = L;
        p.vec_ok = vec_ok_1d(p, true, eb, eb, eb);
        p.ntl = own_lines_1d(p, true, eb, eb, cc.chunk());
        hipError_t e = launch_inv1d_walk(p, dtype, cfg, s);
        return e == hipSuccess ? HAAR_OK : hip_error(e, "inv1d launch");
    }

    const std::vector<Region1D> ps = passes_1d(N, L, depth);
    const int np = (int)ps.size();
    void* scratch = nullptr;
    int64_t half = 0;
    if (np > 1) {
        half = (batch * ps[1].n + 63) & ~(int64_t)63;
        hipError_t e = hipMallocAsync(&scratch, (size_t)(2 * half * 4), s);
        if (e != hipSuccess) return hip_error(e, "hipMallocAsync (deep-transform scratch)");
    }
    auto buf = [&](int k) -> char* { return (char*)scratch + ((k & 1) ? 0 : half) * 4; };

    int rc = HAAR_OK;
    for (int step = 0; step < np && rc == HAAR_OK; ++step) {
        const int k = inverse ? np - 1 - step : step;
        const Region1D& r = ps[k];
        const bool x_f32 = k > 0, ll_f32 = k < np - 1;
        const int ebx = x_f32 ? 4 : eb;
        Pass1D p{};
        p.n = r.n;
        p.batch = batch;
        p.levels = r.levels;
        p.det = const_cast<void*>(inverse ? in : (const void*)out);
        p.det_bstride = N;
        const int64_t nn = (r.n + ((int64_t)1 << r.levels) - 1) >> r.levels;
        void* rptr = k == 0 ? (void*)(inverse ? out : in) : (void*)buf(k);
        const int64_t rbs = k == 0 ? N : r.n;
        if (!inverse) { p.src = rptr; p.src_bstride = rbs; }
        else { p.dst = rptr; p.dst_bstride = rbs; }
        p.ll = k == np - 1 ? (void*)(inverse ? in : out) : (void*)buf(k + 1);
        p.ll_bstride = k == np - 1 ? N : nn;
        p.remap = cc.remap;
        p.chunks_per_item = (r.n + cc.chunk() - 1) / cc.chunk();
        p.total_chunks = p.chunks_per_item * batch;
        p.vec_ok = vec_ok_1d(p, inverse, ebx, eb, ll_f32 ? 4 : eb);
        p.ntl = own_lines_1d(p, inverse, ebx, eb, cc.chunk());
        hipError_t e = inverse ? launch_inv1d(p, dtype, cfg, x_f32, ll_f32, s)
                               : launch_fwd1d(p, dtype, cfg, x_f32, ll_f32, s);
        if (e != hipSuccess) rc = hip_error(e, inverse ? "inv1d launch" : "fwd1d launch");
    }
    if (scratch) {
        hipError_t e = hipFreeAsync(scratch, s);
        if (e != hipSuccess && rc == HAAR_OK) rc = hip_error(e, "hipFreeAsync");
    }
    return rc;
}

static int copy_levels0(const void* in, void* out, int64_t bytes, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(out, in, (size_t)bytes, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? HAAR_OK : hip_error(e, "hipMemcpyAsync (levels = 0)");
}

}  // namespace haar

using namespace haar;

extern "C" {

int haar_max_levels_1d(int64_t length) { return max_levels(length); }

int haar_max_levels_2d(int64_t height, int64_t width) {
    if (height < 1 || width < 1) return -1;
    return max_levels(height > width ? height : width);
}

static int api_1d(const void* in, void* out, int64_t length, int32_t levels, int64_t batch,
                  int32_t dtype, void* stream, bool inverse) {
    if (length < 1) return set_error(HAAR_ERR_SHAPE, "length %lld < 1", (long long)length);
    bool nothing = false;
    int rc = check_common(in, out, length, levels, max_levels(length), batch, dtype, &nothing);
    if (rc != HAAR_OK || nothing) return rc;
    if (rc = fault_injected(); rc != HAAR_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (levels == 0) return copy_levels0(in, out, length * batch * elem_bytes(dtype), s);
    return run_1d(in, out, length, levels, batch, dtype, inverse, s, -1);
}

static int api_2d(const void* in, void* out, int64_t height, int64_t width, int32_t levels,
                  int64_t batch, int32_t dtype, void* stream, bool inverse) {
    if (height < 1 || width < 1)
        return set_error(HAAR_ERR_SHAPE, "height %lld / width %lld < 1", (long long)height,
                         (long long)width);
    if (height > INT64_MAX / width) return set_error(HAAR_ERR_SHAPE, "height * width overflows");
    bool nothing = false;
    int rc = check_common(in, out, height * width, levels, haar_max_levels_2d(height, width), batch,
                          dtype, &nothing);
    if (rc != HAAR_OK || nothing) return rc;
    if (rc = fault_injected(); rc != HAAR_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (levels == 0) return copy_levels0(in, out, height * width * batch * elem_bytes(dtype), s);
    return run_2d(in, out, height, width, levels, batch, dtype, inverse, s, -1);
}

int haar_fwd_1d(const void* x, void* y, int64_t length, int32_t levels, int64_t batch,
                int32_t dtype, void* stream) {
    return api_1d(x, y, length, levels, batch, dtype, stream, false);
}

int haar_inv_1d(const void* y, void* x, int64_t length, int32_t levels, int64_t batch,
                int32_t dtype, void* stream) {
    return api_1d(y, x, length, levels, batch, dtype, stream, true);
}

int haar_fwd_2d(const void* x, void* y, int64_t height, int64_t width, int32_t levels,
                int64_t batch, int32_t dtype, void* stream) {
    return api_2d(x, y, height, width, levels, batch, dtype, stream, false);
}

int haar_inv_2d(const void* y, void* x, int64_t height, int64_t width, int32_t levels,
                int64_t batch, int32_t dtype, void* stream) {
    return api_2d(y, x, height, width, levels, batch, dtype, stream, true);
}

int haar_max_levels_3d(int64_t depth, int64_t height, int64_t width) {
    if (depth < 1 || height < 1 || width < 1) return -1;
    int64_t m = depth > height ? depth : height;
    m = m > width ? m : width;
    return max_levels(m);
}

static int api_3d(const void* in, void* out, int64_t depth, int64_t height, int64_t width,
                  int32_t levels, int64_t batch, int32_t dtype, void* stream, bool inverse) {
    if (depth < 1 || height < 1 || width < 1)
        return set_error(HAAR_ERR_SHAPE, "depth %lld / height %lld / width %lld < 1", (long long)depth,
                         (long long)height, (long long)width);
    if (height > INT64_MAX / width || depth > INT64_MAX / (height * width))
        return set_error(HAAR_ERR_SHAPE, "depth * height * width overflows");
    bool nothing = false;
    int rc = check_common(in, out, depth * height * width, levels,
                          haar_max_levels_3d(depth, height, width), batch, dtype, &nothing);
    if (rc != HAAR_OK || nothing) return rc;
    if (rc = fault_injected(); rc != HAAR_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (levels == 0) return copy_levels0(in, out, depth * height * width * batch * elem_bytes(dtype), s);
    return run_3d(in, out, depth, height, width, levels, batch, dtype, inverse, s);
}

int haar_fwd_3d(const void* x, void* y, int64_t depth, int64_t height, int64_t width, int32_t levels,
                int64_t batch, int32_t dtype, void* stream) {
    return api_3d(x, y, depth, height, width, levels, batch, dtype, stream, false);
}

int haar_inv_3d(const void* y, void* x, int64_t depth, int64_t height, int64_t width, int32_t levels,
                int64_t batch, int32_t dtype, void* stream) {
    return api_3d(y, x, depth, height, width, levels, batch, dtype, stream, true);
}

// Fused shrinkage: the plain-call checks, then mode and thresholds (host
// array, read during the call), then the fused depth.
static int check_shrink(int32_t levels, int32_t mode, const float* thresholds, int max_fused) {
    if (mode != HAAR_SHRINK_HARD && mode != HAAR_SHRINK_SOFT)
        return set_error(HAAR_ERR_ARG, "mode %d is not a haar_shrink_mode", mode);
    if (levels > 0 && !thresholds) return set_error(HAAR_ERR_NULL, "thresholds is NULL");
    for (int j = 0; j < levels; ++j)
        if (!(thresholds[j] >= 0.0f))
            return set_error(HAAR_ERR_ARG, "threshold of level %d is negative or NaN", j + 1);
    if (levels > max_fused)
        return set_error(HAAR_ERR_UNSUPPORTED, "fused shrinkage runs at most %d levels", max_fused);
    return HAAR_OK;
}

int haar_shrink_1d(const void* x, void* y, int64_t length, int32_t levels, int64_t batch,
                   int32_t dtype, int32_t mode, const float* thresholds, void* stream) {
    if (length < 1) return set_error(HAAR_ERR_SHAPE, "length %lld < 1", (long long)length);
    bool nothing = false;
    int rc = check_common(x, y, length, levels, max_levels(length), batch, dtype, &nothing);
    if (rc != HAAR_OK) return rc;
    if ((rc = check_shrink(levels, mode, thresholds, kMaxShrinkLevels)) != HAAR_OK || nothing) return rc;
    if (rc = fault_injected(); rc != HAAR_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (levels == 0) return copy_levels0(x, y, length * batch * elem_bytes(dtype), s);
    return run_shrink_1d(x, y, length, levels, batch, dtype, mode, thresholds, s);
}

int haar_shrink_2d(const void* x, void* y, int64_t height, int64_t width, int32_t levels,
                   int64_t batch, int32_t dtype, int32_t mode, const float* thresholds, void* stream) {
    if (height < 1 || width < 1)
        return set_error(HAAR_ERR_SHAPE, "height %lld / width %lld < 1", (long long)height,
                         (long long)width);
    if (height > INT64_MAX / width) return set_error(HAAR_ERR_SHAPE, "height * width overflows");
    bool nothing = false;
    int rc = check_common(x, y, height * width, levels, haar_max_levels_2d(height, width), batch,
                          dtype, &nothing);
    if (rc != HAAR_OK) return rc;
    if ((rc = check_shrink(levels, mode, thresholds, kMaxShrinkLevels2D)) != HAAR_OK || nothing) return rc;
    if (rc = fault_injected(); rc != HAAR_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (levels == 0) return copy_levels0(x, y, height * width * batch * elem_bytes(dtype), s);
    return run_shrink_2d(x, y, height, width, levels, batch, dtype, mode, thresholds, s);
}

int haar_l1_grad_2d(const void* x, void* grad_x, double* loss, int64_t height, int64_t width,
                    int32_t levels, int64_t batch, int32_t dtype, void* stream) {
    if (height < 1 || width < 1)
        return set_error(HAAR_ERR_SHAPE, "height %lld / width %lld < 1", (long long)height,
                         (long long)width);
    if (height > INT64_MAX / width) return set_error(HAAR_ERR_SHAPE, "height * width overflows");
    bool nothing = false;
    int rc = check_common(x, grad_x, height * width, levels, haar_max_levels_2d(height, width), batch,
                          dtype, &nothing);
    if (rc != HAAR_OK || nothing) return rc;
    if (!loss) return set_error(HAAR_ERR_NULL, "loss is NULL");
    if (levels < 1 || levels > kMaxShrinkLevels2D)
        return set_error(HAAR_ERR_UNSUPPORTED, "the fused loss gradient runs 1..%d levels", kMaxShrinkLevels2D);
    if (rc = fault_injected(); rc != HAAR_OK) return rc;
    return run_l1_grad_2d(x, grad_x, loss, height, width, levels, batch, dtype, (hipStream_t)stream);
}

int haar_l1_grad_2d_noalloc(const void* x, void* grad_x, double* loss, int64_t height, int64_t width,
                            int32_t levels, int64_t batch, int32_t dtype, void* stream) {
    if (height < 1 || width < 1)
        return set_error(HAAR_ERR_SHAPE, "height %lld / width %lld < 1", (long long)height,
                         (long long)width);
    if (height > INT64_MAX / width) return set_error(HAAR_ERR_SHAPE, "height * width overflows");
    bool nothing = false;
    int rc = check_common(x, grad_x, height * width, levels, haar_max_levels_2d(height, width), batch,
                          dtype, &nothing);
    if (rc != HAAR_OK || nothing) return rc;
    if (!loss) return set_error(HAAR_ERR_NULL, "loss is NULL");
    if (levels < 1 || levels > kMaxShrinkLevels2D)
        return set_error(HAAR_ERR_UNSUPPORTED, "the fused loss gradient runs 1..%d levels", kMaxShrinkLevels2D);
    const int64_t parts = l1_grad_partials(height, width, batch, dtype);
    if (parts > kStaticLossPartials)
        return set_error(HAAR_ERR_WORKSPACE,
                         "the call needs %lld tile loss partials; the static scratch holds %lld "
                         "(use haar_l1_grad_2d, or fewer or smaller items per call)",
                         (long long)parts, (long long)kStaticLossPartials);
    if (rc = fault_injected(); rc != HAAR_OK) return rc;
    return run_l1_grad_2d_static(x, grad_x, loss, height, width, levels, batch, dtype, (hipStream_t)stream);
}

size_t haar_direct_workspace_size(int64_t length, int64_t batch) {
    if (length < 1 || batch < 0) return 0;
    return direct_workspace_floats(length, batch) * sizeof(float);
}

int haar_direct_1d(const void* x, void* y, int64_t length, int32_t levels, int64_t batch, int32_t dtype,
                   int32_t inverse, void* workspace, size_t workspace_bytes, void* stream) {
    if (length < 1) return set_error(HAAR_ERR_SHAPE, "length %lld < 1", (long long)length);
    bool nothing = false;
    int rc = check_common(x, y, length, levels, max_levels(length), batch, dtype, &nothing);
    if (rc != HAAR_OK || nothing) return rc;
    if (!workspace) return set_error(HAAR_ERR_NULL, "workspace is NULL");
    if (!aligned(workspace, 4) || workspace_bytes < haar_direct_workspace_size(length, batch))
        return set_error(HAAR_ERR_WORKSPACE, "workspace misaligned or smaller than %zu bytes",
                         haar_direct_workspace_size(length, batch));
    if (rc = fault_injected(); rc != HAAR_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (levels == 0) return copy_levels0(x, y, length * batch * elem_bytes(dtype), s);
    return run_direct_1d(x, y, length, levels, batch, dtype, inverse != 0, (float*)workspace, s);
}

const char* haar_status_string(int status) {
    switch (status) {
        case HAAR_OK: return "HAAR_OK";
        case HAAR_ERR_NULL: return "HAAR_ERR_NULL";
        case HAAR_ERR_DTYPE: return "HAAR_ERR_DTYPE";
        case HAAR_ERR_SHAPE: return "HAAR_ERR_SHAPE";
        case HAAR_ERR_LEVELS: return "HAAR_ERR_LEVELS";
        case HAAR_ERR_ALIAS: return "HAAR_ERR_ALIAS";
        case HAAR_ERR_WORKSPACE: return "HAAR_ERR_WORKSPACE";
        case HAAR_ERR_HIP: return "HAAR_ERR_HIP";
        case HAAR_ERR_PLAN: return "HAAR_ERR_PLAN";
        case HAAR_ERR_UNSUPPORTED: return "HAAR_ERR_UNSUPPORTED";
        case HAAR_ERR_ARG: return "HAAR_ERR_ARG";
        default: return "HAAR_ERR_UNKNOWN";
    }
}

const char* haar_last_error(void) { return g_last_error.c_str(); }

const char* haar_version(void) { return "libhaar 0.1 (gfx950)"; }

}  // extern "C"
