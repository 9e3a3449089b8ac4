// Tile-shape autotuner and the process-wide tuning table.
//
// A table entry maps (dimension, dtype, direction, levels, size class) to a
// tile/chunk configuration index.  haar_tune_2d / haar_tune_1d time every
// candidate on the caller's stream with hipEvents and record the fastest.
// Plain calls and plans consult the table; without an entry they use the
// built-in default.  The table can be written to and read from a small JSON
// file (an object of "key": index pairs).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "haar.h"
#include "haar_internal.h"
#include "haar_kernels.h"

namespace haar {

static std::mutex g_mu;
static std::map<std::string, int> g_table;
static int g_force_2d[3] = {-1, -1, -1};
static int g_force_1d[3] = {-1, -1, -1};

static const char* dtype_name(int d) { return d == 0 ? "f32" : (d == 1 ? "bf16" : "f16"); }

static int size_class(int64_t v) { return max_levels(v); }   // ceil(log2 v)

static std::string key_2d(int dtype, bool inverse, int64_t h, int64_t w, int levels) {
    char b[96];
    snprintf(b, sizeof b, "2d:%s:%s:L%d:h%d:w%d", dtype_name(dtype), inverse ? "inv" : "fwd", levels,
             size_class(h), size_class(w));
    return b;
}

static std::string key_1d(int dtype, bool inverse, int64_t n, int levels) {
    char b[96];
    snprintf(b, sizeof b, "1d:%s:%s:L%d:n%d", dtype_name(dtype), inverse ? "inv" : "fwd", levels,
             size_class(n));
    return b;
}

int choose_config_2d(int dtype, bool inverse, int64_t h, int64_t w, int levels, int fallback) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (dtype >= 0 && dtype < 3 && g_force_2d[dtype] >= 0) return g_force_2d[dtype];
    auto it = g_table.find(key_2d(dtype, inverse, h, w, levels));
    if (it != g_table.end()) return it->second;
    if (fallback >= 0) return fallback;
    // measured defaults (4096^2, 5 levels, cold HBM, one tile per
    // work-group, blocks dealt round-robin to the XCDs):
    //  - FP32 analysis: 32 x 256 tiles, 4 x 4 registers per thread, 512
    //    threads, two-row wavefronts (25.0 us; level 3 by shuffles);
    //  - FP32 synthesis: 64 x 256 tiles, 8 x 4 registers per thread, 512
    //    threads (23.9-24.1 us against 24.5-24.8 us for 32 x 256 with
    //    4 x 4), but only for images of whole tiles whose tile count fills
    //    the resident work-groups an exact number of times: with partial
    //    tiles or a last, partly filled round these large tiles lose
    //    (4096 x 4224: 27.5 against 25.3 us; 4096 x 4352, whole tiles but
    //    1088 of them: 27.4 against 25.0 us);
    //  - 16-bit analysis of rows of 1024 or more: 32 x 512 tiles (BF16),
    //    8 x 8 registers per thread, 256 threads, level 3 in registers
    //    (13.2-13.5 us against 13.8 us for 32 x 256);
    //  - 16-bit synthesis: the same 8 x 8 tiles for images of whole tiles
    //    (13.5 against 14.1-14.3 us), 32 x 512 tiles of 4 x 8 otherwise
    //    (4096 x 4224: 16.3 against 17.9 us).
    if (dtype == 0) {
        if (!inverse) return 14;
        const int64_t tiles = (h / 64) * (w / 256);
        const int64_t resident = 4 * (int64_t)device_cus();
        const bool whole = h % 64 == 0 && w % 256 == 0 && tiles >= resident && tiles % resident == 0;
        return whole ? 17 : 1;
    }
    if (!inverse) return w >= 1024 ? 15 : 0;
    return (w >= 1024 && w % 512 == 0 && h % 32 == 0) ? 15 : 1;
}

int choose_config_1d(int dtype, bool inverse, int64_t n, int levels, int64_t batch) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (dtype >= 0 && dtype < 3 && g_force_1d[dtype] >= 0) return g_force_1d[dtype];
        auto it = g_table.find(key_1d(dtype, inverse, n, levels));
        if (it != g_table.end()) return it->second;
    }
    // default: the smallest chunk that holds the signal, 4096 samples beyond;
    // a deep transform (beyond 12 levels, so it runs a finishing step either
    // way) of fewer than 64 chunks of 4096 in all takes 1024-sample chunks:
    // four times the work-groups for a latency-bound launch (one 65536-sample
    // signal, 16 levels: analysis 8.0 -> 6.7 us, synthesis 5.3 -> 4.4 us)
    if (n <= 1024) return 2;
    if (n <= 2048) return 3;
    if (levels > 12 && batch * ceil_shift_host(n, 12) < 64 && ceil_shift_host(n, 10) <= kFinishMaxHost) return 2;
    return 0;
}

int fault_injected() {
    const char* f = getenv("HAAR_FAULT_INJECT");
    if (f && strcmp(f, "launch") == 0)
        return set_error(HAAR_ERR_HIP, "injected launch failure (HAAR_FAULT_INJECT=launch)");
    return HAAR_OK;
}

// Median of `reps` timed runs of fn() on stream s (after `warm` untimed runs).
template <class F>
static int time_ms(F fn, hipStream_t s, int warm, int reps, float* out_ms) {
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return hip_error(e, "hipEventCreate");
    e = hipEventCreate(&b);
    if (e != hipSuccess) {
        (void)hipEventDestroy(a);
        return hip_error(e, "hipEventCreate");
    }
    int rc = HAAR_OK;
    for (int i = 0; i < warm && rc == HAAR_OK; ++i) rc = fn();
    std::vector<float> ts;
    for (int i = 0; i < reps && rc == HAAR_OK; ++i) {
        (void)hipEventRecord(a, s);
        rc = fn();
        (void)hipEventRecord(b, s);
        e = hipEventSynchronize(b);
        if (e != hipSuccess) {
            rc = hip_error(e, "hipEventSynchronize");
            break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, a, b);
        ts.push_back(ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc == HAAR_OK) {
        std::sort(ts.begin(), ts.end());
        *out_ms = ts[ts.size() / 2];
    }
    return rc;
}

}  // namespace haar

using namespace haar;

extern "C" {

int haar_tune_candidates_2d(int32_t dtype) {
    if (dtype < 0 || dtype > 2) return -1;
    return num_tile_configs_2d(elem_bytes(dtype));
}

const char* haar_tune_candidate_name(int32_t dtype, int32_t index) {
    static thread_local char buf[96];
    if (dtype < 0 || dtype > 2 || index < 0 || index >= num_tile_configs_2d(elem_bytes(dtype)))
        return "";
    const Tile2D t = tile_config_2d(elem_bytes(dtype), index);
    char pers[32] = "";
    if (t.wg_per_cu > 0) snprintf(pers, sizeof pers, ", persistent %d/CU", t.wg_per_cu);
    snprintf(buf, sizeof buf, "tile %dx%d, %d threads, %dx%d per thread%s%s%s", t.th(), t.tw(),
             t.threads(), t.ry, t.rx, t.remap ? ", XCD-contiguous" : "", pers,
             t.map == 1 ? ", wavefront-local analysis" : (t.map == 2 ? ", two-row wavefronts" : ""));
    return buf;
}

int haar_force_config_2d(int32_t dtype, int32_t index) {
    if (dtype < 0 || dtype > 2) return set_error(HAAR_ERR_DTYPE, "dtype %d is not a haar_dtype", dtype);
    if (index < -1 || index >= num_tile_configs_2d(elem_bytes(dtype)))
        return set_error(HAAR_ERR_UNSUPPORTED, "no 2D tile configuration %d", index);
    std::lock_guard<std::mutex> lk(g_mu);
    g_force_2d[dtype] = index;
    return HAAR_OK;
}

int haar_force_config_1d(int32_t dtype, int32_t index) {
    if (dtype < 0 || dtype > 2) return set_error(HAAR_ERR_DTYPE, "dtype %d is not a haar_dtype", dtype);
    if (index < -1 || index >= num_chunk_configs_1d())
        return set_error(HAAR_ERR_UNSUPPORTED, "no 1D chunk configuration %d", index);
    std::lock_guard<std::mutex> lk(g_mu);
    g_force_1d[dtype] = index;
    return HAAR_OK;
}

int haar_tune_candidates_1d(void) { return num_chunk_configs_1d(); }

int haar_tune_2d(int32_t dtype, int32_t inverse, int64_t height, int64_t width, int32_t levels,
                 int64_t batch, void* scratch, size_t scratch_bytes, void* stream,
                 int32_t* choice) {
    if (dtype < 0 || dtype > 2) return set_error(HAAR_ERR_DTYPE, "dtype %d is not a haar_dtype", dtype);
    if (height < 1 || width < 1 || batch < 1)
        return set_error(HAAR_ERR_SHAPE, "tuning needs height, width, batch >= 1");
    const int maxl = max_levels(height > width ? height : width);
    if (levels < 1 || levels > maxl)
        return set_error(HAAR_ERR_LEVELS, "levels %d outside [1, %d]", levels, maxl);
    if (!scratch || !choice) return set_error(HAAR_ERR_NULL, "scratch or choice is NULL");
    const int64_t eb = elem_bytes(dtype);
    const int64_t bytes = batch * height * width * eb;
    if (scratch_bytes < (size_t)(2 * bytes + 16))
        return set_error(HAAR_ERR_WORKSPACE, "tuning scratch needs %lld bytes", (long long)(2 * bytes + 16));
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)(((uintptr_t)scratch + 15) & ~(uintptr_t)15);
    char* in = base;
    char* out = base + ((bytes + 15) & ~(int64_t)15);
    if ((size_t)(out - (char*)scratch) + (size_t)bytes > scratch_bytes)
        return set_error(HAAR_ERR_WORKSPACE, "tuning scratch too small after alignment");
    hipError_t e = hipMemsetAsync(in, 0, (size_t)bytes, s);
    if (e != hipSuccess) return hip_error(e, "hipMemsetAsync");
    const int nc = num_tile_configs_2d((int)eb);
    int best = 0;
    float best_ms = 1e30f;
    for (int c = 0; c < nc; ++c) {
        float ms = 0.0f;
        int rc = time_ms([&]() { return run_2d(in, out, height, width, levels, batch, dtype,
                                               inverse != 0, s, c); },
                         s, 2, 7, &ms);
        if (rc != HAAR_OK) return rc;
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_table[key_2d(dtype, inverse != 0, height, width, levels)] = best;
    }
    *choice = best;
    return HAAR_OK;
}

int haar_tune_1d(int32_t dtype, int32_t inverse, int64_t length, int32_t levels, int64_t batch,
                 void* scratch, size_t scratch_bytes, void* stream, int32_t* choice) {
    if (dtype < 0 || dtype > 2) return set_error(HAAR_ERR_DTYPE, "dtype %d is not a haar_dtype", dtype);
    if (length < 1 || batch < 1) return set_error(HAAR_ERR_SHAPE, "tuning needs length, batch >= 1");
    const int maxl = max_levels(length);
    if (levels < 1 || levels > maxl)
        return set_error(HAAR_ERR_LEVELS, "levels %d outside [1, %d]", levels, maxl);
    if (!scratch || !choice) return set_error(HAAR_ERR_NULL, "scratch or choice is NULL");
    const int64_t eb = elem_bytes(dtype);
    const int64_t bytes = batch * length * eb;
    char* base = (char*)(((uintptr_t)scratch + 15) & ~(uintptr_t)15);
    char* in = base;
    char* out = base + ((bytes + 15) & ~(int64_t)15);
    if (scratch_bytes < (size_t)(2 * bytes + 32) ||
        (size_t)(out - (char*)scratch) + (size_t)bytes > scratch_bytes)
        return set_error(HAAR_ERR_WORKSPACE, "tuning scratch needs %lld bytes", (long long)(2 * bytes + 32));
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemsetAsync(in, 0, (size_t)bytes, s);
    if (e != hipSuccess) return hip_error(e, "hipMemsetAsync");
    const int nc = num_chunk_configs_1d();
    int best = 0;
    float best_ms = 1e30f;
    for (int c = 0; c < nc; ++c) {
        float ms = 0.0f;
        int rc = time_ms([&]() { return run_1d(in, out, length, levels, batch, dtype, inverse != 0,
                                               s, c); },
                         s, 2, 7, &ms);
        if (rc != HAAR_OK) return rc;
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_table[key_1d(dtype, inverse != 0, length, levels)] = best;
    }
    *choice = best;
    return HAAR_OK;
}

int haar_tune_save(const char* path) {
    if (!path) return set_error(HAAR_ERR_NULL, "path is NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    FILE* f = fopen(path, "w");
    if (!f) return set_error(HAAR_ERR_UNSUPPORTED, "cannot open %s for writing", path);
    fprintf(f, "{\n  \"format\": \"libhaar-tuning-1\"");
    for (const auto& kv : g_table) fprintf(f, ",\n  \"%s\": %d", kv.first.c_str(), kv.second);
    fprintf(f, "\n}\n");
    fclose(f);
    return HAAR_OK;
}

// Reads the "key": integer pairs of a file written by haar_tune_save.  A
// missing or malformed file leaves the table unchanged.
int haar_tune_load(const char* path) {
    if (!path) return set_error(HAAR_ERR_NULL, "path is NULL");
    FILE* f = fopen(path, "r");
    if (!f) return set_error(HAAR_ERR_UNSUPPORTED, "cannot open %s", path);
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    fclose(f);
    if (text.find("\"libhaar-tuning-1\"") == std::string::npos)
        return set_error(HAAR_ERR_UNSUPPORTED, "%s is not a libhaar tuning file", path);
    std::map<std::string, int> entries;
    size_t pos = 0;
    while ((pos = text.find('"', pos)) != std::string::npos) {
        const size_t end = text.find('"', pos + 1);
        if (end == std::string::npos) break;
        const std::string key = text.substr(pos + 1, end - pos - 1);
        size_t c = text.find_first_not_of(" \t\r\n", end + 1);
        pos = end + 1;
        if (c == std::string::npos || text[c] != ':') continue;
        c = text.find_first_not_of(" \t\r\n", c + 1);
        if (c == std::string::npos) break;
        if (text[c] == '-' || (text[c] >= '0' && text[c] <= '9')) {
            char* ep = nullptr;
            const long v = strtol(text.c_str() + c, &ep, 10);
            const bool is2d = key.rfind("2d:", 0) == 0, is1d = key.rfind("1d:", 0) == 0;
            if ((is2d && v >= 0 && v < num_tile_configs_2d(4)) ||
                (is1d && v >= 0 && v < num_chunk_configs_1d()))
                entries[key] = (int)v;
            pos = (size_t)(ep - text.c_str());
        }
    }
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto& kv : entries) g_table[kv.first] = kv.second;
    return HAAR_OK;
}

}  // extern "C"
