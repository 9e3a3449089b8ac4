// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace haar {

inline int elem_bytes(int dtype) { return dtype == 0 ? 4 : 2; }

// ceil(n / 2^j) on the host
inline int64_t ceil_shift_host(int64_t n, int j) { return (n + ((int64_t)1 << j) - 1) >> j; }

int set_error(int code, const char* fmt, ...);
int hip_error(hipError_t e, const char* what);
int max_levels(int64_t n);
bool aligned(const void* p, int a);
int device_cus();

// HAAR_FAULT_INJECT=launch makes every transform call fail as if its launch
// had failed (HAAR_ERR_HIP) before anything is enqueued: a host-side way to
// exercise the error path of callers.
int fault_injected();

// Tile / chunk configuration chosen for a problem (tuning table or default).
// fallback >= 0: returned when neither a forced choice nor a tuning-table
// entry exists (plans pass their own default shape).
int choose_config_2d(int dtype, bool inverse, int64_t h, int64_t w, int levels, int fallback = -1);
int choose_config_1d(int dtype, bool inverse, int64_t n, int levels, int64_t batch = 1);

int run_2d(const void* in, void* out, int64_t H, int64_t W, int L, int64_t batch, int dtype,
           bool inverse, hipStream_t s, int cfg_override);
int run_1d(const void* in, void* out, int64_t N, int L, int64_t batch, int dtype, bool inverse,
           hipStream_t s, int cfg_override);

// Separable 3D on [batch][D][H][W]: passes of up to 3 fused levels.
int run_3d(const void* in, void* out, int64_t D, int64_t H, int64_t W, int L, int64_t batch, int dtype,
           bool inverse, hipStream_t s);

// Fused shrinkage (analysis, thresholding of the details, synthesis): one
// chunk of kShrinkChunk samples (1D, levels <= 12) or one 32-row tile (2D,
// levels <= 5) per work-group.
constexpr int kMaxShrinkLevels = 12;
constexpr int kShrinkChunk = 4096, kShrinkChunkThreads = 256;
constexpr int kMaxShrinkLevels2D = 5;
int run_shrink_1d(const void* in, void* out, int64_t n, int L, int64_t batch, int dtype, int mode,
                  const float* thr, hipStream_t s);
// Fused training step of the sparsity loss sum |details| + 0.5 ||LL_L||^2
// through the 2D transform: gradient with respect to the input and the
// loss of each item (levels <= 5).
int run_l1_grad_2d(const void* in, void* out, double* loss, int64_t h, int64_t w, int L, int64_t batch,
                   int dtype, hipStream_t s);
// The same with the loss partials in the library's static device array of
// kStaticLossPartials doubles (no allocation); l1_grad_partials() is the
// number of partials (tiles) a call needs.
constexpr int64_t kStaticLossPartials = (int64_t)1 << 19;
int64_t l1_grad_partials(int64_t h, int64_t w, int64_t batch, int dtype);
int run_l1_grad_2d_static(const void* in, void* out, double* loss, int64_t h, int64_t w, int L,
                          int64_t batch, int dtype, hipStream_t s);
// Direct (convolve-then-decimate) structure, for comparison with the fast bank.
size_t direct_workspace_floats(int64_t n, int64_t batch);
int run_direct_1d(const void* in, void* out, int64_t n, int L, int64_t batch, int dtype, bool inverse,
                  float* ws, hipStream_t s);
int run_shrink_2d(const void* in, void* out, int64_t h, int64_t w, int L, int64_t batch, int dtype,
                  int mode, const float* thr, hipStream_t s);

}  // namespace haar
