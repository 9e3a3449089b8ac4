// Kernels and launchers of the plain 1D transforms (device code of one
// chunk: haar_1d_chunk.h).
#include "haar_1d_chunk.h"

namespace haar {

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
template <class SX, class SD, class SL, int E, int NT>
__global__ __launch_bounds__(NT) void fwd1d_kernel(Pass1D p) {
    using G = Geo1D<SX, E, NT>;
    __shared__ df sm[G::NW];
    const bool remap = p.remap && (int64_t)gridDim.x == p.total_chunks;
    for (int64_t b = blockIdx.x; b < p.total_chunks; b += gridDim.x) {
        const int64_t c = remap ? xcd_tile(b, p.total_chunks) : b;
        const int64_t item = c / p.chunks_per_item, chunk = c - item * p.chunks_per_item;
        const bool full = p.vec_ok && (chunk + 1) * G::C <= p.n;
        if (full)
            fwd1d_chunk<SX, SD, SL, E, NT, true>(p, item, chunk, sm);
        else
            fwd1d_chunk<SX, SD, SL, E, NT, false>(p, item, chunk, sm);
        if (b + gridDim.x < p.total_chunks) __syncthreads();
    }
}

template <class SX, class SD, class SL, int E, int NT, bool WALK>
__global__ __launch_bounds__(NT) void inv1d_kernel(Pass1D p) {
    using G = Geo1D<SX, E, NT>;
    __shared__ float sm[G::NW * 8];
    const bool remap = p.remap && (int64_t)gridDim.x == p.total_chunks;
    for (int64_t b = blockIdx.x; b < p.total_chunks; b += gridDim.x) {
        const int64_t c = remap ? xcd_tile(b, p.total_chunks) : b;
        const int64_t item = c / p.chunks_per_item, chunk = c - item * p.chunks_per_item;
        const bool full = p.vec_ok && (chunk + 1) * G::C <= p.n;
        float top = 0.0f;
        if (WALK)
            top = walk_down<SD>(reinterpret_cast<const typename SD::raw*>(p.det) + item * p.det_bstride,
                                p.n, p.levels_total, p.levels, chunk);
        if (full)
            inv1d_chunk<SX, SD, SL, E, NT, true>(p, item, chunk, sm, WALK, top);
        else
            inv1d_chunk<SX, SD, SL, E, NT, false>(p, item, chunk, sm, WALK, top);
        if (b + gridDim.x < p.total_chunks) __syncthreads();
    }
}

// Levels lc+1..L of each item's prefix, one work-group per item.
// The level-lc approximations come from p.ll (FP32, stride p.ll_bstride)
// when src32, else from the prefix of each item's output.
template <class S>
__global__ __launch_bounds__(256) void finish1d_kernel(Pass1D p, int lc, int L, bool src32) {
    __shared__ df buf0[kFinishMax], buf1[kFinishMax];
    for (int64_t item = blockIdx.x; item < p.batch; item += gridDim.x) {
        const float* a = src32 ? reinterpret_cast<const float*>(p.ll) + item * p.ll_bstride : nullptr;
        finish1d<S>(reinterpret_cast<typename S::raw*>(p.det) + item * p.det_bstride, a, p.n, lc, L,
                    buf0, buf1);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Chunk table and launchers.  Index -> (threads, elements per thread).
// ---------------------------------------------------------------------------
#define HAAR_1D_CHUNKS(X) \
    X(0, 256, 16, 1)      \
    X(1, 1024, 16, 1)     \
    X(2, 64, 16, 1)       \
    X(3, 128, 16, 1)      \
    X(4, 256, 16, 0)

int num_chunk_configs_1d() { return 5; }

Chunk1D chunk_config_1d(int index) {
    switch (index) {
#define X(I, NT_, E_, RM_) \
    case I:                \
        return Chunk1D{NT_, E_, RM_};
        HAAR_1D_CHUNKS(X)
#undef X
        default:
            return Chunk1D{256, 16, 1};
    }
}

template <class SX, class SD, class SL, int NT, int E>
static hipError_t launch1d(const Pass1D& p, bool inverse, hipStream_t s) {
    constexpr int64_t kMaxGrid = 1 << 20;
    const unsigned grid = (unsigned)(p.total_chunks < kMaxGrid ? p.total_chunks : kMaxGrid);
    if (inverse)
        hipLaunchKernelGGL((inv1d_kernel<SX, SD, SL, E, NT, false>), dim3(grid), dim3(NT), 0, s, p);
    else
        hipLaunchKernelGGL((fwd1d_kernel<SX, SD, SL, E, NT>), dim3(grid), dim3(NT), 0, s, p);
    return hipGetLastError();
}

template <class S>
static hipError_t dispatch1d(const Pass1D& p, int cfg, bool inverse, hipStream_t s) {
    switch (cfg) {
#define X(I, NT_, E_, RM_) \
    case I:                \
        return launch1d<S, S, S, NT_, E_>(p, inverse, s);
        HAAR_1D_CHUNKS(X)
#undef X
        default:
            return launch1d<S, S, S, 256, 16>(p, inverse, s);
    }
}

// Passes of a deep reduced-precision transform (FP32 scratch between passes).
template <class S>
static hipError_t dispatch1d_mixed(const Pass1D& p, int cfg, bool x_f32, bool ll_f32, bool inverse,
                                   hipStream_t s) {
    switch (cfg) {
#define X(I, NT_, E_, RM_)                                                       \
    case I:                                                                      \
        if (x_f32 && ll_f32) return launch1d<StF32, S, StF32, NT_, E_>(p, inverse, s); \
        if (x_f32) return launch1d<StF32, S, S, NT_, E_>(p, inverse, s);                \
        return launch1d<S, S, StF32, NT_, E_>(p, inverse, s);
        HAAR_1D_CHUNKS(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
}

static hipError_t dispatch1d_dtype(const Pass1D& p, int dtype, int cfg, bool x_f32, bool ll_f32,
                                   bool inverse, hipStream_t s) {
    if (dtype == 0 || (!x_f32 && !ll_f32)) {
        switch (dtype) {
            case 0: return dispatch1d<StF32>(p, cfg, inverse, s);
            case 1: return dispatch1d<StBF16>(p, cfg, inverse, s);
            case 2: return dispatch1d<StF16>(p, cfg, inverse, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (dtype) {
        case 1: return dispatch1d_mixed<StBF16>(p, cfg, x_f32, ll_f32, inverse, s);
        case 2: return dispatch1d_mixed<StF16>(p, cfg, x_f32, ll_f32, inverse, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fwd1d(const Pass1D& p, int dtype, int cfg, bool x_f32, bool ll_f32, hipStream_t s) {
    return dispatch1d_dtype(p, dtype, cfg, x_f32, ll_f32, false, s);
}

hipError_t launch_inv1d(const Pass1D& p, int dtype, int cfg, bool x_f32, bool ll_f32, hipStream_t s) {
    return dispatch1d_dtype(p, dtype, cfg, x_f32, ll_f32, true, s);
}

template <class S>
static hipError_t finish_t(const Pass1D& p, int lc, int L, bool src32, hipStream_t s) {
    const unsigned grid = (unsigned)(p.batch < (1 << 20) ? p.batch : (1 << 20));
    hipLaunchKernelGGL(finish1d_kernel<S>, dim3(grid), dim3(256), 0, s, p, lc, L, src32);
    return hipGetLastError();
}

hipError_t launch_finish1d(const Pass1D& p, int dtype, int lc, int L, bool src32, hipStream_t s) {
    switch (dtype) {
        case 0: return finish_t<StF32>(p, lc, L, src32, s);
        case 1: return finish_t<StBF16>(p, lc, L, src32, s);
        case 2: return finish_t<StF16>(p, lc, L, src32, s);
        default: return hipErrorInvalidValue;
    }
}

template <class S, int NT, int E>
static hipError_t walk_t(const Pass1D& p, hipStream_t s) {
    constexpr int64_t kMaxGrid = 1 << 20;
    const unsigned grid = (unsigned)(p.total_chunks < kMaxGrid ? p.total_chunks : kMaxGrid);
    hipLaunchKernelGGL((inv1d_kernel<S, S, S, E, NT, true>), dim3(grid), dim3(NT), 0, s, p);
    return hipGetLastError();
}

template <class S>
static hipError_t walk_cfg(const Pass1D& p, int cfg, hipStream_t s) {
    switch (cfg) {
#define X(I, NT_, E_, RM_) \
    case I:                \
        return walk_t<S, NT_, E_>(p, s);
        HAAR_1D_CHUNKS(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_inv1d_walk(const Pass1D& p, int dtype, int cfg, hipStream_t s) {
    switch (dtype) {
        case 0: return walk_cfg<StF32>(p, cfg, s);
        case 1: return walk_cfg<StBF16>(p, cfg, s);
        case 2: return walk_cfg<StF16>(p, cfg, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace haar
