// Kernels and launchers of the plain 1D transforms (device code of one
// chunk: haar_1d_chunk.h).
#include "haar_1d_chunk.h"

namespace haar {

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
// A launch covers chunks [first, first + per) of every item: the complete
// chunks (FULL, vector path) and the ragged last chunk of each item (scalar
// path) run as separate launches, so that neither kernel carries the
// registers of the other path.  ONE: one work-group per chunk (the grid
// covers them all), so the chunk loop runs once and the compiler keeps far
// fewer values live (synthesis of full deep chunks: 35 VGPRs against 104;
// 256 x 65 536 FP32, 16 levels: 38.0 -> 31.1 us, analysis 34.6 -> 33.8 us).
template <class SX, class SD, class SL, int E, int NT, bool FULL, bool ONE = false, bool NTL = false>
__global__ __launch_bounds__(NT) void fwd1d_kernel(Pass1D p, int64_t first, int64_t per, int64_t total) {
    using G = Geo1D<SX, E, NT>;
    __shared__ df sm[G::NW];
    __shared__ float stage[FULL ? NT * E : 1];
    const bool remap = p.remap && (int64_t)gridDim.x == total;
    for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {
        const int64_t c = remap ? xcd_tile(b, total) : b;
        const int64_t item = c / per, chunk = first + (c - item * per);
        fwd1d_chunk<SX, SD, SL, E, NT, FULL, NTL>(p, item, chunk, sm, stage);
        if (ONE) break;
        if (b + gridDim.x < total) __syncthreads();
    }
}

template <class SX, class SD, class SL, int E, int NT, bool FULL, bool WALK, bool DEEP = false, bool ONE = false,
          bool NTL = false>
__global__ __launch_bounds__(NT) void inv1d_kernel(Pass1D p, int64_t first, int64_t per, int64_t total) {
    using G = Geo1D<SX, E, NT>;
    __shared__ float sm[G::NW * 8];
    __shared__ float stage[FULL ? NT * E : 1];
    const bool remap = p.remap && (int64_t)gridDim.x == total;
    for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {
        const int64_t c = remap ? xcd_tile(b, total) : b;
        const int64_t item = c / per, chunk = first + (c - item * per);
        float top = 0.0f;
        if (WALK)
            top = walk_down<SD>(reinterpret_cast<const typename SD::raw*>(p.det) + item * p.det_bstride,
                                p.n, p.levels_total, p.levels, chunk);
        inv1d_chunk<SX, SD, SL, E, NT, FULL, DEEP, NTL>(p, item, chunk, sm, stage, WALK, top);
        if (ONE) break;
        if (b + gridDim.x < total) __syncthreads();
    }
}

// Launch the complete chunks (vector path), then the ragged last chunk of
// every item (or, when the layout forbids vectors, every chunk) on the
// scalar path.
// kfull1 / kpart1: the same kernels for grids of one work-group per chunk.
template <class KFull, class KPart, class KFull1, class KPart1>
static hipError_t launch_split1d(const Pass1D& p, int C, int NT, KFull kfull, KPart kpart, KFull1 kfull1,
                                 KPart1 kpart1, hipStream_t s) {
    constexpr int64_t kMaxGrid = 1 << 20;
    const int64_t nfull = p.vec_ok ? p.n / C : 0, npart = p.chunks_per_item - nfull;
    if (nfull > 0) {
        const int64_t total = nfull * p.batch;
        const unsigned grid = (unsigned)(total < kMaxGrid ? total : kMaxGrid);
        if (total <= kMaxGrid)
            hipLaunchKernelGGL(kfull1, dim3(grid), dim3(NT), 0, s, p, (int64_t)0, nfull, total);
        else
            hipLaunchKernelGGL(kfull, dim3(grid), dim3(NT), 0, s, p, (int64_t)0, nfull, total);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (npart > 0) {
        const int64_t total = npart * p.batch;
        const unsigned grid = (unsigned)(total < kMaxGrid ? total : kMaxGrid);
        if (total <= kMaxGrid)
            hipLaunchKernelGGL(kpart1, dim3(grid), dim3(NT), 0, s, p, nfull, npart, total);
        else
            hipLaunchKernelGGL(kpart, dim3(grid), dim3(NT), 0, s, p, nfull, npart, total);
        return hipGetLastError();
    }
    return hipSuccess;
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
    // full chunks that own whole cache lines read them with nontemporal loads
    if (inverse) {
        if (p.levels > Log2<E>::v) {
            if (p.ntl)
                return launch_split1d(p, NT * E, NT, inv1d_kernel<SX, SD, SL, E, NT, true, false, true>,
                                      inv1d_kernel<SX, SD, SL, E, NT, false, false>,
                                      inv1d_kernel<SX, SD, SL, E, NT, true, false, true, true, true>,
                                      inv1d_kernel<SX, SD, SL, E, NT, false, false, false, true>, s);
            return launch_split1d(p, NT * E, NT, inv1d_kernel<SX, SD, SL, E, NT, true, false, true>,
                                  inv1d_kernel<SX, SD, SL, E, NT, false, false>,
                                  inv1d_kernel<SX, SD, SL, E, NT, true, false, true, true>,
                                  inv1d_kernel<SX, SD, SL, E, NT, false, false, false, true>, s);
        }
        return launch_split1d(p, NT * E, NT, inv1d_kernel<SX, SD, SL, E, NT, true, false>,
                              inv1d_kernel<SX, SD, SL, E, NT, false, false>,
                              inv1d_kernel<SX, SD, SL, E, NT, true, false, false, true>,
                              inv1d_kernel<SX, SD, SL, E, NT, false, false, false, true>, s);
    }
    if (p.ntl)
        return launch_split1d(p, NT * E, NT, fwd1d_kernel<SX, SD, SL, E, NT, true>,
                              fwd1d_kernel<SX, SD, SL, E, NT, false>,
                              fwd1d_kernel<SX, SD, SL, E, NT, true, true, true>,
                              fwd1d_kernel<SX, SD, SL, E, NT, false, true>, s);
    return launch_split1d(p, NT * E, NT, fwd1d_kernel<SX, SD, SL, E, NT, true>,
                          fwd1d_kernel<SX, SD, SL, E, NT, false>,
                          fwd1d_kernel<SX, SD, SL, E, NT, true, true>,
                          fwd1d_kernel<SX, SD, SL, E, NT, false, true>, s);
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
    // the walk covers the whole chunk depth, so full chunks are always deep
    if (p.ntl)
        return launch_split1d(p, NT * E, NT, inv1d_kernel<S, S, S, E, NT, true, true, true>,
                              inv1d_kernel<S, S, S, E, NT, false, true>,
                              inv1d_kernel<S, S, S, E, NT, true, true, true, true, true>,
                              inv1d_kernel<S, S, S, E, NT, false, true, false, true>, s);
    return launch_split1d(p, NT * E, NT, inv1d_kernel<S, S, S, E, NT, true, true, true>,
                          inv1d_kernel<S, S, S, E, NT, false, true>,
                          inv1d_kernel<S, S, S, E, NT, true, true, true, true>,
                          inv1d_kernel<S, S, S, E, NT, false, true, false, true>, s);
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
