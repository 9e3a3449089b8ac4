// Kernels and launchers of the plain 2D transforms (device code of one
// tile: haar_2d_tile.h).
#include "haar_2d_tile.h"

namespace haar {

#ifndef HAAR_MIN_WAVES_2D
#define HAAR_MIN_WAVES_2D 1
#endif


// Tile index -> (item, ty, tx).  EDGE = false: the grid of full tiles (vector
// path); EDGE = true: the right column and bottom row of partial tiles, or
// every tile when the layout is not aligned for vectors (p.vec_ok == 0), on
// the scalar path.
template <bool EDGE>
__device__ __forceinline__ void tile_coords(const Pass2D& p, int64_t tile, int64_t& item,
                                            int64_t& ty, int64_t& tx) {
    if (!EDGE) {
        const int64_t per = p.full_x * p.full_y;
        item = tile / per;
        const int64_t r = tile - item * per;
        ty = r / p.full_x;
        tx = r - ty * p.full_x;
    } else if (!p.vec_ok) {
        item = tile / p.tiles_per_item;
        const int64_t r = tile - item * p.tiles_per_item;
        ty = r / p.tiles_x;
        tx = r - ty * p.tiles_x;
    } else {
        const int64_t right = p.tiles_x > p.full_x ? p.full_y : 0;   // right column, full rows
        const int64_t bottom = p.tiles_y > p.full_y ? p.tiles_x : 0;  // bottom row, all columns
        const int64_t per = right + bottom;
        item = tile / per;
        const int64_t r = tile - item * per;
        if (r < right) {
            ty = r;
            tx = p.full_x;
        } else {
            ty = p.full_y;
            tx = r - right;
        }
    }
}

// Persistent launches (the tuner's persistent configurations, and grids
// beyond kMaxGrid tiles): a work-group walks tiles b, b + G, b + 2G, ...;
// with PIPE it issues the HBM reads of its next tile before it computes and
// writes the current one.  Interior and edge tiles are separate launches.
template <class SX, class SD, class SL, int RY, int RX, int GY, int GX, bool EDGE, bool PIPE, int MAP>
__global__ __launch_bounds__(GY* GX, HAAR_MIN_WAVES_2D) void fwd2d_persistent_kernel(Pass2D p, int64_t ntiles) {
    using G = Geo2D<SX, RY, RX, GY, GX>;
    __shared__ float sm[G::SMEM];
    const bool remap = p.remap && (int64_t)gridDim.x == ntiles;
    int64_t b = blockIdx.x;
    if (b >= ntiles) return;
    int64_t item, ty, tx;
    tile_coords<EDGE>(p, remap ? xcd_tile(b, ntiles) : b, item, ty, tx);
    FwdIn<RY, RX> cur;
    fwd2d_load<SX, RY, RX, GY, GX, !EDGE, MAP>(p, item, ty, tx, cur);
    while (true) {
        const int64_t nb = b + gridDim.x;
        int64_t nitem = 0, nty = 0, ntx = 0;
        FwdIn<RY, RX> nxt;
        if (PIPE && nb < ntiles) {
            tile_coords<EDGE>(p, nb, nitem, nty, ntx);
            fwd2d_load<SX, RY, RX, GY, GX, !EDGE, MAP>(p, nitem, nty, ntx, nxt);
        }
        fwd2d_body<SX, SD, SL, RY, RX, GY, GX, !EDGE, MAP>(p, item, ty, tx, cur, sm);
        if (nb >= ntiles) break;
        __syncthreads();
        if (!PIPE) {
            tile_coords<EDGE>(p, nb, nitem, nty, ntx);
            fwd2d_load<SX, RY, RX, GY, GX, !EDGE, MAP>(p, nitem, nty, ntx, nxt);
        }   // LDS reuse by the next tile
        cur = nxt;
        b = nb;
        item = nitem;
        ty = nty;
        tx = ntx;
    }
}

template <class SX, class SD, class SL, int RY, int RX, int GY, int GX, bool EDGE, bool PIPE>
__global__ __launch_bounds__(GY* GX, HAAR_MIN_WAVES_2D) void inv2d_persistent_kernel(Pass2D p, int64_t ntiles) {
    using In = InvInT<SX, SD, SL, RY, RX, GY, GX>;
    const bool remap = p.remap && (int64_t)gridDim.x == ntiles;
    int64_t b = blockIdx.x;
    if (b >= ntiles) return;
    int64_t item, ty, tx;
    tile_coords<EDGE>(p, remap ? xcd_tile(b, ntiles) : b, item, ty, tx);
    In cur;
    inv2d_load<SX, SD, SL, RY, RX, GY, GX, !EDGE>(p, item, ty, tx, cur);
    while (true) {
        const int64_t nb = b + gridDim.x;
        int64_t nitem = 0, nty = 0, ntx = 0;
        In nxt;
        if (PIPE && nb < ntiles) {
            tile_coords<EDGE>(p, nb, nitem, nty, ntx);
            inv2d_load<SX, SD, SL, RY, RX, GY, GX, !EDGE>(p, nitem, nty, ntx, nxt);
        }
        inv2d_body<SX, SD, SL, RY, RX, GY, GX, !EDGE>(p, item, ty, tx, cur);
        if (nb >= ntiles) break;
        if (!PIPE) {
            tile_coords<EDGE>(p, nb, nitem, nty, ntx);
            inv2d_load<SX, SD, SL, RY, RX, GY, GX, !EDGE>(p, nitem, nty, ntx, nxt);
        }
        cur = nxt;
        b = nb;
        item = nitem;
        ty = nty;
        tx = ntx;
    }
}

// One tile per work-group, every tile of the transform in one launch: the
// first nedge work-groups take the partial tiles (scalar path), the rest the
// full tiles (vector path).  A separate edge launch would wait for the
// interior launch to drain and then run its few hundred work-groups alone,
// each bound by its own memory latency (measured: 4096 x 4128 FP32 analysis
// 40 us in two launches, 33 us in one).  Straight-line code without a tile
// loop also needs fewer registers than the persistent kernels.
template <class SX, class SD, class SL, int RY, int RX, int GY, int GX, int MAP, bool NTL>
__global__ __launch_bounds__(GY* GX, HAAR_MIN_WAVES_2D) void fwd2d_kernel(Pass2D p, int64_t nedge,
                                                                         int64_t ninterior) {
    using G = Geo2D<SX, RY, RX, GY, GX>;
    __shared__ float sm[G::SMEM];
    const int64_t b = blockIdx.x;
    int64_t item, ty, tx;
    FwdIn<RY, RX> in;
    if (b < nedge) {
        tile_coords<true>(p, b, item, ty, tx);
        fwd2d_load<SX, RY, RX, GY, GX, false, MAP, NTL>(p, item, ty, tx, in);
        fwd2d_body<SX, SD, SL, RY, RX, GY, GX, false, MAP>(p, item, ty, tx, in, sm);
    } else {
        const int64_t t = b - nedge;
        // (XCD-contiguous order only when the edge blocks leave the round-robin
        // dealing of blocks to XCDs aligned: block b goes to XCD b mod 8)
        tile_coords<false>(p, (p.remap && (nedge & 7) == 0) ? xcd_tile(t, ninterior) : t, item, ty, tx);
        fwd2d_load<SX, RY, RX, GY, GX, true, MAP, NTL>(p, item, ty, tx, in);
        fwd2d_body<SX, SD, SL, RY, RX, GY, GX, true, MAP>(p, item, ty, tx, in, sm);
    }
}

template <class SX, class SD, class SL, int RY, int RX, int GY, int GX, bool NTL>
__global__ __launch_bounds__(GY* GX, HAAR_MIN_WAVES_2D) void inv2d_kernel(Pass2D p, int64_t nedge,
                                                                         int64_t ninterior) {
    using In = InvInT<SX, SD, SL, RY, RX, GY, GX>;
    const int64_t b = blockIdx.x;
    int64_t item, ty, tx;
    In in;
    if (b < nedge) {
        tile_coords<true>(p, b, item, ty, tx);
        inv2d_load<SX, SD, SL, RY, RX, GY, GX, false, NTL>(p, item, ty, tx, in);
        inv2d_body<SX, SD, SL, RY, RX, GY, GX, false>(p, item, ty, tx, in);
    } else {
        const int64_t t = b - nedge;
        // (XCD-contiguous order only when the edge blocks leave the round-robin
        // dealing of blocks to XCDs aligned: block b goes to XCD b mod 8)
        tile_coords<false>(p, (p.remap && (nedge & 7) == 0) ? xcd_tile(t, ninterior) : t, item, ty, tx);
        inv2d_load<SX, SD, SL, RY, RX, GY, GX, true, NTL>(p, item, ty, tx, in);
        inv2d_body<SX, SD, SL, RY, RX, GY, GX, true>(p, item, ty, tx, in);
    }
}

// ---------------------------------------------------------------------------
// Tile-shape table and launchers
// ---------------------------------------------------------------------------
// Index -> (RY, GY, GX, XCD remap, work-groups per CU, analysis thread map);
// RX = 16 bytes / element size: a thread holds RY rows of one 16-byte
// vector.  Work-groups per CU = 0: one tile
// per work-group; k > 0: a persistent interior grid of k work-groups per
// compute unit.  Map 1: wavefront-local analysis; map 2: two-row
// wavefronts (see thread_rc).
#define HAAR_2D_TILES(X)         \
    X(0, 4, 8, 32, 0, 0, 0)      \
    X(1, 4, 8, 64, 0, 0, 0)      \
    X(2, 4, 8, 32, 0, 4, 0)      \
    X(3, 4, 8, 64, 0, 2, 0)      \
    X(4, 4, 8, 32, 0, 2, 0)      \
    X(5, 4, 8, 32, 1, 0, 0)      \
    X(6, 4, 8, 16, 0, 8, 0)      \
    X(7, 4, 16, 16, 1, 0, 0)     \
    X(8, 4, 8, 64, 0, 0, 1)      \
    X(9, 4, 8, 32, 0, 0, 1)      \
    X(10, 4, 8, 16, 0, 0, 1)     \
    X(11, 4, 8, 8, 0, 0, 1)      \
    X(12, 4, 8, 16, 1, 0, 1)     \
    X(13, 4, 8, 8, 1, 0, 1)      \
    X(14, 4, 8, 64, 0, 0, 2)     \
    X(15, 8, 4, 64, 0, 0, 0)     \
    X(16, 8, 4, 32, 0, 0, 0)     \
    X(17, 8, 8, 64, 0, 0, 0)     \
    X(18, 8, 4, 256, 0, 0, 0)    \
    X(19, 8, 4, 128, 0, 0, 0)

int num_tile_configs_2d(int) { return 20; }

Tile2D tile_config_2d(int elem_bytes, int index) {
    const int rx = 16 / elem_bytes;
    switch (index) {
#define X(I, RY_, GY_, GX_, RM_, WPC_, MAP_) \
    case I:                                  \
        return Tile2D{RY_, rx, GY_, GX_, RM_, WPC_, MAP_};
        HAAR_2D_TILES(X)
#undef X
        default:
            return Tile2D{4, rx, 8, 32, 0, 0, 0};
    }
}

template <class SX, class SD, class SL, int GY, int GX, bool PIPE, int MAP = 0, int RY = 4>
static hipError_t launch2d(const Pass2D& p, bool inverse, hipStream_t s) {
    constexpr int RX = 16 / SX::kBytes;
    constexpr int64_t kMaxGrid = 1 << 20;
    const int64_t interior = p.vec_ok ? p.full_x * p.full_y * p.batch : 0;
    const int64_t edge = p.total_tiles - interior;
    if (p.persist == 0 && p.total_tiles <= kMaxGrid) {
        if (p.total_tiles <= 0) return hipSuccess;
        const unsigned grid = (unsigned)p.total_tiles;
        // tiles that own whole cache lines read them with nontemporal loads;
        // 16-bit passes among them (p.pace) pace their stores: analysis
        // outputs at most 2 operations behind, synthesis outputs 0
        if constexpr (SX::kBytes == 2 && SD::kBytes == 2 && SL::kBytes == 2) {
            if (p.pace) {
                if (inverse)
                    hipLaunchKernelGGL((inv2d_kernel<Paced<SX, 0>, SD, SL, RY, RX, GY, GX, true>), dim3(grid),
                                       dim3(GY * GX), 0, s, p, edge, interior);
                else
                    hipLaunchKernelGGL((fwd2d_kernel<SX, Paced<SD, 2>, Paced<SL, 2>, RY, RX, GY, GX, MAP, true>),
                                       dim3(grid), dim3(GY * GX), 0, s, p, edge, interior);
                return hipGetLastError();
            }
        }
        if (inverse) {
            if (p.ntl)
                hipLaunchKernelGGL((inv2d_kernel<SX, SD, SL, RY, RX, GY, GX, true>), dim3(grid), dim3(GY * GX), 0,
                                   s, p, edge, interior);
            else
                hipLaunchKernelGGL((inv2d_kernel<SX, SD, SL, RY, RX, GY, GX, false>), dim3(grid), dim3(GY * GX),
                                   0, s, p, edge, interior);
        } else {
            if (p.ntl)
                hipLaunchKernelGGL((fwd2d_kernel<SX, SD, SL, RY, RX, GY, GX, MAP, true>), dim3(grid),
                                   dim3(GY * GX), 0, s, p, edge, interior);
            else if (p.wb)
                hipLaunchKernelGGL((fwd2d_kernel<SX, WriteBack<SD>, WriteBack<SL>, RY, RX, GY, GX, MAP, false>),
                                   dim3(grid), dim3(GY * GX), 0, s, p, edge, interior);
            else
                hipLaunchKernelGGL((fwd2d_kernel<SX, SD, SL, RY, RX, GY, GX, MAP, false>), dim3(grid),
                                   dim3(GY * GX), 0, s, p, edge, interior);
        }
        return hipGetLastError();
    }
    if (interior > 0) {
        const int64_t cap = p.persist > 0 ? p.persist : kMaxGrid;
        const unsigned grid = (unsigned)(interior < cap ? interior : cap);
        if (inverse)
            hipLaunchKernelGGL((inv2d_persistent_kernel<SX, SD, SL, RY, RX, GY, GX, false, PIPE>), dim3(grid),
                               dim3(GY * GX), 0, s, p, interior);
        else
            hipLaunchKernelGGL((fwd2d_persistent_kernel<SX, SD, SL, RY, RX, GY, GX, false, PIPE, MAP>),
                               dim3(grid), dim3(GY * GX), 0, s, p, interior);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (edge > 0) {
        const unsigned grid = (unsigned)(edge < kMaxGrid ? edge : kMaxGrid);
        if (inverse)
            hipLaunchKernelGGL((inv2d_persistent_kernel<SX, SD, SL, RY, RX, GY, GX, true, false>), dim3(grid),
                               dim3(GY * GX), 0, s, p, edge);
        else
            hipLaunchKernelGGL((fwd2d_persistent_kernel<SX, SD, SL, RY, RX, GY, GX, true, false, MAP>),
                               dim3(grid), dim3(GY * GX), 0, s, p, edge);
        return hipGetLastError();
    }
    return hipSuccess;
}

template <class S>
static hipError_t dispatch2d(const Pass2D& p, int cfg, bool inverse, hipStream_t s) {
    switch (cfg) {
#define X(I, RY_, GY_, GX_, RM_, WPC_, MAP_) \
    case I:                                  \
        return launch2d<S, S, S, GY_, GX_, (WPC_ > 0), MAP_, RY_>(p, inverse, s);
        HAAR_2D_TILES(X)
#undef X
        default:
            return launch2d<S, S, S, 8, 32, false>(p, inverse, s);
    }
}

// Passes of a deep reduced-precision transform: the region (x_f32) and/or the
// pass's LL (ll_f32) live in FP32 scratch; detail bands keep the storage type.
// These run with the default tile shape.
template <class S>
static hipError_t dispatch2d_mixed(const Pass2D& p, bool x_f32, bool ll_f32, bool inverse,
                                   hipStream_t s) {
    if (x_f32 && ll_f32) return launch2d<StF32, S, StF32, 8, 32, false>(p, inverse, s);
    if (x_f32) return launch2d<StF32, S, S, 8, 32, false>(p, inverse, s);
    return launch2d<S, S, StF32, 8, 32, false>(p, inverse, s);
}

static hipError_t dispatch2d_dtype(const Pass2D& p, int dtype, int cfg, bool x_f32, bool ll_f32,
                                   bool inverse, hipStream_t s) {
    if (dtype == 0 || (!x_f32 && !ll_f32)) {
        switch (dtype) {
            case 0: return dispatch2d<StF32>(p, cfg, inverse, s);
            case 1: return dispatch2d<StBF16>(p, cfg, inverse, s);
            case 2: return dispatch2d<StF16>(p, cfg, inverse, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (dtype) {
        case 1: return dispatch2d_mixed<StBF16>(p, x_f32, ll_f32, inverse, s);
        case 2: return dispatch2d_mixed<StF16>(p, x_f32, ll_f32, inverse, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fwd2d(const Pass2D& p, int dtype, int cfg, bool x_f32, bool ll_f32, hipStream_t s) {
    return dispatch2d_dtype(p, dtype, cfg, x_f32, ll_f32, false, s);
}

hipError_t launch_inv2d(const Pass2D& p, int dtype, int cfg, bool x_f32, bool ll_f32, hipStream_t s) {
    return dispatch2d_dtype(p, dtype, cfg, x_f32, ll_f32, true, s);
}

}  // namespace haar
