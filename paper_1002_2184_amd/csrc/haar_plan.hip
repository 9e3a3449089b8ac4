// Batched transforms of uneven sizes: work-list plans and persistent kernels.
//
// A plan lists the work units of many items (2D: tiles, 1D: chunks), largest
// items first, and one persistent kernel per execute drains the list: every
// work-group claims the next unit with an atomic counter until the list is
// exhausted.  The last work-group to leave resets the counters, so that the
// next execute (or the next replay of a captured graph) starts from zero
// without any memset.
//
// 1D items deeper than one chunk (levels > 12 with 4096-sample chunks):
//   analysis  -- every chunk leaves its level-12 approximation in the item's
//                output (the prefix that the deeper levels later overwrite);
//                a second kernel, one work-group per deep item, computes the
//                remaining levels of that prefix on chip (the kernel boundary
//                orders the writes; no device-scope fences in the hot loop);
//   synthesis -- every chunk derives its own level-12 approximation by
//                walking down its ancestor path from a_L (one synthesis
//                butterfly per level), then runs its 12 on-chip levels.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <numeric>
#include <type_traits>
#include <vector>

#include "haar.h"
#include "haar_1d_chunk.h"
#include "haar_2d_tile.h"
#include "haar_internal.h"

namespace haar {

struct PlanItem2D {
    const void* in;
    void* out;
    int64_t h, w;
    int32_t levels, vec_ok;
};
struct PlanTile2D {
    int32_t item, ty, tx, full;
};
struct PlanItem1D {
    const void* in;
    void* out;
    int64_t n;
    int32_t levels;        // all levels of the item
    int32_t chunk_levels;  // levels done inside one chunk: min(levels, 12)
    int32_t nchunks;
    int32_t vec_ok;
    int64_t a32;           // deep items: offset of their level-12 values in the FP32 area
};
struct PlanChunk1D {
    int32_t item, chunk;
};

constexpr int kPlanNT1 = 256, kPlanE1 = 16;              // 1D chunk: 4096 samples
constexpr int kPlanC1 = kPlanNT1 * kPlanE1, kPlanLogC1 = 12;

// ---------------------------------------------------------------------------
// Counters: ctr[0] = next work unit, ctr[1] = work-groups done.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool claim(unsigned* ctr, unsigned* s_slot, unsigned total, unsigned& unit) {
    if (threadIdx.x == 0) *s_slot = atomicAdd(&ctr[0], 1u);
    __syncthreads();
    unit = *s_slot;
    __syncthreads();
    return unit < total;
}

__device__ __forceinline__ void retire(unsigned* ctr) {
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&ctr[1], 1u) == gridDim.x - 1) {   // every work-group has left the loop
            atomicExch(&ctr[0], 0u);
            atomicExch(&ctr[1], 0u);
        }
    }
}

// ---------------------------------------------------------------------------
// 2D
// ---------------------------------------------------------------------------
// Work-list walk of a plan kernel.  DYN: work-groups claim units with the
// atomic counter (balances units of very different cost); otherwise unit
// b, b + G, b + 2G, ... (no atomics; the units of a plan are nearly uniform
// and sorted largest item first).  The unit index is made wavefront-uniform
// so that the descriptors come through the scalar cache.  REMAP (one unit per
// work-group): work-groups are dealt round-robin to the 8 XCDs, so block b
// takes unit xcd_tile(b), which gives every XCD one contiguous range of the
// list; neighbouring tiles of an image then run on one XCD and share its L2.
// ONE: the grid has one work-group per unit; straight-line code without the
// walk loop, which needs fewer registers.
template <bool DYN, bool REMAP, bool ONE, class F>
__device__ __forceinline__ void walk_units(unsigned n, unsigned* ctr, unsigned* s_slot, F&& body) {
    if constexpr (ONE) {
        const unsigned b = blockIdx.x;
        if (b < n) body(REMAP ? (unsigned)xcd_tile(b, n) : b);
    } else if constexpr (DYN) {
        unsigned unit;
        while (claim(ctr, s_slot, n, unit)) {
            body((unsigned)__builtin_amdgcn_readfirstlane((int)unit));
            __syncthreads();   // LDS reuse by the next unit
        }
        retire(ctr);
    } else {
        const bool remap = REMAP && gridDim.x == n;
        for (unsigned unit = blockIdx.x; unit < n; unit += gridDim.x) {
            body(remap ? (unsigned)xcd_tile(unit, n) : unit);
            __syncthreads();
        }
    }
}

// REMAP: XCD-contiguous units (one work-group per unit): neighbouring tiles of
// an image run on one XCD, so the partial cache lines they share (rows of
// most images start inside a line) are fetched into that XCD's L2 once.
// WB: outputs with write-back stores (WriteBack<S>), so that partial lines
// written by two neighbouring tiles merge in L2 instead of being streamed to
// HBM twice.
// At least 5 wavefronts per SIMD: the 16-bit analysis kernels sit at the
// 96-register boundary of that occupancy.
template <class S, int GY, int GX, bool INV, bool DYN, bool REMAP, bool WB>
__global__ __launch_bounds__(GY* GX) __attribute__((amdgpu_waves_per_eu(5))) void plan2d_kernel(const PlanItem2D* __restrict__ items,
                                                        const PlanTile2D* __restrict__ tiles,
                                                        unsigned ntiles, unsigned* ctr) {
    constexpr int RX = 16 / S::kBytes;
    using SO = std::conditional_t<WB, WriteBack<S>, S>;   // storage of the outputs
    using G = Geo2D<S, 4, RX, GY, GX>;
    __shared__ float sm[G::SMEM];                          // analysis levels 3..L
    __shared__ unsigned s_slot;
    walk_units<DYN, REMAP, false>(ntiles, ctr, &s_slot, [&](unsigned unit) {
        const PlanTile2D d = tiles[unit];
        const PlanItem2D it = items[d.item];
        Pass2D p{};
        p.h = it.h;
        p.w = it.w;
        p.batch = 1;
        p.levels = it.levels;
        p.vec_ok = it.vec_ok;
        if (!INV) {
            p.src = it.in;
            p.det = it.out;
            p.ll = it.out;
            p.src_pitch = p.det_pitch = p.ll_pitch = it.w;
        } else {
            p.det = const_cast<void*>(it.in);
            p.ll = const_cast<void*>(it.in);
            p.dst = it.out;
            p.det_pitch = p.ll_pitch = p.dst_pitch = it.w;
        }
        if (!INV) {
            if (d.full) {
                FwdIn<4, RX> in;
                fwd2d_load<S, 4, RX, GY, GX, true>(p, 0, d.ty, d.tx, in);
                fwd2d_body<S, SO, SO, 4, RX, GY, GX, true>(p, 0, d.ty, d.tx, in, sm);
            } else {
                FwdIn<4, RX> in;
                fwd2d_load<S, 4, RX, GY, GX, false>(p, 0, d.ty, d.tx, in);
                fwd2d_body<S, SO, SO, 4, RX, GY, GX, false>(p, 0, d.ty, d.tx, in, sm);
            }
        } else {
            using In = InvInT<SO, S, S, 4, RX, GY, GX>;
            if (d.full) {
                In in;
                inv2d_load<SO, S, S, 4, RX, GY, GX, true>(p, 0, d.ty, d.tx, in);
                inv2d_body<SO, S, S, 4, RX, GY, GX, true>(p, 0, d.ty, d.tx, in);
            } else {
                In in;
                inv2d_load<SO, S, S, 4, RX, GY, GX, false>(p, 0, d.ty, d.tx, in);
                inv2d_body<SO, S, S, 4, RX, GY, GX, false>(p, 0, d.ty, d.tx, in);
            }
        }
    });
}

// ---------------------------------------------------------------------------
// 1D
// ---------------------------------------------------------------------------
// NTL: every item's chunks own whole cache lines (nontemporal loads).
template <class S, bool INV, bool DYN, bool ONE, bool NTL>
__global__ __launch_bounds__(kPlanNT1) void plan1d_kernel(const PlanItem1D* __restrict__ items,
                                                         const PlanChunk1D* __restrict__ chunks,
                                                         unsigned nunits, unsigned* ctr, float* a32) {
    constexpr int NW = kPlanNT1 / 64;
    __shared__ df smd[NW];
    __shared__ float smf[NW * 8];
    __shared__ float stage[kPlanC1];
    __shared__ unsigned s_slot;
    walk_units<DYN, false, ONE>(nunits, ctr, &s_slot, [&](unsigned unit) {
        const PlanChunk1D d = chunks[unit];
        const PlanItem1D it = items[d.item];
        Pass1D p{};
        p.n = it.n;
        p.batch = 1;
        p.levels = it.chunk_levels;
        p.vec_ok = it.vec_ok;
        const bool full = it.vec_ok && (int64_t)(d.chunk + 1) * kPlanC1 <= it.n;
        if (!INV) {
            // deep items: the chunk's level-12 approximation goes to the
            // FP32 area; a second kernel finishes the deeper levels
            p.src = it.in;
            p.det = it.out;
            if (it.levels > it.chunk_levels) {
                p.ll = a32 + it.a32;
                if (full)
                    fwd1d_chunk<S, S, StF32, kPlanE1, kPlanNT1, true, NTL>(p, 0, d.chunk, smd, stage);
                else
                    fwd1d_chunk<S, S, StF32, kPlanE1, kPlanNT1, false>(p, 0, d.chunk, smd, stage);
            } else {
                p.ll = it.out;
                if (full)
                    fwd1d_chunk<S, S, S, kPlanE1, kPlanNT1, true, NTL>(p, 0, d.chunk, smd, stage);
                else
                    fwd1d_chunk<S, S, S, kPlanE1, kPlanNT1, false>(p, 0, d.chunk, smd, stage);
            }
        } else {
            p.det = const_cast<void*>(it.in);
            p.ll = const_cast<void*>(it.in);
            p.dst = it.out;
            const bool deep = it.levels > it.chunk_levels;
            const float top = deep ? walk_down<S>(reinterpret_cast<const typename S::raw*>(it.in), it.n,
                                                  it.levels, kPlanLogC1, d.chunk)
                                   : 0.0f;
            if (full)
                inv1d_chunk<S, S, S, kPlanE1, kPlanNT1, true, false, NTL>(p, 0, d.chunk, smf, stage, deep, top);
            else
                inv1d_chunk<S, S, S, kPlanE1, kPlanNT1, false>(p, 0, d.chunk, smf, stage, deep, top);
        }
    });
}

// Second kernel of a 1D analysis plan: the levels beyond 12 of each deep
// item, one work-group per item (the kernel boundary orders the chunks'
// writes before these reads).
template <class S>
__global__ __launch_bounds__(256) void plan1d_finish_kernel(const PlanItem1D* __restrict__ items,
                                                            const int32_t* __restrict__ deep,
                                                            unsigned ndeep, const float* a32) {
    __shared__ df buf0[kFinishMax], buf1[kFinishMax];
    for (unsigned i = blockIdx.x; i < ndeep; i += gridDim.x) {
        const PlanItem1D it = items[deep[i]];
        finish1d<S>(reinterpret_cast<typename S::raw*>(it.out), a32 + it.a32, it.n, kPlanLogC1, it.levels,
                    buf0, buf1);
        __syncthreads();
    }
}

}  // namespace haar

using namespace haar;

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct haar_plan {
    int dim = 0;
    int dtype = 0;
    int inverse = 0;
    int cfg = 1;                       // 2D tile configuration (0: 32 rows x 16 vectors, 1: x 32)
    int sched = 0;                     // 0: strided work-list walk, 1: atomic claiming, 2: one unit per
                                       // work-group, 3 (2D): 2 with XCD-contiguous units, write-back stores,
                                       // 4 (2D): 2 with XCD-contiguous units
    std::vector<PlanItem2D> items2;
    std::vector<PlanTile2D> tiles2[2];  // per tile configuration
    std::vector<PlanItem1D> items1;
    std::vector<PlanChunk1D> chunks1;
    std::vector<int32_t> deep1;        // 1D items with more than 12 levels
    size_t off_items = 0, off_units = 0, off_deep = 0, off_a32 = 0, ws_bytes = 0;
    int64_t nunits = 0;
    int grid = 0;
    bool ntl1 = false;                 // 1D: every item's chunks own whole cache lines
    bool uploaded = false;
    const void* uploaded_to = nullptr;
};

namespace {

constexpr int kPlanCfgs2D = 2;          // tile configurations with plan kernels: 0 and 1
constexpr int kPlanScheds1D = 3;        // 0 strided walk, 1 atomic claiming, 2 one unit per work-group
constexpr int kPlanScheds2D = 5;        // the same, 3: 2 with XCD-contiguous units and write-back stores,
                                        // 4: 2 with XCD-contiguous units

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

bool overlap(const void* a, const void* b, uint64_t bytes) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bytes && y < x + bytes;
}

// LDS bytes per compute unit of the current device (cached per device)
int device_lds_per_cu() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 160 * 1024;
    int n = cache[dev].load(std::memory_order_relaxed);
    if (n == 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
            n <= 0)
            n = 160 * 1024;
        cache[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

template <class K>
int grid_for(K kernel, int threads, size_t lds_pad = 0) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds_pad) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return per_cu * device_cus();
}

// Grid of a plan launch: the resident work-groups of the device for the
// persistent schedules (0, 1), one work-group per unit for schedule 2 (the
// strided walk then runs each unit once; capped, beyond which it wraps).
constexpr int64_t kPlanGridCap = (int64_t)1 << 22;

int unit_grid(const haar_plan* pl, unsigned n, int resident);

// launch helpers -------------------------------------------------------------
// Address of a table inside the workspace; a grid query (haar_plan_info)
// passes no workspace, and then no address is formed.
static inline char* ws_at(void* ws, int64_t off) { return ws ? (char*)ws + off : nullptr; }

template <class S>
hipError_t launch_plan2d(const haar_plan* pl, void* ws, hipStream_t s, bool query_only, int* grid) {
    const PlanItem2D* items = (const PlanItem2D*)ws_at(ws, pl->off_items);
    const PlanTile2D* tiles = (const PlanTile2D*)ws_at(ws, pl->off_units);
    unsigned* ctr = (unsigned*)ws;
    const unsigned n = (unsigned)pl->nunits;
    const bool inv = pl->inverse != 0;
    // FP32 synthesis plans in 512-thread tiles run at most three work-groups
    // per CU: LDS that the kernel never touches, allocated at launch, caps
    // the occupancy (the 512 uneven images in FP32: 1.07 -> 1.02 ms).  The
    // analyses did not gain, and the 16-bit plans (256-thread tiles) ran
    // slower capped at 4, 3 or 2 per CU.
    auto lds_pad = [&](int threads, size_t stat) -> size_t {
        if (!inv || S::kBytes != 4 || threads != 512) return 0;
        const size_t want = (size_t)device_lds_per_cu() / 4 + 256;   // three fit in a CU, four do not
        return want > stat ? want - stat : 0;
    };
    auto go = [&](auto kernel, int threads) -> hipError_t {
        hipFuncAttributes fa{};
        const size_t stat = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kernel)) == hipSuccess
                                ? fa.sharedSizeBytes
                                : 0;
        const size_t pad = lds_pad(threads, stat);
        const int g = unit_grid(pl, n, grid_for(kernel, threads, pad));
        if (grid) *grid = g;
        if (query_only) return hipSuccess;
        hipLaunchKernelGGL(kernel, dim3(g), dim3(threads), pad, s, items, tiles, n, ctr);
        return hipGetLastError();
    };
    // schedules: 0 strided walk, 1 claiming, 2 one unit per work-group,
    // 3 the same XCD-contiguous with write-back stores, 4 XCD-contiguous
#define HAAR_PLAN2D_GO(GY_, GX_, DYN_, RM_, WB_)                                               \
    return inv ? go(plan2d_kernel<S, GY_, GX_, true, DYN_, RM_, WB_>, GY_ * GX_)               \
               : go(plan2d_kernel<S, GY_, GX_, false, DYN_, RM_, WB_>, GY_ * GX_)
#define HAAR_PLAN2D_SCHED(GY_, GX_)                                 \
    switch (pl->sched) {                                            \
        case 1: HAAR_PLAN2D_GO(GY_, GX_, true, false, false);       \
        case 3: HAAR_PLAN2D_GO(GY_, GX_, false, true, true);        \
        case 4: HAAR_PLAN2D_GO(GY_, GX_, false, true, false);       \
        default: HAAR_PLAN2D_GO(GY_, GX_, false, false, false);     \
    }
    if (pl->cfg == 0) {
        HAAR_PLAN2D_SCHED(8, 32)
    }
    HAAR_PLAN2D_SCHED(8, 64)
#undef HAAR_PLAN2D_SCHED
#undef HAAR_PLAN2D_GO
}

template <class S>
hipError_t launch_plan1d(const haar_plan* pl, void* ws, hipStream_t s, bool query_only, int* grid) {
    const PlanItem1D* items = (const PlanItem1D*)ws_at(ws, pl->off_items);
    const PlanChunk1D* chunks = (const PlanChunk1D*)ws_at(ws, pl->off_units);
    unsigned* ctr = (unsigned*)ws;
    float* a32 = (float*)ws_at(ws, pl->off_a32);
    const unsigned n = (unsigned)pl->nunits;
    auto go = [&](auto kernel) -> hipError_t {
        const int g = unit_grid(pl, n, grid_for(kernel, kPlanNT1));
        if (grid) *grid = g;
        if (query_only) return hipSuccess;
        hipLaunchKernelGGL(kernel, dim3(g), dim3(kPlanNT1), 0, s, items, chunks, n, ctr, a32);
        return hipGetLastError();
    };
    const bool dyn = pl->sched == 1;
    // synthesis with one work-group per unit: the straight-line kernel (61
    // VGPRs against 105) ran the 1024-signal batch in 0.35 ms against 0.47;
    // the analysis ran slower that way (0.32-0.34 against 0.31 ms)
    const bool one = pl->sched == 2 && (int64_t)n <= kPlanGridCap;
    if (pl->inverse)
        return dyn ? go(plan1d_kernel<S, true, true, false, false>)
                   : one ? (pl->ntl1 ? go(plan1d_kernel<S, true, false, true, true>)
                                     : go(plan1d_kernel<S, true, false, true, false>))
                         : go(plan1d_kernel<S, true, false, false, false>);
    hipError_t e = dyn ? go(plan1d_kernel<S, false, true, false, false>)
                       : pl->ntl1 ? go(plan1d_kernel<S, false, false, false, true>)
                                  : go(plan1d_kernel<S, false, false, false, false>);
    if (e != hipSuccess || query_only || pl->deep1.empty()) return e;
    const int32_t* deep = (const int32_t*)ws_at(ws, pl->off_deep);
    const unsigned nd = (unsigned)pl->deep1.size();
    hipLaunchKernelGGL(plan1d_finish_kernel<S>, dim3(nd), dim3(256), 0, s, items, deep, nd, a32);
    return hipGetLastError();
}

hipError_t launch_plan(const haar_plan* pl, void* ws, hipStream_t s, bool query_only, int* grid) {
    if (pl->dim == 2) {
        switch (pl->dtype) {
            case 0: return launch_plan2d<StF32>(pl, ws, s, query_only, grid);
            case 1: return launch_plan2d<StBF16>(pl, ws, s, query_only, grid);
            default: return launch_plan2d<StF16>(pl, ws, s, query_only, grid);
        }
    }
    switch (pl->dtype) {
        case 0: return launch_plan1d<StF32>(pl, ws, s, query_only, grid);
        case 1: return launch_plan1d<StBF16>(pl, ws, s, query_only, grid);
        default: return launch_plan1d<StF16>(pl, ws, s, query_only, grid);
    }
}

// Plan configurations: 2D, tile shape + 2 * schedule (0..7); 1D, the schedule (0..2).
int plan_configs(const haar_plan* pl) { return pl->dim == 2 ? kPlanScheds2D * kPlanCfgs2D : kPlanScheds1D; }

int unit_grid(const haar_plan* pl, unsigned n, int resident) {
    const int64_t units = std::max<int64_t>(1, n);
    if (pl->sched >= 2) return (int)std::min<int64_t>(units, kPlanGridCap);
    return (int)std::min<int64_t>(resident, units);
}
int plan_config_index(const haar_plan* pl) {
    return pl->dim == 2 ? pl->cfg + kPlanCfgs2D * pl->sched : pl->sched;
}

void layout(haar_plan* pl, size_t item_bytes, size_t nitems, size_t unit_bytes, int64_t nunits,
            size_t counters) {
    pl->off_items = align256(counters * sizeof(unsigned));
    pl->off_units = align256(pl->off_items + item_bytes * nitems);
    pl->ws_bytes = align256(pl->off_units + unit_bytes * (size_t)nunits);
    pl->nunits = nunits;
}

}  // namespace

extern "C" {

int haar_plan_create_2d(const haar_item_2d* items, int64_t count, int32_t dtype, int32_t inverse,
                        haar_plan** out) {
    if (!out) return set_error(HAAR_ERR_NULL, "out is NULL");
    *out = nullptr;
    if (dtype < 0 || dtype > 2) return set_error(HAAR_ERR_DTYPE, "dtype %d is not a haar_dtype", dtype);
    if (count < 1) return set_error(HAAR_ERR_PLAN, "a plan needs at least one item");
    if (!items) return set_error(HAAR_ERR_NULL, "items is NULL");
    const int eb = elem_bytes(dtype);
    for (int64_t i = 0; i < count; ++i) {
        const haar_item_2d& it = items[i];
        if (!it.in || !it.out) return set_error(HAAR_ERR_NULL, "item %lld: NULL pointer", (long long)i);
        if (it.height < 1 || it.width < 1 || it.height > (1 << 30) || it.width > (1 << 30))
            return set_error(HAAR_ERR_SHAPE, "item %lld: bad shape", (long long)i);
        const int maxl = std::min(kMaxPassLevels2D, max_levels(std::max(it.height, it.width)));
        if (it.levels < 1 || it.levels > maxl)
            return set_error(HAAR_ERR_LEVELS, "item %lld: levels %d outside [1, %d]", (long long)i,
                             it.levels, maxl);
        if (overlap(it.in, it.out, (uint64_t)(it.height * it.width * eb)))
            return set_error(HAAR_ERR_ALIAS, "item %lld: input and output overlap", (long long)i);
    }
    haar_plan* pl = new haar_plan();
    pl->dim = 2;
    pl->dtype = dtype;
    pl->inverse = inverse ? 1 : 0;
    // largest items first
    std::vector<int64_t> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
        return items[a].height * items[a].width > items[b].height * items[b].width;
    });
    for (int64_t oi = 0; oi < count; ++oi) {
        const haar_item_2d& it = items[order[oi]];
        PlanItem2D pi{};
        pi.in = it.in;
        pi.out = it.out;
        pi.h = it.height;
        pi.w = it.width;
        pi.levels = it.levels;
        // vector path: needs element-aligned pointers only
        const bool ok = aligned(it.in, eb) && aligned(it.out, eb);
        pi.vec_ok = ok ? 1 : 0;
        pl->items2.push_back(pi);
        for (int c = 0; c < kPlanCfgs2D; ++c) {
            const Tile2D tc = tile_config_2d(eb, c);
            const int64_t tx = (it.width + tc.tw() - 1) / tc.tw(), ty = (it.height + tc.th() - 1) / tc.th();
            for (int64_t y = 0; y < ty; ++y)
                for (int64_t x = 0; x < tx; ++x) {
                    const bool full = ok && (y + 1) * tc.th() <= it.height && (x + 1) * tc.tw() <= it.width;
                    pl->tiles2[c].push_back(PlanTile2D{(int32_t)oi, (int32_t)y, (int32_t)x, full ? 1 : 0});
                }
        }
    }
    if (pl->tiles2[0].size() >= (1u << 31)) {
        delete pl;
        return set_error(HAAR_ERR_SHAPE, "plan has too many tiles");
    }
    // measured defaults (512 uneven images, 4 levels; almost all rows of
    // such images start inside a cache line): the analysis runs one tile per
    // work-group with XCD-contiguous tiles and write-back stores (BF16 0.71
    // ms against 0.87 ms claiming tiles with streaming stores, FP32 1.06
    // against 1.33 ms); the synthesis runs one tile per work-group with
    // streaming stores (BF16 0.72 ms against 0.78 ms with the XCD-contiguous
    // write-back schedule and 0.74 ms XCD-contiguous with streaming stores,
    // although the latter fetches each shared partial line once: 1.4x the
    // algorithmic bytes read with the default order).  Tiles of 32 x 16
    // vectors for 16-bit data, 32 x 32 for FP32.
    const int fb = dtype != 0 ? 0 : 1;
    const int c = choose_config_2d(dtype, inverse != 0, items[order[0]].height, items[order[0]].width,
                                   items[order[0]].levels, fb);
    pl->cfg = tile_config_2d(eb, c).gx == 32 ? 0 : 1;
    pl->sched = inverse ? 2 : 3;
    layout(pl, sizeof(PlanItem2D), pl->items2.size(), sizeof(PlanTile2D),
           (int64_t)std::max(pl->tiles2[0].size(), pl->tiles2[1].size()), 2);
    pl->nunits = (int64_t)pl->tiles2[pl->cfg].size();
    *out = pl;
    return HAAR_OK;
}

int haar_plan_create_1d(const haar_item_1d* items, int64_t count, int32_t dtype, int32_t inverse,
                        haar_plan** out) {
    if (!out) return set_error(HAAR_ERR_NULL, "out is NULL");
    *out = nullptr;
    if (dtype < 0 || dtype > 2) return set_error(HAAR_ERR_DTYPE, "dtype %d is not a haar_dtype", dtype);
    if (count < 1) return set_error(HAAR_ERR_PLAN, "a plan needs at least one item");
    if (!items) return set_error(HAAR_ERR_NULL, "items is NULL");
    const int eb = elem_bytes(dtype);
    int64_t total_chunks = 0;
    for (int64_t i = 0; i < count; ++i) {
        const haar_item_1d& it = items[i];
        if (!it.in || !it.out) return set_error(HAAR_ERR_NULL, "item %lld: NULL pointer", (long long)i);
        if (it.length < 1 || it.length > ((int64_t)1 << 40))
            return set_error(HAAR_ERR_SHAPE, "item %lld: bad length", (long long)i);
        const int maxl = max_levels(it.length);
        if (it.levels < 1 || it.levels > maxl)
            return set_error(HAAR_ERR_LEVELS, "item %lld: levels %d outside [1, %d]", (long long)i,
                             it.levels, maxl);
        if (it.levels > kPlanLogC1 && ceil_shift_host(it.length, kPlanLogC1) > kFinishMax)
            return set_error(HAAR_ERR_UNSUPPORTED,
                             "item %lld: more than 12 levels on more than %d x 4096 samples in a plan",
                             (long long)i, kFinishMax);
        if (it.levels > kPlanLogC1 + 8)
            return set_error(HAAR_ERR_UNSUPPORTED, "item %lld: more than 20 levels in a plan", (long long)i);
        if (overlap(it.in, it.out, (uint64_t)(it.length * eb)))
            return set_error(HAAR_ERR_ALIAS, "item %lld: input and output overlap", (long long)i);
        total_chunks += (it.length + kPlanC1 - 1) / kPlanC1;
    }
    if (total_chunks >= (1ll << 31) || count >= (1ll << 30))
        return set_error(HAAR_ERR_SHAPE, "plan has too many chunks");
    haar_plan* pl = new haar_plan();
    pl->dim = 1;
    pl->dtype = dtype;
    pl->inverse = inverse ? 1 : 0;
    std::vector<int64_t> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return items[a].length > items[b].length; });
    int64_t a32_floats = 0;
    pl->ntl1 = true;
    for (int64_t oi = 0; oi < count; ++oi) {
        const haar_item_1d& it = items[order[oi]];
        // chunk spans of the signal and of its level-1/2 bands on whole lines
        pl->ntl1 = pl->ntl1 && aligned(it.in, 128) && aligned(it.out, 128) && (it.length * eb) % 128 == 0 &&
                   (ceil_shift_host(it.length, 1) * eb) % 128 == 0 &&
                   (ceil_shift_host(it.length, 2) * eb) % 128 == 0;
        PlanItem1D pi{};
        pi.in = it.in;
        pi.out = it.out;
        pi.n = it.length;
        pi.levels = it.levels;
        pi.chunk_levels = std::min(it.levels, kPlanLogC1);
        pi.nchunks = (int32_t)((it.length + kPlanC1 - 1) / kPlanC1);
        const bool ok = aligned(it.in, eb) && aligned(it.out, eb);   // vector path: element alignment
        pi.vec_ok = ok ? 1 : 0;
        pi.a32 = -1;
        if (pi.levels > pi.chunk_levels) {
            pl->deep1.push_back((int32_t)oi);
            pi.a32 = a32_floats;
            a32_floats += (pi.nchunks + 63) & ~63;
        }
        pl->items1.push_back(pi);
        for (int32_t c = 0; c < pi.nchunks; ++c) pl->chunks1.push_back(PlanChunk1D{(int32_t)oi, c});
    }
    layout(pl, sizeof(PlanItem1D), pl->items1.size(), sizeof(PlanChunk1D), (int64_t)pl->chunks1.size(), 2);
    // measured default (1024 signals 2^10..2^20): one chunk per work-group,
    // 0.31 ms against 0.34 ms for the strided persistent walk
    pl->sched = 2;
    pl->off_deep = pl->ws_bytes;
    pl->off_a32 = align256(pl->off_deep + sizeof(int32_t) * (pl->deep1.size() + 1));
    pl->ws_bytes = align256(pl->off_a32 + sizeof(float) * (size_t)a32_floats);
    *out = pl;
    return HAAR_OK;
}

int haar_plan_workspace_size(const haar_plan* plan, size_t* bytes) {
    if (!plan || !bytes) return set_error(HAAR_ERR_NULL, "plan or bytes is NULL");
    *bytes = plan->ws_bytes;
    return HAAR_OK;
}

int haar_plan_upload(haar_plan* plan, void* workspace, void* stream) {
    if (!plan) return set_error(HAAR_ERR_PLAN, "plan is NULL");
    if (!workspace || !aligned(workspace, 256))
        return set_error(HAAR_ERR_WORKSPACE, "workspace is NULL or not 256-byte aligned");
    if (int rc = fault_injected(); rc != HAAR_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)workspace;
    hipError_t e = hipMemsetAsync(ws, 0, plan->off_items, s);
    if (e != hipSuccess) return hip_error(e, "hipMemsetAsync (plan counters)");
    const void* it = plan->dim == 2 ? (const void*)plan->items2.data() : (const void*)plan->items1.data();
    const size_t itb = plan->dim == 2 ? plan->items2.size() * sizeof(PlanItem2D)
                                      : plan->items1.size() * sizeof(PlanItem1D);
    e = hipMemcpyAsync(ws + plan->off_items, it, itb, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_error(e, "hipMemcpyAsync (plan items)");
    if (plan->dim == 2) {
        e = hipMemcpyAsync(ws + plan->off_units, plan->tiles2[plan->cfg].data(),
                           plan->tiles2[plan->cfg].size() * sizeof(PlanTile2D), hipMemcpyHostToDevice, s);
    } else {
        e = hipMemcpyAsync(ws + plan->off_units, plan->chunks1.data(),
                           plan->chunks1.size() * sizeof(PlanChunk1D), hipMemcpyHostToDevice, s);
        if (e == hipSuccess && !plan->deep1.empty())
            e = hipMemcpyAsync(ws + plan->off_deep, plan->deep1.data(),
                               plan->deep1.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
    }
    if (e != hipSuccess) return hip_error(e, "hipMemcpyAsync (plan work-list)");
    plan->uploaded = true;
    plan->uploaded_to = workspace;
    return HAAR_OK;
}

int haar_plan_execute(const haar_plan* plan, void* workspace, void* stream) {
    if (!plan) return set_error(HAAR_ERR_PLAN, "plan is NULL");
    if (!workspace) return set_error(HAAR_ERR_WORKSPACE, "workspace is NULL");
    if (!plan->uploaded || plan->uploaded_to != workspace)
        return set_error(HAAR_ERR_PLAN, "plan was not uploaded to this workspace");
    if (int rc = fault_injected(); rc != HAAR_OK) return rc;
    hipError_t e = launch_plan(plan, workspace, (hipStream_t)stream, false, nullptr);
    return e == hipSuccess ? HAAR_OK : hip_error(e, "plan launch");
}

int haar_plan_info(const haar_plan* plan, int64_t* tiles, int32_t* grid) {
    if (!plan) return set_error(HAAR_ERR_PLAN, "plan is NULL");
    if (tiles) *tiles = plan->nunits;
    if (grid) {
        int g = 0;
        hipError_t e = launch_plan(plan, nullptr, nullptr, true, &g);
        if (e != hipSuccess) return hip_error(e, "occupancy query");
        *grid = g;
    }
    return HAAR_OK;
}

int haar_plan_set_config(haar_plan* plan, int32_t config) {
    if (!plan) return set_error(HAAR_ERR_PLAN, "plan is NULL");
    if (config < 0 || config >= plan_configs(plan))
        return set_error(HAAR_ERR_UNSUPPORTED, "plan configuration %d not available", config);
    if (plan->dim == 2) {
        plan->cfg = config % kPlanCfgs2D;
        plan->sched = config / kPlanCfgs2D;
        plan->nunits = (int64_t)plan->tiles2[plan->cfg].size();
    } else {
        plan->sched = config;
    }
    plan->uploaded = false;          // the work-list may have changed: upload again
    plan->uploaded_to = nullptr;
    return HAAR_OK;
}

int haar_plan_tune(haar_plan* plan, void* workspace, void* stream, int32_t* choice) {
    if (!plan) return set_error(HAAR_ERR_PLAN, "plan is NULL");
    if (!workspace || !choice) return set_error(HAAR_ERR_NULL, "workspace or choice is NULL");
    hipStream_t s = (hipStream_t)stream;
    const int ncfg = plan_configs(plan);
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return set_error(HAAR_ERR_HIP, "hipEventCreate");
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return set_error(HAAR_ERR_HIP, "hipEventCreate");
    }
    int best = plan_config_index(plan), rc = HAAR_OK;
    float best_ms = 1e30f;
    for (int c = 0; c < ncfg && rc == HAAR_OK; ++c) {
        if ((rc = haar_plan_set_config(plan, c)) != HAAR_OK) break;
        if ((rc = haar_plan_upload(plan, workspace, stream)) != HAAR_OK) break;
        for (int i = 0; i < 2 && rc == HAAR_OK; ++i) rc = haar_plan_execute(plan, workspace, stream);
        std::vector<float> ts;
        for (int i = 0; i < 5 && rc == HAAR_OK; ++i) {
            (void)hipEventRecord(a, s);
            rc = haar_plan_execute(plan, workspace, stream);
            (void)hipEventRecord(b, s);
            if (hipEventSynchronize(b) != hipSuccess) rc = set_error(HAAR_ERR_HIP, "hipEventSynchronize");
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, a, b);
            ts.push_back(ms);
        }
        if (rc == HAAR_OK) {
            std::sort(ts.begin(), ts.end());
            if (ts[ts.size() / 2] < best_ms) {
                best_ms = ts[ts.size() / 2];
                best = c;
            }
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc != HAAR_OK) return rc;
    if ((rc = haar_plan_set_config(plan, best)) != HAAR_OK) return rc;
    if ((rc = haar_plan_upload(plan, workspace, stream)) != HAAR_OK) return rc;
    *choice = best;
    return HAAR_OK;
}

int haar_plan_destroy(haar_plan* plan) {
    delete plan;
    return HAAR_OK;
}

}  // extern "C"
