// Host-visible description of the fused passes and their launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace haar {

// One fused 2D pass: `levels` (1..5) levels on an h x w region.
//   analysis : src (region) -> det (detail bands, packed-layout buffer) + ll
//   synthesis: ll + det     -> dst (region)
// Pitches and batch strides are in elements.
struct Pass2D {
    const void* src; int64_t src_pitch, src_bstride;
    void* det;       int64_t det_pitch, det_bstride;
    void* ll;        int64_t ll_pitch, ll_bstride;
    void* dst;       int64_t dst_pitch, dst_bstride;
    int64_t h, w, batch;
    int32_t levels;
    int32_t vec_ok;                         // launch-wide: bases/pitches/band origins aligned
    int64_t tiles_x, tiles_y, tiles_per_item, total_tiles;
    int64_t full_x, full_y;                 // tiles that lie entirely inside the region
    int32_t remap;                          // deal contiguous tile ranges to each XCD
    int64_t persist;                        // interior grid size (0 = one tile per work-group)
    int32_t ntl;                            // every tile owns whole cache lines: nontemporal loads
    int32_t wb;                             // analysis outputs with write-back stores (tiles share lines)
    int32_t pace;                           // 16-bit outputs of an aligned layout: paced stores (with ntl)
};

// One fused 1D pass: `levels` levels on a length-n region (chunks of C).
struct Pass1D {
    const void* src; int64_t src_bstride;
    void* det;       int64_t det_bstride;
    void* ll;        int64_t ll_bstride;
    void* dst;       int64_t dst_bstride;
    int64_t n, batch;
    int32_t levels;
    int32_t vec_ok;
    int64_t chunks_per_item, total_chunks;
    int32_t remap;                          // deal contiguous chunk ranges to each XCD
    int32_t levels_total;                   // synthesis with walk: all levels of the transform
    int32_t ntl;                            // every chunk owns whole cache lines: nontemporal loads
};

// Tile shapes of the 2D kernels (per storage width): rows/cols per thread
// and the thread grid of one work-group.
struct Tile2D {
    int ry, rx, gy, gx;
    int remap;
    int wg_per_cu;                          // persistent interior grid: work-groups per CU
    int map;                                // 1: wavefront-local analysis thread map
    int th() const { return gy * ry; }
    int tw() const { return gx * rx; }
    int threads() const { return gy * gx; }
};

constexpr int kMaxPassLevels2D = 5;

int num_tile_configs_2d(int elem_bytes);
Tile2D tile_config_2d(int elem_bytes, int index);

// dtype: 0 f32, 1 bf16, 2 f16 (storage of the tensors the caller passed).
// x_f32 / ll_f32: the pass's region / deepest approximation lives in FP32
// scratch (passes of a deep reduced-precision transform; default tile shape).
// Return hipError_t of the launch.
hipError_t launch_fwd2d(const Pass2D& p, int dtype, int cfg, bool x_f32, bool ll_f32, hipStream_t s);
hipError_t launch_inv2d(const Pass2D& p, int dtype, int cfg, bool x_f32, bool ll_f32, hipStream_t s);

// 1D chunk kernels: chunk = threads * elems_per_thread; on-chip depth log2(chunk).
struct Chunk1D {
    int threads, ept;
    int remap;
    int chunk() const { return threads * ept; }
};
int num_chunk_configs_1d();
Chunk1D chunk_config_1d(int index);
hipError_t launch_fwd1d(const Pass1D& p, int dtype, int cfg, bool x_f32, bool ll_f32, hipStream_t s);
hipError_t launch_inv1d(const Pass1D& p, int dtype, int cfg, bool x_f32, bool ll_f32, hipStream_t s);
// Deep 1D in two stages.  finish: levels lc+1..L of every item (one
// work-group per item) into the prefix of p.det; the level-lc input is the
// FP32 buffer p.ll when src32, else that prefix itself.
// walk: one synthesis pass whose chunks derive their deepest approximation
// from a_L (p.levels = chunk depth, p.levels_total = L).
constexpr int kFinishMaxHost = 1024;
constexpr int kMaxWalkHost = 24;
hipError_t launch_finish1d(const Pass1D& p, int dtype, int lc, int L, bool src32, hipStream_t s);
hipError_t launch_inv1d_walk(const Pass1D& p, int dtype, int cfg, hipStream_t s);

}  // namespace haar
