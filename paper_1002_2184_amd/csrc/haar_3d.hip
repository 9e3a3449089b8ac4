// Separable 3D Haar transform of volumes [batch][d][h][w], the paper's
// medical-image use carried to volumetric data.  One level applies the fast
// analysis bank (Sec. III, Eq. (11)-(12), Fig. 4) along every x line
// (width), then every y line (height), then every z line (depth) of the
// current LLL region; the next level recurses on the LLL octant.  Synthesis
// (Sec. IV, Eq. (19), Fig. 7) undoes the three axes in reverse, levels L..1.
// Odd counts follow the carry rule of the 1D bank on each axis.
//
// Packed layout: after level j the region [0, D_{j-1}) x [0, H_{j-1}) x
// [0, W_{j-1}) holds eight octants split at D_j = ceil(D_{j-1}/2) (and H_j,
// W_j); octant (bx, by, bz) holds the band that is high-pass along the axes
// whose bit is set.
//
// One work-group owns a tile of 8 x 8 x 64 samples (z, y, x; interior
// tiles of 16-bit data are 128 wide), so a pass fuses three levels.
// Interior tiles run a register path: level 1 inside each thread
// (2 x 2 x 2 blocks), level 2 across lanes with shuffles, level 3 on one
// wavefront through LDS.  Edge tiles (and odd counts) run a generic path
// that takes whole 2 x 2 x 2 blocks per thread, level by level, with the
// carry rule on each axis and only the LLL regions in LDS.  Deeper
// transforms chain passes through scratch; when the region left by the
// first pass is small, all the remaining levels run in one tail launch of
// one work-group per volume.
//
// Arithmetic: samples are widened to FP64, which gfx950 executes at the
// rate of unpacked FP32.  One FP64 add replaces the six-operation pair sum
// that keeps an FP32 approximation exact, the sums of 8 FP32 samples are
// exact, and each output is rounded once to the storage type.  The
// approximation grows by 2^(3/2) per level, so this matters more in 3D than
// in 1D or 2D.
#include <type_traits>
#include <vector>

#include "haar.h"
#include "haar_device.h"
#include "haar_internal.h"

namespace haar {

namespace {

constexpr int kTZ = 8, kTY = 8, kTX = 64;       // generic tile
constexpr int kMaxPassLevels3D = 3;            // log2 of the tile's shortest side
constexpr int kThreads3 = 256;
constexpr double kRs2d = kRsqrt2;               // b00 = a00 = 1/sqrt2
constexpr double kC3 = kRsqrt2 * 0.5;           // (1/sqrt2)^3 = 1/(2 sqrt2)

struct Pass3D {
    // analysis: src (region) -> det (bands) + ll (deepest LLL of the pass)
    // synthesis: ll + det -> dst (region)
    // Strides in elements: plane (z), row (y), item (batch).
    const void* src; int64_t src_p, src_r, src_b;
    void* dst;       int64_t dst_p, dst_r, dst_b;
    void* ll;        int64_t ll_p, ll_r, ll_b;
    void* det;       int64_t det_p, det_r, det_b;
    int64_t d, h, w, batch;                    // region of this pass
    int32_t levels;                            // 1..3
    int64_t ntz, nty, ntx;                     // tiles per axis
    int64_t fz, fy, fx;                        // interior tiles per axis (register path)
    int64_t cx0, ncx;                          // x where interior tiles end; generic tiles after it
    int64_t nfull, nedge;                      // interior / other tiles, all items
};

// Value access of a region, LLL or scratch buffer: storage type S, or FP64
// scratch (DF).
template <class S, bool DF>
__device__ __forceinline__ double ld_val(const void* base, int64_t i) {
    if constexpr (DF)
        return reinterpret_cast<const double*>(base)[i];
    else
        return (double)S::ld(reinterpret_cast<const typename S::raw*>(base)[i]);
}

template <class S, bool DF>
__device__ __forceinline__ void st_val(void* base, int64_t i, double v) {
    if constexpr (DF)
        reinterpret_cast<double*>(base)[i] = v;
    else
        st1_cached<S>(reinterpret_cast<typename S::raw*>(base) + i, (float)v);
}

// Samples i and i + 1 of a row (both when `two`, else i alone): one 8-byte
// store of storage samples or one 16-byte store of FP64 scratch.
template <class S, bool DF>
__device__ __forceinline__ void st_pair(void* base, int64_t i, bool two, double a, double b) {
    if (!two) {
        st_val<S, DF>(base, i, a);
        return;
    }
    if constexpr (DF) {
        double* p = reinterpret_cast<double*>(base) + i;
        p[0] = a;
        p[1] = b;
    } else {
        const float f[2] = {(float)a, (float)b};
        st_vec<S, 2>(reinterpret_cast<typename S::raw*>(base) + i, f);
    }
}

// Butterflies over the three axes of a 2 x 2 x 2 block, index dx | dy<<1 |
// dz<<2.  Analysis leaves at index c the unscaled coefficient that is
// high-pass along the axes whose bit is set in c (pair: (v0 + v1, v1 - v0));
// synthesis applies the transposed stages ((a - d, a + d)).  Multiplying by
// 1/(2 sqrt2) gives the orthonormal values.
template <bool INV, class T>
__device__ __forceinline__ void bfly8(T* q) {
#pragma unroll
    for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (!(i & bit)) {
                const T a = q[i], b = q[i | bit];
                q[i] = INV ? a - b : a + b;
                q[i | bit] = INV ? a + b : b - a;
            }
}

// Sizes of the LLL region after level j of the pass; the high halves of the
// level-j octants start there on each axis.
struct Level3 {
    int64_t D, H, W;
};

__device__ __forceinline__ Level3 level_sizes(const Pass3D& p, int j) {
    return {ceil_shift(p.d, j), ceil_shift(p.h, j), ceil_shift(p.w, j)};
}

// ---------------------------------------------------------------------------
// Generic path (edge tiles, odd counts): one pass per level over the
// level's 2 x 2 x 2 blocks.  A thread takes whole blocks: it reads the
// block's (up to) 8 values, runs the three axis butterflies with the carry
// rule on every axis whose partner is missing, writes the detail octants
// straight to their packed positions and the LLL value to LDS for the next
// level (or to its final place after the pass's last level).  Level 1
// reads the region from memory and the synthesis's level 1 writes it, so
// only the small LLL regions cross LDS, with one barrier per level.
// ---------------------------------------------------------------------------

// Local sample counts of a tile: the tile holds c samples of the region on
// an axis, hence ceil(c / 2^j) samples of the level-j LLL region (tile
// origins are multiples of 2^3).
struct Counts3 {
    int z, y, x;                               // samples of the region in the tile
    __device__ __forceinline__ int cz(int j) const { return (z + (1 << j) - 1) >> j; }
    __device__ __forceinline__ int cy(int j) const { return (y + (1 << j) - 1) >> j; }
    __device__ __forceinline__ int cx(int j) const { return (x + (1 << j) - 1) >> j; }
};

__device__ __forceinline__ Counts3 tile_counts(const Pass3D& p, int64_t oz, int64_t oy, int64_t ox) {
    return {(int)min<int64_t>(kTZ, p.d - oz), (int)min<int64_t>(kTY, p.h - oy),
            (int)min<int64_t>(kTX, p.w - ox)};
}

// Block grid of level j in a tile: (4 x 4 x 32) >> (j - 1) slots; slot s ->
// (bz, by, bx) with bx fastest.  LDS holds the LLL region of each level in
// the same dense layout (pitches YB * XB and XB).
struct Blocks3 {
    int xs, ys;                                // log2 of the slot grid's x and y extent
    __device__ __forceinline__ explicit Blocks3(int j) : xs(6 - j), ys(3 - j) {}
    __device__ __forceinline__ int n() const { return 1 << (xs + ys + ys); }
    __device__ __forceinline__ int bx(int s) const { return s & ((1 << xs) - 1); }
    __device__ __forceinline__ int by(int s) const { return (s >> xs) & ((1 << ys) - 1); }
    __device__ __forceinline__ int bz(int s) const { return s >> (xs + ys); }
    __device__ __forceinline__ int at(int z, int y, int x) const { return (z << (xs + ys)) + (y << xs) + x; }
};
constexpr int kLll1 = 4 * 4 * 32, kLll2 = 2 * 2 * 16;   // LLL regions of levels 1 and 2 in LDS

// Offset of the level-j LLL region (j = 1, 2) in the generic path's LDS.
__device__ __forceinline__ int lll_off(int j) { return j == 1 ? 0 : kLll1; }
constexpr int kSlots1 = kLll1 / kThreads3;              // level-1 blocks per thread

// Analysis butterflies of one block with the carry rule: along an axis
// whose partner is missing (flag false) the value passes unscaled and that
// axis has no detail.  Index dx | dy << 1 | dz << 2; entries of missing
// samples are never used.
__device__ __forceinline__ void block_fwd(double* q, bool fx, bool fy, bool fz) {
    const bool f[3] = {fx, fy, fz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int bit = 1 << a;
        if (!f[a]) continue;
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (!(i & bit)) {
                const double x0 = q[i], x1 = q[i | bit];
                q[i] = (x0 + x1) * kRs2d;              // Eq. (11)
                q[i | bit] = (x1 - x0) * kRs2d;        // Eq. (12)
            }
    }
}

// Synthesis of one block (Eq. (19) per complete axis; carry otherwise).
__device__ __forceinline__ void block_inv(double* q, bool fx, bool fy, bool fz) {
    const bool f[3] = {fx, fy, fz};
#pragma unroll
    for (int a = 2; a >= 0; --a) {
        const int bit = 1 << a;
        if (!f[a]) continue;
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (!(i & bit)) {
                const double lo = q[i], hi = q[i | bit];
                q[i] = (lo - hi) * kRs2d;              // even phase
                q[i | bit] = (lo + hi) * kRs2d;        // odd phase
            }
    }
}

// Packed position of code c of the level-j block (bz, by, bx) in a tile at
// (oz, oy, ox): the low half of an axis at o / 2^j + b, the high half at
// N_j + o / 2^j + b.
__device__ __forceinline__ int64_t octant_pos(const Pass3D& p, const Level3& Lj, int j, int c, int64_t oz,
                                              int64_t oy, int64_t ox, int bz, int by, int bx) {
    const int64_t gz = ((c & 4) ? Lj.D : 0) + (oz >> j) + bz;
    const int64_t gy = ((c & 2) ? Lj.H : 0) + (oy >> j) + by;
    const int64_t gx = ((c & 1) ? Lj.W : 0) + (ox >> j) + bx;
    return gz * p.det_p + gy * p.det_r + gx;
}

template <class S, bool SRCDF, bool LLDF>
__device__ void fwd3d_lds(const Pass3D& p, int64_t item, int64_t oz, int64_t oy, int64_t ox, double* sm) {
    using raw = typename S::raw;
    const Counts3 c = tile_counts(p, oz, oy, ox);
    const int J = p.levels;
    raw* det = reinterpret_cast<raw*>(p.det) + item * p.det_b;
    for (int j = 1; j <= J; ++j) {
        const Blocks3 B(j);
        const Blocks3 P(j - 1 > 0 ? j - 1 : 1);   // layout of the level-(j-1) LLL in LDS
        const int nz = c.cz(j - 1), ny = c.cy(j - 1), nx = c.cx(j - 1);
        const int bz_n = c.cz(j), by_n = c.cy(j), bx_n = c.cx(j);
        const Level3 Lj = level_sizes(p, j);
#pragma unroll
        for (int k = 0; k < kSlots1; ++k) {
            const int s = threadIdx.x + kThreads3 * k;
            if (s >= B.n()) continue;
            const int bx = B.bx(s), by = B.by(s), bz = B.bz(s);
            if (bz >= bz_n || by >= by_n || bx >= bx_n) continue;
            const bool fx = 2 * bx + 1 < nx, fy = 2 * by + 1 < ny, fz = 2 * bz + 1 < nz;
            double q[8];
#pragma unroll
            for (int r = 0; r < 4; ++r) {          // the block's rows (dy, dz)
                const int dy = r & 1, dz = r >> 1;
                q[2 * r] = q[2 * r + 1] = 0.0;
                if ((dy && !fy) || (dz && !fz)) continue;
                const int z = 2 * bz + dz, y = 2 * by + dy, x = 2 * bx;
                if (j == 1) {   // per sample: pair loads measured 3x slower here
                    const int64_t g = item * p.src_b + (oz + z) * p.src_p + (oy + y) * p.src_r + ox + x;
                    q[2 * r] = ld_val<S, SRCDF>(p.src, g);
                    if (fx) q[2 * r + 1] = ld_val<S, SRCDF>(p.src, g + 1);
                } else {
                    const int o = lll_off(j - 1) + P.at(z, y, x);
                    q[2 * r] = sm[o];
                    if (fx) q[2 * r + 1] = sm[o + 1];
                }
            }
            block_fwd(q, fx, fy, fz);
#pragma unroll
            for (int code = 1; code < 8; ++code)
                if ((!(code & 1) || fx) && (!(code & 2) || fy) && (!(code & 4) || fz))
                    st1_cached<S>(det + octant_pos(p, Lj, j, code, oz, oy, ox, bz, by, bx), (float)q[code]);
            if (j == J)
                st_val<S, LLDF>(p.ll, item * p.ll_b + ((oz >> j) + bz) * p.ll_p + ((oy >> j) + by) * p.ll_r +
                                          (ox >> j) + bx, q[0]);
            else
                sm[lll_off(j) + B.at(bz, by, bx)] = q[0];
        }
        if (j < J) __syncthreads();
    }
}

template <class S, bool DSTDF, bool LLDF>
__device__ void inv3d_lds(const Pass3D& p, int64_t item, int64_t oz, int64_t oy, int64_t ox, double* sm) {
    using raw = typename S::raw;
    const Counts3 c = tile_counts(p, oz, oy, ox);
    const int J = p.levels;
    const raw* det = reinterpret_cast<const raw*>(p.det) + item * p.det_b;
    for (int j = J; j >= 1; --j) {
        const Blocks3 B(j);
        const Blocks3 P(j - 1 > 0 ? j - 1 : 1);
        const int nz = c.cz(j - 1), ny = c.cy(j - 1), nx = c.cx(j - 1);
        const int bz_n = c.cz(j), by_n = c.cy(j), bx_n = c.cx(j);
        const Level3 Lj = level_sizes(p, j);
#pragma unroll
        for (int k = 0; k < kSlots1; ++k) {
            const int s = threadIdx.x + kThreads3 * k;
            if (s >= B.n()) continue;
            const int bx = B.bx(s), by = B.by(s), bz = B.bz(s);
            if (bz >= bz_n || by >= by_n || bx >= bx_n) continue;
            const bool fx = 2 * bx + 1 < nx, fy = 2 * by + 1 < ny, fz = 2 * bz + 1 < nz;
            double q[8];
            q[0] = j == J ? ld_val<S, LLDF>(p.ll, item * p.ll_b + ((oz >> j) + bz) * p.ll_p +
                                                      ((oy >> j) + by) * p.ll_r + (ox >> j) + bx)
                          : sm[lll_off(j) + B.at(bz, by, bx)];
#pragma unroll
            for (int code = 1; code < 8; ++code) {
                q[code] = 0.0;
                if ((!(code & 1) || fx) && (!(code & 2) || fy) && (!(code & 4) || fz))
                    q[code] = (double)ld1<S>(det + octant_pos(p, Lj, j, code, oz, oy, ox, bz, by, bx));
            }
            block_inv(q, fx, fy, fz);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int dy = r & 1, dz = r >> 1;
                if ((dy && !fy) || (dz && !fz)) continue;
                const int z = 2 * bz + dz, y = 2 * by + dy, x = 2 * bx;
                if (j == 1) {
                    const int64_t g = item * p.dst_b + (oz + z) * p.dst_p + (oy + y) * p.dst_r + ox + x;
                    st_pair<S, DSTDF>(p.dst, g, fx, q[2 * r], q[2 * r + 1]);
                } else {
                    const int o = lll_off(j - 1) + P.at(z, y, x);
                    sm[o] = q[2 * r];
                    if (fx) sm[o + 1] = q[2 * r + 1];
                }
            }
        }
        if (j > 1) __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Register path for interior tiles.
//
// Thread map (256 threads, 4 wavefronts): tx = lane & 15 owns the RX
// samples x in [RX tx, RX tx + RX) (RX = 16 bytes of storage: 4 FP32 or 8
// BF16/FP16 samples, so an interior tile is 16 RX wide); ty = lane bit 4 |
// wave bit 0 << 1 owns rows 2 ty, 2 ty + 1; tz = lane bit 5 | wave bit 1 << 1
// owns planes 2 tz, 2 tz + 1.  Each load instruction reads four 16-lane row
// segments of 16 RX samples, and each level-1 band store writes four rows of
// 8 RX bytes (128 B in both formats).  A thread's RX/2 blocks of 2 x 2 x 2
// give level 1; the level-2 partners along y and z are lanes ^ 16 and ^ 32
// of the same wavefront; level 3 combines the four wavefronts through LDS.
// ---------------------------------------------------------------------------
struct Map3 {
    int lane, wv, tx, ty, tz;
    bool yo, zo;                               // odd level-1 row / plane of a level-2 pair
};

__device__ __forceinline__ Map3 map3() {
    Map3 m;
    m.lane = threadIdx.x & 63;
    m.wv = threadIdx.x >> 6;
    m.tx = m.lane & 15;
    m.ty = ((m.lane >> 4) & 1) | ((m.wv & 1) << 1);
    m.tz = ((m.lane >> 5) & 1) | ((m.wv >> 1) << 1);
    m.yo = (m.lane >> 4) & 1;
    m.zo = (m.lane >> 5) & 1;
    return m;
}

template <class S, bool RDF>
struct Rx3 {
    // samples per thread along x: 16 bytes of storage, or 4 FP64 values
    // when the region is scratch (a deep pass)
    static constexpr int RX = RDF ? 4 : 16 / S::kBytes;
    static constexpr int NB = RX / 2;          // level-1 blocks per thread
    static constexpr int NP = NB / 2;          // level-2 blocks per thread (along x)
    static constexpr int TX = 16 * RX;         // interior tile width
    static constexpr int X2 = 16 * NP;         // LLL_2 width of a tile
};

template <class S, bool RDF, int LV, bool LLDF>
__device__ void fwd3d_regs(const Pass3D& p, int64_t item, int64_t oz, int64_t oy, int64_t ox, double* sm) {
    using raw = typename S::raw;
    using R = Rx3<S, RDF>;
    constexpr int RX = R::RX, NB = R::NB, NP = R::NP;
    const Map3 m = map3();
    const int64_t sb = item * p.src_b + (oz + 2 * m.tz) * p.src_p + (oy + 2 * m.ty) * p.src_r + ox + RX * m.tx;
    raw* det = reinterpret_cast<raw*>(p.det) + item * p.det_b;

    double v[2][2][RX];
    if constexpr (RDF) {
        const double* src = reinterpret_cast<const double*>(p.src) + sb;
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                for (int e = 0; e < RX; ++e) v[dz][dy][e] = src[dz * p.src_p + dy * p.src_r + e];
    } else {
        const raw* src = reinterpret_cast<const raw*>(p.src) + sb;
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy) {
                float f[RX];
                ld_vec<S, RX>(src + dz * p.src_p + dy * p.src_r, f);
#pragma unroll
                for (int e = 0; e < RX; ++e) v[dz][dy][e] = (double)f[e];
            }
    }

    // level 1: NB blocks per thread
    const Level3 L1 = level_sizes(p, 1);
    double lll[NB];
    float d1[8][NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        double q[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) q[i] = v[i >> 2][(i >> 1) & 1][2 * b + (i & 1)];
        bfly8<false>(q);
        lll[b] = q[0] * kC3;
#pragma unroll
        for (int i = 1; i < 8; ++i) d1[i][b] = (float)(q[i] * kC3);
    }
#pragma unroll
    for (int c = 1; c < 8; ++c) {
        const int64_t gz = ((c >> 2) ? L1.D : 0) + (oz >> 1) + m.tz;
        const int64_t gy = (((c >> 1) & 1) ? L1.H : 0) + (oy >> 1) + m.ty;
        const int64_t gx = ((c & 1) ? L1.W : 0) + (ox >> 1) + NB * m.tx;
        st_vec<S, NB>(det + gz * p.det_p + gy * p.det_r + gx, d1[c]);
    }
    if constexpr (LV == 1) {
        const int64_t g = item * p.ll_b + ((oz >> 1) + m.tz) * p.ll_p + ((oy >> 1) + m.ty) * p.ll_r +
                          (ox >> 1) + NB * m.tx;
        if constexpr (LLDF) {
            double* ll = reinterpret_cast<double*>(p.ll);
#pragma unroll
            for (int b = 0; b < NB; ++b) ll[g + b] = lll[b];
        } else {
            float o[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) o[b] = (float)lll[b];
            st_vec<S, NB>(reinterpret_cast<raw*>(p.ll) + g, o);
        }
        return;
    }

    // level 2: x in the thread, y with lane ^ 16, z with lane ^ 32
    double s[NP], t[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        s[q] = lll[2 * q] + lll[2 * q + 1];
        t[q] = lll[2 * q + 1] - lll[2 * q];
        const double ps = __shfl_xor(s[q], 16), pt = __shfl_xor(t[q], 16);
        s[q] = m.yo ? s[q] - ps : s[q] + ps;
        t[q] = m.yo ? t[q] - pt : t[q] + pt;
        const double zs = __shfl_xor(s[q], 32), zt = __shfl_xor(t[q], 32);
        s[q] = (m.zo ? s[q] - zs : s[q] + zs) * kC3;     // code (L, yo, zo)
        t[q] = (m.zo ? t[q] - zt : t[q] + zt) * kC3;     // code (H, yo, zo)
    }
    const Level3 L2 = level_sizes(p, 2);
    const int y2 = m.ty >> 1, z2 = m.tz >> 1;
    const bool low = !m.yo && !m.zo;           // lanes holding LLL_2
    {
        const int64_t gz = (m.zo ? L2.D : 0) + (oz >> 2) + z2;
        const int64_t gy = (m.yo ? L2.H : 0) + (oy >> 2) + y2;
        raw* row = det + gz * p.det_p + gy * p.det_r + (ox >> 2) + NP * m.tx;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            st1_cached<S>(row + L2.W + q, (float)t[q]);
            if (!low) st1_cached<S>(row + q, (float)s[q]);
        }
    }
    if constexpr (LV == 2) {
        if (low) {
            const int64_t g = item * p.ll_b + ((oz >> 2) + z2) * p.ll_p + ((oy >> 2) + y2) * p.ll_r +
                              (ox >> 2) + NP * m.tx;
#pragma unroll
            for (int q = 0; q < NP; ++q) st_val<S, LLDF>(p.ll, g + q, s[q]);
        }
        return;
    }

    // level 3: LLL_2 of the tile (2 x 2 x X2) through LDS; X2 / 2 threads of
    // wavefront 0 each take one 2 x 2 x 2 block
    constexpr int X2 = R::X2;
    if (low) {
#pragma unroll
        for (int q = 0; q < NP; ++q) sm[(z2 * 2 + y2) * X2 + NP * m.tx + q] = s[q];
    }
    __syncthreads();
    if (threadIdx.x < X2 / 2) {
        const int k = threadIdx.x;
        double q[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) q[i] = sm[((i >> 2) * 2 + ((i >> 1) & 1)) * X2 + 2 * k + (i & 1)];
        bfly8<false>(q);
        const Level3 L3 = level_sizes(p, 3);
#pragma unroll
        for (int c = 1; c < 8; ++c) {
            const int64_t gz = ((c >> 2) ? L3.D : 0) + (oz >> 3);
            const int64_t gy = (((c >> 1) & 1) ? L3.H : 0) + (oy >> 3);
            const int64_t gx = ((c & 1) ? L3.W : 0) + (ox >> 3) + k;
            st1_cached<S>(det + gz * p.det_p + gy * p.det_r + gx, (float)(q[c] * kC3));
        }
        st_val<S, LLDF>(p.ll, item * p.ll_b + (oz >> 3) * p.ll_p + (oy >> 3) * p.ll_r + (ox >> 3) + k,
                        q[0] * kC3);
    }
}

template <class S, bool RDF, int LV, bool LLDF>
__device__ void inv3d_regs(const Pass3D& p, int64_t item, int64_t oz, int64_t oy, int64_t ox, double* sm) {
    using raw = typename S::raw;
    using R = Rx3<S, RDF>;
    constexpr int RX = R::RX, NB = R::NB, NP = R::NP, X2 = R::X2;
    const Map3 m = map3();
    const raw* det = reinterpret_cast<const raw*>(p.det) + item * p.det_b;
    double lll[NB];
    if constexpr (LV == 1) {
        const int64_t g = item * p.ll_b + ((oz >> 1) + m.tz) * p.ll_p + ((oy >> 1) + m.ty) * p.ll_r +
                          (ox >> 1) + NB * m.tx;
#pragma unroll
        for (int b = 0; b < NB; ++b) lll[b] = ld_val<S, LLDF>(p.ll, g + b);
    } else {
        const int y2 = m.ty >> 1, z2 = m.tz >> 1;
        const bool low = !m.yo && !m.zo;
        if constexpr (LV == 3) {
            if (threadIdx.x < X2 / 2) {
                const int k = threadIdx.x;
                const Level3 L3 = level_sizes(p, 3);
                double q[8];
                q[0] = ld_val<S, LLDF>(p.ll, item * p.ll_b + (oz >> 3) * p.ll_p + (oy >> 3) * p.ll_r +
                                                 (ox >> 3) + k);
#pragma unroll
                for (int c = 1; c < 8; ++c) {
                    const int64_t gz = ((c >> 2) ? L3.D : 0) + (oz >> 3);
                    const int64_t gy = (((c >> 1) & 1) ? L3.H : 0) + (oy >> 3);
                    const int64_t gx = ((c & 1) ? L3.W : 0) + (ox >> 3) + k;
                    q[c] = (double)ld1<S>(det + gz * p.det_p + gy * p.det_r + gx);
                }
                bfly8<true>(q);
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    sm[((i >> 2) * 2 + ((i >> 1) & 1)) * X2 + 2 * k + (i & 1)] = q[i] * kC3;
            }
            __syncthreads();
        }
        const Level3 L2 = level_sizes(p, 2);
        const int64_t gz = (m.zo ? L2.D : 0) + (oz >> 2) + z2;
        const int64_t gy = (m.yo ? L2.H : 0) + (oy >> 2) + y2;
        const raw* row = det + gz * p.det_p + gy * p.det_r + (ox >> 2) + NP * m.tx;
        const int64_t gl = item * p.ll_b + ((oz >> 2) + z2) * p.ll_p + ((oy >> 2) + y2) * p.ll_r +
                           (ox >> 2) + NP * m.tx;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            double t = (double)ld1<S>(row + L2.W + q);
            double s;
            if (!low) {
                s = (double)ld1<S>(row + q);
            } else if constexpr (LV == 3) {
                s = sm[(z2 * 2 + y2) * X2 + NP * m.tx + q];
            } else {
                s = ld_val<S, LLDF>(p.ll, gl + q);
            }
            // undo z (lane ^ 32), then y (lane ^ 16): even member a - d, odd a + d
            const double zs = __shfl_xor(s, 32), zt = __shfl_xor(t, 32);
            s = m.zo ? zs + s : s - zs;
            t = m.zo ? zt + t : t - zt;
            const double ys = __shfl_xor(s, 16), yt = __shfl_xor(t, 16);
            s = m.yo ? ys + s : s - ys;
            t = m.yo ? yt + t : t - yt;
            lll[2 * q] = (s - t) * kC3;
            lll[2 * q + 1] = (s + t) * kC3;
        }
    }

    const Level3 L1 = level_sizes(p, 1);
    float d1[8][NB];
#pragma unroll
    for (int c = 1; c < 8; ++c) {
        const int64_t gz = ((c >> 2) ? L1.D : 0) + (oz >> 1) + m.tz;
        const int64_t gy = (((c >> 1) & 1) ? L1.H : 0) + (oy >> 1) + m.ty;
        const int64_t gx = ((c & 1) ? L1.W : 0) + (ox >> 1) + NB * m.tx;
        ld_vec<S, NB>(det + gz * p.det_p + gy * p.det_r + gx, d1[c]);
    }
    // level 1: LLL_1 and the seven detail octants of the NB blocks.  Samples
    // rounded to 16 bits need no more than FP32 here (its error is 2^-16 of
    // their spacing); FP32 and scratch outputs stay in FP64.
    using TV = std::conditional_t<(S::kBytes == 2 && !RDF), float, double>;
    TV v[2][2][RX];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        TV q[8];
        q[0] = (TV)lll[b];
#pragma unroll
        for (int i = 1; i < 8; ++i) q[i] = (TV)d1[i][b];
        bfly8<true>(q);
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i >> 2][(i >> 1) & 1][2 * b + (i & 1)] = q[i] * (TV)kC3;
    }
    const int64_t db = item * p.dst_b + (oz + 2 * m.tz) * p.dst_p + (oy + 2 * m.ty) * p.dst_r + ox + RX * m.tx;
    if constexpr (RDF) {
        double* dst = reinterpret_cast<double*>(p.dst) + db;
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                for (int e = 0; e < RX; ++e) dst[dz * p.dst_p + dy * p.dst_r + e] = v[dz][dy][e];
    } else {
        raw* dst = reinterpret_cast<raw*>(p.dst) + db;
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy) {
                float f[RX];
#pragma unroll
                for (int e = 0; e < RX; ++e) f[e] = (float)v[dz][dy][e];
                st_vec<S, RX>(dst + dz * p.dst_p + dy * p.dst_r, f);
            }
    }
}

// ---------------------------------------------------------------------------
// Kernels.  Interior tiles (the register path) and the other tiles (the LDS
// path) are separate launches, so that each keeps its own register budget.
// Tiles run x-fastest; a grid-stride loop covers grids beyond the cap.
// RDF: the region (analysis source / synthesis destination) is FP64
// scratch; LDF: the pass's deepest LLL is FP64 scratch.
// ---------------------------------------------------------------------------
template <class S, bool RDF>
__device__ __forceinline__ void full_origin(const Pass3D& p, int64_t t, int64_t& item, int64_t& oz,
                                            int64_t& oy, int64_t& ox) {
    ox = (t % p.fx) * Rx3<S, RDF>::TX;
    t /= p.fx;
    oy = (t % p.fy) * kTY;
    t /= p.fy;
    oz = (t % p.fz) * kTZ;
    item = t / p.fz;
}

// Edge tile e of an item (generic tiles, 64 wide): the slab tz >= fz, then
// ty >= fy (tz < fz), then the columns from x = cx0 on (tz < fz, ty < fy),
// where the interior tiles (fx of them, possibly wider) end.
__device__ __forceinline__ void edge_origin(const Pass3D& p, int64_t e, int64_t& item, int64_t& oz,
                                            int64_t& oy, int64_t& ox) {
    const int64_t a = (p.ntz - p.fz) * p.nty * p.ntx;
    const int64_t b = p.fz * (p.nty - p.fy) * p.ntx;
    const int64_t c = p.fz * p.fy * p.ncx;
    const int64_t per = a + b + c;
    item = e / per;
    e -= item * per;
    int64_t tz, ty, tx;
    if (e < a) {
        tx = e % p.ntx;
        ty = (e / p.ntx) % p.nty;
        tz = p.fz + e / (p.ntx * p.nty);
    } else if (e < a + b) {
        e -= a;
        tx = e % p.ntx;
        ty = p.fy + (e / p.ntx) % (p.nty - p.fy);
        tz = e / (p.ntx * (p.nty - p.fy));
    } else {
        e -= a + b;
        oz = (e / (p.ncx * p.fy)) * kTZ;
        oy = ((e / p.ncx) % p.fy) * kTY;
        ox = p.cx0 + (e % p.ncx) * kTX;
        return;
    }
    oz = tz * kTZ;
    oy = ty * kTY;
    ox = tx * kTX;
}

// ONE: the grid covers every tile (one work-group each), so the loop runs
// once and breaks, which keeps fewer values live.
template <class S, bool RDF, int LV, bool LDF, bool ONE = false>
__global__ __launch_bounds__(kThreads3) void fwd3d_full_kernel(Pass3D p) {
    __shared__ double sm[4 * Rx3<S, RDF>::X2];
    for (int64_t t = blockIdx.x; t < p.nfull; t += gridDim.x) {
        int64_t item, oz, oy, ox;
        full_origin<S, RDF>(p, t, item, oz, oy, ox);
        fwd3d_regs<S, RDF, LV, LDF>(p, item, oz, oy, ox, sm);
        if (ONE) break;
        if (LV == 3) __syncthreads();
    }
}

template <class S, bool RDF, int LV, bool LDF, bool ONE = false>
__global__ __launch_bounds__(kThreads3) void inv3d_full_kernel(Pass3D p) {
    __shared__ double sm[4 * Rx3<S, RDF>::X2];
    for (int64_t t = blockIdx.x; t < p.nfull; t += gridDim.x) {
        int64_t item, oz, oy, ox;
        full_origin<S, RDF>(p, t, item, oz, oy, ox);
        inv3d_regs<S, RDF, LV, LDF>(p, item, oz, oy, ox, sm);
        if (ONE) break;
        if (LV == 3) __syncthreads();
    }
}

template <class S, bool RDF, bool LDF>
__global__ __launch_bounds__(kThreads3) void fwd3d_edge_kernel(Pass3D p) {
    __shared__ double sm[kLll1 + kLll2];
    for (int64_t t = blockIdx.x; t < p.nedge; t += gridDim.x) {
        int64_t item, oz, oy, ox;
        edge_origin(p, t, item, oz, oy, ox);
        fwd3d_lds<S, RDF, LDF>(p, item, oz, oy, ox, sm);
        __syncthreads();
    }
}

template <class S, bool RDF, bool LDF>
__global__ __launch_bounds__(kThreads3) void inv3d_edge_kernel(Pass3D p) {
    __shared__ double sm[kLll1 + kLll2];
    for (int64_t t = blockIdx.x; t < p.nedge; t += gridDim.x) {
        int64_t item, oz, oy, ox;
        edge_origin(p, t, item, oz, oy, ox);
        inv3d_lds<S, RDF, LDF>(p, item, oz, oy, ox, sm);
        __syncthreads();
    }
}

constexpr int64_t kGridCap3 = (int64_t)1 << 22;

inline unsigned grid3(int64_t n) { return (unsigned)(n < kGridCap3 ? n : kGridCap3); }

template <class S, bool RDF, bool LDF>
void launch3_full(const Pass3D& p, bool inverse, hipStream_t s) {
    const dim3 g(grid3(p.nfull)), b(kThreads3);
    // without the loop (measured on 4 x 256^3): BF16 synthesis 54.2 -> 51.0
    // us, FP32 analysis 107 -> 106 us (L3) and 133 -> 127 us (L8); the FP32
    // synthesis (95.5 -> 100 us) and the BF16 analysis (51.0 -> 51.8 us)
    // ran slower that way and keep the loop
    const bool one = p.nfull <= kGridCap3 && (inverse ? S::kBytes == 2 : S::kBytes == 4);
    if (one) {
        if (inverse) {
            if (p.levels == 3) hipLaunchKernelGGL((inv3d_full_kernel<S, RDF, 3, LDF, true>), g, b, 0, s, p);
            else if (p.levels == 2) hipLaunchKernelGGL((inv3d_full_kernel<S, RDF, 2, LDF, true>), g, b, 0, s, p);
            else hipLaunchKernelGGL((inv3d_full_kernel<S, RDF, 1, LDF, true>), g, b, 0, s, p);
        } else {
            if (p.levels == 3) hipLaunchKernelGGL((fwd3d_full_kernel<S, RDF, 3, LDF, true>), g, b, 0, s, p);
            else if (p.levels == 2) hipLaunchKernelGGL((fwd3d_full_kernel<S, RDF, 2, LDF, true>), g, b, 0, s, p);
            else hipLaunchKernelGGL((fwd3d_full_kernel<S, RDF, 1, LDF, true>), g, b, 0, s, p);
        }
        return;
    }
    if (inverse) {
        if (p.levels == 3) hipLaunchKernelGGL((inv3d_full_kernel<S, RDF, 3, LDF>), g, b, 0, s, p);
        else if (p.levels == 2) hipLaunchKernelGGL((inv3d_full_kernel<S, RDF, 2, LDF>), g, b, 0, s, p);
        else hipLaunchKernelGGL((inv3d_full_kernel<S, RDF, 1, LDF>), g, b, 0, s, p);
    } else {
        if (p.levels == 3) hipLaunchKernelGGL((fwd3d_full_kernel<S, RDF, 3, LDF>), g, b, 0, s, p);
        else if (p.levels == 2) hipLaunchKernelGGL((fwd3d_full_kernel<S, RDF, 2, LDF>), g, b, 0, s, p);
        else hipLaunchKernelGGL((fwd3d_full_kernel<S, RDF, 1, LDF>), g, b, 0, s, p);
    }
}

template <class S, bool RDF, bool LDF>
void launch3_edge(const Pass3D& p, bool inverse, hipStream_t s) {
    const dim3 g(grid3(p.nedge)), b(kThreads3);
    if (inverse) hipLaunchKernelGGL((inv3d_edge_kernel<S, RDF, LDF>), g, b, 0, s, p);
    else hipLaunchKernelGGL((fwd3d_edge_kernel<S, RDF, LDF>), g, b, 0, s, p);
}

template <class S>
hipError_t launch3_s(const Pass3D& p, bool inverse, bool rdf, bool ldf, hipStream_t s) {
    if (p.nfull > 0) {
        if (rdf) {
            if (ldf) launch3_full<S, true, true>(p, inverse, s);
            else launch3_full<S, true, false>(p, inverse, s);
        } else {
            if (ldf) launch3_full<S, false, true>(p, inverse, s);
            else launch3_full<S, false, false>(p, inverse, s);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (p.nedge > 0) {
        if (rdf) {
            if (ldf) launch3_edge<S, true, true>(p, inverse, s);
            else launch3_edge<S, true, false>(p, inverse, s);
        } else {
            if (ldf) launch3_edge<S, false, true>(p, inverse, s);
            else launch3_edge<S, false, false>(p, inverse, s);
        }
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tail of a deep transform: every level after the first pass, in one launch
// of one work-group per item.  After three levels a volume's LLL region is
// small (a 256^3 volume leaves 32^3), and chained passes over it cost a
// launch and a half-empty tile grid per three levels.  The work-group walks
// the region level by level over the level's 2 x 2 x 2 blocks (carry rule
// on each axis), keeps each level's LLL region in LDS (odd levels in A, even
// levels in B) and writes the detail octants to their packed positions.
// The region comes from (analysis) or goes to (synthesis) the first pass's
// FP64 scratch; the deepest LLL is the call's own output / input.
// ---------------------------------------------------------------------------
constexpr int kTailThreads = 1024;
constexpr int kTailA = 4096, kTailB = 512;     // LDS doubles: LLL after the tail's level 1 / 2

struct Tail3D {
    // the region after the first pass (FP64 scratch, dense per item)
    double* reg; int64_t reg_b;
    void* det; int64_t det_p, det_r, det_b;    // the call's packed buffer (storage type)
    int64_t d, h, w;                           // region
    int32_t levels;                            // levels of the tail
};

// Can the tail of a region of d x h x w run in one work-group per item?
inline bool tail_fits(int64_t d, int64_t h, int64_t w) {
    const int64_t a = ceil_shift_host(d, 1) * ceil_shift_host(h, 1) * ceil_shift_host(w, 1);
    const int64_t b = ceil_shift_host(d, 2) * ceil_shift_host(h, 2) * ceil_shift_host(w, 2);
    return a <= kTailA && b <= kTailB;
}

// Block grid of level j of the tail: the level-(j-1) region and its blocks.
struct TailLevel {
    int nz, ny, nx, bz_n, by_n, bx_n, nb;
    __device__ __forceinline__ TailLevel(const Tail3D& t, int j) {
        nz = (int)ceil_shift(t.d, j - 1);
        ny = (int)ceil_shift(t.h, j - 1);
        nx = (int)ceil_shift(t.w, j - 1);
        bz_n = (nz + 1) >> 1;
        by_n = (ny + 1) >> 1;
        bx_n = (nx + 1) >> 1;
        nb = bz_n * by_n * bx_n;
    }
};

constexpr int kTailSlots = kTailA / kTailThreads;   // blocks per thread at the tail's level 1

template <class S>
__global__ __launch_bounds__(kTailThreads) void fwd3d_tail_kernel(Tail3D t) {
    __shared__ double bufA[kTailA], bufB[kTailB];
    using raw = typename S::raw;
    const int64_t item = blockIdx.x;
    const double* reg = t.reg + item * t.reg_b;
    raw* det = reinterpret_cast<raw*>(t.det) + item * t.det_b;
    Pass3D p{};
    p.d = t.d;
    p.h = t.h;
    p.w = t.w;
    p.det_p = t.det_p;
    p.det_r = t.det_r;
    for (int j = 1; j <= t.levels; ++j) {
        const TailLevel G(t, j);
        const double* in = (j - 1) & 1 ? bufA : bufB;
        double* out = j & 1 ? bufA : bufB;
        const Level3 Lj = level_sizes(p, j);
        for (int s = threadIdx.x; s < G.nb; s += kTailThreads) {
            const int bx = s % G.bx_n, by = (s / G.bx_n) % G.by_n, bz = s / (G.bx_n * G.by_n);
            const bool fx = 2 * bx + 1 < G.nx, fy = 2 * by + 1 < G.ny, fz = 2 * bz + 1 < G.nz;
            double q[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int dx = c & 1, dy = (c >> 1) & 1, dz = c >> 2;
                q[c] = 0.0;
                if ((dx && !fx) || (dy && !fy) || (dz && !fz)) continue;
                const int64_t o = ((int64_t)(2 * bz + dz) * G.ny + 2 * by + dy) * G.nx + 2 * bx + dx;
                q[c] = j == 1 ? reg[o] : in[o];
            }
            block_fwd(q, fx, fy, fz);
#pragma unroll
            for (int code = 1; code < 8; ++code)
                if ((!(code & 1) || fx) && (!(code & 2) || fy) && (!(code & 4) || fz))
                    st1_cached<S>(det + octant_pos(p, Lj, j, code, 0, 0, 0, bz, by, bx), (float)q[code]);
            if (j == t.levels)
                st1_cached<S>(det + (int64_t)bz * t.det_p + (int64_t)by * t.det_r + bx, (float)q[0]);
            else
                out[(bz * G.by_n + by) * G.bx_n + bx] = q[0];
        }
        __syncthreads();
    }
}

// The detail coefficients of this thread's blocks of tail level j (zero
// where the carry rule leaves no partner).
template <class S>
__device__ __forceinline__ void tail_details(const Tail3D& t, const Pass3D& p, const typename S::raw* det, int j,
                                             float (&dv)[kTailSlots][7]) {
    const TailLevel G(t, j);
    const Level3 Lj = level_sizes(p, j);
#pragma unroll
    for (int k = 0; k < kTailSlots; ++k) {
        const int s = threadIdx.x + kTailThreads * k;
#pragma unroll
        for (int code = 1; code < 8; ++code) dv[k][code - 1] = 0.0f;
        if (s >= G.nb) continue;
        const int bx = s % G.bx_n, by = (s / G.bx_n) % G.by_n, bz = s / (G.bx_n * G.by_n);
        const bool fx = 2 * bx + 1 < G.nx, fy = 2 * by + 1 < G.ny, fz = 2 * bz + 1 < G.nz;
#pragma unroll
        for (int code = 1; code < 8; ++code)
            if ((!(code & 1) || fx) && (!(code & 2) || fy) && (!(code & 4) || fz))
                dv[k][code - 1] = ld1<S>(det + octant_pos(p, Lj, j, code, 0, 0, 0, bz, by, bx));
    }
}

template <class S>
__global__ __launch_bounds__(kTailThreads) void inv3d_tail_kernel(Tail3D t) {
    __shared__ double bufA[kTailA], bufB[kTailB];
    using raw = typename S::raw;
    const int64_t item = blockIdx.x;
    double* reg = t.reg + item * t.reg_b;
    const raw* det = reinterpret_cast<const raw*>(t.det) + item * t.det_b;
    Pass3D p{};
    p.d = t.d;
    p.h = t.h;
    p.w = t.w;
    p.det_p = t.det_p;
    p.det_r = t.det_r;
    // the details of level j - 1 are read while level j is undone, so each
    // level waits on LDS and not on a fresh round of HBM reads
    float cur[kTailSlots][7], nxt[kTailSlots][7];
    tail_details<S>(t, p, det, t.levels, cur);
    for (int j = t.levels; j >= 1; --j) {
        if (j > 1) tail_details<S>(t, p, det, j - 1, nxt);
        const TailLevel G(t, j);
        const double* in = j & 1 ? bufA : bufB;               // LLL of level j
        double* out = (j - 1) & 1 ? bufA : bufB;              // LLL of level j - 1
#pragma unroll
        for (int k = 0; k < kTailSlots; ++k) {
            const int s = threadIdx.x + kTailThreads * k;
            if (s >= G.nb) continue;
            const int bx = s % G.bx_n, by = (s / G.bx_n) % G.by_n, bz = s / (G.bx_n * G.by_n);
            const bool fx = 2 * bx + 1 < G.nx, fy = 2 * by + 1 < G.ny, fz = 2 * bz + 1 < G.nz;
            double q[8];
            q[0] = j == t.levels ? (double)ld1<S>(det + (int64_t)bz * t.det_p + (int64_t)by * t.det_r + bx)
                                 : in[(bz * G.by_n + by) * G.bx_n + bx];
#pragma unroll
            for (int code = 1; code < 8; ++code) q[code] = (double)cur[k][code - 1];
            block_inv(q, fx, fy, fz);
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int dx = c & 1, dy = (c >> 1) & 1, dz = c >> 2;
                if ((dx && !fx) || (dy && !fy) || (dz && !fz)) continue;
                const int64_t o = ((int64_t)(2 * bz + dz) * G.ny + 2 * by + dy) * G.nx + 2 * bx + dx;
                if (j == 1)
                    reg[o] = q[c];
                else
                    out[o] = q[c];
            }
        }
        __syncthreads();
        if (j > 1) {
#pragma unroll
            for (int k = 0; k < kTailSlots; ++k)
#pragma unroll
                for (int c = 0; c < 7; ++c) cur[k][c] = nxt[k][c];
        }
    }
}

hipError_t launch_tail3d(const Tail3D& t, int64_t batch, int dtype, bool inverse, hipStream_t s) {
    const dim3 g((unsigned)batch), b(kTailThreads);
    if (dtype == HAAR_F32) {
        if (inverse) hipLaunchKernelGGL(inv3d_tail_kernel<StF32>, g, b, 0, s, t);
        else hipLaunchKernelGGL(fwd3d_tail_kernel<StF32>, g, b, 0, s, t);
    } else if (dtype == HAAR_BF16) {
        if (inverse) hipLaunchKernelGGL(inv3d_tail_kernel<StBF16>, g, b, 0, s, t);
        else hipLaunchKernelGGL(fwd3d_tail_kernel<StBF16>, g, b, 0, s, t);
    } else {
        if (inverse) hipLaunchKernelGGL(inv3d_tail_kernel<StF16>, g, b, 0, s, t);
        else hipLaunchKernelGGL(fwd3d_tail_kernel<StF16>, g, b, 0, s, t);
    }
    return hipGetLastError();
}

struct Region3D {
    int64_t d, h, w;
    int levels;
};

}  // namespace

int run_3d(const void* in, void* out, int64_t D, int64_t H, int64_t W, int L, int64_t batch, int dtype,
           bool inverse, hipStream_t s) {
    std::vector<Region3D> ps;
    {
        int64_t d = D, h = H, w = W;
        for (int left = L; left > 0;) {
            const int lp = left < kMaxPassLevels3D ? left : kMaxPassLevels3D;
            ps.push_back({d, h, w, lp});
            d = ceil_shift_host(d, lp);
            h = ceil_shift_host(h, lp);
            w = ceil_shift_host(w, lp);
            left -= lp;
        }
    }
    // the levels after the first pass run as one tail launch (one
    // work-group per item) when the region left by the first pass is small
    // enough for one work-group and the items fit one grid
    const bool tail = ps.size() > 1 && tail_fits(ps[1].d, ps[1].h, ps[1].w) && batch <= ((int64_t)1 << 30);
    const Region3D rt = tail ? Region3D{ps[1].d, ps[1].h, ps[1].w, L - ps[0].levels} : Region3D{};
    if (tail) ps.resize(1);
    const int np = (int)ps.size();
    // FP64 scratch between passes: two ping-pong buffers sized for the
    // region after the first pass (one when the tail follows that pass)
    void* scratch = nullptr;
    int64_t half = 0;
    if (np > 1 || tail) {
        half = tail ? batch * rt.d * rt.h * rt.w : batch * ps[1].d * ps[1].h * ps[1].w;
        const int nbuf = tail ? 1 : 2;
        hipError_t e = hipMallocAsync(&scratch, (size_t)(nbuf * half * (int64_t)sizeof(double)), s);
        if (e != hipSuccess) return hip_error(e, "hipMallocAsync (3D pass scratch)");
    }
    auto buf = [&](int k) -> void* {
        return (char*)scratch + ((tail || (k & 1)) ? 0 : half) * (int64_t)sizeof(double);
    };
    auto run_tail = [&]() -> int {
        Tail3D t{};
        t.reg = reinterpret_cast<double*>(scratch);
        t.reg_b = rt.d * rt.h * rt.w;
        t.det = const_cast<void*>(inverse ? in : (const void*)out);
        t.det_p = H * W;
        t.det_r = W;
        t.det_b = D * H * W;
        t.d = rt.d;
        t.h = rt.h;
        t.w = rt.w;
        t.levels = rt.levels;
        hipError_t e = launch_tail3d(t, batch, dtype, inverse, s);
        return e == hipSuccess ? HAAR_OK : hip_error(e, inverse ? "inv3d tail launch" : "fwd3d tail launch");
    };

    int rc = HAAR_OK;
    if (tail && inverse) rc = run_tail();
    for (int step = 0; step < np && rc == HAAR_OK; ++step) {
        const int k = inverse ? np - 1 - step : step;
        const Region3D& r = ps[k];
        const bool rdf = k > 0, ldf = k < np - 1 || tail;
        Pass3D p{};
        p.d = r.d;
        p.h = r.h;
        p.w = r.w;
        p.batch = batch;
        p.levels = r.levels;
        p.det = const_cast<void*>(inverse ? in : (const void*)out);
        p.det_p = H * W;
        p.det_r = W;
        p.det_b = D * H * W;
        void* rptr = k == 0 ? (void*)(inverse ? out : in) : buf(k);
        const int64_t rp = k == 0 ? H * W : r.h * r.w, rr = k == 0 ? W : r.w;
        const int64_t rb = k == 0 ? D * H * W : r.d * r.h * r.w;
        const int64_t nd = ceil_shift_host(r.d, r.levels), nh = ceil_shift_host(r.h, r.levels);
        const int64_t nw = ceil_shift_host(r.w, r.levels);
        const bool ll_out = k == np - 1 && !tail;   // the pass's LLL is the call's deepest band
        p.ll = ll_out ? (void*)(inverse ? in : out) : buf(k + 1);
        p.ll_p = ll_out ? H * W : nh * nw;
        p.ll_r = ll_out ? W : nw;
        p.ll_b = ll_out ? D * H * W : nd * nh * nw;
        if (inverse) {
            p.dst = rptr; p.dst_p = rp; p.dst_r = rr; p.dst_b = rb;
        } else {
            p.src = rptr; p.src_p = rp; p.src_r = rr; p.src_b = rb;
        }
        p.ntz = ceil_shift_host(r.d, 3);
        p.nty = ceil_shift_host(r.h, 3);
        p.ntx = ceil_shift_host(r.w, 6);
        // interior tile width: 16 threads of 16 bytes of storage, or of 4
        // FP64 values when the region is scratch
        const int ftx = 16 * (rdf ? 4 : 16 / elem_bytes(dtype));
        p.fz = r.d / kTZ;
        p.fy = r.h / kTY;
        p.fx = r.w / ftx;
        p.cx0 = p.fx * ftx;
        p.ncx = (r.w - p.cx0 + kTX - 1) / kTX;
        p.nfull = p.fz * p.fy * p.fx * batch;
        p.nedge = ((p.ntz - p.fz) * p.nty * p.ntx + p.fz * (p.nty - p.fy) * p.ntx + p.fz * p.fy * p.ncx) * batch;
        hipError_t e;
        if (dtype == HAAR_F32) e = launch3_s<StF32>(p, inverse, rdf, ldf, s);
        else if (dtype == HAAR_BF16) e = launch3_s<StBF16>(p, inverse, rdf, ldf, s);
        else e = launch3_s<StF16>(p, inverse, rdf, ldf, s);
        if (e != hipSuccess) rc = hip_error(e, inverse ? "inv3d launch" : "fwd3d launch");
    }
    if (tail && !inverse && rc == HAAR_OK) rc = run_tail();
    if (scratch) {
        hipError_t e = hipFreeAsync(scratch, s);
        if (e != hipSuccess && rc == HAAR_OK) rc = hip_error(e, "hipFreeAsync");
    }
    return rc;
}

}  // namespace haar
