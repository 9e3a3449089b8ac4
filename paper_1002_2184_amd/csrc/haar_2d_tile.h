// Fused separable 2D Haar analysis / synthesis kernels for gfx950.
//
// One work-group owns one TH x TW tile of the region (TH, TW multiples of
// 32 = 2^5, the largest dependency block of one pass), so a tile needs no
// halo and crosses HBM once: read once, every band written once.
//
// Per thread: an RY x RX register block (16 bytes per row: 4 x f32 or
// 8 x bf16/f16).  Levels 1 and 2 run in registers on 2x2 blocks
// (Eq. (11)-(12) along the width, then along the height, fused into one
// butterfly per 2x2 block with the exact factor 1/2 = b00^2).  The deeper
// levels of the analysis run in wavefront shuffles and in LDS on the tile's
// LL2 or LL3 region; the synthesis derives each thread's LL2 values from
// their ancestor path, with no LDS.  The approximation path of the analysis
// carries compensated FP32 pairs.
//
// Full tiles of element-aligned layouts take the vector path (FULL = true).
// Edge tiles and unaligned layouts take the same code with per-element
// validity (FULL = false), where the odd-size carry rule applies: at an odd
// row/column count the last row/column passes unscaled into the
// approximation.
#pragma once

#include "haar_device.h"
#include "haar_kernels.h"

namespace haar {

// ---------------------------------------------------------------------------
// 2x2 butterflies
// ---------------------------------------------------------------------------
// EX (exact): the approximation path carries a compensated pair (hi + lo),
// rounded once when stored; used whenever the detail bands or the deepest LL
// are stored in FP32.  With 16-bit outputs (EX = false) plain FP32 sums are
// far more accurate than the output format (2^-24 against 2^-9 relative per
// rounding), so the pair is not formed (lo stays zero) and the analysis does
// about a quarter of the vector work less.

// Analysis of a full 2x2 block of exact floats (x00 x01 / x10 x11).
template <bool EX = true>
__device__ __forceinline__ void ana_full_f(float x00, float x01, float x10, float x11, df& ll,
                                           float& hl, float& lh, float& hh) {
    if constexpr (EX)
        ll = df_scale(df_sum4f(x00, x01, x10, x11), 0.5f);
    else
        ll = df{0.5f * ((x00 + x01) + (x10 + x11)), 0.0f};
    const float dr0 = x01 - x00, dr1 = x11 - x10;   // high along width, rows 0/1
    hl = 0.5f * (dr0 + dr1);
    hh = 0.5f * (dr1 - dr0);
    lh = 0.5f * ((x10 - x00) + (x11 - x01));
}

// Analysis of a full 2x2 block of pairs.
template <bool EX = true>
__device__ __forceinline__ void ana_full_df(df x00, df x01, df x10, df x11, df& ll, float& hl,
                                            float& lh, float& hh) {
    if constexpr (EX) {
        ll = df_scale(df_sum4(x00, x01, x10, x11), 0.5f);
        const float dr0 = df_diff(x01, x00), dr1 = df_diff(x11, x10);
        hl = 0.5f * (dr0 + dr1);
        hh = 0.5f * (dr1 - dr0);
        lh = 0.5f * (df_diff(x10, x00) + df_diff(x11, x01));
    } else {
        ana_full_f<false>(x00.hi, x01.hi, x10.hi, x11.hi, ll, hl, lh, hh);
    }
}

// Analysis with the carry rule.  c1: column 2k+1 exists; r1: row 2i+1 exists.
template <bool EX = true>
__device__ __forceinline__ void ana_edge_df(df x00, df x01, df x10, df x11, bool r1, bool c1,
                                            df& ll, float& hl, float& lh, float& hh) {
    if (r1 && c1) {
        ana_full_df<EX>(x00, x01, x10, x11, ll, hl, lh, hh);
    } else if (c1) {            // single row: row pass only, column carried
        if constexpr (EX) {
            ll = df_rs2(df_add(x00, x01));
            hl = df_round(df_rs2(df_from(df_diff(x01, x00))));
        } else {
            ll = df{(x00.hi + x01.hi) * kRs2Hi, 0.0f};
            hl = (x01.hi - x00.hi) * kRs2Hi;
        }
        lh = hh = 0.0f;
    } else if (r1) {            // single column: column pass only, row carried
        if constexpr (EX) {
            ll = df_rs2(df_add(x00, x10));
            lh = df_round(df_rs2(df_from(df_diff(x10, x00))));
        } else {
            ll = df{(x00.hi + x10.hi) * kRs2Hi, 0.0f};
            lh = (x10.hi - x00.hi) * kRs2Hi;
        }
        hl = hh = 0.0f;
    } else {
        ll = x00;
        hl = lh = hh = 0.0f;
    }
}

// The approximation rounded to one float (the pair's sum, or hi alone when
// the pair is not formed).
template <bool EX>
__device__ __forceinline__ float acc_round(df a) {
    if constexpr (EX)
        return df_round(a);
    else
        return a.hi;
}

// Synthesis of one 2x2 block (inverse of the analysis), with the carry rule.
__device__ __forceinline__ void syn_edge(float ll, float hl, float lh, float hh, bool r1, bool c1,
                                         float& x00, float& x01, float& x10, float& x11) {
    if (r1 && c1) {
        const float p = ll - lh, q = ll + lh, r = hl - hh, u = hl + hh;
        x00 = 0.5f * (p - r);
        x01 = 0.5f * (p + r);
        x10 = 0.5f * (q - u);
        x11 = 0.5f * (q + u);
    } else if (c1) {
        x00 = (ll - hl) * kRs2Hi;
        x01 = (ll + hl) * kRs2Hi;
        x10 = x11 = 0.0f;
    } else if (r1) {
        x00 = (ll - lh) * kRs2Hi;
        x10 = (ll + lh) * kRs2Hi;
        x01 = x11 = 0.0f;
    } else {
        x00 = ll;
        x01 = x10 = x11 = 0.0f;
    }
}

// The child (dy, dx) of one synthesis block, with the carry rule: the same
// arithmetic as syn_edge for that output.
__device__ __forceinline__ float syn_child(float ll, float hl, float lh, float hh, bool r1, bool c1,
                                           int dy, int dx) {
    if (r1 && c1) {
        const float base = dy ? ll + lh : ll - lh, tt = dy ? hl + hh : hl - hh;
        return 0.5f * (dx ? base + tt : base - tt);
    }
    if (c1) return (dx ? ll + hl : ll - hl) * kRs2Hi;
    if (r1) return (dy ? ll + lh : ll - lh) * kRs2Hi;
    return ll;
}

// ---------------------------------------------------------------------------
// Analysis tile
// ---------------------------------------------------------------------------
// SX: storage of the region (input of the analysis, output of the synthesis),
// SD: storage of the detail bands, SL: storage of the pass's deepest LL.
// They differ only when a deep transform keeps an intermediate approximation
// in FP32 scratch between passes.
template <class SX, int RY, int RX, int GY, int GX>
struct Geo2D {
    static constexpr int NT = GY * GX, TH = GY * RY, TW = GX * RX;
    static constexpr int B1Y = RY / 2, B1X = RX / 2, B2Y = RY / 4, B2X = RX / 4;
    static constexpr int AN = (TH / 4) * (TW / 4);   // LDS buffer A: LL2 region
    static constexpr int BN = (TH / 8) * (TW / 8);   // LDS buffer B: LL3 region
    static constexpr int SMEM = 2 * AN + 2 * BN;     // floats (hi + lo each)
    static_assert((RY == 4 || RY == 8) && RX * SX::kBytes == 16, "register block is 4 or 8 rows x 16 bytes");
    static_assert(TH % 32 == 0 && TW % 32 == 0, "tile must hold whole 32x32 blocks");
};

// Register block of one analysis tile: the RY x RX input samples of a thread.
template <int RY, int RX>
struct FwdIn {
    float v[RY][RX];
};

// Thread -> register block (row group rg, column group cg) of an analysis
// tile.  MAP 0: row-major over the GY x GX groups (a wavefront spans 64
// column groups, or two rows of 32).  MAP 1 (GY = 8): every wavefront owns an
// 8 x 8 patch of groups, i.e. whole 32-row dependency blocks, so that all
// levels of a full tile stay inside the wavefront.
template <int GY, int GX, int MAP>
__device__ __forceinline__ void thread_rc(int t, int& rg, int& cg) {
    if constexpr (MAP == 0) {
        rg = t / GX;
        cg = t % GX;
    } else if constexpr (MAP == 2) {
        // two-row wavefronts: wavefront w holds row groups 2 (w / 2) and
        // 2 (w / 2) + 1 (lanes 0-31 and 32-63) of column groups
        // 32 (w % 2) .. + 31, so each 2x2 block of LL2 lies in one wavefront
        // while every load and level-1/2 store still covers whole lines
        static_assert(GY == 8 && GX == 64, "two-row wavefronts are defined for 8 x 64 groups");
        const int lane = t & 63, w = t >> 6;
        rg = 2 * (w >> 1) + (lane >> 5);
        cg = 32 * (w & 1) + (lane & 31);
    } else {
        static_assert(GY == 8 && GX % 8 == 0, "wavefront-local tiles are 8 x 8k groups");
        const int lane = t & 63;
        rg = lane >> 3;
        cg = (t >> 6) * 8 + (lane & 7);
    }
}

template <bool EX = true>
__device__ __forceinline__ df shfl_xor_df(df a, int m) {
    if constexpr (EX)
        return df{__shfl_xor(a.hi, m), __shfl_xor(a.lo, m)};
    else
        return df{__shfl_xor(a.hi, m), 0.0f};
}


// NTL: nontemporal vector loads (launches whose tiles own whole cache
// lines, p.ntl; a separate kernel, since a run-time choice between two loads
// that differ only in that hint gets merged into the ordinary one).
template <class SX, int RY, int RX, int GY, int GX, bool FULL, int MAP = 0, bool NTL = false>
__device__ __forceinline__ void fwd2d_load(const Pass2D& p, int64_t item, int64_t ty, int64_t tx,
                                           FwdIn<RY, RX>& in) {
    using G = Geo2D<SX, RY, RX, GY, GX>;
    constexpr int TH = G::TH, TW = G::TW;
    const int t = threadIdx.x;
    int rg, cg;
    thread_rc<GY, GX, MAP>(t, rg, cg);
    const int64_t r0 = ty * TH, c0 = tx * TW;
    const int th = FULL ? TH : (p.h - r0 < TH ? (int)(p.h - r0) : TH);
    const int tw = FULL ? TW : (p.w - c0 < TW ? (int)(p.w - c0) : TW);
    const int lr0 = rg * RY, lc0 = cg * RX;
    const typename SX::raw* src =
        reinterpret_cast<const typename SX::raw*>(p.src) + item * p.src_bstride + r0 * p.src_pitch + c0;
    if (FULL || (lr0 + RY <= th && lc0 + RX <= tw)) {   // whole register block inside
#pragma unroll
        for (int r = 0; r < RY; ++r)
            ld_vec<SX, RX, NTL>(src + (int64_t)(lr0 + r) * p.src_pitch + lc0, in.v[r]);
    } else {
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int c = 0; c < RX; ++c)
                in.v[r][c] = (lr0 + r < th && lc0 + c < tw)
                                 ? ld1<SX>(src + (int64_t)(lr0 + r) * p.src_pitch + lc0 + c)
                                 : 0.0f;
    }
}

template <class SX, class SD, class SL, int RY, int RX, int GY, int GX, bool FULL, int MAP = 0>
__device__ __forceinline__ void fwd2d_body(const Pass2D& p, int64_t item, int64_t ty, int64_t tx,
                                           const FwdIn<RY, RX>& in, float* sm) {
    using G = Geo2D<SX, RY, RX, GY, GX>;
    constexpr int TH = G::TH, TW = G::TW, NT = G::NT;
    constexpr int B1Y = G::B1Y, B1X = G::B1X, B2Y = G::B2Y, B2X = G::B2X;

    const int t = threadIdx.x;
    int rg, cg;
    thread_rc<GY, GX, MAP>(t, rg, cg);
    const int64_t r0 = ty * TH, c0 = tx * TW;
    const int L = p.levels;
    const int th = FULL ? TH : (p.h - r0 < TH ? (int)(p.h - r0) : TH);
    const int tw = FULL ? TW : (p.w - c0 < TW ? (int)(p.w - c0) : TW);
    const int lr0 = rg * RY, lc0 = cg * RX;            // local origin of this thread's block
    // compensated approximation path unless every output of the pass is 16-bit
    constexpr bool EX = SD::kBytes == 4 || SL::kBytes == 4;
    // the whole register block lies inside the region: every 2x2 block of
    // levels 1 and 2 is complete and its bands are written as vectors
    const bool inb = FULL || (lr0 + RY <= th && lc0 + RX <= tw);

    typename SD::raw* det = reinterpret_cast<typename SD::raw*>(p.det) + item * p.det_bstride;
    typename SL::raw* llp = reinterpret_cast<typename SL::raw*>(p.ll) + item * p.ll_bstride;
    const int64_t dp = p.det_pitch, lp = p.ll_pitch;
    const auto& v = in.v;

    // ---- level 1 (registers)
    df a1[B1Y][B1X];
    {
        float hl[B1Y][B1X], lh[B1Y][B1X], hh[B1Y][B1X];
#pragma unroll
        for (int i = 0; i < B1Y; ++i)
#pragma unroll
            for (int k = 0; k < B1X; ++k) {
                if constexpr (FULL) {
                    ana_full_f<EX>(v[2 * i][2 * k], v[2 * i][2 * k + 1], v[2 * i + 1][2 * k],
                               v[2 * i + 1][2 * k + 1], a1[i][k], hl[i][k], lh[i][k], hh[i][k]);
                } else {
                    const bool r1 = lr0 + 2 * i + 1 < th, c1 = lc0 + 2 * k + 1 < tw;
                    ana_edge_df<EX>(df_from(v[2 * i][2 * k]), df_from(v[2 * i][2 * k + 1]),
                                df_from(v[2 * i + 1][2 * k]), df_from(v[2 * i + 1][2 * k + 1]), r1,
                                c1, a1[i][k], hl[i][k], lh[i][k], hh[i][k]);
                }
            }
        const int64_t hs = ceil_shift(p.h, 1), ws = ceil_shift(p.w, 1);
        const int64_t R = (r0 >> 1) + (lr0 >> 1), C = (c0 >> 1) + (lc0 >> 1);
        if (inb) {
#pragma unroll
            for (int i = 0; i < B1Y; ++i) {
                st_vec<SD, B1X>(det + (R + i) * dp + ws + C, hl[i]);
                st_vec<SD, B1X>(det + (hs + R + i) * dp + C, lh[i]);
                st_vec<SD, B1X>(det + (hs + R + i) * dp + ws + C, hh[i]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < B1Y; ++i)
#pragma unroll
                for (int k = 0; k < B1X; ++k) {
                    const int lr = lr0 + 2 * i, lc = lc0 + 2 * k;
                    if (lr < th && lc < tw) {
                        const bool r1 = lr + 1 < th, c1 = lc + 1 < tw;
                        if (c1) st1<SD>(det + (R + i) * dp + ws + C + k, hl[i][k]);
                        if (r1) st1<SD>(det + (hs + R + i) * dp + C + k, lh[i][k]);
                        if (r1 && c1) st1<SD>(det + (hs + R + i) * dp + ws + C + k, hh[i][k]);
                    }
                }
        }
        if (L == 1) {
#pragma unroll
            for (int i = 0; i < B1Y; ++i) {
                if (inb) {
                    float o[B1X];
#pragma unroll
                    for (int k = 0; k < B1X; ++k) o[k] = acc_round<EX>(a1[i][k]);
                    st_vec<SL, B1X>(llp + (R + i) * lp + C, o);
                } else {
#pragma unroll
                    for (int k = 0; k < B1X; ++k)
                        if (lr0 + 2 * i < th && lc0 + 2 * k < tw)
                            st1<SL>(llp + (R + i) * lp + C + k, acc_round<EX>(a1[i][k]));
                }
            }
            return;
        }
    }

    // ---- level 2 (registers)
    df a2[B2Y][B2X];
    {
        float hl[B2Y][B2X], lh[B2Y][B2X], hh[B2Y][B2X];
        const int th1 = (th + 1) >> 1, tw1 = (tw + 1) >> 1;
        const int l1r = lr0 >> 1, l1c = lc0 >> 1;       // local level-1 origin
#pragma unroll
        for (int i = 0; i < B2Y; ++i)
#pragma unroll
            for (int k = 0; k < B2X; ++k) {
                if constexpr (FULL) {
                    ana_full_df<EX>(a1[2 * i][2 * k], a1[2 * i][2 * k + 1], a1[2 * i + 1][2 * k],
                                a1[2 * i + 1][2 * k + 1], a2[i][k], hl[i][k], lh[i][k], hh[i][k]);
                } else {
                    const bool r1 = l1r + 2 * i + 1 < th1, c1 = l1c + 2 * k + 1 < tw1;
                    ana_edge_df<EX>(a1[2 * i][2 * k], a1[2 * i][2 * k + 1], a1[2 * i + 1][2 * k],
                                a1[2 * i + 1][2 * k + 1], r1, c1, a2[i][k], hl[i][k], lh[i][k],
                                hh[i][k]);
                }
            }
        const int64_t hs = ceil_shift(p.h, 2), ws = ceil_shift(p.w, 2);
        const int64_t R = (r0 >> 2) + (lr0 >> 2), C = (c0 >> 2) + (lc0 >> 2);
        if (inb) {
#pragma unroll
            for (int i = 0; i < B2Y; ++i) {
                st_vec<SD, B2X>(det + (R + i) * dp + ws + C, hl[i]);
                st_vec<SD, B2X>(det + (hs + R + i) * dp + C, lh[i]);
                st_vec<SD, B2X>(det + (hs + R + i) * dp + ws + C, hh[i]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < B2Y; ++i)
#pragma unroll
                for (int k = 0; k < B2X; ++k) {
                    const int lr = l1r + 2 * i, lc = l1c + 2 * k;
                    if (lr < th1 && lc < tw1) {
                        const bool r1 = lr + 1 < th1, c1 = lc + 1 < tw1;
                        if (c1) st1<SD>(det + (R + i) * dp + ws + C + k, hl[i][k]);
                        if (r1) st1<SD>(det + (hs + R + i) * dp + C + k, lh[i][k]);
                        if (r1 && c1) st1<SD>(det + (hs + R + i) * dp + ws + C + k, hh[i][k]);
                    }
                }
        }
        if (L == 2) {
#pragma unroll
            for (int i = 0; i < B2Y; ++i) {
                if (inb) {
                    float o[B2X];
#pragma unroll
                    for (int k = 0; k < B2X; ++k) o[k] = acc_round<EX>(a2[i][k]);
                    st_vec<SL, B2X>(llp + (R + i) * lp + C, o);
                } else {
#pragma unroll
                    for (int k = 0; k < B2X; ++k)
                        if (l1r + 2 * i < th1 && l1c + 2 * k < tw1)
                            st1<SL>(llp + (R + i) * lp + C + k, acc_round<EX>(a2[i][k]));
                }
            }
            return;
        }
    }

    if constexpr (FULL && MAP == 1) {
        // Levels 3..L inside the wavefront (a 32 x 8*RX patch of the tile):
        // the 2x2 partners of a level sit at fixed lane distances, so every
        // level is one round of xor-shuffles; no LDS, no barrier.  Shuffles run
        // on all lanes (uniform control flow); the lanes holding a valid
        // coefficient of the level store it.
        const int lane = t & 63, w = t >> 6;
        const int rgl = lane >> 3, cgl = lane & 7;
        constexpr int CS3 = B2X == 1 ? 2 : 1;          // lane distance of adjacent level-3 columns
        df x00, x01, x10, x11;
        if constexpr (B2X == 1) {
            x00 = a2[0][0];
            x01 = shfl_xor_df<EX>(a2[0][0], 1);
            x10 = shfl_xor_df<EX>(a2[0][0], 8);
            x11 = shfl_xor_df<EX>(a2[0][0], 9);
        } else {
            x00 = a2[0][0];
            x01 = a2[0][1];
            x10 = shfl_xor_df<EX>(a2[0][0], 8);
            x11 = shfl_xor_df<EX>(a2[0][1], 8);
        }
        int i = rgl >> 1, k = B2X == 1 ? (cgl >> 1) : cgl;   // level-3 position in the patch
        bool active = (rgl & 1) == 0 && (B2X == 2 || (cgl & 1) == 0);
        const int64_t wc0 = c0 + (int64_t)w * 8 * RX;         // first column of the patch
        df ll;
        float hl, lh, hh;
#pragma unroll
        for (int lev = 3; lev <= kMaxPassLevels2D; ++lev) {
            if (lev > 3) {
                const int cs = CS3 << (lev - 4), rs = 16 << (lev - 4);
                x00 = ll;
                x01 = shfl_xor_df<EX>(ll, cs);
                x10 = shfl_xor_df<EX>(ll, rs);
                x11 = shfl_xor_df<EX>(ll, cs | rs);
                active = active && (i & 1) == 0 && (k & 1) == 0;
                i >>= 1;
                k >>= 1;
            }
            ana_full_df<EX>(x00, x01, x10, x11, ll, hl, lh, hh);
            if (active) {
                const int64_t hs = ceil_shift(p.h, lev), ws = ceil_shift(p.w, lev);
                const int64_t R = (r0 >> lev) + i, C = (wc0 >> lev) + k;
                st1<SD>(det + R * dp + ws + C, hl);
                st1<SD>(det + (hs + R) * dp + C, lh);
                st1<SD>(det + (hs + R) * dp + ws + C, hh);
                if (lev == L) st1<SL>(llp + R * lp + C, acc_round<EX>(ll));
            }
            if (lev == L) return;
        }
        return;
    }

    // ---- levels 3..L.  Buffer A holds LL2 (pitch TW/4), buffer B LL3 (pitch TW/8).
    float* Ahi = sm;
    float* Alo = sm + G::AN;
    float* Bhi = sm + 2 * G::AN;
    float* Blo = Bhi + G::BN;
    int rh = (th + 3) >> 2, rw = (tw + 3) >> 2;   // local region size at level 2
    int first = 3;                                // first level of the single-wave phase
    if constexpr (FULL && RY == 8 && MAP == 0) {
        // Level 3 without LDS: a thread holds LL2 rows 2 rg and 2 rg + 1 of
        // B2X columns.  With B2X = 2 (16-bit data) the 2x2 block of LL2 is the
        // thread's own; with B2X = 1 (FP32) the partner column is in lane ^ 1
        // (column groups are lane-contiguous), so even lanes hold the block.
        const int lane = t & 63;
        df x00, x01, x10, x11;
        bool active;
        int k3;                                   // level-3 column in the tile
        if constexpr (B2X == 1) {
            x00 = a2[0][0];
            x10 = a2[1][0];
            x01 = shfl_xor_df<EX>(a2[0][0], 1);
            x11 = shfl_xor_df<EX>(a2[1][0], 1);
            active = (lane & 1) == 0;
            k3 = cg >> 1;
        } else {
            static_assert(B2X == 2, "16-byte rows hold 1 or 2 LL2 columns");
            x00 = a2[0][0];
            x01 = a2[0][1];
            x10 = a2[1][0];
            x11 = a2[1][1];
            active = true;
            k3 = cg;
        }
        if (active) {
            df ll;
            float hl, lh, hh;
            ana_full_df<EX>(x00, x01, x10, x11, ll, hl, lh, hh);
            const int64_t hs = ceil_shift(p.h, 3), ws = ceil_shift(p.w, 3);
            const int64_t R = (r0 >> 3) + rg, C = (c0 >> 3) + k3;
            st1<SD>(det + R * dp + ws + C, hl);
            st1<SD>(det + (hs + R) * dp + C, lh);
            st1<SD>(det + (hs + R) * dp + ws + C, hh);
            if (L == 3) {
                st1<SL>(llp + R * lp + C, acc_round<EX>(ll));
            } else {
                Bhi[rg * (TW / 8) + k3] = ll.hi;
                if constexpr (EX) Blo[rg * (TW / 8) + k3] = ll.lo;
            }
        }
        if (L == 3) return;
        rh = TH / 8;
        rw = TW / 8;
        first = 4;
    } else if constexpr (FULL && RY == 4 && ((GX == 32 && MAP == 0) || MAP == 2)) {
        // Level 3 inside each wavefront: a wave holds LL2 rows 2q (lanes
        // 0-31) and 2q+1 (lanes 32-63) of 32 column groups (q = w with 32
        // column groups, w / 2 with the two-row map), so every 2x2 block of
        // LL2 lies in one wave: xor-shuffles fetch the partners.
        const int lane = t & 63, w = MAP == 2 ? (t >> 7) : (t >> 6);
        const int cb3 = MAP == 2 ? ((t >> 6) & 1) * 16 * B2X : 0;   // first LL3 column of the wave
        df x00, x01, x10, x11;
        if constexpr (B2X == 1) {
            const df a = a2[0][0];
            x00 = a;
            x01 = shfl_xor_df<EX>(a, 1);
            x10 = shfl_xor_df<EX>(a, 32);
            x11 = shfl_xor_df<EX>(a, 33);
        } else {
            x00 = a2[0][0];
            x01 = a2[0][1];
            x10 = shfl_xor_df<EX>(a2[0][0], 32);
            x11 = shfl_xor_df<EX>(a2[0][1], 32);
        }
        const bool active = B2X == 1 ? (lane & 33) == 0 : lane < 32;
        if (active) {
            const int k = B2X == 1 ? (lane >> 1) : lane;     // level-3 column in the tile
            df ll;
            float hl, lh, hh;
            ana_full_df<EX>(x00, x01, x10, x11, ll, hl, lh, hh);
            const int64_t hs = ceil_shift(p.h, 3), ws = ceil_shift(p.w, 3);
            const int64_t R = (r0 >> 3) + w, C = (c0 >> 3) + cb3 + k;
            if constexpr (MAP == 2) {
                // half lines (the other half comes from the neighbouring
                // wavefront of the same work-group): merged in L2
                st1_cached<SD>(det + R * dp + ws + C, hl);
                st1_cached<SD>(det + (hs + R) * dp + C, lh);
                st1_cached<SD>(det + (hs + R) * dp + ws + C, hh);
            } else {
                st1<SD>(det + R * dp + ws + C, hl);
                st1<SD>(det + (hs + R) * dp + C, lh);
                st1<SD>(det + (hs + R) * dp + ws + C, hh);
            }
            if (L == 3) {
                st1<SL>(llp + R * lp + C, acc_round<EX>(ll));
            } else {
                Bhi[w * (TW / 8) + cb3 + k] = ll.hi;
                if constexpr (EX) Blo[w * (TW / 8) + cb3 + k] = ll.lo;
            }
        }
        if (L == 3) return;
        rh = TH / 8;
        rw = TW / 8;
        first = 4;
    } else {
#pragma unroll
        for (int i = 0; i < B2Y; ++i)
#pragma unroll
            for (int k = 0; k < B2X; ++k) {
                const int idx = ((lr0 >> 2) + i) * (TW / 4) + (lc0 >> 2) + k;
                Ahi[idx] = a2[i][k].hi;
                if constexpr (EX) Alo[idx] = a2[i][k].lo;
            }
    }
    __syncthreads();

    // The remaining levels are small (at most (TH/8) x (TW/8) blocks): the
    // first wavefront does them alone, so the other wavefronts of the
    // work-group can retire.
    if (t >= 64) return;
    constexpr int BH4 = TH / 16, BW4 = TW / 16;      // level-4 blocks of a full tile
    if constexpr (FULL && BH4 * BW4 <= 64 && (BW4 & (BW4 - 1)) == 0) {
        if (first == 4) {
            // Full tile with LL3 (TH/8 x TW/8, pitch TW/8) in LDS: lane
            // i * BW4 + k takes level-4 block (i, k) straight from LDS; level
            // 5 pairs lanes by xor shuffles (column partner lane ^ 1, row
            // partner lane ^ BW4), with no second LDS round trip.  Lanes past
            // the blocks read a valid block again and store nothing.
            constexpr int P3 = TW / 8;
            const int lane = t;
            const int bl = lane < BH4 * BW4 ? lane : lane % (BH4 * BW4);
            const int i = bl / BW4, k = bl % BW4;
            const int i0 = (2 * i) * P3 + 2 * k;
            auto at = [&](int q) { return df{Bhi[q], EX ? Blo[q] : 0.0f}; };
            df ll;
            float hl, lh, hh;
            ana_full_df<EX>(at(i0), at(i0 + 1), at(i0 + P3), at(i0 + P3 + 1), ll, hl, lh, hh);
            const bool own = lane < BH4 * BW4;
            {
                const int64_t hs = ceil_shift(p.h, 4), ws = ceil_shift(p.w, 4);
                const int64_t R = (r0 >> 4) + i, C = (c0 >> 4) + k;
                if (own) {
                    st1_cached<SD>(det + R * dp + ws + C, hl);
                    st1_cached<SD>(det + (hs + R) * dp + C, lh);
                    st1_cached<SD>(det + (hs + R) * dp + ws + C, hh);
                    if (L == 4) st1_cached<SL>(llp + R * lp + C, acc_round<EX>(ll));
                }
            }
            if (L == 4) return;
            static_assert(BH4 % 2 == 0 && BW4 % 2 == 0, "level-5 blocks of a full tile");
            const df x01 = shfl_xor_df<EX>(ll, 1), x10 = shfl_xor_df<EX>(ll, BW4),
                     x11 = shfl_xor_df<EX>(ll, BW4 + 1);
            df l5;
            ana_full_df<EX>(ll, x01, x10, x11, l5, hl, lh, hh);
            if (own && (i & 1) == 0 && (k & 1) == 0) {
                const int64_t hs = ceil_shift(p.h, 5), ws = ceil_shift(p.w, 5);
                const int64_t R = (r0 >> 5) + (i >> 1), C = (c0 >> 5) + (k >> 1);
                st1_cached<SD>(det + R * dp + ws + C, hl);
                st1_cached<SD>(det + (hs + R) * dp + C, lh);
                st1_cached<SD>(det + (hs + R) * dp + ws + C, hh);
                st1_cached<SL>(llp + R * lp + C, acc_round<EX>(l5));
            }
            return;
        }
    }
    for (int lev = first; lev <= L; ++lev) {
        const bool odd = lev & 1;
        const float* ihi = odd ? Ahi : Bhi;
        const float* ilo = odd ? Alo : Blo;
        float* ohi = odd ? Bhi : Ahi;
        float* olo = odd ? Blo : Alo;
        const int pin = TW >> (lev - 1), pout = TW >> lev;
        const int bh = (rh + 1) >> 1, bw = (rw + 1) >> 1;
        const int64_t hs = ceil_shift(p.h, lev), ws = ceil_shift(p.w, lev);
        const int64_t R0 = r0 >> lev, C0 = c0 >> lev;
        for (int b = t; b < bh * bw; b += 64) {
            const int i = b / bw, k = b - i * bw;
            const bool r1 = 2 * i + 1 < rh, c1 = 2 * k + 1 < rw;
            const int i0 = (2 * i) * pin + 2 * k;
            auto lo_at = [&](int q) { return EX ? ilo[q] : 0.0f; };
            const df x00 = {ihi[i0], lo_at(i0)};
            const df x01 = c1 ? df{ihi[i0 + 1], lo_at(i0 + 1)} : df{0.0f, 0.0f};
            const df x10 = r1 ? df{ihi[i0 + pin], lo_at(i0 + pin)} : df{0.0f, 0.0f};
            const df x11 = (r1 && c1) ? df{ihi[i0 + pin + 1], lo_at(i0 + pin + 1)} : df{0.0f, 0.0f};
            df ll;
            float hl, lh, hh;
            ana_edge_df<EX>(x00, x01, x10, x11, r1, c1, ll, hl, lh, hh);
            const int64_t R = R0 + i, C = C0 + k;
            if (c1) st1_cached<SD>(det + R * dp + ws + C, hl);
            if (r1) st1_cached<SD>(det + (hs + R) * dp + C, lh);
            if (r1 && c1) st1_cached<SD>(det + (hs + R) * dp + ws + C, hh);
            if (lev == L) {
                st1_cached<SL>(llp + R * lp + C, acc_round<EX>(ll));
            } else {
                ohi[i * pout + k] = ll.hi;
                if constexpr (EX) olo[i * pout + k] = ll.lo;
            }
        }
        rh = bh;
        rw = bw;
        if (lev < L) {   // LDS written by some lanes, read by others of this wavefront
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

// ---------------------------------------------------------------------------
// Synthesis tile
// ---------------------------------------------------------------------------
// Everything one thread of a synthesis tile reads from HBM: its share of the
// small levels (LL_L and the bands of levels 3..L, one flat index space:
// level by level HL, LH, HH, then LL_L) and the level-1/2 details of its
// register block.
template <int B1Y, int B1X, int B2Y, int B2X>
struct InvIn {
    float walk[10];      // LL_L, then (HL, LH, HH) of levels 3, 4, 5 on the ancestor path of
                         // this thread's LL3 coefficient
    float hl1[B1Y][B1X], lh1[B1Y][B1X], hh1[B1Y][B1X];
    float hl2[B2Y][B2X], lh2[B2Y][B2X], hh2[B2Y][B2X];
};

template <class SX, class SD, class SL, int RY, int RX, int GY, int GX>
using InvInT = InvIn<RY / 2, RX / 2, RY / 4, RX / 4>;

// NTL: nontemporal loads of the level-1/2 band vectors (see fwd2d_load); the
// ancestor-path values, shared by many lanes, stay ordinary loads.
template <class SX, class SD, class SL, int RY, int RX, int GY, int GX, bool FULL, bool NTL = false>
__device__ __forceinline__ void inv2d_load(const Pass2D& p, int64_t item, int64_t ty, int64_t tx,
                                           InvInT<SX, SD, SL, RY, RX, GY, GX>& in) {
    using G = Geo2D<SX, RY, RX, GY, GX>;
    constexpr int TH = G::TH, TW = G::TW;
    constexpr int B1Y = G::B1Y, B1X = G::B1X, B2Y = G::B2Y, B2X = G::B2X;
    const int t = threadIdx.x, rg = t / GX, cg = t % GX;
    const int64_t r0 = ty * TH, c0 = tx * TW;
    const int L = p.levels;
    const int th = FULL ? TH : (p.h - r0 < TH ? (int)(p.h - r0) : TH);
    const int tw = FULL ? TW : (p.w - c0 < TW ? (int)(p.w - c0) : TW);
    const int lr0 = rg * RY, lc0 = cg * RX;
    const int th1 = (th + 1) >> 1, tw1 = (tw + 1) >> 1;
    const bool inb = FULL || (lr0 + RY <= th && lc0 + RX <= tw);   // whole block inside
    // an edge tile's threads whose block lies wholly outside the region have
    // nothing to read or write (the synthesis has no barrier or shuffle)
    if (!FULL && (lr0 >= th || lc0 >= tw)) return;
    const typename SD::raw* det = reinterpret_cast<const typename SD::raw*>(p.det) + item * p.det_bstride;
    const typename SL::raw* llp = reinterpret_cast<const typename SL::raw*>(p.ll) + item * p.ll_bstride;
    const int64_t dp = p.det_pitch, lp = p.ll_pitch;

    // ---- the ancestor path of this thread's LL3 coefficient: LL_L, then
    // (HL, LH, HH) of levels 3..L (many lanes share these addresses, so most
    // requests hit in cache).  Edge tiles load only the coefficients that
    // exist under the carry rule: HL(i, k) of level j needs column 2k + 1 of
    // the level-(j-1) region, LH(i, k) row 2i + 1, HH both.
    if (L >= 3) {
        const int64_t R3 = ((r0 >> 2) + (lr0 >> 2)) >> 1, C3 = ((c0 >> 2) + (lc0 >> 2)) >> 1;
        const int64_t RL = R3 >> (L - 3), CL = C3 >> (L - 3);
        const bool ll_in = FULL || (RL < ceil_shift(p.h, L) && CL < ceil_shift(p.w, L));
        in.walk[0] = ll_in ? ld1<SL>(llp + RL * lp + CL) : 0.0f;
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
            const int j = 3 + jj;
            if (j <= L) {
                const int64_t hs = ceil_shift(p.h, j), ws = ceil_shift(p.w, j);
                const int64_t R = R3 >> (j - 3), C = C3 >> (j - 3);
                if (FULL) {
                    in.walk[1 + 3 * jj] = ld1<SD>(det + R * dp + ws + C);
                    in.walk[2 + 3 * jj] = ld1<SD>(det + (hs + R) * dp + C);
                    in.walk[3 + 3 * jj] = ld1<SD>(det + (hs + R) * dp + ws + C);
                } else {
                    const bool r1 = 2 * R + 1 < ceil_shift(p.h, j - 1);
                    const bool c1 = 2 * C + 1 < ceil_shift(p.w, j - 1);
                    const bool ri = R < hs, ci = C < ws;
                    in.walk[1 + 3 * jj] = (ri && c1) ? ld1<SD>(det + R * dp + ws + C) : 0.0f;
                    in.walk[2 + 3 * jj] = (r1 && ci) ? ld1<SD>(det + (hs + R) * dp + C) : 0.0f;
                    in.walk[3 + 3 * jj] = (r1 && c1) ? ld1<SD>(det + (hs + R) * dp + ws + C) : 0.0f;
                }
            }
        }
    }
    // ---- level-1 details of this thread's block
    {
        const int64_t hs = ceil_shift(p.h, 1), ws = ceil_shift(p.w, 1);
        const int64_t R = (r0 >> 1) + (lr0 >> 1), C = (c0 >> 1) + (lc0 >> 1);
#pragma unroll
        for (int i = 0; i < B1Y; ++i) {
            if (inb) {
                ld_vec<SD, B1X, NTL>(det + (R + i) * dp + ws + C, in.hl1[i]);
                ld_vec<SD, B1X, NTL>(det + (hs + R + i) * dp + C, in.lh1[i]);
                ld_vec<SD, B1X, NTL>(det + (hs + R + i) * dp + ws + C, in.hh1[i]);
            } else {
#pragma unroll
                for (int k = 0; k < B1X; ++k) {
                    const int lr = lr0 + 2 * i, lc = lc0 + 2 * k;
                    const bool ok = lr < th && lc < tw;
                    const bool r1 = ok && lr + 1 < th, c1 = ok && lc + 1 < tw;
                    in.hl1[i][k] = c1 ? ld1<SD>(det + (R + i) * dp + ws + C + k) : 0.0f;
                    in.lh1[i][k] = r1 ? ld1<SD>(det + (hs + R + i) * dp + C + k) : 0.0f;
                    in.hh1[i][k] = (r1 && c1) ? ld1<SD>(det + (hs + R + i) * dp + ws + C + k) : 0.0f;
                }
            }
        }
    }
    // ---- level-2 details (LL1 itself when L == 1, read into hl2's place: see body)
    if (L >= 2) {
        const int64_t hs = ceil_shift(p.h, 2), ws = ceil_shift(p.w, 2);
        const int64_t R = (r0 >> 2) + (lr0 >> 2), C = (c0 >> 2) + (lc0 >> 2);
#pragma unroll
        for (int i = 0; i < B2Y; ++i) {
            if (inb) {
                ld_vec<SD, B2X, NTL>(det + (R + i) * dp + ws + C, in.hl2[i]);
                ld_vec<SD, B2X, NTL>(det + (hs + R + i) * dp + C, in.lh2[i]);
                ld_vec<SD, B2X, NTL>(det + (hs + R + i) * dp + ws + C, in.hh2[i]);
            } else {
#pragma unroll
                for (int k = 0; k < B2X; ++k) {
                    const int lr = (lr0 >> 1) + 2 * i, lc = (lc0 >> 1) + 2 * k;
                    const bool ok = lr < th1 && lc < tw1;
                    const bool r1 = ok && lr + 1 < th1, c1 = ok && lc + 1 < tw1;
                    in.hl2[i][k] = c1 ? ld1<SD>(det + (R + i) * dp + ws + C + k) : 0.0f;
                    in.lh2[i][k] = r1 ? ld1<SD>(det + (hs + R + i) * dp + C + k) : 0.0f;
                    in.hh2[i][k] = (r1 && c1) ? ld1<SD>(det + (hs + R + i) * dp + ws + C + k) : 0.0f;
                }
            }
        }
    }
}

template <class SX, class SD, class SL, int RY, int RX, int GY, int GX, bool FULL>
__device__ __forceinline__ void inv2d_body(const Pass2D& p, int64_t item, int64_t ty, int64_t tx,
                                           const InvInT<SX, SD, SL, RY, RX, GY, GX>& in) {
    using G = Geo2D<SX, RY, RX, GY, GX>;
    constexpr int TH = G::TH, TW = G::TW;
    constexpr int B1Y = G::B1Y, B1X = G::B1X, B2Y = G::B2Y, B2X = G::B2X;

    const int t = threadIdx.x, rg = t / GX, cg = t % GX;
    const int64_t r0 = ty * TH, c0 = tx * TW;
    const int L = p.levels;
    const int th = FULL ? TH : (p.h - r0 < TH ? (int)(p.h - r0) : TH);
    const int tw = FULL ? TW : (p.w - c0 < TW ? (int)(p.w - c0) : TW);
    const int lr0 = rg * RY, lc0 = cg * RX;
    const int th1 = (th + 1) >> 1, tw1 = (tw + 1) >> 1;
    const int th2 = (th + 3) >> 2, tw2 = (tw + 3) >> 2;
    const bool inb = FULL || (lr0 + RY <= th && lc0 + RX <= tw);   // whole block inside
    if (!FULL && (lr0 >= th || lc0 >= tw)) return;                 // nothing of it to write

    const typename SL::raw* llp = reinterpret_cast<const typename SL::raw*>(p.ll) + item * p.ll_bstride;
    typename SX::raw* dst =
        reinterpret_cast<typename SX::raw*>(p.dst) + item * p.dst_bstride + r0 * p.dst_pitch + c0;
    const int64_t lp = p.ll_pitch;
    const auto& hl1 = in.hl1;
    const auto& lh1 = in.lh1;
    const auto& hh1 = in.hh1;
    const auto& hl2 = in.hl2;
    const auto& lh2 = in.lh2;
    const auto& hh2 = in.hh2;
    // ---- LL2 of this thread (B2Y x B2X), or LL1 directly when L == 1
    float ll1[B1Y][B1X];
    if (L >= 2) {
        float ll2[B2Y][B2X];
        const int64_t R = (r0 >> 2) + (lr0 >> 2), C = (c0 >> 2) + (lc0 >> 2);
        if (L >= 3) {
            // walk the ancestor path: LL_L -> ... -> LL3 (one 2x2 synthesis
            // butterfly per level, keeping the child on the path), then the
            // level-3 butterfly gives this thread's LL2 entries.  Edge tiles
            // apply the carry rule at every level (syn_child); the values of
            // a thread whose block lies outside the region are never stored.
            const int64_t R3 = R >> 1, C3 = C >> 1;
            float ll = in.walk[0];
#pragma unroll
            for (int jj = 2; jj >= 1; --jj) {
                const int j = 3 + jj;               // level j -> level j-1 (j = 5, 4)
                if (j <= L) {
                    const int64_t Rj = R3 >> (j - 3), Cj = C3 >> (j - 3);
                    const int dy = (int)((R3 >> (j - 4)) & 1), dx = (int)((C3 >> (j - 4)) & 1);
                    const float hl = in.walk[1 + 3 * jj], lh = in.walk[2 + 3 * jj],
                                hh = in.walk[3 + 3 * jj];
                    if (FULL) {
                        const float base = dy ? ll + lh : ll - lh, tt = dy ? hl + hh : hl - hh;
                        ll = 0.5f * (dx ? base + tt : base - tt);
                    } else {
                        const bool r1 = 2 * Rj + 1 < ceil_shift(p.h, j - 1);
                        const bool c1 = 2 * Cj + 1 < ceil_shift(p.w, j - 1);
                        ll = syn_child(ll, hl, lh, hh, r1, c1, dy, dx);
                    }
                }
            }
            // level 3: the thread's LL2 rows (one, or the two children rows
            // of its LL3 coefficient when RY = 8) and columns
            static_assert(B2Y <= 2 && B2X <= 2, "one LL3 coefficient per thread");
            const float hl = in.walk[1], lh = in.walk[2], hh = in.walk[3];
            const bool r1 = FULL || 2 * R3 + 1 < ceil_shift(p.h, 2);
            const bool c1 = FULL || 2 * C3 + 1 < ceil_shift(p.w, 2);
#pragma unroll
            for (int i = 0; i < B2Y; ++i) {
                const int dy = (int)((R + i) & 1);
#pragma unroll
                for (int k = 0; k < B2X; ++k) {
                    const int dx = (int)((C + k) & 1);
                    if (FULL) {
                        const float base = dy ? ll + lh : ll - lh, tt = dy ? hl + hh : hl - hh;
                        ll2[i][k] = 0.5f * (dx ? base + tt : base - tt);
                    } else {
                        ll2[i][k] = syn_child(ll, hl, lh, hh, r1, c1, dy, dx);
                    }
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < B2Y; ++i)
#pragma unroll
                for (int k = 0; k < B2X; ++k) {
                    const int lr = (lr0 >> 2) + i, lc = (lc0 >> 2) + k;
                    const bool ok = FULL || (lr < th2 && lc < tw2);
                    ll2[i][k] = ok ? ld1<SL>(llp + (R + i) * lp + C + k) : 0.0f;
                }
        }
#pragma unroll
        for (int i = 0; i < B2Y; ++i)
#pragma unroll
            for (int k = 0; k < B2X; ++k) {
                const int lr = (lr0 >> 1) + 2 * i, lc = (lc0 >> 1) + 2 * k;
                const bool r1 = FULL || lr + 1 < th1, c1 = FULL || lc + 1 < tw1;
                syn_edge(ll2[i][k], hl2[i][k], lh2[i][k], hh2[i][k], r1, c1, ll1[2 * i][2 * k],
                         ll1[2 * i][2 * k + 1], ll1[2 * i + 1][2 * k], ll1[2 * i + 1][2 * k + 1]);
            }
    } else {
        const int64_t R = (r0 >> 1) + (lr0 >> 1), C = (c0 >> 1) + (lc0 >> 1);
#pragma unroll
        for (int i = 0; i < B1Y; ++i) {
            if (inb) {
                ld_vec<SL, B1X>(llp + (R + i) * lp + C, ll1[i]);
            } else {
#pragma unroll
                for (int k = 0; k < B1X; ++k) {
                    const bool ok = lr0 + 2 * i < th && lc0 + 2 * k < tw;
                    ll1[i][k] = ok ? ld1<SL>(llp + (R + i) * lp + C + k) : 0.0f;
                }
            }
        }
    }

    // ---- level 1 -> output block
    float v[RY][RX];
#pragma unroll
    for (int i = 0; i < B1Y; ++i)
#pragma unroll
        for (int k = 0; k < B1X; ++k) {
            const bool r1 = FULL || lr0 + 2 * i + 1 < th, c1 = FULL || lc0 + 2 * k + 1 < tw;
            syn_edge(ll1[i][k], hl1[i][k], lh1[i][k], hh1[i][k], r1, c1, v[2 * i][2 * k],
                     v[2 * i][2 * k + 1], v[2 * i + 1][2 * k], v[2 * i + 1][2 * k + 1]);
        }
    if (inb) {
#pragma unroll
        for (int r = 0; r < RY; ++r) st_vec<SX, RX>(dst + (int64_t)(lr0 + r) * p.dst_pitch + lc0, v[r]);
    } else {
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int c = 0; c < RX; ++c)
                if (lr0 + r < th && lc0 + c < tw)
                    st1<SX>(dst + (int64_t)(lr0 + r) * p.dst_pitch + lc0 + c, v[r][c]);
    }
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

}  // namespace haar
