// Fused shrinkage pipelines: analysis, thresholding of the detail
// coefficients, synthesis, in one pass over HBM.
//
// The applications the paper names (Sec. I, Sec. VI: compression and
// analysis of biosignals and medical images) decompose a signal, act on its
// coefficients and reconstruct it.  Run as three calls, that pipeline moves
// every element through HBM three times; here each work-group does all of it
// for one chunk (1D) or tile (2D) on chip:
//   1. the analysis device code of the plain kernels writes the chunk's or
//      tile's coefficients into a packed buffer in LDS (a chunk or tile whose
//      origin is a multiple of 2^L is its own subtree of the transform, and a
//      ragged last chunk or tile follows the same carry rule as the whole
//      signal, so its coefficients are those of the full transform);
//   2. every detail coefficient of level j is thresholded with thr[j-1]
//      (hard: kept when |d| > t, else 0; soft: sign(d) max(|d| - t, 0)); the
//      approximation a_L / LL_L is kept;
//   3. the synthesis device code reads the buffer and writes the output.
// HBM traffic: the input once, the output once.
//
// The same 2D pipeline also runs one training step of the sparsity loss
// sum |details| + 0.5 ||LL_L||^2 (OP = kOpL1): the coefficient operation is
// then the loss gradient (sign of each detail, LL_L itself), the synthesis
// of it is the gradient with respect to the input (the synthesis bank is
// the transpose of the analysis), and every tile adds its share of the
// loss to a per-tile partial sum, reduced per item afterwards in a fixed
// order.
//
// Full 2D tiles and full 1D chunks take register paths instead: the
// synthesis of a thread's block needs exactly the details that the analysis
// of the same block produced, so those stay in registers (thresholded in
// place); only the small deep levels cross LDS (2D: the tile's LL2 region,
// run by one wavefront; 1D: the levels across wavefronts, on one thread).
#include "haar_1d_chunk.h"
#include "haar.h"
#include "haar_2d_tile.h"
#include "haar_internal.h"

#include <atomic>
#include <mutex>

namespace haar {

struct ShrinkArgs {
    float thr[kMaxShrinkLevels];
    int mode;
    double* partial;                         // kOpL1: one loss partial per tile
};

__device__ __forceinline__ float shrink_value(float d, int mode, float t) {
    if (mode == 0) return fabsf(d) > t ? d : 0.0f;
    const float m = fabsf(d) - t;
    return m > 0.0f ? copysignf(m, d) : 0.0f;
}

// Coefficient operations of the 2D pipeline.
constexpr int kOpShrink = 0, kOpL1 = 1;

// A detail coefficient: thresholded, or replaced by its loss gradient
// sign(d) (sign(0) = 0) while |d| joins the loss.
template <int OP>
__device__ __forceinline__ float detail_op(float d, int mode, float t, float& acc) {
    if constexpr (OP == kOpShrink) {
        return shrink_value(d, mode, t);
    } else {
        acc += fabsf(d);
        return d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
    }
}

// LL_L: kept (its loss gradient is itself); 0.5 LL^2 joins the loss.
template <int OP>
__device__ __forceinline__ void ll_op(float v, float& acc) {
    if constexpr (OP == kOpL1) acc += 0.5f * v * v;
}

// Sum of the work-group's loss shares into partial[slot] (FP64, fixed order).
template <int NT>
__device__ __forceinline__ void tile_loss(float acc, double* partial, int64_t slot) {
    __shared__ double red[NT / 64];
    double v = (double)acc;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < NT / 64; ++i) t += red[i];
        partial[slot] = t;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// 1D: chunks of NT * E samples (levels <= log2 of the chunk)
// ---------------------------------------------------------------------------
// FULL: the complete chunks of every item (chunks_per_item = n / C of them);
// otherwise the ragged last chunk of every item (chunks_per_item = 1).
template <class S, int E, int NT, bool FULL>
__global__ __launch_bounds__(NT) void shrink1d_kernel(const void* x, void* y, int64_t n, int L,
                                                      int64_t chunks_per_item, int64_t total,
                                                      ShrinkArgs sh) {
    using G = Geo1D<S, E, NT>;
    constexpr int C = G::C, NW = G::NW;
    __shared__ float buf[C];                 // the chunk's packed coefficients
    __shared__ float stage[FULL ? C : 1];    // lane-contiguous HBM access of full chunks
    __shared__ df smd[NW];
    __shared__ float smf[NW * 8];
    __shared__ float thr[kMaxShrinkLevels];
    if (threadIdx.x < kMaxShrinkLevels) thr[threadIdx.x] = sh.thr[threadIdx.x];
    for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {
        const int64_t item = b / chunks_per_item;
        const int64_t chunk = FULL ? b - item * chunks_per_item : n / C;
        const int64_t c0 = chunk * C;
        const int cl = FULL ? C : (int)(n - c0);
        Pass1D p{};
        p.n = cl;
        p.batch = 1;
        p.levels = L;
        p.vec_ok = 1;
        p.src = reinterpret_cast<const typename S::raw*>(x) + item * n + c0;
        p.det = buf;
        p.ll = buf;
        fwd1d_chunk<S, StLds, StLds, E, NT, FULL>(p, 0, 0, smd, stage);
        __syncthreads();
        // details of level j occupy [ceil(cl / 2^j), ceil(cl / 2^(j-1)))
        for (int i = (int)ceil_shift(cl, L) + (int)threadIdx.x; i < cl; i += NT) {
            int j = 1;
            while (i < ceil_shift(cl, j)) ++j;
            buf[i] = shrink_value(buf[i], sh.mode, thr[j - 1]);
        }
        __syncthreads();
        p.dst = reinterpret_cast<typename S::raw*>(y) + item * n + c0;
        inv1d_chunk<S, StLds, StLds, E, NT, FULL>(p, 0, 0, smf, stage);
        __syncthreads();                     // LDS reuse by the next chunk
    }
}

// Full chunks, register path.  The synthesis of a thread needs exactly the
// details its own analysis produced (in-thread levels in registers,
// wavefront levels at the same lanes), so every coefficient stays in
// registers; only the input / output staging and the levels across
// wavefronts (at most log2(NT/64), on one thread) use LDS.
// ONE: the grid covers every chunk (one work-group each), so the loop runs
// once and breaks, which keeps fewer values live.
template <class S, int E, int NT, bool ONE = false>
__global__ __launch_bounds__(NT) void shrink1d_full_kernel(const void* x, void* y, int64_t n, int L,
                                                           int64_t per, int64_t total, ShrinkArgs sh) {
    using G = Geo1D<S, E, NT>;
    constexpr int C = G::C, LOG_E = G::LOG_E, NW = G::NW;
    __shared__ float stage[C];
    __shared__ df sv[NW];
    __shared__ float sa[NW], sd[NW * 8];
    __shared__ float thr[kMaxShrinkLevels];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (t < kMaxShrinkLevels) thr[t] = sh.thr[t];
    const int mode = sh.mode;
    for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {
        const int64_t item = b / per, c0 = (b - item * per) * C;
        const typename S::raw* src = reinterpret_cast<const typename S::raw*>(x) + item * n + c0;
        typename S::raw* dst = reinterpret_cast<typename S::raw*>(y) + item * n + c0;

        float xv[E];
        ld_chunk_lanes<S, E>(src, stage, xv, lane, wv);
        df s[E];
#pragma unroll
        for (int e = 0; e < E; ++e) s[e] = df_from(xv[e]);

        // ---- analysis, in-thread levels: details (thresholded) stay in dl,
        // level lev at dl[E - (E >> (lev - 1)) + m]
        float dl[E];
#pragma unroll
        for (int lev = 1; lev <= LOG_E; ++lev) {
            if (lev > L) break;
            const int cnt = E >> lev;
            const float tl = sh.thr[lev - 1];
#pragma unroll
            for (int m = 0; m < E / 2; ++m) {
                if (m >= cnt) continue;
                const df a0 = s[2 * m], a1 = s[2 * m + 1];
                dl[E - (E >> (lev - 1)) + m] = shrink_value(f_norm(df_diff(a1, a0), lev), mode, tl);
                s[m] = df_add(a0, a1);
            }
        }

        float a[E];
        if (L <= LOG_E) {
            const int cnt = E >> L;
#pragma unroll
            for (int m = 0; m < E; ++m) a[m] = m < cnt ? df_norm(s[m], L) : 0.0f;
        } else {
            // ---- analysis, wavefront levels (active lanes keep the detail)
            float dw[6];
            df vv = s[0];
#pragma unroll
            for (int st = 0; st < 6; ++st) {
                const int lev = LOG_E + 1 + st;
                dw[st] = 0.0f;
                if (lev > L) continue;
                const int off = 1 << st;
                const df o = {__shfl_xor(vv.hi, off), __shfl_xor(vv.lo, off)};
                if ((lane & ((off << 1) - 1)) == 0) {
                    dw[st] = shrink_value(f_norm(df_diff(o, vv), lev), mode, sh.thr[lev - 1]);
                    vv = df_add(vv, o);
                }
            }
            float v = 0.0f;
            if (L <= LOG_E + 6) {
                v = df_norm(vv, L);
            } else {
                // ---- levels across wavefronts: analysis, threshold, synthesis
                if (lane == 0) sv[wv] = vv;
                __syncthreads();
                if (t == 0) {
                    constexpr int wtop = LOG_E + 6;
                    int cnt = NW;
                    for (int lev = wtop + 1; lev <= L; ++lev) {
                        for (int P = 0; P < cnt / 2; ++P) {
                            const df a0 = sv[2 * P], a1 = sv[2 * P + 1];
                            sd[(lev - wtop - 1) * NW + P] = shrink_value(f_norm(df_diff(a1, a0), lev), mode,
                                                                         thr[lev - 1]);
                            sv[P] = df_add(a0, a1);
                        }
                        cnt >>= 1;
                    }
                    for (int P = 0; P < cnt; ++P) sa[P] = df_norm(sv[P], L);
                    for (int lev = L; lev >= wtop + 1; --lev) {
                        const int pairs = (NW >> (lev - wtop - 1)) >> 1;
                        for (int P = pairs - 1; P >= 0; --P) {
                            const float aa = sa[P], d = sd[(lev - wtop - 1) * NW + P];
                            sa[2 * P] = (aa - d) * kRs2Hi;
                            sa[2 * P + 1] = (aa + d) * kRs2Hi;
                        }
                    }
                }
                __syncthreads();
                if (lane == 0) v = sa[wv];
            }
            // ---- synthesis, wavefront levels
#pragma unroll
            for (int st = 5; st >= 0; --st) {
                const int lev = LOG_E + 1 + st;
                if (lev > L) continue;
                const int off = 1 << st;
                const bool active = (lane & ((off << 1) - 1)) == 0;
                float e0 = v, e1 = 0.0f;
                if (active) {
                    e0 = (v - dw[st]) * kRs2Hi;
                    e1 = (v + dw[st]) * kRs2Hi;
                }
                const float got = __shfl_xor(e1, off);
                if (active)
                    v = e0;
                else if ((lane & ((off << 1) - 1)) == off)
                    v = got;
            }
            a[0] = v;
        }
        // ---- synthesis, in-thread levels
#pragma unroll
        for (int lev = LOG_E; lev >= 1; --lev) {
            if (lev > L) continue;
            const int cnt = E >> lev;
            const float* d = dl + (E - (E >> (lev - 1)));
#pragma unroll
            for (int m = E / 2 - 1; m >= 0; --m) {
                if (m >= cnt) continue;
                const float am = a[m];
                a[2 * m] = (am - d[m]) * kRs2Hi;
                a[2 * m + 1] = (am + d[m]) * kRs2Hi;
            }
        }
        st_chunk_lanes<S, E>(dst, stage, a, lane, wv);
        if (ONE) break;
        __syncthreads();                     // LDS reuse by the next chunk
    }
}

// ---------------------------------------------------------------------------
// 2D: tiles of 32 rows x GX 16-byte vectors (levels <= 5)
// ---------------------------------------------------------------------------
// Partial tiles (right column, bottom row), LDS-buffer path: edge tile e of
// an item is (ty = e, tx = full_x) for e < right, else (ty = full_y,
// tx = e - right).
template <class S, int GY, int GX, int OP>
__global__ __launch_bounds__(GY* GX) void shrink2d_edge_kernel(const void* x, void* y, int64_t h, int64_t w,
                                                               int L, int64_t full_x, int64_t full_y,
                                                               int64_t right, int64_t bottom,
                                                               int64_t total, ShrinkArgs sh,
                                                               int64_t slot0) {
    constexpr int RX = 16 / S::kBytes;
    using G = Geo2D<S, 4, RX, GY, GX>;
    using In = InvInT<S, StLds, StLds, 4, RX, GY, GX>;
    constexpr int TH = G::TH, TW = G::TW, NT = G::NT;
    __shared__ float buf[TH * TW];           // the tile's packed coefficients (pitch TW)
    __shared__ float sm[G::SMEM];            // analysis levels 3..L
    __shared__ float thr[kMaxShrinkLevels];
    if (threadIdx.x < kMaxShrinkLevels) thr[threadIdx.x] = sh.thr[threadIdx.x];
    const int64_t per = right + bottom;
    for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {
        const int64_t item = b / per, e = b - item * per;
        const int64_t ty = e < right ? e : full_y, tx = e < right ? full_x : e - right;
        const int64_t r0 = ty * TH, c0 = tx * TW;
        const int th = h - r0 < TH ? (int)(h - r0) : TH;
        const int tw = w - c0 < TW ? (int)(w - c0) : TW;
        const int64_t origin = item * h * w + r0 * w + c0;

        Pass2D p{};
        p.h = th;
        p.w = tw;
        p.batch = 1;
        p.levels = L;
        p.vec_ok = 1;
        p.src = reinterpret_cast<const typename S::raw*>(x) + origin;
        p.src_pitch = w;
        p.det = buf;
        p.ll = buf;
        p.det_pitch = p.ll_pitch = TW;
        {
            FwdIn<4, RX> in;
            fwd2d_load<S, 4, RX, GY, GX, false>(p, 0, 0, 0, in);
            fwd2d_body<S, StLds, StLds, 4, RX, GY, GX, false>(p, 0, 0, 0, in, sm);
        }
        __syncthreads();
        // level j bands: inside the level-(j-1) LL region, outside level j's
        float acc = 0.0f;
        for (int e = threadIdx.x; e < th * tw; e += NT) {
            const int rr = e / tw, cc = e - rr * tw;
            int j = 1;
            while (j <= L && rr < ceil_shift(th, j) && cc < ceil_shift(tw, j)) ++j;
            float& c = buf[rr * TW + cc];
            if (j <= L)
                c = detail_op<OP>(c, sh.mode, thr[j - 1], acc);
            else
                ll_op<OP>(c, acc);
        }
        __syncthreads();
        if constexpr (OP == kOpL1) tile_loss<NT>(acc, sh.partial, slot0 + b);
        p.dst = reinterpret_cast<typename S::raw*>(y) + origin;
        p.dst_pitch = w;
        {
            In in;
            inv2d_load<S, StLds, StLds, 4, RX, GY, GX, false>(p, 0, 0, 0, in);
            inv2d_body<S, StLds, StLds, 4, RX, GY, GX, false>(p, 0, 0, 0, in);
        }
        __syncthreads();                     // LDS reuse by the next tile
    }
}

// Full tiles, register path.  LL2 region of the tile: RH x RW = (TH/4) x (TW/4).
// ONE: one work-group per tile (see shrink1d_full_kernel).
template <class S, int GY, int GX, int OP, bool ONE = false, bool NTL = false>
__global__ __launch_bounds__(GY* GX) void shrink2d_full_kernel(const void* x, void* y, int64_t h,
                                                               int64_t w, int L, int64_t full_x,
                                                               int64_t full_y, int64_t total,
                                                               ShrinkArgs sh) {
    constexpr int RX = 16 / S::kBytes, RY = 4;
    constexpr int TH = RY * GY, TW = RX * GX;
    constexpr int B1Y = RY / 2, B1X = RX / 2, B2X = RX / 4;
    constexpr int RH = TH / 4, RW = TW / 4;
    // LDS: LL ping-pong (RH x RW each) and the details of levels 3..5
    constexpr int DET = 3 * ((RH / 2) * (RW / 2) + (RH / 4) * (RW / 4) + (RH / 8) * (RW / 8));
    __shared__ float lla[RH * RW], llb[RH * RW], dets[DET];
    __shared__ float thr[kMaxShrinkLevels];
    const int t = threadIdx.x, rg = t / GX, cg = t % GX;
    const int lr0 = rg * RY, lc0 = cg * RX;
    if (t < kMaxShrinkLevels) thr[t] = sh.thr[t];
    const int mode = sh.mode;
    const float t1 = sh.thr[0], t2 = sh.thr[1];
    const int64_t per = full_x * full_y;
    for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {
        const int64_t item = b / per, r = b - item * per;
        const int64_t ty = r / full_x, tx = r - ty * full_x;
        const int64_t origin = item * h * w + ty * TH * w + tx * TW;
        const typename S::raw* src = reinterpret_cast<const typename S::raw*>(x) + origin;
        typename S::raw* dst = reinterpret_cast<typename S::raw*>(y) + origin;

        float v[RY][RX];
#pragma unroll
        for (int i = 0; i < RY; ++i) ld_vec<S, RX, NTL>(src + (int64_t)(lr0 + i) * w + lc0, v[i]);
        float acc = 0.0f;                    // this thread's share of the loss (kOpL1)

        // ---- analysis, levels 1 and 2 (details thresholded in registers)
        df a1[B1Y][B1X];
        float hl1[B1Y][B1X], lh1[B1Y][B1X], hh1[B1Y][B1X];
#pragma unroll
        for (int i = 0; i < B1Y; ++i)
#pragma unroll
            for (int k = 0; k < B1X; ++k) {
                ana_full_f(v[2 * i][2 * k], v[2 * i][2 * k + 1], v[2 * i + 1][2 * k], v[2 * i + 1][2 * k + 1],
                           a1[i][k], hl1[i][k], lh1[i][k], hh1[i][k]);
                hl1[i][k] = detail_op<OP>(hl1[i][k], mode, t1, acc);
                lh1[i][k] = detail_op<OP>(lh1[i][k], mode, t1, acc);
                hh1[i][k] = detail_op<OP>(hh1[i][k], mode, t1, acc);
            }
        float ll1[B1Y][B1X];
        if (L == 1) {
#pragma unroll
            for (int i = 0; i < B1Y; ++i)
#pragma unroll
                for (int k = 0; k < B1X; ++k) {
                    ll1[i][k] = df_round(a1[i][k]);
                    ll_op<OP>(ll1[i][k], acc);
                }
        } else {
            df a2[B2X];
            float hl2[B2X], lh2[B2X], hh2[B2X], ll2[B2X];
#pragma unroll
            for (int k = 0; k < B2X; ++k) {
                ana_full_df(a1[0][2 * k], a1[0][2 * k + 1], a1[1][2 * k], a1[1][2 * k + 1], a2[k], hl2[k],
                            lh2[k], hh2[k]);
                hl2[k] = detail_op<OP>(hl2[k], mode, t2, acc);
                lh2[k] = detail_op<OP>(lh2[k], mode, t2, acc);
                hh2[k] = detail_op<OP>(hh2[k], mode, t2, acc);
                ll2[k] = df_round(a2[k]);
                if (L == 2) ll_op<OP>(ll2[k], acc);
            }
            if (L >= 3) {
                // ---- levels 3..L on the LL2 region, by the first wavefront
#pragma unroll
                for (int k = 0; k < B2X; ++k) lla[(lr0 >> 2) * RW + (lc0 >> 2) + k] = ll2[k];
                __syncthreads();
                if (t < 64) {
                    float* cur = lla;
                    float* nxt = llb;
                    int doff[6];
                    int off = 0, ch = RH, cw = RW;
                    for (int lev = 3; lev <= L; ++lev) {          // analysis + threshold
                        const int bh = ch >> 1, bw = cw >> 1, nb = bh * bw;
                        doff[lev] = off;
                        const float tl = thr[lev - 1];
                        for (int q = t; q < nb; q += 64) {
                            const int i = q / bw, k = q - i * bw;
                            const float x00 = cur[(2 * i) * cw + 2 * k], x01 = cur[(2 * i) * cw + 2 * k + 1];
                            const float x10 = cur[(2 * i + 1) * cw + 2 * k], x11 = cur[(2 * i + 1) * cw + 2 * k + 1];
                            df ll;
                            float hl, lh, hh;
                            ana_full_f(x00, x01, x10, x11, ll, hl, lh, hh);
                            nxt[q] = df_round(ll);
                            dets[off + q] = detail_op<OP>(hl, mode, tl, acc);
                            dets[off + nb + q] = detail_op<OP>(lh, mode, tl, acc);
                            dets[off + 2 * nb + q] = detail_op<OP>(hh, mode, tl, acc);
                        }
                        off += 3 * nb;
                        ch = bh;
                        cw = bw;
                        float* tmp = cur;
                        cur = nxt;
                        nxt = tmp;
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    }
                    if constexpr (OP == kOpL1)                   // LL_L (ch x cw) joins the loss
                        for (int q = t; q < ch * cw; q += 64) ll_op<OP>(cur[q], acc);
                    for (int lev = L; lev >= 3; --lev) {          // synthesis
                        const int bh = ch, bw = cw, nb = bh * bw, ow = 2 * bw;
                        const int o = doff[lev];
                        for (int q = t; q < nb; q += 64) {
                            const int i = q / bw, k = q - i * bw;
                            float x00, x01, x10, x11;
                            syn_edge(cur[q], dets[o + q], dets[o + nb + q], dets[o + 2 * nb + q], true, true,
                                     x00, x01, x10, x11);
                            nxt[(2 * i) * ow + 2 * k] = x00;
                            nxt[(2 * i) * ow + 2 * k + 1] = x01;
                            nxt[(2 * i + 1) * ow + 2 * k] = x10;
                            nxt[(2 * i + 1) * ow + 2 * k + 1] = x11;
                        }
                        ch = 2 * bh;
                        cw = 2 * bw;
                        float* tmp = cur;
                        cur = nxt;
                        nxt = tmp;
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    }
                    // analysis and synthesis swapped the buffers L - 2 times
                    // each: the reconstructed LL2 region (pitch RW) is in lla
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < B2X; ++k) ll2[k] = lla[(lr0 >> 2) * RW + (lc0 >> 2) + k];
            }
            // ---- synthesis, level 2
#pragma unroll
            for (int k = 0; k < B2X; ++k)
                syn_edge(ll2[k], hl2[k], lh2[k], hh2[k], true, true, ll1[0][2 * k], ll1[0][2 * k + 1],
                         ll1[1][2 * k], ll1[1][2 * k + 1]);
        }
        // ---- synthesis, level 1, and the output block
#pragma unroll
        for (int i = 0; i < B1Y; ++i)
#pragma unroll
            for (int k = 0; k < B1X; ++k)
                syn_edge(ll1[i][k], hl1[i][k], lh1[i][k], hh1[i][k], true, true, v[2 * i][2 * k],
                         v[2 * i][2 * k + 1], v[2 * i + 1][2 * k], v[2 * i + 1][2 * k + 1]);
#pragma unroll
        for (int i = 0; i < RY; ++i) st_vec<S, RX>(dst + (int64_t)(lr0 + i) * w + lc0, v[i]);
        if constexpr (OP == kOpL1) tile_loss<GY * GX>(acc, sh.partial, b);
        if (ONE) break;
        if (L >= 3) __syncthreads();         // LDS reuse by the next tile
    }
}

// Loss of each item: its interior tiles' partials [item * per_full, ...) and
// its edge tiles' partials [nfull + item * per_edge, ...), summed in a fixed
// order by one work-group per item.
__global__ __launch_bounds__(256) void l1_loss_reduce_kernel(const double* partial, double* loss,
                                                            int64_t batch, int64_t per_full,
                                                            int64_t per_edge, int64_t nfull) {
    __shared__ double red[4];
    for (int64_t item = blockIdx.x; item < batch; item += gridDim.x) {
        double v = 0.0;
        for (int64_t i = threadIdx.x; i < per_full; i += 256) v += partial[item * per_full + i];
        for (int64_t i = threadIdx.x; i < per_edge; i += 256) v += partial[nfull + item * per_edge + i];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) loss[item] = (red[0] + red[1]) + (red[2] + red[3]);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static ShrinkArgs shrink_args(int L, int mode, const float* thr) {
    ShrinkArgs a{};
    for (int j = 0; j < L && j < kMaxShrinkLevels; ++j) a.thr[j] = thr[j];
    a.mode = mode;
    return a;
}

constexpr int64_t kMaxGridShrink = 1 << 20;

template <class S>
static hipError_t launch_shrink1d(const void* x, void* y, int64_t n, int L, int64_t batch,
                                  const ShrinkArgs& a, hipStream_t s) {
    constexpr int NT = kShrinkChunkThreads, E = kShrinkChunk / kShrinkChunkThreads;
    const int64_t per = n / kShrinkChunk, total = per * batch;
    if (total > 0) {
        const unsigned grid = (unsigned)(total < kMaxGridShrink ? total : kMaxGridShrink);
        if (total <= kMaxGridShrink)
            hipLaunchKernelGGL((shrink1d_full_kernel<S, E, NT, true>), dim3(grid), dim3(NT), 0, s, x, y, n, L,
                               per, total, a);
        else
            hipLaunchKernelGGL((shrink1d_full_kernel<S, E, NT>), dim3(grid), dim3(NT), 0, s, x, y, n, L, per,
                               total, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n % kShrinkChunk != 0) {
        const unsigned grid = (unsigned)(batch < kMaxGridShrink ? batch : kMaxGridShrink);
        hipLaunchKernelGGL((shrink1d_kernel<S, E, NT, false>), dim3(grid), dim3(NT), 0, s, x, y, n, L,
                           (int64_t)1, batch, a);
        return hipGetLastError();
    }
    return hipSuccess;
}

// Tile grid of the 2D pipeline: interior tiles, then the right column and
// the bottom row of partial tiles.
struct ShrinkGrid2D {
    int64_t full_x, full_y, right, bottom;
    int64_t per_full() const { return full_x * full_y; }
    int64_t per_edge() const { return right + bottom; }
};

template <class S>
static ShrinkGrid2D shrink_grid2d(int64_t h, int64_t w) {
    constexpr int TH = 32, TW = 32 * (16 / S::kBytes);
    ShrinkGrid2D g;
    const int64_t tiles_x = (w + TW - 1) / TW, tiles_y = (h + TH - 1) / TH;
    g.full_x = w / TW;
    g.full_y = h / TH;
    g.right = tiles_x > g.full_x ? g.full_y : 0;
    g.bottom = tiles_y > g.full_y ? tiles_x : 0;
    return g;
}

template <class S, int OP>
static hipError_t launch_shrink2d(const void* x, void* y, int64_t h, int64_t w, int L, int64_t batch,
                                  const ShrinkArgs& a, hipStream_t s) {
    constexpr int GY = 8, GX = 32;
    const ShrinkGrid2D g = shrink_grid2d<S>(h, w);
    const int64_t interior = g.per_full() * batch;
    if (interior > 0) {
        const unsigned grid = (unsigned)(interior < kMaxGridShrink ? interior : kMaxGridShrink);
        // one tile per work-group without the loop: FP32 4096^2 L5 shrinkage
        // 26.8 -> 26.1 us, BF16 19.3 -> 17.9 us, BF16 training step of
        // 192 x 512^2 43.0 -> 39.2 us; the FP32 training step ran slower
        // that way (66.0 -> 69.9 us at 8 instead of 6 wavefronts per SIMD)
        const bool one = interior <= kMaxGridShrink && !(OP == kOpL1 && S::kBytes == 4);
        // tile rows on whole 128-byte lines: nontemporal loads for the
        // shrinkage (FP32 4096^2 L5 26.2 -> 25.4 us, BF16 18.1 -> 17.9 us);
        // the training step ran 7 % slower with them and keeps ordinary loads
        const bool ntl = OP == kOpShrink && one && aligned(x, 128) && (w * S::kBytes) % 128 == 0;
        if (ntl)
            hipLaunchKernelGGL((shrink2d_full_kernel<S, GY, GX, OP, true, true>), dim3(grid), dim3(GY * GX), 0,
                               s, x, y, h, w, L, g.full_x, g.full_y, interior, a);
        else if (one)
            hipLaunchKernelGGL((shrink2d_full_kernel<S, GY, GX, OP, true>), dim3(grid), dim3(GY * GX), 0, s, x,
                               y, h, w, L, g.full_x, g.full_y, interior, a);
        else
            hipLaunchKernelGGL((shrink2d_full_kernel<S, GY, GX, OP>), dim3(grid), dim3(GY * GX), 0, s, x, y, h,
                               w, L, g.full_x, g.full_y, interior, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int64_t edge = g.per_edge() * batch;
    if (edge > 0) {
        const unsigned grid = (unsigned)(edge < kMaxGridShrink ? edge : kMaxGridShrink);
        hipLaunchKernelGGL((shrink2d_edge_kernel<S, GY, GX, OP>), dim3(grid), dim3(GY * GX), 0, s, x, y, h,
                           w, L, g.full_x, g.full_y, g.right, g.bottom, edge, a, interior);
        return hipGetLastError();
    }
    return hipSuccess;
}

int run_shrink_1d(const void* in, void* out, int64_t n, int L, int64_t batch, int dtype, int mode,
                  const float* thr, hipStream_t s) {
    const ShrinkArgs a = shrink_args(L, mode, thr);
    hipError_t e;
    switch (dtype) {
        case 0: e = launch_shrink1d<StF32>(in, out, n, L, batch, a, s); break;
        case 1: e = launch_shrink1d<StBF16>(in, out, n, L, batch, a, s); break;
        default: e = launch_shrink1d<StF16>(in, out, n, L, batch, a, s); break;
    }
    return e == hipSuccess ? 0 : hip_error(e, "shrink1d launch");
}

int run_shrink_2d(const void* in, void* out, int64_t h, int64_t w, int L, int64_t batch, int dtype,
                  int mode, const float* thr, hipStream_t s) {
    const ShrinkArgs a = shrink_args(L, mode, thr);
    hipError_t e;
    switch (dtype) {
        case 0: e = launch_shrink2d<StF32, kOpShrink>(in, out, h, w, L, batch, a, s); break;
        case 1: e = launch_shrink2d<StBF16, kOpShrink>(in, out, h, w, L, batch, a, s); break;
        default: e = launch_shrink2d<StF16, kOpShrink>(in, out, h, w, L, batch, a, s); break;
    }
    return e == hipSuccess ? 0 : hip_error(e, "shrink2d launch");
}

// Loss partials of the training step without allocation
// (haar_l1_grad_2d_noalloc): one double per tile in a file-scope device
// array.  Every GPU the library runs on holds its own copy until the process
// ends.  In host code the array's name is a host-side stand-in, not a device
// address: host code uses only the address hipGetSymbolAddress returns for
// the current device, kept per device by static_partials().  Every tile
// writes its own partial before the reduction reads it, so nothing in the
// array has to start at zero; calls that overlap in time on one GPU share it
// and race.
static __device__ __align__(256) double scratch[kStaticLossPartials];

constexpr int kMaxScratchDevices = 64;
static std::atomic<double*> g_scratch_dev[kMaxScratchDevices];
static std::mutex g_scratch_mu;

// Device address of `scratch` on the current device (looked up once per
// device, with that device current).
static int static_partials(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxScratchDevices)
        return set_error(HAAR_ERR_UNSUPPORTED, "device %d beyond the %d devices the static scratch serves", dev,
                         kMaxScratchDevices);
    double* p = g_scratch_dev[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = g_scratch_dev[dev].load(std::memory_order_relaxed);
        if (!p) {
            void* addr = nullptr;
            e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress (static loss partials)");
            if (!addr) return set_error(HAAR_ERR_HIP, "hipGetSymbolAddress returned NULL for the loss partials");
            p = static_cast<double*>(addr);
            g_scratch_dev[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return 0;
}

template <class S>
static int64_t l1_grad_parts_s(int64_t h, int64_t w, int64_t batch) {
    const ShrinkGrid2D g = shrink_grid2d<S>(h, w);
    return (g.per_full() + g.per_edge()) * batch;
}

int64_t l1_grad_partials(int64_t h, int64_t w, int64_t batch, int dtype) {
    return dtype == 0 ? l1_grad_parts_s<StF32>(h, w, batch) : l1_grad_parts_s<StBF16>(h, w, batch);
}

// partial = nullptr: the loss partials live in stream-ordered scratch
// (hipMallocAsync / hipFreeAsync on s); otherwise in the given device array
// of at least l1_grad_partials() doubles.
template <class S>
static int l1_grad_2d_s(const void* in, void* out, double* loss, int64_t h, int64_t w, int L, int64_t batch,
                        double* partial, hipStream_t s) {
    const ShrinkGrid2D g = shrink_grid2d<S>(h, w);
    const int64_t nfull = g.per_full() * batch, nparts = nfull + g.per_edge() * batch;
    ShrinkArgs a{};
    const bool own = partial == nullptr;
    if (own) {
        hipError_t e = hipMallocAsync((void**)&a.partial, (size_t)nparts * sizeof(double), s);
        if (e != hipSuccess) return hip_error(e, "hipMallocAsync (loss partials)");
    } else {
        a.partial = partial;
    }
    hipError_t e = launch_shrink2d<S, kOpL1>(in, out, h, w, L, batch, a, s);
    if (e == hipSuccess) {
        const unsigned grid = (unsigned)(batch < kMaxGridShrink ? batch : kMaxGridShrink);
        hipLaunchKernelGGL(l1_loss_reduce_kernel, dim3(grid), dim3(256), 0, s, a.partial, loss, batch,
                           g.per_full(), g.per_edge(), nfull);
        e = hipGetLastError();
    }
    const hipError_t ef = own ? hipFreeAsync(a.partial, s) : hipSuccess;
    if (e != hipSuccess) return hip_error(e, "l1 gradient launch");
    return ef == hipSuccess ? 0 : hip_error(ef, "hipFreeAsync");
}

static int l1_grad_2d_dtype(const void* in, void* out, double* loss, int64_t h, int64_t w, int L,
                            int64_t batch, int dtype, double* partial, hipStream_t s) {
    switch (dtype) {
        case 0: return l1_grad_2d_s<StF32>(in, out, loss, h, w, L, batch, partial, s);
        case 1: return l1_grad_2d_s<StBF16>(in, out, loss, h, w, L, batch, partial, s);
        default: return l1_grad_2d_s<StF16>(in, out, loss, h, w, L, batch, partial, s);
    }
}

int run_l1_grad_2d(const void* in, void* out, double* loss, int64_t h, int64_t w, int L, int64_t batch,
                   int dtype, hipStream_t s) {
    return l1_grad_2d_dtype(in, out, loss, h, w, L, batch, dtype, nullptr, s);
}

int run_l1_grad_2d_static(const void* in, void* out, double* loss, int64_t h, int64_t w, int L,
                          int64_t batch, int dtype, hipStream_t s) {
    double* partial = nullptr;
    const int rc = static_partials(&partial);
    if (rc != 0) return rc;
    return l1_grad_2d_dtype(in, out, loss, h, w, L, batch, dtype, partial, s);
}

}  // namespace haar
