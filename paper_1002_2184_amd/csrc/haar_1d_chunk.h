// Fused multi-level 1D Haar analysis / synthesis kernels for gfx950.
//
// A work-group owns a chunk of C = NT * E consecutive samples (C = 2^k), so
// the first k levels of the chunk need nothing from outside it.  Per level,
// the polyphase pairs (x[2m], x[2m+1]) give one sum and one difference
// (Eq. (11)-(12), Fig. 4).  Levels run
//   1 .. log2(E)              in registers (each thread holds E samples),
//   log2(E)+1 .. log2(E)+6    across the 64 lanes of a wavefront (xor shuffles),
//   the rest                  across wavefronts through LDS.
// The analysis keeps unnormalised compensated sums S_j (a_j = S_j 2^(-j/2)),
// so no level rounds a 1/sqrt2 factor; details and the final approximation
// are scaled once.  The synthesis (Eq. (19), Fig. 7) runs the same schedule
// backwards in plain FP32.  Odd counts follow the carry rule (the last sample
// of an odd-length level passes unscaled to the next approximation).
#pragma once

#include "haar_device.h"
#include "haar_kernels.h"

namespace haar {

template <int X>
struct Log2 {
    static constexpr int v = 1 + Log2<X / 2>::v;
};
template <>
struct Log2<1> {
    static constexpr int v = 0;
};

// SX: storage of the region (analysis input / synthesis output), SD: detail
// storage, SL: storage of the pass's deepest approximation (FP32 scratch
// between the passes of a deep reduced-precision transform).
template <class SX, int E, int NT>
struct Geo1D {
    static constexpr int C = E * NT, LOG_E = Log2<E>::v, NW = NT / 64, LOG_NW = Log2<NW>::v;
    static constexpr int LOG_C = LOG_E + 6 + LOG_NW;
    static constexpr int VEC = 16 / SX::kBytes;   // region elements per 16-byte access
    static_assert(NT % 64 == 0 && (E * SX::kBytes) % 16 == 0, "chunk geometry");
};

// Store / load N consecutive elements with accesses of at most 16 bytes.
template <class S, int N>
__device__ __forceinline__ void st_span(typename S::raw* p, const float* v) {
    constexpr int V = N < 16 / S::kBytes ? N : 16 / S::kBytes;
#pragma unroll
    for (int q = 0; q < N / V; ++q) st_vec<S, V>(p + q * V, v + q * V);
}
template <class S, int N>
__device__ __forceinline__ void ld_span(const typename S::raw* p, float* v) {
    constexpr int V = N < 16 / S::kBytes ? N : 16 / S::kBytes;
#pragma unroll
    for (int q = 0; q < N / V; ++q) ld_vec<S, V>(p + q * V, v + q * V);
}

// Full chunks read and write HBM lane-contiguously: instruction q of a
// wavefront covers one contiguous span (64 lanes x 16 bytes), which the memory
// system serves far better than a thread-contiguous layout (each thread's E
// samples as consecutive vectors, so that one instruction touches every
// cache line of the wavefront's slice only partly).  The compute layout stays
// thread-contiguous: wavefront w stages its slice of NT/64 ... through LDS
// (`stage`, 64 * E floats per wavefront, wavefront-local ordering only).
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// NTL: nontemporal loads (chunks that own whole cache lines).
template <class SX, int E, bool NTL = false>
__device__ __forceinline__ void ld_chunk_lanes(const typename SX::raw* src, float* stage, float (&x)[E],
                                               int lane, int wv) {
    constexpr int VEC = 16 / SX::kBytes, NV = E / VEC;
    const typename SX::raw* ws = src + (int64_t)wv * 64 * E;
    float* st = stage + wv * 64 * E;
    float v[NV][VEC];
#pragma unroll
    for (int q = 0; q < NV; ++q) ld_vec<SX, VEC, NTL>(ws + (q * 64 + lane) * VEC, v[q]);
#pragma unroll
    for (int q = 0; q < NV; ++q)
#pragma unroll
        for (int e = 0; e < VEC; ++e) st[(q * 64 + lane) * VEC + e] = v[q][e];
    wave_sync_lds();
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = st[lane * E + e];
}

template <class SX, int E>
__device__ __forceinline__ void st_chunk_lanes(typename SX::raw* dst, float* stage, const float (&a)[E],
                                               int lane, int wv) {
    constexpr int VEC = 16 / SX::kBytes, NV = E / VEC;
    typename SX::raw* ws = dst + (int64_t)wv * 64 * E;
    float* st = stage + wv * 64 * E;
#pragma unroll
    for (int e = 0; e < E; ++e) st[lane * E + e] = a[e];
    wave_sync_lds();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        float v[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) v[e] = st[(q * 64 + lane) * VEC + e];
        st_vec<SX, VEC>(ws + (q * 64 + lane) * VEC, v);
    }
}

// ---------------------------------------------------------------------------
// Analysis: in-thread levels (template recursion keeps register indices static)
// ---------------------------------------------------------------------------
// wst: this wavefront's LDS slice (64 * E floats, free once the input has
// been read from it), used to store spans wider than 16 bytes per thread
// lane-contiguously.
template <class SD, int E, bool FULL, int LEV>
__device__ __forceinline__ void fwd_thread_levels(df (&s)[E], int L, int t, int cl, int64_t n,
                                                  int64_t c0, typename SD::raw* det, float* wst) {
    constexpr int LOG_E = Log2<E>::v;
    if constexpr (LEV <= LOG_E) {
        if (LEV > L) return;
        constexpr int CNT = E >> LEV;
        const int len = (int)ceil_shift(cl, LEV - 1);
        float d[CNT];
#pragma unroll
        for (int m = 0; m < CNT; ++m) {
            const df a = s[2 * m], b = s[2 * m + 1];
            const int P = t * CNT + m;
            d[m] = f_norm(df_diff(b, a), LEV);
            if (FULL || 2 * P + 1 < len)
                s[m] = df_add(a, b);
            else if (2 * P < len)
                s[m] = df_s2(a);        // carried: a_j = a_{j-1}  <=>  S_j = sqrt2 S_{j-1}
            else
                s[m] = a;
        }
        typename SD::raw* dp = det + ceil_shift(n, LEV) + (c0 >> LEV) + (int64_t)t * CNT;
        if constexpr (FULL && SD::kStream && CNT * SD::kBytes > 16) {
            constexpr int V = 16 / SD::kBytes;
            const int lane = t & 63;
            typename SD::raw* wb = dp - (int64_t)lane * CNT;   // the wavefront's segment
            wave_sync_lds();                                   // the slice's input reads are done
#pragma unroll
            for (int m = 0; m < CNT; ++m) wst[lane * CNT + m] = d[m];
            wave_sync_lds();
#pragma unroll
            for (int q = 0; q < CNT / V; ++q) {
                float o[V];
#pragma unroll
                for (int e = 0; e < V; ++e) o[e] = wst[(q * 64 + lane) * V + e];
                st_vec<SD, V>(wb + (q * 64 + lane) * V, o);
            }
        } else if constexpr (FULL) {
            st_span<SD, CNT>(dp, d);
        } else {
#pragma unroll
            for (int m = 0; m < CNT; ++m)
                if (2 * (t * CNT + m) + 1 < len) st1<SD>(dp + m, d[m]);
        }
        fwd_thread_levels<SD, E, FULL, LEV + 1>(s, L, t, cl, n, c0, det, wst);
    }
}

// The E >> L approximations of a thread after L <= log2(E) in-thread levels,
// normalised and stored as one span (L is a runtime value: the template
// recursion selects the span length).
template <class SL, int E, int LEV>
__device__ __forceinline__ void st_approx(const df (&s)[E], int L, typename SL::raw* base, int t) {
    if constexpr ((E >> LEV) >= 1) {
        if (L == LEV) {
            constexpr int CNT = E >> LEV;
            float o[CNT];
#pragma unroll
            for (int m = 0; m < CNT; ++m) o[m] = df_norm(s[m], LEV);
            st_span<SL, CNT>(base + (int64_t)t * CNT, o);
            return;
        }
        st_approx<SL, E, LEV + 1>(s, L, base, t);
    }
}

template <class SL, int E, int LEV>
__device__ __forceinline__ void ld_approx(float (&a)[E], int L, const typename SL::raw* base, int t) {
    if constexpr ((E >> LEV) >= 1) {
        if (L == LEV) {
            constexpr int CNT = E >> LEV;
            ld_span<SL, CNT>(base + (int64_t)t * CNT, a);
            return;
        }
        ld_approx<SL, E, LEV + 1>(a, L, base, t);
    }
}

template <class SX, class SD, class SL, int E, int NT, bool FULL, bool NTL = false>
__device__ __forceinline__ void fwd1d_chunk(const Pass1D& p, int64_t item, int64_t chunk, df* sm,
                                            float* stage) {
    using G = Geo1D<SX, E, NT>;
    constexpr int C = G::C, LOG_E = G::LOG_E, VEC = G::VEC;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int L = p.levels;
    const int64_t n = p.n, c0 = chunk * C;
    const int cl = FULL ? C : (n - c0 < C ? (int)(n - c0) : C);
    const typename SX::raw* src = reinterpret_cast<const typename SX::raw*>(p.src) + item * p.src_bstride + c0;
    typename SD::raw* det = reinterpret_cast<typename SD::raw*>(p.det) + item * p.det_bstride;
    typename SL::raw* llp = reinterpret_cast<typename SL::raw*>(p.ll) + item * p.ll_bstride;

    float x[E];
    if constexpr (FULL) {
        ld_chunk_lanes<SX, E, NTL>(src, stage, x, lane, wv);
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = (t * E + e < cl) ? ld1<SX>(src + t * E + e) : 0.0f;
    }
    df s[E];
#pragma unroll
    for (int e = 0; e < E; ++e) s[e] = df_from(x[e]);
    fwd_thread_levels<SD, E, FULL, 1>(s, L, t, cl, n, c0, det, FULL ? stage + wv * 64 * E : nullptr);

    if (L <= LOG_E) {                    // approximations straight from registers
        if constexpr (FULL) {
            st_approx<SL, E, 1>(s, L, llp + (c0 >> L), t);
        } else {
            const int cnt = E >> L;      // runtime count (power of two)
            const int lenL = (int)ceil_shift(cl, L);
#pragma unroll
            for (int m = 0; m < E; ++m)
                if (m < cnt && t * cnt + m < lenL) st1<SL>(llp + (c0 >> L) + t * cnt + m, df_norm(s[m], L));
        }
        return;
    }

    // ---- wavefront levels (xor shuffles)
    df v = s[0];
#pragma unroll
    for (int st = 0; st < 6; ++st) {
        const int lev = LOG_E + 1 + st;
        if (lev > L) break;
        const int off = 1 << st;
        df o;
        o.hi = __shfl_xor(v.hi, off);
        o.lo = __shfl_xor(v.lo, off);
        const bool active = (lane & ((off << 1) - 1)) == 0;
        const int P = t >> (st + 1);
        const int len = (int)ceil_shift(cl, lev - 1);
        if (active && 2 * P < len) {
            if (2 * P + 1 < len) {
                st1<SD>(det + ceil_shift(n, lev) + (c0 >> lev) + P, f_norm(df_diff(o, v), lev));
                v = df_add(v, o);
            } else {
                v = df_s2(v);
            }
        }
    }
    if (L <= LOG_E + 6) {
        const int st = L - LOG_E;
        const int P = t >> st;
        if ((lane & ((1 << st) - 1)) == 0 && P < ceil_shift(cl, L))
            st1<SL>(llp + (c0 >> L) + P, df_norm(v, L));
        return;
    }

    // ---- across wavefronts (LDS, one thread: at most log2(NW) levels)
    if (lane == 0) sm[wv] = v;
    __syncthreads();
    if (t == 0) {
        int cnt = (int)ceil_shift(cl, LOG_E + 6);
        for (int lev = LOG_E + 7; lev <= L; ++lev) {
            const int len = cnt;
            for (int P = 0; 2 * P < len; ++P) {
                const df a = sm[2 * P];
                if (2 * P + 1 < len) {
                    const df b = sm[2 * P + 1];
                    st1<SD>(det + ceil_shift(n, lev) + (c0 >> lev) + P, f_norm(df_diff(b, a), lev));
                    sm[P] = df_add(a, b);
                } else {
                    sm[P] = df_s2(a);
                }
            }
            cnt = (len + 1) >> 1;
        }
        for (int P = 0; P < cnt; ++P) st1<SL>(llp + (c0 >> L) + P, df_norm(sm[P], L));
    }
}

// ---------------------------------------------------------------------------
// Synthesis
// ---------------------------------------------------------------------------
// has_top: the chunk's single deepest approximation (the pass covers the
// whole on-chip depth, so a chunk holds one value at its deepest level) is
// supplied by the caller in `top` instead of being read from p.ll.
// DEEP (full chunks, L > log2(E)): every in-thread level is present and all
// loads are issued as straight-line code (a lane that holds no value of a
// wavefront level reads its group's value: same address, same cache line), so
// that no branch separates them and they overlap in one memory round trip.
template <class SX, class SD, class SL, int E, int NT, bool FULL, bool DEEP = false, bool NTL = false>
__device__ __forceinline__ void inv1d_chunk(const Pass1D& p, int64_t item, int64_t chunk, float* sm,
                                            float* stage, bool has_top = false, float top = 0.0f) {
    static_assert(!DEEP || FULL, "the straight-line loads need a full chunk");
    using G = Geo1D<SX, E, NT>;
    constexpr int C = G::C, LOG_E = G::LOG_E, VEC = G::VEC, NW = G::NW;
    constexpr int VECD = 16 / SD::kBytes;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int L = p.levels;
    const int64_t n = p.n, c0 = chunk * C;
    const int cl = FULL ? C : (n - c0 < C ? (int)(n - c0) : C);
    const typename SD::raw* det = reinterpret_cast<const typename SD::raw*>(p.det) + item * p.det_bstride;
    const typename SL::raw* llp = reinterpret_cast<const typename SL::raw*>(p.ll) + item * p.ll_bstride;
    typename SX::raw* dst = reinterpret_cast<typename SX::raw*>(p.dst) + item * p.dst_bstride + c0;

    // ---- issue every load of this thread first
    // in-thread details: level lev (1..LOG_E) at dl[E - (E >> (lev-1)) + m]
    float dl[E];
#pragma unroll
    for (int lev = 1; lev <= LOG_E; ++lev) {
        if (!DEEP && lev > L) break;
        const int cnt = E >> lev;
        const int len = (int)ceil_shift(cl, lev - 1);
        const typename SD::raw* dp = det + ceil_shift(n, lev) + (c0 >> lev) + (int64_t)t * cnt;
        float* o = dl + (E - (E >> (lev - 1)));
        if constexpr (FULL) {
            if (cnt >= VECD) {
#pragma unroll
                for (int q = 0; q < (E / 2 + VECD - 1) / VECD; ++q)
                    if (q * VECD < cnt) ld_vec<SD, VECD, NTL>(dp + q * VECD, o + q * VECD);
            } else {
#pragma unroll
                for (int m = 0; m < E / 2; ++m)
                    if (m < cnt) o[m] = ld1<SD>(dp + m);
            }
        } else {
#pragma unroll
            for (int m = 0; m < E / 2; ++m)
                if (m < cnt) o[m] = (2 * (t * cnt + m) + 1 < len) ? ld1<SD>(dp + m) : 0.0f;
        }
    }
    // wavefront-level details: level LOG_E+1+st held by lanes with st+1 low zero bits
    float dw[6];
#pragma unroll
    for (int st = 0; st < 6; ++st) {
        const int lev = LOG_E + 1 + st;
        if constexpr (DEEP) {
            const int lv = lev <= L ? lev : L;           // a level of the transform (> LOG_E)
            const int P = t >> (lv - LOG_E);
            dw[st] = ld1<SD>(det + ceil_shift(n, lv) + (c0 >> lv) + P);
        } else {
            dw[st] = 0.0f;
            if (lev <= L && (lane & ((2 << st) - 1)) == 0) {
                const int P = t >> (st + 1);
                if (2 * P + 1 < (int)ceil_shift(cl, lev - 1))
                    dw[st] = ld1<SD>(det + ceil_shift(n, lev) + (c0 >> lev) + P);
            }
        }
    }

    // DEEP: the values of the cross-wavefront levels (details of levels
    // LOG_E+7..L, then a_L) join the same load phase (clamped indices)
    constexpr int LOG_NW = G::LOG_NW;
    float topv[LOG_NW + 1];
    if constexpr (DEEP) {
#pragma unroll
        for (int k = 0; k < LOG_NW; ++k) {
            const int lev = LOG_E + 7 + k;
            const int lv = lev <= L ? lev : L;
            const int nd = (int)ceil_shift(cl, lv - 1) >> 1;
            const int ti = t < nd ? t : nd - 1;
            topv[k] = ld1<SD>(det + ceil_shift(n, lv) + (c0 >> lv) + ti);
        }
        const int na = (int)ceil_shift(cl, L);
        topv[LOG_NW] = has_top ? top : ld1<SL>(llp + (c0 >> L) + (t < na ? t : na - 1));
    }

    float v = 0.0f;   // a_{min(L, LOG_E+6)} value held by wave-level lanes
    if (L > LOG_E + 6) {
        // top levels across wavefronts: sm[0..NW) values, sm[NW..) details
        float* sa = sm;
        float* sd = sm + NW;
        const int wtop = LOG_E + 6;   // deepest wavefront level
        // details of levels top+1..L, packed level after level
        {
            int off = 0;
            for (int lev = wtop + 1; lev <= L; ++lev) {
                const int len = (int)ceil_shift(cl, lev - 1);
                const int nd = len >> 1;
                if constexpr (DEEP) {
                    float tvk = 0.0f;
#pragma unroll
                    for (int k = 0; k < LOG_NW; ++k)
                        if (lev == wtop + 1 + k) tvk = topv[k];
                    if (t < nd) sd[off + t] = tvk;
                } else {
                    if (t < nd) sd[off + t] = ld1<SD>(det + ceil_shift(n, lev) + (c0 >> lev) + t);
                }
                off += NW;
            }
            const int na = (int)ceil_shift(cl, L);
            if constexpr (DEEP) {
                if (t < na) sa[t] = topv[LOG_NW];
            } else {
                if (t < na) sa[t] = has_top ? top : ld1<SL>(llp + (c0 >> L) + t);
            }
        }
        __syncthreads();
        if (t == 0) {
            for (int lev = L; lev >= wtop + 1; --lev) {
                const int len = (int)ceil_shift(cl, lev - 1);
                const float* dd = sd + (lev - wtop - 1) * NW;
                for (int P = ((len + 1) >> 1) - 1; P >= 0; --P) {
                    const float a = sa[P];
                    if (2 * P + 1 < len) {
                        const float d = dd[P];
                        sa[2 * P] = (a - d) * kRs2Hi;
                        sa[2 * P + 1] = (a + d) * kRs2Hi;
                    } else {
                        sa[2 * P] = a;
                    }
                }
            }
        }
        __syncthreads();
        if (lane == 0 && wv < (int)ceil_shift(cl, wtop)) v = sa[wv];
    } else if (DEEP) {
        v = has_top ? top : ld1<SL>(llp + (c0 >> L) + (t >> (L - LOG_E)));
    } else if (L > LOG_E) {
        const int st = L - LOG_E;
        const int P = t >> st;
        if ((lane & ((1 << st) - 1)) == 0 && P < ceil_shift(cl, L))
            v = has_top ? top : ld1<SL>(llp + (c0 >> L) + P);
    }

    // ---- wavefront levels, from the deepest down
#pragma unroll
    for (int st = 5; st >= 0; --st) {
        const int lev = LOG_E + 1 + st;
        if (lev > L) continue;
        const int off = 1 << st;
        const bool active = (lane & ((off << 1) - 1)) == 0;
        const int P = t >> (st + 1);
        const int len = (int)ceil_shift(cl, lev - 1);
        float e0 = v, e1 = 0.0f;
        if (active && 2 * P + 1 < len) {
            e0 = (v - dw[st]) * kRs2Hi;
            e1 = (v + dw[st]) * kRs2Hi;
        }
        const float got = __shfl_xor(e1, off);
        if (active)
            v = e0;
        else if ((lane & ((off << 1) - 1)) == off)
            v = got;
    }

    // ---- in-thread levels
    float a[E];
    if (L > LOG_E) {
        a[0] = v;
    } else if constexpr (FULL) {
        ld_approx<SL, E, 1>(a, L, llp + (c0 >> L), t);
    } else {
        const int cnt = E >> L;
        const int lenL = (int)ceil_shift(cl, L);
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (m < cnt) a[m] = (t * cnt + m < lenL) ? ld1<SL>(llp + (c0 >> L) + t * cnt + m) : 0.0f;
    }
#pragma unroll
    for (int lev = LOG_E; lev >= 1; --lev) {
        if (lev > L) continue;
        const int cnt = E >> lev;
        const int len = (int)ceil_shift(cl, lev - 1);
        const float* d = dl + (E - (E >> (lev - 1)));
#pragma unroll
        for (int m = E / 2 - 1; m >= 0; --m) {
            if (m >= cnt) continue;
            const float am = a[m];
            const int P = t * cnt + m;
            if (FULL || 2 * P + 1 < len) {
                a[2 * m] = (am - d[m]) * kRs2Hi;
                a[2 * m + 1] = (am + d[m]) * kRs2Hi;
            } else {
                a[2 * m] = am;
                a[2 * m + 1] = 0.0f;
            }
        }
    }
    if constexpr (FULL) {
        st_chunk_lanes<SX, E>(dst, stage, a, lane, wv);
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (t * E + e < cl) st1<SX>(dst + t * E + e, a[e]);
    }
}

// ---------------------------------------------------------------------------
// Deep transforms without scratch
// ---------------------------------------------------------------------------
constexpr int kFinishMax = 1024;   // deepest approximations one work-group finishes on chip

// Analysis, second stage: the first stage left the level-`lc` approximations
// of a length-n signal either in FP32 at src32 or, when src32 is null, in
// y[0, n_lc) (the prefix the deeper levels overwrite).  One work-group
// computes levels lc+1..L in LDS (n_lc <= kFinishMax) with unnormalised
// compensated sums as in the chunks, writing into the prefix of y.
template <class S>
__device__ void finish1d(typename S::raw* y, const float* src32, int64_t n, int lc, int L, df* buf0,
                         df* buf1) {
    const int t = threadIdx.x;
    const int64_t m = ceil_shift(n, lc);
    const int lr = L - lc;
    for (int64_t i = t; i < m; i += blockDim.x) buf0[i] = df_from(src32 ? src32[i] : ld1<S>(y + i));
    __syncthreads();
    df* a = buf0;
    df* b = buf1;
    int64_t len = m;
    for (int lev = 1; lev <= lr; ++lev) {
        const int64_t half = len >> 1, na = len - half;   // na = offset of this level's details
        for (int64_t P = t; P < na; P += blockDim.x) {
            if (P < half) {
                st1<S>(y + na + P, f_norm(df_diff(a[2 * P + 1], a[2 * P]), lev));
                b[P] = df_add(a[2 * P], a[2 * P + 1]);
            } else {
                b[P] = df_s2(a[2 * P]);             // carried sample
            }
        }
        __syncthreads();
        df* tmp = a;
        a = b;
        b = tmp;
        len = na;
    }
    for (int64_t P = t; P < len; P += blockDim.x) st1<S>(y + P, df_norm(a[P], lr));
}

// Synthesis: the level-lc approximation with index c of a length-n signal
// transformed to L levels, from a_L down its ancestor path (one synthesis
// butterfly per level; the odd-count carry passes values unchanged).  All
// loads are issued before the arithmetic.  L - lc <= kMaxWalk.
constexpr int kMaxWalk = 24;
template <class S>
__device__ __forceinline__ float walk_down(const typename S::raw* y, int64_t n, int L, int lc,
                                           int64_t c) {
    float dv[kMaxWalk];
#pragma unroll
    for (int q = 0; q < kMaxWalk; ++q) {
        const int j = L - q;                      // detail level
        dv[q] = 0.0f;
        if (j > lc) {
            const int64_t P = c >> (j - lc);
            if (2 * P + 1 < ceil_shift(n, j - 1)) dv[q] = ld1<S>(y + ceil_shift(n, j) + P);
        }
    }
    float a = ld1<S>(y + (c >> (L - lc)));
#pragma unroll
    for (int q = 0; q < kMaxWalk; ++q) {
        const int j = L - q;
        if (j > lc) {
            const int64_t k = c >> (j - 1 - lc);  // index at level j-1
            if (2 * (k >> 1) + 1 < ceil_shift(n, j - 1))
                a = (k & 1) ? (a + dv[q]) * kRs2Hi : (a - dv[q]) * kRs2Hi;
        }
    }
    return a;
}

}  // namespace haar
