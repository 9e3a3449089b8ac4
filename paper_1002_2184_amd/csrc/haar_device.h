// Device helpers for the Haar kernels: storage formats and compensated FP32.
//
// Storage types are read into FP32 registers and written back with
// round-to-nearest-even; all arithmetic is FP32.  The approximation path of
// the analysis bank carries an unevaluated pair (hi + lo) so that the sums of
// the polyphase components (Eq. (11)) are kept to about 48 bits across the
// fused levels and rounded once at the end.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace haar {

constexpr double kRsqrt2 = 0.70710678118654752440084436210485;   // b00 = a00
constexpr double kSqrt2 = 1.4142135623730950488016887242097;
constexpr float kRs2Hi = (float)kRsqrt2;
constexpr float kRs2Lo = (float)(kRsqrt2 - (double)(float)kRsqrt2);
constexpr float kS2Hi = (float)kSqrt2;
constexpr float kS2Lo = (float)(kSqrt2 - (double)(float)kSqrt2);

// ---------------------------------------------------------------------------
// Pair arithmetic (Knuth's TwoSum, Dekker's FastTwoSum, FMA product error).
// ---------------------------------------------------------------------------
struct df {
    float hi, lo;
};

__device__ __forceinline__ df two_sum(float a, float b) {
    const float s = a + b;
    const float bb = s - a;
    const float e = (a - (s - bb)) + (b - bb);
    return {s, e};
}

__device__ __forceinline__ df fast_two_sum(float a, float b) {   // |a| >= |b|
    const float s = a + b;
    return {s, b - (s - a)};
}

__device__ __forceinline__ df df_from(float a) { return {a, 0.0f}; }

__device__ __forceinline__ df df_add(df a, df b) {
    const df s = two_sum(a.hi, b.hi);
    return fast_two_sum(s.hi, s.lo + (a.lo + b.lo));
}

// (a + b + c + d) of four exact floats
__device__ __forceinline__ df df_sum4f(float a, float b, float c, float d) {
    const df s1 = two_sum(a, b);
    const df s2 = two_sum(c, d);
    const df s = two_sum(s1.hi, s2.hi);
    return fast_two_sum(s.hi, s.lo + (s1.lo + s2.lo));
}

__device__ __forceinline__ df df_sum4(df a, df b, df c, df d) {
    const df s1 = two_sum(a.hi, b.hi);
    const df s2 = two_sum(c.hi, d.hi);
    const df s = two_sum(s1.hi, s2.hi);
    const float lo = (s.lo + (s1.lo + s2.lo)) + ((a.lo + b.lo) + (c.lo + d.lo));
    return fast_two_sum(s.hi, lo);
}

__device__ __forceinline__ df df_scale(df a, float p2) {   // exact for a power of two
    return {a.hi * p2, a.lo * p2};
}

// a * (c_hi + c_lo)
__device__ __forceinline__ df df_mul(df a, float c_hi, float c_lo) {
    const float p = a.hi * c_hi;
    const float e = __builtin_fmaf(a.hi, c_hi, -p);
    const float lo = e + (a.hi * c_lo + a.lo * c_hi);
    return fast_two_sum(p, lo);
}

__device__ __forceinline__ df df_rs2(df a) { return df_mul(a, kRs2Hi, kRs2Lo); }
__device__ __forceinline__ df df_s2(df a) { return df_mul(a, kS2Hi, kS2Lo); }

__device__ __forceinline__ float df_round(df a) { return a.hi + a.lo; }

// b - a, rounded once (both pairs)
__device__ __forceinline__ float df_diff(df b, df a) {
    return (b.hi - a.hi) + (b.lo - a.lo);
}

// 2^(-j/2) as a pair (exact power of two for even j)
__device__ __forceinline__ df pow2_half_neg(int j, float& p2) {
    p2 = __builtin_ldexpf(1.0f, -(j >> 1));
    if (j & 1) return {kRs2Hi * p2, kRs2Lo * p2};
    return {p2, 0.0f};
}

// S * 2^(-j/2) rounded once: the normalised approximation from a sum of
// 2^j samples.
__device__ __forceinline__ float df_norm(df s, int j) {
    const float p2 = __builtin_ldexpf(1.0f, -(j >> 1));
    if (j & 1) return df_round(df_mul(df_scale(s, p2), kRs2Hi, kRs2Lo));
    return df_round(df_scale(s, p2));
}

// single float times 2^(-j/2)
__device__ __forceinline__ float f_norm(float d, int j) {
    const float p2 = __builtin_ldexpf(1.0f, -(j >> 1));
    return (j & 1) ? (d * p2) * kRs2Hi : d * p2;
}

// ---------------------------------------------------------------------------
// Storage formats.
// ---------------------------------------------------------------------------
// FP32 -> BF16 with round-to-nearest-even: gfx950's packed conversion
// instruction (v_cvt_pk_bf16_f32) rounds two values at once; NaN stays NaN.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t f32x2_to_bf16x2(float a, float b) {
    const f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}

struct StF32 {
    static constexpr bool kStream = true;   // HBM, addressed through global pointers
    static constexpr bool kNT = true;       // outputs written with streaming stores
    static constexpr int kPace = -1;        // stores not paced (see Paced)
    using raw = float;
    static constexpr int kBytes = 4;
    __device__ __forceinline__ static float ld(raw v) { return v; }
    __device__ __forceinline__ static raw st(float f) { return f; }
};

struct StBF16 {
    static constexpr bool kStream = true;   // HBM, addressed through global pointers
    static constexpr bool kNT = true;       // outputs written with streaming stores
    static constexpr int kPace = -1;        // stores not paced (see Paced)
    using raw = uint16_t;
    static constexpr int kBytes = 2;
    __device__ __forceinline__ static float ld(raw v) { return __uint_as_float((uint32_t)v << 16); }
    __device__ __forceinline__ static raw st(float f) { return f32_to_bf16(f); }
    __device__ __forceinline__ static uint32_t st2(float a, float b) { return f32x2_to_bf16x2(a, b); }
};

// FP32 coefficients of one tile or chunk held on chip (a packed buffer in
// LDS, addressed through generic pointers): ordinary stores.
struct StLds {
    static constexpr bool kStream = false;
    static constexpr bool kNT = false;
    static constexpr int kPace = -1;
    using raw = float;
    static constexpr int kBytes = 4;
    __device__ __forceinline__ static float ld(raw v) { return v; }
    __device__ __forceinline__ static raw st(float f) { return f; }
};

struct StF16 {
    static constexpr bool kStream = true;   // HBM, addressed through global pointers
    static constexpr bool kNT = true;       // outputs written with streaming stores
    static constexpr int kPace = -1;        // stores not paced (see Paced)
    using raw = uint16_t;
    static constexpr int kBytes = 2;
    __device__ __forceinline__ static float ld(raw v) {
        return (float)__builtin_bit_cast(_Float16, v);
    }
    __device__ __forceinline__ static raw st(float f) {
        return __builtin_bit_cast(uint16_t, (_Float16)f);
    }
    __device__ __forceinline__ static uint32_t st2(float a, float b) {
        return (uint32_t)st(a) | ((uint32_t)st(b) << 16);
    }
};

// Outputs are written with nontemporal (streaming) stores: every output
// element is written once and not read again by the kernel, and streaming
// stores avoid allocating the lines in the caches on the way to HBM.
// Inputs use ordinary loads unless HAAR_NT_LOADS is set.
#ifndef HAAR_NT_LOADS
#define HAAR_NT_LOADS 0
#endif

// Vector accesses assume only the alignment of the element type: rows and
// band origins of arbitrary sizes start at any element.  On gfx9 and later
// under ROCm the memory system runs in unaligned-access mode, so these stay
// single 8- or 16-byte instructions whatever the address (a misaligned one
// touches one more cache line).
typedef float v4f __attribute__((ext_vector_type(4), aligned(4)));
typedef float v2f __attribute__((ext_vector_type(2), aligned(4)));
typedef unsigned int v4u __attribute__((ext_vector_type(4), aligned(2)));
typedef unsigned int v2u __attribute__((ext_vector_type(2), aligned(2)));
typedef unsigned int u32e __attribute__((aligned(2)));

// Storage traits that address HBM (kStream) access it through global
// address-space pointers.  A pointer read from a work list (the plans) is
// otherwise generic, and generic (flat) instructions count against both the
// vector-memory and the LDS wait counters.  The LDS trait (StLds) keeps
// generic pointers.
#define HAAR_GLOBAL __attribute__((address_space(1)))

// NT: a nontemporal load, for data that is read once and shares no cache
// line with another work-group's reads.
template <class S, class T, bool NT = false>
__device__ __forceinline__ T ld_s(const T* p) {
    if constexpr (S::kStream) {
        const HAAR_GLOBAL T* g = (const HAAR_GLOBAL T*)p;
        if constexpr (NT || HAAR_NT_LOADS)
            return __builtin_nontemporal_load(g);
        else
            return *g;
    } else {
        return *p;
    }
}

// Load N consecutive elements (N * kBytes in {2, 4, 8, 16}; the pointer
// needs only element alignment) into floats.
template <class S, int N, bool NT = false>
__device__ __forceinline__ void ld_vec(const typename S::raw* p, float* out) {
    constexpr int B = N * S::kBytes;
    static_assert(B == 2 || B == 4 || B == 8 || B == 16, "vector width");
    if constexpr (S::kBytes == 4) {
        if constexpr (N == 4) {
            const v4f v = ld_s<S, v4f, NT>(reinterpret_cast<const v4f*>(p));
            out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
        } else if constexpr (N == 2) {
            const v2f v = ld_s<S, v2f, NT>(reinterpret_cast<const v2f*>(p));
            out[0] = v.x; out[1] = v.y;
        } else {
            out[0] = ld_s<S, float, NT>(reinterpret_cast<const float*>(p));
        }
    } else {
        uint32_t w[B >= 4 ? B / 4 : 1];
        if constexpr (B == 16) {
            const v4u v = ld_s<S, v4u, NT>(reinterpret_cast<const v4u*>(p));
            w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
        } else if constexpr (B == 8) {
            const v2u v = ld_s<S, v2u, NT>(reinterpret_cast<const v2u*>(p));
            w[0] = v.x; w[1] = v.y;
        } else if constexpr (B == 4) {
            w[0] = ld_s<S, u32e, NT>(reinterpret_cast<const u32e*>(p));
        } else {
            out[0] = S::ld(ld_s<S, typename S::raw, NT>(p));
            return;
        }
#pragma unroll
        for (int i = 0; i < N / 2; ++i) {
            out[2 * i] = S::ld((uint16_t)(w[i] & 0xffffu));
            out[2 * i + 1] = S::ld((uint16_t)(w[i] >> 16));
        }
    }
}

template <class S, class T>
__device__ __forceinline__ void st_s(T v, T* p) {
    // s_waitcnt vmcnt(kPace), the other counters left alone (gfx9 encoding:
    // vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8)
    if constexpr (S::kStream && S::kPace >= 0) __builtin_amdgcn_s_waitcnt(0x0F70 | S::kPace);
    if constexpr (S::kStream && S::kNT)
        __builtin_nontemporal_store(v, (HAAR_GLOBAL T*)p);
    else if constexpr (S::kStream)
        *(HAAR_GLOBAL T*)p = v;
    else
        *p = v;
}

// The same storage format written with ordinary (write-back) stores.  When
// rows do not start on cache-line boundaries, the first and last line of
// every row piece of a tile is shared with the neighbouring tile; written
// back through the L2 that both tiles use, the two halves merge there, where
// two streaming partial-line writes would each go to HBM.
template <class S>
struct WriteBack : S {
    static constexpr bool kNT = false;
};

// The same storage format with paced stores: before each store the
// wavefront waits until at most K of its vector-memory operations are still
// outstanding, so that a wavefront never has more than about K + 1 stores in
// flight.  The 16-bit 2D kernels issue many narrow band stores (8 bytes and
// less per lane); left unpaced they queue up in the write path and the whole
// launch runs slower (4096 x 4096 BF16 L5: analysis 13.6-13.7 us unpaced,
// 12.6-12.7 us with K = 2; synthesis 14.8-15.0 us unpaced, 13.8-13.9 us with
// K = 0).  FP32 kernels and the plan kernels ran slower paced.
template <class S, int K>
struct Paced : S {
    static_assert(K >= 0 && K < 16, "vmcnt field");
    static constexpr int kPace = K;
};

template <class S, int N>
__device__ __forceinline__ void st_vec(typename S::raw* p, const float* v) {
    constexpr int B = N * S::kBytes;
    static_assert(B == 2 || B == 4 || B == 8 || B == 16, "vector width");
    if constexpr (S::kBytes == 4) {
        if constexpr (N == 4) {
            v4f o = {v[0], v[1], v[2], v[3]};
            st_s<S>(o, reinterpret_cast<v4f*>(p));
        } else if constexpr (N == 2) {
            v2f o = {v[0], v[1]};
            st_s<S>(o, reinterpret_cast<v2f*>(p));
        } else {
            st_s<S>(v[0], reinterpret_cast<float*>(p));
        }
    } else {
        if constexpr (B == 2) {
            st_s<S>(S::st(v[0]), p);
        } else {
            uint32_t w[B / 4];
#pragma unroll
            for (int i = 0; i < N / 2; ++i)
                w[i] = S::st2(v[2 * i], v[2 * i + 1]);
            if constexpr (B == 16) {
                v4u o = {w[0], w[1], w[2], w[3]};
                st_s<S>(o, reinterpret_cast<v4u*>(p));
            } else if constexpr (B == 8) {
                v2u o = {w[0], w[1]};
                st_s<S>(o, reinterpret_cast<v2u*>(p));
            } else {
                st_s<S>((u32e)w[0], reinterpret_cast<u32e*>(p));
            }
        }
    }
}

template <class S>
__device__ __forceinline__ void st1(typename S::raw* p, float v) { st_s<S>(S::st(v), p); }

// Ordinary (write-back) store of one element.  Used for the short row pieces
// of the deepest 2D levels: these cover only part of a cache line each, and
// partial lines cost less through the caches than streamed.
template <class S>
__device__ __forceinline__ void st1_cached(typename S::raw* p, float v) {
    if constexpr (S::kStream)
        *(HAAR_GLOBAL typename S::raw*)p = S::st(v);
    else
        *p = S::st(v);
}

template <class S>
__device__ __forceinline__ float ld1(const typename S::raw* p) { return S::ld(ld_s<S>(p)); }

// ceil(n / 2^j)
__device__ __forceinline__ int64_t ceil_shift(int64_t n, int j) {
    return (n + ((int64_t)1 << j) - 1) >> j;
}

// Map a block index to a tile index so that the tiles handled by one XCD
// (blocks are dealt round-robin to the 8 XCDs) form one contiguous range:
// neighbouring tiles then share that XCD's L2 for the partial cache lines of
// their small deep-level band segments.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t total) {
    const int64_t q = total >> 3, r = total & 7;
    const int64_t x = b & 7, i = b >> 3;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

}  // namespace haar
