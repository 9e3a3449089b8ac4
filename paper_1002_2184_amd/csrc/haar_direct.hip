// The direct ("original") two-channel filter bank of Fig. 1 / Fig. 2 and
// Fig. 5 / Eq. (13), on the GPU, for comparison with the fast bank.
//
// Analysis level (input a_{j-1} of m samples):
//   filter    y0[k] = b0[0] x[k] + b0[1] x[k-1],  y1[k] = b1[0] x[k] + b1[1] x[k-1]
//             for every k (full rate; x[-1] = 0), taps of Eq. (8)-(9);
//   decimate  a_j[i] = y0[2i+1], d_j[i] = y1[2i+1] (pairs aligned at even
//             indices keep the odd phase); an odd m carries x[m-1] unscaled.
// Synthesis level (Eq. (13), taps of Eq. (17)-(18)):
//   up-sample u0[2i] = a_j[i], u1[2i] = d_j[i], zeros in between;
//   filter    x[k] = a0[0] u0[k] + a0[1] u0[k-1] + a1[0] u1[k] + a1[1] u1[k-1];
//             an odd m carries a_j[last] unscaled.
// Each stage is its own pass and its full-rate streams live in the
// workspace: that is the dataflow of the direct structure, whose cost the
// fast bank (Sec. III-IV) avoids by computing only the decimated outputs.
// (Fused into one kernel, the discarded phase would be dead code and the
// compiler would perform the polyphase reduction itself.)
//
// Precision: the low-pass stream y0 and the approximations passed between
// levels are compensated FP32 pairs (hi, lo), as on the fast path: rounding
// them to FP32 at every level costs about sqrt(L) ulps of the deepest
// approximation, which grows like 2^(L/2) times the signal's mean.
#include "haar_device.h"
#include "haar_internal.h"

namespace haar {

// synthesis taps, FP32 (1/sqrt2 rounded once)
__device__ __forceinline__ float tap_s() { return kRs2Hi; }

// full-rate analysis filtering of m samples per item, one output per thread
// (consecutive lanes, consecutive samples).  Input: storage SI (level 1) or
// a compensated pair buffer (DF, 2 floats per sample); y0 is written as
// pairs (2 floats per sample), y1 as floats.
template <class SI, bool DF>
__global__ __launch_bounds__(256) void direct_filter_kernel(const void* inv, int64_t in_bs, float* y0,
                                                            float* y1, int64_t m, int64_t batch) {
    const int64_t total = m * batch;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t item = g / m, k = g - item * m;
        auto load = [&](int64_t q) -> df {
            if constexpr (DF) {
                const float* p = reinterpret_cast<const float*>(inv) + (item * in_bs + q) * 2;
                return df{p[0], p[1]};
            } else {
                return df_from(ld1<SI>(reinterpret_cast<const typename SI::raw*>(inv) + item * in_bs + q));
            }
        };
        const df cur = load(k);
        const df prev = k > 0 ? load(k - 1) : df{0.0f, 0.0f};
        const df lo = df_rs2(df_add(cur, prev));                       // b0 = [1, 1] / sqrt2
        y0[(item * m + k) * 2] = lo.hi;
        y0[(item * m + k) * 2 + 1] = lo.lo;
        y1[item * m + k] = df_round(df_rs2(df_from(df_diff(cur, prev))));   // b1 = [1, -1] / sqrt2
    }
}

// decimation: keep the odd phase; a_j (pairs) to `aout` (a pair buffer, or
// the final storage when FINAL), d_j to `dout` (stride dout_bs, offset to
// the band); an odd m carries x[m-1] (level input) unscaled
template <class SI, bool DFIN, class SA, bool FINAL, class SD>
__global__ __launch_bounds__(256) void direct_decimate_kernel(const float* y0, const float* y1,
                                                              const void* inv, int64_t in_bs, void* aoutv,
                                                              int64_t aout_bs, typename SD::raw* dout,
                                                              int64_t dout_bs, int64_t m, int64_t batch) {
    const int64_t pairs = m / 2, na = m - pairs;
    const int64_t total = na * batch;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t item = g / na, i = g - item * na;
        df a;
        if (i < pairs) {
            const int64_t k = 2 * i + 1;
            a = df{y0[(item * m + k) * 2], y0[(item * m + k) * 2 + 1]};
            st1<SD>(dout + item * dout_bs + i, y1[item * m + k]);
        } else if constexpr (DFIN) {
            const float* p = reinterpret_cast<const float*>(inv) + (item * in_bs + m - 1) * 2;
            a = df{p[0], p[1]};
        } else {
            a = df_from(ld1<SI>(reinterpret_cast<const typename SI::raw*>(inv) + item * in_bs + m - 1));
        }
        if constexpr (FINAL) {
            st1<SA>(reinterpret_cast<typename SA::raw*>(aoutv) + item * aout_bs + i, df_round(a));
        } else {
            float* p = reinterpret_cast<float*>(aoutv) + (item * aout_bs + i) * 2;
            p[0] = a.hi;
            p[1] = a.lo;
        }
    }
}

// up-sampling of both channels to the full rate (zeros inserted)
template <class SA, class SD>
__global__ __launch_bounds__(256) void direct_upsample_kernel(const typename SA::raw* a, int64_t a_bs,
                                                              const typename SD::raw* d, int64_t d_bs,
                                                              float* u0, float* u1, int64_t m,
                                                              int64_t batch) {
    const int64_t len = 2 * (m / 2);
    const int64_t total = len * batch;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t item = g / len, k = g - item * len;
        const bool even = (k & 1) == 0;
        u0[item * m + k] = even ? ld1<SA>(a + item * a_bs + k / 2) : 0.0f;
        u1[item * m + k] = even ? ld1<SD>(d + item * d_bs + k / 2) : 0.0f;
    }
}

// synthesis filtering and channel sum; an odd m carries a[last] unscaled
template <class SA, class SO>
__global__ __launch_bounds__(256) void direct_synth_filter_kernel(const float* u0, const float* u1,
                                                                  const typename SA::raw* a, int64_t a_bs,
                                                                  typename SO::raw* out, int64_t out_bs,
                                                                  int64_t m, int64_t batch) {
    const int64_t len = 2 * (m / 2);
    const int64_t total = m * batch;
    const float s = tap_s();
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t item = g / m, k = g - item * m;
        float v;
        if (k < len) {
            const float c0 = u0[item * m + k], c1 = u1[item * m + k];
            const float p0 = k > 0 ? u0[item * m + k - 1] : 0.0f;
            const float p1 = k > 0 ? u1[item * m + k - 1] : 0.0f;
            v = (s * c0 + s * p0) + (-s * c1 + s * p1);   // a0 = [s, s], a1 = [-s, s]
        } else {
            v = ld1<SA>(a + item * a_bs + m / 2);
        }
        st1<SO>(out + item * out_bs + k, v);
    }
}

static unsigned grid_of(int64_t work) {
    const int64_t g = (work + 255) / 256;
    return (unsigned)(g < (1 << 20) ? (g > 0 ? g : 1) : (1 << 20));
}

// Workspace (floats): y0 as pairs (2 * batch * n), y1 (batch * n) and two
// approximation buffers of pairs (2 * batch * ceil(n / 2) each).  The
// synthesis uses the first 2 * batch * n floats for u0 / u1 and plain FP32
// approximations in the same two buffers.
size_t direct_workspace_floats(int64_t n, int64_t batch) {
    return (size_t)(3 * batch * n + 4 * batch * ((n + 1) / 2));
}

template <class S>
static hipError_t direct_fwd(const void* xv, void* yv, int64_t n, int L, int64_t batch, float* ws,
                             hipStream_t s) {
    using R = typename S::raw;
    const R* x = (const R*)xv;
    R* y = (R*)yv;
    float* y0 = ws;                                        // pairs
    float* y1 = ws + 2 * batch * n;
    const int64_t half = (n + 1) / 2;
    float* abuf[2] = {ws + 3 * batch * n, ws + 3 * batch * n + 2 * batch * half};   // pairs
    int64_t m = n;
    for (int j = 1; j <= L; ++j) {
        const int64_t nj = m - m / 2;
        const unsigned gf = grid_of(m * batch), gd = grid_of(nj * batch);
        const void* ain = j == 1 ? (const void*)x : (const void*)abuf[j & 1];
        const int64_t ain_bs = j == 1 ? n : half;
        if (j == 1)
            hipLaunchKernelGGL((direct_filter_kernel<S, false>), dim3(gf), dim3(256), 0, s, ain, ain_bs, y0, y1,
                               m, batch);
        else
            hipLaunchKernelGGL((direct_filter_kernel<S, true>), dim3(gf), dim3(256), 0, s, ain, ain_bs, y0, y1,
                               m, batch);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        R* dout = y + nj;                                  // d_j = y[n_j, n_{j-1})
        void* aout = j == L ? (void*)y : (void*)abuf[(j + 1) & 1];
        const int64_t aout_bs = j == L ? n : half;
        if (j == 1 && j == L)
            hipLaunchKernelGGL((direct_decimate_kernel<S, false, S, true, S>), dim3(gd), dim3(256), 0, s, y0,
                               y1, ain, ain_bs, aout, aout_bs, dout, n, m, batch);
        else if (j == 1)
            hipLaunchKernelGGL((direct_decimate_kernel<S, false, S, false, S>), dim3(gd), dim3(256), 0, s, y0,
                               y1, ain, ain_bs, aout, aout_bs, dout, n, m, batch);
        else if (j == L)
            hipLaunchKernelGGL((direct_decimate_kernel<S, true, S, true, S>), dim3(gd), dim3(256), 0, s, y0,
                               y1, ain, ain_bs, aout, aout_bs, dout, n, m, batch);
        else
            hipLaunchKernelGGL((direct_decimate_kernel<S, true, S, false, S>), dim3(gd), dim3(256), 0, s, y0,
                               y1, ain, ain_bs, aout, aout_bs, dout, n, m, batch);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        m = nj;
    }
    return hipSuccess;
}

template <class S>
static hipError_t direct_inv(const void* yv, void* xv, int64_t n, int L, int64_t batch, float* ws,
                             hipStream_t s) {
    using R = typename S::raw;
    const R* y = (const R*)yv;
    R* x = (R*)xv;
    float* u0 = ws;
    float* u1 = ws + batch * n;
    const int64_t half = (n + 1) / 2;
    float* abuf[2] = {ws + 2 * batch * n, ws + 2 * batch * n + batch * half};
    int64_t len[64];
    len[0] = n;
    for (int j = 1; j <= L; ++j) len[j] = len[j - 1] - len[j - 1] / 2;
    for (int j = L; j >= 1; --j) {
        const int64_t m = len[j - 1], nj = len[j];
        const R* d = y + nj;                               // d_j
        const bool first = j == L;                         // a_L comes from y's prefix
        const float* ain = abuf[j & 1];
        if (first)
            hipLaunchKernelGGL((direct_upsample_kernel<S, S>), dim3(grid_of(m * batch)), dim3(256), 0, s, y, n,
                               d, n, u0, u1, m, batch);
        else
            hipLaunchKernelGGL((direct_upsample_kernel<StF32, S>), dim3(grid_of(m * batch)), dim3(256), 0, s,
                               ain, half, d, n, u0, u1, m, batch);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const bool last = j == 1;                          // level 1 writes the output
        if (first && last)
            hipLaunchKernelGGL((direct_synth_filter_kernel<S, S>), dim3(grid_of(m * batch)), dim3(256), 0, s,
                               u0, u1, y, n, x, n, m, batch);
        else if (first)
            hipLaunchKernelGGL((direct_synth_filter_kernel<S, StF32>), dim3(grid_of(m * batch)), dim3(256), 0,
                               s, u0, u1, y, n, abuf[(j + 1) & 1], half, m, batch);
        else if (last)
            hipLaunchKernelGGL((direct_synth_filter_kernel<StF32, S>), dim3(grid_of(m * batch)), dim3(256), 0,
                               s, u0, u1, ain, half, x, n, m, batch);
        else
            hipLaunchKernelGGL((direct_synth_filter_kernel<StF32, StF32>), dim3(grid_of(m * batch)), dim3(256),
                               0, s, u0, u1, ain, half, abuf[(j + 1) & 1], half, m, batch);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int run_direct_1d(const void* in, void* out, int64_t n, int L, int64_t batch, int dtype, bool inverse,
                  float* ws, hipStream_t s) {
    hipError_t e;
    switch (dtype) {
        case 0: e = inverse ? direct_inv<StF32>(in, out, n, L, batch, ws, s) : direct_fwd<StF32>(in, out, n, L, batch, ws, s); break;
        case 1: e = inverse ? direct_inv<StBF16>(in, out, n, L, batch, ws, s) : direct_fwd<StBF16>(in, out, n, L, batch, ws, s); break;
        default: e = inverse ? direct_inv<StF16>(in, out, n, L, batch, ws, s) : direct_fwd<StF16>(in, out, n, L, batch, ws, s); break;
    }
    return e == hipSuccess ? 0 : hip_error(e, "direct-structure launch");
}

}  // namespace haar
