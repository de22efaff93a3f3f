// Line transforms of power-of-two length in LDS, shared by the x/y passes
// and the fused Poisson passes.
//
// DCT-II of a real line x of length L = 2M (Makhoul's reordering):
//   v[m] = x[2m] (m < M), v[m] = x[2L-1-2m] (m >= M),  V = DFT_L(v),
//   X[k] = Re(e^{-i pi k / (2L)} V[k]),  X[L-k] = -Im(e^{-i pi k / (2L)} V[k]).
// V comes from one complex DFT of length M of z[n] = v[2n] + i v[2n+1]
// (real-input packing).  DCT-III inverts these steps; the discrete Hartley
// transform H[k] = (Re F[k] - Im F[k]) / sqrt(L) uses the same packed DFT.
//
// The length-M DFT is a four-step M1 x M2 decomposition: M2 threads per line
// each do an M1-point DFT in registers, multiply by twiddles, exchange
// through LDS once, and finish with M1 / M2 DFTs of length M2 each.
// Twiddles come from a per-axis table tw4[j] = e^{-i pi j / (2L)}, j < 4L.
#pragma once

#include "fft_common.h"

namespace otd {

// Four-step DFT of length M = M1 M2 on one line.  Stage-1 input n comes from
// load(n); on return out[q][k2] = Z[k1 + M1 k2] with k1 = t + M2 q.  The
// line's LDS region s (2M floats) is used for the exchange.  All threads of
// the block must call this (it synchronises the block).
template <int M1, int M2, class Load>
__device__ __forceinline__ void fft_core(float* s, int t, const float2* tw4, Load load,
                                         float2 (&out)[M1 / M2][M2]) {
    constexpr int M = M1 * M2, L = 2 * M;
    float2 a[M1];
#pragma unroll
    for (int n1 = 0; n1 < M1; ++n1) a[n1] = load(M2 * n1 + t);
    dft<M1>(a);
#pragma unroll
    for (int k1 = 1; k1 < M1; ++k1) a[k1] = cmul(a[k1], tw4[(8 * t * k1) & (4 * L - 1)]);
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < M1; ++k1) st2(s, k1 * M2 + t, a[k1]);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < M1 / M2; ++q) {
        const int k1 = t + M2 * q;
#pragma unroll
        for (int n2 = 0; n2 < M2; ++n2) out[q][n2] = ld2(s, k1 * M2 + n2);
        dft<M2>(out[q]);
    }
}

// V[k] of the length-L real DFT from the packed Z (k = 0..M).
template <int M>
__device__ __forceinline__ float2 unpack(const float* s, int k, const float2* tw4) {
    const float2 zk = ld2(s, k & (M - 1));
    const float2 zm = ld2(s, (M - k) & (M - 1));
    const float2 ve = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
    const float2 vo = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
    return k < M ? cadd(ve, cmul(tw4[4 * k], vo)) : csub(ve, vo);
}

// Orthonormal DCT-II of the line s[0..L) in place.
template <int M1, int M2>
__device__ void line_dct2(float* s, int t, const float2* tw4) {
    constexpr int M = M1 * M2, L = 2 * M, T = M2, NK = (M + T) / T;
    auto vidx = [](int m) { return m < M ? 2 * m : 2 * L - 1 - 2 * m; };
    float2 z[M1 / M2][M2];
    fft_core<M1, M2>(s, t, tw4, [&](int n) { return make_float2(s[vidx(2 * n)], s[vidx(2 * n + 1)]); }, z);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < M1 / M2; ++q)
#pragma unroll
        for (int k2 = 0; k2 < M2; ++k2) st2(s, t + M2 * q + M1 * k2, z[q][k2]);
    __syncthreads();
    float xr[NK], xi[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const int k = t + T * j;
        if (k <= M) {
            const float2 w = cmul(tw4[k], unpack<M>(s, k, tw4));
            xr[j] = w.x;
            xi[j] = -w.y;
        }
    }
    __syncthreads();
    const float sc = sqrtf(2.f / L), sc0 = sqrtf(1.f / L);
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const int k = t + T * j;
        if (k <= M) {
            s[k] = (k == 0 ? sc0 : sc) * xr[j];
            if (k > 0 && k < M) s[L - k] = sc * xi[j];
        }
    }
    __syncthreads();
}

// Orthonormal DCT-III (inverse of line_dct2) in place.
template <int M1, int M2>
__device__ void line_dct3(float* s, int t, const float2* tw4) {
    constexpr int M = M1 * M2, L = 2 * M, T = M2, NJ = M / T;
    const float isc = 1.f / sqrtf(2.f / L), isc0 = 1.f / sqrtf(1.f / L);
    auto X = [&](int k) -> float { return k >= L ? 0.f : s[k] * (k == 0 ? isc0 : isc); };
    auto V = [&](int k) -> float2 {
        return cmul(cconj(tw4[k]), make_float2(X(k), -X(L - k)));
    };
    float2 zc[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int k = t + T * j;
        const float2 v = V(k), vm = cconj(V(M - k));
        const float2 ve = make_float2(0.5f * (v.x + vm.x), 0.5f * (v.y + vm.y));
        const float2 vo = cmul(make_float2(0.5f * (v.x - vm.x), 0.5f * (v.y - vm.y)),
                               cconj(tw4[4 * k]));
        const float2 zk = make_float2(ve.x - vo.y, ve.y + vo.x);
        zc[j] = cconj(zk);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NJ; ++j) st2(s, t + T * j, zc[j]);
    __syncthreads();
    float2 r[M1 / M2][M2];
    fft_core<M1, M2>(s, t, tw4, [&](int n) { return ld2(s, n); }, r);
    __syncthreads();
    const float im = 1.f / M;
    auto pos = [](int m) { return m < M ? 2 * m : 2 * (L - 1 - m) + 1; };
#pragma unroll
    for (int q = 0; q < M1 / M2; ++q)
#pragma unroll
        for (int k2 = 0; k2 < M2; ++k2) {
            const int n = t + M2 * q + M1 * k2;
            s[pos(2 * n)] = r[q][k2].x * im;
            s[pos(2 * n + 1)] = -r[q][k2].y * im;
        }
    __syncthreads();
}

// Orthonormal discrete Hartley transform (its own inverse) in place.
template <int M1, int M2>
__device__ void line_dht(float* s, int t, const float2* tw4) {
    constexpr int M = M1 * M2, L = 2 * M, T = M2, NK = (M + T) / T;
    float2 z[M1 / M2][M2];
    fft_core<M1, M2>(s, t, tw4, [&](int n) { return ld2(s, n); }, z);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < M1 / M2; ++q)
#pragma unroll
        for (int k2 = 0; k2 < M2; ++k2) st2(s, t + M2 * q + M1 * k2, z[q][k2]);
    __syncthreads();
    float h0[NK], h1[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const int k = t + T * j;
        if (k <= M) {
            const float2 f = unpack<M>(s, k, tw4);
            h0[j] = f.x - f.y;
            h1[j] = f.x + f.y;
        }
    }
    __syncthreads();
    const float sc = sqrtf(1.f / L);
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const int k = t + T * j;
        if (k <= M) {
            s[k] = sc * h0[j];
            if (k > 0 && k < M) s[L - k] = sc * h1[j];
        }
    }
    __syncthreads();
}

template <int M1, int M2, int KIND>
__device__ __forceinline__ void line_xform(float* s, int t, const float2* tw4) {
    if constexpr (KIND == 0) line_dct2<M1, M2>(s, t, tw4);
    else if constexpr (KIND == 1) line_dct3<M1, M2>(s, t, tw4);
    else line_dht<M1, M2>(s, t, tw4);
}

}  // namespace otd
