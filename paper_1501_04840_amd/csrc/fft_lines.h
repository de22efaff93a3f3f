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
//
// Real-input packing relates the frequencies k and M - k: with
// 2 ve = Z[k] + conj Z[M-k] and 2 vo = -i (Z[k] - conj Z[M-k]),
//   V[k] = ve + w vo,  V[M-k] = conj(ve - w vo),  w = e^{-2 pi i k / L},
// so every thread takes such pairs together (one product serves both, and
// each packed value is read once).  LDS accesses are written as a per-thread
// base pointer plus a compile-time offset, which the hardware encodes in the
// instruction instead of computing an address per access.
#pragma once

#include "fft_common.h"

namespace otd {

// Orders the LDS accesses of the threads of one line.  Every access of a
// power-of-two line transform stays in its line's region, and a line's M2
// threads are consecutive lanes of one wave (M2 divides 64), whose LDS
// instructions the hardware executes in order: a compiler barrier with
// wavefront-scope fences is enough, so the waves of a block do not wait for
// each other inside a transform (each transform still ends with a block
// barrier, after which other lines' data may be read).
__device__ __forceinline__ void line_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Four-step DFT of length M = M1 M2 on one line.  Stage-1 input n = M2 n1 + t
// comes from load(n1) (the caller knows t); on return out[q][k2] =
// Z[k1 + M1 k2] with k1 = t + M2 q.  The line's LDS region s is used for the
// exchange: M1 rows of M2 complex values, each row followed by XP padding
// floats (M1 (2 M2 + XP) floats; XP even).  All threads of the block must
// call this (it synchronises the block); threads with `act` false only take
// part in the synchronisation (their s and out are not touched).
template <int M1, int M2, int XP = 0, class Load>
__device__ __forceinline__ void fft_core(float* s, int t, const float2* tw4, Load load,
                                         float2 (&out)[M1 / M2][M2], bool act = true) {
    constexpr int M = M1 * M2, L = 2 * M, RW = M2 + XP / 2;   // exchange row, complex units
    static_assert(XP % 2 == 0, "exchange padding in whole complex values");
    static_assert(M1 == fft_m1(L) && M1 % 2 == 0, "the split the host's twiddle table is laid out for");
    static_assert(64 % M2 == 0, "a line's threads within one wave (line_sync)");
    float2 a[M1];
    if (act) {
        // this thread's first-stage twiddles, contiguous (16-byte aligned:
        // the table is, and 4 L and t M1 are even), two to a load
        const float4* const tw1 = reinterpret_cast<const float4*>(tw4 + 4 * L + t * M1);
        float4 w[M1 / 2];
#pragma unroll
        for (int i = 0; i < M1 / 2; ++i) w[i] = tw1[i];
#pragma unroll
        for (int n1 = 0; n1 < M1; ++n1) a[n1] = load(n1);
        dft<M1>(a);
#pragma unroll
        for (int k1 = 1; k1 < M1; ++k1)
            a[k1] = cmul(a[k1], k1 & 1 ? make_float2(w[k1 / 2].z, w[k1 / 2].w)
                                       : make_float2(w[k1 / 2].x, w[k1 / 2].y));
    }
    line_sync();
    if (act) {
        float* const sw = s + 2 * t;                  // Z1[k1][t]
#pragma unroll
        for (int k1 = 0; k1 < M1; ++k1) st2(sw, k1 * RW, a[k1]);
    }
    line_sync();
    if (act) {
        const float* const sr = s + 2 * RW * t;       // Z1[t + M2 q][n2]
#pragma unroll
        for (int q = 0; q < M1 / M2; ++q) {
#pragma unroll
            for (int n2 = 0; n2 < M2; ++n2) out[q][n2] = ld2(sr, RW * M2 * q + n2);
            dft<M2>(out[q]);
        }
    }
}

// Stores the stage-2 output out[q][k2] = Z[t + M2 q + M1 k2] to s[2 Z index].
template <int M1, int M2>
__device__ __forceinline__ void store_z(float* s, int t, const float2 (&z)[M1 / M2][M2]) {
    float* const sw = s + 2 * t;
#pragma unroll
    for (int q = 0; q < M1 / M2; ++q)
#pragma unroll
        for (int k2 = 0; k2 < M2; ++k2) st2(sw, M2 * q + M1 * k2, z[q][k2]);
}

// Z[k] and Z[M - k] for k = t + M2 j (j compile-time) from the stored packed
// DFT.  For k = 0 the partner is Z[0] itself.
template <int M, int M2>
__device__ __forceinline__ void load_pair(const float* s, int t, int j, float2& zk, float2& zm) {
    zk = ld2(s + 2 * t, M2 * j);
    if (j == 0) zm = ld2(s, (M - t) & (M - 1));
    else zm = ld2(s - 2 * t, M - M2 * j);
}

// Orthonormal DCT-II of the line s[0..L) in place.  Threads with `act`
// false only take part in the block synchronisation.  The line transforms
// are always inlined, so that s is known to point into LDS and is accessed
// with LDS instructions (32-bit addresses that wrap): s - 4t is below the
// first line's start, which as a 64-bit generic (flat) address would leave
// the LDS aperture.
template <int M1, int M2, int XP = 0>
__device__ __forceinline__ void line_dct2(float* s, int t, const float2* tw4, bool act = true) {
    constexpr int M = M1 * M2, L = 2 * M, T = M2, NP = (M / 2 + T) / T;
    // z[n] = v[2n] + i v[2n+1] with n = M2 n1 + t; v[2n] and v[2n+1] are
    // x[4n], x[4n+2] in the first half (n1 < M1 / 2) and x[2L-1-4n],
    // x[2L-3-4n] in the second.
    const float* const sp = s + 4 * t;
    const float* const sm = s - 4 * t;
    float2 z[M1 / M2][M2];
    fft_core<M1, M2, XP>(s, t, tw4, [&](int n1) {
        return n1 < M1 / 2 ? make_float2(sp[4 * M2 * n1], sp[4 * M2 * n1 + 2])
                           : make_float2(sm[2 * L - 1 - 4 * M2 * n1], sm[2 * L - 3 - 4 * M2 * n1]);
    }, z, act);
    line_sync();
    if (act) store_z<M1, M2>(s, t, z);
    line_sync();
    // 2 V[k] = a and 2 V[M-k] = b; the factor 1/2 is folded into the scales
    const float h = 0.5f * sqrtf(2.f / L), h0 = 0.5f * sqrtf(1.f / L);
    float o[NP][4];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int k = t + T * j;
        if (act && k <= M / 2) {
            float2 zk, zm;
            load_pair<M, T>(s, t, j, zk, zm);
            const float2 ve = make_float2(zk.x + zm.x, zk.y - zm.y);
            const float2 vo = make_float2(zk.y + zm.y, zm.x - zk.x);
            const float2 p = cmul(tw4[4 * k], vo);
            const float2 xa = cmul(tw4[k], cadd(ve, p));
            const float2 xb = cmul(tw4[M - k], make_float2(ve.x - p.x, p.y - ve.y));
            o[j][0] = (k == 0 ? h0 : h) * xa.x;     // X[k]
            o[j][1] = -h * xa.y;                    // X[L-k]
            o[j][2] = h * xb.x;                     // X[M-k]
            o[j][3] = -h * xb.y;                    // X[M+k]
        }
    }
    line_sync();
    float* const op = s + t;
    float* const om = s - t;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int k = t + T * j;
        if (act && k <= M / 2) {
            op[T * j] = o[j][0];
            if (k > 0) om[L - T * j] = o[j][1];
            if (k < M / 2) {
                om[M - T * j] = o[j][2];
                if (k > 0) op[M + T * j] = o[j][3];
            }
        }
    }
    __syncthreads();
}

// Orthonormal DCT-III (inverse of line_dct2) in place.  BLOCK_END false: end
// with a wavefront sync only, for callers that afterwards read nothing but
// the lines of their own wavefront.
template <int M1, int M2, int XP = 0, bool BLOCK_END = true>
__device__ __forceinline__ void line_dct3(float* s, int t, const float2* tw4) {
    constexpr int M = M1 * M2, L = 2 * M, T = M2, NP = (M / 2 + T) / T;
    // inputs scaled by sqrt(L / 2) (sqrt(L) for X[0]); with V(k) =
    // conj(w4_k) (X[k], -X[L-k]), the packed spectrum is
    //   conj Z[k] = conj(ve + i vo),  conj Z[M-k] = ve - i vo,
    //   2 ve = V(k) + conj V(M-k),  2 vo = (V(k) - conj V(M-k)) conj(w_k).
    // The factor sqrt(L / 2) / 2 is applied to the outputs instead.
    const float* const ip = s + t;
    const float* const im_ = s - t;
    float2 zc[NP][2];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int k = t + T * j;
        if (k <= M / 2) {
            const float xk = k == 0 ? 1.41421356237309515f * s[0] : ip[T * j];
            const float xl = j == 0 ? (k == 0 ? 0.f : s[L - t]) : im_[L - T * j];   // X[L-k]
            const float xm = im_[M - T * j];                                         // X[M-k]
            const float xp = ip[M + T * j];                                          // X[M+k]
            const float2 v = cmul(cconj(tw4[k]), make_float2(xk, -xl));
            const float2 w = cmul(cconj(tw4[M - k]), make_float2(xm, -xp));   // V(M-k)
            const float2 ve = make_float2(v.x + w.x, v.y - w.y);
            const float2 vo = cmul(make_float2(v.x - w.x, v.y + w.y), cconj(tw4[4 * k]));
            zc[j][0] = make_float2(ve.x - vo.y, -(ve.y + vo.x));
            zc[j][1] = make_float2(ve.x + vo.y, ve.y - vo.x);
        }
    }
    line_sync();
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int k = t + T * j;
        if (k <= M / 2) {
            st2(s + 2 * t, T * j, zc[j][0]);
            if (k > 0 && k < M / 2) st2(s - 2 * t, M - T * j, zc[j][1]);
        }
    }
    line_sync();
    float2 r[M1 / M2][M2];
    const float* const sl = s + 2 * t;
    fft_core<M1, M2, XP>(s, t, tw4, [&](int n1) { return ld2(sl, M2 * n1); }, r);
    line_sync();
    // output n = t + M2 q + M1 k2: x[pos(2n)] = Re r / M, x[pos(2n+1)] = -Im r / M
    // with pos(m) = 2m (m < M), 2(L-1-m)+1 (m >= M); m < M iff the
    // compile-time part B = 2 (M2 q + M1 k2) is below M
    const float sc = 0.5f * sqrtf(0.5f * L) / M;
    float* const wp = s + 4 * t;
    float* const wm = s - 4 * t;
#pragma unroll
    for (int q = 0; q < M1 / M2; ++q)
#pragma unroll
        for (int k2 = 0; k2 < M2; ++k2) {
            const int B = 2 * (M2 * q + M1 * k2);
            if (B < M) {
                wp[2 * B] = r[q][k2].x * sc;
                wp[2 * B + 2] = -r[q][k2].y * sc;
            } else {
                wm[2 * L - 1 - 2 * B] = r[q][k2].x * sc;
                wm[2 * L - 3 - 2 * B] = -r[q][k2].y * sc;
            }
        }
    if constexpr (BLOCK_END) __syncthreads();
    else line_sync();
}

// Orthonormal discrete Hartley transform (its own inverse) in place.
// Threads with `act` false only take part in the block synchronisation.
template <int M1, int M2>
__device__ __forceinline__ void line_dht(float* s, int t, const float2* tw4, bool act = true) {
    constexpr int M = M1 * M2, L = 2 * M, T = M2, NP = (M / 2 + T) / T;
    float2 z[M1 / M2][M2];
    const float* const sl = s + 2 * t;
    fft_core<M1, M2>(s, t, tw4, [&](int n1) { return ld2(sl, M2 * n1); }, z, act);
    line_sync();
    if (act) store_z<M1, M2>(s, t, z);
    line_sync();
    // 2 F[k] = a and 2 F[M-k] = b; H[k] = (Re F - Im F) / sqrt(L) and
    // H[L-k] = (Re F + Im F) / sqrt(L)
    const float h = 0.5f * sqrtf(1.f / L);
    float o[NP][4];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int k = t + T * j;
        if (act && k <= M / 2) {
            float2 zk, zm;
            load_pair<M, T>(s, t, j, zk, zm);
            const float2 ve = make_float2(zk.x + zm.x, zk.y - zm.y);
            const float2 vo = make_float2(zk.y + zm.y, zm.x - zk.x);
            const float2 p = cmul(tw4[4 * k], vo);
            const float2 a = cadd(ve, p);
            const float2 b = make_float2(ve.x - p.x, p.y - ve.y);
            o[j][0] = h * (a.x - a.y);              // H[k]
            o[j][1] = h * (a.x + a.y);              // H[L-k]
            o[j][2] = h * (b.x - b.y);              // H[M-k]
            o[j][3] = h * (b.x + b.y);              // H[M+k]
        }
    }
    line_sync();
    float* const op = s + t;
    float* const om = s - t;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int k = t + T * j;
        if (act && k <= M / 2) {
            op[T * j] = o[j][0];
            if (k > 0) om[L - T * j] = o[j][1];
            if (k < M / 2) {
                om[M - T * j] = o[j][2];
                if (k > 0) op[M + T * j] = o[j][3];
            }
        }
    }
    __syncthreads();
}

// ---- lines of length L = 2 M with M = M1 M2 not a power of two -----------
// (e.g. the paper's 100-pixel image sides, M = 5 x 10, and the periodic hue
// axes of 180 and 360 bins, M = 6 x 15 and 12 x 15).  The packed complex DFT
// of length M is a four-step M1 x M2 decomposition with M1 <= M2 and M2
// threads per line: thread t does the M1-point DFT of z[M2 n1 + t] in
// registers (the prime-factor DFTs of fft_common.h) and multiplies by
// e^{-2 pi i t k1 / M}; after one exchange through LDS thread t < M1 does the
// M2-point DFT of row k1 = t.  The packing and unpacking steps are those of
// the power-of-two transforms above, with every LDS index formed from the
// line start (no offsets below it).  tw4[j] = e^{-i pi j / (2L)}, j < 4L, as
// for the power-of-two lengths.  Threads with `act` false only take part in
// the block synchronisation.

// On return, threads t < M1 hold out[k2] = Z[t + M1 k2]; load(n1) must give
// z[M2 n1 + t].  The line's LDS region s (2M floats) is used for the exchange.
template <int M1, int M2, class Load>
__device__ __forceinline__ void fft_core_mix(float* s, int t, const float2* tw4, Load load,
                                             float2 (&out)[M2], bool act) {
    static_assert(M1 <= M2, "one stage-2 DFT per thread");
    float2 a[M1];
    if (act) {
#pragma unroll
        for (int n1 = 0; n1 < M1; ++n1) a[n1] = load(n1);
        dftm<M1>(a);
#pragma unroll
        for (int k1 = 1; k1 < M1; ++k1) a[k1] = cmul(a[k1], tw4[8 * t * k1]);   // 8 t k1 < 4L
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int k1 = 0; k1 < M1; ++k1) st2(s, k1 * M2 + t, a[k1]);
    }
    __syncthreads();
    if (act && t < M1) {
#pragma unroll
        for (int n2 = 0; n2 < M2; ++n2) out[n2] = ld2(s, t * M2 + n2);
        dftm<M2>(out);
    }
}

// Orthonormal DCT-II in place (Makhoul's reordering as in line_dct2).
template <int M1, int M2>
__device__ __forceinline__ void line_dct2_mix(float* s, int t, const float2* tw4, bool act = true) {
    constexpr int M = M1 * M2, L = 2 * M, NP = (M / 2 + M2) / M2;
    static_assert(M % 2 == 0, "pairs k, M - k");
    float2 z[M2];
    fft_core_mix<M1, M2>(s, t, tw4, [&](int n1) {
        const int n = M2 * n1 + t;         // v[2n], v[2n+1]
        return n < M / 2 ? make_float2(s[4 * n], s[4 * n + 2])
                         : make_float2(s[2 * L - 1 - 4 * n], s[2 * L - 3 - 4 * n]);
    }, z, act);
    __syncthreads();
    if (act && t < M1) {
#pragma unroll
        for (int k2 = 0; k2 < M2; ++k2) st2(s, t + M1 * k2, z[k2]);
    }
    __syncthreads();
    const float h = 0.5f * sqrtf(2.f / L), h0 = 0.5f * sqrtf(1.f / L);
    float o[NP][4];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int k = t + M2 * j;
        if (act && k <= M / 2) {
            const float2 zk = ld2(s, k), zm = ld2(s, k == 0 ? 0 : M - k);
            const float2 ve = make_float2(zk.x + zm.x, zk.y - zm.y);
            const float2 vo = make_float2(zk.y + zm.y, zm.x - zk.x);
            const float2 p = cmul(tw4[4 * k], vo);
            const float2 xa = cmul(tw4[k], cadd(ve, p));
            const float2 xb = cmul(tw4[M - k], make_float2(ve.x - p.x, p.y - ve.y));
            o[j][0] = (k == 0 ? h0 : h) * xa.x;     // X[k]
            o[j][1] = -h * xa.y;                    // X[L-k]
            o[j][2] = h * xb.x;                     // X[M-k]
            o[j][3] = -h * xb.y;                    // X[M+k]
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int k = t + M2 * j;
        if (act && k <= M / 2) {
            s[k] = o[j][0];
            if (k > 0) s[L - k] = o[j][1];
            if (k < M / 2) {
                s[M - k] = o[j][2];
                if (k > 0) s[M + k] = o[j][3];
            }
        }
    }
    __syncthreads();
}

// Orthonormal DCT-III (inverse of line_dct2_mix) in place, as line_dct3.
template <int M1, int M2>
__device__ __forceinline__ void line_dct3_mix(float* s, int t, const float2* tw4, bool act = true) {
    constexpr int M = M1 * M2, L = 2 * M, NP = (M / 2 + M2) / M2;
    static_assert(M % 2 == 0, "pairs k, M - k");
    float2 zc[NP][2];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int k = t + M2 * j;
        if (act && k <= M / 2) {
            const float xk = k == 0 ? 1.41421356237309515f * s[0] : s[k];
            const float xl = k == 0 ? 0.f : s[L - k];                         // X[L-k]
            const float xm = s[M - k];                                        // X[M-k]
            const float xp = s[M + k];                                        // X[M+k]
            const float2 v = cmul(cconj(tw4[k]), make_float2(xk, -xl));
            const float2 w = cmul(cconj(tw4[M - k]), make_float2(xm, -xp));   // V(M-k)
            const float2 ve = make_float2(v.x + w.x, v.y - w.y);
            const float2 vo = cmul(make_float2(v.x - w.x, v.y + w.y), cconj(tw4[4 * k]));
            zc[j][0] = make_float2(ve.x - vo.y, -(ve.y + vo.x));
            zc[j][1] = make_float2(ve.x + vo.y, ve.y - vo.x);
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int k = t + M2 * j;
        if (act && k <= M / 2) {
            st2(s, k, zc[j][0]);
            if (k > 0 && k < M / 2) st2(s, M - k, zc[j][1]);
        }
    }
    __syncthreads();
    float2 r[M2];
    fft_core_mix<M1, M2>(s, t, tw4, [&](int n1) { return ld2(s, M2 * n1 + t); }, r, act);
    __syncthreads();
    // output n = t + M1 k2: x[pos(2n)] = Re r / M, x[pos(2n+1)] = -Im r / M with
    // pos(m) = 2m (m < M), 2(L-1-m)+1 (m >= M)
    const float sc = 0.5f * sqrtf(0.5f * L) / M;
    if (act && t < M1) {
#pragma unroll
        for (int k2 = 0; k2 < M2; ++k2) {
            const int n = t + M1 * k2;
            if (n < M / 2) {
                s[4 * n] = r[k2].x * sc;
                s[4 * n + 2] = -r[k2].y * sc;
            } else {
                s[2 * L - 1 - 4 * n] = r[k2].x * sc;
                s[2 * L - 3 - 4 * n] = -r[k2].y * sc;
            }
        }
    }
    __syncthreads();
}

// Orthonormal discrete Hartley transform (its own inverse) in place, as
// line_dht.
template <int M1, int M2>
__device__ __forceinline__ void line_dht_mix(float* s, int t, const float2* tw4, bool act = true) {
    constexpr int M = M1 * M2, L = 2 * M, NP = (M / 2 + M2) / M2;
    static_assert(M % 2 == 0, "pairs k, M - k");
    float2 b[M2];
    fft_core_mix<M1, M2>(s, t, tw4, [&](int n1) { return ld2(s, M2 * n1 + t); }, b, act);
    __syncthreads();
    if (act && t < M1) {
#pragma unroll
        for (int k2 = 0; k2 < M2; ++k2) st2(s, t + M1 * k2, b[k2]);
    }
    __syncthreads();
    // 2 F[k] = a and 2 F[M-k] = b for the pairs k <= M / 2 (k = t + M2 j)
    const float h = 0.5f * sqrtf(1.f / L);
    float o[NP][4];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int k = t + M2 * j;
        if (act && k <= M / 2) {
            const float2 zk = ld2(s, k), zm = ld2(s, k == 0 ? 0 : M - k);
            const float2 ve = make_float2(zk.x + zm.x, zk.y - zm.y);
            const float2 vo = make_float2(zk.y + zm.y, zm.x - zk.x);
            const float2 p = cmul(tw4[4 * k], vo);
            const float2 fa = cadd(ve, p);
            const float2 fb = make_float2(ve.x - p.x, p.y - ve.y);
            o[j][0] = h * (fa.x - fa.y);            // H[k]
            o[j][1] = h * (fa.x + fa.y);            // H[L-k]
            o[j][2] = h * (fb.x - fb.y);            // H[M-k]
            o[j][3] = h * (fb.x + fb.y);            // H[M+k]
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int k = t + M2 * j;
        if (act && k <= M / 2) {
            s[k] = o[j][0];
            if (k > 0) s[L - k] = o[j][1];
            if (k < M / 2) {
                s[M - k] = o[j][2];
                if (k > 0) s[M + k] = o[j][3];
            }
        }
    }
    __syncthreads();
}

template <int M1, int M2, int KIND>
__device__ __forceinline__ void line_xform_mix(float* s, int t, const float2* tw4, bool act) {
    if constexpr (KIND == 0) line_dct2_mix<M1, M2>(s, t, tw4, act);
    else if constexpr (KIND == 1) line_dct3_mix<M1, M2>(s, t, tw4, act);
    else line_dht_mix<M1, M2>(s, t, tw4, act);
}

// XP: exchange padding of the DCTs (fft_core); the line's LDS region then
// needs max(2 M, M1 (2 M2 + XP)) floats.
template <int M1, int M2, int KIND, int XP = 0, bool BLOCK_END = true>
__device__ __forceinline__ void line_xform(float* s, int t, const float2* tw4) {
    static_assert(KIND != 2 || XP == 0, "no padded exchange for the Hartley transform");
    static_assert(BLOCK_END || KIND == 1, "a wavefront-sync end only for the DCT-III");
    if constexpr (KIND == 0) line_dct2<M1, M2, XP>(s, t, tw4);
    else if constexpr (KIND == 1) line_dct3<M1, M2, XP, BLOCK_END>(s, t, tw4);
    else line_dht<M1, M2>(s, t, tw4);
}

}  // namespace otd
