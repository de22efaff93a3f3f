// Complex helpers and in-register DFTs shared by the transform kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace otd {

// ---- complex helpers --------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// cos and sin of 2 pi j / 16 (exact constants of the 16th roots of unity)
__device__ __forceinline__ float cos16(int j) {
    constexpr float c1 = 0.923879532511286756f, s1 = 0.382683432365089772f,
                    h = 0.707106781186547524f;
    switch (j & 15) {
        case 0: return 1.f;   case 1: return c1;  case 2: return h;   case 3: return s1;
        case 4: return 0.f;   case 5: return -s1; case 6: return -h;  case 7: return -c1;
        case 8: return -1.f;  case 9: return -c1; case 10: return -h; case 11: return -s1;
        case 12: return 0.f;  case 13: return s1; case 14: return h;  default: return c1;
    }
}
__device__ __forceinline__ float sin16(int j) { return cos16(j - 4); }

// v * e^{-2 pi i J / 16} with the trivial factors (1, -i, -1, i) and the
// eighth roots (1 -+ i) / sqrt 2 taken apart: the general product would
// multiply by exact zeros and ones, which IEEE arithmetic may not drop.
template <int J>
__device__ __forceinline__ float2 twmul(float2 v) {
    constexpr int j = J & 15;
    constexpr float h = 0.707106781186547524f;
    if constexpr (j == 0) return v;
    else if constexpr (j == 4) return make_float2(v.y, -v.x);
    else if constexpr (j == 8) return make_float2(-v.x, -v.y);
    else if constexpr (j == 12) return make_float2(-v.y, v.x);
    else if constexpr (j == 2) return make_float2(h * (v.x + v.y), h * (v.y - v.x));
    else if constexpr (j == 6) return make_float2(h * (v.y - v.x), -h * (v.x + v.y));
    else if constexpr (j == 10) return make_float2(-h * (v.x + v.y), h * (v.x - v.y));
    else if constexpr (j == 14) return make_float2(h * (v.x - v.y), h * (v.x + v.y));
    else return cmul(make_float2(cos16(j), -sin16(j)), v);
}

// a[k + R/2] and a[k] of one radix-2 step, for k < K, with the twiddle of k
// resolved at compile time.
template <int R, int K>
__device__ __forceinline__ void butterflies(float2* a, const float2* e, const float2* o) {
    if constexpr (K > 0) {
        butterflies<R, K - 1>(a, e, o);
        constexpr int k = K - 1;
        const float2 p = twmul<k * (16 / R)>(o[k]);
        a[k] = cadd(e[k], p);
        a[k + R / 2] = csub(e[k], p);
    }
}

// In-register forward DFT of length R (radix-2 decimation in time),
// a[k] <- sum_n a[n] e^{-2 pi i n k / R}; R in {1, 2, 4, 8, 16}.
template <int R>
__device__ __forceinline__ void dft(float2* a) {
    if constexpr (R == 1) {
        return;
    } else if constexpr (R == 2) {
        const float2 u = a[0], v = a[1];
        a[0] = cadd(u, v);
        a[1] = csub(u, v);
    } else {
        float2 e[R / 2], o[R / 2];
#pragma unroll
        for (int i = 0; i < R / 2; ++i) { e[i] = a[2 * i]; o[i] = a[2 * i + 1]; }
        dft<R / 2>(e);
        dft<R / 2>(o);
        butterflies<R, R / 2>(a, e, o);
    }
}

__device__ __forceinline__ float2 ld2(const float* s, int c) { return make_float2(s[2 * c], s[2 * c + 1]); }
__device__ __forceinline__ void st2(float* s, int c, float2 v) { s[2 * c] = v.x; s[2 * c + 1] = v.y; }

}  // namespace otd
