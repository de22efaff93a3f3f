// Complex helpers and in-register DFTs shared by the transform kernels.
#pragma once

#include <hip/hip_runtime.h>

// Multiply-adds are fused only within one source expression (as in the
// stencil kernels): left to the backend, fusion depends on the surrounding
// code, and the same line transform would round differently in different
// kernels.
#pragma clang fp contract(on)

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

// ---- in-register DFTs of lengths with factors 2, 3 and 5 --------------------
// Length 3: X1,2 = a - (b + c) / 2 -+ i (sqrt 3 / 2)(b - c).
__device__ __forceinline__ void dft3(float2* x) {
    constexpr float h = 0.866025403784438647f;   // sqrt(3) / 2
    const float2 t1 = cadd(x[1], x[2]), d = csub(x[1], x[2]);
    const float2 t2 = make_float2(x[0].x - 0.5f * t1.x, x[0].y - 0.5f * t1.y);
    const float2 r = make_float2(h * d.y, -h * d.x);    // -i (sqrt 3 / 2) d
    x[0] = cadd(x[0], t1);
    x[1] = cadd(t2, r);
    x[2] = csub(t2, r);
}

// Length 5 with the symmetric sums t1 = x1 + x4, t2 = x2 + x3 and the
// differences d1 = x1 - x4, d2 = x2 - x3: with c_j = cos(2 pi j / 5) and
// s_j = sin(2 pi j / 5),
//   X1,4 = x0 + c1 t1 + c2 t2 -+ i (s1 d1 + s2 d2),
//   X2,3 = x0 + c2 t1 + c1 t2 -+ i (s2 d1 - s1 d2).
__device__ __forceinline__ void dft5(float2* x) {
    constexpr float c1 = 0.309016994374947424f, c2 = -0.809016994374947424f;
    constexpr float s1 = 0.951056516295153572f, s2 = 0.587785252292473129f;
    const float2 t1 = cadd(x[1], x[4]), t2 = cadd(x[2], x[3]);
    const float2 d1 = csub(x[1], x[4]), d2 = csub(x[2], x[3]);
    const float2 a1 = make_float2(x[0].x + c1 * t1.x + c2 * t2.x, x[0].y + c1 * t1.y + c2 * t2.y);
    const float2 a2 = make_float2(x[0].x + c2 * t1.x + c1 * t2.x, x[0].y + c2 * t1.y + c1 * t2.y);
    const float2 b1 = make_float2(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y);
    const float2 b2 = make_float2(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y);
    x[0] = cadd(x[0], cadd(t1, t2));
    x[1] = make_float2(a1.x + b1.y, a1.y - b1.x);       // a1 - i b1
    x[4] = make_float2(a1.x - b1.y, a1.y + b1.x);       // a1 + i b1
    x[2] = make_float2(a2.x + b2.y, a2.y - b2.x);
    x[3] = make_float2(a2.x - b2.y, a2.y + b2.x);
}

constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }
constexpr int cmodinv(int a, int m) {   // a^-1 mod m (gcd(a, m) = 1, m > 1)
    int r = 1;
    while ((a * r) % m != 1) ++r;
    return r;
}

template <int N>
__device__ __forceinline__ void dftm(float2* a);

// Prime-factor (Good-Thomas) DFT of length N = R S with gcd(R, S) = 1: with
// n = (S n1 + R n2) mod N and k = (S e1 k1 + R e2 k2) mod N, e1 = S^-1 mod R,
// e2 = R^-1 mod S, the exponent n k is S e1 n1 k1 + R e2 n2 k2 mod N, so the
// DFT is R-point DFTs over n1 followed by S-point DFTs over n2, without
// twiddle factors.  All indices are compile-time constants once unrolled.
template <int R, int S>
__device__ __forceinline__ void pfa(float2* a) {
    static_assert(cgcd(R, S) == 1, "prime-factor DFT needs coprime factors");
    constexpr int N = R * S;
    constexpr int e1 = R == 1 ? 0 : cmodinv(S % R, R), e2 = S == 1 ? 0 : cmodinv(R % S, S);
    float2 u[S][R];
#pragma unroll
    for (int n2 = 0; n2 < S; ++n2)
#pragma unroll
        for (int n1 = 0; n1 < R; ++n1) u[n2][n1] = a[(S * n1 + R * n2) % N];
#pragma unroll
    for (int n2 = 0; n2 < S; ++n2) dftm<R>(u[n2]);
    float2 v[R][S];
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1)
#pragma unroll
        for (int n2 = 0; n2 < S; ++n2) v[k1][n2] = u[n2][k1];
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) dftm<S>(v[k1]);
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < S; ++k2) a[(S * e1 * k1 + R * e2 * k2) % N] = v[k1][k2];
}

// In-register forward DFT a[k] <- sum_n a[n] e^{-2 pi i n k / N} for the
// lengths of the mixed-radix line transforms: powers of two up to 16, 3, 5,
// and coprime products of these (6, 10, 12, 15, 20, 30, 60).
template <int N>
__device__ __forceinline__ void dftm(float2* a) {
    if constexpr (N == 1 || N == 2 || N == 4 || N == 8 || N == 16) dft<N>(a);
    else if constexpr (N == 3) dft3(a);
    else if constexpr (N == 5) dft5(a);
    else if constexpr (N % 16 == 0 && cgcd(16, N / 16) == 1) pfa<16, N / 16>(a);
    else if constexpr (N % 8 == 0 && cgcd(8, N / 8) == 1) pfa<8, N / 8>(a);
    else if constexpr (N % 4 == 0 && cgcd(4, N / 4) == 1) pfa<4, N / 4>(a);
    else if constexpr (N % 2 == 0 && cgcd(2, N / 2) == 1) pfa<2, N / 2>(a);
    else if constexpr (N % 3 == 0 && cgcd(3, N / 3) == 1) pfa<3, N / 3>(a);
    else static_assert(N == 1, "dftm: unsupported length");
}

__device__ __forceinline__ float2 ld2(const float* s, int c) { return make_float2(s[2 * c], s[2 * c + 1]); }
__device__ __forceinline__ void st2(float* s, int c, float2 v) { s[2 * c] = v.x; s[2 * c + 1] = v.y; }

}  // namespace otd
