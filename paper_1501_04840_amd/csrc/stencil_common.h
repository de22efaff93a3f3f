// Device helpers shared by the stencil kernels: index maps, the FP64 block
// sum and the pointwise prox of J (Sec. 3, Step 2).
#pragma once

#include "otd_common.h"

// Multiply-adds are fused only within one source expression, never across
// statements: left to the backend, fusion depends on which other values use
// a product, so the instantiation that also forms the residual partials of a
// check iteration would round the state update differently from the one
// that does not, and runs with and without checks would drift apart.
#pragma clang fp contract(on)

namespace otd {

__device__ inline long long cidx(const Geom& g, int b, int k, int c, int p) {
    return (long long)b * g.nc + (long long)k * g.slice + (long long)c * g.plane + p;
}
__device__ inline long long fidx(const Geom& g, int b, int k, int c, int p) {
    return (long long)b * g.nf + (long long)k * g.slice + (long long)c * g.plane + p;
}

// Deterministic FP64 sum over the threads of a block (blockDim.x a multiple
// of 64, at most 1024); the result is valid in thread 0.
__device__ inline double block_sum(double v) {
    __shared__ double red[16];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < nw; ++i) t += red[i];
    return t;
}

// N deterministic FP64 block sums at once (the exchanges of the N values
// interleave); results valid in thread 0.  N <= 8.
template <int N>
__device__ inline void block_sums(double (&v)[N]) {
    __shared__ double red[16][N];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int q = 0; q < N; ++q) v[q] += __shfl_down(v[q], o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < N; ++q) red[w][q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < N; ++q) {
            double t = 0.0;
            for (int i = 0; i < nw; ++i) t += red[i][q];
            v[q] = t;
        }
}

// Pointwise prox of J / sigma (Step 2): (0, 0) if 2 a_f + sigma |a_m|^2 <= 0,
// else v is the positive root of 2 (1 + sigma v)^2 (v - a_f) = sigma |a_m|^2,
// reached by Newton from v0 = max(a_f, 0) + sigma |a_m|^2 / 2 (right of the
// root, where the cubic is increasing and convex: monotone decrease), and
// u = sigma v a_m / (1 + sigma v).
// Closed form of the positive root (OT_PROX_CLOSED, Cardano): with
// w = 1 + sigma v the cubic is w^3 - beta w^2 - gamma = 0, beta = 1 + sigma
// a_f, gamma = sigma^2 |a_m|^2 / 2.  beta > 0: w = beta / 3 + A + beta^2 /
// (9 A), A = cbrt(beta^3 / 27 + gamma / 2 + sqrt(gamma^2 / 4 + gamma beta^3 /
// 27)), a sum of positive terms.  beta <= 0 (gamma > 1 on active nodes):
// s = 1 / w is the positive root of s^3 - 3 P s - 2 H = 0, P = -beta /
// (3 gamma), H = 1 / (2 gamma): s = A + P / A, A = cbrt(H + sqrt(H^2 - P^3))
// when H^2 >= P^3, else s = 2 sqrt(P) cos(acos(H / P^{3/2}) / 3) with the
// argument in (0, 1] (well conditioned).  v = (w - 1) / sigma loses digits
// when sigma v << 1, which the caller's Newton steps restore.  Active nodes
// only (2 a_f + sigma |a_m|^2 > 0).
__device__ inline float prox_root_closed(float a2, float af, float sigma) {
    const float beta = fmaf(sigma, af, 1.f);
    const float gamma = 0.5f * sigma * sigma * a2;
    float w;
    if (beta > 0.f) {
        const float b3 = beta * beta * beta * (1.f / 27.f);
        const float A = cbrtf(b3 + 0.5f * gamma + sqrtf(gamma * (0.25f * gamma + b3)));
        w = beta * (1.f / 3.f) + A + beta * beta / (9.f * A);
    } else {
        const float P = -beta / (3.f * gamma), H = 0.5f / gamma;
        const float disc = H * H - P * P * P;
        float sv;
        if (disc >= 0.f) {
            const float A = cbrtf(H + sqrtf(disc));
            sv = A + P / A;
        } else {
            sv = 2.f * sqrtf(P) * cosf(acosf(fminf(H / (P * sqrtf(P)), 1.f)) * (1.f / 3.f));
        }
        w = 1.f / sv;
    }
    return fmaxf((w - 1.f) / sigma, 0.f);
}

// One Newton step for the cubic g(v) = 2 (1 + sigma v)^2 (v - a_f) -
// sigma |a_m|^2 from v > 0; a step that would leave the positive half-line
// (or is not finite) is not taken.
__device__ inline float prox_newton_step(float vv, float a2, float af, float sigma) {
    const float w = 1.f + sigma * vv;
    const float d = vv - af;
    const float gv = 2.f * w * w * d - sigma * a2;
    const float dg = 4.f * sigma * w * d + 2.f * w * w;
    const float vn = vv - gv / dg;
    return vn > 0.f && vn < 3.0e38f ? vn : vv;
}

__device__ inline void prox_J(float mx, float my, float mc, float af, float sigma,
                              float& ux, float& uy, float& uc, float& v, int kind = 0) {
    const float a2 = mx * mx + my * my + mc * mc;
    if (!(2.f * af + sigma * a2 > 0.f)) {
        ux = uy = uc = v = 0.f;
        return;
    }
    if (kind != 0) {
        float vc = prox_root_closed(a2, af, sigma);
        if (kind == 1 && vc > 0.f) {
            vc = prox_newton_step(vc, a2, af, sigma);
            vc = prox_newton_step(vc, a2, af, sigma);
        }
        if (vc > 0.f || kind == 2) {
            const float sc = sigma * vc / (1.f + sigma * vc);
            ux = sc * mx;
            uy = sc * my;
            uc = sc * mc;
            v = vc;
            return;
        }
        // the closed form rounded a positive root to 0: Newton below
    }
    float vv = fmaxf(af, 0.f) + 0.5f * sigma * a2;
    for (int it = 0; it < 60; ++it) {
        const float w = 1.f + sigma * vv;
        const float d = vv - af;
        const float gv = 2.f * w * w * d - sigma * a2;
        const float dg = 4.f * sigma * w * d + 2.f * w * w;
        float vn = vv - gv / dg;
        if (!(vn < vv)) break;                 // no further decrease: converged
        if (vn <= 0.f) vn = 0.5f * vv;
        const bool done = (vv - vn) <= 1e-6f * vn;
        vv = vn;
        if (done) break;
    }
    const float sc = sigma * vv / (1.f + sigma * vv);
    ux = sc * mx;
    uy = sc * my;
    uc = sc * mc;
    v = vv;
}

}  // namespace otd
