// Device helpers shared by the stencil kernels: index maps, the FP64 block
// sum and the pointwise prox of J (Sec. 3, Step 2).
#pragma once

#include "otd_common.h"

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
__device__ inline void prox_J(float mx, float my, float mc, float af, float sigma,
                              float& ux, float& uy, float& uc, float& v) {
    const float a2 = mx * mx + my * my + mc * mc;
    if (!(2.f * af + sigma * a2 > 0.f)) {
        ux = uy = uc = v = 0.f;
        return;
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
