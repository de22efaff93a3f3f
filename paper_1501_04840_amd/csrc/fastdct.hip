// Fast transforms of power-of-two length for the Poisson solve (Sec. 3 of
// the paper: A A^T is diagonalised by the orthonormal DCT-II C_p along
// Neumann axes and by a real Fourier basis along periodic axes, so the
// pseudo-inverse "can be computed by the FFT and the fast cosine transform").
// The line transforms themselves are in fft_lines.h.
#include "otd_common.h"
#include "fft_lines.h"

#pragma clang fp contract(on)   // as in fft_common.h

namespace otd {

// Planes reduced per block by the plane-sum blocks of k_rows_fft (32 lanes,
// half a wave, per plane).
constexpr int kSumPlanesPerBlock = 8;

// One plane-sum block: kSumPlanesPerBlock planes of `ps` (32 lanes, half a
// wave, per plane) reduced in place into slot 0 of each plane.  No block
// synchronisation: such blocks return independently.
__device__ __forceinline__ void plane_sums_block(const PlaneSums& ps, long long blk) {
    const int l = threadIdx.x & 31;
    const long long q = blk * kSumPlanesPerBlock + (threadIdx.x >> 5);
    const bool live = q < ps.nq;
    double* pp = ps.part + (live ? q : 0) * ps.nbx;
    double acc = 0.0;
    for (int i = l; i < ps.nbx; i += 32 * 16) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int ii = i + 32 * u;
            v[u] = live && ii < ps.nbx ? pp[ii] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) acc += v[u];
    }
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 32);
    // every lane's loads of this plane are consumed above, so slot 0 can be
    // overwritten with the total
    if (live && l == 0) pp[0] = acc;
}

// Contiguous axis: LPB whole rows per block, row pitch L + 1 in LDS.  The
// block's rows are one contiguous span, staged with unrolled loads so that
// every thread keeps all of its loads in flight at once; single floats,
// consecutive over the threads, so that the LDS writes of a wave fall in
// distinct banks (float4 loads written as four floats hit each bank four
// times).  The first
// nsb blocks instead reduce the FP64 plane sums `ps` in place (the first
// forward pass runs between the divergence kernel that writes them and the
// colour/time pass that solves the spatial-DC line from them, so the
// reduction costs no launch and leaves that pass a short serial part).
template <int M1, int M2, int KIND>
__global__ void __launch_bounds__(256) k_rows_fft(float* R, long long rows, const float2* tw4,
                                                  PlaneSums ps, int nsb, RowSkip skip) {
    constexpr int L = 2 * M1 * M2, T = M2, LPB = 256 / T, PITCH = L + 1;
    constexpr int NS = LPB * L / 256;             // floats per thread
    __shared__ float lds[LPB * PITCH];
    if ((int)blockIdx.x < nsb) {
        plane_sums_block(ps, blockIdx.x);
        return;
    }
    const long long r0 = (long long)(blockIdx.x - nsb) * LPB;
    const int nr = (int)min((long long)LPB, rows - r0);
    if (rows_frozen(skip, r0, nr)) return;
    float* g = R + r0 * L;
    float buf[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const int e = threadIdx.x + 256 * j;
        buf[j] = e / L < nr ? g[e] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const int e = threadIdx.x + 256 * j;
        lds[(e / L) * PITCH + (e % L)] = buf[j];
    }
    __syncthreads();
    const int line = threadIdx.x / T, t = threadIdx.x - line * T;
    line_xform<M1, M2, KIND>(lds + line * PITCH, t, tw4);
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const int e = threadIdx.x + 256 * j;
        if (e / L < nr) g[e] = lds[(e / L) * PITCH + (e % L)];
    }
}

// Strided axis: data [outer][L][inner]; a block transforms W = LPB columns,
// stored transposed in LDS (pitch L + 1, conflict-free transposing writes).
// VEC: inner is a multiple of 4, so the tile rows are loaded as float4.
// One-dimensional grid: the first nsb blocks reduce the plane sums `ps` (as
// in k_rows_fft, when this is the first forward pass), then ntiles column
// tiles for each of the outer slabs.
template <int M1, int M2, int KIND, bool VEC>
__global__ void __launch_bounds__(256) k_cols_fft(float* R, long long inner, const float2* tw4,
                                                  PlaneSums ps, int nsb, int ntiles) {
    constexpr int L = 2 * M1 * M2, T = M2, W = 256 / T, PITCH = L + 1;
    constexpr int W4 = W / 4, NV = L * W / 1024, NS = L * W / 256;
    __shared__ float lds[W * PITCH];
    if ((int)blockIdx.x < nsb) {
        plane_sums_block(ps, blockIdx.x);
        return;
    }
    const long long blk = (long long)blockIdx.x - nsb;
    const long long o = blk / ntiles;
    const long long i0 = (blk - o * ntiles) * W;
    const int nw = (int)min((long long)W, inner - i0);
    float* g = R + o * L * inner + i0;
    if constexpr (VEC) {
        float4 buf[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const int e = threadIdx.x + 256 * j;
            const int k = e / W4, i = 4 * (e % W4);
            buf[j] = i < nw ? *reinterpret_cast<const float4*>(g + (long long)k * inner + i)
                            : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const int e = threadIdx.x + 256 * j;
            const int k = e / W4, i = 4 * (e % W4);
            lds[i * PITCH + k] = buf[j].x;
            lds[(i + 1) * PITCH + k] = buf[j].y;
            lds[(i + 2) * PITCH + k] = buf[j].z;
            lds[(i + 3) * PITCH + k] = buf[j].w;
        }
    } else {
        float buf[NS];
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const int e = threadIdx.x + 256 * j;
            const int k = e / W, i = e % W;
            buf[j] = i < nw ? g[(long long)k * inner + i] : 0.f;
        }
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const int e = threadIdx.x + 256 * j;
            lds[(e % W) * PITCH + e / W] = buf[j];
        }
    }
    __syncthreads();
    const int line = threadIdx.x / T, t = threadIdx.x - line * T;
    line_xform<M1, M2, KIND>(lds + line * PITCH, t, tw4);
    if constexpr (VEC) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const int e = threadIdx.x + 256 * j;
            const int k = e / W4, i = 4 * (e % W4);
            if (i < nw)
                *reinterpret_cast<float4*>(g + (long long)k * inner + i) =
                    make_float4(lds[i * PITCH + k], lds[(i + 1) * PITCH + k],
                                lds[(i + 2) * PITCH + k], lds[(i + 3) * PITCH + k]);
        }
    } else {
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const int e = threadIdx.x + 256 * j;
            const int k = e / W, i = e % W;
            if (i < nw) g[(long long)k * inner + i] = lds[i * PITCH + k];
        }
    }
}

// ---- lengths L = 2 M1 M2 with factors 2, 3 and 5 (line_xform_mix) ------------
// 32 lines per block and M2 threads per line (NT = 32 M2 >= 256 threads);
// otherwise as k_rows_fft / k_cols_fft, including the plane-sum blocks
// (their first 256 threads, as there).
constexpr int kMixLines = 32;

template <int M1, int M2, int KIND>
__global__ void __launch_bounds__(kMixLines * M2) k_rows_mix(float* R, long long rows, const float2* tw4,
                                                             PlaneSums ps, int nsb, RowSkip skip) {
    constexpr int L = 2 * M1 * M2, NT = kMixLines * M2, PITCH = L + 1;
    static_assert(NT >= 256 && L % 4 == 0, "block shape");
    __shared__ float lds[kMixLines * PITCH];
    if ((int)blockIdx.x < nsb) {
        if (threadIdx.x < 256) plane_sums_block(ps, blockIdx.x);
        return;
    }
    const long long r0 = (long long)(blockIdx.x - nsb) * kMixLines;
    const int nr = (int)min((long long)kMixLines, rows - r0);
    if (rows_frozen(skip, r0, nr)) return;
    float* g = R + r0 * L;
    const int n4 = nr * L / 4;
    for (int v = threadIdx.x; v < n4; v += NT) {
        const float4 q = reinterpret_cast<const float4*>(g)[v];
        const int e = 4 * v;
        float* d = lds + (e / L) * PITCH + (e % L);
        d[0] = q.x; d[1] = q.y; d[2] = q.z; d[3] = q.w;
    }
    __syncthreads();
    const int line = threadIdx.x / M2, t = threadIdx.x - line * M2;
    line_xform_mix<M1, M2, KIND>(lds + line * PITCH, t, tw4, line < nr);
    for (int v = threadIdx.x; v < n4; v += NT) {
        const int e = 4 * v;
        const float* d = lds + (e / L) * PITCH + (e % L);
        reinterpret_cast<float4*>(g)[v] = make_float4(d[0], d[1], d[2], d[3]);
    }
}

// Strided axis: data [outer][L][inner]; a block transforms 32 columns
// (128 contiguous bytes per row of the tile), stored transposed in LDS.
template <int M1, int M2, int KIND>
__global__ void __launch_bounds__(kMixLines * M2) k_cols_mix(float* R, long long inner, const float2* tw4,
                                                             PlaneSums ps, int nsb, int ntiles) {
    constexpr int L = 2 * M1 * M2, NT = kMixLines * M2, W = kMixLines, PITCH = L + 1;
    static_assert(NT >= 256, "block shape");
    __shared__ float lds[W * PITCH];
    if ((int)blockIdx.x < nsb) {
        if (threadIdx.x < 256) plane_sums_block(ps, blockIdx.x);
        return;
    }
    const long long blk = (long long)blockIdx.x - nsb;
    const long long o = blk / ntiles;
    const long long i0 = (blk - o * ntiles) * W;
    const int nw = (int)min((long long)W, inner - i0);
    float* g = R + o * L * inner + i0;
    for (int e = threadIdx.x; e < L * W; e += NT) {
        const int k = e / W, i = e - k * W;
        if (i < nw) lds[i * PITCH + k] = g[(long long)k * inner + i];
    }
    __syncthreads();
    const int line = threadIdx.x / M2, t = threadIdx.x - line * M2;
    line_xform_mix<M1, M2, KIND>(lds + line * PITCH, t, tw4, line < nw);
    for (int e = threadIdx.x; e < L * W; e += NT) {
        const int k = e / W, i = e - k * W;
        if (i < nw) g[(long long)k * inner + i] = lds[i * PITCH + k];
    }
}

// The (M1, M2) split of each mixed length L = 2 M1 M2.
bool mix_len(int L) { return L == 100 || L == 180 || L == 360; }

template <int M1, int M2>
static void rows_mix_dispatch(float* R, long long rows, const float2* tw, int kind, hipStream_t st,
                              const PlaneSums* sums, RowSkip sk) {
    const PlaneSums ps = sums ? *sums : PlaneSums{nullptr, 0, 0};
    const int nsb = (int)((ps.nq + kSumPlanesPerBlock - 1) / kSumPlanesPerBlock);
    const dim3 grid((unsigned)((rows + kMixLines - 1) / kMixLines + nsb)), block(kMixLines * M2);
    if (kind == 0) hipLaunchKernelGGL((k_rows_mix<M1, M2, 0>), grid, block, 0, st, R, rows, tw, ps, nsb, sk);
    else if (kind == 1) hipLaunchKernelGGL((k_rows_mix<M1, M2, 1>), grid, block, 0, st, R, rows, tw, ps, nsb, sk);
    else hipLaunchKernelGGL((k_rows_mix<M1, M2, 2>), grid, block, 0, st, R, rows, tw, ps, nsb, sk);
}

template <int M1, int M2>
static void cols_mix_dispatch(float* R, long long outer, long long inner, const float2* tw, int kind,
                              hipStream_t st, const PlaneSums* sums) {
    const PlaneSums ps = sums ? *sums : PlaneSums{nullptr, 0, 0};
    const int nsb = (int)((ps.nq + kSumPlanesPerBlock - 1) / kSumPlanesPerBlock);
    const int ntiles = (int)((inner + kMixLines - 1) / kMixLines);
    const dim3 grid((unsigned)(ntiles * outer + nsb)), block(kMixLines * M2);
    if (kind == 0) hipLaunchKernelGGL((k_cols_mix<M1, M2, 0>), grid, block, 0, st, R, inner, tw, ps, nsb, ntiles);
    else if (kind == 1) hipLaunchKernelGGL((k_cols_mix<M1, M2, 1>), grid, block, 0, st, R, inner, tw, ps, nsb, ntiles);
    else hipLaunchKernelGGL((k_cols_mix<M1, M2, 2>), grid, block, 0, st, R, inner, tw, ps, nsb, ntiles);
}

void launch_rows_mix(float* R, long long rows, int L, const float2* tw, int kind, hipStream_t st,
                     const PlaneSums* sums, RowSkip sk) {
    if (L == 100) rows_mix_dispatch<5, 10>(R, rows, tw, kind, st, sums, sk);
    else if (L == 180) rows_mix_dispatch<6, 15>(R, rows, tw, kind, st, sums, sk);
    else rows_mix_dispatch<12, 15>(R, rows, tw, kind, st, sums, sk);
}

void launch_cols_mix(float* R, long long outer, long long inner, int L, const float2* tw, int kind,
                     hipStream_t st, const PlaneSums* sums) {
    if (L == 100) cols_mix_dispatch<5, 10>(R, outer, inner, tw, kind, st, sums);
    else if (L == 180) cols_mix_dispatch<6, 15>(R, outer, inner, tw, kind, st, sums);
    else cols_mix_dispatch<12, 15>(R, outer, inner, tw, kind, st, sums);
}

bool fast_len(int L) { return L >= 32 && L <= 512 && (L & (L - 1)) == 0; }

template <int M1, int M2>
static void rows_dispatch(float* R, long long rows, const float2* tw, int kind, hipStream_t st,
                          const PlaneSums* sums, RowSkip sk) {
    constexpr int LPB = 256 / M2;
    const PlaneSums ps = sums ? *sums : PlaneSums{nullptr, 0, 0};
    const int nsb = (int)((ps.nq + kSumPlanesPerBlock - 1) / kSumPlanesPerBlock);
    const dim3 grid((unsigned)((rows + LPB - 1) / LPB + nsb));
    if (kind == 0) hipLaunchKernelGGL((k_rows_fft<M1, M2, 0>), grid, dim3(256), 0, st, R, rows, tw, ps, nsb, sk);
    else if (kind == 1) hipLaunchKernelGGL((k_rows_fft<M1, M2, 1>), grid, dim3(256), 0, st, R, rows, tw, ps, nsb, sk);
    else hipLaunchKernelGGL((k_rows_fft<M1, M2, 2>), grid, dim3(256), 0, st, R, rows, tw, ps, nsb, sk);
}

template <int M1, int M2, bool VEC>
static void cols_dispatch_v(float* R, long long outer, long long inner, const float2* tw, int kind,
                            hipStream_t st, const PlaneSums* sums) {
    constexpr int W = 256 / M2;
    const PlaneSums ps = sums ? *sums : PlaneSums{nullptr, 0, 0};
    const int nsb = (int)((ps.nq + kSumPlanesPerBlock - 1) / kSumPlanesPerBlock);
    const int ntiles = (int)((inner + W - 1) / W);
    const dim3 grid((unsigned)(ntiles * outer + nsb));
    if (kind == 0) hipLaunchKernelGGL((k_cols_fft<M1, M2, 0, VEC>), grid, dim3(256), 0, st, R, inner, tw, ps, nsb, ntiles);
    else if (kind == 1) hipLaunchKernelGGL((k_cols_fft<M1, M2, 1, VEC>), grid, dim3(256), 0, st, R, inner, tw, ps, nsb, ntiles);
    else hipLaunchKernelGGL((k_cols_fft<M1, M2, 2, VEC>), grid, dim3(256), 0, st, R, inner, tw, ps, nsb, ntiles);
}

template <int M1, int M2>
static void cols_dispatch(float* R, long long outer, long long inner, const float2* tw, int kind,
                          hipStream_t st, const PlaneSums* sums) {
    if (inner % 4 == 0) cols_dispatch_v<M1, M2, true>(R, outer, inner, tw, kind, st, sums);
    else cols_dispatch_v<M1, M2, false>(R, outer, inner, tw, kind, st, sums);
}

// kind: 0 forward DCT-II, 1 inverse (DCT-III), 2 Hartley (either direction)
void launch_rows_fast(float* R, long long rows, int L, const float2* tw, int kind, hipStream_t st,
                      const PlaneSums* sums, RowSkip sk) {
    switch (L) {
        case 32: rows_dispatch<4, 4>(R, rows, tw, kind, st, sums, sk); break;
        case 64: rows_dispatch<8, 4>(R, rows, tw, kind, st, sums, sk); break;
        case 128: rows_dispatch<8, 8>(R, rows, tw, kind, st, sums, sk); break;
        case 256: rows_dispatch<16, 8>(R, rows, tw, kind, st, sums, sk); break;
        default: rows_dispatch<16, 16>(R, rows, tw, kind, st, sums, sk); break;
    }
}

void launch_cols_fast(float* R, long long outer, long long inner, int L, const float2* tw, int kind,
                      hipStream_t st, const PlaneSums* sums) {
    switch (L) {
        case 32: cols_dispatch<4, 4>(R, outer, inner, tw, kind, st, sums); break;
        case 64: cols_dispatch<8, 4>(R, outer, inner, tw, kind, st, sums); break;
        case 128: cols_dispatch<8, 8>(R, outer, inner, tw, kind, st, sums); break;
        case 256: cols_dispatch<16, 8>(R, outer, inner, tw, kind, st, sums); break;
        default: cols_dispatch<16, 16>(R, outer, inner, tw, kind, st, sums); break;
    }
}

}  // namespace otd
