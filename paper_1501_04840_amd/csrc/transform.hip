// Transform passes of the Poisson solve phi = (A A^T)^+ r (Sec. 3, Step 1 and
// Remark 2): A A^T is a sum of one 1D Laplacian per axis, diagonalised by the
// orthonormal DCT-II along Neumann axes (x, y, time) and by a real Fourier
// basis along periodic axes (here the discrete Hartley transform, whose
// basis cas(2 pi j k / n) / sqrt(n) diagonalises the symmetric circulant with
// the same eigenvalues 4 n^2 sin^2(pi j / n) as the Fourier matrix).
//
// Every pass is in place on the centred buffer R and stages its tile in LDS:
//   rows  -- contiguous axis (x): a tile of whole rows;
//   cols  -- strided axis (y):     a tile of L x W columns, W contiguous;
//   tc    -- colour and time lines of W contiguous (x, y) points, with the
//            division by the eigenvalues between forward and inverse; the
//            spatial-DC line (jx, jy) = (0, 0) is solved in FP64 from the
//            FP64 plane sums of r.
// These are dense contractions with the n x n matrix (table T[k][j], lanes
// over j, so table reads are coalesced and LDS reads are broadcasts).
#include "otd_common.h"
#include "fft_common.h"
#include "fft_lines.h"

#pragma clang fp contract(on)   // as in fft_common.h

namespace otd {

constexpr int kT = 256;
constexpr int kTileFloats = 8192;     // 32 KB of LDS per tile buffer

// Forward table = M^T row-major (T[k*n + j] = M[j][k]); inverse table = M.
__device__ inline const float* fwd_tab(const AxisTab& t) { return t.mat; }
__device__ inline const float* inv_tab(const AxisTab& t) { return t.mat + (long long)t.n * t.n; }

__global__ void __launch_bounds__(kT) k_rows(float* R, long long rows, AxisTab t, int inverse,
                                            int rb, RowSkip skip) {
    extern __shared__ float tile[];
    const int L = t.n;
    const long long r0 = (long long)blockIdx.x * rb;
    const int nr = (int)min((long long)rb, rows - r0);
    if (rows_frozen(skip, r0, nr)) return;
    const int cnt = nr * L;
    float* g = R + r0 * L;
    for (int e = threadIdx.x; e < cnt; e += kT) tile[e] = g[e];
    __syncthreads();
    const float* T = inverse ? inv_tab(t) : fwd_tab(t);
    for (int e = threadIdx.x; e < cnt; e += kT) {
        const int r = e / L, j = e - r * L;
        const float* in = tile + r * L;
        float acc = 0.f;
        for (int k = 0; k < L; ++k) acc = fmaf(T[k * L + j], in[k], acc);
        g[e] = acc;
    }
}

// Dense row transform on the matrix cores, for lengths without a fast path
// (the periodic hue axes of 180 and 360 bins, image sides like 100): a block
// owns 32 rows, staged in LDS with zero padding to Lp (a multiple of 32), and
// each of its Lp / 32 waves computes one 32 x 32 output tile of Y = X T with
// MFMA 32x32x2 FP32 steps over k (lane l supplies X[l % 32][k0 + l / 32] and
// T[k0 + l / 32][j0 + l % 32]; the result lands at row 8 (r / 4) + 4 (l / 32)
// + r % 4, column l % 32 of the tile).  The matrix operand comes from L2 in
// chunks of 16 steps whose loads are all in flight before the chunk's MFMAs.
typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int kMfmaRowsMaxL = 480;     // 32 rows of Lp + 1 floats stay under 64 KB

__device__ __forceinline__ int mfma_row(int r, int half) { return (r >> 2) * 8 + half * 4 + (r & 3); }

__global__ void __launch_bounds__(1024) k_rows_mfma(float* R, long long rows, AxisTab t, int inverse,
                                                  int Lp, RowSkip skip) {
    extern __shared__ float xs[];
    const int L = t.n, pitch = Lp + 1, nt = blockDim.x;
    const long long r0 = (long long)blockIdx.x * 32;
    const int nr = (int)min((long long)32, rows - r0);
    if (rows_frozen(skip, r0, nr)) return;
    float* g = R + r0 * L;
    for (int e = threadIdx.x; e < 32 * Lp; e += nt) {
        const int r = e / Lp, k = e - r * Lp;
        xs[r * pitch + k] = (r < nr && k < L) ? g[(long long)r * L + k] : 0.f;
    }
    __syncthreads();
    const float* T = inverse ? inv_tab(t) : fwd_tab(t);      // T[k * L + j]
    const int lane = threadIdx.x & 63, jt = threadIdx.x >> 6, n = lane & 31, half = lane >> 5;
    const int j = jt * 32 + n;
    const bool jin = j < L;
    f32x16 acc = {};
    for (int k0 = 0; k0 < Lp; k0 += 32) {
        float bv[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int k = k0 + 2 * q + half;
            bv[q] = (jin && k < L) ? T[(long long)k * L + j] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q)
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(xs[n * pitch + k0 + 2 * q + half], bv[q], acc,
                                                       0, 0, 0);
    }
    if (!jin) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = mfma_row(r, half);
        if (row < nr) g[(long long)row * L + j] = acc[r];
    }
}

// The same contraction along a strided axis (data [outer][L][inner]): a block
// owns 32 columns i of one outer index, staged as [k][i] (rows of 32
// consecutive floats), and each wave computes one 32-row tile of
// Y[j][i] = sum_k T[k][j] X[k][i] with the matrix as the MFMA A operand (lane
// l supplies T[k0 + l / 32][j0 + l % 32]) and the data as B (X[k0 + l / 32][l % 32]).
__global__ void __launch_bounds__(1024) k_cols_mfma(float* R, long long inner, AxisTab t, int inverse,
                                                  int Lp) {
    extern __shared__ float xs[];
    constexpr int pitch = 33;
    const int L = t.n, nt = blockDim.x;
    const long long o = blockIdx.y;
    const long long i0 = (long long)blockIdx.x * 32;
    const int nw = (int)min((long long)32, inner - i0);
    float* g = R + o * L * inner + i0;
    for (int e = threadIdx.x; e < Lp * 32; e += nt) {
        const int k = e >> 5, i = e & 31;
        xs[k * pitch + i] = (k < L && i < nw) ? g[(long long)k * inner + i] : 0.f;
    }
    __syncthreads();
    const float* T = inverse ? inv_tab(t) : fwd_tab(t);      // T[k * L + j]
    const int lane = threadIdx.x & 63, jt = threadIdx.x >> 6, n = lane & 31, half = lane >> 5;
    const int jA = jt * 32 + n;          // output row supplied by this lane's A value
    f32x16 acc = {};
    for (int k0 = 0; k0 < Lp; k0 += 32) {
        float av[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int k = k0 + 2 * q + half;
            av[q] = (jA < L && k < L) ? T[(long long)k * L + jA] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q)
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[q], xs[(k0 + 2 * q + half) * pitch + n], acc,
                                                       0, 0, 0);
    }
    if (n >= nw) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int jj = jt * 32 + mfma_row(r, half);
        if (jj < L) g[(long long)jj * inner + n] = acc[r];
    }
}

__global__ void __launch_bounds__(kT) k_cols(float* R, long long inner, AxisTab t, int inverse,
                                            int W) {
    extern __shared__ float tile[];
    const int L = t.n;
    const long long o = blockIdx.y;
    const long long i0 = (long long)blockIdx.x * W;
    const int nw = (int)min((long long)W, inner - i0);
    float* g = R + o * L * inner + i0;
    for (int e = threadIdx.x; e < L * W; e += kT) {
        const int k = e / W, i = e - k * W;
        tile[e] = i < nw ? g[(long long)k * inner + i] : 0.f;
    }
    __syncthreads();
    const float* T = inverse ? inv_tab(t) : fwd_tab(t);
    for (int e = threadIdx.x; e < L * W; e += kT) {
        const int j = e / W, i = e - j * W;
        if (i >= nw) continue;
        float acc = 0.f;
        for (int k = 0; k < L; ++k) acc = fmaf(T[k * L + j], tile[k * W + i], acc);
        g[(long long)j * inner + i] = acc;
    }
}

// Slots per plane of the DC-line reduction (1: one thread sums a plane) and
// the doubles of LDS it needs for m = P C planes: the line, its transform
// and the slot sums.
__host__ __device__ constexpr int dc_slots(int m) {
    int S = 16;
    while (S > 1 && m * S > 2048) S >>= 1;
    return S;
}
__host__ __device__ constexpr int dc_scratch_doubles(int m) {
    const int S = dc_slots(m);
    return 2 * m + (S > 1 ? m * S : 0);
}

struct TcArgs {
    Geom g;
    float* R;
    float* Rt;               // fused path: transposed scratch [B][C][X][Y][P]
    AxisTab tx, ty, tc, tt;
    const double* tc64;      // C x C forward matrix M[j][k] (FP64), then the C eigenvalues
    const double* tt64;      // P x P forward matrix M[j][k] (FP64), then the P eigenvalues
    double* part_slice;        // [B][P][C][nbx] FP64 block partials of the plane sums
    int nbx;
    int presummed;           // 1: part_slice[q nbx] already holds the sum of plane q
    const float* frz;        // per problem: nonzero = frozen, skipped (or null)
    int W;
    int premixed;            // fused x pass: r is already in colour modes
    const float2* twt;       // time-axis twiddles e^{-i pi j / (2P)}, j < 4P
};

template <int PT = 0>
__device__ void dc_line_fp64(const TcArgs& a, int b, double* d1, float* ct_out = nullptr);

__global__ void __launch_bounds__(kT) k_tc(TcArgs a) {
    extern __shared__ float lds[];
    const Geom& g = a.g;
    const int P = g.P, C = g.C, W = a.W;
    const int n = P * C * W;
    float* b1 = lds;
    float* b2 = lds + n;
    const int b = blockIdx.y;
    if (a.frz && a.frz[b] != 0.f) return;   // frozen problem (block-uniform)
    const long long i0 = (long long)blockIdx.x * W;
    const int nw = (int)min((long long)W, g.plane - i0);
    float* base = a.R + (long long)b * g.nc + i0;
    // load [k][c][i]
    for (int e = threadIdx.x; e < n; e += kT) {
        const int kc = e / W, i = e - kc * W;
        const int k = kc / C, c = kc - k * C;
        b1[e] = i < nw ? base[(long long)k * g.slice + (long long)c * g.plane + i] : 0.f;
    }
    __syncthreads();
    const float* Tc = fwd_tab(a.tc);
    const float* Tt = fwd_tab(a.tt);
    // forward colour: b2[k][jc][i] = sum_c M_c[jc][c] b1[k][c][i]
    for (int e = threadIdx.x; e < n; e += kT) {
        const int kc = e / W, i = e - kc * W;
        const int k = kc / C, jc = kc - k * C;
        float acc = 0.f;
        for (int c = 0; c < C; ++c) acc = fmaf(Tc[c * C + jc], b1[(k * C + c) * W + i], acc);
        b2[e] = acc;
    }
    __syncthreads();
    // forward time and division: b1[jt][jc][i]
    for (int e = threadIdx.x; e < n; e += kT) {
        const int kc = e / W, i = e - kc * W;
        const int jt = kc / C, jc = kc - jt * C;
        float acc = 0.f;
        for (int k = 0; k < P; ++k) acc = fmaf(Tt[k * P + jt], b2[(k * C + jc) * W + i], acc);
        const long long p = i0 + i;
        const int jy = (int)(p / g.X), jx = (int)(p - (long long)jy * g.X);
        const float lam = (i < nw ? a.tx.lam[jx] + a.ty.lam[jy] : 1.f) + a.tc.lam[jc] +
                          a.tt.lam[jt];
        b1[e] = lam > 0.f ? acc / lam : 0.f;
    }
    __syncthreads();
    const float* Ut = inv_tab(a.tt);
    const float* Uc = inv_tab(a.tc);
    // inverse time: b2[k][jc][i] = sum_jt M_t[jt][k] b1[jt][jc][i]
    for (int e = threadIdx.x; e < n; e += kT) {
        const int kc = e / W, i = e - kc * W;
        const int k = kc / C, jc = kc - k * C;
        float acc = 0.f;
        for (int jt = 0; jt < P; ++jt) acc = fmaf(Ut[jt * P + k], b1[(jt * C + jc) * W + i], acc);
        b2[e] = acc;
    }
    __syncthreads();
    // inverse colour and store (the DC point of block 0 is written below)
    const bool dc_block = blockIdx.x == 0;
    for (int e = threadIdx.x; e < n; e += kT) {
        const int kc = e / W, i = e - kc * W;
        const int k = kc / C, c = kc - k * C;
        if (i >= nw || (dc_block && i == 0)) continue;
        float acc = 0.f;
        for (int jc = 0; jc < C; ++jc) acc = fmaf(Uc[jc * C + c], b2[(k * C + jc) * W + i], acc);
        base[(long long)k * g.slice + (long long)c * g.plane + i] = acc;
    }
    if (!dc_block) return;
    __syncthreads();
    dc_line_fp64(a, b, reinterpret_cast<double*>(lds));
}

// The (colour, time) problem of the spatial-DC line from the FP64 plane
// sums d1[q], q = (k, c), visible to the whole block (d1 and d1 + P C are
// overwritten); output as for dc_line_fp64.  PT > 0: P is the compile-time
// PT, and each thread issues the P loads of its row or column of the FP64
// time matrix at once (one round trip to the cache instead of one per eight
// terms: the time products were the serial part of the one-block solves).
// With TAB the time and colour matrices, each followed by its eigenvalues,
// come from tab (copies in LDS: P P + P doubles, then C C + C), else from
// a.tt64 and a.tc64.  The choice is made at compile time, so that LDS
// copies are read with LDS instructions (a pointer that may be either is a
// flat one, and a flat load waits behind every global load issued before it).
template <int PT, bool TAB = false>
__device__ __forceinline__ void dc_solve_fp64(const TcArgs& a, int b, double* d1, float* ct_out,
                                              const double* tab = nullptr) {
    const Geom& g = a.g;
    const int P = PT > 0 ? PT : g.P, C = g.C;
    const double* Tt = TAB ? tab : a.tt64;
    const double* Tc = TAB ? tab + P * P + P : a.tc64;
    const double* lamt = Tt + P * P;
    const double* lamc = Tc + C * C;
    const int nt = blockDim.x;
    float* base = a.R + (long long)b * g.nc;
    double* d2 = d1 + P * C;
    const int m = P * C;
    for (int e = threadIdx.x; e < m; e += nt) {      // colour forward
        const int k = e / C, jc = e - k * C;
        double acc = 0.0;
        for (int c = 0; c < C; ++c) acc += Tc[jc * C + c] * d1[k * C + c];
        d2[e] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m; e += nt) {      // time forward, divide
        const int jt = e / C, jc = e - jt * C;
        double acc = 0.0;
        if constexpr (PT > 0) {
            double w[PT];
#pragma unroll
            for (int k = 0; k < PT; ++k) w[k] = Tt[jt * PT + k];
#pragma unroll
            for (int k = 0; k < PT; ++k) acc += w[k] * d2[k * C + jc];
        } else {
#pragma unroll 8
            for (int k = 0; k < P; ++k) acc += Tt[jt * P + k] * d2[k * C + jc];
        }
        const double lam = lamc[jc] + lamt[jt];
        d1[e] = lam > 0.0 ? acc / lam : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m; e += nt) {      // time inverse
        const int k = e / C, jc = e - k * C;
        double acc = 0.0;
        if constexpr (PT > 0) {
            double w[PT];
#pragma unroll
            for (int jt = 0; jt < PT; ++jt) w[jt] = Tt[jt * PT + k];
#pragma unroll
            for (int jt = 0; jt < PT; ++jt) acc += w[jt] * d1[jt * C + jc];
        } else {
#pragma unroll 8
            for (int jt = 0; jt < P; ++jt) acc += Tt[jt * P + k] * d1[jt * C + jc];
        }
        d2[e] = acc;
    }
    __syncthreads();
    const double scale = 1.0 / sqrt((double)g.plane);
    if (ct_out) {
        for (int e = threadIdx.x; e < m; e += nt) {
            const int k = e / C, jc = e - k * C;
            ct_out[jc * P + k] = (float)(d2[e] * scale);
        }
        return;
    }
    for (int e = threadIdx.x; e < m; e += nt) {      // colour inverse, store
        const int k = e / C, c = e - k * C;
        double acc = 0.0;
        for (int jc = 0; jc < C; ++jc) acc += Tc[jc * C + c] * d2[k * C + jc];
        base[(long long)k * g.slice + (long long)c * g.plane] = (float)(acc * scale);
    }
}

// dc_solve_fp64 with the tables in LDS (tab as there) for a block of NT >=
// 8 P C threads: every time product (P terms) is split over 8 consecutive
// lanes, P / 8 terms each, and summed by shuffles, so that each phase is a
// few dependent steps instead of P.  Output to ct_out as dc_solve_fp64.
template <int P, int C, int NT>
__device__ __forceinline__ void dc_solve_wide(const TcArgs& a, double* d1, float* ct_out,
                                              const double* tab) {
    constexpr int m = P * C, KL = P / 8;
    static_assert(NT >= 8 * m && P % 8 == 0, "eight lanes per output");
    const double* Tt = tab;
    const double* lamt = tab + P * P;
    const double* Tc = tab + P * P + P;
    const double* lamc = Tc + C * C;
    double* d2 = d1 + m;
    const int tid = threadIdx.x, o = tid >> 3, l = tid & 7;
    if (tid < m) {                                   // colour forward
        const int k = tid / C, jc = tid - k * C;
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < C; ++c) acc += Tc[jc * C + c] * d1[k * C + c];
        d2[tid] = acc;
    }
    __syncthreads();
    if (o < m) {                                     // time forward, divide
        const int jt = o / C, jc = o - jt * C;
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < KL; ++i) {
            const int k = l + 8 * i;
            acc += Tt[jt * P + k] * d2[k * C + jc];
        }
        acc += __shfl_xor(acc, 4, 8);
        acc += __shfl_xor(acc, 2, 8);
        acc += __shfl_xor(acc, 1, 8);
        const double lam = lamc[jc] + lamt[jt];
        if (l == 0) d1[o] = lam > 0.0 ? acc / lam : 0.0;
    }
    __syncthreads();
    if (o < m) {                                     // time inverse
        const int k = o / C, jc = o - k * C;
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < KL; ++i) {
            const int jt = l + 8 * i;
            acc += Tt[jt * P + k] * d1[jt * C + jc];
        }
        acc += __shfl_xor(acc, 4, 8);
        acc += __shfl_xor(acc, 2, 8);
        acc += __shfl_xor(acc, 1, 8);
        if (l == 0) ct_out[jc * P + k] = (float)(acc * (1.0 / sqrt((double)a.g.plane)));
    }
}

// Spatial-DC line (jx, jy) = (0, 0) in FP64: S[k][c] = sum_{x,y} r from the
// FP64 plane sums, then the (colour, time) Poisson problem with eigenvalues
// lam_c + lam_t (zero mode dropped), scaled by 1 / sqrt(X Y); writes the
// line at p = 0 of problem b.  Called by a whole block; d1 holds
// dc_scratch_doubles(P C) doubles.  With ct_out the line is left in colour
// modes and written as ct_out[jc * P + t] (scaled) instead.
template <int PT>
__device__ void dc_line_fp64(const TcArgs& a, int b, double* d1, float* ct_out) {
    const Geom& g = a.g;
    const int P = g.P, C = g.C;
    const int nt = blockDim.x;
    double* d2 = d1 + P * C;
    const int m = P * C;
    // plane sums d1[q], q = (k, c), of the nbx block partials of each plane:
    // S slots per plane each sum every S-th partial (consecutive threads take
    // consecutive slots: coalesced loads, many in flight), then one thread
    // per plane adds its slots from LDS.  No shuffle trees: their chains of
    // dependent exchanges made this block the tail of the whole pass.
    const int S = dc_slots(m);
    const double* part = a.part_slice + (long long)b * m * a.nbx;
    if (a.presummed) {
        for (int q = threadIdx.x; q < m; q += nt) d1[q] = part[(long long)q * a.nbx];
    } else if (S > 1) {
        double* slot = d2 + m;
        for (int e = threadIdx.x; e < m * S; e += nt) {
            const int q = e / S, j = e - q * S;
            const double* pp = part + (long long)q * a.nbx;
            // 16 loads in flight per round trip
            double v[16];
            double acc = 0.0;
            for (int i = j; i < a.nbx; i += 16 * S) {
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int ii = i + u * S;
                    v[u] = ii < a.nbx ? pp[ii] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 16; ++u) acc += v[u];
            }
            slot[e] = acc;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < m; q += nt) {
            double acc = 0.0;
            for (int j = 0; j < S; ++j) acc += slot[q * S + j];
            d1[q] = acc;
        }
    } else {
        for (int q = threadIdx.x; q < m; q += nt) {
            const double* pp = part + (long long)q * a.nbx;
            double acc = 0.0;
            for (int i = 0; i < a.nbx; ++i) acc += pp[i];
            d1[q] = acc;
        }
    }
    __syncthreads();
    dc_solve_fp64<PT>(a, b, d1, ct_out);
}

// dct3_reg<P>(diag(d) dct2_reg<P>(x)) = dct3_reg<P, true>(diag(d s) dct2_reg<P, true>(x))
// with s = dct2_scale<P>(j): the output scales of both and the factor sqrt 2
// the inverse applies to X[0], for a caller that scales every frequency anyway.
template <int P>
__device__ __forceinline__ constexpr float dct2_scale(int j) {
    constexpr float M = P / 2;
    const float sc = 0.5f * __builtin_sqrtf(0.5f * P) / M;
    return j == 0 ? sc * 1.41421356237309515f * 0.5f * __builtin_sqrtf(1.f / P)
                  : sc * 0.5f * __builtin_sqrtf(2.f / P);
}

// Orthonormal DCT-II of a register line of length P (Makhoul's reordering
// and a P/2-point packed DFT; every index is a compile-time constant).  The
// frequencies k and M - k are unpacked together: with 2 ve = Z[k] +
// conj Z[M-k] and 2 vo = -i (Z[k] - conj Z[M-k]), V[k] = ve + w vo and
// V[M-k] = conj(ve - w vo) for w = e^{-2 pi i k / P}.
template <int P, bool RAW = false>
__device__ __forceinline__ void dct2_reg(float (&x)[P], const float2* tw4) {
    constexpr int M = P / 2;
    float2 z[M];
#pragma unroll
    for (int n = 0; n < M; ++n) {
        const int m0 = 2 * n, m1 = 2 * n + 1;
        z[n] = make_float2(x[m0 < M ? 2 * m0 : 2 * P - 1 - 2 * m0],
                           x[m1 < M ? 2 * m1 : 2 * P - 1 - 2 * m1]);
    }
    dft<M>(z);
    // a = 2 V[k], b = 2 V[M-k]: the factor 1/2 is folded into the scales
    // (RAW: no scales, the caller applies dct2_scale)
    const float h = RAW ? 1.f : 0.5f * sqrtf(2.f / P), h0 = RAW ? 1.f : 0.5f * sqrtf(1.f / P);
#pragma unroll
    for (int k = 0; k <= M / 2; ++k) {
        const float2 zk = z[k], zm = z[(M - k) % M];
        const float2 ve = make_float2(zk.x + zm.x, zk.y - zm.y);
        const float2 vo = make_float2(zk.y + zm.y, zm.x - zk.x);
        const float2 p = cmul(tw4[4 * k], vo);
        const float2 xa = cmul(tw4[k], cadd(ve, p));
        const float2 xb = cmul(tw4[M - k], make_float2(ve.x - p.x, p.y - ve.y));
        x[k] = (k == 0 ? h0 : h) * xa.x;
        if (k > 0) x[P - k] = -h * xa.y;
        if (k < M / 2) {
            x[M - k] = h * xb.x;
            if (k > 0) x[M + k] = -h * xb.y;
        }
    }
}

// Orthonormal DCT-III (inverse of dct2_reg) of a register line.  With
// V(k) = conj(w4_k) (X[k], -X[P-k]) on inputs scaled by sqrt(P / 2)
// (sqrt(P) for X[0]): conj Z[k] = conj(ve + i vo) and conj Z[M-k] =
// ve - i vo, 2 ve = V(k) + conj V(M-k), 2 vo = (V(k) - conj V(M-k)) conj(w_k);
// the factor sqrt(P / 2) / 2 is applied to the outputs.
template <int P, bool RAW = false>
__device__ __forceinline__ void dct3_reg(float (&x)[P], const float2* tw4) {
    constexpr int M = P / 2;
    float2 zc[M];
#pragma unroll
    for (int k = 0; k <= M / 2; ++k) {
        const float xk = k == 0 && !RAW ? 1.41421356237309515f * x[0] : x[k];
        const float xl = k == 0 ? 0.f : x[P - k];                 // X[P-k]
        const float2 v = cmul(cconj(tw4[k]), make_float2(xk, -xl));
        const float2 w = cmul(cconj(tw4[M - k]), make_float2(x[M - k], -x[M + k]));   // V(M-k)
        const float2 ve = make_float2(v.x + w.x, v.y - w.y);
        const float2 vo = cmul(make_float2(v.x - w.x, v.y + w.y), cconj(tw4[4 * k]));
        zc[k] = make_float2(ve.x - vo.y, -(ve.y + vo.x));
        if (k > 0 && k < M / 2) zc[M - k] = make_float2(ve.x + vo.y, ve.y - vo.x);
    }
    dft<M>(zc);
    const float sc = RAW ? 1.f : 0.5f * sqrtf(0.5f * P) / M;
#pragma unroll
    for (int n = 0; n < M; ++n) {
        const int m0 = 2 * n, m1 = 2 * n + 1;
        x[m0 < M ? 2 * m0 : 2 * (P - 1 - m0) + 1] = zc[n].x * sc;
        x[m1 < M ? 2 * m1 : 2 * (P - 1 - m1) + 1] = -zc[n].y * sc;
    }
}

// Colour and time pass for power-of-two P: a block covers 64 consecutive
// (x, y) points; wave c loads colour c of them (coalesced) and, after a
// colour transform through LDS, owns colour mode c: time DCT-II in registers,
// division by the eigenvalues of A A^T, inverse DCT; the inverse colour
// transform goes back through LDS.  Block 0 of each problem instead solves
// the spatial-DC line (p = 0) in FP64.
template <int P, int C>
__global__ void __launch_bounds__(64 * C) k_tc_reg(TcArgs a) {
    extern __shared__ double dsh[];
    float* buf = reinterpret_cast<float*>(dsh);        // [C][P][64]
    const Geom& g = a.g;
    const int b = blockIdx.y;
    if (a.frz && a.frz[b] != 0.f) return;   // frozen problem (block-uniform)
    if (blockIdx.x == 0) {
        dc_line_fp64<P>(a, b, dsh);
        return;
    }
    const int lane = threadIdx.x & 63, c = threadIdx.x >> 6;
    const long long p = (long long)(blockIdx.x - 1) * 64 + lane;
    const bool live = p < g.plane;
    float* base = a.R + (long long)b * g.nc + (live ? p : 0) + (long long)c * g.plane;
    float u[P];
#pragma unroll
    for (int k = 0; k < P; ++k) u[k] = live ? base[(long long)k * g.slice] : 0.f;
    if constexpr (C > 1) {
#pragma unroll
        for (int k = 0; k < P; ++k) buf[(c * P + k) * 64 + lane] = u[k];
        __syncthreads();
        const float* Tc = a.tc.mat;                    // Tc[c' * C + jc] = M[jc][c']
#pragma unroll
        for (int k = 0; k < P; ++k) {
            float acc = 0.f;
#pragma unroll
            for (int cc = 0; cc < C; ++cc) acc = fmaf(Tc[cc * C + c], buf[(cc * P + k) * 64 + lane], acc);
            u[k] = acc;
        }
    }
    dct2_reg<P>(u, a.twt);
    const int jy = live ? (int)(p / g.X) : 0, jx = live ? (int)(p - (long long)jy * g.X) : 0;
    const float lc = a.tx.lam[jx] + a.ty.lam[jy] + a.tc.lam[c];
#pragma unroll
    for (int jt = 0; jt < P; ++jt) {
        const float lam = lc + a.tt.lam[jt];     // > 0 except the DC mode of p = 0
        u[jt] = lam > 0.f ? u[jt] * __builtin_amdgcn_rcpf(lam) : 0.f;
    }
    dct3_reg<P>(u, a.twt);
    if constexpr (C > 1) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < P; ++k) buf[(c * P + k) * 64 + lane] = u[k];
        __syncthreads();
        const float* Uc = a.tc.mat + C * C;            // Uc[jc * C + c'] = M[jc][c']
#pragma unroll
        for (int k = 0; k < P; ++k) {
            float acc = 0.f;
#pragma unroll
            for (int jc = 0; jc < C; ++jc) acc = fmaf(Uc[jc * C + c], buf[(jc * P + k) * 64 + lane], acc);
            u[k] = acc;
        }
    }
    if (!live || p == 0) return;
#pragma unroll
    for (int k = 0; k < P; ++k) base[(long long)k * g.slice] = u[k];
}

template <int P, int C>
static void tc_reg_launch(const TcArgs& a, hipStream_t st) {
    const unsigned nb = (unsigned)((a.g.plane + 63) / 64) + 1;
    size_t sh = (size_t)C * P * 64 * sizeof(float);
    const size_t sh64 = (size_t)dc_scratch_doubles(P * C) * sizeof(double);
    if (sh64 > sh) sh = sh64;
    hipLaunchKernelGGL((k_tc_reg<P, C>), dim3(nb, (unsigned)a.g.B), dim3(64 * C), sh, st, a);
}

static bool tc_reg_dispatch(const TcArgs& a, hipStream_t st) {
    if (!a.twt) return false;
    const int P = a.g.P, C = a.g.C;
#define OTD_TC(PP, CC) if (P == PP && C == CC) { tc_reg_launch<PP, CC>(a, st); return true; }
    OTD_TC(8, 1) OTD_TC(16, 1) OTD_TC(32, 1)
    OTD_TC(8, 3) OTD_TC(16, 3) OTD_TC(32, 3)
#undef OTD_TC
    return false;
}

// ---- fused Poisson passes (Neumann x and y of power-of-two length) -------
//
// Three passes instead of five.  A block of the first pass owns one row
// index y of one problem: the P C rows (t, c) of length X are staged in LDS,
// transformed along x (DCT-II), mixed across colours, and written to a
// transposed scratch Rt[b][jc][jx][y][t] (t fastest, so every (jc, jx) gets a
// contiguous run of P values).  A block of the second pass owns one (jc, jx):
// its Y x P values are contiguous in Rt; it transforms along y, then along t
// in registers (one thread per y line), divides by the eigenvalues of A A^T,
// inverts t and y, and writes back in place.  The third pass mirrors the
// first.  The spatial-DC line (jx, jy) = (0, 0) is solved in FP64 from the
// plane sums of r: the first pass reduces the divergence kernel's block
// partials of each plane in place (spread over its row blocks), the second
// leaves the line zero, and every block of the third solves it (a few small
// loads issued before its tile's, so the solve runs while the tile arrives)
// and adds it to the jx = 0 column, where after the inverse y transform it is
// the same value at every y.

constexpr int cmax(int a, int b) { return a > b ? a : b; }

// LDS layout of the lines of length 256 in the fused passes: a row pitch of
// 325 floats and 4 floats of padding after each row of the four-step
// exchange, which takes the line transforms' bank conflicts (8 lines of 8
// threads per wave) to about half of those of the pitch L + 1; other
// lengths keep L + 1 and no padding.
template <int L> constexpr int fused_xp() { return L == 256 ? 4 : 0; }
template <int L> constexpr int fused_pitch() { return L == 256 ? 325 : L + 1; }

// Row block of the x passes for hardware block hw of n: blocks are dispatched
// round-robin over the 8 XCDs (one L2 each), and XCD j gets the j-th
// contiguous eighth of the rows, so that the pieces of the transposed scratch
// one L2 holds (P values per (jc, jx) and row) are contiguous runs in memory
// rather than 128-byte pieces a kilobyte apart.
__device__ __forceinline__ int x_row_block(int hw, int n) {
    const int q = n >> 3, r = n & 7, xcd = hw & 7, slot = hw >> 3;
    return xcd * q + (xcd < r ? xcd : r) + slot;
}

// Slot j < S of a plane's sum of the nbx block partials pp[]: the partials
// j + u S of every run of 16 S, summed in order from `first` (the first run,
// already loaded); as dc_line_fp64 sums them.
template <int S>
__device__ __forceinline__ double plane_slot(const double* pp, int nbx, int j,
                                             const double (&first)[16]) {
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) acc += first[u];
    for (int i = j + 16 * S; i < nbx; i += 16 * S) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int ii = i + u * S;
            v[u] = ii < nbx ? pp[ii] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) acc += v[u];
    }
    return acc;
}

template <int S>
__device__ __forceinline__ void plane_first(const double* pp, int nbx, int j, double (&v)[16]) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int ii = j + u * S;
        v[u] = ii < nbx ? pp[ii] : 0.0;
    }
}

template <int M1, int M2, int C, int P, int PS>
__global__ void __launch_bounds__(PS * C * M2) k_xf_tr(TcArgs a) {
    constexpr int L = 2 * M1 * M2, T = M2, NL = PS * C, NT = NL * T, PITCH = fused_pitch<L>();
    constexpr int XP = fused_xp<L>();
    static_assert(PITCH >= M1 * (2 * M2 + XP), "exchange fits the line");
    constexpr int NE = L / T;                      // tile floats per thread
    static_assert(NE * NT == NL * L && NT % PS == 0, "tile split");
    constexpr int MP = P * C, S = dc_slots(MP);
    static_assert(S >= 2 && S <= NT, "plane-sum slots");
    __shared__ __align__(16) float lds[NL * PITCH];
    __shared__ double pslot[S];
    const Geom& g = a.g;
    const int b = blockIdx.y;
    // block: row index y, time slices t0 .. t0 + PS - 1
    const int nb = g.Y * (P / PS);
    const int lb = x_row_block(blockIdx.x, nb);
    const int y = lb / (P / PS), t0 = (lb - y * (P / PS)) * PS;
    // The plane sums of r for the DC line: this block reduces planes lb,
    // lb + nb, ... < P C in place (the sum replaces the plane's first
    // partial).  The first plane's partials are loaded before the tile, so
    // that waiting for them does not wait for the tile.
    double* const part = a.part_slice + (long long)b * MP * a.nbx;
    const bool psum = lb < MP && (int)threadIdx.x < S;
    double pv[16];
    if (psum) plane_first<S>(part + (long long)lb * a.nbx, a.nbx, threadIdx.x, pv);
    const float* src = a.R + (long long)b * g.nc + (long long)t0 * g.slice + (long long)y * L;
    // Single floats consecutive over the lanes (coalesced, all in flight,
    // conflict-free LDS writes).  When the block is whole wavefronts, each
    // wavefront loads exactly the LW lines it transforms and needs only a
    // wavefront sync before its transform, so that wavefronts whose loads
    // have arrived transform while the others still load; a smaller block
    // stages the tile together.  Offsets within a problem fit in 32 bits (at
    // most 256 x 256 x 3 x 32 values), so the loads take a uniform base and a
    // 32-bit offset.
    constexpr bool PERWAVE = NT % 64 == 0;
    constexpr int LANES = PERWAVE ? 64 : NT, LW = LANES / T;   // lines per staging group
    static_assert(LW * L == LANES * NE, "a group's lines are its lanes' loads");
    const unsigned slice = (unsigned)g.slice, plane = (unsigned)g.plane;
    const unsigned lane = threadIdx.x % LANES, l0 = (threadIdx.x / LANES) * LW;
    float buf[NE];
#pragma unroll
    for (int j = 0; j < NE; ++j) {
        const unsigned e = lane + LANES * j;
        const unsigned line = l0 + e / L, col = e % L, t = line / C, c = line % C;
        buf[j] = src[t * slice + c * plane + col];
    }
    if (psum) pslot[threadIdx.x] = plane_slot<S>(part + (long long)lb * a.nbx, a.nbx, threadIdx.x, pv);
#pragma unroll
    for (int j = 0; j < NE; ++j) {
        const unsigned e = lane + LANES * j;
        lds[(l0 + e / L) * PITCH + (e % L)] = buf[j];
    }
    if constexpr (PERWAVE) line_sync();            // the wavefront's own lines are staged
    else __syncthreads();
    const int line = threadIdx.x / T, tt = threadIdx.x - line * T;
    line_xform<M1, M2, 0, XP>(lds + line * PITCH, tt, a.tx.tw);
    // (the transform ends with a block barrier: pslot is complete)
    if (lb < MP && threadIdx.x == 0) {
        double acc = 0.0;
        for (int j = 0; j < S; ++j) acc += pslot[j];
        part[(long long)lb * a.nbx] = acc;
    }
    // further planes when the row blocks are fewer than the planes
    for (int q = lb + nb; q < MP; q += nb) {
        __syncthreads();                       // pslot is free again
        if ((int)threadIdx.x < S) {
            plane_first<S>(part + (long long)q * a.nbx, a.nbx, threadIdx.x, pv);
            pslot[threadIdx.x] = plane_slot<S>(part + (long long)q * a.nbx, a.nbx, threadIdx.x, pv);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double acc = 0.0;
            for (int j = 0; j < S; ++j) acc += pslot[j];
            part[(long long)q * a.nbx] = acc;
        }
    }
    if (C > 1 && !a.premixed) {
        const float* Tc = a.tc.mat;                    // Tc[c * C + jc] = M_c[jc][c]
        for (int q = threadIdx.x; q < PS * L; q += NT) {
            const int t = q / L, jx = q - t * L;
            float v[C];
#pragma unroll
            for (int c = 0; c < C; ++c) v[c] = lds[(t * C + c) * PITCH + jx];
#pragma unroll
            for (int jc = 0; jc < C; ++jc) {
                float acc = 0.f;
#pragma unroll
                for (int c = 0; c < C; ++c) acc = fmaf(Tc[c * C + jc], v[c], acc);
                lds[(t * C + jc) * PITCH + jx] = acc;
            }
        }
        __syncthreads();
    }
    // transposed store: a thread keeps its slice tq (NT is a multiple of PS)
    // and steps r = jc L + jx by NT / PS; every LDS read before the stores
    const unsigned tq = threadIdx.x % PS, r0 = threadIdx.x / PS, ys = (unsigned)(g.Y * P);
    float* dst = a.Rt + (long long)b * g.nc + (long long)y * P + t0;
#pragma unroll
    for (int j = 0; j < NE; ++j) {
        const unsigned r = r0 + (NT / PS) * j, jx = r % L, jc = r / L;
        buf[j] = lds[(tq * C + jc) * PITCH + jx];
    }
    const unsigned o0 = r0 * ys + tq, step = (NT / PS) * ys;
#pragma unroll
    for (int j = 0; j < NE; ++j) dst[o0 + j * step] = buf[j];
}

template <int M1, int M2, int C, int P, int PS>
__global__ void __launch_bounds__(PS * C * M2) k_xi_tr(TcArgs a) {
    constexpr int L = 2 * M1 * M2, T = M2, NL = PS * C, NT = NL * T, PITCH = fused_pitch<L>();
    constexpr int XP = fused_xp<L>();
    static_assert(PITCH >= M1 * (2 * M2 + XP), "exchange fits the line");
    constexpr int NE = L / T;                      // tile floats per thread
    static_assert(NE * NT == NL * L && NT % PS == 0, "tile split");
    __shared__ __align__(16) float lds[NL * PITCH];
    const Geom& g = a.g;
    // the DC line: plane sums (reduced in place by the forward pass) and the
    // FP64 time and colour tables, staged in LDS
    constexpr int MP = P * C, NTT = P * P + P, NTAB = NTT + C * C + C;
    constexpr int NDC = (MP + NTAB + NT - 1) / NT;     // DC inputs per thread
    __shared__ double dsh[2 * MP + NTAB];
    __shared__ float dcl[MP];                          // the line, [jc][t], scaled
    const int b = blockIdx.y;
    const int lb = x_row_block(blockIdx.x, g.Y * (P / PS));
    const int y = lb / (P / PS), t0 = (lb - y * (P / PS)) * PS;
    // its loads first: waiting for them then does not wait for the tile's
    const double* part = a.part_slice + (long long)b * MP * a.nbx;
    double dv[NDC];
#pragma unroll
    for (int r = 0; r < NDC; ++r) {
        const int i = threadIdx.x + NT * r;
        dv[r] = i < MP ? part[(long long)i * a.nbx]
                       : i < MP + NTT ? a.tt64[i - MP] : i < MP + NTAB ? a.tc64[i - MP - NTT] : 0.0;
    }
    // transposed load, the mirror of the forward pass's store: all loads in
    // flight before the first LDS write
    // (32-bit offsets from a uniform base, as in the forward pass)
    const unsigned tq = threadIdx.x % PS, r0 = threadIdx.x / PS, ys = (unsigned)(g.Y * P);
    const float* src = a.Rt + (long long)b * g.nc + (long long)y * P + t0;
    const unsigned o0 = r0 * ys + tq, step = (NT / PS) * ys;
    float buf[NE];
#pragma unroll
    for (int j = 0; j < NE; ++j) buf[j] = src[o0 + j * step];
    // the DC line while the tile arrives; the plane sums go to dsh[0, MP),
    // the tables behind the solve's scratch
#pragma unroll
    for (int r = 0; r < NDC; ++r) {
        const int i = threadIdx.x + NT * r;
        if (i < MP) dsh[i] = dv[r];
        else if (i < MP + NTAB) dsh[MP + i] = dv[r];
    }
    __syncthreads();
    if constexpr (NT >= 8 * MP) dc_solve_wide<P, C, NT>(a, dsh, dcl, dsh + 2 * MP);
    else dc_solve_fp64<0, true>(a, b, dsh, dcl, dsh + 2 * MP);
#pragma unroll
    for (int j = 0; j < NE; ++j) {
        const unsigned r = r0 + (NT / PS) * j, jx = r % L, jc = r / L;
        lds[(tq * C + jc) * PITCH + jx] = buf[j];
    }
    __syncthreads();
    // after the inverse y transform the line's coefficient c is c / sqrt(Y)
    // at every y (jx = 0 column, colour mode jc)
    if ((int)threadIdx.x < NL) {
        const int t = threadIdx.x / C, jc = threadIdx.x - t * C;
        lds[(t * C + jc) * PITCH] += dcl[jc * P + t0 + t] * (float)(1.0 / sqrt((double)g.Y));
    }
    __syncthreads();
    if constexpr (C > 1) {
        const float* Uc = a.tc.mat + C * C;            // Uc[jc * C + c] = M_c[jc][c]
        for (int q = threadIdx.x; q < PS * L; q += NT) {
            const int t = q / L, jx = q - t * L;
            float v[C];
#pragma unroll
            for (int jc = 0; jc < C; ++jc) v[jc] = lds[(t * C + jc) * PITCH + jx];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                float acc = 0.f;
#pragma unroll
                for (int jc = 0; jc < C; ++jc) acc = fmaf(Uc[jc * C + c], v[jc], acc);
                lds[(t * C + c) * PITCH + jx] = acc;
            }
        }
        __syncthreads();
    }
    // When the block is whole wavefronts, each wavefront stores the LW lines it
    // transformed as soon as they are done (the transform then ends with a
    // wavefront sync, not a block barrier); a smaller block stores together.
    constexpr bool PERWAVE = NT % 64 == 0;
    constexpr int LANES = PERWAVE ? 64 : NT, LW = LANES / T;
    static_assert(LW * L == LANES * NE, "a group's lines are its lanes' stores");
    const int line = threadIdx.x / T, tt = threadIdx.x - line * T;
    line_xform<M1, M2, 1, XP, !PERWAVE>(lds + line * PITCH, tt, a.tx.tw);
    float* dstb = a.R + (long long)b * g.nc + (long long)t0 * g.slice + (long long)y * L;
    const unsigned lane = threadIdx.x % LANES, l0 = (threadIdx.x / LANES) * LW;
#pragma unroll
    for (int j = 0; j < NE; ++j) {
        const unsigned e = lane + LANES * j;
        buf[j] = lds[(l0 + e / L) * PITCH + (e % L)];
    }
#pragma unroll
    for (int j = 0; j < NE; ++j) {
        const unsigned e = lane + LANES * j;
        const unsigned ln = l0 + e / L, col = e % L, ts = ln / C, c = ln % C;
        dstb[ts * (unsigned)g.slice + c * (unsigned)g.plane + col] = buf[j];
    }
}

template <int M1, int M2, int P, int NT>
__global__ void __launch_bounds__(NT) k_yt(TcArgs a) {
    constexpr int L = 2 * M1 * M2, T = M2, PITCH = fused_pitch<L>(), NLINES = cmax(P, NT / T);
    constexpr int XP = fused_xp<L>();
    static_assert(PITCH >= M1 * (2 * M2 + XP), "exchange fits the line");
    constexpr int NV = L * P / (4 * NT);
    static_assert(NV * 4 * NT == L * P, "tile must split into float4 per thread");
    __shared__ __align__(16) float lds[NLINES * PITCH];
    const Geom& g = a.g;
    const int b = blockIdx.y, jc = blockIdx.x / g.X, jx = blockIdx.x - jc * g.X;
    float* base = a.Rt + (long long)b * g.nc + (long long)blockIdx.x * L * P;
    // When the block's lines are exactly P time lines, LW to a wavefront
    // (LW a multiple of 4), each wavefront stages its own lines t0w ..
    // t0w + LW - 1 (LW / 4 float4 per y) and transforms them after a
    // wavefront sync, and stores them after its inverse transform the same
    // way; otherwise the block stages and stores the tile together.
    constexpr int LW = 64 / T;
    constexpr bool PERWAVE = NT % 64 == 0 && NT / T == P && LW % 4 == 0;
    constexpr int H = PERWAVE ? LW / 4 : 1;        // float4 per y and wavefront
    const int lane = (int)(threadIdx.x & 63), t0w = (int)(threadIdx.x >> 6) * LW;
    auto vidx = [&](int j) {                       // float4 index of the j-th load
        if constexpr (PERWAVE) {
            const int q = lane + 64 * j;
            return (q / H) * (P / 4) + t0w / 4 + q % H;
        } else {
            return (int)threadIdx.x + NT * j;
        }
    };
    float4 buf[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) buf[j] = reinterpret_cast<const float4*>(base)[vidx(j)];
    for (int e = P * PITCH + threadIdx.x; e < NLINES * PITCH; e += NT) lds[e] = 0.f;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const int e = 4 * vidx(j);
        const int y = e / P, t = e - y * P;
        lds[t * PITCH + y] = buf[j].x;
        lds[(t + 1) * PITCH + y] = buf[j].y;
        lds[(t + 2) * PITCH + y] = buf[j].z;
        lds[(t + 3) * PITCH + y] = buf[j].w;
    }
    if constexpr (PERWAVE) line_sync();            // the wavefront's own lines are staged
    else __syncthreads();
    const int line = threadIdx.x / T, tt = threadIdx.x - line * T;
    line_xform<M1, M2, 0, XP>(lds + line * PITCH, tt, a.ty.tw);
    const float lcx = a.tx.lam[jx] + a.tc.lam[jc];
    for (int jy = threadIdx.x; jy < L; jy += NT) {
        float u[P];
        if (jx == 0 && jy == 0) {      // the DC line: added by the inverse x pass
#pragma unroll
            for (int t = 0; t < P; ++t) u[t] = 0.f;
        } else {
#pragma unroll
            for (int t = 0; t < P; ++t) u[t] = lds[t * PITCH + jy];
            dct2_reg<P, true>(u, a.twt);
            const float lc = lcx + a.ty.lam[jy];
            // the eigenvalue sum is > 0 off the DC line (every lambda >= 0,
            // and jx or jy is not 0); the transforms' scales ride along
#pragma unroll
            for (int jt = 0; jt < P; ++jt)
                u[jt] = u[jt] * (dct2_scale<P>(jt) * __builtin_amdgcn_rcpf(lc + a.tt.lam[jt]));
            dct3_reg<P, true>(u, a.twt);
        }
#pragma unroll
        for (int t = 0; t < P; ++t) lds[t * PITCH + jy] = u[t];
    }
    __syncthreads();
    line_xform<M1, M2, 1, XP, !PERWAVE>(lds + line * PITCH, tt, a.ty.tw);
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const int e = 4 * vidx(j);
        const int y = e / P, t = e - y * P;
        reinterpret_cast<float4*>(base)[vidx(j)] =
            make_float4(lds[t * PITCH + y], lds[(t + 1) * PITCH + y], lds[(t + 2) * PITCH + y],
                        lds[(t + 3) * PITCH + y]);
    }
}

// Whole Poisson solve of a problem with one spatial axis (Y = C = 1, x of
// power-of-two length 64..256, P in {8, 16, 32}) in one block: the P x X
// tile of r stays in LDS; FP64 sums of its time rows give the spatial-DC
// line, solved in FP64 as in the colour/time pass; the rows are transformed
// along x (Hartley for periodic x, DCT-II for Neumann), every x-frequency
// column along t in registers with the division by the eigenvalues, and the
// rows back along x.  One launch instead of three for each iteration of the
// batched 1D (hue) problems.
template <int M1, int M2, int P, int NT, int KF, int KI>
__global__ void __launch_bounds__(NT) k_p1d(TcArgs a) {
    constexpr int L = 2 * M1 * M2, T = M2, PITCH = L + 1, NLINES = cmax(P, NT / T);
    constexpr int NS = L * P / NT, S = NT / P;
    static_assert(NS * NT == L * P, "tile must split into floats per thread");
    static_assert(S * P == NT && S >= 2, "row-sum slots");
    __shared__ __align__(16) float lds[NLINES * PITCH];
    __shared__ double dsum[NT + 2 * P];
    __shared__ float dcl[P];
    const Geom& g = a.g;
    const int b = blockIdx.x;
    if (a.frz && a.frz[b] != 0.f) return;   // frozen problem (block-uniform)
    float* base = a.R + (long long)b * g.nc;
    // single floats, consecutive over the threads (conflict-free LDS writes)
    float buf[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) buf[j] = base[threadIdx.x + NT * j];
    for (int e = P * PITCH + threadIdx.x; e < NLINES * PITCH; e += NT) lds[e] = 0.f;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const int e = (int)threadIdx.x + NT * j;
        lds[(e / L) * PITCH + (e % L)] = buf[j];
    }
    __syncthreads();
    {   // FP64 sums of the time rows: S slots per row, then one thread per row
        const int t = threadIdx.x / S, q = threadIdx.x - t * S;
        double acc = 0.0;
        for (int x = q; x < L; x += S) acc += (double)lds[t * PITCH + x];
        dsum[threadIdx.x] = acc;
    }
    __syncthreads();
    double* d1 = dsum + NT;
    if (threadIdx.x < P) {
        double acc = 0.0;
        for (int q = 0; q < S; ++q) acc += dsum[threadIdx.x * S + q];
        d1[threadIdx.x] = acc;
    }
    __syncthreads();
    dc_solve_fp64<P>(a, b, d1, dcl);
    __syncthreads();
    const int line = threadIdx.x / T, tt = threadIdx.x - line * T;
    line_xform<M1, M2, KF>(lds + line * PITCH, tt, a.tx.tw);
    for (int jx = threadIdx.x; jx < L; jx += NT) {
        float u[P];
        if (jx == 0) {
#pragma unroll
            for (int t = 0; t < P; ++t) u[t] = dcl[t];
        } else {
#pragma unroll
            for (int t = 0; t < P; ++t) u[t] = lds[t * PITCH + jx];
            dct2_reg<P>(u, a.twt);
            const float lx = a.tx.lam[jx];
#pragma unroll
            for (int jt = 0; jt < P; ++jt)
                u[jt] = u[jt] * __builtin_amdgcn_rcpf(lx + a.tt.lam[jt]);   // lx > 0 off the DC
            dct3_reg<P>(u, a.twt);
        }
#pragma unroll
        for (int t = 0; t < P; ++t) lds[t * PITCH + jx] = u[t];
    }
    __syncthreads();
    line_xform<M1, M2, KI>(lds + line * PITCH, tt, a.tx.tw);
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const int e = (int)threadIdx.x + NT * j;
        base[e] = lds[(e / L) * PITCH + (e % L)];
    }
}

// The one-block solve for an axis whose length 2 M1 M2 is not a power of
// two but has only the factors 2, 3 and 5 (the hue axes of 180 and 360
// bins): as k_p1d, with the mixed-radix transforms of fft_lines.h along x
// (Hartley for periodic x, KF = KI = 2; DCT-II / DCT-III for Neumann x)
// instead of the dense contraction on the matrix cores.  NT threads, a multiple of P and of 64, at least
// P M2; the rows are staged as in k_p1d.
template <int M1, int M2, int P, int NT, int KF, int KI>
__global__ void __launch_bounds__(NT) k_p1d_mix(TcArgs a) {
    constexpr int L = 2 * M1 * M2, T = M2, PITCH = L + 1, S = NT / P;
    static_assert(L % 4 == 0 && S * P == NT && S >= 2 && P * T <= NT, "block shape");
    __shared__ __align__(16) float lds[P * PITCH];
    __shared__ double dsum[NT + 2 * P];
    __shared__ float dcl[P];
    const Geom& g = a.g;
    const int b = blockIdx.x;
    if (a.frz && a.frz[b] != 0.f) return;   // frozen problem (block-uniform)
    float* base = a.R + (long long)b * g.nc;
    // single floats, consecutive over the threads (conflict-free LDS writes),
    // all of a thread's loads in flight at once
    constexpr int NS = (L * P + NT - 1) / NT;
    float buf[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const int e = (int)threadIdx.x + NT * j;
        buf[j] = e < L * P ? base[e] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const int e = (int)threadIdx.x + NT * j;
        if (e < L * P) lds[(e / L) * PITCH + (e % L)] = buf[j];
    }
    __syncthreads();
    {   // FP64 sums of the time rows: S slots per row, then one thread per row
        const int t = threadIdx.x / S, q = threadIdx.x - t * S;
        double acc = 0.0;
        for (int x = q; x < L; x += S) acc += (double)lds[t * PITCH + x];
        dsum[threadIdx.x] = acc;
    }
    __syncthreads();
    double* d1 = dsum + NT;
    if (threadIdx.x < P) {
        double acc = 0.0;
        for (int q = 0; q < S; ++q) acc += dsum[threadIdx.x * S + q];
        d1[threadIdx.x] = acc;
    }
    __syncthreads();
    dc_solve_fp64<P>(a, b, d1, dcl);
    __syncthreads();
    const int line = threadIdx.x / T, tt = threadIdx.x - line * T;
    const bool act = line < P;
    float* const sl = lds + (act ? line : 0) * PITCH;
    line_xform_mix<M1, M2, KF>(sl, tt, a.tx.twm, act);
    for (int jx = threadIdx.x; jx < L; jx += NT) {
        float u[P];
        if (jx == 0) {
#pragma unroll
            for (int t = 0; t < P; ++t) u[t] = dcl[t];
        } else {
#pragma unroll
            for (int t = 0; t < P; ++t) u[t] = lds[t * PITCH + jx];
            dct2_reg<P>(u, a.twt);
            const float lx = a.tx.lam[jx];
#pragma unroll
            for (int jt = 0; jt < P; ++jt)
                u[jt] = u[jt] * __builtin_amdgcn_rcpf(lx + a.tt.lam[jt]);   // lx > 0 off the DC
            dct3_reg<P>(u, a.twt);
        }
#pragma unroll
        for (int t = 0; t < P; ++t) lds[t * PITCH + jx] = u[t];
    }
    __syncthreads();
    line_xform_mix<M1, M2, KI>(sl, tt, a.tx.twm, act);
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const int e = (int)threadIdx.x + NT * j;
        if (e < L * P) base[e] = lds[(e / L) * PITCH + (e % L)];
    }
}

// The same one-block solve for one spatial axis without a fast transform
// (e.g. 180 or 360 periodic bins), X <= kMfmaRowsMaxL: the P time rows,
// padded with zero rows to 32, are the A operand of the dense x contraction
// on the matrix cores (as in k_rows_mfma: 2 Lp threads, one wave per 32
// output columns), forward and inverse, with the time pass and the FP64 DC
// line between them in LDS.
// k_p1d_dense: at most 8 waves (up to 256 VGPRs; with 2 Lp threads the
// register DCT along t spilled), each computing up to two 32-column tiles,
// so Lp <= 512; X <= 416 keeps the dynamic LDS (32 padded rows of Lp + 1
// floats plus the FP64 scratch) under 64 KB.
constexpr int kP1dDenseThreads = 512;
constexpr int kP1dDenseMaxL = 416;

template <int P>
__global__ void __launch_bounds__(kP1dDenseThreads) k_p1d_dense(TcArgs a, int Lp) {
    extern __shared__ double dyn[];
    const Geom& g = a.g;
    const int L = g.X, pitch = Lp + 1, nt = blockDim.x, S = nt / 32;
    const int nwave = nt >> 6, ntile = Lp / 32;       // a wave computes tiles w, w + nwave
    double* dsum = dyn;                               // [nt]
    double* d1 = dsum + nt;                           // [2 P]
    float* dcl = reinterpret_cast<float*>(d1 + 2 * P);   // [P]
    float* xs = dcl + P;                              // [32][pitch]
    const int b = blockIdx.x;
    if (a.frz && a.frz[b] != 0.f) return;   // frozen problem (block-uniform)
    float* base = a.R + (long long)b * g.nc;
    for (int e = threadIdx.x; e < 32 * Lp; e += nt) {
        const int r = e / Lp, k = e - r * Lp;
        xs[r * pitch + k] = (r < P && k < L) ? base[(long long)r * L + k] : 0.f;
    }
    __syncthreads();
    {   // FP64 sums of the time rows (S slots per row of the 32), the DC line
        const int t = threadIdx.x / S, q = threadIdx.x - t * S;
        double acc = 0.0;
        for (int x = q; x < L; x += S) acc += (double)xs[t * pitch + x];
        dsum[threadIdx.x] = acc;
    }
    __syncthreads();
    if (threadIdx.x < P) {
        double acc = 0.0;
        for (int q = 0; q < S; ++q) acc += dsum[threadIdx.x * S + q];
        d1[threadIdx.x] = acc;
    }
    __syncthreads();
    dc_solve_fp64<P>(a, b, d1, dcl);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n = lane & 31, half = lane >> 5;
    for (int pass = 0; pass < 2; ++pass) {
        const float* T = pass ? inv_tab(a.tx) : fwd_tab(a.tx);   // T[k * L + j]
        f32x16 acc[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            acc[i] = f32x16{};
            const int tile = wave + i * nwave;
            if (tile >= ntile) continue;                 // wave-uniform
            const int j = tile * 32 + n;
            const bool jin = j < L;
            for (int k0 = 0; k0 < Lp; k0 += 32) {
                float bv[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int k = k0 + 2 * q + half;
                    bv[q] = (jin && k < L) ? T[(long long)k * L + j] : 0.f;
                }
#pragma unroll
                for (int q = 0; q < 16; ++q)
                    acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(xs[n * pitch + k0 + 2 * q + half],
                                                                  bv[q], acc[i], 0, 0, 0);
            }
        }
        if (pass == 1) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int j = (wave + i * nwave) * 32 + n;
                if (wave + i * nwave < ntile && j < L)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int row = mfma_row(r, half);
                        if (row < P) base[(long long)row * L + j] = acc[i][r];
                    }
            }
            break;
        }
        __syncthreads();                    // every wave has read xs
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int tile = wave + i * nwave;
            if (tile >= ntile) continue;
            const int j = tile * 32 + n;
#pragma unroll
            for (int r = 0; r < 16; ++r) xs[mfma_row(r, half) * pitch + j] = j < L ? acc[i][r] : 0.f;
        }
        __syncthreads();
        for (int jx = threadIdx.x; jx < L; jx += nt) {
            float u[P];
            if (jx == 0) {
#pragma unroll
                for (int t = 0; t < P; ++t) u[t] = dcl[t];
            } else {
#pragma unroll
                for (int t = 0; t < P; ++t) u[t] = xs[t * pitch + jx];
                dct2_reg<P>(u, a.twt);
                const float lx = a.tx.lam[jx];
#pragma unroll
                for (int jt2 = 0; jt2 < P; ++jt2)
                    u[jt2] = u[jt2] * __builtin_amdgcn_rcpf(lx + a.tt.lam[jt2]);   // lx > 0 off the DC
                dct3_reg<P>(u, a.twt);
            }
#pragma unroll
            for (int t = 0; t < P; ++t) xs[t * pitch + jx] = u[t];
        }
        __syncthreads();
    }
}

template <int M1, int M2, int P>
static void p1d_launch(const TcArgs& a, hipStream_t st) {
    constexpr int NT = cmax(64, P * M2);
    const dim3 grid((unsigned)a.g.B);
    if (a.g.perx)
        hipLaunchKernelGGL((k_p1d<M1, M2, P, NT, 2, 2>), grid, dim3(NT), 0, st, a);
    else
        hipLaunchKernelGGL((k_p1d<M1, M2, P, NT, 0, 1>), grid, dim3(NT), 0, st, a);
}

template <int P>
static bool p1d_dispatch(const TcArgs& a, hipStream_t st) {
    switch (a.g.X) {
        case 64: p1d_launch<8, 4, P>(a, st); return true;
        case 128: p1d_launch<8, 8, P>(a, st); return true;
        case 256: p1d_launch<16, 8, P>(a, st); return true;
        default: return false;
    }
}

template <int M1, int M2, int P>
static void p1d_mix_launch(const TcArgs& a, hipStream_t st) {
    constexpr int NT0 = P * M2, NT = (NT0 + 63) / 64 * 64;
    static_assert(NT % P == 0, "row-sum slots");
    if (a.g.perx)
        hipLaunchKernelGGL((k_p1d_mix<M1, M2, P, NT, 2, 2>), dim3((unsigned)a.g.B), dim3(NT), 0, st, a);
    else
        hipLaunchKernelGGL((k_p1d_mix<M1, M2, P, NT, 0, 1>), dim3((unsigned)a.g.B), dim3(NT), 0, st, a);
}

template <int P>
static void p1d_mix_dispatch(const TcArgs& a, hipStream_t st) {
    if (a.g.X == 100) p1d_mix_launch<5, 10, P>(a, st);
    else if (a.g.X == 180) p1d_mix_launch<6, 15, P>(a, st);
    else p1d_mix_launch<12, 15, P>(a, st);
}

bool poisson_1d_ok(const Geom& g, const AxisTab& tx, const AxisTab& tt) {
    if (g.Y != 1 || g.C != 1 || !tt.tw || !(g.P == 8 || g.P == 16 || g.P == 32)) return false;
    if (tx.tw) return g.X == 64 || g.X == 128 || g.X == 256;
    return g.X >= 2 && g.X <= kP1dDenseMaxL;
}

template <int P>
static void p1d_dense_launch(const TcArgs& a, hipStream_t st) {
    const int Lp = (a.g.X + 31) / 32 * 32, nt = std::min(2 * Lp, kP1dDenseThreads);
    const size_t sh = ((size_t)nt + 2 * P) * sizeof(double) + (size_t)P * sizeof(float) +
                      (size_t)32 * (Lp + 1) * sizeof(float);
    hipLaunchKernelGGL((k_p1d_dense<P>), dim3((unsigned)a.g.B), dim3(nt), sh, st, a, Lp);
}

void launch_poisson_1d(const Geom& g, float* R, const AxisTab& tx, const AxisTab& ty,
                       const AxisTab& tc, const AxisTab& tt, const double* tc64,
                       const double* tt64, const float* frz, hipStream_t st) {
    TcArgs a{};
    a.g = g; a.R = R; a.tx = tx; a.ty = ty; a.tc = tc; a.tt = tt;
    a.tc64 = tc64;
    a.tt64 = tt64;
    a.frz = frz;
    a.twt = tt.tw;
    if (!tx.tw && tx.twm) {
        if (g.P == 8) p1d_mix_dispatch<8>(a, st);
        else if (g.P == 16) p1d_mix_dispatch<16>(a, st);
        else p1d_mix_dispatch<32>(a, st);
        return;
    }
    if (!tx.tw) {
        if (g.P == 8) p1d_dense_launch<8>(a, st);
        else if (g.P == 16) p1d_dense_launch<16>(a, st);
        else p1d_dense_launch<32>(a, st);
        return;
    }
    if (g.P == 8) p1d_dispatch<8>(a, st);
    else if (g.P == 16) p1d_dispatch<16>(a, st);
    else p1d_dispatch<32>(a, st);
}

// Time slices per block of the x passes: all of them (blocks of half the
// slices write 64-byte runs and measured slower at 256 x 256 x 3 x 32).
template <int M1, int M2, int C, int P>
static void xpair_launch(const TcArgs& a, int inverse, hipStream_t st) {
    constexpr int PS = P, NT = PS * C * M2;
    const unsigned nb = (unsigned)a.g.Y * (P / PS);
    if (!inverse)
        hipLaunchKernelGGL((k_xf_tr<M1, M2, C, P, PS>), dim3(nb, (unsigned)a.g.B), dim3(NT), 0, st,
                           a);
    else
        hipLaunchKernelGGL((k_xi_tr<M1, M2, C, P, PS>), dim3(nb, (unsigned)a.g.B), dim3(NT), 0, st,
                           a);
}

template <int C, int P>
static bool x_dispatch(const TcArgs& a, int inverse, hipStream_t st) {
    switch (a.g.X) {
        case 32: xpair_launch<4, 4, C, P>(a, inverse, st); return true;
        case 64: xpair_launch<8, 4, C, P>(a, inverse, st); return true;
        case 128: xpair_launch<8, 8, C, P>(a, inverse, st); return true;
        case 256: xpair_launch<16, 8, C, P>(a, inverse, st); return true;
        default: return false;
    }
}

template <int P>
static bool y_dispatch(const TcArgs& a, hipStream_t st) {
    const dim3 grid((unsigned)(a.g.C * a.g.X), (unsigned)a.g.B);
    switch (a.g.Y) {
        case 32: hipLaunchKernelGGL((k_yt<4, 4, P, cmax(64, P * 4)>), grid, dim3(cmax(64, P * 4)), 0, st, a); return true;
        case 64: hipLaunchKernelGGL((k_yt<8, 4, P, cmax(64, P * 4)>), grid, dim3(cmax(64, P * 4)), 0, st, a); return true;
        case 128: hipLaunchKernelGGL((k_yt<8, 8, P, cmax(64, P * 8)>), grid, dim3(cmax(64, P * 8)), 0, st, a); return true;
        case 256: hipLaunchKernelGGL((k_yt<16, 8, P, cmax(64, P * 8)>), grid, dim3(cmax(64, P * 8)), 0, st, a); return true;
        default: return false;
    }
}

bool fused_poisson_ok(const Geom& g, const AxisTab& tx, const AxisTab& ty, const AxisTab& tt) {
    auto len_ok = [](int n) { return n == 32 || n == 64 || n == 128 || n == 256; };
    return len_ok(g.X) && len_ok(g.Y) && !g.perx && !g.pery && tx.tw && ty.tw && tt.tw &&
           (g.P == 8 || g.P == 16 || g.P == 32) && (g.C == 1 || g.C == 3);
}

static TcArgs fused_args(const Geom& g, float* R, float* Rt, const AxisTab& tx,
                         const AxisTab& ty, const AxisTab& tc, const AxisTab& tt,
                         const double* tc64, const double* tt64, double* part_slice,
                         int nbx) {
    TcArgs a{};
    a.g = g; a.R = R; a.Rt = Rt; a.tx = tx; a.ty = ty; a.tc = tc; a.tt = tt;
    a.tc64 = tc64;
    a.tt64 = tt64;
    a.part_slice = part_slice;
    a.nbx = nbx;
    a.twt = tt.tw;
    return a;
}

void launch_fused_x(const Geom& g, float* R, float* Rt, const AxisTab& tx,
                    const AxisTab& ty, const AxisTab& tc, const AxisTab& tt, const double* tc64,
                    const double* tt64, double* part_slice, int nbx, int inverse,
                    bool premixed, hipStream_t st) {
    TcArgs a = fused_args(g, R, Rt, tx, ty, tc, tt, tc64, tt64, part_slice, nbx);
    a.premixed = !inverse && premixed;
#define OTD_FX(CC, PP) if (g.C == CC && g.P == PP) { x_dispatch<CC, PP>(a, inverse, st); return; }
    OTD_FX(1, 8) OTD_FX(1, 16) OTD_FX(1, 32) OTD_FX(3, 8) OTD_FX(3, 16) OTD_FX(3, 32)
#undef OTD_FX
}

void launch_fused_yt(const Geom& g, float* Rt, const AxisTab& tx, const AxisTab& ty,
                     const AxisTab& tc, const AxisTab& tt, hipStream_t st) {
    const TcArgs a = fused_args(g, nullptr, Rt, tx, ty, tc, tt, nullptr, nullptr, nullptr, 0);
    if (g.P == 8) y_dispatch<8>(a, st);
    else if (g.P == 16) y_dispatch<16>(a, st);
    else y_dispatch<32>(a, st);
}

bool launch_rows(float* R, long long rows, const AxisTab& t, int inverse, hipStream_t st,
                 const PlaneSums* sums, RowSkip skip) {
    if (t.tw) {
        launch_rows_fast(R, rows, t.n, t.tw, t.periodic ? 2 : (inverse ? 1 : 0), st, sums, skip);
        return sums != nullptr;
    }
    if (t.twm) {
        launch_rows_mix(R, rows, t.n, t.twm, t.periodic ? 2 : (inverse ? 1 : 0), st, sums, skip);
        return sums != nullptr;
    }
    const int L = t.n;
    if (L <= kMfmaRowsMaxL) {
        const int Lp = (L + 31) / 32 * 32;
        const size_t sh = (size_t)32 * (Lp + 1) * sizeof(float);
        hipLaunchKernelGGL(k_rows_mfma, dim3((unsigned)((rows + 31) / 32)), dim3(2 * Lp), sh, st, R,
                           rows, t, inverse, Lp, skip);
        return false;
    }
    int rb = kTileFloats / L;
    if (rb < 1) rb = 1;
    const long long nb = (rows + rb - 1) / rb;
    const size_t sh = (size_t)rb * L * sizeof(float);
    hipLaunchKernelGGL(k_rows, dim3((unsigned)nb), dim3(kT), sh, st, R, rows, t, inverse, rb, skip);
    return false;
}

bool launch_cols(float* R, long long outer, long long inner, const AxisTab& t, int inverse,
                 hipStream_t st, const PlaneSums* sums) {
    if (t.tw) {
        launch_cols_fast(R, outer, inner, t.n, t.tw, t.periodic ? 2 : (inverse ? 1 : 0), st, sums);
        return sums != nullptr;
    }
    if (t.twm) {
        launch_cols_mix(R, outer, inner, t.n, t.twm, t.periodic ? 2 : (inverse ? 1 : 0), st, sums);
        return sums != nullptr;
    }
    const int L = t.n;
    if (L <= kMfmaRowsMaxL) {
        const int Lp = (L + 31) / 32 * 32;
        const size_t sh = (size_t)Lp * 33 * sizeof(float);
        hipLaunchKernelGGL(k_cols_mfma, dim3((unsigned)((inner + 31) / 32), (unsigned)outer),
                           dim3(2 * Lp), sh, st, R, inner, t, inverse, Lp);
        return false;
    }
    int W = 64;
    while (W > 1 && L * W > kTileFloats) W >>= 1;
    const long long nb = (inner + W - 1) / W;
    const size_t sh = (size_t)L * W * sizeof(float);
    hipLaunchKernelGGL(k_cols, dim3((unsigned)nb, (unsigned)outer), dim3(kT), sh, st, R, inner,
                       t, inverse, W);
    return false;
}

void launch_tc(const Geom& g, float* R, const AxisTab& tx, const AxisTab& ty, const AxisTab& tc,
               const AxisTab& tt, const double* tc64, const double* tt64,
               double* part_slice, int nbx, int presummed, const float* frz,
               hipStream_t st) {
    TcArgs a{};
    a.g = g; a.R = R; a.tx = tx; a.ty = ty; a.tc = tc; a.tt = tt;
    a.tc64 = tc64;
    a.tt64 = tt64;
    a.part_slice = part_slice;
    a.nbx = nbx;
    a.presummed = presummed;
    a.frz = frz;
    a.twt = tt.tw;
    if (tc_reg_dispatch(a, st)) return;
    int W = 64;
    while (W > 1 && 2 * g.P * g.C * W > 2 * kTileFloats) W >>= 1;
    a.W = W;
    const long long nb = (g.plane + W - 1) / W;
    size_t sh = (size_t)2 * g.P * g.C * W * sizeof(float);
    const size_t sh64 = (size_t)dc_scratch_doubles(g.P * g.C) * sizeof(double);
    if (sh64 > sh) sh = sh64;
    hipLaunchKernelGGL(k_tc, dim3((unsigned)nb, (unsigned)g.B), dim3(kT), sh, st, a);
}

}  // namespace otd
