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

namespace otd {

constexpr int kT = 256;
constexpr int kTileFloats = 8192;     // 32 KB of LDS per tile buffer

// Forward table = M^T row-major (T[k*n + j] = M[j][k]); inverse table = M.
__device__ inline const float* fwd_tab(const AxisTab& t) { return t.mat; }
__device__ inline const float* inv_tab(const AxisTab& t) { return t.mat + (long long)t.n * t.n; }

__global__ void __launch_bounds__(kT) k_rows(float* R, long long rows, AxisTab t, int inverse,
                                            int rb) {
    extern __shared__ float tile[];
    const int L = t.n;
    const long long r0 = (long long)blockIdx.x * rb;
    const int nr = (int)min((long long)rb, rows - r0);
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

struct TcArgs {
    Geom g;
    float* R;
    AxisTab tx, ty, tc, tt;
    const double* tc64;      // C x C forward matrix M[j][k] (FP64)
    const double* tt64;      // P x P forward matrix M[j][k] (FP64)
    const double* lamc64;
    const double* lamt64;
    const double* part_slice;
    int nbx;
    int W;
};

__global__ void __launch_bounds__(kT) k_tc(TcArgs a) {
    extern __shared__ float lds[];
    const Geom& g = a.g;
    const int P = g.P, C = g.C, W = a.W;
    const int n = P * C * W;
    float* b1 = lds;
    float* b2 = lds + n;
    const int b = blockIdx.y;
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
    // spatial-DC line in FP64: S[k][c] = sum_{x,y} r, then the (c, t) Poisson
    // problem with eigenvalues lam_c + lam_t, scaled by 1 / sqrt(X Y).
    __syncthreads();
    double* d1 = reinterpret_cast<double*>(lds);
    double* d2 = d1 + P * C;
    const int m = P * C;
    for (int e = threadIdx.x; e < m; e += kT) {
        const double* pp = a.part_slice + ((long long)b * m + e) * a.nbx;
        double s = 0.0;
        for (int j = 0; j < a.nbx; ++j) s += pp[j];
        d1[e] = s;                                   // [k][c]
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m; e += kT) {      // colour forward
        const int k = e / C, jc = e - k * C;
        double acc = 0.0;
        for (int c = 0; c < C; ++c) acc += a.tc64[jc * C + c] * d1[k * C + c];
        d2[e] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m; e += kT) {      // time forward, divide
        const int jt = e / C, jc = e - jt * C;
        double acc = 0.0;
        for (int k = 0; k < P; ++k) acc += a.tt64[jt * P + k] * d2[k * C + jc];
        const double lam = a.lamc64[jc] + a.lamt64[jt];
        d1[e] = lam > 0.0 ? acc / lam : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m; e += kT) {      // time inverse
        const int k = e / C, jc = e - k * C;
        double acc = 0.0;
        for (int jt = 0; jt < P; ++jt) acc += a.tt64[jt * P + k] * d1[jt * C + jc];
        d2[e] = acc;
    }
    __syncthreads();
    const double scale = 1.0 / sqrt((double)g.plane);
    for (int e = threadIdx.x; e < m; e += kT) {      // colour inverse, store
        const int k = e / C, c = e - k * C;
        double acc = 0.0;
        for (int jc = 0; jc < C; ++jc) acc += a.tc64[jc * C + c] * d2[k * C + jc];
        base[(long long)k * g.slice + (long long)c * g.plane] = (float)(acc * scale);
    }
}

void launch_rows(float* R, long long rows, const AxisTab& t, int inverse, hipStream_t st) {
    const int L = t.n;
    int rb = kTileFloats / L;
    if (rb < 1) rb = 1;
    const long long nb = (rows + rb - 1) / rb;
    const size_t sh = (size_t)rb * L * sizeof(float);
    hipLaunchKernelGGL(k_rows, dim3((unsigned)nb), dim3(kT), sh, st, R, rows, t, inverse, rb);
}

void launch_cols(float* R, long long outer, long long inner, const AxisTab& t, int inverse,
                 hipStream_t st) {
    const int L = t.n;
    int W = 64;
    while (W > 1 && L * W > kTileFloats) W >>= 1;
    const long long nb = (inner + W - 1) / W;
    const size_t sh = (size_t)L * W * sizeof(float);
    hipLaunchKernelGGL(k_cols, dim3((unsigned)nb, (unsigned)outer), dim3(kT), sh, st, R, inner,
                       t, inverse, W);
}

void launch_tc(const Geom& g, float* R, const AxisTab& tx, const AxisTab& ty, const AxisTab& tc,
               const AxisTab& tt, const double* tc64, const double* tt64,
               const double* part_slice, int nbx, hipStream_t st) {
    TcArgs a;
    a.g = g; a.R = R; a.tx = tx; a.ty = ty; a.tc = tc; a.tt = tt;
    a.tc64 = tc64;
    a.tt64 = tt64;
    a.lamc64 = tc64 + (long long)g.C * g.C;
    a.lamt64 = tt64 + (long long)g.P * g.P;
    a.part_slice = part_slice;
    a.nbx = nbx;
    int W = 64;
    while (W > 1 && 2 * g.P * g.C * W > 2 * kTileFloats) W >>= 1;
    a.W = W;
    const long long nb = (g.plane + W - 1) / W;
    size_t sh = (size_t)2 * g.P * g.C * W * sizeof(float);
    const size_t sh64 = (size_t)2 * g.P * g.C * sizeof(double);
    if (sh64 > sh) sh = sh64;
    hipLaunchKernelGGL(k_tc, dim3((unsigned)nb, (unsigned)g.B), dim3(kT), sh, st, a);
}

}  // namespace otd
