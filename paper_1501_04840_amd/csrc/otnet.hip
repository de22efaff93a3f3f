// Kernels of the warm-start network: convolutions as implicit GEMMs on the
// gfx950 matrix cores (BF16 operands, FP32 accumulation) and the pooling,
// upsampling, loss, optimiser and layout pieces around them.
#include "net_common.h"

namespace otn {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kThreads = 256;
constexpr int BK = 32;          // K depth of one LDS stage
constexpr int LDK = BK + 8;     // LDS row pitch (elements): 80 bytes

// Round to nearest even (finite inputs).
__device__ inline bf16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}
__device__ inline float bf2f(bf16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline void unpack8(const uint4& v, float* f) {
    const bf16_t* h = reinterpret_cast<const bf16_t*>(&v);
#pragma unroll
    for (int q = 0; q < 8; ++q) f[q] = bf2f(h[q]);
}
__device__ inline uint4 pack8(const float* f) {
    uint4 v;
    bf16_t* h = reinterpret_cast<bf16_t*>(&v);
#pragma unroll
    for (int q = 0; q < 8; ++q) h[q] = f2bf(f[q]);
    return v;
}

// Eight consecutive K entries (one tap, channels c..c+7) of row `pix` of the
// gathered operand; zero outside the image or past k_end.
__device__ inline uint4 conv_gather(const ConvArgs& a, int pix, int k, int k_end) {
    uint4 v = make_uint4(0, 0, 0, 0);
    if (pix >= a.M || k >= k_end) return v;
    const int tap = k / a.cin, c = k - tap * a.cin;
    const int hw = a.H * a.W;
    const int b = pix / hw, r = pix - b * hw;
    int y = r / a.W, x = r - (r / a.W) * a.W;
    if (a.taps == 9) {
        y += tap / 3 - 1;
        x += tap % 3 - 1;
        if (y < 0 || y >= a.H || x < 0 || x >= a.W) return v;
    }
    return *reinterpret_cast<const uint4*>(a.src + ((long long)(b * a.H + y) * a.W + x) * a.src_ld + c);
}

// Eight consecutive rows i0..i0+7 (one tap, channels c..c+7, or the ones row)
// of the weight-gradient operand at pixel q.
__device__ inline uint4 wgrad_gather(const ConvArgs& a, int i0, int q, int k_end) {
    uint4 v = make_uint4(0, 0, 0, 0);
    const int rows = a.taps * a.cin;
    if (q >= k_end || i0 > rows) return v;
    if (i0 == rows) {                       // bias row: (1, 0, ..., 0)
        v.x = 0x3F80u;
        return v;
    }
    const int tap = i0 / a.cin, c = i0 - tap * a.cin;
    const int hw = a.H * a.W;
    const int b = q / hw, r = q - b * hw;
    int y = r / a.W, x = r - (r / a.W) * a.W;
    if (a.taps == 9) {
        y += tap / 3 - 1;
        x += tap % 3 - 1;
        if (y < 0 || y >= a.H || x < 0 || x >= a.W) return v;
    }
    return *reinterpret_cast<const uint4*>(a.src + ((long long)(b * a.H + y) * a.W + x) * a.src_ld + c);
}

// Block tile BM x BN, four waves of 32 x 32 each (WN = BN / 32 along N).
// Per K stage the block stages A (BM x BK) and B (BN x BK) in LDS with K
// contiguous; a wave issues BK / 16 MFMA 32x32x16 on its sub-tile.
// Lane l of a wave holds A rows (l mod 32), K entries 8 (l / 32) + 0..7; the
// accumulator entry r of lane l is row 8 (r / 4) + 4 (l / 32) + r mod 4,
// column l mod 32.
template <int BM, int BN, int MODE, int EPI>
__global__ void __launch_bounds__(kThreads) k_conv(ConvArgs a) {
    static_assert(BM * BN == 4 * 32 * 32, "four 32x32 wave tiles");
    __shared__ __attribute__((aligned(16))) bf16_t As[BM * LDK];
    __shared__ __attribute__((aligned(16))) bf16_t Bs[BN * LDK];
    constexpr int WN = BN / 32;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    int k_begin = 0, k_end = a.K;
    if (MODE == MODE_WGRAD) {
        k_begin = blockIdx.z * a.ksplit;
        k_end = min(a.K, k_begin + a.ksplit);
    }
    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;

    for (int k0 = k_begin; k0 < k_end; k0 += BK) {
        if (MODE == MODE_CONV) {
#pragma unroll
            for (int e = t; e < BM * BK / 8; e += kThreads) {
                const int i = e / (BK / 8), kr = (e % (BK / 8)) * 8;
                const uint4 v = conv_gather(a, m0 + i, k0 + kr, k_end);
                *reinterpret_cast<uint4*>(&As[i * LDK + kr]) = v;
            }
#pragma unroll
            for (int e = t; e < BN * BK / 8; e += kThreads) {
                const int j = e / (BK / 8), kr = (e % (BK / 8)) * 8;
                uint4 v = make_uint4(0, 0, 0, 0);
                if (n0 + j < a.N && k0 + kr < k_end)
                    v = *reinterpret_cast<const uint4*>(a.wmat + (long long)(n0 + j) * a.K + k0 + kr);
                *reinterpret_cast<uint4*>(&Bs[j * LDK + kr]) = v;
            }
        } else {
#pragma unroll
            for (int e = t; e < BM * BK / 8; e += kThreads) {
                const int kk = e / (BM / 8), ir = (e % (BM / 8)) * 8;
                const uint4 v = wgrad_gather(a, m0 + ir, k0 + kk, k_end);
                const bf16_t* h = reinterpret_cast<const bf16_t*>(&v);
#pragma unroll
                for (int q = 0; q < 8; ++q) As[(ir + q) * LDK + kk] = h[q];
            }
#pragma unroll
            for (int e = t; e < BN * BK / 8; e += kThreads) {
                const int kk = e / (BN / 8), jr = (e % (BN / 8)) * 8;
                uint4 v = make_uint4(0, 0, 0, 0);
                if (k0 + kk < k_end && n0 + jr < a.N)
                    v = *reinterpret_cast<const uint4*>(a.dz + (long long)(k0 + kk) * a.dz_ld + n0 + jr);
                const bf16_t* h = reinterpret_cast<const bf16_t*>(&v);
#pragma unroll
                for (int q = 0; q < 8; ++q) Bs[(jr + q) * LDK + kk] = h[q];
            }
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < BK; ks += 16) {
            const int kq = ks + 8 * (lane >> 5);
            const bf16x8 fa = *reinterpret_cast<const bf16x8*>(&As[(wm * 32 + (lane & 31)) * LDK + kq]);
            const bf16x8 fb = *reinterpret_cast<const bf16x8*>(&Bs[(wn * 32 + (lane & 31)) * LDK + kq]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa, fb, acc, 0, 0, 0);
        }
        __syncthreads();
    }

    const int col = n0 + wn * 32 + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        if (row >= a.M || col >= a.dst_n) continue;
        float v = acc[r];
        if (EPI == EPI_PART) {
            reinterpret_cast<float*>(a.dst)[((long long)blockIdx.z * a.M + row) * a.N + col] = v;
            continue;
        }
        const long long o = (long long)row * a.dst_ld + a.dst_off + col;
        if (EPI == EPI_RELU || EPI == EPI_F32) v += a.bias[col];
        if (EPI == EPI_RELU) v = fmaxf(v, 0.f);
        if (EPI == EPI_MASK && !(bf2f(a.mask[(long long)row * a.mask_ld + col]) > 0.f)) v = 0.f;
        if (EPI == EPI_F32)
            reinterpret_cast<float*>(a.dst)[o] = v;
        else
            reinterpret_cast<bf16_t*>(a.dst)[o] = f2bf(v);
    }
}

template <int BM, int BN>
void conv_dispatch(const ConvArgs& a, int mode, int epi, dim3 grid, hipStream_t st) {
    if (mode == MODE_WGRAD) {
        hipLaunchKernelGGL((k_conv<BM, BN, MODE_WGRAD, EPI_PART>), grid, dim3(kThreads), 0, st, a);
        return;
    }
    switch (epi) {
        case EPI_RELU:
            hipLaunchKernelGGL((k_conv<BM, BN, MODE_CONV, EPI_RELU>), grid, dim3(kThreads), 0, st, a);
            break;
        case EPI_F32:
            hipLaunchKernelGGL((k_conv<BM, BN, MODE_CONV, EPI_F32>), grid, dim3(kThreads), 0, st, a);
            break;
        case EPI_PLAIN:
            hipLaunchKernelGGL((k_conv<BM, BN, MODE_CONV, EPI_PLAIN>), grid, dim3(kThreads), 0, st, a);
            break;
        default:
            hipLaunchKernelGGL((k_conv<BM, BN, MODE_CONV, EPI_MASK>), grid, dim3(kThreads), 0, st, a);
            break;
    }
}

__global__ void __launch_bounds__(kThreads) k_wgrad_reduce(const float* part, int splits,
                                                          long long mn, float* out) {
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= mn) return;
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += part[z * mn + i];
    out[i] = s;
}

__global__ void __launch_bounds__(kThreads) k_pack_input(const float* x, int in_ch, long long npix,
                                                        bf16_t* out, int ld) {
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= npix * ld) return;
    const long long p = i / ld;
    const int c = (int)(i - p * ld);
    out[i] = c < in_ch ? f2bf(x[p * in_ch + c]) : (bf16_t)0;
}

// dst[b][y][x][c] = mean of the 2x2 source block (8 channels per thread).
__global__ void __launch_bounds__(kThreads) k_pool(View src, int C, int nb, int H, int W,
                                                  bf16_t* dst) {
    const int h = H / 2, w = W / 2, c8 = C / 8;
    const long long n = (long long)nb * h * w * c8;
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const int c = (int)(i % c8) * 8;
    const long long p = i / c8;
    const int x = (int)(p % w), y = (int)((p / w) % h), b = (int)(p / ((long long)w * h));
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
            const long long q = ((long long)(b * H + 2 * y + dy) * W + 2 * x + dx);
            float f[8];
            unpack8(*reinterpret_cast<const uint4*>(src.ptr + q * src.ld + c), f);
#pragma unroll
            for (int e = 0; e < 8; ++e) acc[e] += f[e];
        }
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[e] *= 0.25f;
    *reinterpret_cast<uint4*>(dst + p * C + c) = pack8(acc);
}

// dst (2h x 2w, channels [0, C)) = nearest upsampling of src (h x w x C).
__global__ void __launch_bounds__(kThreads) k_upsample(const bf16_t* src, int C, int nb, int h,
                                                      int w, View dst) {
    const int H = 2 * h, W = 2 * w, c8 = C / 8;
    const long long n = (long long)nb * H * W * c8;
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const int c = (int)(i % c8) * 8;
    const long long p = i / c8;
    const int x = (int)(p % W), y = (int)((p / W) % H), b = (int)(p / ((long long)W * H));
    const long long q = (long long)(b * h + y / 2) * w + x / 2;
    *reinterpret_cast<uint4*>(dst.ptr + p * dst.ld + c) =
        *reinterpret_cast<const uint4*>(src + q * C + c);
}

// out (h x w x C) = (sum of the 2x2 block of g's channels [0, C)) masked by
// hlow > 0: the gradient through upsampling into the ReLU that fed it.
__global__ void __launch_bounds__(kThreads) k_up_bwd(View g, int C, int nb, int h, int w,
                                                    const bf16_t* hlow, bf16_t* out) {
    const int W = 2 * w, c8 = C / 8;
    const long long n = (long long)nb * h * w * c8;
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const int c = (int)(i % c8) * 8;
    const long long p = i / c8;
    const int x = (int)(p % w), y = (int)((p / w) % h), b = (int)(p / ((long long)w * h));
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
            const long long q = (long long)(b * 2 * h + 2 * y + dy) * W + 2 * x + dx;
            float f[8];
            unpack8(*reinterpret_cast<const uint4*>(g.ptr + q * g.ld + c), f);
#pragma unroll
            for (int e = 0; e < 8; ++e) acc[e] += f[e];
        }
    float m[8];
    unpack8(*reinterpret_cast<const uint4*>(hlow + p * C + c), m);
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[e] = m[e] > 0.f ? acc[e] : 0.f;
    *reinterpret_cast<uint4*>(out + p * C + c) = pack8(acc);
}

// out (H x W x C) = (gpool at the pooled pixel / 4 + gcat) masked by cat > 0:
// the two gradient paths into an encoder level's output, through its ReLU.
__global__ void __launch_bounds__(kThreads) k_merge(const bf16_t* gpool, View gcat, View cat, int C,
                                                   int nb, int H, int W, bf16_t* out) {
    const int c8 = C / 8;
    const long long n = (long long)nb * H * W * c8;
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const int c = (int)(i % c8) * 8;
    const long long p = i / c8;
    const int x = (int)(p % W), y = (int)((p / W) % H), b = (int)(p / ((long long)W * H));
    const long long q = (long long)(b * (H / 2) + y / 2) * (W / 2) + x / 2;
    float a[8], g[8], m[8];
    unpack8(*reinterpret_cast<const uint4*>(gpool + q * C + c), a);
    unpack8(*reinterpret_cast<const uint4*>(gcat.ptr + p * gcat.ld + c), g);
    unpack8(*reinterpret_cast<const uint4*>(cat.ptr + p * cat.ld + c), m);
#pragma unroll
    for (int e = 0; e < 8; ++e) a[e] = m[e] > 0.f ? 0.25f * a[e] + g[e] : 0.f;
    *reinterpret_cast<uint4*>(out + p * C + c) = pack8(a);
}

__device__ inline double block_sum_d(double v) {
    __shared__ double red[kThreads / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < kThreads / 64; ++q) s += red[q];
    return s;
}

constexpr int kLossPer = 16;    // elements per thread of the loss kernel

// dy = d loss / d y (BF16, padded channels 0) and the loss per block (FP64).
__global__ void __launch_bounds__(kThreads) k_loss(const float* y, const float* t, const float* cw,
                                                  int out_ch, int out_p, long long npix,
                                                  bf16_t* dy, double* part) {
    const long long n = npix * out_p;
    const long long base = (long long)blockIdx.x * kThreads * kLossPer;
    const double inv = 1.0 / (double)npix;
    double s = 0.0;
    for (int e = 0; e < kLossPer; ++e) {
        const long long i = base + (long long)e * kThreads + threadIdx.x;
        if (i >= n) break;
        const long long p = i / out_p;
        const int c = (int)(i - p * out_p);
        float g = 0.f;
        if (c < out_ch) {
            const float d = y[p * out_ch + c] - t[p * out_ch + c];
            s += (double)cw[c] * (double)d * (double)d * inv;
            g = (float)(2.0 * cw[c] * inv) * d;
        }
        dy[i] = f2bf(g);
    }
    s = block_sum_d(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kThreads) k_sum(const double* part, int n, double* out) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kThreads) s += part[i];
    s = block_sum_d(s);
    if (threadIdx.x == 0) *out = s;
}

__global__ void __launch_bounds__(kThreads) k_adam(float* p, float* m, float* v, const float* g,
                                                  long long n, float lr, float b1, float b2,
                                                  float eps, float c1, float c2) {
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// BF16 copies of one layer's weights w[tap][ci][co]: wf[co][tap][ci] for the
// forward GEMM and wb[ci][taps-1-tap][co] for the input-gradient GEMM.
__global__ void __launch_bounds__(kThreads) k_export(const float* w, int taps, int cin, int cout,
                                                    bf16_t* wf, bf16_t* wb) {
    const long long n = (long long)taps * cin * cout;
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const int co = (int)(i % cout);
    const int ci = (int)((i / cout) % cin);
    const int tap = (int)(i / ((long long)cout * cin));
    const bf16_t h = f2bf(w[i]);
    wf[((long long)co * taps + tap) * cin + ci] = h;
    wb[((long long)ci * taps + (taps - 1 - tap)) * cout + co] = h;
}

// One layer between the flat exchange layout (cin_o, cout_o) and the padded
// device layout (cin_p, cout_p); padded entries read as 0.
__global__ void __launch_bounds__(kThreads) k_param_map(const float* src, float* dst, int taps,
                                                       int cin_o, int cout_o, int cin_p,
                                                       int cout_p, int to_padded) {
    const long long np = (long long)taps * cin_p * cout_p + cout_p;
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= np) return;
    const long long nw = (long long)taps * cin_p * cout_p;
    long long o = -1;
    if (i < nw) {
        const int co = (int)(i % cout_p);
        const int ci = (int)((i / cout_p) % cin_p);
        const int tap = (int)(i / ((long long)cout_p * cin_p));
        if (co < cout_o && ci < cin_o) o = ((long long)tap * cin_o + ci) * cout_o + co;
    } else {
        const int co = (int)(i - nw);
        if (co < cout_o) o = (long long)taps * cin_o * cout_o + co;
    }
    if (to_padded)
        dst[i] = o >= 0 ? src[o] : 0.f;
    else if (o >= 0)
        dst[o] = src[i];
}

// ---- solver glue ----------------------------------------------------------

// x[b][y][x] = (f0 channels, f1 channels, then base channels if base is given).
__global__ void __launch_bounds__(kThreads) k_warm_inputs(WarmGeom g, int nb, const float* f0,
                                                         const float* f1, const float* base,
                                                         float* x) {
    const long long plane = (long long)g.X * g.Y;
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= nb * plane) return;
    const long long b = i / plane, p = i - b * plane;
    const int nch = g.C * (g.P - 1) + 3 * g.C * g.P;
    const int in_ch = 2 * g.C + (base ? nch : 0);
    float* o = x + i * in_ch;
    for (int c = 0; c < g.C; ++c) {
        o[c] = f0[(b * g.C + c) * plane + p];
        o[g.C + c] = f1[(b * g.C + c) * plane + p];
    }
    if (base)
        for (int q = 0; q < nch; ++q) o[2 * g.C + q] = base[i * nch + q];
}

// One thread per pixel; mode 0 writes the target (state minus base) from
// the state, mode 1 the state from a network output (plus base).
template <int MODE>
__global__ void __launch_bounds__(kThreads) k_warm_map(WarmGeom g, int nb, const float* f0,
                                                      const float* f1, const float* Fr, float* Fw,
                                                      long long sF, const float* Mxr,
                                                      const float* Myr, const float* Mcr,
                                                      float* Mxw, float* Myw, float* Mcw,
                                                      long long sM, const float* yr,
                                                      const float* base, float* tw) {
    const long long plane = (long long)g.X * g.Y;
    const long long slice = plane * g.C;
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= nb * plane) return;
    const long long b = i / plane, p = i - b * plane;
    const int x = (int)(p % g.X), y = (int)(p / g.X);
    const int P = g.P, C = g.C;
    const int nch = C * (P - 1) + 3 * C * P;
    const long long tb = i * nch;
    for (int k = 1; k < P; ++k) {
        const float s = (float)k / (float)P;
        for (int c = 0; c < C; ++c) {
            const long long e = (b * C + c) * plane + p;
            const float lin = (1.f - s) * f0[e] + s * f1[e];
            const long long fi = b * sF + k * slice + (long long)c * plane + p;
            const long long ti = tb + (k - 1) * C + c;
            const float bs = base ? base[ti] : 0.f;
            if (MODE == 0)
                tw[ti] = Fr[fi] - lin - bs;
            else
                Fw[fi] = lin + yr[ti] + bs;
        }
    }
    const long long o0 = (long long)C * (P - 1);
    for (int q = 0; q < 3; ++q) {
        const bool wallrow = (q == 0 && !g.perx && x == 0) || (q == 1 && !g.pery && y == 0);
        for (int k = 0; k < P; ++k)
            for (int c = 0; c < C; ++c) {
                const bool wall = wallrow || (q == 2 && !g.perc && c == 0);
                const long long mi = b * sM + k * slice + (long long)c * plane + p;
                const long long ti = tb + o0 + ((long long)q * P + k) * C + c;
                const float bs = base ? base[ti] : 0.f;
                if (MODE == 0) {
                    const float* M = q == 0 ? Mxr : (q == 1 ? Myr : Mcr);
                    tw[ti] = wall ? 0.f : M[mi] - bs;
                } else {
                    float* M = q == 0 ? Mxw : (q == 1 ? Myw : Mcw);
                    M[mi] = wall ? 0.f : yr[ti] + bs;
                }
            }
    }
}

// fc = 2 x 2 block means of f (coarse X, Y of gc; the fine grid is twice as
// wide and high).
__global__ void __launch_bounds__(kThreads) k_restrict(WarmGeom gc, int nb, const float* f,
                                                      float* fc) {
    const long long pc = (long long)gc.X * gc.Y;
    const long long n = nb * gc.C * pc;
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const long long bc = i / pc, p = i - bc * pc;
    const int x = (int)(p % gc.X), y = (int)(p / gc.X);
    const int X = 2 * gc.X;
    const float* s = f + bc * 4 * pc + (long long)(2 * y) * X + 2 * x;
    fc[i] = 0.25f * (s[0] + s[1] + s[X] + s[X + 1]);
}

// Linear interpolation weight and the two neighbours of position u on an
// axis of n samples at integer positions (clamped at the ends, or wrapped).
struct Lerp {
    int a, b;
    float w;
};
__device__ inline Lerp lerp_at(float u, int n, int periodic) {
    int i0 = (int)floorf(u);
    Lerp r;
    r.w = u - (float)i0;
    if (periodic) {
        r.a = ((i0 % n) + n) % n;
        r.b = (r.a + 1) % n;
    } else {
        r.a = min(max(i0, 0), n - 1);
        r.b = min(max(i0 + 1, 0), n - 1);
    }
    return r;
}

// Prolong a coarse state (X/2, Y/2, same C, P_c steps) to the fine grid:
// bilinear in space for cell-centred values, linear between faces for the
// staggered momenta (walls read as 0), linear in time.  Writes the unknown
// slices of F and every slot of Mx, My, Mc.
__global__ void __launch_bounds__(kThreads) k_prolong(WarmGeom gc, WarmGeom gf, int nb,
                                                     const float* Fc, long long sFc,
                                                     const float* Mxc, const float* Myc,
                                                     const float* Mcc, long long sMc, float* F,
                                                     long long sF, float* Mx, float* My,
                                                     float* Mc, long long sM) {
    const long long plane = (long long)gf.X * gf.Y;
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= nb * plane) return;
    const long long b = i / plane, p = i - b * plane;
    const int x = (int)(p % gf.X), y = (int)(p / gf.X);
    const long long pc = (long long)gc.X * gc.Y, slc = pc * gc.C, slf = plane * gf.C;
    const float rt = (float)gc.P / (float)gf.P;
    // cell-centred positions of this fine cell on the coarse grid
    const Lerp cx = lerp_at(0.5f * x - 0.25f, gc.X, gf.perx);
    const Lerp cy = lerp_at(0.5f * y - 0.25f, gc.Y, gf.pery);
    auto centred = [&](const float* A, long long off) -> float {
        const float* r0 = A + off + (long long)cy.a * gc.X;
        const float* r1 = A + off + (long long)cy.b * gc.X;
        const float v0 = (1.f - cx.w) * r0[cx.a] + cx.w * r0[cx.b];
        const float v1 = (1.f - cx.w) * r1[cx.a] + cx.w * r1[cx.b];
        return (1.f - cy.w) * v0 + cy.w * v1;
    };
    // coarse face value along an axis: slot j of n faces, walls at 0 and n
    auto face = [&](const float* row, int j, int n, int stride, int periodic) -> float {
        if (periodic) return row[(long long)(((j % n) + n) % n) * stride];
        return (j <= 0 || j >= n) ? 0.f : row[(long long)j * stride];
    };
    for (int k = 1; k < gf.P; ++k) {
        float s = k * rt;
        int j0 = min((int)floorf(s), gc.P - 1);
        const float a = s - (float)j0;
        for (int c = 0; c < gf.C; ++c) {
            const long long o0 = b * sFc + j0 * slc + (long long)c * pc;
            const float v = (1.f - a) * centred(Fc, o0) + a * centred(Fc, o0 + slc);
            F[b * sF + k * slf + (long long)c * plane + p] = v;
        }
    }
    for (int k = 0; k < gf.P; ++k) {
        const Lerp ct = lerp_at((k + 0.5f) * rt - 0.5f, gc.P, 0);
        for (int c = 0; c < gf.C; ++c) {
            const long long mi = b * sM + k * slf + (long long)c * plane + p;
            float vt[3] = {0.f, 0.f, 0.f};
            for (int h = 0; h < 2; ++h) {
                const int kc = h ? ct.b : ct.a;
                const float wt = h ? ct.w : 1.f - ct.w;
                const long long oc = b * sMc + kc * slc + (long long)c * pc;
                // x faces: fine slot x sits at coarse face position x / 2
                {
                    const int j0 = x >> 1;
                    const float w = (x & 1) ? 0.5f : 0.f;
                    const float* r0 = Mxc + oc + (long long)cy.a * gc.X;
                    const float* r1 = Mxc + oc + (long long)cy.b * gc.X;
                    const float v0 = (1.f - w) * face(r0, j0, gc.X, 1, gf.perx) + w * face(r0, j0 + 1, gc.X, 1, gf.perx);
                    const float v1 = (1.f - w) * face(r1, j0, gc.X, 1, gf.perx) + w * face(r1, j0 + 1, gc.X, 1, gf.perx);
                    vt[0] += wt * ((1.f - cy.w) * v0 + cy.w * v1);
                }
                {
                    const int j0 = y >> 1;
                    const float w = (y & 1) ? 0.5f : 0.f;
                    const float* c0 = Myc + oc + cx.a;
                    const float* c1 = Myc + oc + cx.b;
                    const float v0 = (1.f - w) * face(c0, j0, gc.Y, gc.X, gf.pery) + w * face(c0, j0 + 1, gc.Y, gc.X, gf.pery);
                    const float v1 = (1.f - w) * face(c1, j0, gc.Y, gc.X, gf.pery) + w * face(c1, j0 + 1, gc.Y, gc.X, gf.pery);
                    vt[1] += wt * ((1.f - cx.w) * v0 + cx.w * v1);
                }
                vt[2] += wt * centred(Mcc, oc);
            }
            const bool wx = !gf.perx && x == 0, wy = !gf.pery && y == 0, wc = !gf.perc && c == 0;
            Mx[mi] = wx ? 0.f : vt[0];
            My[mi] = wy ? 0.f : vt[1];
            Mc[mi] = wc ? 0.f : vt[2];
        }
    }
}

inline unsigned blocks(long long n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

void launch_conv(const ConvArgs& a, int mode, int epi, int splits, hipStream_t st) {
    const bool narrow = a.N <= 32;
    if (narrow) {
        const dim3 grid((a.M + 127) / 128, (a.N + 31) / 32, mode == MODE_WGRAD ? splits : 1);
        conv_dispatch<128, 32>(a, mode, epi, grid, st);
    } else {
        const dim3 grid((a.M + 63) / 64, (a.N + 63) / 64, mode == MODE_WGRAD ? splits : 1);
        conv_dispatch<64, 64>(a, mode, epi, grid, st);
    }
}

void launch_wgrad_reduce(const float* part, int splits, int M, int N, float* out, hipStream_t st) {
    const long long mn = (long long)M * N;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(blocks(mn)), dim3(kThreads), 0, st, part, splits, mn, out);
}

void launch_pack_input(const float* x, int in_ch, long long npix, bf16_t* out, int ld,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_pack_input, dim3(blocks(npix * ld)), dim3(kThreads), 0, st, x, in_ch, npix,
                       out, ld);
}

void launch_pool(View src, int C, int nb, int H, int W, bf16_t* dst, hipStream_t st) {
    const long long n = (long long)nb * (H / 2) * (W / 2) * (C / 8);
    hipLaunchKernelGGL(k_pool, dim3(blocks(n)), dim3(kThreads), 0, st, src, C, nb, H, W, dst);
}

void launch_upsample(const bf16_t* src, int C, int nb, int h, int w, View dst, hipStream_t st) {
    const long long n = (long long)nb * 4 * h * w * (C / 8);
    hipLaunchKernelGGL(k_upsample, dim3(blocks(n)), dim3(kThreads), 0, st, src, C, nb, h, w, dst);
}

void launch_up_bwd(View g, int C, int nb, int h, int w, const bf16_t* hlow, bf16_t* out,
                   hipStream_t st) {
    const long long n = (long long)nb * h * w * (C / 8);
    hipLaunchKernelGGL(k_up_bwd, dim3(blocks(n)), dim3(kThreads), 0, st, g, C, nb, h, w, hlow, out);
}

void launch_merge(const bf16_t* gpool, View gcat, View cat, int C, int nb, int H, int W,
                  bf16_t* out, hipStream_t st) {
    const long long n = (long long)nb * H * W * (C / 8);
    hipLaunchKernelGGL(k_merge, dim3(blocks(n)), dim3(kThreads), 0, st, gpool, gcat, cat, C, nb, H,
                       W, out);
}

int loss_blocks(long long n) { return (int)((n + kThreads * kLossPer - 1) / (kThreads * kLossPer)); }

void launch_loss(const float* y, const float* t, const float* cw, int out_ch, int out_p,
                 long long npix, bf16_t* dy, double* part, hipStream_t st) {
    hipLaunchKernelGGL(k_loss, dim3(loss_blocks(npix * out_p)), dim3(kThreads), 0, st, y, t, cw,
                       out_ch, out_p, npix, dy, part);
}

void launch_sum(const double* part, int n, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(kThreads), 0, st, part, n, out);
}

void launch_adam(float* p, float* m, float* v, const float* g, long long n, float lr, float b1,
                 float b2, float eps, float c1, float c2, hipStream_t st) {
    hipLaunchKernelGGL(k_adam, dim3(blocks(n)), dim3(kThreads), 0, st, p, m, v, g, n, lr, b1, b2,
                       eps, c1, c2);
}

void launch_export(const float* w, int taps, int cin, int cout, bf16_t* wf, bf16_t* wb,
                   hipStream_t st) {
    const long long n = (long long)taps * cin * cout;
    hipLaunchKernelGGL(k_export, dim3(blocks(n)), dim3(kThreads), 0, st, w, taps, cin, cout, wf, wb);
}

void launch_param_map(const float* src, float* dst, int taps, int cin_o, int cout_o, int cin_p,
                      int cout_p, int to_padded, hipStream_t st) {
    const long long n = (long long)taps * cin_p * cout_p + cout_p;
    hipLaunchKernelGGL(k_param_map, dim3(blocks(n)), dim3(kThreads), 0, st, src, dst, taps, cin_o,
                       cout_o, cin_p, cout_p, to_padded);
}

void launch_warm_inputs(const WarmGeom& g, int nb, const float* f0, const float* f1,
                        const float* base, float* x, hipStream_t st) {
    const long long n = (long long)nb * g.X * g.Y;
    hipLaunchKernelGGL(k_warm_inputs, dim3(blocks(n)), dim3(kThreads), 0, st, g, nb, f0, f1, base, x);
}

void launch_warm_targets(const WarmGeom& g, int nb, const float* f0, const float* f1,
                         const float* F, long long sF, const float* Mx, const float* My,
                         const float* Mc, long long sM, const float* base, float* t,
                         hipStream_t st) {
    const long long n = (long long)nb * g.X * g.Y;
    hipLaunchKernelGGL(k_warm_map<0>, dim3(blocks(n)), dim3(kThreads), 0, st, g, nb, f0, f1, F,
                       (float*)nullptr, sF, Mx, My, Mc, (float*)nullptr, (float*)nullptr,
                       (float*)nullptr, sM, (const float*)nullptr, base, t);
}

void launch_warm_state(const WarmGeom& g, int nb, const float* f0, const float* f1,
                       const float* y, const float* base, float* F, long long sF, float* Mx,
                       float* My, float* Mc, long long sM, hipStream_t st) {
    const long long n = (long long)nb * g.X * g.Y;
    hipLaunchKernelGGL(k_warm_map<1>, dim3(blocks(n)), dim3(kThreads), 0, st, g, nb, f0, f1,
                       (const float*)nullptr, F, sF, (const float*)nullptr, (const float*)nullptr,
                       (const float*)nullptr, Mx, My, Mc, sM, y, base, (float*)nullptr);
}

void launch_restrict(const WarmGeom& gc, int nb, const float* f, float* fc, hipStream_t st) {
    const long long n = (long long)nb * gc.C * gc.X * gc.Y;
    hipLaunchKernelGGL(k_restrict, dim3(blocks(n)), dim3(kThreads), 0, st, gc, nb, f, fc);
}

void launch_prolong(const WarmGeom& gc, const WarmGeom& gf, int nb, const float* Fc,
                    long long sFc, const float* Mxc, const float* Myc, const float* Mcc,
                    long long sMc, float* F, long long sF, float* Mx, float* My, float* Mc,
                    long long sM, hipStream_t st) {
    const long long n = (long long)nb * gf.X * gf.Y;
    hipLaunchKernelGGL(k_prolong, dim3(blocks(n)), dim3(kThreads), 0, st, gc, gf, nb, Fc, sFc, Mxc,
                       Myc, Mcc, sMc, F, sF, Mx, My, Mc, sM);
}

}  // namespace otn
