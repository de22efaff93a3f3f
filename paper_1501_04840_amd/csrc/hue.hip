// Hue image pipeline of Sec. 5: hexcone hue of 8-bit RGB pixels, periodic
// hue histogram, strict order of the pixels, and the frame for a target
// density by exact circular histogram specification (the readings are listed
// in ot_hue.h).
//
// Device layout (one caller-owned workspace, carved by ot_hue_create): the
// hue bits, two sort-key buffers, two index buffers (the first also holds the
// ranks) u32 [N], the radix histograms int32 [256][tiles] and their digit
// totals, the source counts int32 [n]; per frame, the target counts and their
// inclusive cumulative sums int32 [n] and the shift one int64.  The strict
// order is a stable LSD radix sort of 24-bit keys written here: three passes
// of 8 bits, each a histogram kernel, a scan kernel and a scatter kernel
// whose blocks rank their tile stably in LDS (wave ballots per round) and
// write every digit's run contiguously; the last pass writes each pixel's
// rank instead of the order.  Per call of F frames: one planning
// kernel of F blocks (target counts, median shift) and one streaming kernel
// over the pixels in raster order with the frames along grid y, four pixels
// per thread (reads 3 bytes of RGB, the 4-byte hue kept from the source's
// sort keys and the 4-byte rank, writes 3 bytes and optionally the 4-byte
// bin).
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <new>

#include "../../include/ot_hue.h"

namespace {

constexpr int kMaxBins = 4096;
constexpr long long kMaxPix = 1LL << 30;
constexpr int kThreads = 256;
constexpr int kPlanThreads = 1024;
constexpr unsigned kKeyBlocks = 2048;     // 8 blocks per compute unit
constexpr unsigned kRenderBlocks = 4096;  // 16 blocks per compute unit, per frame
constexpr int kMaxFrames = 65535;         // frames per call (grid y)
constexpr unsigned kConvBlocks = 8192;    // RGB<->HSV grid-stride launches
// radix sort of the 24-bit hue keys: 3 passes of 8-bit digits over tiles of
// kSortThreads x kSortItems keys
constexpr int kSortThreads = 512;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kRadix = 256;
constexpr int kKeyBits = 24;

// Every FP32 step below is one rounded operation in the written order: no
// contraction of a product and a sum into a fused multiply-add.
struct Hue {
    float h;
    int hi, lo;
};

__device__ __forceinline__ Hue hue_of(int r, int g, int b) {
#pragma clang fp contract(off)
    // one division: the sector's signed difference over max - min (selects,
    // not branches, so a wave with mixed sectors divides once)
    Hue o;
    o.hi = max(max(r, g), b);
    o.lo = min(min(r, g), b);
    const bool rs = o.hi == r, gs = !rs && o.hi == g;
    const int num = rs ? g - b : (gs ? b - r : r - g);
    const float d = o.hi > o.lo ? (float)(o.hi - o.lo) : 1.f;
    const float q = (float)num / d;
    float h6 = rs ? (q < 0.f ? q + 6.f : q) : (gs ? q + 2.f : q + 4.f);
    h6 = o.hi > o.lo ? h6 : 0.f;
    float h = h6 / 6.f;
    h = h >= 1.f ? h - 1.f : h;
    o.h = h + 0.f;        // no negative zero in the sort key
    return o;
}

__device__ __forceinline__ int bin_of(float h, int n) {
#pragma clang fp contract(off)
    const float x = h * (float)n;
    return min((int)floorf(x), n - 1);
}

__device__ __forceinline__ unsigned char to_u8(float v) {
#pragma clang fp contract(off)
    float r = floorf(v + 0.5f);
    r = fminf(fmaxf(r, 0.f), 255.f);
    return (unsigned char)(int)r;
}

// Hexcone inverse with the max channel hi and the min channel lo kept.
__device__ __forceinline__ void rgb_of(float h, int hi, int lo, unsigned char* o) {
#pragma clang fp contract(off)
    const float hf = (float)hi, lf = (float)lo;
    const float d = hf - lf;
    const float h6 = h * 6.f;
    int i = (int)floorf(h6);
    i = min(max(i, 0), 5);
    const float f = h6 - (float)i;
    const float x = d * f;
    const float up = lf + x, down = hf - x;
    float r, g, b;
    switch (i) {
        case 0: r = hf; g = up; b = lf; break;
        case 1: r = down; g = hf; b = lf; break;
        case 2: r = lf; g = hf; b = up; break;
        case 3: r = lf; g = down; b = hf; break;
        case 4: r = up; g = lf; b = hf; break;
        default: r = hf; g = lf; b = down; break;
    }
    o[0] = to_u8(r);
    o[1] = to_u8(g);
    o[2] = to_u8(b);
}

// HSV of 8-bit RGB: the hexcone hue above, saturation (max - min) / max (0
// for black), value max / 255; float [N][3].
__global__ void __launch_bounds__(kThreads) k_rgb_to_hsv(const unsigned char* __restrict__ rgb,
                                                         long long N, float* hsv) {
#pragma clang fp contract(off)
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += stride) {
        const unsigned char* c = rgb + 3 * p;
        const Hue u = hue_of(c[0], c[1], c[2]);
        const float hf = (float)u.hi;
        const float d = hf - (float)u.lo;
        hsv[3 * p] = u.h;
        hsv[3 * p + 1] = u.hi > 0 ? d / hf : 0.f;
        hsv[3 * p + 2] = hf / 255.f;
    }
}

// 8-bit RGB of float HSV by the textbook hexcone (h wrapped into [0, 1), s
// and v clamped to [0, 1], non-finite input black), channels rounded to
// nearest.
__global__ void __launch_bounds__(kThreads) k_hsv_to_rgb(const float* __restrict__ hsv,
                                                         long long N, unsigned char* rgb) {
#pragma clang fp contract(off)
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += stride) {
        float h = hsv[3 * p], s = hsv[3 * p + 1], v = hsv[3 * p + 2];
        const bool bad = !(isfinite(h) && isfinite(s) && isfinite(v));
        h = bad ? 0.f : h;
        s = fminf(fmaxf(bad ? 0.f : s, 0.f), 1.f);
        v = fminf(fmaxf(bad ? 0.f : v, 0.f), 1.f);
        h = h - floorf(h);
        h = h >= 1.f ? h - 1.f : h;
        const float h6 = h * 6.f;
        const int i = min(max((int)floorf(h6), 0), 5);
        const float f = h6 - (float)i;
        const float pp = v * (1.f - s);
        const float sf = s * f;
        const float qq = v * (1.f - sf);
        const float g1 = 1.f - f;
        const float sg = s * g1;
        const float tt = v * (1.f - sg);
        float r, g, b;
        switch (i) {
            case 0: r = v; g = tt; b = pp; break;
            case 1: r = qq; g = v; b = pp; break;
            case 2: r = pp; g = v; b = tt; break;
            case 3: r = pp; g = qq; b = v; break;
            case 4: r = tt; g = pp; b = v; break;
            default: r = v; g = pp; b = qq; break;
        }
        unsigned char* o = rgb + 3 * p;
        o[0] = to_u8(r * 255.f);
        o[1] = to_u8(g * 255.f);
        o[2] = to_u8(b * 255.f);
    }
}

__global__ void k_fill_i32(int* p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Hue sort key (the FP32 bit pattern: monotone for hues >= 0), raster index,
// and the bin histogram (per-block LDS counts over a grid-stride loop, then
// one global add per bin and block).  Four pixels per thread; VEC: the image
// is 4-byte aligned, so a group of four moves as one 12-byte load and two
// 16-byte stores (the tail group and unaligned images go pixel by pixel).
// Sort key: floor(h 2^24), exact (a power-of-two scaling).  Distinct hues of
// 8-bit RGB differ by at least 1 / (6 * 255^2) (differences of fractions
// with denominators <= 255, over 6), far above 2^-24 plus the few ulps of
// their FP32 rounding, and equal hues give equal floats, so this 24-bit key
// orders pixels exactly as the hue does, in three radix passes instead of
// four.
__device__ __forceinline__ unsigned sort_key(float h) {
    return (unsigned)(h * 16777216.f);
}

template <bool VEC>
__global__ void __launch_bounds__(kThreads) k_hue_keys(const unsigned char* __restrict__ rgb,
                                                       long long N, int n, unsigned* keys,
                                                       unsigned* skey, int* counts) {
    __shared__ int hist[kMaxBins];
    for (int k = threadIdx.x; k < n; k += blockDim.x) hist[k] = 0;
    __syncthreads();
    const long long groups = (N + 3) / 4;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long gi = (long long)blockIdx.x * blockDim.x + threadIdx.x; gi < groups;
         gi += stride) {
        const long long p0 = 4 * gi;
        if (VEC && p0 + 4 <= N) {
            union { uint3 v; unsigned char b[12]; } in;
            in.v = *reinterpret_cast<const uint3*>(rgb + 3 * p0);
            uint4 kv, sv;
            unsigned* ku = reinterpret_cast<unsigned*>(&kv);
            unsigned* su = reinterpret_cast<unsigned*>(&sv);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const Hue u = hue_of(in.b[3 * i], in.b[3 * i + 1], in.b[3 * i + 2]);
                ku[i] = __float_as_uint(u.h);
                su[i] = sort_key(u.h);
                atomicAdd(&hist[bin_of(u.h, n)], 1);
            }
            *reinterpret_cast<uint4*>(keys + p0) = kv;
            *reinterpret_cast<uint4*>(skey + p0) = sv;
        } else {
            for (long long p = p0; p < p0 + 4 && p < N; ++p) {
                const unsigned char* c = rgb + 3 * p;
                const Hue u = hue_of(c[0], c[1], c[2]);
                keys[p] = __float_as_uint(u.h);
                skey[p] = sort_key(u.h);
                atomicAdd(&hist[bin_of(u.h, n)], 1);
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += blockDim.x)
        if (hist[k]) atomicAdd(&counts[k], hist[k]);
}

// ---- stable LSD radix sort of the 24-bit keys ------------------------------
// Tile i holds keys [i T, (i + 1) T) of the current order, T = kSortTile;
// thread t takes element r kSortThreads + t of its tile in round r, so the
// order (round, wave, lane) is the tile's element order.

// hist[d][tile] = number of keys of digit d in the tile.
__global__ void __launch_bounds__(kSortThreads) k_sort_hist(const unsigned* __restrict__ keys,
                                                            long long N, int shift, int ntiles,
                                                            int* hist) {
    __shared__ int cnt[kRadix];
    const int t = threadIdx.x;
    if (t < kRadix) cnt[t] = 0;
    __syncthreads();
    const long long base = (long long)blockIdx.x * kSortTile;
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const long long e = base + r * kSortThreads + t;
        if (e < N) atomicAdd(&cnt[(keys[e] >> shift) & (kRadix - 1)], 1);
    }
    __syncthreads();
    if (t < kRadix) hist[(long long)t * ntiles + blockIdx.x] = cnt[t];
}

// Block d: exclusive prefix sums of hist[d][0..ntiles) in place (the start of
// each tile's run of digit d among all keys of digit d) and totals[d].
__global__ void __launch_bounds__(kRadix) k_sort_scan(int* hist, int ntiles, int* totals) {
    __shared__ int part[kRadix];
    const int t = threadIdx.x;
    int* h = hist + (long long)blockIdx.x * ntiles;
    const int per = (ntiles + kRadix - 1) / kRadix;
    const int i0 = t * per, i1 = min(i0 + per, ntiles);
    int sum = 0;
    for (int i = i0; i < i1; ++i) sum += h[i];
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < kRadix; off <<= 1) {       // inclusive scan of the parts
        const int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - sum;
    for (int i = i0; i < i1; ++i) {
        const int v = h[i];
        h[i] = run;
        run += v;
    }
    if (t == kRadix - 1) totals[blockIdx.x] = part[t];
}

// Exclusive scan of v over the kRadix threads t < kRadix of the block (all
// threads of the block call it); returns the value for t < kRadix.
__device__ __forceinline__ int radix_scan(int v, int* sh) {
    const int t = threadIdx.x;
    if (t < kRadix) sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kRadix; off <<= 1) {
        const int a = (t < kRadix && t >= off) ? sh[t - off] : 0;
        __syncthreads();
        if (t < kRadix) sh[t] += a;
        __syncthreads();
    }
    const int r = t < kRadix ? sh[t] - v : 0;
    __syncthreads();
    return r;
}

// One radix pass: every key goes to position off[d] + pre[d][tile] + (its
// stable rank among the tile's keys of digit d), off[d] the number of keys of
// smaller digits.  FIRST: the input index is the element's own position (the
// raster index); LAST: writes rank_out[index] = position instead of the
// sorted keys and indices.
template <bool FIRST, bool LAST>
__global__ void __launch_bounds__(kSortThreads) k_sort_scatter(
    const unsigned* __restrict__ kin, const unsigned* __restrict__ iin, unsigned* kout,
    unsigned* iout, unsigned* rank_out, long long N, int shift, int ntiles,
    const int* __restrict__ pre, const int* __restrict__ totals) {
    __shared__ int cnt[kSortWaves][kRadix];
    __shared__ int run[kRadix], dbase[kRadix], dstart[kRadix], sh[kRadix];
    __shared__ unsigned sk[kSortTile], si[kSortTile];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const long long tile = blockIdx.x, base = tile * kSortTile;
    // global start of this tile's run of each digit
    {
        const int tot = t < kRadix ? totals[t] : 0;
        const int off = radix_scan(tot, sh);
        if (t < kRadix) {
            dbase[t] = off + pre[(long long)t * ntiles + tile];
            run[t] = 0;
        }
    }
    unsigned key[kSortItems], idx[kSortItems];
    int rk[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const long long e = base + r * kSortThreads + t;
        const bool valid = e < N;
        key[r] = valid ? kin[e] : 0u;
        idx[r] = valid ? (FIRST ? (unsigned)e : iin[e]) : 0u;
    }
    const unsigned long long lt = (1ull << lane) - 1ull;
    for (int r = 0; r < kSortItems; ++r) {
        for (int i = t; i < kSortWaves * kRadix; i += kSortThreads) (&cnt[0][0])[i] = 0;
        __syncthreads();
        const bool valid = base + r * kSortThreads + t < N;
        const int d = (int)((key[r] >> shift) & (kRadix - 1));
        // lanes of this wave with the same digit
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const unsigned long long m = __ballot(valid && bit);
            peers &= bit ? m : ~m;
        }
        const int lr = __popcll(peers & lt);
        if (valid && lr == 0) cnt[w][d] = __popcll(peers);
        __syncthreads();
        if (t < kRadix) {          // digit t: start of each wave's keys in this round
            int s0 = run[t];
#pragma unroll
            for (int q = 0; q < kSortWaves; ++q) {
                const int c = cnt[q][t];
                cnt[q][t] = s0;
                s0 += c;
            }
            run[t] = s0;
        }
        __syncthreads();
        rk[r] = valid ? cnt[w][d] + lr : 0;
        __syncthreads();
    }
    // the tile sorted by digit in LDS: digit runs in order, each stable
    {
        const int st = radix_scan(t < kRadix ? run[t] : 0, sh);
        if (t < kRadix) dstart[t] = st;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        if (base + r * kSortThreads + t < N) {
            const int d = (int)((key[r] >> shift) & (kRadix - 1));
            const int p = dstart[d] + rk[r];
            sk[p] = key[r];
            si[p] = idx[r];
        }
    }
    __syncthreads();
    const int nh = (int)min((long long)kSortTile, N - base);
    for (int j = t; j < nh; j += kSortThreads) {
        const unsigned k = sk[j];
        const int d = (int)((k >> shift) & (kRadix - 1));
        const long long pos = (long long)dbase[d] + (j - dstart[d]);
        if (LAST) {
            rank_out[si[j]] = (unsigned)pos;
        } else {
            kout[pos] = k;
            iout[pos] = si[j];
        }
    }
}

__global__ void k_hue_density(const int* __restrict__ counts, int n, long long N, float* dens) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dens[k] = (float)((double)counts[k] * ((double)n / (double)N));
}

// Exclusive prefix sums of two integer arrays of n <= kMaxBins entries held
// kBinsPerThread per thread (Hillis-Steele over the per-thread totals).
constexpr int kBinsPerThread = kMaxBins / kPlanThreads;

__device__ __forceinline__ void block_scan2(int& x, int& y, int* sx, int* sy) {
    const int t = threadIdx.x;
    sx[t] = x;
    sy[t] = y;
    __syncthreads();
    for (int off = 1; off < kPlanThreads; off <<= 1) {
        const int ax = t >= off ? sx[t - off] : 0, ay = t >= off ? sy[t - off] : 0;
        __syncthreads();
        sx[t] += ax;
        sy[t] += ay;
        __syncthreads();
    }
    x = t ? sx[t - 1] : 0;              // exclusive
    y = t ? sy[t - 1] : 0;
    __syncthreads();
}

// One block: target counts by largest remainder, the inclusive cumulative
// target counts, and the shift (lower median of the edge differences).
// The remainder ranks take bins strided over the block (t + 1024 i), the
// prefix sums blocked (kBinsPerThread t + i).  The FP64 mass is summed bin by
// bin in index order (one thread, from LDS); the integer sums and prefix sums
// are exact in any order.
__global__ void __launch_bounds__(kPlanThreads) k_hue_plan(const float* __restrict__ target,
                                                           const int* __restrict__ cs, int n,
                                                           long long N, int* ct_out,
                                                           int* cum_out, long long* shift) {
    {   // block f plans frame f
        const long long f = blockIdx.x;
        target += f * n;
        ct_out += f * n;
        cum_out += f * n;
        shift += f;
    }
    __shared__ double rem[kMaxBins];
    __shared__ int ct[kMaxBins];
    __shared__ int sx[kPlanThreads], sy[kPlanThreads];
    __shared__ double S_sh;
    __shared__ unsigned long long fl_sh;
    int* D = reinterpret_cast<int*>(rem);   // edge differences, once rem is consumed
    const int t = threadIdx.x;
    // the target, negative and non-finite entries as zero, staged in rem
    for (int k = t; k < n; k += blockDim.x) {
        const float v = target[k];
        rem[k] = (isfinite(v) && v > 0.f) ? (double)v : 0.0;
    }
    if (t == 0) fl_sh = 0;
    __syncthreads();
    if (t == 0) {                       // the mass, bin by bin in index order
        double S = 0.0;
#pragma unroll 8
        for (int k = 0; k < n; ++k) S += rem[k];
        S_sh = S;
    }
    __syncthreads();
    const double S = S_sh;
    const bool keep = !(S > 0.0);
    int fsum = 0;
    for (int k = t; k < n; k += blockDim.x) {
        if (keep) {
            ct[k] = cs[k];
            rem[k] = 0.0;
        } else {
            const double x = ((double)N * rem[k]) / S;
            const double c = floor(x);
            ct[k] = (int)c;
            rem[k] = x - c;
        }
        fsum += ct[k];
    }
    atomicAdd(&fl_sh, (unsigned long long)fsum);
    __syncthreads();
    const long long left = keep ? 0 : N - (long long)fl_sh;
    // the `left` largest remainders (ties: lower bin) get one more pixel;
    // bins strided over the block, the rank loop unrolled so that its LDS
    // loads overlap
    int add[kBinsPerThread];
#pragma unroll
    for (int q = 0; q < kBinsPerThread; ++q) {
        const int k = t + q * kPlanThreads;
        add[q] = 0;
        if (k < n && left > 0) {
            const double rk = rem[k];
            int rank = 0;
#pragma unroll 8
            for (int j = 0; j < n; ++j) {
                const double rj = rem[j];
                rank += (rj > rk || (rj == rk && j < k)) ? 1 : 0;
            }
            add[q] = rank < left ? 1 : 0;
        }
    }
    __syncthreads();                    // every read of rem is done
#pragma unroll
    for (int q = 0; q < kBinsPerThread; ++q) {
        const int k = t + q * kPlanThreads;
        if (k < n) ct[k] += add[q];
    }
    __syncthreads();
    int cst[kBinsPerThread], ctt[kBinsPerThread];
    int xs = 0, xt = 0;
#pragma unroll
    for (int q = 0; q < kBinsPerThread; ++q) {
        const int k = kBinsPerThread * t + q;
        cst[q] = k < n ? cs[k] : 0;
        ctt[q] = k < n ? ct[k] : 0;
        xs += cst[q];
        xt += ctt[q];
    }
    block_scan2(xs, xt, sx, sy);
#pragma unroll
    for (int q = 0; q < kBinsPerThread; ++q) {
        const int k = kBinsPerThread * t + q;
        if (k < n) {
            D[k] = xs - xt;             // before bin k
            xs += cst[q];
            xt += ctt[q];
            cum_out[k] = xt;
            ct_out[k] = ctt[q];
        }
    }
    __syncthreads();
    const int m = (n - 1) / 2;          // lower median: the value of rank m
    for (int e = t; e < n; e += blockDim.x) {
        const int de = D[e];
        int rank = 0;
#pragma unroll 8
        for (int j = 0; j < n; ++j) {
            const int dj = D[j];
            rank += (dj < de || (dj == de && j < e)) ? 1 : 0;
        }
        if (rank == m) *shift = de;
    }
}

// Output bin of a pixel of rank rk: the first bin whose cumulative count
// exceeds q = (rk - s) mod N, i.e. the number of cumulative counts <= q.  cl
// holds the n nondecreasing counts padded with INT_MAX to pw = 2^ceil(log2 n)
// entries, so the branch-free search needs no bounds test; W pixels in
// lockstep so that their LDS loads overlap.
template <int W>
__device__ __forceinline__ void out_bins(const unsigned* rk, int s, int N, const int* cl, int n,
                                         int pw, int* lo) {
    // N <= 2^30: rank - s lies in (-2^30, 2^31 - 1), so 32-bit arithmetic
    int q[W];
#pragma unroll
    for (int i = 0; i < W; ++i) {
        q[i] = (int)rk[i] - s;          // rank in [0, N), shift in (-N, N)
        q[i] = q[i] < 0 ? q[i] + N : (q[i] >= N ? q[i] - N : q[i]);
        lo[i] = 0;
    }
    for (int half = pw >> 1; half > 0; half >>= 1) {
#pragma unroll
        for (int i = 0; i < W; ++i) lo[i] += cl[lo[i] + half - 1] <= q[i] ? half : 0;
    }
#pragma unroll
    for (int i = 0; i < W; ++i) lo[i] = min(lo[i] + (cl[lo[i]] <= q[i] ? 1 : 0), n - 1);
}

// One pixel of a frame: its hue h (the source's sort key, computed once per
// source) moved to the output bin, RGB rebuilt with the max and min channels.
__device__ __forceinline__ void paint_px(const unsigned char* c, float h, int kout, int n,
                                         unsigned char* o) {
#pragma clang fp contract(off)
    const int r = c[0], g = c[1], b = c[2];
    const int ksrc = bin_of(h, n);
    float h2 = h + (float)(kout - ksrc) / (float)n;
    if (h2 >= 1.f) h2 = h2 - 1.f;
    if (h2 < 0.f) h2 = h2 + 1.f;
    if (h2 >= 1.f) h2 = h2 - 1.f;
    rgb_of(h2, max(max(r, g), b), min(min(r, g), b), o);
}

// One frame over the pixels in raster order, four pixels per thread in a
// grid-stride loop.  VEC: the image pointers are 4-byte aligned (and bins_out
// 16-byte aligned), so a group of four moves as 12 bytes of RGB, 16 bytes of
// rank and 16 bytes of bins; the tail group and unaligned images go pixel by
// pixel.
template <bool VEC>
__global__ void __launch_bounds__(kThreads) k_hue_render(const unsigned char* __restrict__ rgb,
                                                         const unsigned* __restrict__ hue,
                                                         const unsigned* __restrict__ rank,
                                                         const int* __restrict__ cum,
                                                         const long long* __restrict__ shift,
                                                         int n, long long N, unsigned char* out,
                                                         int* bins_out) {
    {   // blockIdx.y: the frame
        const long long f = blockIdx.y;
        cum += f * n;
        shift += f;
        out += f * 3 * N;
        if (bins_out) bins_out += f * N;
    }
    extern __shared__ int cl[];        // [pw]: cumulative counts, INT_MAX padding
    const int pw = n > 1 ? 1 << (32 - __clz(n - 1)) : 1;
    for (int k = threadIdx.x; k < pw; k += blockDim.x) cl[k] = k < n ? cum[k] : INT_MAX;
    __syncthreads();
    const int s32 = (int)*shift, N32 = (int)N;
    const long long groups = (N + 3) / 4;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long gi = (long long)blockIdx.x * blockDim.x + threadIdx.x; gi < groups;
         gi += stride) {
        const long long p0 = 4 * gi;
        if (VEC && p0 + 4 <= N) {
            union { uint3 v; unsigned char b[12]; } in, o;
            union { uint4 v; unsigned u[4]; } rk, hu;
            in.v = *reinterpret_cast<const uint3*>(rgb + 3 * p0);
            rk.v = *reinterpret_cast<const uint4*>(rank + p0);
            hu.v = *reinterpret_cast<const uint4*>(hue + p0);
            int kb[4];
            out_bins<4>(rk.u, s32, N32, cl, n, pw, kb);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                paint_px(in.b + 3 * i, __uint_as_float(hu.u[i]), kb[i], n, o.b + 3 * i);
            *reinterpret_cast<uint3*>(out + 3 * p0) = o.v;
            if (bins_out) *reinterpret_cast<int4*>(bins_out + p0) = make_int4(kb[0], kb[1], kb[2], kb[3]);
        } else {
            for (long long p = p0; p < p0 + 4 && p < N; ++p) {
                const unsigned r1 = rank[p];
                int k;
                out_bins<1>(&r1, s32, N32, cl, n, pw, &k);
                paint_px(rgb + 3 * p, __uint_as_float(hue[p]), k, n, out + 3 * p);
                if (bins_out) bins_out[p] = k;
            }
        }
    }
}

unsigned blocks_for(long long n, int t) { return (unsigned)((n + t - 1) / t); }

// Workspace carve of a renderer (256-byte aligned pieces).
struct HueLayout {
    size_t keys, skey, skey2, idxa, idxb, hist, totals, counts, ct, cum, shift, total;
    int ntiles;
};

HueLayout hue_layout(long long N, int n, int frames) {
    HueLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = (o + bytes + 255) / 256 * 256; return r; };
    const size_t w = (size_t)N * sizeof(unsigned);
    L.ntiles = (int)((N + kSortTile - 1) / kSortTile);
    L.keys = take(w);
    L.skey = take(w);
    L.skey2 = take(w);
    L.idxa = take(w);
    L.idxb = take(w);
    L.hist = take((size_t)kRadix * L.ntiles * sizeof(int));
    L.totals = take(kRadix * sizeof(int));
    L.counts = take((size_t)n * sizeof(int));
    L.ct = take((size_t)frames * n * sizeof(int));
    L.cum = take((size_t)frames * n * sizeof(int));
    L.shift = take((size_t)frames * sizeof(long long));
    L.total = o;
    return L;
}

int hue_check(long long npix, int nbins, int frames) {
    if (npix < 1 || npix > kMaxPix || nbins < 2 || nbins > kMaxBins || frames < 1 ||
        frames > kMaxFrames)
        return OT_ERR_SHAPE;
    return OT_OK;
}

}  // namespace

struct ot_hue {
    long long N = 0;
    int n = 0;
    int cap = 0;                        // frames the plan arrays hold
    int ntiles = 0;
    hipStream_t st = nullptr;
    // keys: each pixel's hue (FP32 bits, raster order, read by the frames);
    // skey/skey2: 24-bit sort keys, idxa/idxb: the sort's raster indices
    // (idxb holds the ranks once the sort is done)
    unsigned *keys = nullptr, *skey = nullptr, *skey2 = nullptr, *idxa = nullptr, *idxb = nullptr;
    unsigned* rank = nullptr;
    int *hist = nullptr, *totals = nullptr;
    int *counts = nullptr, *ct = nullptr, *cum = nullptr;
    long long* shift = nullptr;
    const unsigned char* src = nullptr;
    bool have_source = false;
    int planned = 0;                    // frames of the last plan (0: none)
};

extern "C" {

int ot_hue_workspace_size(long long npix, int nbins, int max_frames, size_t* bytes) {
    if (!bytes) return OT_ERR_PARAM;
    const int st = hue_check(npix, nbins, max_frames);
    if (st != OT_OK) return st;
    *bytes = hue_layout(npix, nbins, max_frames).total;
    return OT_OK;
}

int ot_hue_create(long long npix, int nbins, int max_frames, void* stream, void* workspace,
                  size_t ws_bytes, ot_hue** out) {
    if (!out) return OT_ERR_PARAM;
    *out = nullptr;
    const int st = hue_check(npix, nbins, max_frames);
    if (st != OT_OK) return st;
    const HueLayout L = hue_layout(npix, nbins, max_frames);
    if (!workspace || ws_bytes < L.total || (uintptr_t)workspace % 256 != 0) return OT_ERR_SHAPE;
    ot_hue* h = new (std::nothrow) ot_hue;
    if (!h) return OT_ERR_PARAM;
    char* ws = (char*)workspace;
    h->N = npix;
    h->n = nbins;
    h->cap = max_frames;
    h->ntiles = L.ntiles;
    h->st = (hipStream_t)stream;
    h->keys = (unsigned*)(ws + L.keys);
    h->skey = (unsigned*)(ws + L.skey);
    h->skey2 = (unsigned*)(ws + L.skey2);
    h->idxa = (unsigned*)(ws + L.idxa);
    h->idxb = (unsigned*)(ws + L.idxb);
    h->rank = h->idxb;
    h->hist = (int*)(ws + L.hist);
    h->totals = (int*)(ws + L.totals);
    h->counts = (int*)(ws + L.counts);
    h->ct = (int*)(ws + L.ct);
    h->cum = (int*)(ws + L.cum);
    h->shift = (long long*)(ws + L.shift);
    *out = h;
    return OT_OK;
}

void ot_hue_destroy(ot_hue* h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->st);
    delete h;
}

int ot_hue_set_source(ot_hue* h, const unsigned char* rgb) {
    if (!h || !rgb) return OT_ERR_PARAM;
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(h->n, kThreads)), dim3(kThreads), 0, h->st,
                       h->counts, h->n, 0);
    const unsigned kb = blocks_for((h->N + 3) / 4, kThreads);
    const dim3 kgrid(kb < kKeyBlocks ? kb : kKeyBlocks);
    if ((uintptr_t)rgb % 4 == 0)
        hipLaunchKernelGGL(k_hue_keys<true>, kgrid, dim3(kThreads), 0, h->st, rgb, h->N, h->n,
                           h->keys, h->skey, h->counts);
    else
        hipLaunchKernelGGL(k_hue_keys<false>, kgrid, dim3(kThreads), 0, h->st, rgb, h->N, h->n,
                           h->keys, h->skey, h->counts);
    // stable radix sort of the 24-bit keys (sort_key): equal hues keep raster
    // order.  Pass 0: keys skey -> skey2, raster indices (implicit) -> idxb;
    // pass 1: skey2 -> skey, idxb -> idxa; pass 2 reads skey and idxa and
    // writes each pixel's rank into idxb.
    const unsigned* kin[3] = {h->skey, h->skey2, h->skey};
    unsigned* kout[3] = {h->skey2, h->skey, nullptr};
    const unsigned* iin[3] = {nullptr, h->idxb, h->idxa};
    unsigned* iout[3] = {h->idxb, h->idxa, nullptr};
    for (int pass = 0; pass < kKeyBits / 8; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_sort_hist, dim3(h->ntiles), dim3(kSortThreads), 0, h->st, kin[pass],
                           h->N, shift, h->ntiles, h->hist);
        hipLaunchKernelGGL(k_sort_scan, dim3(kRadix), dim3(kRadix), 0, h->st, h->hist, h->ntiles,
                           h->totals);
        if (pass == 0)
            hipLaunchKernelGGL((k_sort_scatter<true, false>), dim3(h->ntiles), dim3(kSortThreads), 0,
                               h->st, kin[0], nullptr, kout[0], iout[0], nullptr, h->N, shift,
                               h->ntiles, h->hist, h->totals);
        else if (pass == 1)
            hipLaunchKernelGGL((k_sort_scatter<false, false>), dim3(h->ntiles), dim3(kSortThreads),
                               0, h->st, kin[1], iin[1], kout[1], iout[1], nullptr, h->N, shift,
                               h->ntiles, h->hist, h->totals);
        else
            hipLaunchKernelGGL((k_sort_scatter<false, true>), dim3(h->ntiles), dim3(kSortThreads),
                               0, h->st, kin[2], iin[2], nullptr, nullptr, h->idxb, h->N, shift,
                               h->ntiles, h->hist, h->totals);
    }
    if (hipGetLastError() != hipSuccess) return OT_ERR_HIP;
    h->rank = h->idxb;
    h->src = rgb;
    h->have_source = true;
    h->planned = 0;
    return OT_OK;
}

int ot_hue_histogram(ot_hue* h, int* counts, float* density) {
    if (!h) return OT_ERR_PARAM;
    if (!h->have_source) return OT_ERR_STATE;
    if (counts &&
        hipMemcpyAsync(counts, h->counts, h->n * sizeof(int), hipMemcpyDeviceToDevice, h->st) !=
            hipSuccess)
        return OT_ERR_HIP;
    if (density)
        hipLaunchKernelGGL(k_hue_density, dim3(blocks_for(h->n, kThreads)), dim3(kThreads), 0,
                           h->st, h->counts, h->n, h->N, density);
    return hipGetLastError() == hipSuccess ? OT_OK : OT_ERR_HIP;
}

int ot_hue_plan(ot_hue* h, const float* targets, int frames) {
    if (!h || !targets || frames < 1 || frames > kMaxFrames) return OT_ERR_PARAM;
    if (!h->have_source) return OT_ERR_STATE;
    if (frames > h->cap) {
        h->planned = 0;
        return OT_ERR_SHAPE;
    }
    hipLaunchKernelGGL(k_hue_plan, dim3(frames), dim3(kPlanThreads), 0, h->st, targets, h->counts,
                       h->n, h->N, h->ct, h->cum, h->shift);
    if (hipGetLastError() != hipSuccess) return OT_ERR_HIP;
    h->planned = frames;
    return OT_OK;
}

int ot_hue_apply(ot_hue* h, unsigned char* rgb_out, int* bins_out) {
    if (!h || !rgb_out) return OT_ERR_PARAM;
    if (!h->planned) return OT_ERR_STATE;
    const int F = h->planned;
    const unsigned gb = blocks_for((h->N + 3) / 4, kThreads);
    const dim3 grid(gb < kRenderBlocks ? gb : kRenderBlocks, (unsigned)F);
    // every frame's image 4-byte aligned and bins 16-byte aligned
    const bool vec = ((uintptr_t)h->src % 4 == 0) && ((uintptr_t)rgb_out % 4 == 0) &&
                     ((uintptr_t)bins_out % 16 == 0) &&
                     (F == 1 || ((3 * h->N) % 4 == 0 && (!bins_out || h->N % 4 == 0)));
    // LDS: the cumulative counts padded to the next power of two (<= 16 KB)
    const size_t lds = sizeof(int) * (h->n > 1 ? (size_t)1 << (32 - __builtin_clz(h->n - 1)) : 1);
    if (vec)
        hipLaunchKernelGGL(k_hue_render<true>, grid, dim3(kThreads), lds, h->st, h->src, h->keys,
                           h->rank,
                           h->cum, h->shift, h->n, h->N, rgb_out, bins_out);
    else
        hipLaunchKernelGGL(k_hue_render<false>, grid, dim3(kThreads), lds, h->st, h->src, h->keys,
                           h->rank,
                           h->cum, h->shift, h->n, h->N, rgb_out, bins_out);
    return hipGetLastError() == hipSuccess ? OT_OK : OT_ERR_HIP;
}

int ot_hue_render(ot_hue* h, const float* targets, int frames, unsigned char* rgb_out,
                  int* bins_out) {
    if (!h || !targets || !rgb_out) return OT_ERR_PARAM;
    const int st = ot_hue_plan(h, targets, frames);
    return st != OT_OK ? st : ot_hue_apply(h, rgb_out, bins_out);
}

int ot_hue_plan_info(ot_hue* h, int frame, int* counts, long long* shift) {
    if (!h) return OT_ERR_PARAM;
    if (!h->planned) return OT_ERR_STATE;
    if (frame < 0 || frame >= h->planned) return OT_ERR_PARAM;
    if (counts && hipMemcpyAsync(counts, h->ct + (size_t)frame * h->n, h->n * sizeof(int),
                                 hipMemcpyDeviceToHost, h->st) != hipSuccess)
        return OT_ERR_HIP;
    if (shift && hipMemcpyAsync(shift, h->shift + frame, sizeof(long long),
                                hipMemcpyDeviceToHost, h->st) != hipSuccess)
        return OT_ERR_HIP;
    return hipStreamSynchronize(h->st) == hipSuccess ? OT_OK : OT_ERR_HIP;
}

int ot_hue_rgb_to_hsv(const unsigned char* rgb, long long npix, float* hsv, void* stream) {
    if (npix < 0 || (npix > 0 && (!rgb || !hsv))) return OT_ERR_PARAM;
    if (npix == 0) return OT_OK;
    const unsigned gb = blocks_for(npix, kThreads);
    hipLaunchKernelGGL(k_rgb_to_hsv, dim3(gb < kConvBlocks ? gb : kConvBlocks), dim3(kThreads), 0,
                       (hipStream_t)stream, rgb, npix, hsv);
    return hipGetLastError() == hipSuccess ? OT_OK : OT_ERR_HIP;
}

int ot_hue_hsv_to_rgb(const float* hsv, long long npix, unsigned char* rgb, void* stream) {
    if (npix < 0 || (npix > 0 && (!rgb || !hsv))) return OT_ERR_PARAM;
    if (npix == 0) return OT_OK;
    const unsigned gb = blocks_for(npix, kThreads);
    hipLaunchKernelGGL(k_hsv_to_rgb, dim3(gb < kConvBlocks ? gb : kConvBlocks), dim3(kThreads), 0,
                       (hipStream_t)stream, hsv, npix, rgb);
    return hipGetLastError() == hipSuccess ? OT_OK : OT_ERR_HIP;
}

}  // extern "C"
