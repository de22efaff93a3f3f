// Hue image pipeline of Sec. 5: hexcone hue of 8-bit RGB pixels, periodic
// hue histogram, strict order of the pixels, and the frame for a target
// density by exact circular histogram specification (the readings are listed
// in ot_hue.h).
//
// Device layout: keys/order/rank are u32 [N]; counts, target counts and the
// inclusive cumulative target counts are int32 [n]; the shift is one int64.
// Per frame: one single-block planning kernel (target counts, median shift)
// and one streaming kernel over the pixels in raster order (reads 3 bytes of
// RGB and the 4-byte rank, writes 3 bytes and optionally the 4-byte bin).
#include <hip/hip_runtime.h>
#include <hipcub/device/device_radix_sort.hpp>

#include <new>

#include "../../include/ot_hue.h"

namespace {

constexpr int kMaxBins = 4096;
constexpr long long kMaxPix = 1LL << 30;
constexpr int kThreads = 256;
constexpr int kPlanThreads = 1024;
constexpr unsigned kKeyBlocks = 2048;     // 8 blocks per compute unit

// Every FP32 step below is one rounded operation in the written order: no
// contraction of a product and a sum into a fused multiply-add.
struct Hue {
    float h;
    int hi, lo;
};

__device__ __forceinline__ Hue hue_of(int r, int g, int b) {
#pragma clang fp contract(off)
    Hue o;
    o.hi = max(max(r, g), b);
    o.lo = min(min(r, g), b);
    const float d = (float)(o.hi - o.lo);
    float h6;
    if (o.hi == o.lo) {
        h6 = 0.f;
    } else if (o.hi == r) {
        h6 = (float)(g - b) / d;
        if (h6 < 0.f) h6 = h6 + 6.f;
    } else if (o.hi == g) {
        h6 = (float)(b - r) / d + 2.f;
    } else {
        h6 = (float)(r - g) / d + 4.f;
    }
    float h = h6 / 6.f;
    if (h >= 1.f) h = h - 1.f;
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

__global__ void k_fill_i32(int* p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Hue sort key (the FP32 bit pattern: monotone for hues >= 0), raster index,
// and the bin histogram (per-block LDS counts over a grid-stride loop, then
// one global add per bin and block).
__global__ void __launch_bounds__(kThreads) k_hue_keys(const unsigned char* __restrict__ rgb,
                                                       long long N, int n, unsigned* keys,
                                                       unsigned* idx, int* counts) {
    __shared__ int hist[kMaxBins];
    for (int k = threadIdx.x; k < n; k += blockDim.x) hist[k] = 0;
    __syncthreads();
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += stride) {
        const unsigned char* c = rgb + 3 * p;
        const Hue u = hue_of(c[0], c[1], c[2]);
        keys[p] = __float_as_uint(u.h);
        idx[p] = (unsigned)p;
        atomicAdd(&hist[bin_of(u.h, n)], 1);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += blockDim.x)
        if (hist[k]) atomicAdd(&counts[k], hist[k]);
}

__global__ void k_hue_rank(const unsigned* __restrict__ order, long long N, unsigned* rank) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < N) rank[order[j]] = (unsigned)j;
}

__global__ void k_hue_density(const int* __restrict__ counts, int n, long long N, float* dens) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dens[k] = (float)((double)counts[k] * ((double)n / (double)N));
}

// One block: target counts by largest remainder, the inclusive cumulative
// target counts, and the shift (lower median of the edge differences).
__global__ void __launch_bounds__(kPlanThreads) k_hue_plan(const float* __restrict__ target,
                                                           const int* __restrict__ cs, int n,
                                                           long long N, int* ct_out,
                                                           int* cum_out, long long* shift) {
    __shared__ double rem[kMaxBins];
    __shared__ int ct[kMaxBins];
    int* D = reinterpret_cast<int*>(rem);   // edge differences, once rem is consumed
    __shared__ double S_sh;
    __shared__ long long left_sh;
    const int t = threadIdx.x;
    if (t == 0) {                       // the density's mass, bin by bin in order
        double S = 0.0;
        for (int k = 0; k < n; ++k) {
            const float v = target[k];
            if (isfinite(v) && v > 0.f) S += (double)v;
        }
        S_sh = S;
    }
    __syncthreads();
    const double S = S_sh;
    const bool keep = !(S > 0.0);
    for (int k = t; k < n; k += blockDim.x) {
        if (keep) {
            ct[k] = cs[k];
            rem[k] = 0.0;
        } else {
            const float v = target[k];
            const double hv = (isfinite(v) && v > 0.f) ? (double)v : 0.0;
            const double x = ((double)N * hv) / S;
            const double c = floor(x);
            ct[k] = (int)c;
            rem[k] = x - c;
        }
    }
    __syncthreads();
    if (t == 0) {
        long long sum = 0;
        for (int k = 0; k < n; ++k) sum += ct[k];
        left_sh = keep ? 0 : N - sum;
    }
    __syncthreads();
    const long long left = left_sh;
    // the `left` largest remainders (ties: lower bin) get one more pixel
    int add[kMaxBins / kPlanThreads];
#pragma unroll
    for (int q = 0; q < kMaxBins / kPlanThreads; ++q) {
        const int k = t + q * kPlanThreads;
        add[q] = 0;
        if (k < n && left > 0) {
            const double rk = rem[k];
            int rank = 0;
            for (int j = 0; j < n; ++j) {
                const double rj = rem[j];
                rank += (rj > rk || (rj == rk && j < k)) ? 1 : 0;
            }
            add[q] = rank < left ? 1 : 0;
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kMaxBins / kPlanThreads; ++q) {
        const int k = t + q * kPlanThreads;
        if (k < n) ct[k] += add[q];
    }
    __syncthreads();
    if (t == 0) {                       // edge differences and cumulative counts
        long long es = 0, et = 0;
        for (int k = 0; k < n; ++k) {
            D[k] = (int)(es - et);
            es += cs[k];
            et += ct[k];
            cum_out[k] = (int)et;
            ct_out[k] = ct[k];
        }
    }
    __syncthreads();
    const int m = (n - 1) / 2;          // lower median: the value of rank m
    for (int e = t; e < n; e += blockDim.x) {
        const int de = D[e];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const int dj = D[j];
            rank += (dj < de || (dj == de && j < e)) ? 1 : 0;
        }
        if (rank == m) *shift = de;
    }
}

// One frame: each pixel in raster order takes the target bin holding
// position (rank - s) mod N of the cumulative target counts.
__global__ void __launch_bounds__(kThreads) k_hue_render(const unsigned char* __restrict__ rgb,
                                                         const unsigned* __restrict__ rank,
                                                         const int* __restrict__ cum,
                                                         const long long* __restrict__ shift,
                                                         int n, long long N, unsigned char* out,
                                                         int* bins_out) {
#pragma clang fp contract(off)
    __shared__ int cl[kMaxBins];
    for (int k = threadIdx.x; k < n; k += blockDim.x) cl[k] = cum[k];
    __syncthreads();
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    long long q = (long long)rank[p] - *shift;     // rank in [0, N), shift in (-N, N)
    if (q < 0) q += N;
    else if (q >= N) q -= N;
    int lo = 0, hi = n - 1;            // first bin whose cumulative count exceeds q
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((long long)cl[mid] > q) hi = mid;
        else lo = mid + 1;
    }
    const int kout = lo;
    const unsigned char* c = rgb + 3 * p;
    const Hue u = hue_of(c[0], c[1], c[2]);
    const int ksrc = bin_of(u.h, n);
    float h2 = u.h + (float)(kout - ksrc) / (float)n;
    if (h2 >= 1.f) h2 = h2 - 1.f;
    if (h2 < 0.f) h2 = h2 + 1.f;
    if (h2 >= 1.f) h2 = h2 - 1.f;
    rgb_of(h2, u.hi, u.lo, out + 3 * p);
    if (bins_out) bins_out[p] = kout;
}

unsigned blocks_for(long long n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

struct ot_hue {
    long long N = 0;
    int n = 0;
    hipStream_t st = nullptr;
    unsigned *keys = nullptr, *keys2 = nullptr, *idx = nullptr, *order = nullptr, *rank = nullptr;
    int *counts = nullptr, *ct = nullptr, *cum = nullptr;
    long long* shift = nullptr;
    void* temp = nullptr;
    size_t temp_bytes = 0;
    const unsigned char* src = nullptr;
    bool have_source = false, have_frame = false;
};

static void hue_free(ot_hue* h) {
    void* bufs[] = {h->keys, h->keys2, h->idx, h->order, h->rank, h->counts,
                    h->ct, h->cum, h->shift, h->temp};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
}

extern "C" {

int ot_hue_create(long long npix, int nbins, void* stream, ot_hue** out) {
    if (!out) return OT_ERR_PARAM;
    *out = nullptr;
    if (npix < 1 || npix > kMaxPix || nbins < 2 || nbins > kMaxBins) return OT_ERR_SHAPE;
    ot_hue* h = new (std::nothrow) ot_hue;
    if (!h) return OT_ERR_HIP;
    h->N = npix;
    h->n = nbins;
    h->st = (hipStream_t)stream;
    const size_t w = (size_t)npix * sizeof(unsigned);
    bool ok = hipMalloc(&h->keys, w) == hipSuccess && hipMalloc(&h->keys2, w) == hipSuccess &&
              hipMalloc(&h->idx, w) == hipSuccess && hipMalloc(&h->order, w) == hipSuccess &&
              hipMalloc(&h->rank, w) == hipSuccess &&
              hipMalloc(&h->counts, nbins * sizeof(int)) == hipSuccess &&
              hipMalloc(&h->ct, nbins * sizeof(int)) == hipSuccess &&
              hipMalloc(&h->cum, nbins * sizeof(int)) == hipSuccess &&
              hipMalloc(&h->shift, sizeof(long long)) == hipSuccess;
    if (ok)
        ok = hipcub::DeviceRadixSort::SortPairs(nullptr, h->temp_bytes, h->keys, h->keys2, h->idx,
                                                h->order, (int)npix, 0, 30, h->st) == hipSuccess &&
             hipMalloc(&h->temp, h->temp_bytes ? h->temp_bytes : 1) == hipSuccess;
    if (!ok) {
        hue_free(h);
        delete h;
        return OT_ERR_HIP;
    }
    *out = h;
    return OT_OK;
}

void ot_hue_destroy(ot_hue* h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->st);
    hue_free(h);
    delete h;
}

int ot_hue_set_source(ot_hue* h, const unsigned char* rgb) {
    if (!h || !rgb) return OT_ERR_PARAM;
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(h->n, kThreads)), dim3(kThreads), 0, h->st,
                       h->counts, h->n, 0);
    const unsigned kb = blocks_for(h->N, kThreads);
    hipLaunchKernelGGL(k_hue_keys, dim3(kb < kKeyBlocks ? kb : kKeyBlocks), dim3(kThreads), 0, h->st,
                       rgb, h->N, h->n, h->keys, h->idx, h->counts);
    // hues lie in [0, 1): their FP32 patterns are below 2^30
    if (hipcub::DeviceRadixSort::SortPairs(h->temp, h->temp_bytes, h->keys, h->keys2, h->idx,
                                           h->order, (int)h->N, 0, 30, h->st) != hipSuccess)
        return OT_ERR_HIP;
    hipLaunchKernelGGL(k_hue_rank, dim3(blocks_for(h->N, kThreads)), dim3(kThreads), 0, h->st,
                       h->order, h->N, h->rank);
    if (hipGetLastError() != hipSuccess) return OT_ERR_HIP;
    h->src = rgb;
    h->have_source = true;
    h->have_frame = false;
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

int ot_hue_render(ot_hue* h, const float* target, unsigned char* rgb_out, int* bins_out) {
    if (!h || !target || !rgb_out) return OT_ERR_PARAM;
    if (!h->have_source) return OT_ERR_STATE;
    hipLaunchKernelGGL(k_hue_plan, dim3(1), dim3(kPlanThreads), 0, h->st, target, h->counts, h->n,
                       h->N, h->ct, h->cum, h->shift);
    hipLaunchKernelGGL(k_hue_render, dim3(blocks_for(h->N, kThreads)), dim3(kThreads), 0, h->st,
                       h->src, h->rank, h->cum, h->shift, h->n, h->N, rgb_out, bins_out);
    if (hipGetLastError() != hipSuccess) return OT_ERR_HIP;
    h->have_frame = true;
    return OT_OK;
}

int ot_hue_plan_info(ot_hue* h, int* counts, long long* shift) {
    if (!h) return OT_ERR_PARAM;
    if (!h->have_frame) return OT_ERR_STATE;
    if (counts && hipMemcpyAsync(counts, h->ct, h->n * sizeof(int), hipMemcpyDeviceToHost,
                                 h->st) != hipSuccess)
        return OT_ERR_HIP;
    if (shift && hipMemcpyAsync(shift, h->shift, sizeof(long long), hipMemcpyDeviceToHost,
                                h->st) != hipSuccess)
        return OT_ERR_HIP;
    return hipStreamSynchronize(h->st) == hipSuccess ? OT_OK : OT_ERR_HIP;
}

}  // extern "C"
