// Internal interface between the network host code and its kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace otn {

typedef uint16_t bf16_t;   // BF16 storage (upper half of an IEEE float)

enum { MODE_CONV = 0, MODE_WGRAD = 1 };
enum { EPI_RELU = 0, EPI_F32 = 1, EPI_PLAIN = 2, EPI_MASK = 3, EPI_PART = 4 };

// One implicit GEMM of a convolution layer.
//   MODE_CONV:  out[p][n] = sum_k A[p][k] W[n][k],  A[p][(tap, c)] = src at
//               pixel p shifted by tap, channel c (0 outside the image);
//               forward (W = weights) and input gradient (W = flipped
//               transposed weights, src = output gradient) alike.
//   MODE_WGRAD: part[z][i][n] = sum over pixels q in split z of
//               A[i][q] dz[q][n], A[(tap, c)][q] = src at q shifted by tap,
//               plus a row of ones (i = taps * cin) that yields the bias
//               gradient.
struct ConvArgs {
    const bf16_t* src;
    int src_ld;            // pixel stride of src (elements)
    int cin;               // gathered channels (multiple of 8)
    int taps;              // 9 or 1
    const bf16_t* wmat;    // MODE_CONV: [N][K] with K = taps * cin
    const bf16_t* dz;      // MODE_WGRAD: [pixels][dz_ld]
    int dz_ld;
    int nb, H, W;
    int M, N, K;
    void* dst;
    int dst_ld, dst_off, dst_n;
    const float* bias;
    const bf16_t* mask;    // EPI_MASK: [pixels][mask_ld]
    int mask_ld;
    int ksplit;            // MODE_WGRAD: pixels per split
};

// A channels-last view: element (pixel p, channel c) at ptr[p * ld + c].
struct View {
    bf16_t* ptr;
    int ld;
};

void launch_conv(const ConvArgs& a, int mode, int epi, int splits, hipStream_t st);
void launch_wgrad_reduce(const float* part, int splits, int M, int N, float* out, hipStream_t st);
void launch_pack_input(const float* x, int in_ch, long long npix, bf16_t* out, int ld,
                       hipStream_t st);
void launch_pool(View src, int C, int nb, int H, int W, bf16_t* dst, hipStream_t st);
void launch_upsample(const bf16_t* src, int C, int nb, int h, int w, View dst, hipStream_t st);
void launch_up_bwd(View g, int C, int nb, int h, int w, const bf16_t* hlow, bf16_t* out,
                   hipStream_t st);
void launch_merge(const bf16_t* gpool, View gcat, View cat, int C, int nb, int H, int W,
                  bf16_t* out, hipStream_t st);
int loss_blocks(long long n);
void launch_loss(const float* y, const float* t, const float* cw, int out_ch, int out_p,
                 long long npix, bf16_t* dy, double* part, hipStream_t st);
void launch_sum(const double* part, int n, double* out, hipStream_t st);
void launch_adam(float* p, float* m, float* v, const float* g, long long n, float lr, float b1,
                 float b2, float eps, float c1, float c2, hipStream_t st);
void launch_export(const float* w, int taps, int cin, int cout, bf16_t* wf, bf16_t* wb,
                   hipStream_t st);
void launch_param_map(const float* src, float* dst, int taps, int cin_o, int cout_o, int cin_p,
                      int cout_p, int to_padded, hipStream_t st);

// solver glue
struct WarmGeom {
    int X, Y, C, P;
    int perx, pery, perc;
};
void launch_warm_inputs(const WarmGeom& g, int nb, const float* f0, const float* f1,
                        const float* base, float* x, hipStream_t st);
void launch_warm_targets(const WarmGeom& g, int nb, const float* f0, const float* f1,
                         const float* F, long long sF, const float* Mx, const float* My,
                         const float* Mc, long long sM, const float* base, float* t,
                         hipStream_t st);
void launch_warm_state(const WarmGeom& g, int nb, const float* f0, const float* f1,
                       const float* y, const float* base, float* F, long long sF, float* Mx,
                       float* My, float* Mc, long long sM, hipStream_t st);
void launch_restrict(const WarmGeom& gc, int nb, const float* f, float* fc, hipStream_t st);
void launch_prolong(const WarmGeom& gc, const WarmGeom& gf, int nb, const float* Fc,
                    long long sFc, const float* Mxc, const float* Myc, const float* Mcc,
                    long long sMc, float* F, long long sF, float* Mx, float* My, float* Mc,
                    long long sM, hipStream_t st);

}  // namespace otn
