/*
 * ot_net.h -- learned warm start for the dynamic transport solver.
 *
 * The paper has no learned component; Algorithm 1 starts from zero.  This
 * library adds a small convolutional encoder-decoder that predicts the
 * initial primal iterate of Algorithm 1 from the two end densities, trained
 * on the GPU by its own kernels on pairs that the solver itself produced.
 * The solver then starts from that iterate with the dual that makes it a
 * fixed point of the prox step (OT_INIT_PRIMAL_DUAL in ot_dyn.h) and is
 * certified by the same residual tolerances as a cold start; a caller falls
 * back to a cold start when a warm run does not certify.
 *
 * Network (channels-last tensors [batch][H][W][channels], FP32 at the API):
 *   encoder levels l = 0..levels-1 of width w_l = base * 2^l, each two 3x3
 *   convolutions (zero padding, bias, ReLU), 2x2 average pooling between
 *   levels; decoder levels l = levels-2..0, each nearest 2x upsampling,
 *   concatenation [upsampled, encoder output of level l] and two 3x3
 *   convolutions with ReLU; a 1x1 output convolution without activation.
 *   Weights and activations are BF16 on the device, accumulation is FP32,
 *   the master weights and the Adam moments are FP32.
 *
 * Parameters are exchanged as one flat FP32 device vector: per layer in
 * execution order, the weights [k][k][C_in][C_out] (row-major) and then the
 * biases [C_out].
 *
 * Loss: sum over output channels c of cw[c] * sum over pixels of
 * (y - t)^2 / (batch * H * W).
 *
 * All pointers are device pointers unless stated; work is ordered on the
 * stream given at creation.  Status codes are those of ot_dyn.h.
 */
#ifndef OT_NET_H
#define OT_NET_H

#include <stddef.h>

#include "ot_dyn.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ot_net_desc {
    int H, W;              /* input resolution; multiples of 2^(levels-1)   */
    int in_ch, out_ch;     /* channels of the input and of the output        */
    int base, levels;      /* widths base * 2^l for l < levels (1..5)        */
    int max_batch;         /* largest batch passed to forward / grad / train */
    double beta1, beta2, eps;  /* Adam constants                             */
} ot_net_desc;

typedef struct ot_net ot_net;

/* Defaults: base 32, levels 4, Adam (0.9, 0.999, 1e-8). */
int ot_net_default_desc(int H, int W, int in_ch, int out_ch, int max_batch, ot_net_desc* d);

/* Number of FP32 entries of the flat parameter vector. */
int ot_net_param_count(const ot_net_desc* d, long long* count);

/* Bytes of device workspace (activations, gradients, BF16 weight copies,
 * master weights, Adam moments) the caller must provide. */
int ot_net_workspace_size(const ot_net_desc* d, size_t* bytes);

/* Carve the caller's workspace (256-byte aligned, >= workspace_size bytes;
 * owned by the caller, used until ot_net_destroy).  Parameters start at
 * zero: call ot_net_set_params before use. */
int ot_net_create(const ot_net_desc* d, void* stream, void* workspace, size_t ws_bytes,
                  ot_net** out);

/* Load the flat FP32 parameters (device); resets the Adam moments and the
 * step counter.  Asynchronous on the net's stream. */
int ot_net_set_params(ot_net* n, const float* params);

/* Write the FP32 master parameters to `params` (device). */
int ot_net_get_params(ot_net* n, float* params);

/* y[batch][H][W][out_ch] = network(x[batch][H][W][in_ch]).  1 <= batch <=
 * max_batch.  Asynchronous. */
int ot_net_forward(ot_net* n, int batch, const float* x, float* y);

/* Loss of the batch against the target t[batch][H][W][out_ch] with channel
 * weights cw[out_ch] (device), and its gradient with respect to the
 * parameters into grad (device, flat layout; may be NULL).  When loss is
 * non-NULL the call waits for the stream and stores the loss (host). */
int ot_net_grad(ot_net* n, int batch, const float* x, const float* t, const float* cw,
                float* grad, double* loss);

/* One Adam step with learning rate lr on the batch (gradient as in
 * ot_net_grad).  loss as in ot_net_grad. */
int ot_net_train_step(ot_net* n, int batch, const float* x, const float* t, const float* cw,
                      float lr, double* loss);

int ot_net_destroy(ot_net* n);
const char* ot_net_last_error(const ot_net* n);

/* ---- solver glue: the network's input and output for a problem of desc d --
 *
 * f0, f1: [batch][C][Y][X] end densities.  F, Mx, My, Mc: solver state in
 * the layout of ot_dyn.h; problem b starts at F + b * sF and M* + b * sM
 * (element strides), so both the plain batched buffers and the packed
 * state of ot_dyn_batch_get_state are accepted.
 *
 * Input channels (2C): f0 then f1.  Output channels (C(P-1) + 3CP):
 *   [0, C(P-1))              f at k/P, k = 1..P-1, minus the linear
 *                             interpolation (1 - k/P) f0 + (k/P) f1;
 *   then Mx, My, Mc, each P slots of C channels (slot k, colour c at
 *   k * C + c), wall slots included (they read as 0).
 */

/* Network input x[batch][Y][X][2C (+ OUT)]: f0, f1 and, when base is not
 * NULL, the OUT = C(P-1) + 3CP channels of base[batch][Y][X][OUT] (a state
 * in the target layout, e.g. a prolonged coarse solution). */
int ot_warm_inputs(const ot_dyn_desc* d, int batch, const float* f0, const float* f1,
                   const float* base, float* x, void* stream);

/* Training target t[batch][Y][X][OUT] from a solver state, minus base when
 * base is not NULL. */
int ot_warm_targets(const ot_dyn_desc* d, int batch, const float* f0, const float* f1,
                    const float* F, long long sF, const float* Mx, const float* My,
                    const float* Mc, long long sM, const float* base, float* t, void* stream);

/* Solver state from a network output y (layout of the targets; base added
 * when not NULL): writes the unknown slices of F and every slot of Mx, My,
 * Mc (wall slots 0).  F's end slices are written by ot_dyn_init. */
int ot_warm_state(const ot_dyn_desc* d, int batch, const float* f0, const float* f1,
                  const float* y, const float* base, float* F, long long sF, float* Mx,
                  float* My, float* Mc, long long sM, void* stream);

/* Coarse densities fc[batch][C][Y/2][X/2] = 2 x 2 block means of
 * f[batch][C][Y][X] (X, Y of the fine desc, both even).  Means keep the
 * total mass of a unit domain. */
int ot_warm_restrict(const ot_dyn_desc* fine, int batch, const float* f, float* fc,
                     void* stream);

/* Prolong a coarse solver state (X/2, Y/2, the same C and boundary
 * conditions, any P) to the fine grid: bilinear in space for cell-centred
 * values (Neumann ends clamped, periodic ends wrapped), linear between
 * faces for the staggered momenta (walls read as 0), linear in time.
 * Writes the unknown slices of F and every slot of Mx, My, Mc; strides as
 * above for both states. */
int ot_warm_prolong(const ot_dyn_desc* coarse, const ot_dyn_desc* fine, int batch,
                    const float* Fc, long long sFc, const float* Mxc, const float* Myc,
                    const float* Mcc, long long sMc, float* F, long long sF, float* Mx,
                    float* My, float* Mc, long long sM, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* OT_NET_H */
