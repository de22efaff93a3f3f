// Shared declarations of the HIP kernels and the host plan code.
//
// Layout (FP32, x fastest, batch outermost):
//   centred fields   [B][P][C][Y][X]   (duals b, b_bar, the residual r / phi,
//                                       the staggered work arrays a_*)
//   F                [B][P+1][C][Y][X] (times 0..P; 0 and P are f0 and f1)
//   Mx, My, Mc       [B][P][C][Y][X]   (slot i = face between cells i-1, i)
// The work array a_f uses the centred shape with slice k holding time k
// (slot 0 unused), so that a_f and F share (k, c, y, x) offsets.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace otd {

struct Geom {
    int B, X, Y, C, P;
    int perx, pery, perc;        // 1 if the axis is periodic (size > 1 only)
    float sx, sy, sc, st;        // difference factors n / extent, P
    long long plane;             // X * Y
    long long slice;             // C * X * Y
    long long nc;                // P * slice   (centred, per problem)
    long long nf;                // (P + 1) * slice (F, per problem)
};

// Reduction slots written by the update kernel (one FP64 partial per block).
enum RedSlot {
    RS_DB2 = 0,     // sum |b_new - b|^2  = |K x + c - z|^2
    RS_Z2,          // sum |z|^2
    RS_DX2,         // sum |x_new - x_old|^2
    RS_X2,          // sum |x_new|^2
    RS_J,           // sum J(z)
    RS_COUNT
};

// Transform tables (device), one set per axis; `n` = 1 means absent.
struct AxisTab {
    int n;
    int periodic;
    const float* mat;    // n x n forward matrix M[j][k] (row j = frequency)
    const float* lam;    // n eigenvalues of A A^T along this axis
    const float2* tw;    // fast path: tw[j] = e^{-i pi j / (2n)}, j < 4n; else null
    const float2* twm;   // mixed-radix path (mix_len(n)): the same table; else null
};

struct StepArgs {
    Geom g;
    float tau_sigma;     // tau * sigma (the same for every problem)
    int prox;            // root of the prox cubic: OT_PROX_NEWTON or OT_PROX_CLOSED
    const float* sig;    // sigma per problem [B] (device; residual balancing)
    const float* frz;    // per problem [B]: nonzero = frozen (a certified member of a
                         // batch): the initialisation kernels skip it
    const float* frz_run;  // the same flags for the iteration kernels, or null for a
                           // plan outside a batch (no frozen problems; the kernels
                           // then start without waiting for a flag load)
    float theta;
    // state
    float* F; float* Mx; float* My; float* Mc;
    float* b[4]; float* bb[4];
    float* A[4];         // staggered work arrays a_x, a_y, a_c, a_f
    float* R;            // residual r, transformed in place into phi_1
    float* R2;           // refinement: residual of x' = a + grad phi_1 -> phi_2
    float* Phi;          // carried potential (sum of the previous phi_1), or null
    double* part_slice;  // [B*P*C][nbx] FP64 block partials of the plane sums of r
    double* part_red;    // [RS_COUNT][B][P*C*nbx] FP64 residual partials
    double* part_mass;   // [B*P*C][nbx] FP64 slice sums of f_new
    double* part_div;    // [B*P*C][nbx] FP64 sum of (A x - f_b^-)^2
    int nbx;             // blocks per (b, k, c) slice in the stencil kernels
    int row_bx;          // block width of the row stencil kernels (64, 128 or 256)
    // forward transform along x folded into the divergence kernels (their
    // block owns whole rows of every colour): x twiddles of the fast path,
    // or null when the x pass runs on its own; kind 0 DCT-II, 2 Hartley
    const float2* twx;
    int xkind;
    // the fused Poisson solve: the divergence kernels write r already
    // transformed across colours, cmix[c C + jc] = M_c[jc][c] (else null)
    const float* cmix;
    // nonzero: the iteration's fields are stored non-temporally (fields of
    // 16 MB and more, whose working set the caches cannot hold)
    int nt_store;
};

// ---- stencil kernels (stencil.hip) -------------------------------------
// mode 0: a from (x, b_bar); writes A and r into R.  mode 1 (refinement):
// residual of x' = A + grad R into R2.  mode 2: as mode 0 with a + grad Phi.
void launch_div(const StepArgs& s, int mode, hipStream_t st);
// x = a + grad(phi_1) (+ grad(phi_2) if nphi == 2 or 4), prox, dual update;
// nphi == 3 and 4 also add the potentials into Phi; residual partials if
// `check`.
void launch_update(const StepArgs& s, int check, int nphi, hipStream_t st);
// Row-marching variants (stencil_rows.hip), used when 1 <= C <= 4: one
// thread per (b, k, y, x) for all colours, XCD-aware block order.  Their
// plane partial stride is Y * ceil(X / row_bx); row_block(X) is the default
// width (X rounded up to a multiple of 64, at most 256).
int row_block(int X);
bool rows_ok(const Geom& g);
void launch_div_rows(const StepArgs& s, int mode, hipStream_t st);
// The forward x transform can be folded into the row divergence kernels
// (StepArgs::twx): rows of fast length 64, 128 or 256, one block per row.
bool div_fold_ok(const Geom& g, int row_bx, const AxisTab& tx);
void launch_update_rows(const StepArgs& s, int check, int nphi, hipStream_t st);
// FP64 partials of |A x - f_b^-|^2 and of the slice masses of F.
void launch_resid_div(const StepArgs& s, hipStream_t st);
// FP64 partials of the residual slots RS_DB2, RS_Z2, RS_X2 and RS_J (RS_DX2
// zero) of the current state, z = prox(K x + c + b), nothing written but
// part_red: one partial per block of the per-node grid, [RS_COUNT][B][P C
// ceil(X Y / 256)].
void launch_resid_state(const StepArgs& s, hipStream_t st);
// Boundary slices, wall slots and (optionally) zero unknowns; zeroes Phi
// when it is set.
void launch_init_state(const StepArgs& s, const float* f0, const float* f1,
                       int zero_unknowns, hipStream_t st);
// b = b_bar = grad J(K x + c) / sigma from a caller-filled primal.
// vfloor: per problem, the density floor of the velocity u / v (device)
void launch_init_dual(const StepArgs& s, const double* vfloor, hipStream_t st);
// zero the dual fields
void launch_zero_dual(const StepArgs& s, hipStream_t st);
// b and b_bar of problem q times fac[q] (device [B]): keeps the unscaled dual
// sigma b when sigma changes
void launch_scale_dual(const StepArgs& s, const float* fac, hipStream_t st);
// The pointwise prox on n nodes (am, u: [3][n]; af, v: [n]), `kind` as
// OT_PROX_* (ot_dyn_prox_eval).
void launch_prox_eval(int kind, long long n, const float* am, const float* af, float sigma,
                      float* u, float* v, hipStream_t st);
// FP64 mass partials and input checks of f0, f1 ([B][C][Y][X]).
void launch_boundary_stats(const Geom& g, const float* f0, const float* f1,
                           double* part, int nblk, hipStream_t st);

// ---- transforms (transform.hip) ----------------------------------------
// FP64 plane sums reduced in place: part[q nbx] = sum_i part[q nbx + i] for
// every plane q < nq (the layout of StepArgs::part_slice).
struct PlaneSums {
    double* part;
    long long nq;
    int nbx;
};
// Rows of a row pass that belong to frozen problems: frz[b] nonzero for
// problem b, rpp rows per problem (null frz: none).
struct RowSkip {
    const float* frz;
    long long rpp;
};
// True when rows [r0, r0 + n) all belong to frozen problems (block-uniform
// when r0 and n are).
__device__ inline bool rows_frozen(const RowSkip& k, long long r0, int n) {
    if (!k.frz) return false;
    for (long long b = r0 / k.rpp; b <= (r0 + n - 1) / k.rpp; ++b)
        if (k.frz[b] == 0.f) return false;
    return true;
}
// Forward or inverse orthonormal transform along x (contiguous rows).  With
// `sums`, the fast path also reduces those plane sums (extra blocks of the
// same launch) and returns true; otherwise it returns false and leaves them.
// Blocks whose rows all belong to problems frozen in `skip` do nothing.
bool launch_rows(float* R, long long rows, const AxisTab& t, int inverse, hipStream_t st,
                 const PlaneSums* sums = nullptr, RowSkip skip = RowSkip{nullptr, 1});
// Forward or inverse transform along a strided axis: data [outer][L][inner].
// With `sums`, the fast path also reduces those plane sums (as launch_rows)
// and returns true.
bool launch_cols(float* R, long long outer, long long inner, const AxisTab& t,
                 int inverse, hipStream_t st, const PlaneSums* sums = nullptr);
// Colour and time transforms, division by the eigenvalues of A A^T, inverse
// transforms; the spatial-DC line is solved in FP64 from the slice sums
// (already reduced to part_slice[q nbx] when `presummed`).
void launch_tc(const Geom& g, float* R, const AxisTab& tx, const AxisTab& ty,
               const AxisTab& tc, const AxisTab& tt, const double* tc64,
               const double* tt64, double* part_slice, int nbx, int presummed,
               const float* frz, hipStream_t st);

// Fused Poisson passes (transform.hip) for Neumann x and y of length 32..256,
// P in {8, 16, 32}, C in {1, 3}: x (+ colour) pass with a transposed write to
// Rt ([B][C][X][Y][P]; the forward pass also reduces the plane sums of r in
// part_slice in place; with premixed r is already in colour modes, see
// StepArgs::cmix), the y + t pass in place on Rt, and the mirrored inverse,
// which also solves the spatial-DC line in FP64 and adds it.
bool fused_poisson_ok(const Geom& g, const AxisTab& tx, const AxisTab& ty, const AxisTab& tt);
void launch_fused_x(const Geom& g, float* R, float* Rt, const AxisTab& tx,
                    const AxisTab& ty, const AxisTab& tc, const AxisTab& tt, const double* tc64,
                    const double* tt64, double* part_slice, int nbx, int inverse,
                    bool premixed, hipStream_t st);
void launch_fused_yt(const Geom& g, float* Rt, const AxisTab& tx, const AxisTab& ty,
                     const AxisTab& tc, const AxisTab& tt, hipStream_t st);

// Whole Poisson solve of problems with one spatial axis (transform.hip):
// Y = C = 1, P in {8, 16, 32}, X in {64, 128, 256} with its fast transform
// or X <= 480 with the dense transform on the matrix cores; one block per
// problem, frozen problems skipped.
// Lengths L = 2 M1 M2 (factors 2, 3 and 5) with mixed-radix line transforms
// (x and y passes, one-block 1D solve) instead of dense contractions: 100,
// 180 and 360.
bool mix_len(int n);
void launch_rows_mix(float* R, long long rows, int L, const float2* tw, int kind, hipStream_t st,
                     const PlaneSums* sums, RowSkip sk);
void launch_cols_mix(float* R, long long outer, long long inner, int L, const float2* tw, int kind,
                     hipStream_t st, const PlaneSums* sums);
bool poisson_1d_ok(const Geom& g, const AxisTab& tx, const AxisTab& tt);
void launch_poisson_1d(const Geom& g, float* R, const AxisTab& tx, const AxisTab& ty,
                       const AxisTab& tc, const AxisTab& tt, const double* tc64,
                       const double* tt64, const float* frz, hipStream_t st);

// Fast power-of-two passes (fastdct.hip); kind 0 DCT-II, 1 DCT-III, 2 Hartley.
bool fast_len(int L);
// The four-step split M1 x M2 (M1 M2 = L / 2) of the power-of-two line
// transforms of length L (32..512), shared by the kernels and the host: the
// fast twiddle table of an axis has, after its 4 L entries, the first-stage
// twiddles e^{-2 pi i t k1 / (L / 2)} at [4 L + t M1 + k1], t < M2, k1 < M1.
__host__ __device__ constexpr int fft_m1(int L) { return L == 32 ? 4 : L <= 128 ? 8 : 16; }
void launch_rows_fast(float* R, long long rows, int L, const float2* tw, int kind, hipStream_t st,
                      const PlaneSums* sums = nullptr, RowSkip skip = RowSkip{nullptr, 1});
void launch_cols_fast(float* R, long long outer, long long inner, int L, const float2* tw, int kind,
                      hipStream_t st, const PlaneSums* sums = nullptr);

// ---- plan internals used by the batched solver (plan.cpp) ---------------
}  // namespace otd
struct ot_dyn_plan;
struct ot_dyn_report;
namespace otd {
void plan_iterate(ot_dyn_plan* p, float* F, float* Mx, float* My, float* Mc, bool check);
int plan_collect(ot_dyn_plan* p, float* F, float* Mx, float* My, float* Mc);
void plan_apply_tuning(ot_dyn_plan* p, int row_bx, int dense_xy);
bool plan_has_fast_xy(const ot_dyn_plan* p);
// Marks a batch group's plan: its iteration kernels read the frozen flags
// (call before the first launch or capture).
void plan_enable_freeze(ot_dyn_plan* p);
void plan_problem(const ot_dyn_plan* p, int b, ot_dyn_report* rep);
void plan_add_iters(ot_dyn_plan* p, int n);
// Freezes problem b (frozen[b] nonzero) or releases it; uploads on the
// plan's stream only when a flag changes.
int plan_freeze(ot_dyn_plan* p, const std::vector<char>& frozen);
// True while the launch sequence of the next iteration may differ from the
// one after it (adaptive refinement; the refined start of OT_REFINE_CARRY):
// a captured graph of iterations must then be captured again.
bool plan_launch_varies(const ot_dyn_plan* p);
// Restart the problems b with which[b] nonzero from Algorithm 1's cold
// start (state, dual, carried potential, step sizes) and release them; the
// others keep their state and frozen flags.  Synchronises the plan's stream.
int plan_restart_cold(ot_dyn_plan* p, float* F, float* Mx, float* My, float* Mc,
                      const std::vector<char>& which);
// Copy the dual b of problem b to (to_packed = 1) or from (0, also b_bar) a
// packed [4][P][C][Y][X] array; asynchronous on the plan's stream.
int plan_copy_dual(ot_dyn_plan* p, int b, float* packed, int to_packed);

// ---- reductions (stencil.hip) ------------------------------------------
// out[q] = sum_j part[q * n + j] in FP64, for q < nq.
void launch_reduce(const double* part, long long n, int nq, double* out, hipStream_t st);

}  // namespace otd
