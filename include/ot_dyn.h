/*
 * ot_dyn.h -- C ABI of the MI355X (gfx950) dynamic optimal transport solver.
 *
 * The library runs Algorithm 1 of Fitschen, Laus and Steidl, "Dynamic
 * Optimal Transport with Mixed Boundary Conditions for Color Image
 * Processing" (the PDHG iteration of Sec. 3) on the staggered grid of Sec. 2
 * extended to 4D (Remark 2): Neumann boundaries in x, y and time, periodic
 * (by default) in the colour axis.  Each iteration is
 *   Step 1  a = x - tau sigma K^T b_bar;  x = a - A^T (A A^T)^+ (A a - f_b^-)
 *           (the pseudo-inverse by fast transforms, Sec. 3 and Remark 2),
 *   Step 2  z = prox of J / sigma at K x + c + b (the cubic of Sec. 3),
 *   Steps 3-4  b += K x + c - z;  b_bar = b + theta (b - b_old).
 *
 * Conventions for every entry point:
 *   - All functions return an int status: 0 = OT_OK, < 0 an error, > 0 a
 *     warning.  No exception or longjmp crosses this boundary.
 *   - Pointers named f0, f1, F, Mx, My, Mc, workspace are DEVICE pointers
 *     (hipMalloc'd or torch CUDA tensors on the plan's device).  Pointers to
 *     ot_dyn_desc, ot_dyn_report and ot_dyn_plan* are HOST pointers.
 *   - The library never allocates device memory: all device storage is the
 *     caller's (state buffers and one workspace of ot_dyn_workspace_size
 *     bytes, 256-byte aligned).  The plan object is host memory owned by the
 *     library (ot_dyn_create / ot_dyn_destroy).
 *   - A plan is bound to one HIP stream; calls on one plan must not overlap
 *     from several host threads.
 *
 * Buffer layout (FP32, x fastest, `batch` independent problems of the same
 * shape stacked outermost):
 *   F   [batch][P+1][C][Y][X]  density at times k/P.  Slices 0 and P hold f0
 *                              and f1 (written by ot_dyn_init, read-only to
 *                              the solver); slices 1..P-1 are the unknowns.
 *   Mx  [batch][P][C][Y][X]    x-momentum at half-time (k+1/2)/P; slot x is
 *                              the face between cells x-1 and x.  Neumann:
 *                              slot 0 is the wall and stays 0 (face X is
 *                              implicit).  Periodic: slot 0 is the face
 *                              between cells X-1 and 0.
 *   My  [batch][P][C][Y][X]    same along y.
 *   Mc  [batch][P][C][Y][X]    same along the colour axis.
 */
#ifndef OT_DYN_H
#define OT_DYN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define OT_OK               0
#define OT_NOT_CONVERGED    1   /* warning: max_iters reached before tolerance */
#define OT_ERR_PARAM       -1   /* tau, sigma, theta, tolerances out of range  */
#define OT_ERR_SHAPE       -2   /* sizes out of range or buffer too small      */
#define OT_ERR_INPUT       -3   /* negative or non-finite density              */
#define OT_ERR_MASS        -4   /* |M0 - M1| / M0 above tol_mass               */
#define OT_ERR_HIP         -5   /* a HIP runtime call failed                   */
#define OT_ERR_NONFINITE   -6   /* non-finite residual during the iteration    */
#define OT_ERR_STATE       -7   /* call out of order (e.g. step before init)   */

/* boundary condition of a spatial axis (Sec. 2: kappa = 1 Neumann, 0 periodic) */
#define OT_BC_NEUMANN   0
#define OT_BC_PERIODIC  1

/* initialisation modes of ot_dyn_init */
#define OT_INIT_COLD         0  /* Algorithm 1: m = 0, f = 0, b = b_bar = 0          */
#define OT_INIT_PRIMAL       1  /* caller-filled (F, M), b = b_bar = 0               */
#define OT_INIT_PRIMAL_DUAL  2  /* caller-filled (F, M); b = b_bar = grad J(Kx+c)/sigma,
                                   the centred density floored at 1e-3 times
                                   the mean of f0 (near-vacuum nodes)        */
/* Flag, OR-ed into OT_INIT_PRIMAL or OT_INIT_PRIMAL_DUAL (ot_dyn_init,
 * ot_dyn_batch_set_state): the next ot_dyn_solve / ot_dyn_batch_solve
 * certifies the warm start or falls back to Algorithm 1's cold start.  A
 * warm-started problem that is not certified within max_iters (or whose
 * residual turns non-finite) is initialised cold and solved again with a
 * budget of another max_iters; its report has fallback = 1 and counts the
 * iterations of both runs.  The flag is consumed by that one solve. */
#define OT_INIT_FALLBACK     4

/* FP32 accuracy of the projection onto the continuity constraint (Sec. 3,
 * Step 1: x = a - A^T (A A^T)^+ (A a - f_b^-)).  The transform solve in FP32
 * leaves an error proportional to |A a - f_b^-|; the modes differ in how it
 * is reduced.  The projection is affine and Pi(a) = Pi(a - A^T Phi) for any
 * potential Phi, which OT_REFINE_CARRY uses with the previous iteration's
 * potential: the residual it solves for then vanishes as the iteration
 * converges (one transform solve per iteration; the default). */
#define OT_REFINE_OFF       0  /* one FP32 solve of the full residual            */
#define OT_REFINE_ALWAYS    1  /* second solve for the residual of the first     */
#define OT_REFINE_ADAPTIVE  2  /* OFF until max(r_prim, r_dual) < 1e-4, then ALWAYS */
#define OT_REFINE_CARRY     3  /* one solve, started from the carried potential  */

/* Root of the prox cubic 2 (1 + sigma v)^2 (v - a_f) = sigma |a_m|^2
 * (ot_dyn_desc.prox).  NEWTON: monotone Newton steps from the right of the
 * root to relative change 1e-6.  CLOSED: Cardano's formula in w = 1 + sigma v
 * (for 1 + sigma a_f <= 0 in s = 1 / w, where the positive root is well
 * conditioned), then one Newton step in v, which restores the digits that
 * v = (w - 1) / sigma loses in FP32 when sigma v << 1. */
#define OT_PROX_NEWTON      0
#define OT_PROX_CLOSED      1
#define OT_PROX_CLOSED_RAW  2  /* ot_dyn_prox_eval only: no Newton step */

typedef struct ot_dyn_desc {
    int X, Y, C, P;        /* grid: X x Y pixels, C channels, P time steps; an
                              axis of size 1 is absent.  P >= 2.              */
    int bc[3];             /* per spatial axis (x, y, colour): OT_BC_*        */
    double extent[3];      /* physical length per spatial axis (default 1):
                              the difference factor is size / extent          */
    double tau, sigma;     /* step sizes, tau * sigma < 1 (Algorithm 1)       */
    double theta;          /* extrapolation, 0 <= theta <= 1 (1 in the paper) */
    int check_every;       /* ot_dyn_solve: residual check interval (>= 1)    */
    double tol_res;        /* stop when max(r_prim, r_dual) < tol_res ...     */
    double tol_div;        /* ... and r_div < tol_div                         */
    double tol_mass;       /* admissible |M0 - M1| / M0 of the end densities  */
    int refine;            /* FP32 accuracy of the projection: OT_REFINE_*  */
    int batch;             /* number of stacked problems of this shape (>= 1) */
    int adapt;             /* step sizes: 0 fixed (tau, sigma as given), 1
                              balanced per problem at residual checks (sigma
                              halved or doubled towards r_prim ~ r_dual, at
                              most 4 times, none once both are below 3e-5);
                              tau sigma stays fixed.  Helps 1D periodic (hue)
                              problems, slows the RGB ones: off by default */
    int prox;              /* root of the prox cubic (Sec. 3, Step 2):
                              OT_PROX_NEWTON or OT_PROX_CLOSED */
    int carry_refine;      /* OT_REFINE_CARRY: the first carry_refine
                              iterations after ot_dyn_init also run the
                              refinement solve (early on the carried
                              potential predicts little); >= 0, default 64 */
} ot_dyn_desc;

typedef struct ot_dyn_report {
    int iterations;        /* iterations run by this call                     */
    int converged;         /* 1 if the tolerances were met                    */
    int total_iterations;  /* iterations since the last ot_dyn_init           */
    int worst_problem;     /* batch index with the largest residual           */
    double r_prim;         /* ||Kx + c - z|| / ||z||          (max over batch) */
    double r_dual;         /* ||x_new - x_old|| / ||x_new||   (max over batch) */
    double r_div;          /* ||A x - f_b^-|| / ||f_b^-||     (max over batch) */
    double cost;           /* cell volume * sum J(z)  (problem 0)             */
    double e_mass;         /* max_k |sum f(., k/P) - M0| / M0 (max over batch) */
    double mass0, mass1;   /* FP64 masses of f0 and f1 (problem 0)            */
    double ms;             /* wall time of the call in milliseconds           */
    int fallback;          /* 1 if a warm start was abandoned for a cold start
                              (OT_INIT_FALLBACK); batches: the count        */
} ot_dyn_report;

typedef struct ot_dyn_plan ot_dyn_plan;

/* Fill *d with the defaults for an X x Y x C x P grid: bc = {Neumann,
 * Neumann, periodic}, extent = 1, tau = 10, sigma = 0.099, theta = 1,
 * check_every = 50, tol_res = 1e-6, tol_div = 1e-6, tol_mass = 1e-5,
 * refine = OT_REFINE_CARRY, batch = 1, adapt = 0, prox = OT_PROX_NEWTON,
 * carry_refine = 64. */
int ot_dyn_default_desc(ot_dyn_desc* d, int X, int Y, int C, int P);

/* Bytes of device workspace a plan for *d needs (OT_ERR_SHAPE/PARAM if *d
 * is invalid). */
int ot_dyn_workspace_size(const ot_dyn_desc* d, size_t* bytes);

/* Create a plan for *d bound to `stream` (a hipStream_t; NULL = default
 * stream) over the caller's device workspace of ws_bytes bytes.  Uploads
 * the transform tables (DCT-II along Neumann axes, discrete Hartley along
 * periodic axes -- a real basis that diagonalises the periodic Laplacian
 * like the Fourier matrix of Sec. 3 -- and the eigenvalues of A A^T).
 * On error *out is NULL. */
int ot_dyn_create(const ot_dyn_desc* d, void* stream, void* workspace,
                  size_t ws_bytes, ot_dyn_plan** out);

/* Copy the end densities f0, f1 ([batch][C][Y][X], device) into the plan
 * (Sec. 2: f^0, f^1 >= 0 with equal l1 mass), compute their FP64 masses and
 * check them.  Returns OT_ERR_INPUT for a negative or non-finite value and
 * OT_ERR_MASS when |M0 - M1| / M0 > tol_mass; synchronises the stream. */
int ot_dyn_set_boundary(ot_dyn_plan* p, const float* f0, const float* f1);

/* Initialise the iteration state.  Writes slices 0 and P of F, the Neumann
 * wall slots of Mx/My/Mc and, for OT_INIT_COLD, zeros the unknowns
 * (Algorithm 1 initialisation).  The duals live in the workspace.  `mode`
 * is one of OT_INIT_*, optionally with OT_INIT_FALLBACK (warm modes only). */
int ot_dyn_init(ot_dyn_plan* p, int mode, float* F, float* Mx, float* My, float* Mc);

/* Run `iters` iterations of Algorithm 1 on the plan's stream without host
 * synchronisation.  (F, Mx, My, Mc) must be the buffers passed to
 * ot_dyn_init (or copies of them); they are updated in place. */
int ot_dyn_step(ot_dyn_plan* p, float* F, float* Mx, float* My, float* Mc, int iters);

/* Iterate until certified (max(r_prim, r_dual) < tol_res and r_div <
 * tol_div, checked every check_every iterations) or max_iters.  Returns
 * OT_OK when certified, OT_NOT_CONVERGED otherwise, OT_ERR_NONFINITE on a
 * non-finite residual.  Synchronous.  rep may be NULL. */
int ot_dyn_solve(ot_dyn_plan* p, float* F, float* Mx, float* My, float* Mc,
                 int max_iters, ot_dyn_report* rep);

/* Residuals of the current state (x, b) without iterating: the state is
 * left bitwise unchanged.  FP64 reductions; synchronous.  Fills
 *   r_div, e_mass   of x, as at a residual check;
 *   r_prim, cost    from z = prox of J / sigma at K x + c + b (Sec. 3,
 *                   Step 2): r_prim = ||K x + c - z|| / ||z|| and cost = cell
 *                   volume * sum J(z); both vanish / reach the minimum at a
 *                   fixed point of Algorithm 1;
 *   r_dual          needs the previous iterate: the value of the last residual
 *                   check since ot_dyn_init, or -1 if there was none.
 * iterations = 0, converged = 0. */
int ot_dyn_residuals(ot_dyn_plan* p, float* F, float* Mx, float* My, float* Mc,
                     ot_dyn_report* rep);

/* ---- phase timing ----------------------------------------------------
 * When a phase is enabled, every launch of it by ot_dyn_step / ot_dyn_solve
 * is bracketed by two HIP events recorded on the plan's stream.  Phases:   */
#define OT_PHASE_DIV      0  /* adjoint averages and divergence: a, r (Step 1)    */
#define OT_PHASE_XFORM_X  1  /* transforms along x (forward and inverse)          */
#define OT_PHASE_XFORM_Y  2  /* transforms along y (forward and inverse)          */
#define OT_PHASE_TC       3  /* colour/time transforms and eigenvalue division    */
#define OT_PHASE_REFINE   4  /* refinement: residual of a + grad phi_1           */
#define OT_PHASE_UPDATE   5  /* x = a + grad phi(s), prox, dual steps (Steps 2-4) */
#define OT_PHASE_COUNT    6

/* Enable event timing for the phases in bit mask `mask` (0 disables) and
 * reset the accumulators. */
int ot_dyn_profile(ot_dyn_plan* p, int mask);

/* The dual iterate b of Algorithm 1 (Steps 2-4), copied to or from b
 * [batch][4][P][C][Y][X] (device; components x, y, colour, time of the
 * centred grid).  ot_dyn_set_dual also sets b_bar = b; call it after
 * ot_dyn_init to start from a given primal-dual pair.  Asynchronous on the
 * plan's stream. */
int ot_dyn_get_dual(ot_dyn_plan* p, float* b);
int ot_dyn_set_dual(ot_dyn_plan* p, const float* b);

/* The extrapolated dual b_bar = b + theta (b - b_old) of Step 4, which the
 * next iteration's Step 1 reads, copied to b_bar [batch][4][P][C][Y][X]
 * (device); with b (ot_dyn_get_dual) and (F, M) it is the whole state the
 * next iteration depends on (up to FP32 rounding of the projection).
 * Asynchronous on the plan's stream. */
int ot_dyn_get_dual_bar(ot_dyn_plan* p, float* b_bar);

/* Synchronise the stream and return, per phase (n <= OT_PHASE_COUNT
 * entries), the accumulated milliseconds and launch counts since the last
 * ot_dyn_profile call.  ms and launches are host arrays of n entries. */
int ot_dyn_profile_read(ot_dyn_plan* p, double* ms, long long* launches, int n);

/* Release the plan (host memory only; device buffers stay the caller's). */
int ot_dyn_destroy(ot_dyn_plan* p);

/* ---- batched problems of uneven sizes ---------------------------------
 * Many independent problems (RGB images of different resolutions, 1D
 * periodic hue histograms of different bin counts -- Sec. 5 of the paper
 * transports such histograms with X = bins, Y = C = 1, bc[0] periodic)
 * solved together.  Problems are grouped by shape; each group is one batched
 * plan, and a chunk of iterations of every active group is captured into
 * one HIP graph with a branch per group (each on the group's own stream).
 * Per-group launch shapes can be autotuned.
 *
 * dims: host array of count x 4 ints (X, Y, C, P) per problem.  The other
 * descriptor fields (bc, extent, tau, sigma, theta, tolerances, refine,
 * check_every) come from *base; base->batch is ignored.
 *
 * Packed device layout of the caller's arrays (problem i in order):
 *   f0, f1 : C*Y*X floats each at offset off_h[i]
 *   F      : (P+1)*C*Y*X floats at offset off_F[i]
 *   M      : 3*P*C*Y*X floats at offset off_M[i] (Mx, then My, then Mc)
 * with the per-problem layouts of the single-problem API. */
typedef struct ot_dyn_batch ot_dyn_batch;

int ot_dyn_batch_workspace_size(const ot_dyn_desc* base, int count, const int* dims,
                                size_t* bytes);

/* Create the batch over the caller's workspace (no device allocation; the
 * batch creates one HIP stream per shape group, all of default priority). */
int ot_dyn_batch_create(const ot_dyn_desc* base, int count, const int* dims, void* stream,
                        void* workspace, size_t ws_bytes, ot_dyn_batch** out);

/* Packed offsets (host arrays of count + 1 entries; the last is the total). */
int ot_dyn_batch_offsets(const ot_dyn_batch* bt, long long* off_h, long long* off_F,
                         long long* off_M);

/* Gather the packed end densities into the groups and check them per
 * problem (as ot_dyn_set_boundary). */
int ot_dyn_batch_set_boundary(ot_dyn_batch* bt, const float* f0, const float* f1);

/* Autotune each group's launch shapes (row-stencil block width, FFT or dense
 * x/y transforms) by timing `trials` iterations per candidate on the group's
 * own buffers; results are cached in the file named by the environment
 * variable OT_DYN_TUNE_CACHE when it is set.  Leaves the state cold-started. */
int ot_dyn_batch_autotune(ot_dyn_batch* bt, int trials);

/* Start the next ot_dyn_batch_solve from the caller's packed F and M
 * (device, layout of ot_dyn_batch_get_state) instead of a cold start: the
 * state is copied and initialised with `mode` (OT_INIT_PRIMAL or
 * OT_INIT_PRIMAL_DUAL, see ot_dyn_init, optionally with OT_INIT_FALLBACK:
 * then each problem not certified from its warm start is restarted cold).  Problems whose packed state is
 * not wanted warm can be given a cold state (zeros).  Consumed by the next
 * solve. */
int ot_dyn_batch_set_state(ot_dyn_batch* bt, const float* F, const float* M, int mode);

/* Cold-start every problem (or start from the state of
 * ot_dyn_batch_set_state) and iterate (graph chunks of `chunk` iterations,
 * residuals checked after each chunk) until every problem is certified or
 * max_iters.  A certified problem is frozen at the check that certified it:
 * its state (ot_dyn_batch_get_state) and report are those of that check
 * while the rest of its shape group iterates on.  rep (may be NULL)
 * receives the batch totals: iterations, the
 * number certified in `converged`, the worst residuals and the wall time.
 * Returns OT_OK when all are certified, OT_NOT_CONVERGED otherwise.  With
 * the environment variable OT_DYN_VERBOSE set, one progress line per chunk
 * goes to stderr. */
int ot_dyn_batch_solve(ot_dyn_batch* bt, int max_iters, int chunk, ot_dyn_report* rep);

/* Per-problem result of the last solve: iterations until certified (or run),
 * residuals, cost, masses. */
int ot_dyn_batch_problem(const ot_dyn_batch* bt, int i, ot_dyn_report* rep);

/* Scatter the solution into the caller's packed F and M (device). */
int ot_dyn_batch_get_state(ot_dyn_batch* bt, float* F, float* M);

/* Packed duals (see ot_dyn_get_dual): problem i occupies 4 P_i C_i Y_i X_i
 * floats at 4/3 of its offset in the packed M.  ot_dyn_batch_set_dual
 * follows ot_dyn_batch_set_state (mode OT_INIT_PRIMAL) and replaces the
 * starting dual (and b_bar) of the next solve. */
int ot_dyn_batch_get_dual(ot_dyn_batch* bt, float* Bd);
int ot_dyn_batch_set_dual(ot_dyn_batch* bt, const float* Bd);

/* Selected launch shape of the group holding problem i: row_bx is the block
 * width of the row stencils (64, 128, 256); dense_xy the transform path (0
 * fused three-pass Poisson solve where it applies, else five FFT passes; 1
 * dense x/y contractions; 2 five FFT passes).  For problems with one spatial
 * axis (Y = C = 1, P in {8, 16, 32}) paths 0 and 2 solve the whole Poisson
 * problem in one block per problem (fast transform for X in {64, 128, 256},
 * dense contraction on the matrix cores for other X up to 416). */
int ot_dyn_batch_tuning(const ot_dyn_batch* bt, int i, int* row_bx, int* dense_xy);

int ot_dyn_batch_destroy(ot_dyn_batch* bt);

/* Last error message recorded on the batch (never NULL). */
const char* ot_dyn_batch_last_error(const ot_dyn_batch* bt);

/* ---- solve without device allocation -----------------------------------
 * For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): Algorithm 1 from its cold start to the
 * certificate, as ot_dyn_create + ot_dyn_set_boundary + ot_dyn_init
 * (OT_INIT_COLD) + ot_dyn_solve + ot_dyn_destroy, with the plan's workspace
 * in a device array of OT_DYN_STATIC_BYTES owned by the library (one per
 * GPU, held until the process ends) instead of the caller's.  The caller
 * passes inputs and outputs only: f0, f1 [batch][C][Y][X] and F, Mx, My, Mc
 * (layouts above), device pointers on the current device; `stream` as in
 * ot_dyn_create.  Results are those of the calls it stands for.  Calls no
 * hipMalloc, hipFree or other allocating routine.  Synchronous.
 * Returns OT_ERR_SHAPE when ot_dyn_workspace_size(d) exceeds
 * OT_DYN_STATIC_BYTES (e.g. 64 x 64 x 3 x 16 needs 12.2 MiB, 128 x 128 x 3
 * x 16 49 MiB: use ot_dyn_create with a workspace), OT_ERR_PARAM for null
 * pointers or max_iters < 1, else the status of ot_dyn_solve.  Every call
 * on one GPU uses the same array: calls that overlap on one GPU (several
 * host threads or streams) race and must be serialised by the caller. */
#define OT_DYN_STATIC_BYTES (32u << 20)
int ot_dyn_solve_static(const ot_dyn_desc* d, void* stream, const float* f0, const float* f1,
                        float* F, float* Mx, float* My, float* Mc, int max_iters,
                        ot_dyn_report* rep);

/* Static description of a status code. */
/* Pointwise prox of J / sigma (Sec. 3, Step 2) on n nodes, as the update
 * kernels compute it: (u, v) = argmin |u|^2 / (2 v) + sigma/2 |u - a_m|^2 +
 * sigma/2 (v - a_f)^2, (0, 0) where 2 a_f + sigma |a_m|^2 <= 0.  am and u are
 * device arrays [3][n] (the three momentum components, each contiguous), af
 * and v device arrays [n]; the caller owns them all.  kind: OT_PROX_NEWTON,
 * OT_PROX_CLOSED, or OT_PROX_CLOSED_RAW (the closed form without its Newton
 * step, for accuracy comparisons).  Asynchronous on `stream` (a hipStream_t,
 * NULL = default stream).  OT_ERR_PARAM for a null pointer, n < 0, sigma
 * <= 0 or an unknown kind; OT_ERR_HIP if the launch fails. */
int ot_dyn_prox_eval(int kind, long long n, const float* am, const float* af, float sigma,
                     float* u, float* v, void* stream);

const char* ot_dyn_status_str(int status);

/* Last error message recorded on the plan (never NULL). */
const char* ot_dyn_last_error(const ot_dyn_plan* p);

#ifdef __cplusplus
}
#endif

#endif /* OT_DYN_H */
