// Host side of the C ABI: plan creation over a caller-owned workspace, the
// launch sequence of one PDHG iteration (Algorithm 1 of the paper, Sec. 3),
// FP64 residual reductions and the certified solve loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/ot_dyn.h"
#include "otd_common.h"

using namespace otd;

struct ot_dyn_plan {
    ot_dyn_desc d;
    Geom g;
    hipStream_t stream;
    char* ws;
    size_t ws_bytes;
    // workspace carve
    float* b[4];
    float* bb[4];
    float* A[4];
    float* R;
    float* R2;
    float* Phi;              // carried potential (OT_REFINE_CARRY), else null
    float* Rt;               // fused Poisson passes: transposed scratch [B][C][X][Y][P]
    bool fused;              // the fused three-pass Poisson solve applies
    bool freezable;          // a batch group's plan: its problems can be frozen
    bool p1d;                // one spatial axis: the one-block Poisson solve applies
    bool xfold;              // the divergence kernels also do the forward x transform
    float* sig;              // sigma per problem [B] (device)
    float* fac;              // dual rescale factors per problem [B] (device)
    float* frz;              // frozen flags per problem [B] (device; batches)
    float* f0;
    float* f1;
    AxisTab tab[4];          // x, y, c, t
    double* tc64;
    double* tt64;
    double* part_slice;
    double* part_red;
    double* part_div;
    double* part_mass;
    double* part_bnd;
    double* red_out;
    int nbx;                 // plane-partial stride of the divergence kernels
    int nbx_node;            // blocks per plane of the per-node kernels
    long long nred;          // residual partials per problem of the update kernel
    int nblk_bnd;
    // launch shapes (autotuned): row-stencil block width, dense x/y transforms
    int row_bx;
    int dense_xy;
    const float2* tw_fast[2];    // fast-path twiddles of x and y (null if absent)
    const float2* tw_mix[2];     // mixed-radix twiddles of x and y (null if absent)
    // host state
    bool have_boundary;
    bool have_init;
    int total_iters;
    int it_next;             // index of the next iteration to be issued
    bool fallback_armed;     // OT_INIT_FALLBACK: the next solve may restart cold
    int checks;              // residual checks since the last ot_dyn_init
    int last_solve_iters;    // iterations of the last certified-solve loop
    std::vector<double> mass0, mass1, fbm2;
    std::vector<double> vfloor;     // per problem: 1e-3 * mean of f0 (warm-start dual)
    std::vector<double> r_prim, r_dual, r_div, cost, e_mass;
    std::vector<float> sig_h, fac_h;     // sigma per problem and rescale factors
    std::vector<float> frz_h;            // frozen flags (host copy of frz)
    std::vector<int> n_adapt, last_adapt;   // per problem: changes, iteration of the last
    double last_res;         // max(r_prim, r_dual) of the last check
    std::string err;
    // phase timing
    int prof_mask;
    std::vector<hipEvent_t> ev_pool;
    std::vector<int> ev_phase;   // phase of each recorded (start, stop) pair
    size_t ev_used;              // events in use (2 per launch)
    double prof_ms[OT_PHASE_COUNT];
    long long prof_n[OT_PHASE_COUNT];
};

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t off_b, off_bb, off_A, off_R, off_R2, off_Phi, off_Rt, off_sig, off_f,
        off_tab[4], off_tw[4], off_tc64, off_tt64;
    size_t off_pslice, off_pred, off_pdiv, off_pmass, off_pbnd, off_red;
    size_t total;
    int nbx, nbx_node, nblk_bnd;
    long long nred;
};

int axis_size(const ot_dyn_desc& d, int a) { return a == 0 ? d.X : (a == 1 ? d.Y : d.C); }

Geom make_geom(const ot_dyn_desc& d) {
    Geom g;
    g.B = d.batch; g.X = d.X; g.Y = d.Y; g.C = d.C; g.P = d.P;
    g.perx = d.X > 1 && d.bc[0] == OT_BC_PERIODIC;
    g.pery = d.Y > 1 && d.bc[1] == OT_BC_PERIODIC;
    g.perc = d.C > 1 && d.bc[2] == OT_BC_PERIODIC;
    g.sx = (float)(d.X / d.extent[0]);
    g.sy = (float)(d.Y / d.extent[1]);
    g.sc = (float)(d.C / d.extent[2]);
    g.st = (float)d.P;
    g.plane = (long long)d.X * d.Y;
    g.slice = g.plane * d.C;
    g.nc = g.slice * d.P;
    g.nf = g.slice * (d.P + 1);
    return g;
}

int validate(const ot_dyn_desc* d, std::string* why) {
    if (!d) { if (why) *why = "null descriptor"; return OT_ERR_PARAM; }
    if (d->X < 1 || d->Y < 1 || d->C < 1 || d->P < 2 || d->batch < 1) {
        if (why) *why = "sizes must satisfy X, Y, C >= 1, P >= 2, batch >= 1";
        return OT_ERR_SHAPE;
    }
    if (d->X > 8192 || d->Y > 8192 || d->C > 64 || d->P > 1024 ||
        (long long)d->P * d->C > 8192) {
        if (why) *why = "sizes beyond the supported range (X, Y <= 8192, C <= 64, P <= 1024, P*C <= 8192)";
        return OT_ERR_SHAPE;
    }
    const long long slices = (long long)d->batch * d->P * d->C;
    if (slices > 65535) {
        if (why) *why = "batch * P * C must not exceed 65535";
        return OT_ERR_SHAPE;
    }
    for (int a = 0; a < 3; ++a) {
        if (d->bc[a] != OT_BC_NEUMANN && d->bc[a] != OT_BC_PERIODIC) {
            if (why) *why = "bc must be OT_BC_NEUMANN or OT_BC_PERIODIC";
            return OT_ERR_PARAM;
        }
        if (!(d->extent[a] > 0.0) || !std::isfinite(d->extent[a])) {
            if (why) *why = "extent must be positive and finite";
            return OT_ERR_PARAM;
        }
    }
    if (!(d->tau > 0.0) || !(d->sigma > 0.0) || !(d->tau * d->sigma < 1.0) ||
        !std::isfinite(d->tau) || !std::isfinite(d->sigma)) {
        if (why) *why = "need tau > 0, sigma > 0 and tau * sigma < 1";
        return OT_ERR_PARAM;
    }
    if (!(d->theta >= 0.0 && d->theta <= 1.0)) {
        if (why) *why = "theta must lie in [0, 1]";
        return OT_ERR_PARAM;
    }
    if (d->check_every < 1 || !(d->tol_res > 0.0) || !(d->tol_div > 0.0) ||
        !(d->tol_mass >= 0.0) || d->refine < OT_REFINE_OFF || d->refine > OT_REFINE_CARRY ||
        d->adapt < 0 || d->adapt > 1 || d->prox < OT_PROX_NEWTON || d->prox > OT_PROX_CLOSED ||
        d->carry_refine < 0) {
        if (why) *why = "need check_every >= 1, tol_res > 0, tol_div > 0, tol_mass >= 0, refine in {0,1,2,3}, adapt in {0,1}, prox in {0,1}, carry_refine >= 0";
        return OT_ERR_PARAM;
    }
    return OT_OK;
}

Layout layout_of(const ot_dyn_desc& d) {
    const Geom g = make_geom(d);
    Layout L;
    const long long ncT = (long long)g.B * g.nc;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
    L.off_b = take(4 * ncT * sizeof(float));
    L.off_bb = take(4 * ncT * sizeof(float));
    L.off_A = take(4 * ncT * sizeof(float));
    L.off_R = take(ncT * sizeof(float));
    L.off_R2 = take(ncT * sizeof(float));
    L.off_Phi = take(d.refine == OT_REFINE_CARRY ? ncT * sizeof(float) : 0);
    L.off_sig = take(3 * (size_t)g.B * sizeof(float));   // sigma, rescale, frozen
    L.off_Rt = take(ncT * sizeof(float));
    L.off_f = take(2 * (size_t)g.B * g.slice * sizeof(float));
    const int ns[4] = {d.X, d.Y, d.C, d.P};
    for (int a = 0; a < 4; ++a) {
        L.off_tab[a] = take((2 * (size_t)ns[a] * ns[a] + ns[a]) * sizeof(float));
        L.off_tw[a] = take((4 * (size_t)ns[a] + ns[a] / 2) * 2 * sizeof(float));
    }
    L.off_tc64 = take(((size_t)d.C * d.C + d.C) * sizeof(double));
    L.off_tt64 = take(((size_t)d.P * d.P + d.P) * sizeof(double));
    // FP64 partials: per-node kernels write one per 256 nodes of a plane; the
    // row kernels one per row segment and colour (plane stride Y * nxb)
    L.nbx_node = (int)((g.plane + 255) / 256);
    if (rows_ok(g)) {
        // sized for the narrowest row block (64), the most partials
        const int nxb = (g.X + 63) / 64;
        L.nbx = g.Y * nxb;
        L.nred = (long long)g.Y * g.P * nxb;
    } else {
        L.nbx = L.nbx_node;
        L.nred = (long long)g.P * g.C * L.nbx_node;
    }
    const size_t nnode = (size_t)g.B * g.P * g.C * L.nbx_node;
    L.off_pslice = take((size_t)g.B * g.P * g.C * L.nbx * sizeof(double));
    // the residual partials also hold one per block of the per-node state
    // residual kernel (ot_dyn_residuals)
    const long long nred_cap = std::max<long long>(L.nred, (long long)g.P * g.C * L.nbx_node);
    L.off_pred = take(RS_COUNT * (size_t)g.B * nred_cap * sizeof(double));
    L.off_pdiv = take(nnode * sizeof(double));
    L.off_pmass = take(nnode * sizeof(double));
    L.nblk_bnd = (int)std::min<long long>(64, (g.slice + 255) / 256);
    L.off_pbnd = take(5 * (size_t)g.B * L.nblk_bnd * sizeof(double));
    L.off_red = take(((size_t)RS_COUNT * g.B + g.B + (size_t)g.B * g.P + 5 * g.B) * sizeof(double));
    L.total = o;
    return L;
}

// Orthonormal DCT-II (Neumann axis, Sec. 3: C_p) or discrete Hartley
// (periodic axis) matrix M[j][k], built in FP64.
void axis_matrix(int n, int periodic, std::vector<double>& M) {
    M.assign((size_t)n * n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) {
            double v;
            if (periodic) {
                const long long jk = ((long long)j * k) % n;
                const double ang = 2.0 * pi * (double)jk / n;
                v = (std::cos(ang) + std::sin(ang)) / std::sqrt((double)n);
            } else {
                const long long q = ((long long)j * (2 * k + 1)) % (4LL * n);
                v = std::sqrt(2.0 / n) * std::cos(pi * (double)q / (2.0 * n));
                if (j == 0) v /= std::sqrt(2.0);
            }
            M[(size_t)j * n + k] = v;
        }
}

// Eigenvalues of s^2 Delta along one axis: 4 s^2 sin^2(pi j / n) periodic,
// 4 s^2 sin^2(pi j / (2 n)) Neumann (Sec. 3).
void axis_eigs(int n, int periodic, double s, std::vector<double>& lam) {
    lam.assign(n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int j = 0; j < n; ++j) {
        const double sn = std::sin(pi * j / (periodic ? n : 2.0 * n));
        lam[j] = 4.0 * s * s * sn * sn;
    }
}

int hip_fail(ot_dyn_plan* p, hipError_t e, const char* what) {
    if (p) p->err = std::string(what) + ": " + hipGetErrorString(e);
    return OT_ERR_HIP;
}

#define HIPCHK(p, call)                                  \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(p, e_, #call); \
    } while (0)

StepArgs step_args(ot_dyn_plan* p, float* F, float* Mx, float* My, float* Mc) {
    StepArgs s;
    s.g = p->g;
    s.tau_sigma = (float)(p->d.tau * p->d.sigma);
    s.prox = p->d.prox;
    s.sig = p->sig;
    s.frz = p->frz;
    s.frz_run = p->freezable ? p->frz : nullptr;
    s.theta = (float)p->d.theta;
    s.F = F; s.Mx = Mx; s.My = My; s.Mc = Mc;
    for (int q = 0; q < 4; ++q) { s.b[q] = p->b[q]; s.bb[q] = p->bb[q]; s.A[q] = p->A[q]; }
    s.R = p->R;
    s.R2 = p->R2;
    s.Phi = p->Phi;
    s.part_slice = p->part_slice;
    s.part_red = p->part_red;
    s.part_mass = p->part_mass;
    s.part_div = p->part_div;
    s.nbx = p->nbx;
    s.row_bx = p->row_bx;
    s.twx = p->xfold ? p->tab[0].tw : nullptr;
    s.xkind = p->tab[0].periodic ? 2 : 0;
    s.cmix = p->fused && p->g.C > 1 ? p->tab[2].mat : nullptr;
    s.nt_store = (long long)p->g.B * p->g.nc * (long long)sizeof(float) >= (16ll << 20) ? 1 : 0;
    return s;
}

hipEvent_t next_event(ot_dyn_plan* p) {
    if (p->ev_used == p->ev_pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        p->ev_pool.push_back(e);
    }
    return p->ev_pool[p->ev_used++];
}

// Launch `fn`, bracketed by events when `phase` is being timed.
template <class Fn>
void timed(ot_dyn_plan* p, int phase, Fn&& fn) {
    if (!((p->prof_mask >> phase) & 1)) { fn(); return; }
    hipEvent_t a = next_event(p), b = next_event(p);
    if (!a || !b) { fn(); return; }
    hipEventRecord(a, p->stream);
    fn();
    hipEventRecord(b, p->stream);
    p->ev_phase.push_back(phase);
}

// phi = (A A^T)^+ r in place on R.
void poisson(ot_dyn_plan* p, float* R) {
    const Geom& g = p->g;
    hipStream_t st = p->stream;
    const long long B = g.B;
    if (p->p1d) {
        timed(p, OT_PHASE_TC, [&] {
            launch_poisson_1d(g, R, p->tab[0], p->tab[1], p->tab[2], p->tab[3], p->tc64, p->tt64,
                              p->freezable ? p->frz : nullptr, st);
        });
        return;
    }
    if (p->fused) {     // three passes: x (+ colour), y + t, inverse x (+ colour)
        auto x_pass = [&](int inverse) {
            // the divergence kernels wrote r in colour modes (StepArgs::cmix)
            launch_fused_x(g, R, p->Rt, p->tab[0], p->tab[1], p->tab[2], p->tab[3],
                           p->tc64, p->tt64, p->part_slice, p->nbx, inverse, g.C > 1, st);
        };
        timed(p, OT_PHASE_XFORM_X, [&] { x_pass(0); });
        timed(p, OT_PHASE_TC, [&] {
            launch_fused_yt(g, p->Rt, p->tab[0], p->tab[1], p->tab[2], p->tab[3], st);
        });
        timed(p, OT_PHASE_XFORM_X, [&] { x_pass(1); });
        return;
    }
    // the first forward pass also reduces the FP64 plane sums of r that the
    // colour/time pass needs for the spatial-DC line (fast lengths only);
    // when the divergence kernel has done the forward x transform (xfold),
    // the first pass is the one along y
    bool presummed = false;
    const PlaneSums ps{p->part_slice, B * g.P * g.C, p->nbx};
    // rows of frozen problems are skipped (rows per problem: P C Y)
    const RowSkip skip{p->freezable ? p->frz : nullptr, (long long)g.P * g.C * g.Y};
    if (g.X > 1 && !p->xfold)
        timed(p, OT_PHASE_XFORM_X, [&] {
            presummed = launch_rows(R, B * g.P * g.C * g.Y, p->tab[0], 0, st, &ps, skip);
        });
    if (g.Y > 1)
        timed(p, OT_PHASE_XFORM_Y, [&] {
            const bool s1 = launch_cols(R, B * g.P * g.C, g.X, p->tab[1], 0, st,
                                        presummed ? nullptr : &ps);
            presummed = presummed || s1;
        });
    timed(p, OT_PHASE_TC, [&] {
        launch_tc(g, R, p->tab[0], p->tab[1], p->tab[2], p->tab[3], p->tc64, p->tt64,
                  p->part_slice, p->nbx, presummed ? 1 : 0, p->freezable ? p->frz : nullptr, st);
    });
    if (g.Y > 1)
        timed(p, OT_PHASE_XFORM_Y, [&] { launch_cols(R, B * g.P * g.C, g.X, p->tab[1], 1, st); });
    if (g.X > 1)
        timed(p, OT_PHASE_XFORM_X, [&] {
            launch_rows(R, B * g.P * g.C * g.Y, p->tab[0], 1, st, nullptr, skip);
        });
}

// Launch shapes: the row-stencil block width (64, 128 or 256; 0 = default)
// and the transform path: dense_xy 0 = fused three-pass solve where it
// applies (else five FFT passes), 1 = dense x/y passes, 2 = five FFT passes.
void apply_tuning(ot_dyn_plan* p, int row_bx, int dense_xy) {
    const Geom& g = p->g;
    if (row_bx <= 0) row_bx = row_block(g.X);
    p->row_bx = row_bx;
    p->dense_xy = dense_xy;
    if (rows_ok(g)) {
        const int nxb = (g.X + row_bx - 1) / row_bx;
        p->nbx = g.Y * nxb;
        p->nred = (long long)g.Y * g.P * nxb;
    }
    for (int a = 0; a < 2; ++a) {
        p->tab[a].tw = dense_xy == 1 ? nullptr : p->tw_fast[a];
        p->tab[a].twm = dense_xy == 1 ? nullptr : p->tw_mix[a];
    }
    // the fused passes use one block per row index and problem: measured
    // faster than the five passes at 64 x 64 and 128 x 128 (alone and
    // batched) and, since the FP64 DC line's loads are all in flight, for one
    // 256 x 256 problem as well (1.3% per iteration against the five passes
    // with the forward x transform folded into the divergence kernel)
    // problems with one spatial axis: the whole solve in one block per problem
    p->p1d = dense_xy != 1 && poisson_1d_ok(g, p->tab[0], p->tab[3]);
    p->fused = dense_xy == 0 && fused_poisson_ok(g, p->tab[0], p->tab[1], p->tab[3]);
    // the five-pass solve with rows of one block each: the divergence
    // kernels write r already transformed along x (one pass fewer)
    p->xfold = !p->p1d && !p->fused && g.X > 1 && div_fold_ok(g, row_bx, p->tab[0]);
}

bool refine_now(const ot_dyn_plan* p) {
    if (p->d.refine == OT_REFINE_ALWAYS) return true;
    if (p->d.refine == OT_REFINE_ADAPTIVE) return p->last_res < 1e-4;
    return false;
}

// One iteration of Algorithm 1; residual partials when `check`.
void iterate(ot_dyn_plan* p, const StepArgs& s, bool check) {
    hipStream_t st = p->stream;
    const int it = p->it_next++;
    if (p->d.refine == OT_REFINE_CARRY) {
        // The projection is affine with Pi(a) = Pi(a + grad Phi) for any Phi
        // (A^T annihilates constants and (A A^T)^+ A A^T Phi = Phi up to a
        // constant), so start from the previous iterations' potential: a' =
        // a + grad Phi, r' = A a' - f_b^-, phi_1 = (A A^T)^+ r', x = a' +
        // grad phi_1, Phi += phi_1.  r' vanishes as the iterates converge,
        // and with it the FP32 error of the transform solve.
        timed(p, OT_PHASE_DIV, [&] { launch_div(s, 2, st); });
        poisson(p, p->R);
        // early on the iterates move fast and the carried potential predicts
        // little: the residual it leaves is as large as the plain one
        const bool refine = it < p->d.carry_refine;
        if (refine) {   // r'' = A (a' + grad phi_1) - f_b^-, phi_2 = (A A^T)^+ r''
            timed(p, OT_PHASE_REFINE, [&] { launch_div(s, 1, st); });
            poisson(p, p->R2);
        }
        timed(p, OT_PHASE_UPDATE, [&] { launch_update(s, check ? 1 : 0, refine ? 4 : 3, st); });
        return;
    }
    // a = x - tau sigma K^T b_bar, r = A a - f_b^-
    timed(p, OT_PHASE_DIV, [&] { launch_div(s, 0, st); });
    poisson(p, p->R);                      // phi_1 = (A A^T)^+ r
    const bool refine = refine_now(p);
    if (refine) {                          // FP32 refinement of the projection:
        // r' = A (a + grad phi_1) - f_b^-, phi_2 = (A A^T)^+ r'
        timed(p, OT_PHASE_REFINE, [&] { launch_div(s, 1, st); });
        poisson(p, p->R2);
    }
    // x = a + grad phi_1 (+ grad phi_2); prox; duals
    timed(p, OT_PHASE_UPDATE, [&] { launch_update(s, check ? 1 : 0, refine ? 2 : 1, st); });
}

// Reduce the residual partials of the last check iteration and of the
// divergence/mass kernel, then fill the per-problem host arrays.
int collect(ot_dyn_plan* p, const StepArgs& s, bool have_iter) {
    const Geom& g = p->g;
    hipStream_t st = p->stream;
    const int B = g.B;
    const long long nslot = (long long)g.P * g.C * p->nbx_node;  // per problem
    launch_resid_div(s, st);
    double* out_red = p->red_out;
    double* out_div = out_red + RS_COUNT * B;
    double* out_mass = out_div + B;
    if (have_iter) launch_reduce(p->part_red, p->nred, RS_COUNT * B, out_red, st);
    launch_reduce(p->part_div, nslot, B, out_div, st);
    launch_reduce(p->part_mass, (long long)g.C * p->nbx_node, B * g.P, out_mass, st);
    std::vector<double> h((size_t)RS_COUNT * B + B + (size_t)B * g.P);
    HIPCHK(p, hipMemcpyAsync(h.data(), out_red, h.size() * sizeof(double),
                             hipMemcpyDeviceToHost, st));
    HIPCHK(p, hipStreamSynchronize(st));
    HIPCHK(p, hipGetLastError());
    const double vol = [&] {
        double v = 1.0 / g.P;
        for (int a = 0; a < 3; ++a) v *= p->d.extent[a] / axis_size(p->d, a);
        return v;
    }();
    bool finite = true;
    for (int b = 0; b < B; ++b) {
        if (have_iter) {
            const double db2 = h[RS_DB2 * B + b], z2 = h[RS_Z2 * B + b];
            const double dx2 = h[RS_DX2 * B + b], x2 = h[RS_X2 * B + b];
            p->r_prim[b] = std::sqrt(db2) / std::max(std::sqrt(z2), 1e-300);
            p->r_dual[b] = std::sqrt(dx2) / std::max(std::sqrt(x2), 1e-300);
            p->cost[b] = vol * h[RS_J * B + b];
        }
        p->r_div[b] = std::sqrt(h[RS_COUNT * B + b]) / std::max(std::sqrt(p->fbm2[b]), 1e-300);
        double em = 0.0;
        for (int k = 1; k < g.P; ++k) {
            const double mk = h[(size_t)RS_COUNT * B + B + (size_t)b * g.P + k];
            em = std::max(em, std::fabs(mk - p->mass0[b]) / p->mass0[b]);
            if (!std::isfinite(mk)) finite = false;
        }
        p->e_mass[b] = em;
        if (!std::isfinite(p->r_prim[b]) || !std::isfinite(p->r_dual[b]) ||
            !std::isfinite(p->r_div[b]) || !std::isfinite(p->cost[b]))
            finite = false;
    }
    if (have_iter) p->checks += 1;
    if (!finite) {
        p->err = "non-finite residual";
        return OT_ERR_NONFINITE;
    }
    return OT_OK;
}

// Residuals of the current state without iterating (ot_dyn_residuals):
// r_div and the slice masses as in collect(), r_prim and the cost from z =
// prox(K x + c + b).  Nothing of the state is written.
int collect_state(ot_dyn_plan* p, const StepArgs& s) {
    const Geom& g = p->g;
    hipStream_t st = p->stream;
    const int B = g.B;
    const long long nslot = (long long)g.P * g.C * p->nbx_node;  // per problem
    launch_resid_div(s, st);
    launch_resid_state(s, st);
    double* out_red = p->red_out;
    double* out_div = out_red + RS_COUNT * B;
    double* out_mass = out_div + B;
    launch_reduce(p->part_red, nslot, RS_COUNT * B, out_red, st);
    launch_reduce(p->part_div, nslot, B, out_div, st);
    launch_reduce(p->part_mass, (long long)g.C * p->nbx_node, B * g.P, out_mass, st);
    std::vector<double> h((size_t)RS_COUNT * B + B + (size_t)B * g.P);
    HIPCHK(p, hipMemcpyAsync(h.data(), out_red, h.size() * sizeof(double),
                             hipMemcpyDeviceToHost, st));
    HIPCHK(p, hipStreamSynchronize(st));
    HIPCHK(p, hipGetLastError());
    double vol = 1.0 / g.P;
    for (int a = 0; a < 3; ++a) vol *= p->d.extent[a] / axis_size(p->d, a);
    bool finite = true;
    for (int b = 0; b < B; ++b) {
        const double db2 = h[RS_DB2 * B + b], z2 = h[RS_Z2 * B + b];
        p->r_prim[b] = std::sqrt(db2) / std::max(std::sqrt(z2), 1e-300);
        p->cost[b] = vol * h[RS_J * B + b];
        if (p->checks == 0) p->r_dual[b] = -1.0;
        p->r_div[b] = std::sqrt(h[RS_COUNT * B + b]) / std::max(std::sqrt(p->fbm2[b]), 1e-300);
        double em = 0.0;
        for (int k = 1; k < g.P; ++k) {
            const double mk = h[(size_t)RS_COUNT * B + B + (size_t)b * g.P + k];
            em = std::max(em, std::fabs(mk - p->mass0[b]) / p->mass0[b]);
            if (!std::isfinite(mk)) finite = false;
        }
        p->e_mass[b] = em;
        if (!std::isfinite(p->r_prim[b]) || !std::isfinite(p->r_div[b]) ||
            !std::isfinite(p->cost[b]))
            finite = false;
    }
    if (!finite) {
        p->err = "non-finite residual";
        return OT_ERR_NONFINITE;
    }
    return OT_OK;
}

// Residual balancing of the step sizes (desc.adapt), per problem, after a
// residual check: tau sigma stays fixed and sigma halves when the primal
// iterate lags (r_dual > 4 r_prim: a larger primal step tau) or doubles when
// the constraint residual lags (r_prim > 4 r_dual).  The unscaled dual
// sigma b is kept, so b and b_bar are rescaled.  A problem changes at most
// every kAdaptGap iterations and kAdaptMax times, within 64x of the given
// sigma, and no more once max(r_prim, r_dual) < kAdaptStop: near the fixed
// point a change of steps perturbs the iteration, and problems whose steps
// kept changing there stalled just above the tolerance (measured on the
// 1024 hue problems: 4 changes at most and no change below 3e-5 certify 1023
// of them in 4.6 s, 16 changes without that bound 1019 in 5.4 s).  Certified
// problems keep their sigma.
constexpr int kAdaptGap = 200;
constexpr int kAdaptMax = 4;
constexpr double kAdaptStop = 3e-5;

int adapt_steps(ot_dyn_plan* p, const StepArgs& s) {
    if (!p->d.adapt) return OT_OK;
    const float s0 = (float)p->d.sigma;
    bool any = false;
    for (int b = 0; b < p->g.B; ++b) {
        p->fac_h[b] = 1.f;
        const bool done = std::max(p->r_prim[b], p->r_dual[b]) < p->d.tol_res &&
                          p->r_div[b] < p->d.tol_div;
        if (done || p->n_adapt[b] >= kAdaptMax || p->total_iters - p->last_adapt[b] < kAdaptGap ||
            std::max(p->r_prim[b], p->r_dual[b]) < kAdaptStop)
            continue;
        float f = 1.f;
        if (p->r_dual[b] > 4.0 * p->r_prim[b] && p->sig_h[b] > s0 / 64.f) f = 2.f;
        else if (p->r_prim[b] > 4.0 * p->r_dual[b] && p->sig_h[b] < s0 * 64.f) f = 0.5f;
        if (f == 1.f) continue;
        p->sig_h[b] /= f;
        p->fac_h[b] = f;
        p->n_adapt[b] += 1;
        p->last_adapt[b] = p->total_iters;
        any = true;
    }
    if (!any) return OT_OK;
    const size_t B = (size_t)p->g.B;
    HIPCHK(p, hipMemcpyAsync(p->sig, p->sig_h.data(), B * sizeof(float), hipMemcpyHostToDevice,
                             p->stream));
    HIPCHK(p, hipMemcpyAsync(p->fac, p->fac_h.data(), B * sizeof(float), hipMemcpyHostToDevice,
                             p->stream));
    launch_scale_dual(s, p->fac, p->stream);
    HIPCHK(p, hipGetLastError());
    return OT_OK;
}

void fill_report(const ot_dyn_plan* p, ot_dyn_report* rep) {
    if (!rep) return;
    const int B = p->g.B;
    int worst = 0;
    double wv = -HUGE_VAL;
    rep->r_prim = rep->r_dual = rep->r_div = rep->e_mass = -HUGE_VAL;
    for (int b = 0; b < B; ++b) {
        rep->r_prim = std::max(rep->r_prim, p->r_prim[b]);
        rep->r_dual = std::max(rep->r_dual, p->r_dual[b]);
        rep->r_div = std::max(rep->r_div, p->r_div[b]);
        rep->e_mass = std::max(rep->e_mass, p->e_mass[b]);
        const double v = std::max(p->r_prim[b], p->r_dual[b]);
        if (v > wv) { wv = v; worst = b; }
    }
    rep->worst_problem = worst;
    rep->cost = p->cost[0];
    rep->mass0 = p->mass0[0];
    rep->mass1 = p->mass1[0];
    rep->total_iterations = p->total_iters;
}

int solve_loop(ot_dyn_plan* p, const StepArgs& s, int max_iters);

}  // namespace

extern "C" {

int ot_dyn_default_desc(ot_dyn_desc* d, int X, int Y, int C, int P) {
    if (!d) return OT_ERR_PARAM;
    std::memset(d, 0, sizeof(*d));
    d->X = X; d->Y = Y; d->C = C; d->P = P;
    d->bc[0] = OT_BC_NEUMANN; d->bc[1] = OT_BC_NEUMANN; d->bc[2] = OT_BC_PERIODIC;
    d->extent[0] = d->extent[1] = d->extent[2] = 1.0;
    d->tau = 10.0; d->sigma = 0.099; d->theta = 1.0;
    d->check_every = 50;
    d->tol_res = 1e-6; d->tol_div = 1e-6; d->tol_mass = 1e-5;
    d->refine = OT_REFINE_CARRY;
    d->batch = 1;
    d->adapt = 0;
    d->prox = OT_PROX_NEWTON;
    d->carry_refine = 64;
    return OT_OK;
}

int ot_dyn_workspace_size(const ot_dyn_desc* d, size_t* bytes) {
    const int st = validate(d, nullptr);
    if (st != OT_OK) return st;
    if (!bytes) return OT_ERR_PARAM;
    *bytes = layout_of(*d).total;
    return OT_OK;
}

int ot_dyn_create(const ot_dyn_desc* d, void* stream, void* workspace, size_t ws_bytes,
                  ot_dyn_plan** out) {
    if (!out) return OT_ERR_PARAM;
    *out = nullptr;
    const int st = validate(d, nullptr);
    if (st != OT_OK) return st;
    const Layout L = layout_of(*d);
    if (!workspace || ws_bytes < L.total || ((uintptr_t)workspace % kAlign) != 0)
        return OT_ERR_SHAPE;
    ot_dyn_plan* p = new (std::nothrow) ot_dyn_plan();
    if (!p) return OT_ERR_PARAM;
    p->d = *d;
    p->g = make_geom(*d);
    p->stream = (hipStream_t)stream;
    p->ws = (char*)workspace;
    p->ws_bytes = ws_bytes;
    const long long ncT = (long long)p->g.B * p->g.nc;
    for (int q = 0; q < 4; ++q) {
        p->b[q] = (float*)(p->ws + L.off_b) + q * ncT;
        p->bb[q] = (float*)(p->ws + L.off_bb) + q * ncT;
        p->A[q] = (float*)(p->ws + L.off_A) + q * ncT;
    }
    p->R = (float*)(p->ws + L.off_R);
    p->R2 = (float*)(p->ws + L.off_R2);
    p->Phi = d->refine == OT_REFINE_CARRY ? (float*)(p->ws + L.off_Phi) : nullptr;
    p->sig = (float*)(p->ws + L.off_sig);
    p->Rt = (float*)(p->ws + L.off_Rt);
    p->fused = false;
    p->p1d = false;
    p->xfold = false;
    p->freezable = false;
    p->fac = p->sig + p->g.B;
    p->frz = p->sig + 2 * (size_t)p->g.B;
    p->f0 = (float*)(p->ws + L.off_f);
    p->f1 = p->f0 + (long long)p->g.B * p->g.slice;
    p->tc64 = (double*)(p->ws + L.off_tc64);
    p->tt64 = (double*)(p->ws + L.off_tt64);
    p->part_slice = (double*)(p->ws + L.off_pslice);
    p->part_red = (double*)(p->ws + L.off_pred);
    p->part_div = (double*)(p->ws + L.off_pdiv);
    p->part_mass = (double*)(p->ws + L.off_pmass);
    p->part_bnd = (double*)(p->ws + L.off_pbnd);
    p->red_out = (double*)(p->ws + L.off_red);
    p->nbx = L.nbx;
    p->nbx_node = L.nbx_node;
    p->nred = L.nred;
    p->nblk_bnd = L.nblk_bnd;
    const int B = p->g.B;
    p->mass0.assign(B, 0); p->mass1.assign(B, 0); p->fbm2.assign(B, 0);
    p->vfloor.assign(B, 0);
    p->r_prim.assign(B, 0); p->r_dual.assign(B, 0); p->r_div.assign(B, 0);
    p->cost.assign(B, 0); p->e_mass.assign(B, 0);
    p->sig_h.assign(B, (float)d->sigma); p->fac_h.assign(B, 1.f);
    p->frz_h.assign(B, 0.f);
    p->n_adapt.assign(B, 0); p->last_adapt.assign(B, 0);
    p->last_res = 1.0;
    p->total_iters = 0;
    p->it_next = 0;
    p->fallback_armed = false;
    p->checks = 0;
    p->last_solve_iters = 0;
    p->have_boundary = p->have_init = false;
    p->prof_mask = 0;
    p->ev_used = 0;
    for (int q = 0; q < OT_PHASE_COUNT; ++q) { p->prof_ms[q] = 0.0; p->prof_n[q] = 0; }

    // transform tables, built in FP64 and uploaded once
    const int ns[4] = {d->X, d->Y, d->C, d->P};
    const int per[4] = {p->g.perx, p->g.pery, p->g.perc, 0};
    const double sc[4] = {d->X / d->extent[0], d->Y / d->extent[1], d->C / d->extent[2],
                          (double)d->P};
    std::vector<double> M, lam;
    for (int a = 0; a < 4; ++a) {
        const int n = ns[a];
        axis_matrix(n, per[a], M);
        axis_eigs(n, per[a], sc[a], lam);
        std::vector<float> h(2 * (size_t)n * n + n);
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                h[(size_t)k * n + j] = (float)M[(size_t)j * n + k];              // M^T
                h[(size_t)n * n + (size_t)k * n + j] = (float)M[(size_t)k * n + j];  // M
            }
        for (int j = 0; j < n; ++j) h[2 * (size_t)n * n + j] = (float)lam[j];
        float* dst = (float*)(p->ws + L.off_tab[a]);
        hipError_t e = hipMemcpyAsync(dst, h.data(), h.size() * sizeof(float),
                                      hipMemcpyHostToDevice, p->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) { delete p; return OT_ERR_HIP; }
        p->tab[a].n = n;
        p->tab[a].periodic = per[a];
        p->tab[a].mat = dst;
        p->tab[a].lam = dst + 2 * (size_t)n * n;
        // twiddles e^{-i pi j / (2n)}, j < 4n, for the power-of-two fast paths
        const bool fast = (a < 2 && fast_len(n)) || (a == 3 && (n == 8 || n == 16 || n == 32));
        // the same table for the mixed-radix transforms of x and y
        const bool mixed = a < 2 && !fast && mix_len(n);
        p->tab[a].tw = nullptr;
        p->tab[a].twm = nullptr;
        if (fast || mixed) {
            std::vector<float> tw(2 * (4 * (size_t)n + n / 2));
            const double pi = 3.14159265358979323846;
            for (int j = 0; j < 4 * n; ++j) {
                tw[2 * j] = (float)std::cos(pi * j / (2.0 * n));
                tw[2 * j + 1] = (float)-std::sin(pi * j / (2.0 * n));
            }
            if (fast && a < 2) {   // the first-stage twiddles of the line transforms
                const int M1 = fft_m1(n), M2 = n / (2 * M1);
                for (int t = 0; t < M2; ++t)
                    for (int k1 = 0; k1 < M1; ++k1) {
                        const int j = (8 * t * k1) % (4 * n), q = 4 * n + t * M1 + k1;
                        tw[2 * q] = tw[2 * j];
                        tw[2 * q + 1] = tw[2 * j + 1];
                    }
            }
            float* tdst = (float*)(p->ws + L.off_tw[a]);
            e = hipMemcpyAsync(tdst, tw.data(), tw.size() * sizeof(float), hipMemcpyHostToDevice,
                               p->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
            if (e != hipSuccess) { delete p; return OT_ERR_HIP; }
            if (fast) p->tab[a].tw = (const float2*)tdst;
            else p->tab[a].twm = (const float2*)tdst;
        }
        if (a < 2) { p->tw_fast[a] = p->tab[a].tw; p->tw_mix[a] = p->tab[a].twm; }
        if (a == 2 || a == 3) {
            std::vector<double> h64((size_t)n * n + n);
            std::copy(M.begin(), M.end(), h64.begin());
            std::copy(lam.begin(), lam.end(), h64.begin() + (size_t)n * n);
            double* d64 = a == 2 ? p->tc64 : p->tt64;
            e = hipMemcpyAsync(d64, h64.data(), h64.size() * sizeof(double),
                               hipMemcpyHostToDevice, p->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
            if (e != hipSuccess) { delete p; return OT_ERR_HIP; }
        }
    }
    {   // no problem starts frozen (ot_dyn_init also releases them)
        hipError_t e = hipMemcpyAsync(p->frz, p->frz_h.data(), p->frz_h.size() * sizeof(float),
                                      hipMemcpyHostToDevice, p->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) { delete p; return OT_ERR_HIP; }
    }
    apply_tuning(p, 0, 0);
    *out = p;
    return OT_OK;
}

int ot_dyn_set_boundary(ot_dyn_plan* p, const float* f0, const float* f1) {
    if (!p || !f0 || !f1) return OT_ERR_PARAM;
    const Geom& g = p->g;
    const int B = g.B;
    hipStream_t st = p->stream;
    const size_t bytes = (size_t)B * g.slice * sizeof(float);
    HIPCHK(p, hipMemcpyAsync(p->f0, f0, bytes, hipMemcpyDeviceToDevice, st));
    HIPCHK(p, hipMemcpyAsync(p->f1, f1, bytes, hipMemcpyDeviceToDevice, st));
    launch_boundary_stats(g, p->f0, p->f1, p->part_bnd, p->nblk_bnd, st);
    launch_reduce(p->part_bnd, p->nblk_bnd, 5 * B, p->red_out, st);
    std::vector<double> h(5 * (size_t)B);
    HIPCHK(p, hipMemcpyAsync(h.data(), p->red_out, h.size() * sizeof(double),
                             hipMemcpyDeviceToHost, st));
    HIPCHK(p, hipStreamSynchronize(st));
    HIPCHK(p, hipGetLastError());
    p->have_boundary = false;
    for (int b = 0; b < B; ++b) {
        const double m0 = h[b], m1 = h[B + b], bad = h[2 * B + b];
        if (bad > 0.0 || !std::isfinite(m0) || !std::isfinite(m1) || !(m0 > 0.0)) {
            char buf[160];
            std::snprintf(buf, sizeof buf, "problem %d: negative or non-finite density (%.0f entries)", b, bad);
            p->err = buf;
            return OT_ERR_INPUT;
        }
        if (std::fabs(m0 - m1) / m0 > p->d.tol_mass) {
            char buf[160];
            std::snprintf(buf, sizeof buf, "problem %d: |M0 - M1| / M0 = %.3e exceeds tol_mass", b,
                          std::fabs(m0 - m1) / m0);
            p->err = buf;
            return OT_ERR_MASS;
        }
        p->mass0[b] = m0;
        p->mass1[b] = m1;
        p->vfloor[b] = 1e-3 * m0 / (double)g.slice;
        p->fbm2[b] = (double)g.st * g.st * (h[3 * B + b] + h[4 * B + b]);
    }
    p->have_boundary = true;
    return OT_OK;
}

int ot_dyn_init(ot_dyn_plan* p, int mode, float* F, float* Mx, float* My, float* Mc) {
    if (!p || !F || !Mx || !My || !Mc) return OT_ERR_PARAM;
    if (!p->have_boundary) { p->err = "ot_dyn_set_boundary must succeed first"; return OT_ERR_STATE; }
    const bool fallback = (mode & OT_INIT_FALLBACK) != 0;
    mode &= ~OT_INIT_FALLBACK;
    if (mode < OT_INIT_COLD || mode > OT_INIT_PRIMAL_DUAL || (fallback && mode == OT_INIT_COLD)) {
        p->err = "mode must be OT_INIT_COLD, OT_INIT_PRIMAL or OT_INIT_PRIMAL_DUAL (the last two "
                 "optionally with OT_INIT_FALLBACK)";
        return OT_ERR_PARAM;
    }
    const StepArgs s = step_args(p, F, Mx, My, Mc);
    std::fill(p->sig_h.begin(), p->sig_h.end(), (float)p->d.sigma);
    std::fill(p->n_adapt.begin(), p->n_adapt.end(), 0);
    std::fill(p->last_adapt.begin(), p->last_adapt.end(), 0);
    HIPCHK(p, hipMemcpyAsync(p->sig, p->sig_h.data(), p->sig_h.size() * sizeof(float),
                             hipMemcpyHostToDevice, p->stream));
    std::fill(p->frz_h.begin(), p->frz_h.end(), 0.f);
    HIPCHK(p, hipMemcpyAsync(p->frz, p->frz_h.data(), p->frz_h.size() * sizeof(float),
                             hipMemcpyHostToDevice, p->stream));
    launch_init_state(s, p->f0, p->f1, mode == OT_INIT_COLD ? 1 : 0, p->stream);
    if (mode == OT_INIT_PRIMAL_DUAL) {
        // the boundary-statistics scratch is free after set_boundary
        HIPCHK(p, hipMemcpyAsync(p->part_bnd, p->vfloor.data(), p->vfloor.size() * sizeof(double),
                                 hipMemcpyHostToDevice, p->stream));
        launch_init_dual(s, p->part_bnd, p->stream);
    }
    else launch_zero_dual(s, p->stream);
    HIPCHK(p, hipGetLastError());
    p->have_init = true;
    p->total_iters = 0;
    p->it_next = 0;
    p->last_res = 1.0;
    p->checks = 0;
    p->fallback_armed = fallback;
    return OT_OK;
}

int ot_dyn_step(ot_dyn_plan* p, float* F, float* Mx, float* My, float* Mc, int iters) {
    if (!p || !F || !Mx || !My || !Mc || iters < 0) return OT_ERR_PARAM;
    if (!p->have_init) { p->err = "ot_dyn_init must succeed first"; return OT_ERR_STATE; }
    const StepArgs s = step_args(p, F, Mx, My, Mc);
    for (int i = 0; i < iters; ++i) iterate(p, s, false);
    p->total_iters += iters;
    HIPCHK(p, hipGetLastError());
    return OT_OK;
}

int ot_dyn_solve(ot_dyn_plan* p, float* F, float* Mx, float* My, float* Mc, int max_iters,
                 ot_dyn_report* rep) {
    if (!p || !F || !Mx || !My || !Mc || max_iters < 1) return OT_ERR_PARAM;
    if (!p->have_init) { p->err = "ot_dyn_init must succeed first"; return OT_ERR_STATE; }
    const auto t0 = std::chrono::steady_clock::now();
    const StepArgs s = step_args(p, F, Mx, My, Mc);
    const bool fallback_armed = p->fallback_armed;
    p->fallback_armed = false;
    int status = solve_loop(p, s, max_iters);
    int done = p->last_solve_iters;
    bool fell_back = false;
    if (fallback_armed && (status == OT_NOT_CONVERGED || status == OT_ERR_NONFINITE)) {
        // the warm start did not certify: Algorithm 1 from its cold start
        const int st = ot_dyn_init(p, OT_INIT_COLD, F, Mx, My, Mc);
        if (st != OT_OK) return st;
        status = solve_loop(p, s, max_iters);
        done += p->last_solve_iters;
        fell_back = true;
    }
    if (rep) {
        fill_report(p, rep);
        rep->iterations = done;
        rep->converged = status == OT_OK;
        rep->fallback = fell_back ? 1 : 0;
        rep->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

}  // extern "C"

namespace {

// The certified-solve loop of ot_dyn_solve: chunks of check_every iterations,
// the last of each with the residual reductions.
int solve_loop(ot_dyn_plan* p, const StepArgs& s, int max_iters) {
    int done = 0, status = OT_NOT_CONVERGED;
    while (done < max_iters) {
        const int chunk = std::min(p->d.check_every, max_iters - done);
        for (int i = 0; i + 1 < chunk; ++i) iterate(p, s, false);
        iterate(p, s, true);
        done += chunk;
        p->total_iters += chunk;
        const int cs = collect(p, s, true);
        if (cs != OT_OK) { status = cs; break; }
        double worst = 0.0, worst_div = 0.0;
        for (int b = 0; b < p->g.B; ++b) {
            worst = std::max(worst, std::max(p->r_prim[b], p->r_dual[b]));
            worst_div = std::max(worst_div, p->r_div[b]);
        }
        p->last_res = worst;
        if (worst < p->d.tol_res && worst_div < p->d.tol_div) { status = OT_OK; break; }
        const int as = adapt_steps(p, s);
        if (as != OT_OK) { status = as; break; }
    }
    p->last_solve_iters = done;
    return status;
}

}  // namespace

extern "C" {

int ot_dyn_residuals(ot_dyn_plan* p, float* F, float* Mx, float* My, float* Mc,
                     ot_dyn_report* rep) {
    if (!p || !F || !Mx || !My || !Mc) return OT_ERR_PARAM;
    if (!p->have_init) { p->err = "ot_dyn_init must succeed first"; return OT_ERR_STATE; }
    const auto t0 = std::chrono::steady_clock::now();
    const StepArgs s = step_args(p, F, Mx, My, Mc);
    const int cs = collect_state(p, s);
    if (rep) {
        fill_report(p, rep);
        rep->iterations = 0;
        rep->converged = 0;
        rep->fallback = 0;
        rep->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return cs;
}

int ot_dyn_get_dual_bar(ot_dyn_plan* p, float* b_bar) {
    if (!p || !b_bar) return OT_ERR_PARAM;
    if (!p->have_init) { p->err = "ot_dyn_init must succeed first"; return OT_ERR_STATE; }
    const size_t nc = (size_t)p->g.nc, w = nc * sizeof(float);
    for (int q = 0; q < 4; ++q)
        HIPCHK(p, hipMemcpy2DAsync(b_bar + q * nc, 4 * w, p->bb[q], w, w, p->g.B,
                                   hipMemcpyDeviceToDevice, p->stream));
    return OT_OK;
}

int ot_dyn_get_dual(ot_dyn_plan* p, float* b) {
    if (!p || !b) return OT_ERR_PARAM;
    if (!p->have_init) { p->err = "ot_dyn_init must succeed first"; return OT_ERR_STATE; }
    const size_t nc = (size_t)p->g.nc, w = nc * sizeof(float);
    for (int q = 0; q < 4; ++q)
        HIPCHK(p, hipMemcpy2DAsync(b + q * nc, 4 * w, p->b[q], w, w, p->g.B, hipMemcpyDeviceToDevice,
                                   p->stream));
    return OT_OK;
}

int ot_dyn_set_dual(ot_dyn_plan* p, const float* b) {
    if (!p || !b) return OT_ERR_PARAM;
    if (!p->have_init) { p->err = "ot_dyn_init must succeed first"; return OT_ERR_STATE; }
    const size_t nc = (size_t)p->g.nc, w = nc * sizeof(float);
    for (int q = 0; q < 4; ++q) {
        HIPCHK(p, hipMemcpy2DAsync(p->b[q], w, b + q * nc, 4 * w, w, p->g.B, hipMemcpyDeviceToDevice,
                                   p->stream));
        HIPCHK(p, hipMemcpy2DAsync(p->bb[q], w, b + q * nc, 4 * w, w, p->g.B, hipMemcpyDeviceToDevice,
                                   p->stream));
    }
    return OT_OK;
}

int ot_dyn_profile(ot_dyn_plan* p, int mask) {
    if (!p) return OT_ERR_PARAM;
    HIPCHK(p, hipStreamSynchronize(p->stream));
    p->prof_mask = mask;
    p->ev_used = 0;
    p->ev_phase.clear();
    for (int q = 0; q < OT_PHASE_COUNT; ++q) { p->prof_ms[q] = 0.0; p->prof_n[q] = 0; }
    return OT_OK;
}

int ot_dyn_profile_read(ot_dyn_plan* p, double* ms, long long* launches, int n) {
    if (!p || n < 0 || n > OT_PHASE_COUNT || (n > 0 && (!ms || !launches))) return OT_ERR_PARAM;
    HIPCHK(p, hipStreamSynchronize(p->stream));
    for (size_t i = 0; i < p->ev_phase.size(); ++i) {
        float t = 0.f;
        HIPCHK(p, hipEventElapsedTime(&t, p->ev_pool[2 * i], p->ev_pool[2 * i + 1]));
        p->prof_ms[p->ev_phase[i]] += t;
        p->prof_n[p->ev_phase[i]] += 1;
    }
    p->ev_phase.clear();
    p->ev_used = 0;
    for (int q = 0; q < n; ++q) { ms[q] = p->prof_ms[q]; launches[q] = p->prof_n[q]; }
    return OT_OK;
}

int ot_dyn_destroy(ot_dyn_plan* p) {
    if (!p) return OT_OK;
    (void)hipStreamSynchronize(p->stream);
    for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
    delete p;
    return OT_OK;
}

const char* ot_dyn_status_str(int status) {
    switch (status) {
        case OT_OK: return "ok";
        case OT_NOT_CONVERGED: return "not converged within max_iters";
        case OT_ERR_PARAM: return "invalid parameter";
        case OT_ERR_SHAPE: return "invalid shape or buffer size";
        case OT_ERR_INPUT: return "negative or non-finite input density";
        case OT_ERR_MASS: return "masses of f0 and f1 differ beyond tol_mass";
        case OT_ERR_HIP: return "HIP runtime error";
        case OT_ERR_NONFINITE: return "non-finite residual";
        case OT_ERR_STATE: return "call out of order";
        default: return "unknown status";
    }
}

const char* ot_dyn_last_error(const ot_dyn_plan* p) {
    return p ? p->err.c_str() : "null plan";
}

int ot_dyn_prox_eval(int kind, long long n, const float* am, const float* af, float sigma,
                     float* u, float* v, void* stream) {
    if (!am || !af || !u || !v || n < 0 || !(sigma > 0.f) || kind < OT_PROX_NEWTON ||
        kind > OT_PROX_CLOSED_RAW || n > (long long)0xffffffffLL * 256)
        return OT_ERR_PARAM;
    launch_prox_eval(kind, n, am, af, sigma, u, v, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? OT_OK : OT_ERR_HIP;
}

}  // extern "C"

// ---- internal hooks for the batched solver (batch.cpp) ---------------------
namespace otd {

void plan_iterate(ot_dyn_plan* p, float* F, float* Mx, float* My, float* Mc, bool check) {
    const StepArgs s = step_args(p, F, Mx, My, Mc);
    iterate(p, s, check);
}

int plan_collect(ot_dyn_plan* p, float* F, float* Mx, float* My, float* Mc) {
    const StepArgs s = step_args(p, F, Mx, My, Mc);
    int st = collect(p, s, true);
    if (st == OT_OK) st = adapt_steps(p, s);
    double worst = 0.0;
    for (int b = 0; b < p->g.B; ++b) worst = std::max(worst, std::max(p->r_prim[b], p->r_dual[b]));
    p->last_res = worst;
    return st;
}

void plan_apply_tuning(ot_dyn_plan* p, int row_bx, int dense_xy) { apply_tuning(p, row_bx, dense_xy); }

int plan_freeze(ot_dyn_plan* p, const std::vector<char>& frozen) {
    bool changed = false;
    for (int b = 0; b < p->g.B; ++b) {
        const float v = frozen[b] ? 1.f : 0.f;
        changed = changed || v != p->frz_h[b];
        p->frz_h[b] = v;
    }
    if (changed)
        HIPCHK(p, hipMemcpyAsync(p->frz, p->frz_h.data(), p->frz_h.size() * sizeof(float),
                                 hipMemcpyHostToDevice, p->stream));
    return OT_OK;
}

void plan_enable_freeze(ot_dyn_plan* p) { p->freezable = true; }

bool plan_has_fast_xy(const ot_dyn_plan* p) {
    return p->tw_fast[0] || p->tw_fast[1] || p->tw_mix[0] || p->tw_mix[1];
}

void plan_problem(const ot_dyn_plan* p, int b, ot_dyn_report* rep) {
    rep->r_prim = p->r_prim[b];
    rep->r_dual = p->r_dual[b];
    rep->r_div = p->r_div[b];
    rep->cost = p->cost[b];
    rep->e_mass = p->e_mass[b];
    rep->mass0 = p->mass0[b];
    rep->mass1 = p->mass1[b];
}

void plan_add_iters(ot_dyn_plan* p, int n) { p->total_iters += n; }

bool plan_launch_varies(const ot_dyn_plan* p) {
    if (p->d.refine == OT_REFINE_ADAPTIVE) return true;
    return p->d.refine == OT_REFINE_CARRY && p->it_next < p->d.carry_refine;
}

int plan_restart_cold(ot_dyn_plan* p, float* F, float* Mx, float* My, float* Mc,
                      const std::vector<char>& which) {
    // the init kernels skip frozen problems: freeze all but `which` for them
    const StepArgs s = step_args(p, F, Mx, My, Mc);
    const std::vector<float> keep = p->frz_h;
    for (int b = 0; b < p->g.B; ++b) {
        p->frz_h[b] = which[b] ? 0.f : 1.f;
        if (!which[b]) continue;
        p->sig_h[b] = (float)p->d.sigma;
        p->n_adapt[b] = 0;
        p->last_adapt[b] = p->total_iters;
    }
    const size_t nb = p->frz_h.size() * sizeof(float);
    HIPCHK(p, hipMemcpyAsync(p->sig, p->sig_h.data(), nb, hipMemcpyHostToDevice, p->stream));
    HIPCHK(p, hipMemcpyAsync(p->frz, p->frz_h.data(), nb, hipMemcpyHostToDevice, p->stream));
    launch_init_state(s, p->f0, p->f1, 1, p->stream);
    launch_zero_dual(s, p->stream);
    HIPCHK(p, hipGetLastError());
    HIPCHK(p, hipStreamSynchronize(p->stream));
    for (int b = 0; b < p->g.B; ++b) p->frz_h[b] = which[b] ? 0.f : keep[b];
    HIPCHK(p, hipMemcpyAsync(p->frz, p->frz_h.data(), nb, hipMemcpyHostToDevice, p->stream));
    HIPCHK(p, hipStreamSynchronize(p->stream));
    p->it_next = 0;        // the restarted problems refine their start again
    p->last_res = 1.0;
    return OT_OK;
}

int plan_copy_dual(ot_dyn_plan* p, int b, float* packed, int to_packed) {
    if (b < 0 || b >= p->g.B) return OT_ERR_PARAM;
    const size_t nc = (size_t)p->g.nc, w = nc * sizeof(float);
    for (int q = 0; q < 4; ++q) {
        if (to_packed) {
            HIPCHK(p, hipMemcpyAsync(packed + q * nc, p->b[q] + b * nc, w, hipMemcpyDeviceToDevice,
                                     p->stream));
        } else {
            HIPCHK(p, hipMemcpyAsync(p->b[q] + b * nc, packed + q * nc, w, hipMemcpyDeviceToDevice,
                                     p->stream));
            HIPCHK(p, hipMemcpyAsync(p->bb[q] + b * nc, packed + q * nc, w, hipMemcpyDeviceToDevice,
                                     p->stream));
        }
    }
    return OT_OK;
}

}  // namespace otd
