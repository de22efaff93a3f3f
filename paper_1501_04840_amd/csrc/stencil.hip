// Staggered-grid stencil kernels of one PDHG iteration (Algorithm 1 of the
// paper, Sec. 3) and the FP64 reductions.
//
// One thread per centred node (b, k, c, y, x); a block covers 256 nodes of
// one (b, k, c) plane, so consecutive lanes read consecutive x (coalesced)
// and each block owns exactly one FP64 partial per reduced quantity.
// Neighbour faces along x and y are re-read by the neighbouring lanes' loads
// (L1/L2 hits); along colour and time they are separate planes.
#include "otd_common.h"
#include "stencil_common.h"

#pragma clang fp contract(on)   // as in stencil_common.h: fusion within an expression only

namespace otd {

constexpr int kBlock = 256;

struct Node {
    int b, k, c, p, y, x;
    long long cb;        // centred offset of plane (b, k, c)
    bool live;
};

__device__ inline Node node_of(const Geom& g) {
    Node n;
    const int s = blockIdx.y;
    const int pc = g.P * g.C;
    n.b = s / pc;
    const int rem = s - n.b * pc;
    n.k = rem / g.C;
    n.c = rem - n.k * g.C;
    n.p = blockIdx.x * kBlock + threadIdx.x;
    n.live = n.p < g.plane;
    n.y = n.live ? n.p / g.X : 0;
    n.x = n.live ? n.p - n.y * g.X : 0;
    n.cb = (long long)n.b * g.nc + (long long)n.k * g.slice + (long long)n.c * g.plane;
    return n;
}

// ---- the staggered work array a (Step 1 input) ---------------------------
// a = x - tau sigma K^T b_bar on unknown faces; walls and absent faces are 0.
// MODE 0 computes it from (x, b_bar).  MODE 1 (refinement) reads the first
// projection x' = a + grad phi_1 from A and phi_1 = R on the fly.  MODE 2
// adds the gradient of the carried potential Phi to the MODE 0 value.
template <int MODE>
struct FaceA {
    const StepArgs& s;
    const Node& n;
    float ts;   // tau sigma / 2

    __device__ float x(int xx) const {
        const Geom& g = s.g;
        if (!g.perx) { if (xx <= 0 || xx >= g.X) return 0.f; }
        else if (xx == g.X) xx = 0;
        const long long row = n.cb + (long long)n.y * g.X;
        const int xm = xx == 0 ? g.X - 1 : xx - 1;
        if (MODE == 1) return s.A[0][row + xx] + g.sx * (s.R[row + xx] - s.R[row + xm]);
        const float v = s.Mx[row + xx] - ts * (s.bb[0][row + xm] + s.bb[0][row + xx]);
        return MODE == 2 ? v + g.sx * (s.Phi[row + xx] - s.Phi[row + xm]) : v;
    }
    __device__ float y(int yy) const {
        const Geom& g = s.g;
        if (!g.pery) { if (yy <= 0 || yy >= g.Y) return 0.f; }
        else if (yy == g.Y) yy = 0;
        const long long i = n.cb + (long long)yy * g.X + n.x;
        const int ym = yy == 0 ? g.Y - 1 : yy - 1;
        const long long im = n.cb + (long long)ym * g.X + n.x;
        if (MODE == 1) return s.A[1][i] + g.sy * (s.R[i] - s.R[im]);
        const float v = s.My[i] - ts * (s.bb[1][im] + s.bb[1][i]);
        return MODE == 2 ? v + g.sy * (s.Phi[i] - s.Phi[im]) : v;
    }
    __device__ float c(int cc) const {
        const Geom& g = s.g;
        if (!g.perc) { if (cc <= 0 || cc >= g.C) return 0.f; }
        else if (cc == g.C) cc = 0;
        const long long i = cidx(g, n.b, n.k, cc, n.p);
        const int cm = cc == 0 ? g.C - 1 : cc - 1;
        const long long im = cidx(g, n.b, n.k, cm, n.p);
        if (MODE == 1) return s.A[2][i] + g.sc * (s.R[i] - s.R[im]);
        const float v = s.Mc[i] - ts * (s.bb[2][im] + s.bb[2][i]);
        return MODE == 2 ? v + g.sc * (s.Phi[i] - s.Phi[im]) : v;
    }
    __device__ float f(int kk) const {   // time kk in [0, P]
        const Geom& g = s.g;
        if (kk == 0 || kk == g.P) return s.F[fidx(g, n.b, kk, n.c, n.p)];
        const long long i = cidx(g, n.b, kk, n.c, n.p);
        const long long im = cidx(g, n.b, kk - 1, n.c, n.p);
        if (MODE == 1) return s.A[3][i] + g.st * (s.R[i] - s.R[im]);
        const float v = s.F[fidx(g, n.b, kk, n.c, n.p)] - ts * (s.bb[3][im] + s.bb[3][i]);
        return MODE == 2 ? v + g.st * (s.Phi[i] - s.Phi[im]) : v;
    }
};

// r = A a - f_b^- (Step 1) with f_b^- folded in through F[0], F[P], and its
// FP64 plane sums.  MODE 0 and MODE 2 write the own faces of a to A and r to
// R; MODE 1 writes the residual of the first projection to R2.
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_div(StepArgs s) {
    const Geom& g = s.g;
    const Node n = node_of(g);
    if (s.frz_run && s.frz_run[n.b] != 0.f) return;   // frozen problem (block-uniform)
    double acc = 0.0;
    if (n.live) {
        FaceA<MODE> a{s, n, 0.5f * s.tau_sigma};
        const float ax0 = a.x(n.x), ay0 = a.y(n.y), ac0 = a.c(n.c), af0 = a.f(n.k);
        const float ax1 = a.x(n.x + 1), ay1 = a.y(n.y + 1), ac1 = a.c(n.c + 1);
        const float af1 = a.f(n.k + 1);
        const float r = g.sx * (ax1 - ax0) + g.sy * (ay1 - ay0) + g.sc * (ac1 - ac0) +
                        g.st * (af1 - af0);
        const long long i = n.cb + n.p;
        if (MODE != 1) {
            s.A[0][i] = ax0;
            s.A[1][i] = ay0;
            s.A[2][i] = ac0;
            s.A[3][i] = n.k > 0 ? af0 : 0.f;
            s.R[i] = r;
        } else {
            s.R2[i] = r;
        }
        acc = (double)r;
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) s.part_slice[(long long)blockIdx.y * s.nbx + blockIdx.x] = t;
}

// x^{r+1} = a + grad phi_1 (+ grad phi_2 when refined, NPHI 2 or 4),
// z = prox(K x + c + b), b and b_bar updates.  NPHI 3 and 4: the carried
// potential Phi takes the potentials on.
template <int CHECK, int NPHI_>
__global__ void __launch_bounds__(kBlock) k_update(StepArgs s) {
    constexpr int NPHI = NPHI_ == 4 ? 2 : (NPHI_ == 3 ? 1 : NPHI_);
    constexpr bool CARRY = NPHI_ >= 3;
    const Geom& g = s.g;
    const Node n = node_of(g);
    if (s.frz_run && s.frz_run[n.b] != 0.f) return;   // frozen problem (block-uniform)
    double db2 = 0, z2 = 0, dx2 = 0, x2 = 0, jj = 0;
    if (n.live) {
        const long long i = n.cb + n.p;
        const long long row = n.cb + (long long)n.y * g.X;
        const float* R = s.R;
        const float* R2 = s.R2;
        // grad of phi_1 (+ phi_2) between centred offsets j and jm
        auto dphi = [&](long long j, long long jm) -> float {
            return NPHI == 2 ? (R[j] - R[jm]) + (R2[j] - R2[jm]) : R[j] - R[jm];
        };
        auto mx = [&](int xx) -> float {
            if (!g.perx) { if (xx <= 0 || xx >= g.X) return 0.f; }
            else if (xx == g.X) xx = 0;
            const int xm = xx == 0 ? g.X - 1 : xx - 1;
            return s.A[0][row + xx] + g.sx * dphi(row + xx, row + xm);
        };
        auto my = [&](int yy) -> float {
            if (!g.pery) { if (yy <= 0 || yy >= g.Y) return 0.f; }
            else if (yy == g.Y) yy = 0;
            const int ym = yy == 0 ? g.Y - 1 : yy - 1;
            const long long j = n.cb + (long long)yy * g.X + n.x;
            return s.A[1][j] + g.sy * dphi(j, n.cb + (long long)ym * g.X + n.x);
        };
        auto mc = [&](int cc) -> float {
            if (!g.perc) { if (cc <= 0 || cc >= g.C) return 0.f; }
            else if (cc == g.C) cc = 0;
            const int cm = cc == 0 ? g.C - 1 : cc - 1;
            const long long j = cidx(g, n.b, n.k, cc, n.p);
            return s.A[2][j] + g.sc * dphi(j, cidx(g, n.b, n.k, cm, n.p));
        };
        auto ff = [&](int kk) -> float {
            if (kk == 0 || kk == g.P) return s.F[fidx(g, n.b, kk, n.c, n.p)];
            const long long j = cidx(g, n.b, kk, n.c, n.p);
            return s.A[3][j] + g.st * dphi(j, cidx(g, n.b, kk - 1, n.c, n.p));
        };
        const float mx0 = mx(n.x), my0 = my(n.y), mc0 = mc(n.c), f0 = ff(n.k);
        const float mx1 = mx(n.x + 1), my1 = my(n.y + 1), mc1 = mc(n.c + 1);
        const float f1 = ff(n.k + 1);
        // K x + c at the node
        const float kx = 0.5f * (mx0 + mx1), ky = 0.5f * (my0 + my1);
        const float kc = 0.5f * (mc0 + mc1), kf = 0.5f * (f0 + f1);
        const float bx = s.b[0][i], by = s.b[1][i], bc = s.b[2][i], bf = s.b[3][i];
        const float amx = kx + bx, amy = ky + by, amc = kc + bc, amf = kf + bf;
        float ux, uy, uc, vv;
        prox_J(amx, amy, amc, amf, s.sig[n.b], ux, uy, uc, vv, s.prox);
        const float nbx = amx - ux, nby = amy - uy, nbc = amc - uc, nbf = amf - vv;
        const float th = s.theta;
        s.b[0][i] = nbx; s.bb[0][i] = nbx + th * (nbx - bx);
        s.b[1][i] = nby; s.bb[1][i] = nby + th * (nby - by);
        s.b[2][i] = nbc; s.bb[2][i] = nbc + th * (nbc - bc);
        s.b[3][i] = nbf; s.bb[3][i] = nbf + th * (nbf - bf);
        const long long fi = fidx(g, n.b, n.k, n.c, n.p);
        if (CHECK) {
            const float ox = s.Mx[i], oy = s.My[i], oc = s.Mc[i];
            const float of = n.k > 0 ? s.F[fi] : 0.f;
            const float nf = n.k > 0 ? f0 : 0.f;
            const double ddx = (double)mx0 - ox, ddy = (double)my0 - oy;
            const double ddc = (double)mc0 - oc, ddf = (double)nf - of;
            dx2 = ddx * ddx + ddy * ddy + ddc * ddc + ddf * ddf;
            x2 = (double)mx0 * mx0 + (double)my0 * my0 + (double)mc0 * mc0 + (double)nf * nf;
            const double ex = (double)nbx - bx, ey = (double)nby - by;
            const double ec = (double)nbc - bc, ef = (double)nbf - bf;
            db2 = ex * ex + ey * ey + ec * ec + ef * ef;
            const double u2 = (double)ux * ux + (double)uy * uy + (double)uc * uc;
            z2 = u2 + (double)vv * vv;
            jj = vv > 0.f ? u2 / (2.0 * vv) : 0.0;
        }
        s.Mx[i] = mx0;
        s.My[i] = my0;
        s.Mc[i] = mc0;
        if (n.k > 0) s.F[fi] = f0;
        if (CARRY) s.Phi[i] = s.Phi[i] + (NPHI == 2 ? R[i] + R2[i] : R[i]);
    }
    if (CHECK) {
        const long long nblk = (long long)gridDim.x * gridDim.y;
        const long long o = (long long)blockIdx.y * gridDim.x + blockIdx.x;
        const double vals[RS_COUNT] = {db2, z2, dx2, x2, jj};
        for (int q = 0; q < RS_COUNT; ++q) {
            const double t = block_sum(vals[q]);
            if (threadIdx.x == 0) s.part_red[q * nblk + o] = t;
        }
    }
}

// FP64 partials of |A x - f_b^-|^2 and of the plane sums of F (slices 0..P-1).
__global__ void __launch_bounds__(kBlock) k_resid_div(StepArgs s) {
    const Geom& g = s.g;
    const Node n = node_of(g);
    double r2 = 0.0, mass = 0.0;
    if (n.live) {
        // a = x: reuse the MODE 1 face reader on the state itself
        const long long row = n.cb + (long long)n.y * g.X;
        auto fx = [&](int xx) -> float {
            if (!g.perx) { if (xx <= 0 || xx >= g.X) return 0.f; }
            else if (xx == g.X) xx = 0;
            return s.Mx[row + xx];
        };
        auto fy = [&](int yy) -> float {
            if (!g.pery) { if (yy <= 0 || yy >= g.Y) return 0.f; }
            else if (yy == g.Y) yy = 0;
            return s.My[n.cb + (long long)yy * g.X + n.x];
        };
        auto fc = [&](int cc) -> float {
            if (!g.perc) { if (cc <= 0 || cc >= g.C) return 0.f; }
            else if (cc == g.C) cc = 0;
            return s.Mc[cidx(g, n.b, n.k, cc, n.p)];
        };
        const float f0 = s.F[fidx(g, n.b, n.k, n.c, n.p)];
        const float f1 = s.F[fidx(g, n.b, n.k + 1, n.c, n.p)];
        const double r = (double)g.sx * ((double)fx(n.x + 1) - fx(n.x)) +
                         (double)g.sy * ((double)fy(n.y + 1) - fy(n.y)) +
                         (double)g.sc * ((double)fc(n.c + 1) - fc(n.c)) +
                         (double)g.st * ((double)f1 - f0);
        r2 = r * r;
        mass = f0;
    }
    const long long o = (long long)blockIdx.y * gridDim.x + blockIdx.x;
    double t = block_sum(r2);
    if (threadIdx.x == 0) s.part_div[o] = t;
    t = block_sum(mass);
    if (threadIdx.x == 0) s.part_mass[o] = t;
}

// Residuals of the current state (x, b) without iterating: z = prox(K x +
// c + b) at the node (Sec. 3, Step 2), then |K x + c - z|^2, |z|^2, J(z) and
// |x|^2 over the node's own faces.  Reads only; one FP64 partial per block
// and slot in part_red ([RS_COUNT][B][P C nblk]).
__global__ void __launch_bounds__(kBlock) k_resid_state(StepArgs s) {
    const Geom& g = s.g;
    const Node n = node_of(g);
    double db2 = 0.0, z2 = 0.0, x2 = 0.0, jj = 0.0;
    if (n.live) {
        const long long row = n.cb + (long long)n.y * g.X;
        auto fx = [&](int xx) -> float {
            if (!g.perx) { if (xx <= 0 || xx >= g.X) return 0.f; }
            else if (xx == g.X) xx = 0;
            return s.Mx[row + xx];
        };
        auto fy = [&](int yy) -> float {
            if (!g.pery) { if (yy <= 0 || yy >= g.Y) return 0.f; }
            else if (yy == g.Y) yy = 0;
            return s.My[n.cb + (long long)yy * g.X + n.x];
        };
        auto fc = [&](int cc) -> float {
            if (!g.perc) { if (cc <= 0 || cc >= g.C) return 0.f; }
            else if (cc == g.C) cc = 0;
            return s.Mc[cidx(g, n.b, n.k, cc, n.p)];
        };
        const float mx0 = fx(n.x), my0 = fy(n.y), mc0 = fc(n.c);
        const float f0 = s.F[fidx(g, n.b, n.k, n.c, n.p)];
        const float f1 = s.F[fidx(g, n.b, n.k + 1, n.c, n.p)];
        const float kx = 0.5f * (mx0 + fx(n.x + 1)), ky = 0.5f * (my0 + fy(n.y + 1));
        const float kc = 0.5f * (mc0 + fc(n.c + 1)), kf = 0.5f * (f0 + f1);
        const long long i = n.cb + n.p;
        float ux, uy, uc, vv;
        prox_J(kx + s.b[0][i], ky + s.b[1][i], kc + s.b[2][i], kf + s.b[3][i], s.sig[n.b], ux, uy,
               uc, vv, s.prox);
        const double ex = (double)kx - ux, ey = (double)ky - uy, ec = (double)kc - uc;
        const double ef = (double)kf - vv;
        db2 = ex * ex + ey * ey + ec * ec + ef * ef;
        const double u2 = (double)ux * ux + (double)uy * uy + (double)uc * uc;
        z2 = u2 + (double)vv * vv;
        jj = vv > 0.f ? u2 / (2.0 * vv) : 0.0;
        const double nf = n.k > 0 ? (double)f0 : 0.0;
        x2 = (double)mx0 * mx0 + (double)my0 * my0 + (double)mc0 * mc0 + nf * nf;
    }
    const long long nblk = (long long)gridDim.x * gridDim.y;
    const long long o = (long long)blockIdx.y * gridDim.x + blockIdx.x;
    const double vals[RS_COUNT] = {db2, z2, 0.0, x2, jj};
    for (int q = 0; q < RS_COUNT; ++q) {
        const double t = block_sum(vals[q]);
        if (threadIdx.x == 0) s.part_red[q * nblk + o] = t;
    }
}

// Boundary slices of F, Neumann wall slots, optional zero unknowns; frozen
// problems are left alone (ot_dyn_init releases every problem first).
__global__ void __launch_bounds__(kBlock) k_init_state(StepArgs s, const float* f0,
                                                       const float* f1, int zero) {
    const Geom& g = s.g;
    const Node n = node_of(g);
    if (!n.live || s.frz[n.b] != 0.f) return;
    const long long i = n.cb + n.p;
    const long long e = (long long)n.b * g.slice + (long long)n.c * g.plane + n.p;
    if (n.k == 0) s.F[fidx(g, n.b, 0, n.c, n.p)] = f0[e];
    if (n.k == g.P - 1) s.F[fidx(g, n.b, g.P, n.c, n.p)] = f1[e];
    if (s.Phi) s.Phi[i] = 0.f;
    if (zero) {
        s.Mx[i] = 0.f; s.My[i] = 0.f; s.Mc[i] = 0.f;
        if (n.k > 0) s.F[fidx(g, n.b, n.k, n.c, n.p)] = 0.f;
    } else {
        if (!g.perx && n.x == 0) s.Mx[i] = 0.f;
        if (!g.pery && n.y == 0) s.My[i] = 0.f;
        if (!g.perc && n.c == 0) s.Mc[i] = 0.f;
    }
}

__global__ void __launch_bounds__(kBlock) k_zero_dual(StepArgs s) {
    const Geom& g = s.g;
    const Node n = node_of(g);
    if (!n.live || s.frz[n.b] != 0.f) return;
    const long long i = n.cb + n.p;
    for (int q = 0; q < 4; ++q) { s.b[q][i] = 0.f; s.bb[q][i] = 0.f; }
}

__global__ void __launch_bounds__(kBlock) k_scale_dual(StepArgs s, const float* fac) {
    const Geom& g = s.g;
    const Node n = node_of(g);
    if (!n.live) return;
    const long long i = n.cb + n.p;
    const float f = fac[n.b];
    for (int q = 0; q < 4; ++q) { s.b[q][i] *= f; s.bb[q][i] *= f; }
}

// b = b_bar = grad J(K x + c) / sigma (the dual that makes a given primal a
// fixed point of Steps 2-4 where v > 0), with v floored at vfloor[b]: at
// nodes of (near) vacuum the fixed-point dual is not the gradient, and the
// floor keeps the velocity u / v there near 0 instead of blowing it up.
__global__ void __launch_bounds__(kBlock) k_init_dual(StepArgs s, const double* vfloor) {
    const Geom& g = s.g;
    const Node n = node_of(g);
    if (!n.live) return;
    const long long i = n.cb + n.p;
    const long long row = n.cb + (long long)n.y * g.X;
    auto fx = [&](int xx) -> float {
        if (!g.perx) { if (xx <= 0 || xx >= g.X) return 0.f; }
        else if (xx == g.X) xx = 0;
        return s.Mx[row + xx];
    };
    auto fy = [&](int yy) -> float {
        if (!g.pery) { if (yy <= 0 || yy >= g.Y) return 0.f; }
        else if (yy == g.Y) yy = 0;
        return s.My[n.cb + (long long)yy * g.X + n.x];
    };
    auto fc = [&](int cc) -> float {
        if (!g.perc) { if (cc <= 0 || cc >= g.C) return 0.f; }
        else if (cc == g.C) cc = 0;
        return s.Mc[cidx(g, n.b, n.k, cc, n.p)];
    };
    const float ux = 0.5f * (fx(n.x) + fx(n.x + 1));
    const float uy = 0.5f * (fy(n.y) + fy(n.y + 1));
    const float uc = 0.5f * (fc(n.c) + fc(n.c + 1));
    float v = 0.5f * (s.F[fidx(g, n.b, n.k, n.c, n.p)] + s.F[fidx(g, n.b, n.k + 1, n.c, n.p)]);
    v = fmaxf(v, (float)vfloor[n.b]);
    const float is = 1.f / (s.sig[n.b] * v);
    const float bx = ux * is, by = uy * is, bc = uc * is;
    const float bf = -(ux * ux + uy * uy + uc * uc) * 0.5f * is / v;
    s.b[0][i] = bx; s.bb[0][i] = bx;
    s.b[1][i] = by; s.bb[1][i] = by;
    s.b[2][i] = bc; s.bb[2][i] = bc;
    s.b[3][i] = bf; s.bb[3][i] = bf;
}

// part layout: [5][B][nblk]: sum f0, sum f1, count of invalid entries,
// sum f0^2, sum f1^2.
__global__ void __launch_bounds__(kBlock) k_boundary_stats(Geom g, const float* f0,
                                                           const float* f1, double* part) {
    const int b = blockIdx.y;
    const long long n = g.slice;
    double s0 = 0, s1 = 0, bad = 0, q0 = 0, q1 = 0;
    for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < n;
         e += (long long)gridDim.x * kBlock) {
        const float a = f0[b * n + e], c = f1[b * n + e];
        if (!(a >= 0.f) || !(c >= 0.f) || !isfinite(a) || !isfinite(c)) bad += 1.0;
        s0 += a;
        s1 += c;
        q0 += (double)a * a;
        q1 += (double)c * c;
    }
    const long long nb = gridDim.x, o = (long long)b * nb + blockIdx.x;
    const long long q = (long long)g.B * nb;
    const double vals[5] = {s0, s1, bad, q0, q1};
    for (int i = 0; i < 5; ++i) {
        const double t = block_sum(vals[i]);
        if (threadIdx.x == 0) part[i * q + o] = t;
    }
}

__global__ void __launch_bounds__(kBlock) k_reduce(const double* part, long long n, double* out) {
    const int q = blockIdx.x;
    double acc = 0.0;
    for (long long j = threadIdx.x; j < n; j += kBlock) acc += part[q * n + j];
    const double t = block_sum(acc);
    if (threadIdx.x == 0) out[q] = t;
}

// ---- launchers ------------------------------------------------------------

static dim3 node_grid(const Geom& g) {
    return dim3((unsigned)((g.plane + kBlock - 1) / kBlock), (unsigned)(g.B * g.P * g.C));
}

void launch_div(const StepArgs& s, int mode, hipStream_t st) {
    if (rows_ok(s.g)) { launch_div_rows(s, mode, st); return; }
    if (mode == 0) hipLaunchKernelGGL(k_div<0>, node_grid(s.g), dim3(kBlock), 0, st, s);
    else if (mode == 1) hipLaunchKernelGGL(k_div<1>, node_grid(s.g), dim3(kBlock), 0, st, s);
    else hipLaunchKernelGGL(k_div<2>, node_grid(s.g), dim3(kBlock), 0, st, s);
}

void launch_update(const StepArgs& s, int check, int nphi, hipStream_t st) {
    if (rows_ok(s.g)) { launch_update_rows(s, check, nphi, st); return; }
    const dim3 gr = node_grid(s.g), bl(kBlock);
    if (nphi == 2) {
        if (check) hipLaunchKernelGGL((k_update<1, 2>), gr, bl, 0, st, s);
        else hipLaunchKernelGGL((k_update<0, 2>), gr, bl, 0, st, s);
    } else if (nphi == 3) {
        if (check) hipLaunchKernelGGL((k_update<1, 3>), gr, bl, 0, st, s);
        else hipLaunchKernelGGL((k_update<0, 3>), gr, bl, 0, st, s);
    } else if (nphi == 4) {
        if (check) hipLaunchKernelGGL((k_update<1, 4>), gr, bl, 0, st, s);
        else hipLaunchKernelGGL((k_update<0, 4>), gr, bl, 0, st, s);
    } else {
        if (check) hipLaunchKernelGGL((k_update<1, 1>), gr, bl, 0, st, s);
        else hipLaunchKernelGGL((k_update<0, 1>), gr, bl, 0, st, s);
    }
}

__global__ void __launch_bounds__(kBlock) k_prox_eval(int kind, long long n, const float* am,
                                                    const float* af, float sigma, float* u,
                                                    float* v) {
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    float ux, uy, uc, vv;
    prox_J(am[i], am[n + i], am[2 * n + i], af[i], sigma, ux, uy, uc, vv, kind);
    u[i] = ux;
    u[n + i] = uy;
    u[2 * n + i] = uc;
    v[i] = vv;
}

void launch_prox_eval(int kind, long long n, const float* am, const float* af, float sigma,
                      float* u, float* v, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_prox_eval, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                       kind, n, am, af, sigma, u, v);
}

void launch_resid_div(const StepArgs& s, hipStream_t st) {
    hipLaunchKernelGGL(k_resid_div, node_grid(s.g), dim3(kBlock), 0, st, s);
}

void launch_resid_state(const StepArgs& s, hipStream_t st) {
    hipLaunchKernelGGL(k_resid_state, node_grid(s.g), dim3(kBlock), 0, st, s);
}

void launch_init_state(const StepArgs& s, const float* f0, const float* f1,
                       int zero_unknowns, hipStream_t st) {
    hipLaunchKernelGGL(k_init_state, node_grid(s.g), dim3(kBlock), 0, st, s, f0, f1,
                       zero_unknowns);
}

void launch_init_dual(const StepArgs& s, const double* vfloor, hipStream_t st) {
    hipLaunchKernelGGL(k_init_dual, node_grid(s.g), dim3(kBlock), 0, st, s, vfloor);
}

void launch_zero_dual(const StepArgs& s, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_dual, node_grid(s.g), dim3(kBlock), 0, st, s);
}

void launch_scale_dual(const StepArgs& s, const float* fac, hipStream_t st) {
    hipLaunchKernelGGL(k_scale_dual, node_grid(s.g), dim3(kBlock), 0, st, s, fac);
}

void launch_boundary_stats(const Geom& g, const float* f0, const float* f1, double* part,
                           int nblk, hipStream_t st) {
    hipLaunchKernelGGL(k_boundary_stats, dim3(nblk, g.B), dim3(kBlock), 0, st, g, f0, f1,
                       part);
}

void launch_reduce(const double* part, long long n, int nq, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce, dim3(nq), dim3(kBlock), 0, st, part, n, out);
}

}  // namespace otd
