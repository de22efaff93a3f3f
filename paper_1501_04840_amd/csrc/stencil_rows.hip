// Stencil kernels of one PDHG iteration (Algorithm 1 of the paper, Sec. 3)
// laid out for the MI355X cache hierarchy.
//
// A thread owns the node (b, k, y, x) for all C colours, so the colour faces
// (periodic: face c between channels c-1 and c) come from registers.  A
// block covers one x-row segment; blocks are ordered with time fastest, then
// y, then problem, and the hardware block id is remapped so that each of the
// 8 XCDs (one L2 each) walks a contiguous range of that order: the k+1 row is
// the next block and the y+1 row is P blocks later on the same XCD, so the
// neighbour reads of the staggered stencils are L2 hits instead of refetches.
#include "otd_common.h"
#include "fft_lines.h"
#include "stencil_common.h"

#pragma clang fp contract(on)   // as in stencil_common.h: fusion within an expression only

namespace otd {

// Hardware blocks are dispatched round-robin over the 8 XCDs; give XCD j the
// j-th contiguous eighth of the logical order.
__device__ inline long long xcd_remap(long long hw, long long n) {
    const long long q = n >> 3, r = n & 7, xcd = hw & 7, slot = hw >> 3;
    return xcd * q + (xcd < r ? xcd : r) + slot;
}

struct RowCtx {
    int b, k, y, x, xb;
    long long L;         // logical block id
    long long i0;        // centred offset of (b, k, c = 0, y, x)
    long long f0;        // F offset of (b, k, c = 0, y, x)
    bool live;
};

__device__ inline RowCtx row_ctx(const Geom& g, int nxb) {
    RowCtx r;
    r.L = xcd_remap(blockIdx.x, gridDim.x);
    long long t = r.L;
    r.xb = (int)(t % nxb); t /= nxb;
    r.k = (int)(t % g.P); t /= g.P;
    r.y = (int)(t % g.Y); t /= g.Y;
    r.b = (int)t;
    r.x = r.xb * blockDim.x + threadIdx.x;
    r.live = r.x < g.X;
    const long long p = (long long)r.y * g.X + (r.live ? r.x : 0);
    r.i0 = (long long)r.b * g.nc + (long long)r.k * g.slice + p;
    r.f0 = (long long)r.b * g.nf + (long long)r.k * g.slice + p;
    return r;
}

// Neighbour offsets of a node within its plane, with the Neumann walls.
struct Nbr {
    long long dxm, dxp, dym, dyp;   // offsets of the x-1, x+1, y-1, y+1 cells (wrapped)
    bool wx0, wx1, wy0, wy1;        // own / next face is a Neumann wall (value 0)
};

__device__ inline Nbr neighbours(const Geom& g, int x, int y) {
    Nbr n;
    n.dxm = x == 0 ? g.X - 1 : -1;
    n.dxp = x + 1 == g.X ? -(long long)(g.X - 1) : 1;
    n.dym = y == 0 ? (long long)(g.Y - 1) * g.X : -(long long)g.X;
    n.dyp = y + 1 == g.Y ? -(long long)(g.Y - 1) * g.X : (long long)g.X;
    n.wx0 = !g.perx && x == 0;
    n.wx1 = !g.perx && x + 1 == g.X;
    n.wy0 = !g.pery && y == 0;
    n.wy1 = !g.pery && y + 1 == g.Y;
    return n;
}

// Stores of the iteration's fields that a later kernel reads (a' and the
// state, duals and carried potential), marked non-temporal when the fields
// are too large for the caches to hold an iteration's working set
// (StepArgs::nt_store; the kernels take it as the template parameter NT: a
// branch per store measured 4% slower).  Measured at 256 x 256 x 3 x 32: the storing kernel
// takes a little longer, the kernel that reads the fields next is faster by
// more (the update's stores made the divergence kernel 8 us faster); at
// 100 x 100 x 3 x 32, whose fields stay cached, they made the iteration 13%
// slower.  r, which the Poisson solve's first pass reads right away, keeps
// normal stores.
template <bool NT>
__device__ __forceinline__ void st_f(float* p, float v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// The residual of a node in colour modes for the fused Poisson solve: out
// at colour stride plane gets sum_c M_c[jc][c] r[c] (cm[c C + jc] =
// M_c[jc][c]), the colour transform the solve's first pass would apply (the
// same products in the same order).
template <int C>
__device__ __forceinline__ void colour_modes(const float (&cm)[C * C], const float (&r)[C],
                                             float* out, long long plane) {
#pragma unroll
    for (int jc = 0; jc < C; ++jc) {
        float acc = 0.f;
#pragma unroll
        for (int c = 0; c < C; ++c) acc = fmaf(cm[c * C + jc], r[c], acc);
        out[(long long)jc * plane] = acc;
    }
}

// Short vectors of NX nodes consecutive along x (16-byte accesses for NX = 4).
template <int NX>
using fvec = float __attribute__((ext_vector_type(NX)));

template <int NX>
__device__ __forceinline__ fvec<NX> ld_v(const float* p) {
    return *reinterpret_cast<const fvec<NX>*>(p);
}

// Non-temporal vector load, for a field the kernel reads once at the node
// and no other wavefront reads in this kernel.
template <int NX>
__device__ __forceinline__ fvec<NX> ld_ntv(const float* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const fvec<NX>*>(p));
}

template <int NX, bool NT>
__device__ __forceinline__ void st_v(float* p, fvec<NX> v) {
    if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<fvec<NX>*>(p));
    else *reinterpret_cast<fvec<NX>*>(p) = v;
}

// The value of v held by the lane d places away along the wavefront (d = +-1,
// wrapping across the 64 lanes).
__device__ __forceinline__ float lane_rot(float v, int d) {
    return __shfl(v, ((int)(threadIdx.x & 63) + d) & 63, 64);
}

// r = A a - f_b^- with a = x - tau sigma K^T b_bar (MODE 0: also writes a to A
// and r to R), a = A + grad phi_1 (MODE 1, refinement: writes r to R2) or
// a = x - tau sigma K^T b_bar + grad Phi with the carried potential Phi
// (MODE 2: writes a to A and r to R), and the FP64 plane sums of r (one
// partial per block and colour).  XL > 0: the block owns whole rows of
// length XL (one per colour), and r is written already transformed along x
// (the first pass of the Poisson solve of Sec. 3: DCT-II for XK = 0, discrete
// Hartley for XK = 2) from the rows staged in LDS.
template <int MODE, int C, int XL, int XK, bool NT>
__global__ void __launch_bounds__(256) k_div_rows(StepArgs s, int nxb) {
    const Geom& g = s.g;
    const RowCtx r = row_ctx(g, nxb);
    constexpr int XP = XL + 1;                     // LDS row pitch
    __shared__ float xl[XL > 0 ? C * XP : 1];
    if (s.frz_run && s.frz_run[r.b] != 0.f) return;   // frozen problem (block-uniform)
    const float ts = 0.5f * s.tau_sigma;
    // the colour transform of r (fused Poisson solve), read before the first
    // store: the compiler cannot tell the stores from these loads
    float cm[C * C];
    const bool mix = XL == 0 && C > 1 && s.cmix != nullptr;
#pragma unroll
    for (int q = 0; q < C * C; ++q) cm[q] = mix ? s.cmix[q] : 0.f;
    float rv[C];
#pragma unroll
    for (int c = 0; c < C; ++c) rv[c] = 0.f;
    if (r.live) {
        const Nbr nb = neighbours(g, r.x, r.y);
        const long long sl = g.slice;
        const bool k0 = r.k == 0, k1 = r.k + 1 == g.P;
        if constexpr (MODE != 1) {
            // Every operand of all colours is loaded before the first store:
            // the stores to A and R may alias the inputs as far as the
            // compiler knows, and interleaving would serialise the colours.
            constexpr bool Q = MODE == 2;
            const long long dtm = k0 ? 0 : -sl, dtp = k1 ? 0 : sl;   // clamped time steps
            float X0[C], X1[C], Y0[C], Y1[C], MC[C], T0[C], T1[C];
            float BXm[C], BXc[C], BXp[C], BYm[C], BYc[C], BYp[C], BC[C], BTm[C], BTc[C], BTp[C];
            float Qc[C], Qxm[C], Qxp[C], Qym[C], Qyp[C], Qtm[C], Qtp[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const long long i = r.i0 + (long long)c * g.plane;
                const long long fi = r.f0 + (long long)c * g.plane;
                X0[c] = s.Mx[i]; X1[c] = s.Mx[i + nb.dxp];
                Y0[c] = s.My[i]; Y1[c] = s.My[i + nb.dyp];
                MC[c] = s.Mc[i];
                T0[c] = s.F[fi]; T1[c] = s.F[fi + sl];
                BXm[c] = s.bb[0][i + nb.dxm]; BXc[c] = s.bb[0][i]; BXp[c] = s.bb[0][i + nb.dxp];
                BYm[c] = s.bb[1][i + nb.dym]; BYc[c] = s.bb[1][i]; BYp[c] = s.bb[1][i + nb.dyp];
                BC[c] = s.bb[2][i];
                BTm[c] = s.bb[3][i + dtm]; BTc[c] = s.bb[3][i]; BTp[c] = s.bb[3][i + dtp];
                if constexpr (Q) {
                    const float* P = s.Phi;
                    Qc[c] = P[i];
                    Qxm[c] = P[i + nb.dxm]; Qxp[c] = P[i + nb.dxp];
                    Qym[c] = P[i + nb.dym]; Qyp[c] = P[i + nb.dyp];
                    Qtm[c] = P[i + dtm]; Qtp[c] = P[i + dtp];
                }
            }
            float acv[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int cm = c == 0 ? C - 1 : c - 1;
                float v = MC[c] - ts * (BC[cm] + BC[c]);
                if constexpr (Q) v += g.sc * (Qc[c] - Qc[cm]);
                acv[c] = ((!g.perc && c == 0) || C == 1) ? 0.f : v;
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                float ax0 = X0[c] - ts * (BXm[c] + BXc[c]);
                float ax1 = X1[c] - ts * (BXc[c] + BXp[c]);
                float ay0 = Y0[c] - ts * (BYm[c] + BYc[c]);
                float ay1 = Y1[c] - ts * (BYc[c] + BYp[c]);
                float af0 = T0[c] - ts * (BTm[c] + BTc[c]);
                float af1 = T1[c] - ts * (BTc[c] + BTp[c]);
                if constexpr (Q) {           // + grad Phi on the unknown faces
                    ax0 += g.sx * (Qc[c] - Qxm[c]);
                    ax1 += g.sx * (Qxp[c] - Qc[c]);
                    ay0 += g.sy * (Qc[c] - Qym[c]);
                    ay1 += g.sy * (Qyp[c] - Qc[c]);
                    af0 += g.st * (Qc[c] - Qtm[c]);
                    af1 += g.st * (Qtp[c] - Qc[c]);
                }
                ax0 = nb.wx0 ? 0.f : ax0;
                ax1 = nb.wx1 ? 0.f : ax1;
                ay0 = nb.wy0 ? 0.f : ay0;
                ay1 = nb.wy1 ? 0.f : ay1;
                af0 = k0 ? T0[c] : af0;      // boundary slices are data
                af1 = k1 ? T1[c] : af1;
                const float ac1 = C == 1 ? 0.f
                                  : (c + 1 < C ? acv[(c + 1) % C] : (g.perc ? acv[0] : 0.f));
                const float rr = g.sx * (ax1 - ax0) + g.sy * (ay1 - ay0) + g.sc * (ac1 - acv[c]) +
                                 g.st * (af1 - af0);
                const long long i = r.i0 + (long long)c * g.plane;
                st_f<NT>(s.A[0] + i, ax0);
                st_f<NT>(s.A[1] + i, ay0);
                st_f<NT>(s.A[2] + i, acv[c]);
                st_f<NT>(s.A[3] + i, k0 ? 0.f : af0);
                if constexpr (XL > 0) xl[c * XP + r.x] = rr;
                else if (!mix) s.R[i] = rr;
                rv[c] = rr;
            }
            if (mix) colour_modes<C>(cm, rv, s.R + r.i0, g.plane);
        } else {
            // colour faces first: own face c of every colour, into registers
            float acv[C];
            {
                float w[C];
#pragma unroll
                for (int c = 0; c < C; ++c) w[c] = s.R[r.i0 + (long long)c * g.plane];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const int cm = c == 0 ? C - 1 : c - 1;
                    const long long i = r.i0 + (long long)c * g.plane;
                    const float v = s.A[2][i] + g.sc * (w[c] - w[cm]);
                    acv[c] = ((!g.perc && c == 0) || C == 1) ? 0.f : v;
                }
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const long long i = r.i0 + (long long)c * g.plane;
                const long long fi = r.f0 + (long long)c * g.plane;
                const float* R = s.R;
                const float pc = R[i];
                const float ax0 = nb.wx0 ? 0.f : s.A[0][i] + g.sx * (pc - R[i + nb.dxm]);
                const float ax1 = nb.wx1 ? 0.f : s.A[0][i + nb.dxp] + g.sx * (R[i + nb.dxp] - pc);
                const float ay0 = nb.wy0 ? 0.f : s.A[1][i] + g.sy * (pc - R[i + nb.dym]);
                const float ay1 = nb.wy1 ? 0.f : s.A[1][i + nb.dyp] + g.sy * (R[i + nb.dyp] - pc);
                const float af0 = k0 ? s.F[fi] : s.A[3][i] + g.st * (pc - R[i - sl]);
                const float af1 = k1 ? s.F[fi + sl] : s.A[3][i + sl] + g.st * (R[i + sl] - pc);
                const float ac1 = C == 1 ? 0.f
                                  : (c + 1 < C ? acv[(c + 1) % C] : (g.perc ? acv[0] : 0.f));
                const float rr = g.sx * (ax1 - ax0) + g.sy * (ay1 - ay0) + g.sc * (ac1 - acv[c]) +
                                 g.st * (af1 - af0);
                if constexpr (XL > 0) xl[c * XP + r.x] = rr;
                else if (!mix) s.R2[i] = rr;
                rv[c] = rr;
            }
            if (mix) colour_modes<C>(cm, rv, s.R2 + r.i0, g.plane);
        }
    }
    const long long col = (long long)r.y * nxb + r.xb;
    double sums[C];
#pragma unroll
    for (int c = 0; c < C; ++c) sums[c] = (double)rv[c];
    block_sums(sums);
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < C; ++c)
            s.part_slice[(((long long)r.b * g.P + r.k) * C + c) * s.nbx + col] = sums[c];
    if constexpr (XL > 0) {
        // the C rows of r along x, M2 threads per row (block_sums has
        // synchronised the block since the rows were staged)
        constexpr int M1 = XL == 256 ? 16 : 8, M2 = XL == 64 ? 4 : 8;
        const int line = threadIdx.x / M2, t = threadIdx.x - line * M2;
        const bool act = line < C;
        float* const sl = xl + (act ? line : 0) * XP;
        if constexpr (XK == 0) line_dct2<M1, M2>(sl, t, s.twx, act);
        else line_dht<M1, M2>(sl, t, s.twx, act);
        float* const out = MODE == 1 ? s.R2 : s.R;
#pragma unroll
        for (int c = 0; c < C; ++c) out[r.i0 + (long long)c * g.plane] = xl[c * XP + r.x];
    }
}

// k_div_rows without the folded x transform (XL = 0) for rows of X = 64 NX
// nodes (128 or 256), laid out as k_update_vec: a wavefront per row, NX
// nodes per lane, NX-wide accesses, x neighbours by lane rotation, one
// colour's loads at a time after the colour faces.  The same expressions per
// node as k_div_rows; the FP64 plane sums of r are per row (wavefront), the
// slots k_div_rows fills with one block per row.
template <int MODE, int C, bool NT, int NX>
__global__ void __launch_bounds__(256) k_div_vec(StepArgs s) {
    using V = fvec<NX>;
    const Geom& g = s.g;
    const long long nrows = (long long)g.B * g.Y * g.P;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const long long row = xcd_remap(blockIdx.x, gridDim.x) * (long long)(blockDim.x >> 6) + w;
    if (row >= nrows) return;
    const int k = (int)(row % g.P), y = (int)((row / g.P) % g.Y), b = (int)(row / ((long long)g.P * g.Y));
    if (s.frz_run && s.frz_run[b] != 0.f) return;   // frozen problem (wave-uniform)
    const float ts = 0.5f * s.tau_sigma;
    float cm[C * C];
    const bool mix = C > 1 && s.cmix != nullptr;
#pragma unroll
    for (int q = 0; q < C * C; ++q) cm[q] = mix ? s.cmix[q] : 0.f;
    const int lane = (int)(threadIdx.x & 63);
    const long long p = (long long)y * g.X + (long long)lane * NX;
    const long long i0 = (long long)b * g.nc + (long long)k * g.slice + p;
    const long long f00 = (long long)b * g.nf + (long long)k * g.slice + p;
    const long long sl = g.slice;
    const bool k0 = k == 0, k1 = k + 1 == g.P;
    const long long dtm = k0 ? 0 : -sl, dtp = k1 ? 0 : sl;   // clamped time steps
    const long long dym = y == 0 ? (long long)(g.Y - 1) * g.X : -(long long)g.X;
    const long long dyp = y + 1 == g.Y ? -(long long)(g.Y - 1) * g.X : (long long)g.X;
    const bool wy0 = !g.pery && y == 0, wy1 = !g.pery && y + 1 == g.Y;
    const bool wx0 = !g.perx && lane == 0, wx1 = !g.perx && lane == 63;   // row ends
    V rv[C];
    if constexpr (MODE != 1) {
        constexpr bool Q = MODE == 2;
        // colour faces of a: own face c of every colour
        V BC[C], Qc[C], acv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            BC[c] = ld_ntv<NX>(s.bb[2] + i0 + (long long)c * g.plane);
            if constexpr (Q) Qc[c] = ld_v<NX>(s.Phi + i0 + (long long)c * g.plane);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int cm_ = c == 0 ? C - 1 : c - 1;
            const V MC = ld_ntv<NX>(s.Mc + i0 + (long long)c * g.plane);
#pragma unroll
            for (int e = 0; e < NX; ++e) {
                float v = MC[e] - ts * (BC[cm_][e] + BC[c][e]);
                if constexpr (Q) v += g.sc * (Qc[c][e] - Qc[cm_][e]);
                acv[c][e] = ((!g.perc && c == 0) || C == 1) ? 0.f : v;
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const long long i = i0 + (long long)c * g.plane;
            const long long fi = f00 + (long long)c * g.plane;
            const V X0 = ld_ntv<NX>(s.Mx + i);
            const V Y0 = ld_v<NX>(s.My + i), Y1 = ld_v<NX>(s.My + i + dyp);
            const V T0 = ld_v<NX>(s.F + fi), T1 = ld_v<NX>(s.F + fi + sl);
            const V BXc = ld_ntv<NX>(s.bb[0] + i);
            const V BYm = ld_v<NX>(s.bb[1] + i + dym), BYc = ld_v<NX>(s.bb[1] + i);
            const V BYp = ld_v<NX>(s.bb[1] + i + dyp);
            const V BTm = ld_v<NX>(s.bb[3] + i + dtm), BTc = ld_v<NX>(s.bb[3] + i);
            const V BTp = ld_v<NX>(s.bb[3] + i + dtp);
            V Qym, Qyp, Qtm, Qtp;
            if constexpr (Q) {
                Qym = ld_v<NX>(s.Phi + i + dym); Qyp = ld_v<NX>(s.Phi + i + dyp);
                Qtm = ld_v<NX>(s.Phi + i + dtm); Qtp = ld_v<NX>(s.Phi + i + dtp);
            }
            // x neighbours beyond the lane's nodes
            const float x1n = lane_rot(X0[0], 1);
            const float bxm = lane_rot(BXc[NX - 1], -1), bxp = lane_rot(BXc[0], 1);
            const float qxm = Q ? lane_rot(Qc[c][NX - 1], -1) : 0.f;
            const float qxp = Q ? lane_rot(Qc[c][0], 1) : 0.f;
            const V ac1v = C == 1 ? V(0.f)
                                  : (c + 1 < C ? acv[(c + 1) % C] : (g.perc ? acv[0] : V(0.f)));
            V o0, o1, o3;
#pragma unroll
            for (int e = 0; e < NX; ++e) {
                const float x1 = e + 1 < NX ? X0[e + 1] : x1n;
                const float bm = e > 0 ? BXc[e - 1] : bxm, bp = e + 1 < NX ? BXc[e + 1] : bxp;
                float ax0 = X0[e] - ts * (bm + BXc[e]);
                float ax1 = x1 - ts * (BXc[e] + bp);
                float ay0 = Y0[e] - ts * (BYm[e] + BYc[e]);
                float ay1 = Y1[e] - ts * (BYc[e] + BYp[e]);
                float af0 = T0[e] - ts * (BTm[e] + BTc[e]);
                float af1 = T1[e] - ts * (BTc[e] + BTp[e]);
                if constexpr (Q) {           // + grad Phi on the unknown faces
                    const float qc = Qc[c][e];
                    const float qm = e > 0 ? Qc[c][e - 1] : qxm;
                    const float qp = e + 1 < NX ? Qc[c][e + 1] : qxp;
                    ax0 += g.sx * (qc - qm);
                    ax1 += g.sx * (qp - qc);
                    ay0 += g.sy * (qc - Qym[e]);
                    ay1 += g.sy * (Qyp[e] - qc);
                    af0 += g.st * (qc - Qtm[e]);
                    af1 += g.st * (Qtp[e] - qc);
                }
                ax0 = e == 0 && wx0 ? 0.f : ax0;
                ax1 = e + 1 == NX && wx1 ? 0.f : ax1;
                ay0 = wy0 ? 0.f : ay0;
                ay1 = wy1 ? 0.f : ay1;
                af0 = k0 ? T0[e] : af0;      // boundary slices are data
                af1 = k1 ? T1[e] : af1;
                const float ac1 = ac1v[e];
                rv[c][e] = g.sx * (ax1 - ax0) + g.sy * (ay1 - ay0) + g.sc * (ac1 - acv[c][e]) +
                           g.st * (af1 - af0);
                o0[e] = ax0; o1[e] = ay0; o3[e] = k0 ? 0.f : af0;
            }
            st_v<NX, NT>(s.A[0] + i, o0);
            st_v<NX, NT>(s.A[1] + i, o1);
            st_v<NX, NT>(s.A[2] + i, acv[c]);
            st_v<NX, NT>(s.A[3] + i, o3);
        }
    } else {
        // colour faces first: own face c of every colour
        V W[C], acv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) W[c] = ld_v<NX>(s.R + i0 + (long long)c * g.plane);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int cm_ = c == 0 ? C - 1 : c - 1;
            const V A2 = ld_v<NX>(s.A[2] + i0 + (long long)c * g.plane);
#pragma unroll
            for (int e = 0; e < NX; ++e) {
                const float v = A2[e] + g.sc * (W[c][e] - W[cm_][e]);
                acv[c][e] = ((!g.perc && c == 0) || C == 1) ? 0.f : v;
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const long long i = i0 + (long long)c * g.plane;
            const long long fi = f00 + (long long)c * g.plane;
            const V A0 = ld_v<NX>(s.A[0] + i);
            const V A1c = ld_v<NX>(s.A[1] + i), A1p = ld_v<NX>(s.A[1] + i + dyp);
            const V T0 = k0 ? ld_v<NX>(s.F + fi) : ld_v<NX>(s.A[3] + i);
            const V T1 = k1 ? ld_v<NX>(s.F + fi + sl) : ld_v<NX>(s.A[3] + i + sl);
            const V Rym = ld_v<NX>(s.R + i + dym), Ryp = ld_v<NX>(s.R + i + dyp);
            const V Rtm = ld_v<NX>(s.R + i + dtm), Rtp = ld_v<NX>(s.R + i + dtp);
            const float rxm = lane_rot(W[c][NX - 1], -1), rxp = lane_rot(W[c][0], 1);
            const float a0p = lane_rot(A0[0], 1);
            const V ac1v = C == 1 ? V(0.f)
                                  : (c + 1 < C ? acv[(c + 1) % C] : (g.perc ? acv[0] : V(0.f)));
#pragma unroll
            for (int e = 0; e < NX; ++e) {
                const float pc = W[c][e];
                const float rm = e > 0 ? W[c][e - 1] : rxm, rp = e + 1 < NX ? W[c][e + 1] : rxp;
                const float a0n = e + 1 < NX ? A0[e + 1] : a0p;
                const float ax0 = e == 0 && wx0 ? 0.f : A0[e] + g.sx * (pc - rm);
                const float ax1 = e + 1 == NX && wx1 ? 0.f : a0n + g.sx * (rp - pc);
                const float ay0 = wy0 ? 0.f : A1c[e] + g.sy * (pc - Rym[e]);
                const float ay1 = wy1 ? 0.f : A1p[e] + g.sy * (Ryp[e] - pc);
                const float af0 = k0 ? T0[e] : T0[e] + g.st * (pc - Rtm[e]);
                const float af1 = k1 ? T1[e] : T1[e] + g.st * (Rtp[e] - pc);
                const float ac1 = ac1v[e];
                rv[c][e] = g.sx * (ax1 - ax0) + g.sy * (ay1 - ay0) + g.sc * (ac1 - acv[c][e]) +
                           g.st * (af1 - af0);
            }
        }
    }
    float* const out = MODE == 1 ? s.R2 : s.R;
    if (mix) {
#pragma unroll
        for (int jc = 0; jc < C; ++jc) {
            V acc;
#pragma unroll
            for (int e = 0; e < NX; ++e) {
                float a = 0.f;
#pragma unroll
                for (int c = 0; c < C; ++c) a = fmaf(cm[c * C + jc], rv[c][e], a);
                acc[e] = a;
            }
            *reinterpret_cast<V*>(out + i0 + (long long)jc * g.plane) = acc;
        }
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c) *reinterpret_cast<V*>(out + i0 + (long long)c * g.plane) = rv[c];
    }
    double sums[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        double t = 0.0;
#pragma unroll
        for (int e = 0; e < NX; ++e) t += (double)rv[c][e];
        sums[c] = t;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int c = 0; c < C; ++c) sums[c] += __shfl_down(sums[c], o, 64);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < C; ++c)
            s.part_slice[(((long long)b * g.P + k) * C + c) * s.nbx + y] = sums[c];
}

// x = a + grad phi_1 (+ grad phi_2 when NPHI is 2 or 4), z = prox(K x + c +
// b), b and b_bar updates, for all colours of a node; residual partials when
// CHECK.  NPHI 3 and 4 (carried potential) also add the potentials into Phi
// at the own node.
// FP64 residual sums of a check iteration (the RedSlot quantities).
struct ResidSums {
    double db2 = 0, z2 = 0, dx2 = 0, x2 = 0, jj = 0;
};

// Steps 2 and 3 of Algorithm 1 at one node, given the new x on the node's
// lower and upper faces (mx0/mx1, my0/my1, mc0/mc1, f0/f1) and the dual bo:
// z = prox of J at K x + c + bo, the new dual bn = K x + c + bo - z and its
// extrapolation bbn = bn + theta (bn - bo).  With CHECK the residual sums take
// the node's terms, o holding the old x on the lower faces (f at k = 0, the
// boundary slice, counts as 0).
template <bool CHECK>
__device__ __forceinline__ void node_dual(float mx0, float mx1, float my0, float my1, float mc0,
                                          float mc1, float f0, float f1, bool k0,
                                          const float (&bo)[4], const float (&o)[4], float sigma,
                                          float th, int prox, float (&bn)[4], float (&bbn)[4],
                                          ResidSums& rs) {
    // K x + c at the node, plus b
    const float bx = bo[0], by = bo[1], bc = bo[2], bf = bo[3];
    const float amx = 0.5f * (mx0 + mx1) + bx, amy = 0.5f * (my0 + my1) + by;
    const float amc = 0.5f * (mc0 + mc1) + bc, amf = 0.5f * (f0 + f1) + bf;
    float ux, uy, uc, vv;
    prox_J(amx, amy, amc, amf, sigma, ux, uy, uc, vv, prox);
    bn[0] = amx - ux; bn[1] = amy - uy; bn[2] = amc - uc; bn[3] = amf - vv;
#pragma unroll
    for (int q = 0; q < 4; ++q) bbn[q] = bn[q] + th * (bn[q] - bo[q]);
    if constexpr (CHECK) {
        const float nf = k0 ? 0.f : f0;
        const double ddx = (double)mx0 - o[0], ddy = (double)my0 - o[1];
        const double ddc = (double)mc0 - o[2], ddf = (double)nf - o[3];
        rs.dx2 += ddx * ddx + ddy * ddy + ddc * ddc + ddf * ddf;
        rs.x2 += (double)mx0 * mx0 + (double)my0 * my0 + (double)mc0 * mc0 + (double)nf * nf;
        const double ex = (double)bn[0] - bx, ey = (double)bn[1] - by;
        const double ec = (double)bn[2] - bc, ef = (double)bn[3] - bf;
        rs.db2 += ex * ex + ey * ey + ec * ec + ef * ef;
        const double u2 = (double)ux * ux + (double)uy * uy + (double)uc * uc;
        rs.z2 += u2 + (double)vv * vv;
        rs.jj += vv > 0.f ? u2 / (2.0 * vv) : 0.0;
    }
}

template <int CHECK, int NPHI_, int C, bool NT>
__global__ void __launch_bounds__(256) k_update_rows(StepArgs s, int nxb) {
    constexpr int NPHI = NPHI_ == 4 ? 2 : (NPHI_ == 3 ? 1 : NPHI_);
    constexpr bool CARRY = NPHI_ >= 3;
    constexpr bool TWO = NPHI == 2;
    const Geom& g = s.g;
    const RowCtx r = row_ctx(g, nxb);
    if (s.frz_run && s.frz_run[r.b] != 0.f) return;   // frozen problem (block-uniform)
    ResidSums rs;
    if (r.live) {
        const Nbr nb = neighbours(g, r.x, r.y);
        const long long sl = g.slice;
        const bool k0 = r.k == 0, k1 = r.k + 1 == g.P;
        const long long dtm = k0 ? 0 : -sl, dtp = k1 ? 0 : sl;   // clamped time steps
        // Loads of all colours first (the stores below may alias them as far
        // as the compiler knows).  Time faces read the boundary slice of F
        // at k = 0 and k = P, else the work array a.
        float A0c[C], A0p[C], A1c[C], A1p[C], A2c[C], T0[C], T1[C];
        float Rc[C], Rxm[C], Rxp[C], Rym[C], Ryp[C], Rtm[C], Rtp[C];
        float Sc[C], Sxm[C], Sxp[C], Sym[C], Syp[C], Stm[C], Stp[C];   // phi_2
        float B0[C], B1[C], B2[C], B3[C], Qc[C], O0[C], O1[C], O2[C], O3[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const long long i = r.i0 + (long long)c * g.plane;
            const long long fi = r.f0 + (long long)c * g.plane;
            A0c[c] = s.A[0][i]; A0p[c] = s.A[0][i + nb.dxp];
            A1c[c] = s.A[1][i]; A1p[c] = s.A[1][i + nb.dyp];
            A2c[c] = s.A[2][i];
            T0[c] = k0 ? s.F[fi] : s.A[3][i];
            T1[c] = k1 ? s.F[fi + sl] : s.A[3][i + sl];
            const float* R = s.R;
            Rc[c] = R[i];
            Rxm[c] = R[i + nb.dxm]; Rxp[c] = R[i + nb.dxp];
            Rym[c] = R[i + nb.dym]; Ryp[c] = R[i + nb.dyp];
            Rtm[c] = R[i + dtm]; Rtp[c] = R[i + dtp];
            if constexpr (TWO) {
                const float* R2 = s.R2;
                Sc[c] = R2[i];
                Sxm[c] = R2[i + nb.dxm]; Sxp[c] = R2[i + nb.dxp];
                Sym[c] = R2[i + nb.dym]; Syp[c] = R2[i + nb.dyp];
                Stm[c] = R2[i + dtm]; Stp[c] = R2[i + dtp];
            }
            B0[c] = s.b[0][i]; B1[c] = s.b[1][i]; B2[c] = s.b[2][i]; B3[c] = s.b[3][i];
            if constexpr (CARRY) Qc[c] = s.Phi[i];
            if constexpr (CHECK) {
                O0[c] = s.Mx[i]; O1[c] = s.My[i]; O2[c] = s.Mc[i];
                O3[c] = k0 ? 0.f : s.F[fi];
            }
        }
        // grad of the potential(s) between a cell pair (lo, hi): phi_2 (the
        // refinement) is much smaller than phi_1, so difference the two
        // separately and keep its low-order bits
        auto dphi = [&](float hi, float lo, float hi2, float lo2) -> float {
            return TWO ? (hi - lo) + (hi2 - lo2) : hi - lo;
        };
        float mcv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int cm = c == 0 ? C - 1 : c - 1;
            const float v = A2c[c] + g.sc * dphi(Rc[c], Rc[cm], TWO ? Sc[c] : 0.f, TWO ? Sc[cm] : 0.f);
            mcv[c] = ((!g.perc && c == 0) || C == 1) ? 0.f : v;
        }
        const float th = s.theta;
        const float sigma = s.sig[r.b];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const long long i = r.i0 + (long long)c * g.plane;
            const long long fi = r.f0 + (long long)c * g.plane;
            const float s0 = TWO ? Sc[c] : 0.f;
            const float mx0 = nb.wx0 ? 0.f : A0c[c] + g.sx * dphi(Rc[c], Rxm[c], s0, TWO ? Sxm[c] : 0.f);
            const float mx1 = nb.wx1 ? 0.f : A0p[c] + g.sx * dphi(Rxp[c], Rc[c], TWO ? Sxp[c] : 0.f, s0);
            const float my0 = nb.wy0 ? 0.f : A1c[c] + g.sy * dphi(Rc[c], Rym[c], s0, TWO ? Sym[c] : 0.f);
            const float my1 = nb.wy1 ? 0.f : A1p[c] + g.sy * dphi(Ryp[c], Rc[c], TWO ? Syp[c] : 0.f, s0);
            const float f0 = k0 ? T0[c] : T0[c] + g.st * dphi(Rc[c], Rtm[c], s0, TWO ? Stm[c] : 0.f);
            const float f1 = k1 ? T1[c] : T1[c] + g.st * dphi(Rtp[c], Rc[c], TWO ? Stp[c] : 0.f, s0);
            const float mc0 = mcv[c];
            const float mc1 = C == 1 ? 0.f
                              : (c + 1 < C ? mcv[(c + 1) % C] : (g.perc ? mcv[0] : 0.f));
            const float bo[4] = {B0[c], B1[c], B2[c], B3[c]};
            const float o[4] = {CHECK ? O0[c] : 0.f, CHECK ? O1[c] : 0.f,
                                CHECK ? O2[c] : 0.f, CHECK ? O3[c] : 0.f};
            float bn[4], bbn[4];
            node_dual<CHECK != 0>(mx0, mx1, my0, my1, mc0, mc1, f0, f1, k0, bo, o, sigma, th,
                                  s.prox, bn, bbn, rs);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                st_f<NT>(s.b[q] + i, bn[q]);
                st_f<NT>(s.bb[q] + i, bbn[q]);
            }
            st_f<NT>(s.Mx + i, mx0);
            st_f<NT>(s.My + i, my0);
            st_f<NT>(s.Mc + i, mc0);
            if (!k0) st_f<NT>(s.F + fi, f0);
            if (CARRY) st_f<NT>(s.Phi + i, Qc[c] + (TWO ? Rc[c] + Sc[c] : Rc[c]));
        }
    }
    if (CHECK) {
        double vals[RS_COUNT] = {rs.db2, rs.z2, rs.dx2, rs.x2, rs.jj};
        block_sums(vals);
        if (threadIdx.x == 0)
            for (int q = 0; q < RS_COUNT; ++q) s.part_red[q * (long long)gridDim.x + r.L] = vals[q];
    }
}

// k_update_rows for rows of X = 64 NX nodes (128 or 256): a wavefront owns a
// row (b, k, y), lane l the NX nodes from x = NX l, and every field access
// is an NX-wide vector (one 16-byte access per lane for NX = 4 instead of
// four 4-byte ones).  The x neighbours in the adjacent lanes come by a lane
// rotation, which wraps at the row ends as the periodic x axis does (a
// Neumann wall zeroes the face there).  Same arithmetic per node as
// k_update_rows (node_dual, the same expressions).  Iterations without a residual check only: with the FP64 sums the
// kernel would need more than 256 VGPRs, and a check iteration runs
// k_update_rows, whose partials with one block per row are per row.
template <int NPHI_, int C, bool NT, int NX>
__global__ void __launch_bounds__(256) k_update_vec(StepArgs s) {
    constexpr int NPHI = NPHI_ == 4 ? 2 : (NPHI_ == 3 ? 1 : NPHI_);
    constexpr bool CARRY = NPHI_ >= 3;
    constexpr bool TWO = NPHI == 2;
    using V = fvec<NX>;
    const Geom& g = s.g;
    const long long nrows = (long long)g.B * g.Y * g.P;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const long long row = xcd_remap(blockIdx.x, gridDim.x) * (long long)(blockDim.x >> 6) + w;
    if (row >= nrows) return;
    const int k = (int)(row % g.P), y = (int)((row / g.P) % g.Y), b = (int)(row / ((long long)g.P * g.Y));
    if (s.frz_run && s.frz_run[b] != 0.f) return;   // frozen problem (wave-uniform)
    const int lane = (int)(threadIdx.x & 63);
    const long long p = (long long)y * g.X + (long long)lane * NX;
    const long long i0 = (long long)b * g.nc + (long long)k * g.slice + p;
    const long long f00 = (long long)b * g.nf + (long long)k * g.slice + p;
    const long long sl = g.slice;
    const bool k0 = k == 0, k1 = k + 1 == g.P;
    const long long dtm = k0 ? 0 : -sl, dtp = k1 ? 0 : sl;   // clamped time steps
    const long long dym = y == 0 ? (long long)(g.Y - 1) * g.X : -(long long)g.X;
    const long long dyp = y + 1 == g.Y ? -(long long)(g.Y - 1) * g.X : (long long)g.X;
    const bool wy0 = !g.pery && y == 0, wy1 = !g.pery && y + 1 == g.Y;
    const bool wx0 = !g.perx && lane == 0, wx1 = !g.perx && lane == 63;   // row ends
    auto dphi = [&](float hi, float lo, float hi2, float lo2) -> float {
        return TWO ? (hi - lo) + (hi2 - lo2) : hi - lo;
    };
    // r (and phi_2) at the node for every colour, and the colour faces of x
    V Rc[C], Sc[C], mcv[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        Rc[c] = ld_v<NX>(s.R + i0 + (long long)c * g.plane);
        if constexpr (TWO) Sc[c] = ld_v<NX>(s.R2 + i0 + (long long)c * g.plane);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int cm = c == 0 ? C - 1 : c - 1;
        const V a2 = ld_v<NX>(s.A[2] + i0 + (long long)c * g.plane);
#pragma unroll
        for (int e = 0; e < NX; ++e) {
            const float v = a2[e] + g.sc * dphi(Rc[c][e], Rc[cm][e], TWO ? Sc[c][e] : 0.f,
                                                TWO ? Sc[cm][e] : 0.f);
            mcv[c][e] = ((!g.perc && c == 0) || C == 1) ? 0.f : v;
        }
    }
    const float th = s.theta;
    const float sigma = s.sig[b];
    ResidSums rs;   // unused: check iterations run k_update_rows
    // One colour at a time: its loads, then its stores (which the compiler
    // must keep ahead of the next colour's loads), so a wavefront holds one
    // colour's vectors.
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const long long i = i0 + (long long)c * g.plane;
        const long long fi = f00 + (long long)c * g.plane;
        const V A0c = ld_v<NX>(s.A[0] + i);
        const V A1c = ld_v<NX>(s.A[1] + i), A1p = ld_v<NX>(s.A[1] + i + dyp);
        const V T0 = k0 ? ld_v<NX>(s.F + fi) : ld_v<NX>(s.A[3] + i);
        const V T1 = k1 ? ld_v<NX>(s.F + fi + sl) : ld_v<NX>(s.A[3] + i + sl);
        const V Rym = ld_v<NX>(s.R + i + dym), Ryp = ld_v<NX>(s.R + i + dyp);
        const V Rtm = ld_v<NX>(s.R + i + dtm), Rtp = ld_v<NX>(s.R + i + dtp);
        V Sym, Syp, Stm, Stp, Qc;
        if constexpr (TWO) {
            Sym = ld_v<NX>(s.R2 + i + dym); Syp = ld_v<NX>(s.R2 + i + dyp);
            Stm = ld_v<NX>(s.R2 + i + dtm); Stp = ld_v<NX>(s.R2 + i + dtp);
        }
        const V B0 = ld_v<NX>(s.b[0] + i), B1 = ld_v<NX>(s.b[1] + i);
        const V B2 = ld_v<NX>(s.b[2] + i), B3 = ld_v<NX>(s.b[3] + i);
        if constexpr (CARRY) Qc = ld_v<NX>(s.Phi + i);
        // x neighbours beyond the lane's nodes
        const float rxm = lane_rot(Rc[c][NX - 1], -1), rxp = lane_rot(Rc[c][0], 1);
        const float a0p = lane_rot(A0c[0], 1);
        const float sxm = TWO ? lane_rot(Sc[c][NX - 1], -1) : 0.f;
        const float sxp = TWO ? lane_rot(Sc[c][0], 1) : 0.f;
        const V mc1v = C == 1 ? V(0.f)
                              : (c + 1 < C ? mcv[(c + 1) % C] : (g.perc ? mcv[0] : V(0.f)));
        V nb[4], nbb[4], vmx, vmy, vmc, vf, vq;
#pragma unroll
        for (int e = 0; e < NX; ++e) {
            const float rc = Rc[c][e];
            const float rm = e > 0 ? Rc[c][e - 1] : rxm, rp = e + 1 < NX ? Rc[c][e + 1] : rxp;
            const float s0 = TWO ? Sc[c][e] : 0.f;
            const float sm = TWO ? (e > 0 ? Sc[c][e - 1] : sxm) : 0.f;
            const float sp = TWO ? (e + 1 < NX ? Sc[c][e + 1] : sxp) : 0.f;
            const float a0n = e + 1 < NX ? A0c[e + 1] : a0p;
            const bool w0 = e == 0 && wx0, w1 = e + 1 == NX && wx1;
            const float mx0 = w0 ? 0.f : A0c[e] + g.sx * dphi(rc, rm, s0, sm);
            const float mx1 = w1 ? 0.f : a0n + g.sx * dphi(rp, rc, sp, s0);
            const float my0 = wy0 ? 0.f : A1c[e] + g.sy * dphi(rc, Rym[e], s0, TWO ? Sym[e] : 0.f);
            const float my1 = wy1 ? 0.f : A1p[e] + g.sy * dphi(Ryp[e], rc, TWO ? Syp[e] : 0.f, s0);
            const float f0 = k0 ? T0[e] : T0[e] + g.st * dphi(rc, Rtm[e], s0, TWO ? Stm[e] : 0.f);
            const float f1 = k1 ? T1[e] : T1[e] + g.st * dphi(Rtp[e], rc, TWO ? Stp[e] : 0.f, s0);
            const float mc0 = mcv[c][e], mc1 = mc1v[e];
            const float bo[4] = {B0[e], B1[e], B2[e], B3[e]};
            const float o[4] = {0.f, 0.f, 0.f, 0.f};
            float bn[4], bbn[4];
            node_dual<false>(mx0, mx1, my0, my1, mc0, mc1, f0, f1, k0, bo, o, sigma, th, s.prox,
                             bn, bbn, rs);
#pragma unroll
            for (int q = 0; q < 4; ++q) { nb[q][e] = bn[q]; nbb[q][e] = bbn[q]; }
            vmx[e] = mx0; vmy[e] = my0; vmc[e] = mc0; vf[e] = f0;
            if constexpr (CARRY) vq[e] = Qc[e] + (TWO ? rc + s0 : rc);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            st_v<NX, NT>(s.b[q] + i, nb[q]);
            st_v<NX, NT>(s.bb[q] + i, nbb[q]);
        }
        st_v<NX, NT>(s.Mx + i, vmx);
        st_v<NX, NT>(s.My + i, vmy);
        st_v<NX, NT>(s.Mc + i, vmc);
        if (!k0) st_v<NX, NT>(s.F + fi, vf);
        if constexpr (CARRY) st_v<NX, NT>(s.Phi + i, vq);
    }
}

int row_block(int X) {
    int b = ((X + 63) / 64) * 64;
    return b > 256 ? 256 : b;
}

bool rows_ok(const Geom& g) { return g.C >= 1 && g.C <= 4; }

static dim3 row_grid(const Geom& g, int nxb) {
    return dim3((unsigned)((long long)g.B * g.Y * g.P * nxb));
}

// The vector kernels apply when a row is one wavefront of NX-node vectors
// (X = 128 or 256 with one block per row, so that the plane and residual
// partials keep the per-row layout) and every field is aligned to the
// vector (a null field counts as aligned).  Returns NX, or 0.
static int row_vec_nx(const StepArgs& s) {
    const Geom& g = s.g;
    const int bx = s.row_bx > 0 ? s.row_bx : row_block(g.X);
    if (bx != g.X || (g.X != 128 && g.X != 256)) return 0;
    const int nx = g.X / 64;
    const uintptr_t m = (uintptr_t)(4 * nx) - 1;
    uintptr_t any = (uintptr_t)s.F | (uintptr_t)s.Mx | (uintptr_t)s.My | (uintptr_t)s.Mc |
                    (uintptr_t)s.R | (uintptr_t)s.R2 | (uintptr_t)s.Phi;
    for (int q = 0; q < 4; ++q) any |= (uintptr_t)s.b[q] | (uintptr_t)s.bb[q] | (uintptr_t)s.A[q];
    return (any & m) == 0 ? nx : 0;
}

// Grid of the vector kernels: one row (wavefront) per block.  Blocks of 2
// and 4 rows (consecutive times) measured slower at 256 x 256 x 3 x 32
// (0.2422 and 0.2410 against 0.2403 ms per iteration); the kernels take any
// multiple of 64 threads.
static void vec_grid(const Geom& g, dim3& gr, dim3& bl) {
    gr = dim3((unsigned)((long long)g.B * g.Y * g.P));
    bl = dim3(64);
}

template <int C, bool NT, int NX>
static void div_vec_n(const StepArgs& s, int mode, hipStream_t st) {
    dim3 gr, bl;
    vec_grid(s.g, gr, bl);
    if (mode == 0) hipLaunchKernelGGL((k_div_vec<0, C, NT, NX>), gr, bl, 0, st, s);
    else if (mode == 1) hipLaunchKernelGGL((k_div_vec<1, C, NT, NX>), gr, bl, 0, st, s);
    else hipLaunchKernelGGL((k_div_vec<2, C, NT, NX>), gr, bl, 0, st, s);
}

template <int C>
static void div_vec_c(const StepArgs& s, int mode, int nx, hipStream_t st) {
    if (s.nt_store) {
        if (nx == 4) div_vec_n<C, true, 4>(s, mode, st);
        else div_vec_n<C, true, 2>(s, mode, st);
    } else {
        if (nx == 4) div_vec_n<C, false, 4>(s, mode, st);
        else div_vec_n<C, false, 2>(s, mode, st);
    }
}

template <int C, int XL, int XK>
static void div_rows_x(const StepArgs& s, int mode, int nxb, int bx, hipStream_t st) {
    const dim3 gr = row_grid(s.g, nxb), bl(bx);
    if (s.nt_store) {
        if (mode == 0) hipLaunchKernelGGL((k_div_rows<0, C, XL, XK, true>), gr, bl, 0, st, s, nxb);
        else if (mode == 1) hipLaunchKernelGGL((k_div_rows<1, C, XL, XK, true>), gr, bl, 0, st, s, nxb);
        else hipLaunchKernelGGL((k_div_rows<2, C, XL, XK, true>), gr, bl, 0, st, s, nxb);
    } else {
        if (mode == 0) hipLaunchKernelGGL((k_div_rows<0, C, XL, XK, false>), gr, bl, 0, st, s, nxb);
        else if (mode == 1) hipLaunchKernelGGL((k_div_rows<1, C, XL, XK, false>), gr, bl, 0, st, s, nxb);
        else hipLaunchKernelGGL((k_div_rows<2, C, XL, XK, false>), gr, bl, 0, st, s, nxb);
    }
}

template <int C, int XL>
static void div_rows_k(const StepArgs& s, int mode, int nxb, int bx, hipStream_t st) {
    if (s.xkind == 0) div_rows_x<C, XL, 0>(s, mode, nxb, bx, st);
    else div_rows_x<C, XL, 2>(s, mode, nxb, bx, st);
}

template <int C>
static void div_rows_c(const StepArgs& s, int mode, hipStream_t st) {
    const int bx = s.row_bx > 0 ? s.row_bx : row_block(s.g.X), nxb = (s.g.X + bx - 1) / bx;
    if (!s.twx) {
        const int nx = row_vec_nx(s);
        if (nx) div_vec_c<C>(s, mode, nx, st);
        else div_rows_x<C, 0, 0>(s, mode, nxb, bx, st);
        return;
    }
    switch (s.g.X) {     // div_fold_ok: X == bx in {64, 128, 256}
        case 64: div_rows_k<C, 64>(s, mode, nxb, bx, st); break;
        case 128: div_rows_k<C, 128>(s, mode, nxb, bx, st); break;
        default: div_rows_k<C, 256>(s, mode, nxb, bx, st); break;
    }
}

bool div_fold_ok(const Geom& g, int row_bx, const AxisTab& tx) {
    const int bx = row_bx > 0 ? row_bx : row_block(g.X);
    return rows_ok(g) && tx.tw != nullptr && bx == g.X && (g.X == 64 || g.X == 128 || g.X == 256);
}

template <int C, bool NT, int NX>
static void update_vec_n(const StepArgs& s, int nphi, hipStream_t st) {
    dim3 gr, bl;
    vec_grid(s.g, gr, bl);
    if (nphi == 2) hipLaunchKernelGGL((k_update_vec<2, C, NT, NX>), gr, bl, 0, st, s);
    else if (nphi == 3) hipLaunchKernelGGL((k_update_vec<3, C, NT, NX>), gr, bl, 0, st, s);
    else if (nphi == 4) hipLaunchKernelGGL((k_update_vec<4, C, NT, NX>), gr, bl, 0, st, s);
    else hipLaunchKernelGGL((k_update_vec<1, C, NT, NX>), gr, bl, 0, st, s);
}

template <int C, bool NT>
static void update_rows_n(const StepArgs& s, int check, int nphi, hipStream_t st) {
    const int nx = check ? 0 : row_vec_nx(s);
    if (nx == 4) { update_vec_n<C, NT, 4>(s, nphi, st); return; }
    if (nx == 2) { update_vec_n<C, NT, 2>(s, nphi, st); return; }
    const int bx = s.row_bx > 0 ? s.row_bx : row_block(s.g.X), nxb = (s.g.X + bx - 1) / bx;
    const dim3 gr = row_grid(s.g, nxb), bl(bx);
    if (nphi == 2) {
        if (check) hipLaunchKernelGGL((k_update_rows<1, 2, C, NT>), gr, bl, 0, st, s, nxb);
        else hipLaunchKernelGGL((k_update_rows<0, 2, C, NT>), gr, bl, 0, st, s, nxb);
    } else if (nphi == 3) {
        if (check) hipLaunchKernelGGL((k_update_rows<1, 3, C, NT>), gr, bl, 0, st, s, nxb);
        else hipLaunchKernelGGL((k_update_rows<0, 3, C, NT>), gr, bl, 0, st, s, nxb);
    } else if (nphi == 4) {
        if (check) hipLaunchKernelGGL((k_update_rows<1, 4, C, NT>), gr, bl, 0, st, s, nxb);
        else hipLaunchKernelGGL((k_update_rows<0, 4, C, NT>), gr, bl, 0, st, s, nxb);
    } else {
        if (check) hipLaunchKernelGGL((k_update_rows<1, 1, C, NT>), gr, bl, 0, st, s, nxb);
        else hipLaunchKernelGGL((k_update_rows<0, 1, C, NT>), gr, bl, 0, st, s, nxb);
    }
}

template <int C>
static void update_rows_c(const StepArgs& s, int check, int nphi, hipStream_t st) {
    if (s.nt_store) update_rows_n<C, true>(s, check, nphi, st);
    else update_rows_n<C, false>(s, check, nphi, st);
}

void launch_div_rows(const StepArgs& s, int mode, hipStream_t st) {
    switch (s.g.C) {
        case 1: div_rows_c<1>(s, mode, st); break;
        case 2: div_rows_c<2>(s, mode, st); break;
        case 3: div_rows_c<3>(s, mode, st); break;
        default: div_rows_c<4>(s, mode, st); break;
    }
}

void launch_update_rows(const StepArgs& s, int check, int nphi, hipStream_t st) {
    switch (s.g.C) {
        case 1: update_rows_c<1>(s, check, nphi, st); break;
        case 2: update_rows_c<2>(s, check, nphi, st); break;
        case 3: update_rows_c<3>(s, check, nphi, st); break;
        default: update_rows_c<4>(s, check, nphi, st); break;
    }
}

}  // namespace otd
