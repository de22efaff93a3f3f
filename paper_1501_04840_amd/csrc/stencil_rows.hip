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
#include "stencil_common.h"

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

// r = A a - f_b^- with a = x - tau sigma K^T b_bar (MODE 0: also writes a to A
// and r to R), a = A + grad phi_1 (MODE 1, refinement: writes r to R2) or
// a = x - tau sigma K^T b_bar + grad Phi with the carried potential Phi
// (MODE 2: writes a to A and r to R), and the FP64 plane sums of r (one
// partial per block and colour).
template <int MODE, int C>
__global__ void __launch_bounds__(256) k_div_rows(StepArgs s, int nxb) {
    const Geom& g = s.g;
    const RowCtx r = row_ctx(g, nxb);
    const float ts = 0.5f * s.tau_sigma;
    float rv[C];
#pragma unroll
    for (int c = 0; c < C; ++c) rv[c] = 0.f;
    if (r.live) {
        const Nbr nb = neighbours(g, r.x, r.y);
        const long long sl = g.slice;
        const bool k0 = r.k == 0, k1 = r.k + 1 == g.P;
        // colour faces first: own face c of every colour, into registers
        float acv[C];
        {
            float w[C], q[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const long long i = r.i0 + (long long)c * g.plane;
                w[c] = MODE == 1 ? s.R[i] : s.bb[2][i];
                q[c] = MODE == 2 ? s.Phi[i] : 0.f;
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int cm = c == 0 ? C - 1 : c - 1;
                const long long i = r.i0 + (long long)c * g.plane;
                const bool wall = !g.perc && c == 0;
                float v;
                if (MODE == 1) v = s.A[2][i] + g.sc * (w[c] - w[cm]);
                else v = s.Mc[i] - ts * (w[cm] + w[c]);
                if (MODE == 2) v += g.sc * (q[c] - q[cm]);
                acv[c] = (wall || C == 1) ? 0.f : v;
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const long long i = r.i0 + (long long)c * g.plane;
            const long long fi = r.f0 + (long long)c * g.plane;
            float ax0, ax1, ay0, ay1, af0, af1;
            if (MODE != 1) {
                const float* bx = s.bb[0];
                const float* by = s.bb[1];
                const float* bt = s.bb[3];
                const float bxc = bx[i], byc = by[i];
                ax0 = nb.wx0 ? 0.f : s.Mx[i] - ts * (bx[i + nb.dxm] + bxc);
                ax1 = nb.wx1 ? 0.f : s.Mx[i + nb.dxp] - ts * (bxc + bx[i + nb.dxp]);
                ay0 = nb.wy0 ? 0.f : s.My[i] - ts * (by[i + nb.dym] + byc);
                ay1 = nb.wy1 ? 0.f : s.My[i + nb.dyp] - ts * (byc + by[i + nb.dyp]);
                const float btc = bt[i];
                af0 = k0 ? s.F[fi] : s.F[fi] - ts * (bt[i - sl] + btc);
                af1 = k1 ? s.F[fi + sl] : s.F[fi + sl] - ts * (btc + bt[i + sl]);
                if (MODE == 2) {           // + grad Phi on the unknown faces
                    const float* Q = s.Phi;
                    const float qc = Q[i];
                    if (!nb.wx0) ax0 += g.sx * (qc - Q[i + nb.dxm]);
                    if (!nb.wx1) ax1 += g.sx * (Q[i + nb.dxp] - qc);
                    if (!nb.wy0) ay0 += g.sy * (qc - Q[i + nb.dym]);
                    if (!nb.wy1) ay1 += g.sy * (Q[i + nb.dyp] - qc);
                    if (!k0) af0 += g.st * (qc - Q[i - sl]);
                    if (!k1) af1 += g.st * (Q[i + sl] - qc);
                }
            } else {
                const float* R = s.R;
                const float pc = R[i];
                ax0 = nb.wx0 ? 0.f : s.A[0][i] + g.sx * (pc - R[i + nb.dxm]);
                ax1 = nb.wx1 ? 0.f : s.A[0][i + nb.dxp] + g.sx * (R[i + nb.dxp] - pc);
                ay0 = nb.wy0 ? 0.f : s.A[1][i] + g.sy * (pc - R[i + nb.dym]);
                ay1 = nb.wy1 ? 0.f : s.A[1][i + nb.dyp] + g.sy * (R[i + nb.dyp] - pc);
                af0 = k0 ? s.F[fi] : s.A[3][i] + g.st * (pc - R[i - sl]);
                af1 = k1 ? s.F[fi + sl] : s.A[3][i + sl] + g.st * (R[i + sl] - pc);
            }
            const float ac1 = C == 1 ? 0.f
                              : (c + 1 < C ? acv[(c + 1) % C] : (g.perc ? acv[0] : 0.f));
            const float rr = g.sx * (ax1 - ax0) + g.sy * (ay1 - ay0) + g.sc * (ac1 - acv[c]) +
                             g.st * (af1 - af0);
            if (MODE != 1) {
                s.A[0][i] = ax0;
                s.A[1][i] = ay0;
                s.A[2][i] = acv[c];
                s.A[3][i] = k0 ? 0.f : af0;
                s.R[i] = rr;
            } else {
                s.R2[i] = rr;
            }
            rv[c] = rr;
        }
    }
    const long long col = (long long)r.y * nxb + r.xb;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const double t = block_sum((double)rv[c]);
        if (threadIdx.x == 0)
            s.part_slice[(((long long)r.b * g.P + r.k) * C + c) * s.nbx + col] = t;
    }
}

// x = a + grad phi_1 (+ grad phi_2 when NPHI is 2 or 4), z = prox(K x + c +
// b), b and b_bar updates, for all colours of a node; residual partials when
// CHECK.  NPHI 3 and 4 (carried potential) also add the potentials into Phi
// at the own node.
template <int CHECK, int NPHI_, int C>
__global__ void __launch_bounds__(256) k_update_rows(StepArgs s, int nxb) {
    constexpr int NPHI = NPHI_ == 4 ? 2 : (NPHI_ == 3 ? 1 : NPHI_);
    constexpr bool CARRY = NPHI_ >= 3;
    const Geom& g = s.g;
    const RowCtx r = row_ctx(g, nxb);
    double db2 = 0, z2 = 0, dx2 = 0, x2 = 0, jj = 0;
    if (r.live) {
        const Nbr nb = neighbours(g, r.x, r.y);
        const long long sl = g.slice;
        const bool k0 = r.k == 0, k1 = r.k + 1 == g.P;
        // phi_2 (the refinement) is much smaller than phi_1: difference the
        // two separately so that its low-order bits survive
        float ph[C], ph2[C], mcv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            ph[c] = s.R[r.i0 + (long long)c * g.plane];
            ph2[c] = NPHI == 2 ? s.R2[r.i0 + (long long)c * g.plane] : 0.f;
        }
        // grad of the potential from the own node (value pair p1, p2) to j
        auto dfrom = [&](float p1, float p2, long long j) -> float {
            return NPHI == 2 ? (p1 - s.R[j]) + (p2 - s.R2[j]) : p1 - s.R[j];
        };
        auto dto = [&](long long j, float p1, float p2) -> float {
            return NPHI == 2 ? (s.R[j] - p1) + (s.R2[j] - p2) : s.R[j] - p1;
        };
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int cm = c == 0 ? C - 1 : c - 1;
            const bool wall = !g.perc && c == 0;
            const float d = NPHI == 2 ? (ph[c] - ph[cm]) + (ph2[c] - ph2[cm]) : ph[c] - ph[cm];
            const float v = s.A[2][r.i0 + (long long)c * g.plane] + g.sc * d;
            mcv[c] = (wall || C == 1) ? 0.f : v;
        }
        const float th = s.theta;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const long long i = r.i0 + (long long)c * g.plane;
            const long long fi = r.f0 + (long long)c * g.plane;
            const float pc = ph[c], pc2 = ph2[c];
            const float mx0 = nb.wx0 ? 0.f : s.A[0][i] + g.sx * dfrom(pc, pc2, i + nb.dxm);
            const float mx1 = nb.wx1 ? 0.f : s.A[0][i + nb.dxp] + g.sx * dto(i + nb.dxp, pc, pc2);
            const float my0 = nb.wy0 ? 0.f : s.A[1][i] + g.sy * dfrom(pc, pc2, i + nb.dym);
            const float my1 = nb.wy1 ? 0.f : s.A[1][i + nb.dyp] + g.sy * dto(i + nb.dyp, pc, pc2);
            const float f0 = k0 ? s.F[fi] : s.A[3][i] + g.st * dfrom(pc, pc2, i - sl);
            const float f1 = k1 ? s.F[fi + sl] : s.A[3][i + sl] + g.st * dto(i + sl, pc, pc2);
            const float mc0 = mcv[c];
            const float mc1 = C == 1 ? 0.f
                              : (c + 1 < C ? mcv[(c + 1) % C] : (g.perc ? mcv[0] : 0.f));
            // K x + c at the node, plus b
            const float bx = s.b[0][i], by = s.b[1][i], bc = s.b[2][i], bf = s.b[3][i];
            const float amx = 0.5f * (mx0 + mx1) + bx, amy = 0.5f * (my0 + my1) + by;
            const float amc = 0.5f * (mc0 + mc1) + bc, amf = 0.5f * (f0 + f1) + bf;
            float ux, uy, uc, vv;
            prox_J(amx, amy, amc, amf, s.sigma, ux, uy, uc, vv);
            const float nbx = amx - ux, nby = amy - uy, nbc = amc - uc, nbf = amf - vv;
            s.b[0][i] = nbx; s.bb[0][i] = nbx + th * (nbx - bx);
            s.b[1][i] = nby; s.bb[1][i] = nby + th * (nby - by);
            s.b[2][i] = nbc; s.bb[2][i] = nbc + th * (nbc - bc);
            s.b[3][i] = nbf; s.bb[3][i] = nbf + th * (nbf - bf);
            if (CHECK) {
                const float ox = s.Mx[i], oy = s.My[i], oc = s.Mc[i];
                const float of = k0 ? 0.f : s.F[fi];
                const float nf = k0 ? 0.f : f0;
                const double ddx = (double)mx0 - ox, ddy = (double)my0 - oy;
                const double ddc = (double)mc0 - oc, ddf = (double)nf - of;
                dx2 += ddx * ddx + ddy * ddy + ddc * ddc + ddf * ddf;
                x2 += (double)mx0 * mx0 + (double)my0 * my0 + (double)mc0 * mc0 + (double)nf * nf;
                const double ex = (double)nbx - bx, ey = (double)nby - by;
                const double ec = (double)nbc - bc, ef = (double)nbf - bf;
                db2 += ex * ex + ey * ey + ec * ec + ef * ef;
                const double u2 = (double)ux * ux + (double)uy * uy + (double)uc * uc;
                z2 += u2 + (double)vv * vv;
                jj += vv > 0.f ? u2 / (2.0 * vv) : 0.0;
            }
            s.Mx[i] = mx0;
            s.My[i] = my0;
            s.Mc[i] = mc0;
            if (!k0) s.F[fi] = f0;
            if (CARRY) s.Phi[i] = s.Phi[i] + (NPHI == 2 ? pc + pc2 : pc);
        }
    }
    if (CHECK) {
        const double vals[RS_COUNT] = {db2, z2, dx2, x2, jj};
        for (int q = 0; q < RS_COUNT; ++q) {
            const double t = block_sum(vals[q]);
            if (threadIdx.x == 0) s.part_red[q * (long long)gridDim.x + r.L] = t;
        }
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

template <int C>
static void div_rows_c(const StepArgs& s, int mode, hipStream_t st) {
    const int bx = s.row_bx > 0 ? s.row_bx : row_block(s.g.X), nxb = (s.g.X + bx - 1) / bx;
    if (mode == 0) hipLaunchKernelGGL((k_div_rows<0, C>), row_grid(s.g, nxb), dim3(bx), 0, st, s, nxb);
    else if (mode == 1) hipLaunchKernelGGL((k_div_rows<1, C>), row_grid(s.g, nxb), dim3(bx), 0, st, s, nxb);
    else hipLaunchKernelGGL((k_div_rows<2, C>), row_grid(s.g, nxb), dim3(bx), 0, st, s, nxb);
}

template <int C>
static void update_rows_c(const StepArgs& s, int check, int nphi, hipStream_t st) {
    const int bx = s.row_bx > 0 ? s.row_bx : row_block(s.g.X), nxb = (s.g.X + bx - 1) / bx;
    const dim3 gr = row_grid(s.g, nxb), bl(bx);
    if (nphi == 2) {
        if (check) hipLaunchKernelGGL((k_update_rows<1, 2, C>), gr, bl, 0, st, s, nxb);
        else hipLaunchKernelGGL((k_update_rows<0, 2, C>), gr, bl, 0, st, s, nxb);
    } else if (nphi == 3) {
        if (check) hipLaunchKernelGGL((k_update_rows<1, 3, C>), gr, bl, 0, st, s, nxb);
        else hipLaunchKernelGGL((k_update_rows<0, 3, C>), gr, bl, 0, st, s, nxb);
    } else if (nphi == 4) {
        if (check) hipLaunchKernelGGL((k_update_rows<1, 4, C>), gr, bl, 0, st, s, nxb);
        else hipLaunchKernelGGL((k_update_rows<0, 4, C>), gr, bl, 0, st, s, nxb);
    } else {
        if (check) hipLaunchKernelGGL((k_update_rows<1, 1, C>), gr, bl, 0, st, s, nxb);
        else hipLaunchKernelGGL((k_update_rows<0, 1, C>), gr, bl, 0, st, s, nxb);
    }
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
