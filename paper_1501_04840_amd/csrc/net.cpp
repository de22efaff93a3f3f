// Host side of the warm-start network: layer table, workspace carve, the
// forward and backward schedules and the C ABI of ot_net.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/ot_net.h"
#include "net_common.h"

using namespace otn;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
int pad8(int c) { return (c + 7) / 8 * 8; }

struct Layer {
    int taps, cin_o, cout_o, cin_p, cout_p;
    long long off_o;      // offset in the exchanged flat vector
    long long off_p;      // offset in the padded device vector (weights, then biases)
    long long off_w;      // offset of this layer's BF16 copies
    long long np() const { return (long long)taps * cin_p * cout_p + cout_p; }
    long long nw() const { return (long long)taps * cin_p * cout_p; }
};

// Layer list in execution order: encoder (2 per level), decoder (2 per level
// but the last), output layer.
std::vector<Layer> make_layers(const ot_net_desc& d) {
    std::vector<Layer> L;
    auto add = [&](int taps, int ci, int co) {
        Layer l{};
        l.taps = taps;
        l.cin_o = ci;
        l.cout_o = co;
        l.cin_p = pad8(ci);
        l.cout_p = pad8(co);
        L.push_back(l);
    };
    int c = d.in_ch;
    for (int l = 0; l < d.levels; ++l) {
        const int w = d.base << l;
        add(9, c, w);
        add(9, w, w);
        c = w;
    }
    for (int l = d.levels - 2; l >= 0; --l) {
        const int w = d.base << l;
        add(9, c + w, w);
        add(9, w, w);
        c = w;
    }
    add(1, c, d.out_ch);
    long long oo = 0, op = 0, ow = 0;
    for (auto& l : L) {
        l.off_o = oo;
        l.off_p = op;
        l.off_w = ow;
        oo += (long long)l.taps * l.cin_o * l.cout_o + l.cout_o;
        op += l.np();
        ow += l.nw();
    }
    return L;
}

int check_desc(const ot_net_desc* d) {
    if (!d) return OT_ERR_PARAM;
    if (d->levels < 1 || d->levels > 5 || d->base < 8 || d->base % 8 || d->in_ch < 1 ||
        d->out_ch < 1 || d->max_batch < 1 || d->H < 1 || d->W < 1)
        return OT_ERR_SHAPE;
    const int f = 1 << (d->levels - 1);
    if (d->H % f || d->W % f) return OT_ERR_SHAPE;
    if (!(d->beta1 >= 0 && d->beta1 < 1 && d->beta2 >= 0 && d->beta2 < 1 && d->eps > 0))
        return OT_ERR_PARAM;
    return OT_OK;
}

// Split of a weight-gradient GEMM over the pixels.
// `bound` is an upper bound of `splits` over every K up to the one given.
struct Split {
    int splits, ksplit, bound;
};
Split wgrad_split(int M, int N, int K) {
    const int bm = N <= 32 ? 128 : 64, bn = N <= 32 ? 32 : 64;
    const long long tiles = (long long)((M + bm - 1) / bm) * ((N + bn - 1) / bn);
    int s = (int)std::max(1LL, (1024 + tiles - 1) / tiles);
    s = std::min(s, std::max(1, K / 256));
    int ks = (K + s - 1) / s;
    ks = (ks + 31) / 32 * 32;
    return {(K + ks - 1) / ks, ks, s};
}

}  // namespace

struct ot_net {
    ot_net_desc d;
    hipStream_t st;
    std::vector<Layer> layers;
    long long np_o = 0, np_p = 0, nw = 0;
    // parameters and optimiser
    float *master = nullptr, *mom1 = nullptr, *mom2 = nullptr, *grad = nullptr;
    bf16_t *wf = nullptr, *wb = nullptr;
    int step = 0;
    // activations per level: a (first conv), cat (up | encoder output), bot
    // (encoder output at the bottom), pool (pooled input), da, db (decoder)
    std::vector<bf16_t*> a, cat, pool, da, db;
    bf16_t* bot = nullptr;
    bf16_t* x8 = nullptr;
    float* y = nullptr;
    bf16_t* dy = nullptr;
    // gradients per level
    std::vector<bf16_t*> gcat, gz1, gz2, gpool;
    float* part = nullptr;
    long long part_cap = 0;
    double* lpart = nullptr;
    double* lsum = nullptr;
    int lblocks = 0;
    std::string err;
};

namespace {

// Workspace layout; with n == nullptr only the size is computed.
size_t carve(const ot_net_desc& d, ot_net* n, char* base) {
    const auto layers = make_layers(d);
    long long np = 0, nw = 0;
    for (auto& l : layers) {
        np += l.np();
        nw += l.nw();
    }
    size_t o = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + o : nullptr;
        o = align_up(o + bytes);
        return p;
    };
    const long long B = d.max_batch;
    const int L = d.levels;
    float* master = (float*)take(np * 4);
    float* m1 = (float*)take(np * 4);
    float* m2 = (float*)take(np * 4);
    float* gr = (float*)take(np * 4);
    bf16_t* wf = (bf16_t*)take(nw * 2);
    bf16_t* wb = (bf16_t*)take(nw * 2);
    std::vector<bf16_t*> a(L), cat(L), pool(L), da(L), db(L), gcat(L), gz1(L), gz2(L), gpool(L);
    bf16_t* bot = nullptr;
    const int cin0 = pad8(d.in_ch), coutp = pad8(d.out_ch);
    for (int l = 0; l < L; ++l) {
        const long long P = B * (d.H >> l) * (d.W >> l);
        const int w = d.base << l, up = l + 1 < L ? d.base << (l + 1) : 0;
        a[l] = (bf16_t*)take(P * w * 2);
        if (l + 1 < L) {
            cat[l] = (bf16_t*)take(P * (up + w) * 2);
            gcat[l] = (bf16_t*)take(P * (up + w) * 2);
            da[l] = (bf16_t*)take(P * w * 2);
            db[l] = (bf16_t*)take(P * w * 2);
        } else {
            bot = (bf16_t*)take(P * w * 2);
        }
        if (l > 0) {
            pool[l] = (bf16_t*)take(P * (d.base << (l - 1)) * 2);
            gpool[l] = (bf16_t*)take(P * (d.base << (l - 1)) * 2);
        }
        gz1[l] = (bf16_t*)take(P * w * 2);
        gz2[l] = (bf16_t*)take(P * w * 2);
    }
    const long long P0 = B * d.H * d.W;
    bf16_t* x8 = (bf16_t*)take(P0 * cin0 * 2);
    float* y = (float*)take(P0 * d.out_ch * 4);
    bf16_t* dy = (bf16_t*)take(P0 * coutp * 2);
    // split-K partials: the largest weight-gradient GEMM at the full batch
    long long cap = 0;
    for (size_t i = 0; i < layers.size(); ++i) {
        const Layer& ly = layers[i];
        int lev;
        if (i < (size_t)2 * L) lev = (int)i / 2;
        else if (i + 1 < layers.size()) lev = L - 2 - (int)(i - 2 * L) / 2;
        else lev = 0;
        const int K = (int)(B * (d.H >> lev) * (d.W >> lev));
        const int M = ly.taps * ly.cin_p + 1;
        const Split s = wgrad_split(M, ly.cout_p, K);
        cap = std::max(cap, (long long)s.bound * M * ly.cout_p);
    }
    float* part = (float*)take(cap * 4);
    const int lb = loss_blocks(P0 * coutp);
    double* lpart = (double*)take((size_t)lb * 8);
    double* lsum = (double*)take(8);
    if (n) {
        n->layers = layers;
        n->np_p = np;
        n->nw = nw;
        n->master = master;
        n->mom1 = m1;
        n->mom2 = m2;
        n->grad = gr;
        n->wf = wf;
        n->wb = wb;
        n->a = a;
        n->cat = cat;
        n->pool = pool;
        n->da = da;
        n->db = db;
        n->bot = bot;
        n->gcat = gcat;
        n->gz1 = gz1;
        n->gz2 = gz2;
        n->gpool = gpool;
        n->x8 = x8;
        n->y = y;
        n->dy = dy;
        n->part = part;
        n->part_cap = cap;
        n->lpart = lpart;
        n->lsum = lsum;
        n->lblocks = lb;
    }
    return o;
}

int hipfail(ot_net* n, hipError_t e, const char* what) {
    n->err = std::string(what) + ": " + hipGetErrorString(e);
    return OT_ERR_HIP;
}

int enc(const ot_net* n, int l, int s) { (void)n; return 2 * l + s; }
int dec(const ot_net* n, int l, int s) { return 2 * n->d.levels + 2 * (n->d.levels - 2 - l) + s; }
int head(const ot_net* n) { return 2 * n->d.levels + 2 * (n->d.levels - 1); }

const float* bias_of(const ot_net* n, const Layer& l) { return n->master + l.off_p + l.nw(); }

// out = conv(src) with the layer's weights; epi EPI_RELU (BF16 out) or
// EPI_F32 (FP32 out, no activation).
void conv_fwd(ot_net* n, int li, int nb, int lev, View src, void* dst, int dst_ld, int dst_off,
              int dst_n, int epi) {
    const Layer& l = n->layers[li];
    ConvArgs a{};
    a.src = src.ptr;
    a.src_ld = src.ld;
    a.cin = l.cin_p;
    a.taps = l.taps;
    a.wmat = n->wf + l.off_w;
    a.nb = nb;
    a.H = n->d.H >> lev;
    a.W = n->d.W >> lev;
    a.M = nb * a.H * a.W;
    a.N = l.cout_p;
    a.K = l.taps * l.cin_p;
    a.dst = dst;
    a.dst_ld = dst_ld;
    a.dst_off = dst_off;
    a.dst_n = dst_n;
    a.bias = bias_of(n, l);
    launch_conv(a, MODE_CONV, epi, 1, n->st);
}

// Input gradient: dst = conv^T(dz), masked by mask > 0 when mask is given.
void conv_bwd_data(ot_net* n, int li, int nb, int lev, const bf16_t* dz, bf16_t* dst, int dst_ld,
                   const bf16_t* mask, int mask_ld) {
    const Layer& l = n->layers[li];
    ConvArgs a{};
    a.src = dz;
    a.src_ld = l.cout_p;
    a.cin = l.cout_p;
    a.taps = l.taps;
    a.wmat = n->wb + l.off_w;
    a.nb = nb;
    a.H = n->d.H >> lev;
    a.W = n->d.W >> lev;
    a.M = nb * a.H * a.W;
    a.N = l.cin_p;
    a.K = l.taps * l.cout_p;
    a.dst = dst;
    a.dst_ld = dst_ld;
    a.dst_off = 0;
    a.dst_n = l.cin_p;
    a.mask = mask;
    a.mask_ld = mask_ld;
    launch_conv(a, MODE_CONV, mask ? EPI_MASK : EPI_PLAIN, 1, n->st);
}

// Weight and bias gradient of layer li into n->grad.
int conv_wgrad(ot_net* n, int li, int nb, int lev, View src, const bf16_t* dz) {
    const Layer& l = n->layers[li];
    ConvArgs a{};
    a.src = src.ptr;
    a.src_ld = src.ld;
    a.cin = l.cin_p;
    a.taps = l.taps;
    a.dz = dz;
    a.dz_ld = l.cout_p;
    a.nb = nb;
    a.H = n->d.H >> lev;
    a.W = n->d.W >> lev;
    a.M = l.taps * l.cin_p + 1;
    a.N = l.cout_p;
    a.K = nb * a.H * a.W;
    const Split s = wgrad_split(a.M, a.N, a.K);
    if ((long long)s.splits * a.M * a.N > n->part_cap) {
        n->err = "internal: weight-gradient partials exceed the workspace";
        return OT_ERR_SHAPE;
    }
    a.ksplit = s.ksplit;
    a.dst = n->part;
    a.dst_ld = a.N;
    a.dst_n = a.N;
    launch_conv(a, MODE_WGRAD, EPI_PART, s.splits, n->st);
    launch_wgrad_reduce(n->part, s.splits, a.M, a.N, n->grad + l.off_p, n->st);
    return OT_OK;
}

// Forward pass into n's activations; the output (FP32, out_ch channels) goes
// to y.
void forward(ot_net* n, int nb, const float* x, float* y) {
    const ot_net_desc& d = n->d;
    const int L = d.levels;
    const int cin0 = pad8(d.in_ch);
    launch_pack_input(x, d.in_ch, (long long)nb * d.H * d.W, n->x8, cin0, n->st);
    View in{n->x8, cin0};
    for (int l = 0; l < L; ++l) {
        const int w = d.base << l;
        const int up = l + 1 < L ? d.base << (l + 1) : 0;
        conv_fwd(n, enc(n, l, 0), nb, l, in, n->a[l], w, 0, w, EPI_RELU);
        if (l + 1 < L) {
            conv_fwd(n, enc(n, l, 1), nb, l, View{n->a[l], w}, n->cat[l], up + w, up, w, EPI_RELU);
            launch_pool(View{n->cat[l] + up, up + w}, w, nb, d.H >> l, d.W >> l, n->pool[l + 1], n->st);
            in = View{n->pool[l + 1], w};
        } else {
            conv_fwd(n, enc(n, l, 1), nb, l, View{n->a[l], w}, n->bot, w, 0, w, EPI_RELU);
        }
    }
    const bf16_t* low = n->bot;
    for (int l = L - 2; l >= 0; --l) {
        const int w = d.base << l, up = d.base << (l + 1);
        launch_upsample(low, up, nb, d.H >> (l + 1), d.W >> (l + 1), View{n->cat[l], up + w}, n->st);
        conv_fwd(n, dec(n, l, 0), nb, l, View{n->cat[l], up + w}, n->da[l], w, 0, w, EPI_RELU);
        conv_fwd(n, dec(n, l, 1), nb, l, View{n->da[l], w}, n->db[l], w, 0, w, EPI_RELU);
        low = n->db[l];
    }
    conv_fwd(n, head(n), nb, 0, View{const_cast<bf16_t*>(low), d.base}, y, d.out_ch, 0, d.out_ch,
             EPI_F32);
}

// Backward pass from n->dy; weight gradients into n->grad (padded layout).
int backward(ot_net* n, int nb) {
    const ot_net_desc& d = n->d;
    const int L = d.levels;
    const int cin0 = pad8(d.in_ch);
    int st;
    // output layer
    const bf16_t* hin = L > 1 ? n->db[0] : n->bot;
    if ((st = conv_wgrad(n, head(n), nb, 0, View{const_cast<bf16_t*>(hin), d.base}, n->dy)) != OT_OK) return st;
    conv_bwd_data(n, head(n), nb, 0, n->dy, n->gz1[0], d.base, hin, d.base);
    bf16_t* dz = n->gz1[0];          // gradient at the pre-activation of the layer producing hin
    for (int l = 0; l + 1 < L; ++l) {
        const int w = d.base << l, up = d.base << (l + 1);
        if ((st = conv_wgrad(n, dec(n, l, 1), nb, l, View{n->da[l], w}, dz)) != OT_OK) return st;
        conv_bwd_data(n, dec(n, l, 1), nb, l, dz, n->gz2[l], w, n->da[l], w);
        if ((st = conv_wgrad(n, dec(n, l, 0), nb, l, View{n->cat[l], up + w}, n->gz2[l])) != OT_OK) return st;
        conv_bwd_data(n, dec(n, l, 0), nb, l, n->gz2[l], n->gcat[l], up + w, nullptr, 0);
        const bf16_t* lowh = l + 2 < L ? n->db[l + 1] : n->bot;
        launch_up_bwd(View{n->gcat[l], up + w}, up, nb, d.H >> (l + 1), d.W >> (l + 1), lowh,
                      n->gz1[l + 1], n->st);
        dz = n->gz1[l + 1];
    }
    for (int l = L - 1; l >= 0; --l) {
        const int w = d.base << l, up = l + 1 < L ? d.base << (l + 1) : 0;
        if (l + 1 < L) {
            launch_merge(n->gpool[l + 1], View{n->gcat[l] + up, up + w}, View{n->cat[l] + up, up + w},
                         w, nb, d.H >> l, d.W >> l, n->gz1[l], n->st);
            dz = n->gz1[l];
        }
        if ((st = conv_wgrad(n, enc(n, l, 1), nb, l, View{n->a[l], w}, dz)) != OT_OK) return st;
        conv_bwd_data(n, enc(n, l, 1), nb, l, dz, n->gz2[l], w, n->a[l], w);
        const View in = l == 0 ? View{n->x8, cin0} : View{n->pool[l], d.base << (l - 1)};
        if ((st = conv_wgrad(n, enc(n, l, 0), nb, l, in, n->gz2[l])) != OT_OK) return st;
        if (l > 0)
            conv_bwd_data(n, enc(n, l, 0), nb, l, n->gz2[l], n->gpool[l], d.base << (l - 1), nullptr, 0);
    }
    return OT_OK;
}

void export_weights(ot_net* n) {
    for (auto& l : n->layers)
        launch_export(n->master + l.off_p, l.taps, l.cin_p, l.cout_p, n->wf + l.off_w,
                      n->wb + l.off_w, n->st);
}

int loss_and_grad(ot_net* n, int nb, const float* x, const float* t, const float* cw, double* loss) {
    const ot_net_desc& d = n->d;
    if (nb < 1 || nb > d.max_batch) { n->err = "batch outside [1, max_batch]"; return OT_ERR_SHAPE; }
    if (!x || !t || !cw) { n->err = "null input"; return OT_ERR_PARAM; }
    forward(n, nb, x, n->y);
    const long long npix = (long long)nb * d.H * d.W;
    launch_loss(n->y, t, cw, d.out_ch, pad8(d.out_ch), npix, n->dy, n->lpart, n->st);
    const int st = backward(n, nb);
    if (st != OT_OK) return st;
    if (loss) {
        launch_sum(n->lpart, loss_blocks(npix * pad8(d.out_ch)), n->lsum, n->st);
        hipError_t e = hipMemcpyAsync(loss, n->lsum, sizeof(double), hipMemcpyDeviceToHost, n->st);
        if (e == hipSuccess) e = hipStreamSynchronize(n->st);
        if (e != hipSuccess) return hipfail(n, e, "loss readback");
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hipfail(n, e, "kernel launch");
    return OT_OK;
}

otn::WarmGeom warm_geom(const ot_dyn_desc* d) {
    otn::WarmGeom g;
    g.X = d->X;
    g.Y = d->Y;
    g.C = d->C;
    g.P = d->P;
    g.perx = d->bc[0] == OT_BC_PERIODIC;
    g.pery = d->bc[1] == OT_BC_PERIODIC;
    g.perc = d->bc[2] == OT_BC_PERIODIC;
    return g;
}

int warm_check(const ot_dyn_desc* d, int batch) {
    if (!d || batch < 1) return OT_ERR_PARAM;
    if (d->X < 1 || d->Y < 1 || d->C < 1 || d->P < 2) return OT_ERR_SHAPE;
    return OT_OK;
}

}  // namespace

extern "C" {

int ot_net_default_desc(int H, int W, int in_ch, int out_ch, int max_batch, ot_net_desc* d) {
    if (!d) return OT_ERR_PARAM;
    std::memset(d, 0, sizeof(*d));
    d->H = H;
    d->W = W;
    d->in_ch = in_ch;
    d->out_ch = out_ch;
    d->base = 32;
    d->levels = 4;
    d->max_batch = max_batch;
    d->beta1 = 0.9;
    d->beta2 = 0.999;
    d->eps = 1e-8;
    return check_desc(d);
}

int ot_net_param_count(const ot_net_desc* d, long long* count) {
    const int st = check_desc(d);
    if (st != OT_OK) return st;
    if (!count) return OT_ERR_PARAM;
    long long c = 0;
    for (auto& l : make_layers(*d)) c += (long long)l.taps * l.cin_o * l.cout_o + l.cout_o;
    *count = c;
    return OT_OK;
}

int ot_net_workspace_size(const ot_net_desc* d, size_t* bytes) {
    const int st = check_desc(d);
    if (st != OT_OK) return st;
    if (!bytes) return OT_ERR_PARAM;
    *bytes = carve(*d, nullptr, nullptr);
    return OT_OK;
}

int ot_net_create(const ot_net_desc* d, void* stream, void* workspace, size_t ws_bytes,
                  ot_net** out) {
    if (!out) return OT_ERR_PARAM;
    *out = nullptr;
    int st = check_desc(d);
    if (st != OT_OK) return st;
    const size_t need = carve(*d, nullptr, nullptr);
    if (!workspace || ws_bytes < need || ((uintptr_t)workspace % kAlign) != 0) return OT_ERR_SHAPE;
    ot_net* n = new (std::nothrow) ot_net();
    if (!n) return OT_ERR_PARAM;
    n->d = *d;
    n->st = (hipStream_t)stream;
    carve(*d, n, (char*)workspace);
    ot_net_param_count(d, &n->np_o);
    // zero parameters and moments, then the BF16 copies
    hipError_t e = hipMemsetAsync(n->master, 0, n->np_p * 4, n->st);
    if (e == hipSuccess) e = hipMemsetAsync(n->mom1, 0, n->np_p * 4, n->st);
    if (e == hipSuccess) e = hipMemsetAsync(n->mom2, 0, n->np_p * 4, n->st);
    if (e != hipSuccess) {
        delete n;
        return OT_ERR_HIP;
    }
    export_weights(n);
    *out = n;
    return OT_OK;
}

int ot_net_set_params(ot_net* n, const float* params) {
    if (!n || !params) return OT_ERR_PARAM;
    for (auto& l : n->layers)
        launch_param_map(params + l.off_o, n->master + l.off_p, l.taps, l.cin_o, l.cout_o, l.cin_p,
                         l.cout_p, 1, n->st);
    hipError_t e = hipMemsetAsync(n->mom1, 0, n->np_p * 4, n->st);
    if (e == hipSuccess) e = hipMemsetAsync(n->mom2, 0, n->np_p * 4, n->st);
    if (e != hipSuccess) return hipfail(n, e, "reset moments");
    n->step = 0;
    export_weights(n);
    e = hipGetLastError();
    return e == hipSuccess ? OT_OK : hipfail(n, e, "set_params");
}

int ot_net_get_params(ot_net* n, float* params) {
    if (!n || !params) return OT_ERR_PARAM;
    for (auto& l : n->layers)
        launch_param_map(n->master + l.off_p, params + l.off_o, l.taps, l.cin_o, l.cout_o, l.cin_p,
                         l.cout_p, 0, n->st);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? OT_OK : hipfail(n, e, "get_params");
}

int ot_net_forward(ot_net* n, int batch, const float* x, float* y) {
    if (!n || !x || !y) return OT_ERR_PARAM;
    if (batch < 1 || batch > n->d.max_batch) { n->err = "batch outside [1, max_batch]"; return OT_ERR_SHAPE; }
    forward(n, batch, x, y);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? OT_OK : hipfail(n, e, "forward");
}

int ot_net_grad(ot_net* n, int batch, const float* x, const float* t, const float* cw,
                float* grad, double* loss) {
    if (!n) return OT_ERR_PARAM;
    const int st = loss_and_grad(n, batch, x, t, cw, loss);
    if (st != OT_OK) return st;
    if (grad) {
        for (auto& l : n->layers)
            launch_param_map(n->grad + l.off_p, grad + l.off_o, l.taps, l.cin_o, l.cout_o, l.cin_p,
                             l.cout_p, 0, n->st);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hipfail(n, e, "grad export");
    }
    return OT_OK;
}

int ot_net_train_step(ot_net* n, int batch, const float* x, const float* t, const float* cw,
                      float lr, double* loss) {
    if (!n) return OT_ERR_PARAM;
    if (!(lr > 0.f) || !std::isfinite(lr)) { n->err = "learning rate must be positive"; return OT_ERR_PARAM; }
    const int st = loss_and_grad(n, batch, x, t, cw, loss);
    if (st != OT_OK) return st;
    n->step += 1;
    const double b1 = n->d.beta1, b2 = n->d.beta2;
    const float c1 = (float)(1.0 - std::pow(b1, n->step));
    const float c2 = (float)(1.0 - std::pow(b2, n->step));
    launch_adam(n->master, n->mom1, n->mom2, n->grad, n->np_p, lr, (float)b1, (float)b2,
                (float)n->d.eps, c1, c2, n->st);
    export_weights(n);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? OT_OK : hipfail(n, e, "train step");
}

int ot_net_destroy(ot_net* n) {
    if (!n) return OT_OK;
    (void)hipStreamSynchronize(n->st);
    delete n;
    return OT_OK;
}

const char* ot_net_last_error(const ot_net* n) { return n ? n->err.c_str() : "null net"; }

int ot_warm_inputs(const ot_dyn_desc* d, int batch, const float* f0, const float* f1,
                   const float* base, float* x, void* stream) {
    int st = warm_check(d, batch);
    if (st != OT_OK) return st;
    if (!f0 || !f1 || !x) return OT_ERR_PARAM;
    launch_warm_inputs(warm_geom(d), batch, f0, f1, base, x, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? OT_OK : OT_ERR_HIP;
}

int ot_warm_targets(const ot_dyn_desc* d, int batch, const float* f0, const float* f1,
                    const float* F, long long sF, const float* Mx, const float* My,
                    const float* Mc, long long sM, const float* base, float* t, void* stream) {
    int st = warm_check(d, batch);
    if (st != OT_OK) return st;
    if (!f0 || !f1 || !F || !Mx || !My || !Mc || !t) return OT_ERR_PARAM;
    const long long slice = (long long)d->X * d->Y * d->C;
    if (sF < slice * (d->P + 1) || sM < slice * d->P) return OT_ERR_SHAPE;
    launch_warm_targets(warm_geom(d), batch, f0, f1, F, sF, Mx, My, Mc, sM, base, t,
                        (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? OT_OK : OT_ERR_HIP;
}

int ot_warm_state(const ot_dyn_desc* d, int batch, const float* f0, const float* f1,
                  const float* y, const float* base, float* F, long long sF, float* Mx,
                  float* My, float* Mc, long long sM, void* stream) {
    int st = warm_check(d, batch);
    if (st != OT_OK) return st;
    if (!f0 || !f1 || !F || !Mx || !My || !Mc || !y) return OT_ERR_PARAM;
    const long long slice = (long long)d->X * d->Y * d->C;
    if (sF < slice * (d->P + 1) || sM < slice * d->P) return OT_ERR_SHAPE;
    launch_warm_state(warm_geom(d), batch, f0, f1, y, base, F, sF, Mx, My, Mc, sM,
                      (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? OT_OK : OT_ERR_HIP;
}

int ot_warm_restrict(const ot_dyn_desc* fine, int batch, const float* f, float* fc, void* stream) {
    int st = warm_check(fine, batch);
    if (st != OT_OK) return st;
    if (!f || !fc) return OT_ERR_PARAM;
    if (fine->X % 2 || fine->Y % 2) return OT_ERR_SHAPE;
    otn::WarmGeom gc = warm_geom(fine);
    gc.X /= 2;
    gc.Y /= 2;
    launch_restrict(gc, batch, f, fc, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? OT_OK : OT_ERR_HIP;
}

int ot_warm_prolong(const ot_dyn_desc* coarse, const ot_dyn_desc* fine, int batch,
                    const float* Fc, long long sFc, const float* Mxc, const float* Myc,
                    const float* Mcc, long long sMc, float* F, long long sF, float* Mx,
                    float* My, float* Mc, long long sM, void* stream) {
    int st = warm_check(coarse, batch);
    if (st == OT_OK) st = warm_check(fine, batch);
    if (st != OT_OK) return st;
    if (!Fc || !Mxc || !Myc || !Mcc || !F || !Mx || !My || !Mc) return OT_ERR_PARAM;
    if (fine->X != 2 * coarse->X || fine->Y != 2 * coarse->Y || fine->C != coarse->C)
        return OT_ERR_SHAPE;
    for (int a = 0; a < 3; ++a)
        if (fine->bc[a] != coarse->bc[a]) return OT_ERR_SHAPE;
    const long long slc = (long long)coarse->X * coarse->Y * coarse->C;
    const long long slf = (long long)fine->X * fine->Y * fine->C;
    if (sFc < slc * (coarse->P + 1) || sMc < slc * coarse->P || sF < slf * (fine->P + 1) ||
        sM < slf * fine->P)
        return OT_ERR_SHAPE;
    launch_prolong(warm_geom(coarse), warm_geom(fine), batch, Fc, sFc, Mxc, Myc, Mcc, sMc, F, sF,
                   Mx, My, Mc, sM, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? OT_OK : OT_ERR_HIP;
}

}  // extern "C"
