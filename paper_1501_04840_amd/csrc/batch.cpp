// Batched solver for many independent problems of uneven sizes.
//
// Problems are grouped by shape (X, Y, C, P); a group is one batched plan
// over group-contiguous buffers inside the caller's workspace.  A chunk of
// iterations of every active group is captured into one HIP graph with a
// branch per group (the batch's stream forks into the groups' streams and
// joins them), so the per-kernel launch cost is paid once per graph.  The
// branches overlap little on the GPU: the tail of a batch, where a few
// problems of several groups remain, costs about the sum of the groups'
// launch latencies per iteration.  After each chunk the FP64 residuals of
// every problem are collected and certified problems are recorded; a group
// whose problems are all certified leaves the graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/ot_dyn.h"
#include "otd_common.h"

using namespace otd;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Group {
    ot_dyn_desc d;                 // shape, batch = members
    std::vector<int> members;      // problem ids in group order
    hipStream_t side = nullptr;
    ot_dyn_plan* plan = nullptr;
    size_t off_state = 0, off_plan = 0, plan_bytes = 0;
    float *F = nullptr, *Mx = nullptr, *My = nullptr, *Mc = nullptr;
    float *f0 = nullptr, *f1 = nullptr;
    bool active = true;
    std::vector<int> conv_iter;    // per member: iteration of certification, -1 if none
    std::vector<char> fell_back;   // per member: restarted cold after its warm start
    std::vector<int> deadline;     // per member: last iteration of its current run
    std::vector<int> stopped;      // per member: iteration it stopped uncertified, -1 if running
    std::vector<ot_dyn_report> rep;
    int row_bx = 0, dense_xy = 0;
    long long slice() const { return (long long)d.X * d.Y * d.C; }
    long long nc() const { return slice() * d.P; }
    long long nf() const { return slice() * (d.P + 1); }
};

struct Plan {
    std::vector<Group> groups;
    std::vector<int> group_of, index_in_group;
    std::vector<long long> off_h, off_F, off_M;
    size_t total = 0;
};

int check_dims(int count, const int* dims) {
    if (count < 1 || !dims) return OT_ERR_PARAM;
    for (int i = 0; i < count; ++i) {
        const int* q = dims + 4 * i;
        if (q[0] < 1 || q[1] < 1 || q[2] < 1 || q[3] < 2) return OT_ERR_SHAPE;
    }
    return OT_OK;
}

// Group the problems by shape and lay out the workspace.
int make_plan(const ot_dyn_desc* base, int count, const int* dims, Plan* out) {
    int st = check_dims(count, dims);
    if (st != OT_OK) return st;
    std::map<std::vector<int>, int> key;
    Plan P;
    P.group_of.resize(count);
    P.index_in_group.resize(count);
    for (int i = 0; i < count; ++i) {
        const std::vector<int> k(dims + 4 * i, dims + 4 * i + 4);
        auto it = key.find(k);
        int gi;
        if (it == key.end()) {
            gi = (int)P.groups.size();
            key[k] = gi;
            Group g;
            g.d = *base;
            g.d.X = k[0]; g.d.Y = k[1]; g.d.C = k[2]; g.d.P = k[3];
            P.groups.push_back(g);
        } else {
            gi = it->second;
        }
        P.group_of[i] = gi;
        P.index_in_group[i] = (int)P.groups[gi].members.size();
        P.groups[gi].members.push_back(i);
    }
    size_t o = 0;
    for (auto& g : P.groups) {
        g.d.batch = (int)g.members.size();
        size_t pb = 0;
        st = ot_dyn_workspace_size(&g.d, &pb);
        if (st != OT_OK) return st;
        const long long B = g.d.batch;
        g.off_state = o;
        o = align_up(o + (size_t)B * (g.nf() + 3 * g.nc() + 2 * g.slice()) * sizeof(float));
        g.off_plan = o;
        g.plan_bytes = pb;
        o = align_up(o + pb);
    }
    P.total = o;
    P.off_h.assign(count + 1, 0);
    P.off_F.assign(count + 1, 0);
    P.off_M.assign(count + 1, 0);
    for (int i = 0; i < count; ++i) {
        const long long sl = (long long)dims[4 * i] * dims[4 * i + 1] * dims[4 * i + 2];
        const long long p = dims[4 * i + 3];
        P.off_h[i + 1] = P.off_h[i] + sl;
        P.off_F[i + 1] = P.off_F[i] + (p + 1) * sl;
        P.off_M[i + 1] = P.off_M[i] + 3 * p * sl;
    }
    *out = std::move(P);
    return OT_OK;
}

}  // namespace

struct ot_dyn_batch {
    ot_dyn_desc base;
    hipStream_t user;          // the caller's stream (inputs are ordered on it)
    hipStream_t stream;        // the batch's own stream: graph capture and replay
    char* ws;
    int count;
    Plan P;
    bool have_boundary = false;
    bool warm = false;         // the next solve starts from ot_dyn_batch_set_state
    bool fallback = false;     // ... and restarts uncertified problems cold (OT_INIT_FALLBACK)
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;
    int graph_chunk = 0;
    bool graph_varies = false;     // launch sequence changes after this graph
    std::vector<int> graph_groups;
    hipGraph_t graph = nullptr;    // one chunk of every active group, a branch each
    hipGraphExec_t exec = nullptr;
    std::string err;
};

namespace {

int hipfail(ot_dyn_batch* bt, hipError_t e, const char* what) {
    bt->err = std::string(what) + ": " + hipGetErrorString(e);
    return OT_ERR_HIP;
}
#define BCHK(bt, call)                                          \
    do {                                                        \
        hipError_t e_ = (call);                                 \
        if (e_ != hipSuccess) return hipfail(bt, e_, #call);    \
    } while (0)

void drop_graph(ot_dyn_batch* bt) {
    if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
    if (bt->graph) (void)hipGraphDestroy(bt->graph);
    bt->exec = nullptr;
    bt->graph = nullptr;
    bt->graph_groups.clear();
    bt->graph_chunk = 0;
}

// Capture `chunk` iterations (the last one with residual partials) of every
// active group into one graph: the batch's stream forks into the groups'
// streams (event record / wait), each group's chunk is a branch, and the
// branches join back, so the graph holds independent chains that the
// runtime can run concurrently.
int build_graph(ot_dyn_batch* bt, int chunk) {
    drop_graph(bt);
    bool varies = false;
    std::vector<int> act;
    for (size_t gi = 0; gi < bt->P.groups.size(); ++gi)
        if (bt->P.groups[gi].active) act.push_back((int)gi);
    if (act.empty()) return OT_OK;
    BCHK(bt, hipStreamBeginCapture(bt->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipEventRecord(bt->ev_fork, bt->stream);
    for (size_t i = 0; e == hipSuccess && i < act.size(); ++i) {
        Group& g = bt->P.groups[act[i]];
        varies = varies || plan_launch_varies(g.plan);
        e = hipStreamWaitEvent(g.side, bt->ev_fork, 0);
        if (e != hipSuccess) break;
        for (int it = 0; it < chunk; ++it)
            plan_iterate(g.plan, g.F, g.Mx, g.My, g.Mc, it + 1 == chunk);
        e = hipEventRecord(bt->ev_join[act[i]], g.side);
        if (e == hipSuccess) e = hipStreamWaitEvent(bt->stream, bt->ev_join[act[i]], 0);
    }
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(bt->stream, &graph);
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hipfail(bt, e, "capture of the groups' chunk");
    }
    if (e2 != hipSuccess) return hipfail(bt, e2, "hipStreamEndCapture");
    bt->graph = graph;
    BCHK(bt, hipGraphInstantiate(&bt->exec, graph, nullptr, nullptr, 0));
    bt->graph_groups = act;
    bt->graph_chunk = chunk;
    bt->graph_varies = varies;
    return OT_OK;
}

std::string tune_key(const ot_dyn_desc& d) {
    char b[160];
    std::snprintf(b, sizeof b, "%d,%d,%d,%d,%d,%d,%d%d%d", d.X, d.Y, d.C, d.P, d.batch, d.refine,
                  d.bc[0], d.bc[1], d.bc[2]);
    return b;
}

std::map<std::string, std::pair<int, int>> load_cache(const char* path) {
    std::map<std::string, std::pair<int, int>> m;
    if (!path) return m;
    std::ifstream in(path);
    std::string k;
    int a, b;
    while (in >> k >> a >> b) m[k] = {a, b};
    return m;
}

void save_cache(const char* path, const std::map<std::string, std::pair<int, int>>& m) {
    if (!path) return;
    std::ofstream out(path);
    for (auto& kv : m) out << kv.first << " " << kv.second.first << " " << kv.second.second << "\n";
}

}  // namespace

extern "C" {

int ot_dyn_batch_workspace_size(const ot_dyn_desc* base, int count, const int* dims,
                                size_t* bytes) {
    if (!base || !bytes) return OT_ERR_PARAM;
    Plan P;
    const int st = make_plan(base, count, dims, &P);
    if (st != OT_OK) return st;
    *bytes = P.total;
    return OT_OK;
}

int ot_dyn_batch_create(const ot_dyn_desc* base, int count, const int* dims, void* stream,
                        void* workspace, size_t ws_bytes, ot_dyn_batch** out) {
    if (!base || !out) return OT_ERR_PARAM;
    *out = nullptr;
    Plan P;
    int st = make_plan(base, count, dims, &P);
    if (st != OT_OK) return st;
    if (!workspace || ws_bytes < P.total || ((uintptr_t)workspace % kAlign) != 0) return OT_ERR_SHAPE;
    ot_dyn_batch* bt = new (std::nothrow) ot_dyn_batch();
    if (!bt) return OT_ERR_PARAM;
    bt->base = *base;
    bt->user = (hipStream_t)stream;
    bt->stream = nullptr;
    bt->ws = (char*)workspace;
    bt->count = count;
    bt->P = std::move(P);
    auto fail = [&](int code) { ot_dyn_batch_destroy(bt); return code; };
    if (hipStreamCreateWithFlags(&bt->stream, hipStreamNonBlocking) != hipSuccess) return fail(OT_ERR_HIP);
    if (hipEventCreateWithFlags(&bt->ev_fork, hipEventDisableTiming) != hipSuccess) return fail(OT_ERR_HIP);
    bt->ev_join.assign(bt->P.groups.size(), nullptr);
    for (size_t gi = 0; gi < bt->P.groups.size(); ++gi) {
        Group& g = bt->P.groups[gi];
        if (hipEventCreateWithFlags(&bt->ev_join[gi], hipEventDisableTiming) != hipSuccess)
            return fail(OT_ERR_HIP);
        if (hipStreamCreateWithFlags(&g.side, hipStreamNonBlocking) != hipSuccess) return fail(OT_ERR_HIP);
        const long long B = g.d.batch;
        float* s = (float*)(bt->ws + g.off_state);
        g.F = s;
        g.Mx = g.F + B * g.nf();
        g.My = g.Mx + B * g.nc();
        g.Mc = g.My + B * g.nc();
        g.f0 = g.Mc + B * g.nc();
        g.f1 = g.f0 + B * g.slice();
        st = ot_dyn_create(&g.d, g.side, bt->ws + g.off_plan, g.plan_bytes, &g.plan);
        if (st != OT_OK) return fail(st);
        plan_enable_freeze(g.plan);
        g.conv_iter.assign(g.members.size(), -1);
        g.fell_back.assign(g.members.size(), 0);
        g.rep.assign(g.members.size(), ot_dyn_report{});
    }
    *out = bt;
    return OT_OK;
}

int ot_dyn_batch_offsets(const ot_dyn_batch* bt, long long* off_h, long long* off_F,
                         long long* off_M) {
    if (!bt) return OT_ERR_PARAM;
    for (int i = 0; i <= bt->count; ++i) {
        if (off_h) off_h[i] = bt->P.off_h[i];
        if (off_F) off_F[i] = bt->P.off_F[i];
        if (off_M) off_M[i] = bt->P.off_M[i];
    }
    return OT_OK;
}

int ot_dyn_batch_set_boundary(ot_dyn_batch* bt, const float* f0, const float* f1) {
    if (!bt || !f0 || !f1) return OT_ERR_PARAM;
    bt->have_boundary = false;
    BCHK(bt, hipStreamSynchronize(bt->user));      // inputs were produced on the caller's stream
    for (auto& g : bt->P.groups) {
        const size_t bytes = g.slice() * sizeof(float);
        for (size_t j = 0; j < g.members.size(); ++j) {
            const int i = g.members[j];
            BCHK(bt, hipMemcpyAsync(g.f0 + j * g.slice(), f0 + bt->P.off_h[i], bytes,
                                    hipMemcpyDeviceToDevice, g.side));
            BCHK(bt, hipMemcpyAsync(g.f1 + j * g.slice(), f1 + bt->P.off_h[i], bytes,
                                    hipMemcpyDeviceToDevice, g.side));
        }
        const int st = ot_dyn_set_boundary(g.plan, g.f0, g.f1);
        if (st != OT_OK) {
            bt->err = ot_dyn_last_error(g.plan);
            return st;
        }
    }
    bt->have_boundary = true;
    return OT_OK;
}

int ot_dyn_batch_autotune(ot_dyn_batch* bt, int trials) {
    if (!bt || trials < 1) return OT_ERR_PARAM;
    if (!bt->have_boundary) { bt->err = "set the boundary first"; return OT_ERR_STATE; }
    const char* path = std::getenv("OT_DYN_TUNE_CACHE");
    auto cache = load_cache(path);
    hipEvent_t t0, t1;
    BCHK(bt, hipEventCreate(&t0));
    BCHK(bt, hipEventCreate(&t1));
    int status = OT_OK;
    for (auto& g : bt->P.groups) {
        const std::string key = tune_key(g.d);
        auto it = cache.find(key);
        if (it != cache.end()) {
            g.row_bx = it->second.first;
            g.dense_xy = it->second.second;
            plan_apply_tuning(g.plan, g.row_bx, g.dense_xy);
            continue;
        }
        std::vector<int> bxs;
        const int def = row_block(g.d.X);
        for (int bx : {64, 128, 256})
            if (bx <= def) bxs.push_back(bx);
        std::vector<int> dens = {0};
        if (plan_has_fast_xy(g.plan)) { dens.push_back(1); dens.push_back(2); }
        float best = 1e30f;
        int bbx = def, bdn = 0;
        for (int bx : bxs)
            for (int dn : dens) {
                plan_apply_tuning(g.plan, bx, dn);
                int st = ot_dyn_init(g.plan, OT_INIT_COLD, g.F, g.Mx, g.My, g.Mc);
                if (st != OT_OK) { status = st; break; }
                for (int w = 0; w < 2; ++w) plan_iterate(g.plan, g.F, g.Mx, g.My, g.Mc, false);
                if (hipEventRecord(t0, g.side) != hipSuccess) { status = OT_ERR_HIP; break; }
                for (int w = 0; w < trials; ++w) plan_iterate(g.plan, g.F, g.Mx, g.My, g.Mc, false);
                if (hipEventRecord(t1, g.side) != hipSuccess ||
                    hipEventSynchronize(t1) != hipSuccess) { status = OT_ERR_HIP; break; }
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, t0, t1);
                if (ms < best) { best = ms; bbx = bx; bdn = dn; }
            }
        if (status != OT_OK) break;
        g.row_bx = bbx;
        g.dense_xy = bdn;
        plan_apply_tuning(g.plan, bbx, bdn);
        cache[key] = {bbx, bdn};
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (status != OT_OK) return status;
    save_cache(path, cache);
    drop_graph(bt);
    bt->warm = false;
    for (auto& g : bt->P.groups) {
        const int st = ot_dyn_init(g.plan, OT_INIT_COLD, g.F, g.Mx, g.My, g.Mc);
        if (st != OT_OK) return st;
    }
    BCHK(bt, hipDeviceSynchronize());
    return OT_OK;
}

int ot_dyn_batch_solve(ot_dyn_batch* bt, int max_iters, int chunk, ot_dyn_report* rep) {
    if (!bt || max_iters < 1 || chunk < 1) return OT_ERR_PARAM;
    if (!bt->have_boundary) { bt->err = "set the boundary first"; return OT_ERR_STATE; }
    const auto t0 = std::chrono::steady_clock::now();
    const bool verbose = std::getenv("OT_DYN_VERBOSE") != nullptr;
    drop_graph(bt);
    for (auto& g : bt->P.groups) {
        if (!bt->warm) {
            const int st = ot_dyn_init(g.plan, OT_INIT_COLD, g.F, g.Mx, g.My, g.Mc);
            if (st != OT_OK) return st;
        }
        g.active = true;
        std::fill(g.conv_iter.begin(), g.conv_iter.end(), -1);
        std::fill(g.fell_back.begin(), g.fell_back.end(), 0);
        g.deadline.assign(g.members.size(), max_iters);
        g.stopped.assign(g.members.size(), -1);
        const int st = plan_freeze(g.plan, std::vector<char>(g.members.size(), 0));
        if (st != OT_OK) return st;
    }
    // OT_INIT_FALLBACK: a warm start that is not certified by its deadline
    // (or turns non-finite) restarts cold with a deadline max_iters later
    const bool fallback = bt->warm && bt->fallback;
    bt->warm = false;
    bt->fallback = false;
    for (auto& g : bt->P.groups) BCHK(bt, hipStreamSynchronize(g.side));
    int done = 0;
    while (true) {
        // next residual check: one chunk on, or the earliest deadline of a
        // member still running
        int next = done + chunk;
        bool running = false;
        for (auto& g : bt->P.groups) {
            if (!g.active) continue;
            for (size_t j = 0; j < g.members.size(); ++j)
                if (g.conv_iter[j] < 0 && g.stopped[j] < 0) {
                    next = std::min(next, g.deadline[j]);
                    running = true;
                }
        }
        if (!running) break;
        const int k = next - done;
        if (bt->graph_groups.empty() || bt->graph_chunk != k || bt->graph_varies) {
            const int st = build_graph(bt, k);
            if (st != OT_OK) return st;
        }
        // work the last check left on the groups' streams (step rescaling,
        // frozen flags) precedes the graph
        for (int gi : bt->graph_groups) BCHK(bt, hipStreamSynchronize(bt->P.groups[gi].side));
        BCHK(bt, hipGraphLaunch(bt->exec, bt->stream));
        BCHK(bt, hipStreamSynchronize(bt->stream));
        done += k;
        bool changed = false;
        for (int gi : bt->graph_groups) {
            Group& g = bt->P.groups[gi];
            plan_add_iters(g.plan, k);
            const int st = plan_collect(g.plan, g.F, g.Mx, g.My, g.Mc);
            if (st != OT_OK && st != OT_ERR_NONFINITE) { bt->err = ot_dyn_last_error(g.plan); return st; }
            const size_t n = g.members.size();
            std::vector<char> restart(n, 0);
            bool any_restart = false, any_running = false;
            for (size_t j = 0; j < n; ++j) {
                if (g.conv_iter[j] >= 0 || g.stopped[j] >= 0) continue;   // frozen: report kept
                ot_dyn_report& r = g.rep[j];
                plan_problem(g.plan, (int)j, &r);
                const bool finite = std::isfinite(r.r_prim) && std::isfinite(r.r_dual) &&
                                    std::isfinite(r.r_div) && std::isfinite(r.cost);
                const bool ok = finite && std::max(r.r_prim, r.r_dual) < g.d.tol_res &&
                                r.r_div < g.d.tol_div;
                if (ok) {
                    g.conv_iter[j] = done;
                } else if (!finite || done >= g.deadline[j]) {
                    if (fallback && !g.fell_back[j]) {
                        restart[j] = 1;
                        any_restart = true;
                        g.fell_back[j] = 1;
                        g.deadline[j] = done + max_iters;
                    } else if (!finite) {
                        char buf[160];
                        std::snprintf(buf, sizeof buf, "problem %d: non-finite residual",
                                      g.members[j]);
                        bt->err = buf;
                        return OT_ERR_NONFINITE;
                    } else {
                        g.stopped[j] = done;
                    }
                }
                r.iterations = g.conv_iter[j] >= 0 ? g.conv_iter[j] : done;
                r.converged = g.conv_iter[j] >= 0;
                r.total_iterations = done;
                r.fallback = g.fell_back[j];
                any_running = any_running || (g.conv_iter[j] < 0 && g.stopped[j] < 0);
            }
            if (!any_running) { g.active = false; changed = true; continue; }
            // certified (and stopped) members keep their state: the stencil
            // and colour/time kernels of the remaining chunks skip them
            std::vector<char> frozen(n);
            for (size_t j = 0; j < n; ++j) frozen[j] = g.conv_iter[j] >= 0 || g.stopped[j] >= 0;
            int fst = plan_freeze(g.plan, frozen);
            if (fst == OT_OK && any_restart) {
                fst = plan_restart_cold(g.plan, g.F, g.Mx, g.My, g.Mc, restart);
                changed = true;
            }
            if (fst != OT_OK) { bt->err = ot_dyn_last_error(g.plan); return fst; }
        }
        if (changed) drop_graph(bt);
        if (verbose) {
            int nconv = 0, nact = 0;
            for (auto& g : bt->P.groups) {
                nact += g.active;
                for (int c : g.conv_iter) nconv += c >= 0;
            }
            const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            std::fprintf(stderr, "ot_dyn_batch: %d iterations, %d/%d certified, %d groups active, %.2f s\n",
                         done, nconv, bt->count, nact, el);
        }
    }
    int nconv = 0;
    for (auto& g : bt->P.groups)
        for (int c : g.conv_iter) nconv += c >= 0;
    const int status = nconv == bt->count ? OT_OK : OT_NOT_CONVERGED;
    if (rep) {
        std::memset(rep, 0, sizeof(*rep));
        int worst = 0, nfb = 0;
        double wv = -1.0;
        for (int i = 0; i < bt->count; ++i) {
            const Group& g = bt->P.groups[bt->P.group_of[i]];
            const ot_dyn_report& r = g.rep[bt->P.index_in_group[i]];
            nfb += r.fallback;
            rep->r_prim = std::max(rep->r_prim, r.r_prim);
            rep->r_dual = std::max(rep->r_dual, r.r_dual);
            rep->r_div = std::max(rep->r_div, r.r_div);
            rep->e_mass = std::max(rep->e_mass, r.e_mass);
            const double v = std::max(r.r_prim, r.r_dual);
            if (v > wv) { wv = v; worst = i; }
        }
        rep->iterations = done;
        rep->total_iterations = done;
        rep->converged = nconv;
        rep->fallback = nfb;
        rep->worst_problem = worst;
        rep->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

int ot_dyn_batch_problem(const ot_dyn_batch* bt, int i, ot_dyn_report* rep) {
    if (!bt || !rep || i < 0 || i >= bt->count) return OT_ERR_PARAM;
    const Group& g = bt->P.groups[bt->P.group_of[i]];
    *rep = g.rep[bt->P.index_in_group[i]];
    return OT_OK;
}

int ot_dyn_batch_get_state(ot_dyn_batch* bt, float* F, float* M) {
    if (!bt || !F || !M) return OT_ERR_PARAM;
    for (auto& g : bt->P.groups) {
        for (size_t j = 0; j < g.members.size(); ++j) {
            const int i = g.members[j];
            BCHK(bt, hipMemcpyAsync(F + bt->P.off_F[i], g.F + j * g.nf(), g.nf() * sizeof(float),
                                    hipMemcpyDeviceToDevice, g.side));
            float* m = M + bt->P.off_M[i];
            const float* src[3] = {g.Mx, g.My, g.Mc};
            for (int q = 0; q < 3; ++q)
                BCHK(bt, hipMemcpyAsync(m + q * g.nc(), src[q] + j * g.nc(), g.nc() * sizeof(float),
                                        hipMemcpyDeviceToDevice, g.side));
        }
        BCHK(bt, hipStreamSynchronize(g.side));
    }
    return OT_OK;
}

int ot_dyn_batch_set_state(ot_dyn_batch* bt, const float* F, const float* M, int mode) {
    if (!bt || !F || !M) return OT_ERR_PARAM;
    const bool fallback = (mode & OT_INIT_FALLBACK) != 0;
    mode &= ~OT_INIT_FALLBACK;
    if (mode != OT_INIT_PRIMAL && mode != OT_INIT_PRIMAL_DUAL) {
        bt->err = "set_state takes OT_INIT_PRIMAL or OT_INIT_PRIMAL_DUAL (optionally with "
                  "OT_INIT_FALLBACK)";
        return OT_ERR_PARAM;
    }
    if (!bt->have_boundary) { bt->err = "set the boundary first"; return OT_ERR_STATE; }
    bt->warm = false;
    BCHK(bt, hipStreamSynchronize(bt->user));      // the state was produced on the caller's stream
    for (auto& g : bt->P.groups) {
        for (size_t j = 0; j < g.members.size(); ++j) {
            const int i = g.members[j];
            BCHK(bt, hipMemcpyAsync(g.F + j * g.nf(), F + bt->P.off_F[i], g.nf() * sizeof(float),
                                    hipMemcpyDeviceToDevice, g.side));
            const float* m = M + bt->P.off_M[i];
            float* dst[3] = {g.Mx, g.My, g.Mc};
            for (int q = 0; q < 3; ++q)
                BCHK(bt, hipMemcpyAsync(dst[q] + j * g.nc(), m + q * g.nc(), g.nc() * sizeof(float),
                                        hipMemcpyDeviceToDevice, g.side));
        }
        const int st = ot_dyn_init(g.plan, mode, g.F, g.Mx, g.My, g.Mc);
        if (st != OT_OK) {
            bt->err = ot_dyn_last_error(g.plan);
            return st;
        }
        BCHK(bt, hipStreamSynchronize(g.side));
    }
    bt->warm = true;
    bt->fallback = fallback;
    return OT_OK;
}

// Packed duals: problem i at 4 / 3 of its offset in the packed M.
int ot_dyn_batch_get_dual(ot_dyn_batch* bt, float* Bd) {
    if (!bt || !Bd) return OT_ERR_PARAM;
    for (auto& g : bt->P.groups) {
        for (size_t j = 0; j < g.members.size(); ++j) {
            const int i = g.members[j];
            const int st = plan_copy_dual(g.plan, (int)j, Bd + bt->P.off_M[i] / 3 * 4, 1);
            if (st != OT_OK) { bt->err = ot_dyn_last_error(g.plan); return st; }
        }
        BCHK(bt, hipStreamSynchronize(g.side));
    }
    return OT_OK;
}

int ot_dyn_batch_set_dual(ot_dyn_batch* bt, const float* Bd) {
    if (!bt || !Bd) return OT_ERR_PARAM;
    if (!bt->warm) { bt->err = "set_dual follows set_state"; return OT_ERR_STATE; }
    BCHK(bt, hipStreamSynchronize(bt->user));
    for (auto& g : bt->P.groups) {
        for (size_t j = 0; j < g.members.size(); ++j) {
            const int i = g.members[j];
            const int st = plan_copy_dual(g.plan, (int)j, const_cast<float*>(Bd + bt->P.off_M[i] / 3 * 4), 0);
            if (st != OT_OK) { bt->err = ot_dyn_last_error(g.plan); return st; }
        }
        BCHK(bt, hipStreamSynchronize(g.side));
    }
    return OT_OK;
}

int ot_dyn_batch_tuning(const ot_dyn_batch* bt, int i, int* row_bx, int* dense_xy) {
    if (!bt || i < 0 || i >= bt->count) return OT_ERR_PARAM;
    const Group& g = bt->P.groups[bt->P.group_of[i]];
    if (row_bx) *row_bx = g.row_bx > 0 ? g.row_bx : row_block(g.d.X);
    if (dense_xy) *dense_xy = g.dense_xy;
    return OT_OK;
}

int ot_dyn_batch_destroy(ot_dyn_batch* bt) {
    if (!bt) return OT_OK;
    drop_graph(bt);
    for (auto& g : bt->P.groups) {
        if (g.side) (void)hipStreamSynchronize(g.side);
        if (g.plan) ot_dyn_destroy(g.plan);
        if (g.side) (void)hipStreamDestroy(g.side);
    }
    for (hipEvent_t e : bt->ev_join)
        if (e) (void)hipEventDestroy(e);
    if (bt->ev_fork) (void)hipEventDestroy(bt->ev_fork);
    if (bt->stream) {
        (void)hipStreamSynchronize(bt->stream);
        (void)hipStreamDestroy(bt->stream);
    }
    delete bt;
    return OT_OK;
}

const char* ot_dyn_batch_last_error(const ot_dyn_batch* bt) {
    return bt ? bt->err.c_str() : "null batch";
}

}  // extern "C"
