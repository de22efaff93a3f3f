// ot_dyn_solve_static: the certified cold-start solve over a library-owned
// device workspace, for callers that cannot allocate device memory.
//
// The workspace is one file-scope device array of OT_DYN_STATIC_BYTES per
// GPU (loaded with the library's code object, held until the process ends).
// In host code the array's name is only a host-side stand-in: its device
// address is taken once per device with hipGetSymbolAddress and only that
// address is handed to the plan and its kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ot_dyn.h"

namespace {

static __device__ __align__(256) char scratch[OT_DYN_STATIC_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};   // device address of `scratch`, per device

// Device address of the current device's array (looked up on the first call
// on that device, with it current).
int scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return OT_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return OT_ERR_HIP;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return OT_OK;
}

}  // namespace

extern "C" int ot_dyn_solve_static(const ot_dyn_desc* d, void* stream, const float* f0,
                                   const float* f1, float* F, float* Mx, float* My, float* Mc,
                                   int max_iters, ot_dyn_report* rep) {
    if (!d || !f0 || !f1 || !F || !Mx || !My || !Mc || max_iters < 1) return OT_ERR_PARAM;
    size_t need = 0;
    int st = ot_dyn_workspace_size(d, &need);
    if (st != OT_OK) return st;
    if (need > (size_t)OT_DYN_STATIC_BYTES) return OT_ERR_SHAPE;
    void* ws = nullptr;
    st = scratch_address(&ws);
    if (st != OT_OK) return st;
    ot_dyn_plan* p = nullptr;
    st = ot_dyn_create(d, stream, ws, OT_DYN_STATIC_BYTES, &p);
    if (st != OT_OK) return st;
    st = ot_dyn_set_boundary(p, f0, f1);
    if (st == OT_OK) st = ot_dyn_init(p, OT_INIT_COLD, F, Mx, My, Mc);
    if (st == OT_OK) st = ot_dyn_solve(p, F, Mx, My, Mc, max_iters, rep);
    ot_dyn_destroy(p);
    return st;
}
