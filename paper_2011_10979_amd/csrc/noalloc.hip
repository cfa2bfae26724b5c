// flow_solve_static: the plain solve for callers that cannot allocate device memory.  Its working
// set (pyramids, linearisation, state, reduction partials) lives in one file-scope device array of
// kStaticBytes per GPU instead of a context arena; the kernels are the plain solve's, launched
// directly with the built-in kernel plan.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>
#include <tuple>

#include "runtime.hpp"

namespace flowmi {

namespace {

constexpr size_t kStaticBytes = FLOW_STATIC_BYTES;
// head of the array: a~ slots, tile-queue counters, energy partials and totals
constexpr size_t kAtOff = 0, kQueueOff = 256, kPartialOff = 512;
constexpr size_t kOutOff = kPartialOff + sizeof(double) * kEnergyTerms * kEnergyBlocks;
constexpr size_t kHeadBytes = (kOutOff + sizeof(double) * kEnergyTerms + 255) & ~(size_t)255;
static_assert(kHeadBytes + 256 < kStaticBytes, "workspace head");

// Host code must not take this array's address directly (that is a host-side stand-in): the
// device address of each GPU's copy comes from hipGetSymbolAddress, once per device.
__device__ __align__(256) char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};

flow_status scratch_ptr(int dev, char** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(FLOW_E_INVAL, "device index beyond the static workspaces");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(FLOW_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_ptr[dev] = (char*)p;
    }
    *out = g_ptr[dev];
    return FLOW_OK;
}

}  // namespace

size_t static_workspace_need(int H, int W, const flow_params& p) { return kHeadBytes + layout_bytes(H, W, p); }
size_t static_workspace_bytes() { return kStaticBytes; }

}  // namespace flowmi

using namespace flowmi;

#define HIP_TRY(expr)                                           \
    do {                                                        \
        hipError_t _e = (expr);                                 \
        if (_e != hipSuccess) return hip_fail(_e, #expr);       \
    } while (0)

extern "C" flow_status flow_static_bytes(int32_t H, int32_t W, const flow_params* p, uint64_t* need,
                                         uint64_t* limit) {
    flow_status st = validate(p);
    if (st != FLOW_OK) return st;
    if (H < 2 || W < 2 || H > FLOW_MAX_SIDE || W > FLOW_MAX_SIDE) return fail(FLOW_E_INVAL, "bad shape");
    if (need) *need = static_workspace_need(H, W, *p);
    if (limit) *limit = static_workspace_bytes();
    return FLOW_OK;
}

extern "C" flow_status flow_solve_static(const float* I0, const float* I1, int32_t H, int32_t W, int64_t ld,
                                         const flow_params* p, float* u, float* v, int64_t ld_uv, flow_result* res,
                                         void* stream) {
    if (!I0 || !I1 || !u || !v) return fail(FLOW_E_INVAL, "NULL device pointer");
    flow_status st = validate(p);
    if (st != FLOW_OK) return st;
    st = validate_shape(H, W, ld, p->levels);
    if (st != FLOW_OK) return st;
    if (ld_uv < W) return fail(FLOW_E_INVAL, "ld_uv smaller than W");
    if (p->tol != 0.0) return fail(FLOW_E_INVAL, "flow_solve_static runs a fixed iteration count (tol must be 0)");
    const size_t need = static_workspace_need(H, W, *p);
    if (need > static_workspace_bytes())
        return fail(FLOW_E_NOMEM, "working set of " + std::to_string(need) + " bytes exceeds the " +
                                      std::to_string(static_workspace_bytes()) + "-byte static workspace");
    for (auto [ptr, l, name] : {std::make_tuple((const void*)I0, ld, "I0"), std::make_tuple((const void*)I1, ld, "I1"),
                                std::make_tuple((const void*)u, ld_uv, "u"), std::make_tuple((const void*)v, ld_uv, "v")}) {
        st = check_extent(ptr, H, W, l, sizeof(float), name);
        if (st != FLOW_OK) return st;
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    char* base = nullptr;
    st = scratch_ptr(dev, &base);
    if (st != FLOW_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const bool f16 = p->storage == FLOW_STORE_F16;

    // the head of the workspace: every word that must start at zero is cleared here by a kernel
    // (the a~ slots are also cleared by the level start and the linearisation themselves)
    Scratch sc;
    sc.at = (float*)(base + kAtOff);
    sc.queue = (unsigned*)(base + kQueueOff);
    sc.e_partial = (double*)(base + kPartialOff);
    sc.e_out = (double*)(base + kOutOff);
    launch_reset_u32((unsigned*)(base + kAtOff), 128, s);     // a~ slots and queue counters
    DevArena arena;
    arena.base = base + kHeadBytes;
    arena.bytes = static_workspace_bytes() - kHeadBytes;
    std::vector<LevelPlanes> Ls;
    st = build_layout(arena, H, W, *p, Ls);
    if (st != FLOW_OK) return st;
    SolvePlan plan;
    st = make_plan(Ls, *p, sc, plan, nullptr, false);    // built-in choices, direct tiling: no tables
    if (st != FLOW_OK) return st;

    launch_import(I0, H, W, ld, Ls[0].I0, Ls[0].ld, f16, s);
    launch_import(I1, H, W, ld, Ls[0].I1, Ls[0].ld, f16, s);
    st = enqueue_core(Ls, *p, sc, s, nullptr, nullptr, &plan);
    if (st != FLOW_OK) return st;
    const int fb = sc.final_buf;
    launch_copy2d(level_flow(Ls[0], *p, 1, fb), H, W, Ls[0].ld, u, ld_uv, s, level_inc(Ls[0], *p, 1, fb));
    launch_copy2d(level_flow(Ls[0], *p, 2, fb), H, W, Ls[0].ld, v, ld_uv, s, level_inc(Ls[0], *p, 2, fb));
    HIP_TRY(hipGetLastError());
    if (!res) return FLOW_OK;
    double h[kEnergyTerms];
    HIP_TRY(hipMemcpyAsync(h, sc.e_out, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    fill_result(h, res);
    if (!std::isfinite(h[0] + h[1]) || !std::isfinite(h[2]) || h[7] != 0.0)
        return fail(FLOW_E_NONFINITE, "energy or gap is not finite");
    return FLOW_OK;
}
