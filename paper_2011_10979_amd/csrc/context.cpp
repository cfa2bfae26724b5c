// flow_ctx: arena management, graph cache, timers and the plain solve.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <sstream>

#include "runtime.hpp"

namespace flowmi {

#define HIP_TRY(expr)                                           \
    do {                                                        \
        hipError_t _e = (expr);                                 \
        if (_e != hipSuccess) return hip_fail(_e, #expr);       \
    } while (0)

flow_status Scratch::alloc() {
    release();
    HIP_TRY(hipMalloc(&at, 256));
    HIP_TRY(hipMalloc(&queue, 256));
    HIP_TRY(hipMemset(queue, 0, 256));
    HIP_TRY(hipMalloc(&e_partial, sizeof(double) * kEnergyTerms * kEnergyBlocks));
    HIP_TRY(hipMalloc(&e_out, sizeof(double) * kEnergyTerms));
    HIP_TRY(hipMemset(at, 0, 256));
    return FLOW_OK;
}

void Scratch::release() {
    for (void* p : {(void*)at, (void*)queue, (void*)e_partial, (void*)e_out})
        if (p) hipFree(p);
    at = nullptr;
    queue = nullptr;
    e_partial = nullptr;
    e_out = nullptr;
}

size_t Scratch::bytes() const {
    if (!at) return 0;
    return 512 + sizeof(double) * kEnergyTerms * (kEnergyBlocks + 1);
}

hipEvent_t WarpTimers::get() {
    if (used == pool.size()) {
        hipEvent_t e;
        hipEventCreate(&e);
        pool.push_back(e);
    }
    return pool[used++];
}

void WarpTimers::reset() {
    pairs.clear();
    used = 0;
    for (auto& l : iters) l = 0;
    for (auto& l : kernels) l = 0;
}

void WarpTimers::begin(int level, hipStream_t s) {
    Pair p{get(), get(), level};
    hipEventRecord(p.a, s);
    pairs.push_back(p);
}

void WarpTimers::end(int level, hipStream_t s) {
    (void)level;
    hipEventRecord(pairs.back().b, s);
}

WarpTimers::~WarpTimers() {
    for (auto e : pool) hipEventDestroy(e);
}

void fill_result(const double* h, flow_result* r) {
    if (!r) return;
    r->tv = h[0];
    r->data = h[1];
    r->energy = h[0] + h[1];
    r->dual = h[2];
    r->gap = r->energy - r->dual;
    r->residual = std::sqrt(h[3]);
}

flow_status StopTest::check(Scratch& sc, hipStream_t s, bool* converged) {
    HIP_TRY(hipMemcpyAsync(host, sc.e_out, sizeof(double) * kEnergyTerms, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double energy = host[0] + host[1];
    const double gap = energy - host[2];
    *converged = std::isfinite(gap) && energy > 0 && std::fabs(gap) <= tol * energy;
    return FLOW_OK;
}

std::string graph_key(int H, int W, const flow_params& p, const void* arena, int tune_epoch) {
    std::ostringstream o;
    o.precision(17);
    o << H << ',' << W << ',' << p.scheme << ',' << p.lambda << ',' << p.beta << ',' << p.c << ',' << p.relax << ','
      << p.sigma << ',' << p.tau << ',' << p.gs_sweeps << ',' << p.intensity_scale << ',' << p.levels << ','
      << p.warps << ',' << p.iters << ',' << p.storage << ',' << arena << ",tb" << g_tb_mode << ',' << g_tb_k
      << ",rows" << g_admm_rows_override << ",pdr" << g_pdr_mode << ',' << g_pdr_k << ",te" << tune_epoch;
    return o.str();
}

flow_status OpScratch::ensure() {
    if (!e_partial) {
        HIP_TRY(hipMalloc(&e_partial, sizeof(double) * kEnergyTerms * kEnergyBlocks));
        HIP_TRY(hipMalloc(&e_out, sizeof(double) * kEnergyTerms));
    }
    return FLOW_OK;
}

OpScratch& op_scratch() {
    static std::map<int, OpScratch> per_device;
    int dev = 0;
    hipGetDevice(&dev);
    return per_device[dev];
}

}  // namespace flowmi

using namespace flowmi;

flow_status flow_ctx::init_scratch() {
    HIP_TRY(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipHostMalloc((void**)&host_out, sizeof(double) * kEnergyTerms * 2, hipHostMallocDefault));
    HIP_TRY(hipEventCreate(&ev_total[0]));
    HIP_TRY(hipEventCreate(&ev_total[1]));
    return scratch.alloc();
}

size_t flow_ctx::bytes_in_use() const { return arena.bytes + scratch.bytes() + flowmi::batch_bytes(batch); }

void flow_ctx::drop_graphs() {
    for (auto& kv : graphs) {
        if (kv.second.exec) hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) hipGraphDestroy(kv.second.graph);
    }
    graphs.clear();
    plans.clear();
}

flow_status flow_ctx::ensure_arena(size_t need) {
    if (arena.bytes >= need) return FLOW_OK;
    if (budget && need + scratch.bytes() + batch_bytes(batch) > budget)
        return fail(FLOW_E_NOMEM, "working set of " + std::to_string(need) + " bytes exceeds the HBM budget");
    drop_graphs();
    if (arena.base) {
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipFree(arena.base));
        arena.base = nullptr;
        arena.bytes = 0;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, need);
    if (e != hipSuccess) return fail(FLOW_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    arena.base = p;
    arena.bytes = need;
    return FLOW_OK;
}

flow_status flow_ctx::solve(const float* I0, const float* I1, int H, int W, int64_t ld, const flow_params& p,
                            float* u, float* v, int64_t ld_uv, flow_result* res, hipStream_t s) {
    const bool f16 = p.storage == FLOW_STORE_F16;
    flow_status st = ensure_arena(layout_bytes(H, W, p));
    if (st != FLOW_OK) return st;
    std::vector<LevelPlanes> Ls;
    st = build_layout(arena, H, W, p, Ls);
    if (st != FLOW_OK) return st;

    launch_import(I0, H, W, ld, Ls[0].I0, Ls[0].ld, f16, s);
    launch_import(I1, H, W, ld, Ls[0].I1, Ls[0].ld, f16, s);
    if (stats_enabled) HIP_TRY(hipEventRecord(ev_total[0], s));

    const bool use_graph = p.use_graph && p.tol == 0.0;
    const std::string key = graph_key(H, W, p, arena.base, tune_epoch);
    auto pit = plans.find(key);
    if (pit == plans.end()) {
        std::unique_ptr<SolvePlan> plan(new SolvePlan());
        st = make_plan(Ls, p, scratch, *plan, &tuned);
        if (st != FLOW_OK) return st;
        pit = plans.emplace(key, std::move(plan)).first;
    }
    const SolvePlan* plan = pit->second.get();
    int final_buf = 0;
    bool replayed = false;
    timers.reset();
    if (use_graph) {
        auto it = graphs.find(key);
        if (it == graphs.end()) {
            GraphEntry g;
            HIP_TRY(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
            flow_status cst = enqueue_core(Ls, p, scratch, cap_stream, nullptr, nullptr, plan);
            hipGraph_t graph = nullptr;
            hipError_t ee = hipStreamEndCapture(cap_stream, &graph);
            if (cst != FLOW_OK) {
                if (graph) hipGraphDestroy(graph);
                return cst;
            }
            if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
            g.graph = graph;
            HIP_TRY(hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0));
            g.final_buf = scratch.final_buf;
            it = graphs.emplace(key, g).first;
        }
        HIP_TRY(hipGraphLaunch(it->second.exec, s));
        final_buf = it->second.final_buf;
        replayed = true;
    } else {
        StopTest stop;
        stop.tol = p.tol;
        stop.host = host_out + kEnergyTerms;
        st = enqueue_core(Ls, p, scratch, s, stats_enabled ? &timers : nullptr, p.tol > 0 ? &stop : nullptr, plan);
        if (st != FLOW_OK) return st;
        final_buf = scratch.final_buf;
    }
    if (stats_enabled) HIP_TRY(hipEventRecord(ev_total[1], s));

    launch_copy2d(level_flow(Ls[0], p, 1, final_buf), H, W, Ls[0].ld, u, ld_uv, s, level_inc(Ls[0], p, 1, final_buf));
    launch_copy2d(level_flow(Ls[0], p, 2, final_buf), H, W, Ls[0].ld, v, ld_uv, s, level_inc(Ls[0], p, 2, final_buf));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(host_out, scratch.e_out, sizeof(double) * kEnergyTerms, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));

    if (stats_enabled) {
        flow_stats S{};
        S.levels = (int)Ls.size();
        int64_t pxi = 0;
        for (int l = 0; l < S.levels; ++l) {
            S.H[l] = Ls[l].H;
            S.level_px[l] = (int64_t)Ls[l].H * Ls[l].W;
            S.W[l] = Ls[l].W;
            S.iterations[l] = replayed ? (int64_t)p.warps * p.iters : timers.iters[l];
            S.launches[l] = replayed ? 0 : timers.kernels[l];
            pxi += (int64_t)Ls[l].H * Ls[l].W * S.iterations[l];
        }
        for (auto& pr : timers.pairs) {
            float ms = 0.f;
            hipEventElapsedTime(&ms, pr.a, pr.b);
            S.iter_ms[pr.level] += ms;
        }
        float tot = 0.f;
        hipEventElapsedTime(&tot, ev_total[0], ev_total[1]);
        S.total_ms = tot;
        S.px_iter = pxi;
        S.graph_replayed = replayed ? 1 : 0;
        last_stats = S;
    }
    fill_result(host_out, res);
    if (!std::isfinite(host_out[0] + host_out[1]) || !std::isfinite(host_out[2]) || host_out[7] != 0.0)
        return fail(FLOW_E_NONFINITE, "energy or gap is not finite");
    return FLOW_OK;
}

flow_ctx::~flow_ctx() {
    hipDeviceSynchronize();
    flowmi::destroy_batch(batch);
    drop_graphs();
    if (arena.base) hipFree(arena.base);
    scratch.release();
    if (host_out) hipHostFree(host_out);
    if (cap_stream) hipStreamDestroy(cap_stream);
    for (auto e : ev_total)
        if (e) hipEventDestroy(e);
}
