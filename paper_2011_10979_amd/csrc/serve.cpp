// Serving engine: continuous batching of frame pairs that arrive over time.
//
// Requests are queued on submit and admitted, in arrival order, when a slot (at most max_active
// pairs in flight) and room in the engine's HBM arena (first-fit, the pair's whole working set)
// are free.  Each call to flow_server_step runs one epoch: every admitted pair advances by one warp
// of its coarse-to-fine solve (Sec. 4) -- level start where due, linearisation (which commits the
// previous warp's increment), the warp's iterations -- and all pairs share each launch: item tables map work-groups to pairs for
// the elementwise steps, and one K-iteration tile launch covers the tiles of every pair's current
// level.  Newly admitted pairs are imported and get their pyramids in the same epoch.  A pair that
// finishes level 0 has its energy computed and its flow exported in that epoch; its memory and slot
// are released once the epoch's event has completed.  Pairs at different levels and warps share
// launches, so a pair's arithmetic is the same as alone (each pair has its own a~ slots, energy
// partials and state direction; the K of a launch only decides how far tile halos are recomputed):
// a served result is bitwise the same alone or in any mix.
//
// Epochs are double-buffered: the host builds epoch e + 1's tables while the device runs epoch e,
// and blocks only when it needs epoch e - 1's buffers again.  An epoch's K-iteration tile launches
// (about iters / K of them, the bulk of its launches) are replayed from a captured graph: the tile
// count, the level descriptors and the tiles sit at fixed offsets of the buffer set's table, the
// kernels read the tile count there, and the launches use a fixed persistent grid, so one graph
// per buffer set and stage choice (K, order, width) serves every epoch; the few elementwise
// launches, whose grids follow the epoch's item tables, stay direct.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "multi.hpp"
#include "runtime.hpp"

namespace flowmi {

int g_serve_graph = 1;

#define HIP_TRY(expr)                                           \
    do {                                                        \
        hipError_t _e = (expr);                                 \
        if (_e != hipSuccess) return hip_fail(_e, #expr);       \
    } while (0)

namespace {

struct Req {
    flow_pair q{};
    int levels = 0;
    size_t bytes = 0;
    size_t off = 0;
    int slot = -1;
    std::vector<LevelPlanes> L;
    int l = 0, w = 0;          // cursor: next warp w of level l
    int cur = 0;               // state buffer holding the current iterate
    int cur_coarse = 0;        // state buffer of the finished coarser level
    bool imported = false;
    bool done = false;
    flow_status status = FLOW_OK;
};

struct Epoch {
    hipEvent_t ev = nullptr;
    bool in_flight = false;
    std::vector<uint64_t> finishing;
};

}  // namespace

}  // namespace flowmi

using namespace flowmi;

struct flow_server {
    int device = 0;
    flow_params p{};
    hipStream_t s = nullptr;
    int max_active = 0;
    DevArena arena;
    RangeAlloc ralloc;
    size_t bytes_in_use = 0;
    DevBuf dyn;                    // a~ slots, energy partials and sums per slot, queue counters
    size_t at_off = 0, epart_off = 0, eout_off = 0, cnt_off = 0;
    DevBuf tab[2];
    PinnedBuf htab[2], he[2];
    // fixed offsets in an epoch's table: the tile count at 0, the level descriptors at kDescsAt
    // (room for two per pair in flight), the tiles at tiles_at()
    static constexpr size_t kDescsAt = 256;
    static constexpr size_t kDescBytes = sizeof(TbLevel) > sizeof(PdrTbLevel) ? sizeof(TbLevel) : sizeof(PdrTbLevel);
    size_t tiles_at() const {
        return (kDescsAt + kDescBytes * 2 * (size_t)max_active + 255) & ~(size_t)255;
    }
    hipStream_t cs = nullptr;      // capture stream (default priority)
    struct TileGraph {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::map<std::tuple<int, int, int, int, int, int>, TileGraph> graphs[2];   // (K, order, ew, code, launches, grid)
    void drop_graphs(int b);
    flow_status tile_launches(int b, const StageChoice& ch, int ntiles, int lpw, unsigned* d_cnt);
    Epoch ep[2];
    std::deque<uint64_t> queue;
    std::map<uint64_t, Req> reqs;
    std::vector<uint64_t> active;
    std::vector<int> free_slots;
    uint64_t next_ticket = 1;
    flow_server_stats st{};

    flow_status init(const flow_params& prm, size_t budget, int maxa, hipStream_t stream);
    flow_status retire(int b);
    flow_status admit();
    flow_status step(int32_t* n_active, int32_t* n_queued);
    ~flow_server();
};

flow_status flow_server::init(const flow_params& prm, size_t budget, int maxa, hipStream_t stream) {
    p = prm;
    s = stream;
    max_active = maxa;
    void* a = nullptr;
    hipError_t e = hipMalloc(&a, budget);
    if (e != hipSuccess) return fail(FLOW_E_NOMEM, std::string("hipMalloc(serving arena): ") + hipGetErrorString(e));
    arena.base = a;
    arena.bytes = budget;
    ralloc.reset(budget);
    size_t o = 0;
    auto take = [&](size_t b) { const size_t r = o; o = (o + b + 255) & ~(size_t)255; return r; };
    at_off = take(sizeof(float) * 2 * maxa);
    epart_off = take(sizeof(double) * kEnergyTerms * kEnergyBlocks * maxa);
    eout_off = take(sizeof(double) * kEnergyTerms * maxa);
    cnt_off = take(sizeof(unsigned) * 2 * std::max(1, p.iters) * kNq);
    flow_status r = dyn.ensure(o, "serving scalars");
    if (r != FLOW_OK) return r;
    for (int b = 0; b < 2; ++b) {
        HIP_TRY(hipEventCreateWithFlags(&ep[b].ev, hipEventDisableTiming));
        r = he[b].ensure(sizeof(double) * kEnergyTerms * maxa);
        if (r != FLOW_OK) return r;
    }
    for (int k = maxa - 1; k >= 0; --k) free_slots.push_back(k);
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    st.arena_bytes = budget;
    return FLOW_OK;
}

void flow_server::drop_graphs(int b) {
    for (auto& kv : graphs[b]) {
        if (kv.second.exec) hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) hipGraphDestroy(kv.second.graph);
    }
    graphs[b].clear();
}

// The epoch's tile launches over the tables of buffer set b (already uploaded on s): replayed from
// the graph of this stage choice, captured on first use, or launched directly.
flow_status flow_server::tile_launches(int b, const StageChoice& ch, int ntiles, int lpw, unsigned* d_cnt) {
    const TbTile* tiles = (const TbTile*)(tab[b].d + tiles_at());
    const TbLevel* descs = (const TbLevel*)(tab[b].d + kDescsAt);
    if (!g_serve_graph) {
        if (ch.order == ORDER_QUEUE) launch_reset_u32(d_cnt, lpw * kNq, s);
        enqueue_tile_warp(tiles, ntiles, tile_grid(ch, ntiles), descs, ch, p, 0, 0, d_cnt, s);
        return FLOW_OK;
    }
    // the grid: 512 work-groups (two of 1024 threads per CU) pulling from the queues, or for table
    // order one work-group per tile, rounded up to a power of two (at least 64) so that a few
    // graphs cover every table size and at most half of a launch's work-groups exit at once
    int grid = 512;
    if (ch.order != ORDER_QUEUE) {
        grid = 64;
        while (grid < ntiles) grid *= 2;
    }
    const auto key = std::make_tuple(ch.K, ch.order, ch.ew, ch.tnt, lpw, grid);
    auto it = graphs[b].find(key);
    if (it == graphs[b].end()) {
        TileGraph g;
        HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        if (ch.order == ORDER_QUEUE) launch_reset_u32(d_cnt, lpw * kNq, cs);
        enqueue_tile_warp(tiles, 0, grid, descs, ch, p, 0, 0, d_cnt, cs, (const int*)tab[b].d);
        hipError_t e = hipStreamEndCapture(cs, &g.graph);
        if (e != hipSuccess) {
            if (g.graph) hipGraphDestroy(g.graph);
            return hip_fail(e, "hipStreamEndCapture(serving tile launches)");
        }
        e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            hipGraphDestroy(g.graph);
            return hip_fail(e, "hipGraphInstantiate(serving tile launches)");
        }
        it = graphs[b].emplace(key, g).first;
        st.graphs_captured++;
    }
    HIP_TRY(hipGraphLaunch(it->second.exec, s));
    return FLOW_OK;
}

flow_server::~flow_server() {
    if (s) hipStreamSynchronize(s);
    for (int b = 0; b < 2; ++b) drop_graphs(b);
    if (cs) hipStreamDestroy(cs);
    for (auto& x : ep)
        if (x.ev) hipEventDestroy(x.ev);
    if (arena.base) hipFree(arena.base);
    dyn.release();
    for (int b = 0; b < 2; ++b) {
        tab[b].release();
        htab[b].release();
        he[b].release();
    }
}

// Epoch b has completed on the device: results of its finishing pairs, memory and slots back.
flow_status flow_server::retire(int b) {
    Epoch& E = ep[b];
    if (!E.in_flight) return FLOW_OK;
    HIP_TRY(hipEventSynchronize(E.ev));
    const double* h = (const double*)he[b].h;
    for (uint64_t t : E.finishing) {
        Req& r = reqs[t];
        const double* e = h + (size_t)r.slot * kEnergyTerms;
        fill_result(e, r.q.res);
        if (!std::isfinite(e[0] + e[1]) || !std::isfinite(e[2]) || e[7] != 0.0) r.status = FLOW_E_NONFINITE;
        r.done = true;
        ralloc.release(r.off, r.bytes);
        bytes_in_use -= r.bytes;
        free_slots.push_back(r.slot);
        r.L.clear();
        st.completed++;
    }
    E.finishing.clear();
    E.in_flight = false;
    return FLOW_OK;
}

flow_status flow_server::admit() {
    while (!queue.empty() && (int)active.size() < max_active && !free_slots.empty()) {
        Req& r = reqs[queue.front()];
        size_t off = 0;
        if (!ralloc.alloc(r.bytes, off)) break;   // arrival order: later requests wait behind this one
        flow_params pk = p;
        pk.levels = r.levels;
        DevArena sub{(char*)arena.base + off, r.bytes};
        flow_status rs = build_layout(sub, r.q.H, r.q.W, pk, r.L);
        if (rs != FLOW_OK) {
            ralloc.release(off, r.bytes);
            return rs;
        }
        r.off = off;
        r.slot = free_slots.back();
        free_slots.pop_back();
        r.l = r.levels - 1;
        r.w = 0;
        r.cur = 0;
        r.imported = false;
        bytes_in_use += r.bytes;
        st.peak_bytes_in_use = std::max(st.peak_bytes_in_use, bytes_in_use);
        active.push_back(queue.front());
        queue.pop_front();
        st.admitted++;
    }
    st.peak_active = std::max<int32_t>(st.peak_active, (int32_t)active.size());
    return FLOW_OK;
}

static void run_items(BatchOp op, const char* base, const BLaunch& L, bool f16, hipStream_t s) {
    if (L.n > 0) launch_batched(op, base + L.items, (const int*)(base + L.off), L.n, L.total, f16, s);
}

flow_status flow_server::step(int32_t* n_active, int32_t* n_queued) {
    const int b = (int)(st.epochs & 1);
    flow_status r = retire(b);                                   // the epoch that used these buffers
    if (r != FLOW_OK) return r;
    if (ep[b ^ 1].in_flight && hipEventQuery(ep[b ^ 1].ev) == hipSuccess) {
        r = retire(b ^ 1);
        if (r != FLOW_OK) return r;
    }
    r = admit();
    if (r != FLOW_OK) return r;
    if (active.empty() && !queue.empty() && ep[b ^ 1].in_flight) {
        r = retire(b ^ 1);                                       // memory held by finishing pairs
        if (r == FLOW_OK) r = admit();
        if (r != FLOW_OK) return r;
    }
    if (active.empty()) {
        if (n_active) *n_active = 0;
        if (n_queued) *n_queued = (int32_t)queue.size();
        return FLOW_OK;
    }
    const bool hw = p.beta > 0;
    const bool f16 = p.storage == FLOW_STORE_F16;
    float* d_at = (float*)(dyn.d + at_off);
    double* d_epart = (double*)(dyn.d + epart_off);
    double* d_eout = (double*)(dyn.d + eout_off);
    unsigned* d_cnt = (unsigned*)(dyn.d + cnt_off) + (size_t)b * std::max(1, p.iters) * kNq;

    // ---- tables of this epoch
    std::vector<CopyArgs> imp;
    std::vector<int> imp_bl;
    std::vector<DerivArgs> der;
    std::vector<int> der_bl;
    int lmax_new = 0;
    for (uint64_t t : active) {
        Req& q = reqs[t];
        if (q.imported) continue;
        const LevelPlanes& L0 = q.L[0];
        const float off = f16 ? kFrameOffsetF16 : 0.f;
        imp.push_back(CopyArgs{q.q.I0, q.q.H, q.q.W, q.q.ld, L0.I0, L0.ld, off});
        imp.push_back(CopyArgs{q.q.I1, q.q.H, q.q.W, q.q.ld, L0.I1, L0.ld, off});
        imp_bl.push_back(blocks_of(q.q.H, q.q.W));
        imp_bl.push_back(blocks_of(q.q.H, q.q.W));
        lmax_new = std::max(lmax_new, q.levels);
        for (const LevelPlanes& L : q.L) {
            der.push_back(DerivArgs{L.I1, L.H, L.W, L.ld, L.Dx, L.Dy, L.ld, L.I1lo});
            der_bl.push_back(blocks_of(L.H, L.W));
        }
    }
    std::vector<std::vector<DownArgs>> down(std::max(1, lmax_new));
    std::vector<std::vector<int>> down_bl(std::max(1, lmax_new));
    for (int l = 1; l < lmax_new; ++l) {
        for (uint64_t t : active) {
            Req& q = reqs[t];
            if (q.imported || q.levels <= l) continue;
            const LevelPlanes& F = q.L[l - 1];
            const LevelPlanes& C = q.L[l];
            down[l].push_back(DownArgs{F.I0, F.H, F.W, F.ld, C.I0, C.ld, F.I0lo, C.I0lo});
            down[l].push_back(DownArgs{F.I1, F.H, F.W, F.ld, C.I1, C.ld, F.I1lo, C.I1lo});
            down_bl[l].push_back(blocks_of(C.H, C.W));
            down_bl[l].push_back(blocks_of(C.H, C.W));
        }
    }

    Shapes shapes;
    for (uint64_t t : active) {
        const LevelPlanes& L = reqs[t].L[reqs[t].l];
        shapes.emplace_back(L.H, L.W);
    }
    const bool pd = pd_state(p);
    StageChoice ch;
    if (!pd) {
        ch = default_stage_choice(shapes, hw, p.iters);
        if (g_batch_order >= 0) ch.order = g_batch_order;
        if (g_batch_ew > 0) ch.ew = g_batch_ew;
        if (g_batch_k > 0) ch.K = g_batch_k;
        if (g_batch_nt > 0) ch.tnt = g_batch_nt;
        ch = fit_stage_choice(ch, shapes, hw);
    } else {
        // pDR / ALG1: 1024-thread tiles; every admitted pair's levels take tiles at K = 1 (submit
        // checks it), so a K >= 1 exists
        ch.K = pd_shared_k(shapes, p);
        ch.nt = 1024;
        if (ch.K < 1) return fail(FLOW_E_INVAL, "a served level takes no pDR / ALG1 tiles");
    }
    const int lpw = launches_per_warp(p.iters, ch.K);

    std::vector<LevelInitArgs> init;
    std::vector<int> init_bl;
    std::vector<LinArgs> lin;
    std::vector<int> bl;
    std::vector<TbLevel> descs(pd ? 0 : 2 * active.size());
    std::vector<PdrTbLevel> pdescs(pd ? 2 * active.size() : 0);
    std::vector<TbTile> tiles;
    std::vector<EnergyArgs> en;
    std::vector<int> en_bl;
    std::vector<CopyArgs> exp;
    std::vector<int> exp_bl;
    std::vector<uint64_t> finishing;
    Scratch none;
    for (size_t i = 0; i < active.size(); ++i) {
        Req& q = reqs[active[i]];
        const int l = q.l;
        const LevelPlanes& L = q.L[l];
        float* at2 = d_at + 2 * q.slot;
        if (q.w == 0) {
            LevelInitArgs ia{};
            ia.H = L.H; ia.W = L.W; ia.ld = L.ld;
            if (l < q.levels - 1) {
                const LevelPlanes& C = q.L[l + 1];
                ia.uc = level_flow(C, p, 1, q.cur_coarse);
                ia.vc = level_flow(C, p, 2, q.cur_coarse);
                ia.ucd = level_inc(C, p, 1, q.cur_coarse);
                ia.vcd = level_inc(C, p, 2, q.cur_coarse);
                ia.wc = hw ? level_flow(C, p, 0, q.cur_coarse) : nullptr;
                ia.Hc = C.H; ia.Wc = C.W; ia.ldc = C.ld;
            }
            int nz = 0;
            if (!pd) {
                ia.set_flow[0] = hw ? L.st[0][0] : nullptr;
                ia.set_flow[1] = L.U0[0];
                ia.set_flow[2] = L.U0[1];
                for (int k = 3; k < 10; ++k)
                    if (L.st[0][k]) ia.zero[nz++] = L.st[0][k];
            } else {                            // X = X bar = the upsampled flow, y bar = 0, Theta = 0
                ia.set_flow[0] = hw ? L.Xs[0][0] : nullptr;
                ia.set_flow[1] = L.Xs[0][1];
                ia.set_flow[2] = L.Xs[0][2];
                ia.copy_flow[0] = hw ? L.Xbs[0][0] : nullptr;
                ia.copy_flow[1] = L.Xbs[0][1];
                ia.copy_flow[2] = L.Xbs[0][2];
                for (int k = 0; k < 6; ++k)
                    if (L.ybs[0][k]) ia.zero[nz++] = L.ybs[0][k];
                ia.zero[nz++] = L.s_out;
            }
            ia.nzero = nz;
            ia.clear_scalar = at2;
            init.push_back(ia);
            init_bl.push_back(blocks_of(L.H, L.W));
        }
        LinArgs la{};
        la.I0 = L.I0; la.I1 = L.I1; la.Dx = L.Dx; la.Dy = L.Dy;
        la.I0lo = L.I0lo; la.I1lo = L.I1lo;
        if (!pd) {
            la.u0 = L.U0[0];
            la.v0 = L.U0[1];
            if (q.w > 0) {                      // commit the previous warp's increment on the way
                la.pend_u = L.st[q.cur][1];
                la.pend_v = L.st[q.cur][2];
            }
            la.zero_u = L.st[q.cur][1];
            la.zero_v = L.st[q.cur][2];
        } else {                                // linearise around X; keep a copy of the point for I_t
            la.u0 = L.Xs[q.cur][1];
            la.v0 = L.Xs[q.cur][2];
            la.keep_u = L.U0[0];
            la.keep_v = L.U0[1];
        }
        la.Ix = L.Ix; la.Iy = L.Iy; la.It = L.It;
        la.at = at2 + (q.w & 1);
        la.at_clear = at2 + ((q.w + 1) & 1);
        la.H = L.H; la.W = L.W; la.ld = L.ld;
        la.kappa = (float)p.intensity_scale;
        la.beta = (float)p.beta;
        la.rel = 1;
        lin.push_back(la);
        bl.push_back(lin_blocks_of(L.H, L.W));
        // descriptors in the pair's own direction: launch direction 0 reads state buffer q.cur
        if (!pd) {
            TbLevel d[2];
            fill_tb_level(d, L, at2 + (q.w & 1));
            descs[2 * i] = d[q.cur];
            descs[2 * i + 1] = d[q.cur ^ 1];
            level_tiles(L.H, L.W, hw, ch, (int)i, tiles);
        } else {
            PdrTbPlan one;
            one.th = one.tw = 1;
            pdescs[2 * i] = pdr_tb_args(L, p, one, q.cur, 1).lvl;
            pdescs[2 * i + 1] = pdr_tb_args(L, p, one, q.cur ^ 1, 1).lvl;
            const PdrTbPlan T = plan_pd_tiles(L.H, L.W, hw, pd_halo(p, std::min(ch.K, 64)), ch.K, 0, 1024);
            if (!T.tb) return fail(FLOW_E_INVAL, "a served level takes no pDR / ALG1 tiles");
            for (int y = 0; y < L.H; y += T.th)
                for (int x = 0; x < L.W; x += T.tw)
                    tiles.push_back(TbTile{(int)i, y, x, std::min(T.th, L.H - y), std::min(T.tw, L.W - x)});
        }
        const int after = q.cur ^ (lpw & 1);
        if (l == 0 && q.w == p.warps - 1) {
            EnergyArgs e = energy_args(L, p, after, none);
            e.partial = d_epart + (size_t)q.slot * kEnergyTerms * kEnergyBlocks;
            e.out = d_eout + (size_t)q.slot * kEnergyTerms;
            en.push_back(e);
            en_bl.push_back(energy_blocks(L.H, L.W));
            exp.push_back(CopyArgs{level_flow(L, p, 1, after), L.H, L.W, L.ld, q.q.u, q.q.ld_uv, 0.f,
                                   level_inc(L, p, 1, after)});
            exp.push_back(CopyArgs{level_flow(L, p, 2, after), L.H, L.W, L.ld, q.q.v, q.q.ld_uv, 0.f,
                                   level_inc(L, p, 2, after)});
            exp_bl.push_back(blocks_of(L.H, L.W));
            exp_bl.push_back(blocks_of(L.H, L.W));
            finishing.push_back(active[i]);
        }
    }
    // The epoch's table, one upload: [tile count | level descriptors (room for max_active pairs) |
    // tiles | item tables].  The first three sit at the same offsets in every epoch, which the
    // graphs of the tile launches rely on; a table buffer that has to grow moves, and the graphs
    // recorded over the old one are dropped.
    const int ntiles = (int)tiles.size();
    TableBuilder T;
    T.h.assign(tiles_at(), 0);
    std::memcpy(T.h.data(), &ntiles, sizeof(int));
    if (!pd) std::memcpy(T.h.data() + kDescsAt, descs.data(), sizeof(TbLevel) * descs.size());
    else std::memcpy(T.h.data() + kDescsAt, pdescs.data(), sizeof(PdrTbLevel) * pdescs.size());
    const size_t tiles_off = T.put(tiles);
    const BLaunch l_imp = T.launch(imp, imp_bl);
    std::vector<BLaunch> l_down(std::max(1, lmax_new));
    for (int l = 1; l < lmax_new; ++l) l_down[l] = T.launch(down[l], down_bl[l]);
    const BLaunch l_der = T.launch(der, der_bl);
    const BLaunch l_init = T.launch(init, init_bl);
    const BLaunch l_lin = T.launch(lin, bl);
    const BLaunch l_en = T.launch(en, en_bl);
    const BLaunch l_exp = T.launch(exp, exp_bl);

    r = htab[b].ensure(T.h.size());
    if (r != FLOW_OK) return r;
    {
        const char* old = tab[b].d;
        r = tab[b].ensure(T.h.size(), "serving tables");
        if (r != FLOW_OK) return r;
        if (tab[b].d != old) drop_graphs(b);
    }
    std::memcpy(htab[b].h, T.h.data(), T.h.size());
    HIP_TRY(hipSetDevice(device));
    HIP_TRY(hipMemcpyAsync(tab[b].d, htab[b].h, T.h.size(), hipMemcpyHostToDevice, s));
    (void)tiles_off;   // == tiles_at(): T.h held exactly the aligned prefix before the put

    // ---- launches
    const char* tb = tab[b].d;
    run_items(BatchOp::Copy, tb, l_imp, f16, s);
    for (int l = 1; l < lmax_new; ++l) run_items(BatchOp::Downsample, tb, l_down[l], f16, s);
    run_items(BatchOp::Derivatives, tb, l_der, f16, s);
    run_items(BatchOp::LevelInit, tb, l_init, false, s);
    run_items(BatchOp::Linearize, tb, l_lin, f16, s);
    if (!pd) {
        r = tile_launches(b, ch, ntiles, lpw, d_cnt);
        if (r != FLOW_OK) return r;
    } else if (ntiles > 0) {
        // pDR / ALG1 tile launches, direct: direction 0 reads each pair's current state buffer
        PdrTbArgs a{};
        pd_tile_scalars(a, p);
        a.tiles = (const TbTile*)(tb + tiles_at());
        a.ntiles = ntiles;
        a.levels = (const PdrTbLevel*)(tb + kDescsAt);
        int dir = 0;
        for (int k = 0; k < p.iters;) {
            a.K = std::min(ch.K, p.iters - k);
            a.dir = dir;
            if (p.scheme == FLOW_ALG1) launch_alg1_tb(a, hw, ch.nt, s);
            else launch_pdr_tb(a, hw, ch.nt, s);
            dir ^= 1;
            k += a.K;
        }
    }
    if (l_en.n > 0)
        launch_energy_batched((const EnergyArgs*)(tb + l_en.items), (const int*)(tb + l_en.off), l_en.n, l_en.total, s);
    run_items(BatchOp::Copy, tb, l_exp, false, s);
    if (!finishing.empty())
        HIP_TRY(hipMemcpyAsync(he[b].h, d_eout, sizeof(double) * kEnergyTerms * max_active, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(ep[b].ev, s));
    ep[b].in_flight = true;
    ep[b].finishing = finishing;

    // ---- cursors
    std::vector<uint64_t> still;
    for (uint64_t t : active) {
        Req& q = reqs[t];
        q.imported = true;
        q.cur ^= lpw & 1;
        if (++q.w == p.warps) {
            q.w = 0;
            if (q.l == 0) continue;            // finished: results once this epoch completes
            q.cur_coarse = q.cur;
            q.cur = 0;
            --q.l;
        }
        still.push_back(t);
    }
    active.swap(still);
    st.epochs++;
    if (n_active) *n_active = (int32_t)active.size();
    if (n_queued) *n_queued = (int32_t)queue.size();
    return FLOW_OK;
}

extern "C" {

flow_status flow_server_create(flow_ctx* ctx, const flow_params* p, size_t hbm_budget, int32_t max_active,
                               void* stream, flow_server** out) {
    if (!ctx || !out) return fail(FLOW_E_INVAL, "NULL argument");
    *out = nullptr;
    flow_status r = validate(p);
    if (r != FLOW_OK) return r;
    if (p->tol > 0) return fail(FLOW_E_INVAL, "the serving engine runs a fixed iteration count (tol = 0)");
    if (max_active < 1 || max_active > 4096) return fail(FLOW_E_INVAL, "max_active must be in [1, 4096]");
    if (hbm_budget == 0) hbm_budget = (size_t)8 << 30;
    HIP_TRY(hipSetDevice(ctx->device));
    std::unique_ptr<flow_server> srv(new flow_server());
    srv->device = ctx->device;
    r = srv->init(*p, hbm_budget, max_active, (hipStream_t)stream);
    if (r != FLOW_OK) return r;
    *out = srv.release();
    return FLOW_OK;
}

flow_status flow_working_set_bytes(int32_t H, int32_t W, const flow_params* p, int32_t levels, uint64_t* bytes) {
    if (!bytes) return fail(FLOW_E_INVAL, "bytes is NULL");
    flow_status r = validate(p);
    if (r != FLOW_OK) return r;
    if (levels < 0 || levels > FLOW_MAX_LEVELS) return fail(FLOW_E_INVAL, "levels out of range");
    flow_params pk = *p;
    if (levels > 0) pk.levels = levels;
    r = validate_shape(H, W, W, pk.levels);
    if (r != FLOW_OK) return r;
    *bytes = (layout_bytes(H, W, pk) + 255) & ~(size_t)255;
    return FLOW_OK;
}

flow_status flow_server_destroy(flow_server* srv) {
    if (!srv) return FLOW_OK;
    hipSetDevice(srv->device);
    delete srv;
    return FLOW_OK;
}

flow_status flow_server_submit(flow_server* srv, const flow_pair* pair, uint64_t* ticket) {
    if (!srv || !pair || !ticket) return fail(FLOW_E_INVAL, "NULL argument");
    HIP_TRY(hipSetDevice(srv->device));
    flow_status r = validate_pair(*pair, srv->p, "");
    if (r != FLOW_OK) return r;
    Req q;
    q.q = *pair;
    q.levels = pair->levels > 0 ? pair->levels : srv->p.levels;
    flow_params pk = srv->p;
    pk.levels = q.levels;
    if (pd_state(pk) && !pd_pair_tileable(pair->H, pair->W, q.levels, pk))
        return fail(FLOW_E_INVAL, "the pDR halo of this many sweeps outgrows a tile at some level of the pair");
    q.bytes = (layout_bytes(pair->H, pair->W, pk) + 255) & ~(size_t)255;
    if (q.bytes > srv->arena.bytes)
        return fail(FLOW_E_NOMEM, "pair working set of " + std::to_string(q.bytes) + " bytes exceeds the serving budget");
    const uint64_t t = srv->next_ticket++;
    srv->reqs.emplace(t, std::move(q));
    srv->queue.push_back(t);
    srv->st.submitted++;
    *ticket = t;
    return FLOW_OK;
}

flow_status flow_server_step(flow_server* srv, int32_t* active, int32_t* queued) {
    if (!srv) return fail(FLOW_E_INVAL, "server is NULL");
    HIP_TRY(hipSetDevice(srv->device));
    return srv->step(active, queued);
}

flow_status flow_server_poll(flow_server* srv, uint64_t ticket, int32_t* done) {
    if (!srv || !done) return fail(FLOW_E_INVAL, "NULL argument");
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return fail(FLOW_E_NOTFOUND, "unknown or already collected ticket");
    for (int b = 0; b < 2 && !it->second.done; ++b) {
        // a finishing epoch that has completed on the device hands its results over now
        Epoch& E = srv->ep[b];
        if (E.in_flight && hipEventQuery(E.ev) == hipSuccess) {
            flow_status r = srv->retire(b);
            if (r != FLOW_OK) return r;
        }
    }
    *done = it->second.done ? 1 : 0;
    if (!it->second.done) return FLOW_OK;
    const flow_status st = it->second.status;
    srv->reqs.erase(it);
    if (st != FLOW_OK) return fail(st, "non-finite energy or gap");
    return FLOW_OK;
}

flow_status flow_server_drain(flow_server* srv) {
    if (!srv) return fail(FLOW_E_INVAL, "server is NULL");
    HIP_TRY(hipSetDevice(srv->device));
    int32_t a = 0, q = 0;
    do {
        flow_status r = srv->step(&a, &q);
        if (r != FLOW_OK) return r;
    } while (a > 0 || q > 0);
    for (int b = 0; b < 2; ++b) {
        flow_status r = srv->retire(b);
        if (r != FLOW_OK) return r;
    }
    return FLOW_OK;
}

flow_status flow_server_get_stats(const flow_server* srv, flow_server_stats* out) {
    if (!srv || !out) return fail(FLOW_E_INVAL, "NULL argument");
    *out = srv->st;
    out->active = (int32_t)srv->active.size();
    out->queued = (int32_t)srv->queue.size();
    out->bytes_in_use = srv->bytes_in_use;
    return FLOW_OK;
}

}  // extern "C"
