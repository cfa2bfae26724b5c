// Batched solve of many pairs of uneven sizes on one GPU: the coarse-to-fine solve of Sec. 4 for
// every pair, advanced together.  Stage s works on pyramid level l = Lmax-1-s of every pair that has
// it, so all pairs reach level 0 in the last stage.  Every step of a stage is ONE launch over all
// its pairs: the elementwise steps (import, downsample, derivatives, level start, linearisation,
// energy, export) through item tables in which a block-offset prefix maps each work-group
// to its pair, and each block of K iterations through the K-iteration tile kernel over a table of
// (pair-level, tile) entries, taken in XCD order or drained from per-XCD work queues.
//
// Determinism: a pair's arithmetic never depends on the other pairs of the batch (each pair has
// its own a~ slots and energy partials, every tile is computed by the same kernel instantiation, and
// the K of a launch only decides how far a tile's halo is recomputed), so a pair's results are
// bitwise the same alone or in any batch, for any stage choice.
//
// pDR and ALG1 (state X, X bar, y bar) take the same stages with their own tile kernels in table
// order: 1024-thread tiles with one red and one black cell per thread (ALG1: its own tiles), the
// plain path's built-in K per launch, or the whole warp in one launch where every level of the
// stage fits one tile.  Every pDR tile shape and K computes each cell with the same expressions, so
// a batched pDR pair is bitwise the plain pDR tile solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

#include "multi.hpp"
#include "runtime.hpp"

namespace flowmi {

#define HIP_TRY(expr)                                           \
    do {                                                        \
        hipError_t _e = (expr);                                 \
        if (_e != hipSuccess) return hip_fail(_e, #expr);       \
    } while (0)

// One stage: pyramid level l of every pair that has it.
struct BStage {
    int l = 0;                          // pyramid level (0 = finest)
    std::vector<int> pairs;             // pairs that have level l
    std::string key;                    // level shapes of the stage (tuning key)
    StageChoice ch;
    int lpw = 0;                        // tile launches per warp
    int tile_off = 0, ntiles = 0, grid = 0;
    int counter_off = 0;                // first counter of the stage's queue launches
    bool pd = false;                    // pDR / ALG1 stage: tile kernels of that scheme, work-group code pd_nt
    int pd_nt = 1024;
    BLaunch init;
    std::vector<BLaunch> lin;           // per warp
};

// Working set and launch plan of one batch composition.
struct BatchPlan {
    std::string key;
    int n = 0, lmax = 0;
    std::vector<int> H, W, levels;
    std::vector<std::vector<LevelPlanes>> L;   // [pair][level]
    std::vector<BStage> stages;                // coarsest first
    std::vector<BLaunch> down;                 // [level], level >= 1
    BLaunch deriv, energy;
    int ncounters = 0;
    int final_cur = 0;                         // state buffer of the level-0 result
    // device scalars (in BatchState::dyn): a~ slots, energy partials and sums, queue counters
    size_t at_off = 0, epart_off = 0, eout_off = 0, cnt_off = 0, dyn_bytes = 0;
    size_t descs_off = 0, tiles_off = 0;       // tile-kernel tables in BatchState::tab
    size_t pdescs_off = 0;                     // pDR / ALG1 level descriptors in BatchState::tab
    BLaunch imp, exp;                          // import / export launches in BatchState::io
    size_t io_bytes = 0;
};

struct BatchState {
    DevArena arena;
    DevBuf dyn, tab, io;
    PinnedBuf h_io, h_e;
    std::unique_ptr<BatchPlan> plan;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string graph_key;
    std::map<std::string, StageChoice> tuned;  // per stage key
    int tune_epoch = 0;
    std::vector<hipEvent_t> ev;                // stage timers of instrumented solves

    void drop_graph() {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        graph_key.clear();
    }
    size_t bytes() const { return arena.bytes + dyn.bytes + tab.bytes + io.bytes; }
    ~BatchState() {
        hipDeviceSynchronize();
        drop_graph();
        if (arena.base) hipFree(arena.base);
        dyn.release();
        tab.release();
        io.release();
        h_io.release();
        h_e.release();
        for (auto e : ev) hipEventDestroy(e);
    }
};

void destroy_batch(BatchState* b) { delete b; }
size_t batch_bytes(const BatchState* b) { return b ? b->bytes() : 0; }

int g_batch_order = -1;
int g_batch_k = 0;
int g_batch_ew = 0;
int g_batch_nt = 0;

namespace {

std::string stage_key(const std::vector<std::pair<int, int>>& shapes, bool hw, int iters) {
    std::vector<std::pair<int, int>> s = shapes;
    std::sort(s.begin(), s.end());
    std::ostringstream o;
    o << (hw ? "w" : "") << "i" << iters << ":";
    for (auto& x : s) o << x.first << "x" << x.second << ",";
    return o.str();
}

Shapes stage_shapes(const BatchPlan& P, const BStage& S) {
    Shapes s;
    for (int k : S.pairs) s.emplace_back(P.L[k][S.l].H, P.L[k][S.l].W);
    return s;
}

bool stage_fits(const BatchPlan& P, const BStage& S, bool hw, int K, int ew, int nt) {
    return shapes_fit(stage_shapes(P, S), hw, K, ew, nt);
}

void stage_tiles(const BatchPlan& P, const BStage& S, bool hw, const StageChoice& ch,
                 const std::vector<int>& desc_id, std::vector<TbTile>& out) {
    for (int k : S.pairs)
        level_tiles(P.L[k][S.l].H, P.L[k][S.l].W, hw, ch, desc_id[k * FLOW_MAX_LEVELS + S.l], out);
}

}  // namespace

}  // namespace flowmi

using namespace flowmi;

namespace {

flow_status validate_pairs(int n, const flow_pair* pairs, const flow_params& p) {
    for (int k = 0; k < n; ++k) {
        flow_status st = validate_pair(pairs[k], p, "pair " + std::to_string(k) + ": ");
        if (st != FLOW_OK) return st;
    }
    return FLOW_OK;
}

std::string batch_key(int n, const flow_pair* pairs, const flow_params& p) {
    std::ostringstream o;
    o.precision(17);
    o << n << ";bo" << g_batch_order << ",bk" << g_batch_k << ",be" << g_batch_ew << ",bn" << g_batch_nt << ';' << p.scheme << ',' << p.lambda << ',' << p.beta << ',' << p.c << ',' << p.relax << ','
      << p.intensity_scale << ',' << p.levels << ',' << p.warps << ',' << p.iters << ',' << p.storage << ','
      << p.sigma << ',' << p.tau << ',' << p.gs_sweeps << ',' << p.alg1_tau << ',' << p.alg1_sigma << ';';
    for (int k = 0; k < n; ++k) o << pairs[k].H << 'x' << pairs[k].W << 'l' << pairs[k].levels << ',';
    return o.str();
}

// Tiles of pDR / ALG1 stage S for work-group code nt and K iterations per launch (levels that fit
// one tile take one); false if some level takes no tiles.
bool pd_stage_tiles(const BatchPlan& P, const BStage& S, const flow_params& p, int nt, int K,
                    const std::vector<int>& desc_id, std::vector<TbTile>& out) {
    const bool hw = p.beta > 0;
    std::vector<PdrTbPlan> plans;
    for (int k : S.pairs) {
        const LevelPlanes& L = P.L[k][S.l];
        plans.push_back(plan_pd_tiles(L.H, L.W, hw, pd_halo(p, std::min(K, 64)), K, 0, nt));
        if (!plans.back().tb) return false;
    }
    for (size_t i = 0; i < S.pairs.size(); ++i) {
        const int k = S.pairs[i];
        const LevelPlanes& L = P.L[k][S.l];
        const int th = plans[i].th, tw = plans[i].tw;
        for (int y = 0; y < L.H; y += th)
            for (int x = 0; x < L.W; x += tw) {
                TbTile t;
                t.level = desc_id[k * FLOW_MAX_LEVELS + S.l];
                t.y0 = y;
                t.x0 = x;
                t.th = std::min(th, L.H - y);
                t.tw = std::min(tw, L.W - x);
                out.push_back(t);
            }
    }
    return true;
}

// Every level of pDR / ALG1 stage S fits one tile of work-group code nt.
bool pd_stage_resident(const BatchPlan& P, const BStage& S, bool hw, int nt) {
    for (int k : S.pairs)
        if (!pd_fits(hw, nt, P.L[k][S.l].H, P.L[k][S.l].W)) return false;
    return true;
}

// Work-group codes a pDR / ALG1 stage may take: 1024 and 512 threads with one cell of each colour
// per thread; pDR also the wave-row tiles of 128 x 32 and 64 x 32 cells, and without the w block
// 1024 and 512 threads with two cells of each colour and the wave-row tiles of 128 x 48 and 64 x 48.
std::vector<int> pd_codes(const flow_params& p) {
    if (p.scheme == FLOW_PDR && !(p.beta > 0)) return {1024, 512, 2048, 513, 4098, 6145, 3074, 2050};
    if (p.scheme == FLOW_PDR) return {1024, 512, 4098, 2050};
    if (!(p.beta > 0)) return {1024, 512, 3074, 2050};              // ALG1
    return {1024, 512, 2050};
}

// pDR / ALG1 stage: the tuned choice (work-group code and K) where one is recorded for the stage's
// shapes and still fits, else 1024-thread tiles with the plain path's built-in K, lowered until
// every level takes tiles (the whole warp in one launch where every level fits one tile).
// Appends the stage's tiles; false if some level takes no tiles even at K = 1 (callers check
// beforehand with pd_batch_tileable).
bool plan_pd_stage(const BatchPlan& P, BStage& S, const flow_params& p, const std::vector<int>& desc_id,
                   const std::map<std::string, StageChoice>& tuned, std::vector<TbTile>& tiles) {
    const bool hw = p.beta > 0;
    S.pd = true;
    S.ch = StageChoice();
    S.tile_off = (int)tiles.size();
    auto it = tuned.find(S.key);
    bool ok = false;
    if (it != tuned.end()) {
        const std::vector<int> codes = pd_codes(p);
        if (std::find(codes.begin(), codes.end(), it->second.nt) != codes.end() &&
            pd_stage_tiles(P, S, p, it->second.nt, it->second.K, desc_id, tiles)) {
            S.ch = it->second;
            ok = true;
        } else {
            tiles.resize(S.tile_off);
        }
    }
    if (!ok) {
        S.ch.nt = 1024;
        S.ch.K = pd_stage_resident(P, S, hw, 1024) ? std::max(1, p.iters)
                                                   : (p.scheme == FLOW_ALG1 ? kAlg1DefaultK : kPdrDefaultK);
        for (;; --S.ch.K) {
            if (pd_stage_tiles(P, S, p, 1024, S.ch.K, desc_id, tiles)) {
                ok = true;
                break;
            }
            tiles.resize(S.tile_off);
            if (S.ch.K <= 1) break;
        }
        if (!ok) return false;
    }
    S.ch.order = ORDER_TABLE;
    S.pd_nt = S.ch.nt;
    S.lpw = launches_per_warp(p.iters, S.ch.K);
    S.ntiles = (int)tiles.size() - S.tile_off;
    S.grid = S.ntiles;
    return true;
}

// Every level of every pair takes pDR / ALG1 tiles at one iteration per launch (with many sweeps
// the pDR halo can outgrow a tile; such batches are solved as plain solves in turn).
bool pd_batch_tileable(int n, const flow_pair* pairs, const flow_params& p) {
    for (int k = 0; k < n; ++k)
        if (!pd_pair_tileable(pairs[k].H, pairs[k].W, pairs[k].levels > 0 ? pairs[k].levels : p.levels, p)) return false;
    return true;
}

// Lays the pairs out in the batch arena and builds every table of the launch sequence.
flow_status build_plan(flow_ctx* ctx, BatchState& B, int n, const flow_pair* pairs, const flow_params& p) {
    const bool hw = p.beta > 0;
    const bool pd = pd_state(p);
    const bool f16 = p.storage == FLOW_STORE_F16;
    std::unique_ptr<BatchPlan> P(new BatchPlan());
    P->key = batch_key(n, pairs, p);
    P->n = n;
    // arena: the pairs' working sets back to back
    std::vector<size_t> off(n + 1, 0);
    for (int k = 0; k < n; ++k) {
        flow_params pk = p;
        pk.levels = pairs[k].levels > 0 ? pairs[k].levels : p.levels;
        P->H.push_back(pairs[k].H);
        P->W.push_back(pairs[k].W);
        P->levels.push_back(pk.levels);
        off[k + 1] = off[k] + ((layout_bytes(pairs[k].H, pairs[k].W, pk) + 255) & ~(size_t)255);
    }
    const size_t need = off[n];
    if (B.arena.bytes < need) {
        if (ctx->budget && need + ctx->bytes_in_use() - B.arena.bytes > ctx->budget)
            return fail(FLOW_E_NOMEM, "batch working set of " + std::to_string(need) + " bytes exceeds the HBM budget");
        B.drop_graph();
        if (B.arena.base) {
            HIP_TRY(hipDeviceSynchronize());
            HIP_TRY(hipFree(B.arena.base));
            B.arena.base = nullptr;
            B.arena.bytes = 0;
        }
        void* a = nullptr;
        hipError_t e = hipMalloc(&a, need);
        if (e != hipSuccess) return fail(FLOW_E_NOMEM, std::string("hipMalloc(batch arena): ") + hipGetErrorString(e));
        B.arena.base = a;
        B.arena.bytes = need;
    }
    P->L.resize(n);
    for (int k = 0; k < n; ++k) {
        flow_params pk = p;
        pk.levels = P->levels[k];
        DevArena sub{(char*)B.arena.base + off[k], off[k + 1] - off[k]};
        flow_status st = build_layout(sub, pairs[k].H, pairs[k].W, pk, P->L[k]);
        if (st != FLOW_OK) return st;
        P->lmax = std::max(P->lmax, P->levels[k]);
    }

    // stages, their choices and tile counts
    std::vector<int> desc_id(n * FLOW_MAX_LEVELS, -1);
    int ndesc = 0;
    for (int k = 0; k < n; ++k)
        for (int l = 0; l < P->levels[k]; ++l) desc_id[k * FLOW_MAX_LEVELS + l] = ndesc++;
    std::vector<TbTile> tiles;
    int ncounters = 0;
    for (int l = P->lmax - 1; l >= 0; --l) {
        BStage S;
        S.l = l;
        std::vector<std::pair<int, int>> shapes;
        for (int k = 0; k < n; ++k)
            if (P->levels[k] > l) {
                S.pairs.push_back(k);
                shapes.emplace_back(P->L[k][l].H, P->L[k][l].W);
            }
        S.key = stage_key(shapes, hw, p.iters);
        if (pd) {
            S.key = (p.scheme == FLOW_ALG1 ? std::string("a:") : "p" + std::to_string(p.gs_sweeps) + ":") + S.key;
            if (!plan_pd_stage(*P, S, p, desc_id, B.tuned, tiles))
                return fail(FLOW_E_INVAL, "a level of the batch takes no pDR / ALG1 tiles");
            P->stages.push_back(S);
            continue;
        }
        auto it = B.tuned.find(S.key);
        S.ch = (it != B.tuned.end() && shapes_fit(shapes, hw, it->second.K, it->second.ew, it->second.tnt))
                   ? it->second : default_stage_choice(shapes, hw, p.iters);
        // process-wide overrides (tests and experiments); K is lowered until every level fits
        if (g_batch_order >= 0) S.ch.order = g_batch_order;
        if (g_batch_ew > 0) S.ch.ew = g_batch_ew;
        if (g_batch_k > 0) S.ch.K = g_batch_k;
        if (g_batch_nt > 0) S.ch.tnt = g_batch_nt;
        S.ch = fit_stage_choice(S.ch, shapes, hw);
        S.lpw = launches_per_warp(p.iters, S.ch.K);
        S.tile_off = (int)tiles.size();
        stage_tiles(*P, S, hw, S.ch, desc_id, tiles);
        S.ntiles = (int)tiles.size() - S.tile_off;
        S.grid = tile_grid(S.ch, S.ntiles);
        if (S.ch.order == ORDER_QUEUE) {
            S.counter_off = ncounters;
            ncounters += p.warps * S.lpw * kNq;
        }
        P->stages.push_back(S);
    }
    P->ncounters = ncounters;

    // device scalars
    size_t o = 0;
    auto take = [&](size_t b) { const size_t r = o; o = (o + b + 255) & ~(size_t)255; return r; };
    P->at_off = take(sizeof(float) * 2 * n);
    P->epart_off = take(sizeof(double) * kEnergyTerms * kEnergyBlocks * n);
    P->eout_off = take(sizeof(double) * kEnergyTerms * n);
    P->cnt_off = take(sizeof(unsigned) * std::max(1, ncounters));
    P->dyn_bytes = o;
    {
        flow_status st = B.dyn.ensure(P->dyn_bytes, "batch scalars");
        if (st != FLOW_OK) return st;
    }
    float* d_at = (float*)(B.dyn.d + P->at_off);
    double* d_epart = (double*)(B.dyn.d + P->epart_off);
    double* d_eout = (double*)(B.dyn.d + P->eout_off);

    // tables
    TableBuilder T;
    if (!pd) {
        std::vector<TbLevel> descs(2 * std::max(1, ndesc));
        for (int k = 0; k < n; ++k)
            for (int l = 0; l < P->levels[k]; ++l)
                fill_tb_level(&descs[2 * desc_id[k * FLOW_MAX_LEVELS + l]], P->L[k][l], d_at + 2 * k);
        P->descs_off = T.put(descs);
    } else {
        // direction d reads state set d and writes the other
        std::vector<PdrTbLevel> descs(2 * std::max(1, ndesc));
        PdrTbPlan one;
        one.th = one.tw = 1;
        for (int k = 0; k < n; ++k)
            for (int l = 0; l < P->levels[k]; ++l)
                for (int d = 0; d < 2; ++d)
                    descs[2 * desc_id[k * FLOW_MAX_LEVELS + l] + d] = pdr_tb_args(P->L[k][l], p, one, d, 1).lvl;
        P->pdescs_off = T.put(descs);
    }
    P->tiles_off = T.put(tiles);
    // pyramid
    P->down.resize(P->lmax);
    for (int l = 1; l < P->lmax; ++l) {
        std::vector<DownArgs> it;
        std::vector<int> bl;
        for (int k = 0; k < n; ++k) {
            if (P->levels[k] <= l) continue;
            const LevelPlanes& F = P->L[k][l - 1];
            const LevelPlanes& C = P->L[k][l];
            it.push_back(DownArgs{F.I0, F.H, F.W, F.ld, C.I0, C.ld, F.I0lo, C.I0lo});
            it.push_back(DownArgs{F.I1, F.H, F.W, F.ld, C.I1, C.ld, F.I1lo, C.I1lo});
            bl.push_back(blocks_of(C.H, C.W));
            bl.push_back(blocks_of(C.H, C.W));
        }
        P->down[l] = T.launch(it, bl);
    }
    {
        std::vector<DerivArgs> it;
        std::vector<int> bl;
        for (int k = 0; k < n; ++k)
            for (int l = 0; l < P->levels[k]; ++l) {
                const LevelPlanes& L = P->L[k][l];
                it.push_back(DerivArgs{L.I1, L.H, L.W, L.ld, L.Dx, L.Dy, L.ld, L.I1lo});
                bl.push_back(blocks_of(L.H, L.W));
            }
        P->deriv = T.launch(it, bl);
    }
    // stages: level start, per-warp linearisation (committing the previous warp); the state buffer after each warp
    // follows from the number of tile launches (every pair of a stage has the same schedule)
    std::vector<int> final_cur_of_stage(P->lmax, 0);
    for (BStage& S : P->stages) {
        const int l = S.l;
        std::vector<LevelInitArgs> init;
        std::vector<int> bl;
        for (int k : S.pairs) {
            const LevelPlanes& L = P->L[k][l];
            LevelInitArgs ia{};
            ia.H = L.H; ia.W = L.W; ia.ld = L.ld;
            if (l < P->levels[k] - 1) {
                const LevelPlanes& C = P->L[k][l + 1];
                const int cc = final_cur_of_stage[l + 1];
                ia.uc = level_flow(C, p, 1, cc);
                ia.vc = level_flow(C, p, 2, cc);
                ia.ucd = level_inc(C, p, 1, cc);
                ia.vcd = level_inc(C, p, 2, cc);
                ia.wc = hw ? level_flow(C, p, 0, cc) : nullptr;
                ia.Hc = C.H; ia.Wc = C.W; ia.ldc = C.ld;
            }
            int nz = 0;
            if (!pd) {
                ia.set_flow[0] = hw ? L.st[0][0] : nullptr;
                ia.set_flow[1] = L.U0[0];
                ia.set_flow[2] = L.U0[1];
                for (int q = 3; q < 10; ++q)
                    if (L.st[0][q]) ia.zero[nz++] = L.st[0][q];
            } else {                     // X = X bar = the upsampled flow, y bar = 0, Theta = 0
                ia.set_flow[0] = hw ? L.Xs[0][0] : nullptr;
                ia.set_flow[1] = L.Xs[0][1];
                ia.set_flow[2] = L.Xs[0][2];
                ia.copy_flow[0] = hw ? L.Xbs[0][0] : nullptr;
                ia.copy_flow[1] = L.Xbs[0][1];
                ia.copy_flow[2] = L.Xbs[0][2];
                for (int q = 0; q < 6; ++q)
                    if (L.ybs[0][q]) ia.zero[nz++] = L.ybs[0][q];
                ia.zero[nz++] = L.s_out;
            }
            ia.nzero = nz;
            ia.clear_scalar = d_at + 2 * k;
            init.push_back(ia);
            bl.push_back(blocks_of(L.H, L.W));
        }
        S.init = T.launch(init, bl);
        int cur = 0;
        std::vector<int> lbl;
        for (int k : S.pairs) lbl.push_back(lin_blocks_of(P->L[k][l].H, P->L[k][l].W));
        for (int w = 0; w < p.warps; ++w) {
            std::vector<LinArgs> lin;
            for (int k : S.pairs) {
                const LevelPlanes& L = P->L[k][l];
                LinArgs la{};
                la.I0 = L.I0; la.I1 = L.I1; la.Dx = L.Dx; la.Dy = L.Dy;
                la.I0lo = L.I0lo; la.I1lo = L.I1lo;
                if (!pd) {
                    la.u0 = L.U0[0];
                    la.v0 = L.U0[1];
                    if (w > 0) {         // commit the previous warp's increment on the way
                        la.pend_u = L.st[cur][1];
                        la.pend_v = L.st[cur][2];
                    }
                    la.zero_u = L.st[cur][1];
                    la.zero_v = L.st[cur][2];
                } else {                 // linearise around X; keep a copy of the point for I_t
                    la.u0 = L.Xs[cur][1];
                    la.v0 = L.Xs[cur][2];
                    la.keep_u = L.U0[0];
                    la.keep_v = L.U0[1];
                }
                la.Ix = L.Ix; la.Iy = L.Iy; la.It = L.It;
                la.at = d_at + 2 * k + (w & 1);
                la.at_clear = d_at + 2 * k + ((w + 1) & 1);
                la.H = L.H; la.W = L.W; la.ld = L.ld;
                la.kappa = (float)p.intensity_scale;
                la.beta = (float)p.beta;
                la.rel = 1;
                lin.push_back(la);
            }
            S.lin.push_back(T.launch(lin, lbl));
            cur ^= S.lpw & 1;
        }
        final_cur_of_stage[l] = cur;
    }
    P->final_cur = final_cur_of_stage[0];
    {
        // energy of every pair at the end of level 0 (flow = U0 + the last warp's increment)
        Scratch dummy;
        std::vector<EnergyArgs> it;
        std::vector<int> bl;
        for (int k = 0; k < n; ++k) {
            const LevelPlanes& L = P->L[k][0];
            EnergyArgs e = energy_args(L, p, P->final_cur, dummy);
            e.partial = d_epart + (size_t)k * kEnergyTerms * kEnergyBlocks;
            e.out = d_eout + (size_t)k * kEnergyTerms;
            it.push_back(e);
            bl.push_back(energy_blocks(L.H, L.W));
        }
        P->energy = T.launch(it, bl);
    }
    {
        flow_status st = B.tab.ensure(T.h.size(), "batch tables");
        if (st != FLOW_OK) return st;
        HIP_TRY(hipMemcpy(B.tab.d, T.h.data(), T.h.size(), hipMemcpyHostToDevice));
    }
    // io table: import (I0, I1 -> level 0) and export (U0 -> u, v) items, rewritten per call; the
    // block offsets depend on the composition only and are written once into the staging copy
    {
        std::vector<int> bl;
        for (int k = 0; k < n; ++k) {
            bl.push_back(blocks_of(pairs[k].H, pairs[k].W));
            bl.push_back(blocks_of(pairs[k].H, pairs[k].W));
        }
        std::vector<CopyArgs> blank(2 * n);
        TableBuilder io;
        P->imp = io.launch(blank, bl);
        P->exp = io.launch(blank, bl);
        P->io_bytes = io.h.size();
        flow_status st = B.io.ensure(P->io_bytes, "batch io table");
        if (st != FLOW_OK) return st;
        st = B.h_io.ensure(P->io_bytes);
        if (st != FLOW_OK) return st;
        std::memcpy(B.h_io.h, io.h.data(), io.h.size());
    }
    B.plan = std::move(P);
    return FLOW_OK;
}

// Fills the per-call import / export items (caller pointers) into the pinned staging table.
void fill_io(BatchState& B, int n, const flow_pair* pairs, const flow_params& p) {
    const BatchPlan& P = *B.plan;
    CopyArgs* ci = (CopyArgs*)(B.h_io.h + P.imp.items);
    CopyArgs* ce = (CopyArgs*)(B.h_io.h + P.exp.items);
    for (int k = 0; k < n; ++k) {
        const LevelPlanes& L = P.L[k][0];
        const flow_pair& q = pairs[k];
        const float off = p.storage == FLOW_STORE_F16 ? kFrameOffsetF16 : 0.f;
        ci[2 * k] = CopyArgs{q.I0, q.H, q.W, q.ld, L.I0, L.ld, off};
        ci[2 * k + 1] = CopyArgs{q.I1, q.H, q.W, q.ld, L.I1, L.ld, off};
        // the flow is U0 plus the last warp's pending increment (pDR / ALG1: X)
        ce[2 * k] = CopyArgs{level_flow(L, p, 1, P.final_cur), q.H, q.W, L.ld, q.u, q.ld_uv, 0.f,
                             level_inc(L, p, 1, P.final_cur)};
        ce[2 * k + 1] = CopyArgs{level_flow(L, p, 2, P.final_cur), q.H, q.W, L.ld, q.v, q.ld_uv, 0.f,
                                 level_inc(L, p, 2, P.final_cur)};
    }
}

void run_b(BatchOp op, const char* base, const BLaunch& L, bool f16, hipStream_t s) {
    launch_batched(op, base + L.items, (const int*)(base + L.off), L.n, L.total, f16, s);
}

// The tile launches of one warp of stage S (returns the state buffer after them).
int enqueue_stage_iters(const BatchState& B, const BStage& S, const flow_params& p, int w, int cur, hipStream_t s) {
    const BatchPlan& P = *B.plan;
    if (S.pd) {
        PdrTbArgs a{};
        pd_tile_scalars(a, p);
        a.tiles = (const TbTile*)(B.tab.d + P.tiles_off) + S.tile_off;
        a.ntiles = S.ntiles;
        a.levels = (const PdrTbLevel*)(B.tab.d + P.pdescs_off);
        int dir = cur;
        for (int k = 0; k < p.iters;) {
            a.K = std::min(S.ch.K, p.iters - k);
            a.dir = dir;
            if (p.scheme == FLOW_ALG1) launch_alg1_tb(a, p.beta > 0, S.pd_nt, s);
            else launch_pdr_tb(a, p.beta > 0, S.pd_nt, s);
            dir ^= 1;
            k += a.K;
        }
        return dir;
    }
    unsigned* counters = (unsigned*)(B.dyn.d + P.cnt_off) + S.counter_off + w * S.lpw * kNq;
    return enqueue_tile_warp((const TbTile*)(B.tab.d + P.tiles_off) + S.tile_off, S.ntiles, S.grid,
                             (const TbLevel*)(B.tab.d + P.descs_off), S.ch, p, w & 1, cur, counters, s);
}

void enqueue_batch(const BatchState& B, const flow_params& p, hipStream_t s, hipEvent_t* ev) {
    const BatchPlan& P = *B.plan;
    const bool f16 = p.storage == FLOW_STORE_F16;
    const char* tab = B.tab.d;
    run_b(BatchOp::Copy, B.io.d, P.imp, f16, s);                         // import
    if (P.ncounters > 0) launch_reset_u32((unsigned*)(B.dyn.d + P.cnt_off), P.ncounters, s);
    for (int l = 1; l < P.lmax; ++l) run_b(BatchOp::Downsample, tab, P.down[l], f16, s);
    run_b(BatchOp::Derivatives, tab, P.deriv, f16, s);
    int si = 0;
    for (const BStage& S : P.stages) {
        run_b(BatchOp::LevelInit, tab, S.init, false, s);
        int cur = 0;
        for (int w = 0; w < p.warps; ++w) {
            run_b(BatchOp::Linearize, tab, S.lin[w], f16, s);
            // instrumented solves time the iteration launches alone, warp by warp
            if (ev) hipEventRecord(ev[2 * (si * p.warps + w)], s);
            cur = enqueue_stage_iters(B, S, p, w, cur, s);
            if (ev) hipEventRecord(ev[2 * (si * p.warps + w) + 1], s);
            if (S.l == 0 && w == p.warps - 1)
                launch_energy_batched((const EnergyArgs*)(tab + P.energy.items), (const int*)(tab + P.energy.off),
                                      P.energy.n, P.energy.total, s);
        }
        ++si;
    }
    run_b(BatchOp::Copy, B.io.d, P.exp, false, s);                       // export
}

BatchState& batch_of(flow_ctx* ctx) {
    if (!ctx->batch) ctx->batch = new BatchState();
    return *ctx->batch;
}

flow_status prepare(flow_ctx* ctx, int n, const flow_pair* pairs, const flow_params& p) {
    BatchState& B = batch_of(ctx);
    const std::string key = batch_key(n, pairs, p) + "|te" + std::to_string(B.tune_epoch);
    if (B.plan && B.plan->key == key) return FLOW_OK;
    B.drop_graph();
    B.plan.reset();
    flow_status st = build_plan(ctx, B, n, pairs, p);
    if (st != FLOW_OK) return st;
    B.plan->key = key;
    return FLOW_OK;
}

}  // namespace

extern "C" flow_status flow_solve_batched(flow_ctx* ctx, int32_t n, const flow_pair* pairs, const flow_params* p,
                                          void* stream) {
    if (!ctx) return fail(FLOW_E_INVAL, "ctx is NULL");
    if (n < 0 || (n > 0 && !pairs)) return fail(FLOW_E_INVAL, "bad batch arguments");
    flow_status st = validate(p);
    if (st != FLOW_OK) return st;
    st = validate_pairs(n, pairs, *p);
    if (st != FLOW_OK) return st;
    if (n == 0) return FLOW_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    if (p->tol > 0 || (pd_state(*p) && !pd_batch_tileable(n, pairs, *p))) {
        // stopping tests, and pDR with a halo no tile holds: plain solves in turn
        for (int32_t k = 0; k < n; ++k) {
            flow_params pk = *p;
            if (pairs[k].levels > 0) pk.levels = pairs[k].levels;
            const flow_pair& q = pairs[k];
            st = flow_solve(ctx, q.I0, q.I1, q.H, q.W, q.ld, &pk, q.u, q.v, q.ld_uv, q.res, stream);
            if (st != FLOW_OK) return st;
        }
        return FLOW_OK;
    }
    st = prepare(ctx, n, pairs, *p);
    if (st != FLOW_OK) return st;
    BatchState& B = *ctx->batch;
    const BatchPlan& P = *B.plan;
    fill_io(B, n, pairs, *p);
    HIP_TRY(hipMemcpyAsync(B.io.d, B.h_io.h, P.io_bytes, hipMemcpyHostToDevice, s));
    const bool timed = ctx->stats_enabled;
    if (timed) HIP_TRY(hipEventRecord(ctx->ev_total[0], s));
    const bool use_graph = p->use_graph && !timed;
    if (use_graph) {
        if (!B.exec) {
            HIP_TRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
            enqueue_batch(B, *p, ctx->cap_stream, nullptr);
            hipGraph_t g = nullptr;
            HIP_TRY(hipStreamEndCapture(ctx->cap_stream, &g));
            B.graph = g;
            HIP_TRY(hipGraphInstantiate(&B.exec, g, nullptr, nullptr, 0));
        }
        HIP_TRY(hipGraphLaunch(B.exec, s));
    } else {
        while (B.ev.size() < 2 * P.stages.size() * (size_t)p->warps) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            B.ev.push_back(e);
        }
        enqueue_batch(B, *p, s, timed ? B.ev.data() : nullptr);
    }
    HIP_TRY(hipGetLastError());
    if (timed) HIP_TRY(hipEventRecord(ctx->ev_total[1], s));
    st = B.h_e.ensure(sizeof(double) * kEnergyTerms * n);
    if (st != FLOW_OK) return st;
    HIP_TRY(hipMemcpyAsync(B.h_e.h, B.dyn.d + P.eout_off, sizeof(double) * kEnergyTerms * n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (timed) {
        flow_stats S{};
        S.levels = P.lmax;
        int64_t pxi = 0;
        for (size_t si = 0; si < P.stages.size(); ++si) {
            const BStage& G = P.stages[si];
            int64_t px = 0;
            for (int k : G.pairs) px += (int64_t)P.L[k][G.l].H * P.L[k][G.l].W;
            S.level_px[G.l] = px;
            S.H[G.l] = 0;
            S.W[G.l] = 0;
            S.iterations[G.l] = (int64_t)p->warps * p->iters;
            S.launches[G.l] = (int64_t)p->warps * G.lpw;
            float ms = 0.f;
            for (int w = 0; w < p->warps; ++w) {
                float wms = 0.f;
                hipEventElapsedTime(&wms, B.ev[2 * (si * p->warps + w)], B.ev[2 * (si * p->warps + w) + 1]);
                ms += wms;
            }
            S.iter_ms[G.l] = ms;
            pxi += px * S.iterations[G.l];
        }
        float tot = 0.f;
        hipEventElapsedTime(&tot, ctx->ev_total[0], ctx->ev_total[1]);
        S.total_ms = tot;
        S.px_iter = pxi;
        S.graph_replayed = 0;
        ctx->last_stats = S;
    }
    bool finite = true;
    const double* h = (const double*)B.h_e.h;
    for (int k = 0; k < n; ++k) {
        const double* e = h + (size_t)k * kEnergyTerms;
        fill_result(e, pairs[k].res);
        if (!std::isfinite(e[0] + e[1]) || !std::isfinite(e[2]) || e[7] != 0.0) finite = false;
    }
    if (!finite) return fail(FLOW_E_NONFINITE, "non-finite energy or gap in a batched pair");
    return FLOW_OK;
}

extern "C" flow_status flow_tune_batched_stage(flow_ctx* ctx, int32_t n, const flow_pair* pairs, const flow_params* p,
                                               int32_t level, int32_t order, int32_t K, int32_t ew) {
    if (!ctx) return fail(FLOW_E_INVAL, "ctx is NULL");
    if (n < 1 || !pairs) return fail(FLOW_E_INVAL, "bad batch arguments");
    flow_status st = validate(p);
    if (st != FLOW_OK) return st;
    st = validate_pairs(n, pairs, *p);
    if (st != FLOW_OK) return st;
    if (level < 0 || level >= FLOW_MAX_LEVELS) return fail(FLOW_E_INVAL, "level out of range");
    if (pd_state(*p)) {
        // pDR / ALG1 stage: order is the work-group code (the report's "nt"), ew is not used
        const std::vector<int> codes = pd_codes(*p);
        if (std::find(codes.begin(), codes.end(), order) == codes.end())
            return fail(FLOW_E_INVAL, "pDR / ALG1 stage: order must be one of the scheme's tile codes (the report's nt)");
        if (K < 1) return fail(FLOW_E_INVAL, "K must be >= 1");
        const bool hw = p->beta > 0;
        Shapes shapes;
        for (int32_t k = 0; k < n; ++k) {
            const int lv = pairs[k].levels > 0 ? pairs[k].levels : p->levels;
            if (lv > level) shapes.push_back(level_shapes(pairs[k].H, pairs[k].W, lv)[level]);
        }
        if (shapes.empty()) return fail(FLOW_E_INVAL, "no pair of the batch has that level");
        const int kk = std::min<int>(K, std::max(1, p->iters));
        for (const auto& sh : shapes)
            if (!plan_pd_tiles(sh.first, sh.second, hw, pd_halo(*p, kk), kk, 0, order).tb)
                return fail(FLOW_E_INVAL, "a level of the stage takes no tiles of that code and K");
        BatchState& B = batch_of(ctx);
        StageChoice c;
        c.nt = order;
        c.K = kk;
        const std::string pre = p->scheme == FLOW_ALG1 ? std::string("a:") : "p" + std::to_string(p->gs_sweeps) + ":";
        B.tuned[pre + stage_key(shapes, hw, p->iters)] = c;
        B.tune_epoch++;
        B.drop_graph();
        B.plan.reset();
        return FLOW_OK;
    }
    if (order != ORDER_TABLE && order != ORDER_QUEUE && !is_rows_code(order))
        return fail(FLOW_E_INVAL, "order: 0 table, 1 work queue, or a wave-row code 2049 / 3073 / 4097 (table order)");
    if (K < 1 || ew < 16 || ew > 512) return fail(FLOW_E_INVAL, "K must be >= 1 and ew in [16, 512]");
    const int nt = is_rows_code(order) ? order : kBatchNt;
    if (is_rows_code(nt) && ew > kWave) return fail(FLOW_E_INVAL, "the wave-row tiles take ew <= 64");
    const bool hw = p->beta > 0;
    Shapes shapes;
    for (int32_t k = 0; k < n; ++k) {
        const int lv = pairs[k].levels > 0 ? pairs[k].levels : p->levels;
        if (lv > level) shapes.push_back(level_shapes(pairs[k].H, pairs[k].W, lv)[level]);
    }
    if (shapes.empty()) return fail(FLOW_E_INVAL, "no pair of the batch has that level");
    if (!shapes_fit(shapes, hw, K, ew, nt))
        return fail(FLOW_E_INVAL, "a level of the stage takes no tiles of that K and width");
    BatchState& B = batch_of(ctx);
    StageChoice c;
    c.order = is_rows_code(order) ? ORDER_TABLE : order;
    c.K = K;
    c.ew = ew;
    c.tnt = nt;
    B.tuned[stage_key(shapes, hw, p->iters)] = c;
    B.tune_epoch++;
    B.drop_graph();
    B.plan.reset();
    return FLOW_OK;
}

extern "C" flow_status flow_autotune_batched(flow_ctx* ctx, int32_t n, const flow_pair* pairs, const flow_params* p,
                                             void* stream) {
    if (!ctx) return fail(FLOW_E_INVAL, "ctx is NULL");
    if (n < 0 || (n > 0 && !pairs)) return fail(FLOW_E_INVAL, "bad batch arguments");
    flow_status st = validate(p);
    if (st != FLOW_OK) return st;
    st = validate_pairs(n, pairs, *p);
    if (st != FLOW_OK) return st;
    if (n == 0 || p->iters < 1) return FLOW_OK;
    if (pd_state(*p) && !pd_batch_tileable(n, pairs, *p)) return FLOW_OK;   // plain solves in turn
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    st = prepare(ctx, n, pairs, *p);
    if (st != FLOW_OK) return st;
    BatchState& B = *ctx->batch;
    BatchPlan& P = *B.plan;
    const bool hw = p->beta > 0;
    const bool f16 = p->storage == FLOW_STORE_F16;
    fill_io(B, n, pairs, *p);
    HIP_TRY(hipMemcpyAsync(B.io.d, B.h_io.h, P.io_bytes, hipMemcpyHostToDevice, s));
    const char* tab = B.tab.d;
    run_b(BatchOp::Copy, B.io.d, P.imp, f16, s);
    for (int l = 1; l < P.lmax; ++l) run_b(BatchOp::Downsample, tab, P.down[l], f16, s);
    run_b(BatchOp::Derivatives, tab, P.deriv, f16, s);
    std::vector<int> desc_id(n * FLOW_MAX_LEVELS, -1);
    int ndesc = 0;
    for (int k = 0; k < n; ++k)
        for (int l = 0; l < P.levels[k]; ++l) desc_id[k * FLOW_MAX_LEVELS + l] = ndesc++;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    // candidate tables live in a temporary buffer; the plan's own tables stay as they are
    DevBuf tmp_tiles, tmp_cnt;
    st = tmp_cnt.ensure(256, "tuning counters");
    std::map<std::string, StageChoice> chosen;
    std::ostringstream rep;                       // the report flow_get_tuning returns afterwards
    rep << "{\"stages\": [";
    for (BStage& S : P.stages) {
        if (st != FLOW_OK) break;
        run_b(BatchOp::LevelInit, tab, S.init, false, s);
        run_b(BatchOp::Linearize, tab, S.lin[0], f16, s);
        if (S.pd) {
            // pDR / ALG1: work-group code x K (pDR 1 .. 4, ALG1 the launch-count values up to 10),
            // and the whole warp per launch where every level fits one tile of that code
            std::vector<StageChoice> pc;
            const std::vector<int> pks = p->scheme == FLOW_ALG1 ? launch_ks(p->iters, 1, 10) : std::vector<int>{1, 2, 3, 4};
            for (int nt : pd_codes(*p)) {
                std::vector<int> kk = pks;
                if (pd_stage_resident(P, S, hw, nt)) kk.push_back(p->iters);
                for (int K : kk) {
                    StageChoice c;
                    c.nt = nt;
                    c.K = K;
                    pc.push_back(c);
                }
            }
            double pbest = 1e30;
            StageChoice pbestc = S.ch;
            for (const StageChoice& c : pc) {
                std::vector<TbTile> tl;
                if (!pd_stage_tiles(P, S, *p, c.nt, c.K, desc_id, tl)) continue;
                st = tmp_tiles.ensure(sizeof(TbTile) * tl.size(), "tuning tiles");
                if (st != FLOW_OK) break;
                HIP_TRY(hipMemcpy(tmp_tiles.d, tl.data(), sizeof(TbTile) * tl.size(), hipMemcpyHostToDevice));
                PdrTbArgs a{};
                pd_tile_scalars(a, *p);
                a.tiles = (const TbTile*)tmp_tiles.d;
                a.ntiles = (int)tl.size();
                a.levels = (const PdrTbLevel*)(tab + P.pdescs_off);
                float best_ms = 1e30f;
                for (int rep_i = 0; rep_i < 4; ++rep_i) {         // the first run is a warm-up
                    HIP_TRY(hipEventRecord(e0, s));
                    int dir = 0;
                    for (int k = 0; k < p->iters;) {
                        a.K = std::min(c.K, p->iters - k);
                        a.dir = dir;
                        if (p->scheme == FLOW_ALG1) launch_alg1_tb(a, hw, c.nt, s);
                        else launch_pdr_tb(a, hw, c.nt, s);
                        dir ^= 1;
                        k += a.K;
                    }
                    HIP_TRY(hipEventRecord(e1, s));
                    HIP_TRY(hipEventSynchronize(e1));
                    float ms = 0.f;
                    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                    if (rep_i > 0) best_ms = std::min(best_ms, ms);
                }
                HIP_TRY(hipGetLastError());
                if (best_ms < pbest) {
                    pbest = best_ms;
                    pbestc = c;
                }
            }
            chosen[S.key] = pbestc;
            rep << (&S == &P.stages.front() ? "" : ", ") << "{\"level\": " << S.l << ", \"pairs\": " << S.pairs.size()
                << ", \"nt\": " << pbestc.nt << ", \"K\": " << pbestc.K << ", \"us_per_warp\": " << 1e3 * pbest << "}";
            continue;
        }
        // the general tiles in table and queue order, and the wave-row tiles (table order only)
        std::vector<StageChoice> cands;
        const std::vector<int> ks = launch_ks(p->iters, 2, 10);
        for (int nt : {kBatchNt, 2049, 3073, 4097})
            for (int order : {ORDER_TABLE, ORDER_QUEUE}) {
                if (is_rows_code(nt) && order != ORDER_TABLE) continue;
                if (shapes_all_resident(stage_shapes(P, S), hw, nt)) {
                    StageChoice c;
                    c.order = order;
                    c.K = p->iters;
                    c.tnt = nt;
                    cands.push_back(c);
                }
                for (int K : ks)
                    for (int ew : {64, 128}) {
                        if (is_rows_code(nt) && ew > kWave) continue;
                        if (stage_fits(P, S, hw, K, ew, nt)) {
                            StageChoice c;
                            c.order = order;
                            c.K = K;
                            c.ew = ew;
                            c.tnt = nt;
                            cands.push_back(c);
                        }
                    }
            }
        double best = 1e30;
        StageChoice bestc = S.ch;
        for (const StageChoice& c : cands) {
            std::vector<TbTile> tl;
            stage_tiles(P, S, hw, c, desc_id, tl);
            st = tmp_tiles.ensure(sizeof(TbTile) * tl.size(), "tuning tiles");
            if (st != FLOW_OK) break;
            HIP_TRY(hipMemcpy(tmp_tiles.d, tl.data(), sizeof(TbTile) * tl.size(), hipMemcpyHostToDevice));
            BStage T = S;
            T.ch = c;
            T.lpw = launches_per_warp(p->iters, c.K);
            T.ntiles = (int)tl.size();
            T.grid = c.order == ORDER_QUEUE ? std::max(1, std::min(T.ntiles, 512)) : T.ntiles;
            AdmmIterArgs co{};
            fill_admm_coeffs(co, *p);
            float best_ms = 1e30f;
            for (int rep = 0; rep < 4; ++rep) {               // the first run is a warm-up
                HIP_TRY(hipEventRecord(e0, s));
                int cur = 0, k = 0;
                while (k < p->iters) {
                    const int kk = std::min(c.K, p->iters - k);
                    TbArgs a{};
                    a.tiles = (const TbTile*)tmp_tiles.d;
                    a.ntiles = T.ntiles;
                    a.levels = (const TbLevel*)(tab + P.descs_off);
                    a.at_slot = 0;
                    a.dir = cur;
                    a.K = kk;
                    a.c = co.c; a.lam = co.lam; a.beta = co.beta; a.inv_ac = co.inv_ac; a.c_rho_s = co.c_rho_s;
                    a.cA = co.cA; a.cB = co.cB; a.cC = co.cC;
                    if (c.order == ORDER_QUEUE) {
                        launch_reset_u32((unsigned*)tmp_cnt.d, kNq, s);
                        a.queue = (unsigned*)tmp_cnt.d;
                        a.nq = std::min(kNq, T.grid);
                    } else {
                        a.nq = 1;
                    }
                    launch_admm_tb(a, hw, c.tnt, T.grid, s);
                    cur ^= 1;
                    k += kk;
                }
                HIP_TRY(hipEventRecord(e1, s));
                HIP_TRY(hipEventSynchronize(e1));
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                if (rep > 0) best_ms = std::min(best_ms, ms);
            }
            HIP_TRY(hipGetLastError());
            if (best_ms < best) {
                best = best_ms;
                bestc = c;
            }
        }
        chosen[S.key] = bestc;
        rep << (&S == &P.stages.front() ? "" : ", ") << "{\"level\": " << S.l << ", \"pairs\": " << S.pairs.size()
            << ", \"order\": " << bestc.order << ", \"nt\": " << bestc.tnt << ", \"K\": " << bestc.K << ", \"ew\": " << bestc.ew
            << ", \"us_per_warp\": " << 1e3 * best << "}";
    }
    rep << "]}";
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    tmp_tiles.release();
    tmp_cnt.release();
    if (st != FLOW_OK) return st;
    for (auto& kv : chosen) B.tuned[kv.first] = kv.second;
    ctx->tune_report = rep.str();
    B.tune_epoch++;
    B.drop_graph();
    B.plan.reset();
    return FLOW_OK;
}
