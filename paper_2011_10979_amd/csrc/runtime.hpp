// Host-side structures of the runtime: arena layout of one pair, small per-context device
// buffers, event timers, the stopping test and the context itself.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/flow.h"
#include "kernels.hpp"

namespace flowmi {

flow_status fail(flow_status st, const std::string& msg);
// Schemes whose state is (X, X bar, y) in the pDR planes: pDR and ALG1.
inline bool pd_state(const flow_params& p) { return p.scheme == FLOW_PDR || p.scheme == FLOW_ALG1; }
flow_status hip_fail(hipError_t e, const char* what);
int64_t pitch_of(int W);
flow_status check_extent(const void* ptr, int H, int W, int64_t ld, size_t elem, const char* name);
std::vector<std::pair<int, int>> level_shapes(int H, int W, int levels);
flow_status validate(const flow_params* p);
flow_status validate_shape(int H, int W, int64_t ld, int levels);

struct DevArena {
    void* base = nullptr;
    size_t bytes = 0;
};

// Planes of one pyramid level (pitch ld elements; pyramid planes are FP32 or FP16).
struct LevelPlanes {
    int H = 0, W = 0;
    int64_t ld = 0;
    void *I0 = nullptr, *I1 = nullptr, *Dx = nullptr, *Dy = nullptr;
    float *I0lo = nullptr, *I1lo = nullptr;   // low parts of float-float image levels (FP32 storage, levels >= 1)
    float *Ix = nullptr, *Iy = nullptr, *It = nullptr;
    float* st[2][10] = {};                // ADMM ping-pong: w, du, dv, px, py, q1x, q1y, q2x, q2y, s
    float* U0[2] = {};                    // linearisation point (u0, v0); ADMM: the flow without the pending increment
    // pDR, two state sets (the tile kernel reads one and writes the other): X = (w, u, v),
    // X bar, y bar = (p_x, p_y, q1x, q1y, q2x, q2y); b is the three-pass kernels' work plane
    float *Xs[2][3] = {}, *Xbs[2][3] = {}, *ybs[2][6] = {}, *b[3] = {}, *s_out = nullptr;
};

// Small device buffers used by the reductions of one solve stream.
struct Scratch {
    float* at = nullptr;              // two a~ slots: warp w of a level uses slot w % 2
    double* e_partial = nullptr;
    double* e_out = nullptr;
    unsigned* queue = nullptr;        // work counter of the tile kernel (reset at the start of a solve)
    int final_buf = 0;
    flow_status alloc();
    void release();
    size_t bytes() const;
};

// Events around each warp's block of iteration kernels, summed per level.
struct WarpTimers {
    struct Pair { hipEvent_t a, b; int level; };
    std::vector<Pair> pairs;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    int64_t iters[FLOW_MAX_LEVELS] = {};      // inner iterations per level
    int64_t kernels[FLOW_MAX_LEVELS] = {};    // iteration-kernel launches per level
    int cur_level = 0;
    hipEvent_t get();
    void reset();
    void begin(int level, hipStream_t s);
    void end(int level, hipStream_t s);
    void count(int level, int64_t n, int64_t k) { iters[level] += n; kernels[level] += k; }
    ~WarpTimers();
};

struct StopTest {
    double tol = 0.0;
    double* host = nullptr;   // pinned, kEnergyTerms doubles
    flow_status check(Scratch& sc, hipStream_t s, bool* converged);
};

struct SolvePlan;
size_t layout_bytes(int H, int W, const flow_params& p);
flow_status build_layout(DevArena& arena, int H, int W, const flow_params& p, std::vector<LevelPlanes>& out);
void fill_admm_coeffs(AdmmIterArgs& a, const flow_params& p);
flow_status enqueue_core(std::vector<LevelPlanes>& Ls, const flow_params& p, Scratch& sc, hipStream_t s,
                         WarpTimers* timers, StopTest* stop, const SolvePlan* plan);
const float* level_flow(const LevelPlanes& L, const flow_params& p, int k, int cur);
const float* level_inc(const LevelPlanes& L, const flow_params& p, int k, int cur);
EnergyArgs energy_args(const LevelPlanes& L, const flow_params& p, int cur, Scratch& sc);
void fill_result(const double* h, flow_result* r);
std::string graph_key(int H, int W, const flow_params& p, const void* arena, int tune_epoch);

// Lazily allocated buffers for the operator-level entry points (per device, process lifetime).
struct OpScratch {
    double* e_partial = nullptr;
    double* e_out = nullptr;
    flow_status ensure();
};
OpScratch& op_scratch();

// pDR: the three-pass iteration (nullptr plan) or K-iteration tiles of one level (direct tiling).
struct PdrTbPlan {
    bool tb = false;
    bool resident = false;     // one tile covers the level: a whole warp per launch
    int nt = 1024;             // work-group size: 1024 or 512 threads
    int K = 1;                 // iterations per launch
    int th = 0, tw = 0;
};
PdrTbPlan plan_pd_tiles(int H, int W, bool hw, int halo, int K, int ew_target, int nt = 1024);
std::string pd_tune_key(int H, int W, const flow_params& p);
int pd_halo(const flow_params& p, int K);
extern int g_pdr_mode;
extern int g_pdr_k;

// Per-level choice between the one-pass kernel and K-iteration tiles.
struct LevelTbPlan {
    bool tb = false;           // false: one launch of the one-pass kernel per iteration
    bool resident = false;     // one tile covers the level: all iterations of a warp in one launch
    int nt = 256;              // work-group size of the tile kernel
    int K = 1;                 // iterations per launch
    int th = 0, tw = 0;        // output tile
    int tile_off = 0, ntiles = 0;
    int rows = 0;              // one-pass kernel strip height (0 = built-in)
};
// Autotuned kernel choice of one level shape (see flow_autotune).
struct TunedChoice {
    int mode = 0;              // ADMM: 1 one-pass, 2 tiles/256, 3 tiles/1024, 4 small tiles/1024;
                               // pDR: 1 three-pass, 5 tiles (K = 0: resident)
    int K = 0, rows = 0;
    double us_per_iter = 0;
};
std::string tune_key(int H, int W, bool hw, int iters);
// Iterations per launch worth timing for `iters` iterations per warp: for each launch count n the
// smallest K that covers the warp in n launches, ceil(iters / n), within [kmin, kmax] (ascending).
// A larger K with the same launch count only widens the halo (50 iterations: K = 12 and 10 both
// take five launches).
std::vector<int> launch_ks(int iters, int kmin, int kmax);
extern int g_tb_mode;
extern int g_tb_k;
extern int g_batch_order;   // batched tile launches: -1 tuned / built-in, 0 table order, 1 work queue
extern int g_batch_k;       // 0 tuned / built-in, else iterations per batched tile launch
extern int g_batch_ew;      // 0 tuned / built-in, else extended tile width target
extern int g_batch_nt;      // 0 tuned / built-in, else the ADMM tile code of every batched / served stage
extern int g_serve_graph;   // 1 (default): serving epochs replay their tile launches from graphs
LevelTbPlan plan_level(int H, int W, bool hw, int iters, int mode, int kreq, int ew = 0);
// Tiles of work-group size nt (256, 1024, 1025) for K iterations per launch with extended tiles about
// ew_target wide (0: built-in); K is lowered until the tile fits; resident if the level fits one tile.
LevelTbPlan plan_tiles(int H, int W, bool hw, int nt, int K, int ew_target);
LevelTbPlan plan_level_tuned(int H, int W, bool hw, int iters, const std::map<std::string, TunedChoice>* tuned);
void append_tiles(const LevelTbPlan& P, int level_id, int H, int W, std::vector<TbTile>& out);
void fill_tb_level(TbLevel* d, const LevelPlanes& L, const float* at2);
int tb_grid(const LevelTbPlan& P, int ntiles);

struct TbTables {
    TbTile* d_tiles = nullptr;
    TbLevel* d_levels = nullptr;
    size_t bytes = 0;
    flow_status upload(const std::vector<TbTile>& tiles, const std::vector<TbLevel>& levels);
    void release();
    ~TbTables() { release(); }
};

// Iteration plan of one solve shape: a plan per level and the device tables of the tile kernel.
struct SolvePlan {
    std::vector<LevelTbPlan> levels;
    std::vector<PdrTbPlan> pdr;    // per level (pDR)
    std::unique_ptr<TbTables> tables;
};

// upload = false: the level plans only (direct tiling reads no device table), nothing allocated
flow_status make_plan(std::vector<LevelPlanes>& Ls, const flow_params& p, Scratch& sc, SolvePlan& out,
                      const std::map<std::string, TunedChoice>* tuned, bool upload = true);
PdrTbPlan plan_pdr_level(int H, int W, const flow_params& p, const std::map<std::string, TunedChoice>* tuned);
int enqueue_pdr_tiles(const LevelPlanes& L, const flow_params& p, const PdrTbPlan& T, int cur, int64_t n,
                      hipStream_t s, int64_t* launches);
PdrArgs pdr_args(const LevelPlanes& L, const flow_params& p, int cur);
PdrTbArgs pdr_tb_args(const LevelPlanes& L, const flow_params& p, const PdrTbPlan& T, int cur, int K);
// The scheme's scalars of a pDR / ALG1 tile launch (sweeps, steps, lambda, beta).
void pd_tile_scalars(PdrTbArgs& a, const flow_params& p);
// Built-in iterations per pDR / ALG1 tile launch.
constexpr int kPdrDefaultK = 2;
constexpr int kAlg1DefaultK = 4;
void enqueue_pdr_iter(const PdrArgs& a, int sweeps, bool hw, hipStream_t s);
int enqueue_admm_iters(const LevelPlanes& L, const flow_params& p, const LevelTbPlan* P, int rows_hint, int cur,
                       int64_t n, int at_slot, const float* at2, hipStream_t s, int64_t* launches = nullptr);
TbArgs tb_args(const SolvePlan& plan, const LevelTbPlan& P, const LevelPlanes& L, const flow_params& p, int cur,
               int K, int at_slot, const float* at2);

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int final_buf = 0;
};

struct BatchState;   // batch.cpp
void destroy_batch(BatchState* b);
size_t batch_bytes(const BatchState* b);

}  // namespace flowmi

struct flow_ctx {
    int device = 0;
    size_t budget = 0;
    flowmi::DevArena arena;
    flowmi::Scratch scratch;
    double* host_out = nullptr;           // pinned
    hipStream_t cap_stream = nullptr;
    std::map<std::string, flowmi::GraphEntry> graphs;
    std::map<std::string, std::unique_ptr<flowmi::SolvePlan>> plans;
    std::map<std::string, flowmi::TunedChoice> tuned;     // per level shape, from flow_autotune
    int tune_epoch = 0;
    std::string tune_report;                             // JSON of the last flow_autotune
    bool stats_enabled = false;
    flow_stats last_stats{};
    flowmi::WarpTimers timers;
    hipEvent_t ev_total[2] = {nullptr, nullptr};
    flowmi::BatchState* batch = nullptr;

    flow_status init_scratch();
    size_t bytes_in_use() const;
    flow_status ensure_arena(size_t need);
    void drop_graphs();
    flow_status solve(const float* I0, const float* I1, int H, int W, int64_t ld, const flow_params& p, float* u,
                      float* v, int64_t ld_uv, flow_result* res, hipStream_t s);
    ~flow_ctx();
};
