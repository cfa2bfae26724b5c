// Host runtime behind the C ABI of include/flow.h: parameter checks, the device arena of one
// solve, the coarse-to-fine launch sequence (Sec. 4), hipGraph capture / replay of that sequence,
// and the operator-level entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/flow.h"
#include "kernels.hpp"
#include "runtime.hpp"

namespace flowmi {

thread_local std::string g_last_error;

flow_status fail(flow_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

flow_status hip_fail(hipError_t e, const char* what) {
    return fail(FLOW_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                           \
    do {                                                        \
        hipError_t _e = (expr);                                 \
        if (_e != hipSuccess) return hip_fail(_e, #expr);       \
    } while (0)

int64_t pitch_of(int W) { return ((int64_t)W + 63) / 64 * 64; }

// A caller plane of H rows, W used columns and pitch ld elements must lie inside the device
// allocation that contains its first element; a plane that runs past it would make the kernels
// write outside the caller's memory, so it is rejected before anything is launched.
flow_status check_extent(const void* ptr, int H, int W, int64_t ld, size_t elem, const char* name) {
    if (!ptr) return fail(FLOW_E_INVAL, std::string(name) + " is NULL");
    if (H > FLOW_MAX_SIDE || W > FLOW_MAX_SIDE)
        return fail(FLOW_E_INVAL, std::string(name) + ": a side above FLOW_MAX_SIDE pixels");
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    hipError_t e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)ptr);
    if (e != hipSuccess || !base) {
        (void)hipGetLastError();
        return fail(FLOW_E_INVAL, std::string(name) + " is not device memory of this GPU");
    }
    const uintptr_t lo = (uintptr_t)ptr, b = (uintptr_t)base;
    const uintptr_t need = lo + ((size_t)(H - 1) * (size_t)ld + (size_t)W) * elem;
    if (lo < b || need > b + size)
        return fail(FLOW_E_INVAL, std::string(name) + ": H x W plane with this pitch runs past its allocation");
    return FLOW_OK;
}

std::vector<std::pair<int, int>> level_shapes(int H, int W, int levels) {
    std::vector<std::pair<int, int>> s;
    s.emplace_back(H, W);
    for (int l = 1; l < levels; ++l) s.emplace_back((s.back().first + 1) / 2, (s.back().second + 1) / 2);
    return s;
}

flow_status validate(const flow_params* p) {
    if (!p) return fail(FLOW_E_INVAL, "params is NULL");
    if (p->struct_size != sizeof(flow_params)) return fail(FLOW_E_INVAL, "params.struct_size mismatch");
    if (p->scheme < FLOW_PADMM || p->scheme > FLOW_ALG1) return fail(FLOW_E_INVAL, "unknown scheme");
    if (!(p->lambda > 0)) return fail(FLOW_E_INVAL, "lambda must be > 0");
    if (!(p->beta >= 0)) return fail(FLOW_E_INVAL, "beta must be >= 0");
    if (!(p->c > 0)) return fail(FLOW_E_INVAL, "c must be > 0");
    if (p->scheme == FLOW_PADMM && !(p->relax > 0 && p->relax < (1.0 + std::sqrt(5.0)) / 2.0))
        return fail(FLOW_E_INVAL, "rpADMMI relaxation r must lie in (0, (1+sqrt 5)/2)");
    if (p->scheme == FLOW_RPADMM2 && !(p->relax > 0 && p->relax < 2.0))
        return fail(FLOW_E_INVAL, "rpADMMII relaxation rho must lie in (0, 2)");
    if (!(p->sigma > 0) || !(p->tau > 0)) return fail(FLOW_E_INVAL, "sigma and tau must be > 0");
    if (p->scheme == FLOW_ALG1 && !(p->alg1_tau > 0 && p->alg1_sigma > 0 && 8.0 * p->alg1_tau * p->alg1_sigma <= 1.0 + 1e-9))
        return fail(FLOW_E_INVAL, "ALG1 steps must be > 0 with 8 alg1_tau alg1_sigma <= 1");
    if (p->gs_sweeps < 1) return fail(FLOW_E_INVAL, "gs_sweeps must be >= 1");
    if (!(p->intensity_scale > 0)) return fail(FLOW_E_INVAL, "intensity_scale must be > 0");
    if (p->levels < 1 || p->levels > FLOW_MAX_LEVELS) return fail(FLOW_E_INVAL, "levels out of range");
    if (p->warps < 1) return fail(FLOW_E_INVAL, "warps must be >= 1");
    if (p->iters < 0) return fail(FLOW_E_INVAL, "iters must be >= 0");
    if (p->storage != FLOW_STORE_F32 && p->storage != FLOW_STORE_F16) return fail(FLOW_E_INVAL, "bad storage");
    if (!(p->tol >= 0)) return fail(FLOW_E_INVAL, "tol must be >= 0");
    if (p->tol > 0 && p->check_every < 1) return fail(FLOW_E_INVAL, "check_every must be >= 1");
    return FLOW_OK;
}

flow_status validate_shape(int H, int W, int64_t ld, int levels) {
    if (H < 2 || W < 2) return fail(FLOW_E_INVAL, "H and W must be >= 2");
    // 2-D launch grids put H / 4 in the grid's y dimension (limit 65535 work-groups)
    if (H > FLOW_MAX_SIDE || W > FLOW_MAX_SIDE) return fail(FLOW_E_INVAL, "H and W must be at most FLOW_MAX_SIDE");
    if (ld < W) return fail(FLOW_E_INVAL, "pitch smaller than W");
    auto s = level_shapes(H, W, levels).back();
    if (s.first < 2 || s.second < 2) return fail(FLOW_E_INVAL, "coarsest level has a side < 2");
    return FLOW_OK;
}

// ---------------------------------------------------------------------------------------------
// Layout of one pair's working set: pyramid, linearisation and scheme state per level.
// ---------------------------------------------------------------------------------------------
size_t layout_bytes(int H, int W, const flow_params& p) {
    const bool f16 = p.storage == FLOW_STORE_F16;
    const bool pdr = pd_state(p);
    const bool hw = p.beta > 0;
    size_t total = 0;
    int lev = 0;
    for (auto [h, w] : level_shapes(H, W, p.levels)) {
        const size_t plane = (size_t)h * pitch_of(w) * 4;
        const size_t pyr = (size_t)h * pitch_of(w) * (f16 ? 2 : 4);
        total += 4 * pyr + 5 * plane;   // pyramid, linearisation, linearisation point
        if (!f16 && lev++ > 0) total += 2 * plane;   // low parts of the float-float image levels
        if (pdr) total += (size_t)(hw ? 2 * (3 + 3 + 6) + 3 + 1 : 2 * (2 + 2 + 4) + 2 + 1) * plane;
        else total += (size_t)2 * (hw ? 10 : 7) * plane;
        total += 48 * 256;  // alignment slack: every plane starts on a 256-byte boundary
    }
    return total;
}

flow_status build_layout(DevArena& arena, int H, int W, const flow_params& p, std::vector<LevelPlanes>& out) {
    const bool f16 = p.storage == FLOW_STORE_F16;
    const bool pdr = pd_state(p);
    const bool hw = p.beta > 0;
    out.clear();
    char* cur = (char*)arena.base;
    char* end = cur + arena.bytes;
    bool short_of_space = false;
    auto take = [&](size_t n) -> void* {
        char* q = (char*)(((uintptr_t)cur + 255) & ~(uintptr_t)255);
        if (q + n > end) {
            short_of_space = true;
            return nullptr;
        }
        cur = q + n;
        return q;
    };
    for (auto [h, w] : level_shapes(H, W, p.levels)) {
        LevelPlanes L{};
        L.H = h;
        L.W = w;
        L.ld = pitch_of(w);
        const size_t plane = (size_t)h * L.ld * 4;
        const size_t pyr = (size_t)h * L.ld * (f16 ? 2 : 4);
        L.I0 = take(pyr);
        L.I1 = take(pyr);
        if (!f16 && !out.empty()) {
            L.I0lo = (float*)take(plane);
            L.I1lo = (float*)take(plane);
        }
        L.Dx = take(pyr);
        L.Dy = take(pyr);
        L.Ix = (float*)take(plane);
        L.Iy = (float*)take(plane);
        L.It = (float*)take(plane);
        L.U0[0] = (float*)take(plane);
        L.U0[1] = (float*)take(plane);
        if (!pdr) {
            for (int b = 0; b < 2; ++b)
                for (int k = 0; k < 10; ++k) {
                    const bool wk = k == 0 || k == 3 || k == 4;   // w, px, py
                    L.st[b][k] = (!wk || hw) ? (float*)take(plane) : nullptr;
                }
        } else {
            for (int k = 0; k < 3; ++k) {
                const bool need = k > 0 || hw;
                for (int c = 0; c < 2; ++c) {
                    L.Xs[c][k] = need ? (float*)take(plane) : nullptr;
                    L.Xbs[c][k] = need ? (float*)take(plane) : nullptr;
                }
                L.b[k] = need ? (float*)take(plane) : nullptr;
            }
            for (int c = 0; c < 2; ++c)
                for (int k = 0; k < 6; ++k) L.ybs[c][k] = (k >= 2 || hw) ? (float*)take(plane) : nullptr;
            L.s_out = (float*)take(plane);
        }
        if (short_of_space) return fail(FLOW_E_NOMEM, "arena too small for layout");
        out.push_back(L);
    }
    return FLOW_OK;
}

// ---------------------------------------------------------------------------------------------
// Launch sequence
// ---------------------------------------------------------------------------------------------
AdmmIterArgs admm_args(const LevelPlanes& L, int from, const flow_params& p, const float* at) {
    AdmmIterArgs a{};
    const float* const* in = L.st[from];
    float* const* out = L.st[from ^ 1];
    a.w = in[0]; a.u = in[1]; a.v = in[2]; a.px = in[3]; a.py = in[4];
    a.q1x = in[5]; a.q1y = in[6]; a.q2x = in[7]; a.q2y = in[8]; a.s = in[9];
    a.wo = out[0]; a.uo = out[1]; a.vo = out[2]; a.pxo = out[3]; a.pyo = out[4];
    a.q1xo = out[5]; a.q1yo = out[6]; a.q2xo = out[7]; a.q2yo = out[8]; a.so = out[9];
    a.Ix = L.Ix; a.Iy = L.Iy; a.It = L.It; a.at = at;
    a.u0 = L.U0[0]; a.v0 = L.U0[1];
    a.H = L.H; a.W = L.W; a.ld = L.ld;
    fill_admm_coeffs(a, p);
    return a;
}

void fill_admm_coeffs(AdmmIterArgs& a, const flow_params& p) {
    const double c = p.c;
    a.c = (float)c;
    a.lam = (float)p.lambda;
    a.beta = (float)p.beta;
    a.inv_ac = (float)(1.0 / (8.0 * c));
    if (p.scheme == FLOW_RPADMM2) {
        a.c_rho_s = (float)(c * p.relax);
        a.cA = (float)(c * p.relax);
        a.cB = (float)c;
        a.cC = (float)(c * (1.0 - p.relax));
    } else {
        a.c_rho_s = (float)c;
        a.cA = (float)(c * p.relax);
        a.cB = (float)(c * p.relax);
        a.cC = 0.f;
    }
}

PdrArgs pdr_args(const LevelPlanes& L, const flow_params& p, int cur) {
    PdrArgs a{};
    float* const* X = L.Xs[cur];
    float* const* Xb = L.Xbs[cur];
    float* const* yb = L.ybs[cur];
    a.w = X[0]; a.u = X[1]; a.v = X[2];
    a.wb = Xb[0]; a.ub = Xb[1]; a.vb = Xb[2];
    a.pbx = yb[0]; a.pby = yb[1]; a.qb1x = yb[2]; a.qb1y = yb[3]; a.qb2x = yb[4]; a.qb2y = yb[5];
    a.bw = L.b[0]; a.bu = L.b[1]; a.bv = L.b[2];
    a.s_out = L.s_out;
    a.Ix = L.Ix; a.Iy = L.Iy; a.It = L.It;
    a.u0 = L.U0[0]; a.v0 = L.U0[1];
    a.H = L.H; a.W = L.W; a.ld = L.ld;
    if (p.scheme == FLOW_ALG1) {
        a.sigma = (float)p.alg1_sigma;
        a.tau = (float)p.alg1_tau;
        a.stt = 0.f;
    } else {
        a.sigma = (float)p.sigma; a.tau = (float)p.tau; a.stt = (float)(p.sigma * p.tau);
    }
    a.lam = (float)p.lambda; a.beta = (float)p.beta;
    return a;
}

void enqueue_pdr_iter(const PdrArgs& a, int sweeps, bool hw, hipStream_t s) {
    launch_pdr_rhs_red(a, hw, s);
    PdrArgs c = a;
    for (int k = 0; k < sweeps; ++k) {
        c.colour = 1;
        launch_pdr_colour(c, hw, s);                 // black
        if (k < sweeps - 1) {
            c.colour = 0;
            launch_pdr_colour(c, hw, s);             // red (the last red is fused into the final pass)
        }
    }
    launch_pdr_final(a, hw, s);
}

// Flow component k (0 = w, 1 = u, 2 = v) of a level: pDR keeps X; the ADMM family keeps the
// flow in U0 (plus the pending increment, see level_inc) and w in its current state buffer `cur`.
const float* level_flow(const LevelPlanes& L, const flow_params& p, int k, int cur) {
    if (pd_state(p)) return L.Xs[cur][k];
    if (k > 0) return L.U0[k - 1];
    return L.st[cur][0];
}

// Pending increment of flow component k (ADMM family, u and v: the last warp's du, dv in state
// buffer `cur`, not yet added to U0); nullptr where the flow is stored whole.
const float* level_inc(const LevelPlanes& L, const flow_params& p, int k, int cur) {
    if (pd_state(p) || k == 0) return nullptr;
    return L.st[cur][k];
}

EnergyArgs energy_args(const LevelPlanes& L, const flow_params& p, int cur, Scratch& sc) {
    EnergyArgs e{};
    if (pd_state(p)) {
        float* const* X = L.Xs[cur];
        float* const* yb = L.ybs[cur];
        e.w = X[0]; e.u = X[1]; e.v = X[2];
        e.px = yb[0]; e.py = yb[1]; e.q1x = yb[2]; e.q1y = yb[3]; e.q2x = yb[4]; e.q2y = yb[5];
        e.s = L.s_out;
        e.pdr_tau = p.scheme == FLOW_PDR ? (float)p.tau : 0.f;   // ALG1 keeps y itself
        e.lu0 = L.U0[0]; e.lv0 = L.U0[1];
    } else {
        // flow = U0 + the warp's increment (not yet committed)
        float* const* st = L.st[cur];
        e.w = st[0]; e.u = L.U0[0]; e.v = L.U0[1]; e.du = st[1]; e.dv = st[2];
        e.px = st[3]; e.py = st[4]; e.q1x = st[5]; e.q1y = st[6]; e.q2x = st[7]; e.q2y = st[8]; e.s = st[9];
        e.pdr_tau = 0.f;
    }
    e.Ix = L.Ix; e.Iy = L.Iy; e.It = L.It;
    e.H = L.H; e.W = L.W; e.ld = L.ld;
    e.lam = (float)p.lambda; e.beta = (float)p.beta;
    e.partial = sc.e_partial; e.out = sc.e_out;
    return e;
}

// Tile plan of every level plus the device tables the tile kernel reads (ADMM family only).
flow_status make_plan(std::vector<LevelPlanes>& Ls, const flow_params& p, Scratch& sc, SolvePlan& out,
                      const std::map<std::string, TunedChoice>* tuned, bool upload) {
    out.levels.clear();
    out.pdr.clear();
    if (pd_state(p)) {
        for (const LevelPlanes& L : Ls) out.pdr.push_back(plan_pdr_level(L.H, L.W, p, tuned));
        return FLOW_OK;
    }
    const bool hw = p.beta > 0;
    std::vector<TbTile> tiles;
    std::vector<TbLevel> descs(2 * Ls.size());
    for (size_t l = 0; l < Ls.size(); ++l) {
        LevelTbPlan P = plan_level_tuned(Ls[l].H, Ls[l].W, hw, p.iters, tuned);
        if (P.tb) {
            P.tile_off = (int)tiles.size();
            append_tiles(P, (int)l, Ls[l].H, Ls[l].W, tiles);
            P.ntiles = (int)tiles.size() - P.tile_off;
        }
        fill_tb_level(&descs[2 * l], Ls[l], sc.at);
        out.levels.push_back(P);
    }
    if (!upload) return FLOW_OK;
    out.tables.reset(new TbTables());
    return out.tables->upload(tiles, descs);
}

TbArgs tb_args(const SolvePlan& plan, const LevelTbPlan& P, const LevelPlanes& L, const flow_params& p, int cur,
               int K, int at_slot, const float* at2) {
    AdmmIterArgs co{};
    fill_admm_coeffs(co, p);
    TbArgs a{};
    (void)plan;
    a.ntiles = P.ntiles;
    a.dir = cur;
    a.K = K;
    a.at_slot = at_slot;
    a.queue = nullptr;                 // one level per launch: direct mode
    a.c = co.c; a.lam = co.lam; a.beta = co.beta; a.inv_ac = co.inv_ac; a.c_rho_s = co.c_rho_s;
    a.cA = co.cA; a.cB = co.cB; a.cC = co.cC;
    TbLevel d[2];
    fill_tb_level(d, L, at2);
    a.lvl = d[cur];
    a.th = P.th;
    a.tw = P.tw;
    a.ntx = (L.W + P.tw - 1) / P.tw;
    return a;
}

// `n` ADMM-family iterations of level L starting from state buffer `cur`, with the kernel choice
// of plan P (nullptr: one-pass kernel, strip height rows_hint); returns the buffer holding the result.
int enqueue_admm_iters(const LevelPlanes& L, const flow_params& p, const LevelTbPlan* P, int rows_hint, int cur,
                       int64_t n, int at_slot, const float* at2, hipStream_t s, int64_t* launches) {
    const bool hw = p.beta > 0;
    int64_t t = 0;
    while (t < n) {
        if (P) {
            const int kk = (int)std::min<int64_t>(P->resident ? n - t : P->K, n - t);
            launch_admm_tb(tb_args(SolvePlan(), *P, L, p, cur, kk, at_slot, at2), hw, P->nt, P->ntiles, s);
            t += kk;
        } else {
            AdmmIterArgs ai = admm_args(L, cur, p, at2 + at_slot);
            ai.rows = rows_hint;
            launch_admm_iter(ai, hw, s);
            t += 1;
        }
        if (launches) ++*launches;
        cur ^= 1;
    }
    return cur;
}

int g_pdr_mode = 0;   // pDR iteration kernel: 0 built-in (tiles), 1 three-pass, 5 tiles of 1024 threads, 6 of 512,
                      // 10 / 11 tiles of 1024 / 512 threads with two cells of each colour per thread (beta = 0),
                      // 12 / 13 wave-row tiles of 128 x 32 / 128 x 48 cells (13: beta = 0), 14 / 15 of
                      // 64 x 48 / 64 x 32 cells, one per lane (14: beta = 0)
int g_pdr_k = 0;      // iterations per pDR tile launch (0 = built-in)

std::string pd_tune_key(int H, int W, const flow_params& p) {
    const std::string k = tune_key(H, W, p.beta > 0, p.iters);
    return p.scheme == FLOW_ALG1 ? k + "a" : k + "p" + std::to_string(p.gs_sweeps);
}

// Halo of a K-iteration tile with (X, X bar, y) state, summed over both sides of an axis.
int pd_halo(const flow_params& p, int K) {
    return p.scheme == FLOW_ALG1 ? 2 * alg1_halo(K) : pdr_halo_lo(p.gs_sweeps, K) + pdr_halo_hi(p.gs_sweeps, K);
}

PdrTbPlan plan_pdr_level(int H, int W, const flow_params& p, const std::map<std::string, TunedChoice>* tuned) {
    const bool hw = p.beta > 0;
    const bool alg1 = p.scheme == FLOW_ALG1;
    int mode = alg1 ? 0 : g_pdr_mode, K = alg1 ? 0 : g_pdr_k;
    if (mode == 0 && tuned) {
        auto it = tuned->find(pd_tune_key(H, W, p));
        if (it != tuned->end()) {
            mode = it->second.mode;
            K = it->second.K;
        }
    }
    if (alg1 && mode == 1) mode = 5;                 // ALG1 has no three-pass form
    if ((mode == 10 || mode == 11) && (alg1 || hw)) mode -= 5;   // two cells per colour: pDR without w only
    if ((mode == 12 || mode == 13) && alg1) mode = 5;            // cell-pair wave-row tiles: pDR only
    if (mode == 13 && hw) mode = 12;                             // 128 x 48 cells without the w block only
    if (mode == 14 && hw) mode = 15;                             // 64 x 48 cells without the w block only
    if (mode == 1 || p.iters < 1) return PdrTbPlan();
    const int nt = mode == 6 ? 512 : mode == 10 ? 2048 : mode == 11 ? 513 : mode == 12 ? 4098 : mode == 13 ? 6145
                 : mode == 14 ? 3074 : mode == 15 ? 2050 : 1024;
    const int kdef = alg1 ? kAlg1DefaultK : kPdrDefaultK;
    const int k0 = K > 0 ? K : kdef;
    PdrTbPlan T = plan_pd_tiles(H, W, hw, pd_halo(p, k0), k0, 0, nt);
    if (T.resident && K == 0) T.K = p.iters;        // the whole warp in one launch
    if (!T.tb) {                                     // the halo does not fit: fewer iterations per launch
        for (int k = k0 - 1; k >= 1 && !T.tb; --k) T = plan_pd_tiles(H, W, hw, pd_halo(p, k), k, 0, nt);
    }
    return T;
}

PdrTbArgs pdr_tb_args(const LevelPlanes& L, const flow_params& p, const PdrTbPlan& T, int cur, int K) {
    PdrTbArgs a{};
    const int xs[3] = {1, 2, 0};                    // kernel order u, v, w <- layout order w, u, v
    const int ys[6] = {2, 3, 4, 5, 0, 1};           // q1x q1y q2x q2y p_x p_y <- p_x p_y q1x q1y q2x q2y
    for (int c = 0; c < 3; ++c) {
        a.lvl.x_in[c] = L.Xs[cur][xs[c]];
        a.lvl.xb_in[c] = L.Xbs[cur][xs[c]];
        a.lvl.x_out[c] = L.Xs[cur ^ 1][xs[c]];
        a.lvl.xb_out[c] = L.Xbs[cur ^ 1][xs[c]];
    }
    for (int c = 0; c < 6; ++c) {
        a.lvl.y_in[c] = L.ybs[cur][ys[c]];
        a.lvl.y_out[c] = L.ybs[cur ^ 1][ys[c]];
    }
    a.lvl.Ix = L.Ix; a.lvl.Iy = L.Iy; a.lvl.It = L.It;
    a.lvl.u0 = L.U0[0]; a.lvl.v0 = L.U0[1];
    a.lvl.s_out = L.s_out;
    a.lvl.H = L.H; a.lvl.W = L.W; a.lvl.ld = L.ld;
    a.K = K;
    a.th = T.th; a.tw = T.tw;
    a.ntx = (L.W + T.tw - 1) / T.tw;
    a.ntiles = a.ntx * ((L.H + T.th - 1) / T.th);
    pd_tile_scalars(a, p);
    return a;
}

void pd_tile_scalars(PdrTbArgs& a, const flow_params& p) {
    a.sweeps = p.gs_sweeps;
    if (p.scheme == FLOW_ALG1) {
        a.sigma = (float)p.alg1_sigma;
        a.tau = (float)p.alg1_tau;
        a.stt = 0.f;
    } else {
        a.sigma = (float)p.sigma; a.tau = (float)p.tau; a.stt = (float)(p.sigma * p.tau);
    }
    a.lam = (float)p.lambda; a.beta = (float)p.beta;
}

// `n` pDR or ALG1 iterations of level L on K-iteration tiles starting from state set `cur`; returns
// the set holding the result.
int enqueue_pdr_tiles(const LevelPlanes& L, const flow_params& p, const PdrTbPlan& T, int cur, int64_t n,
                      hipStream_t s, int64_t* launches) {
    int64_t t = 0;
    while (t < n) {
        const int kk = (int)std::min<int64_t>(T.resident ? n - t : T.K, n - t);
        if (p.scheme == FLOW_ALG1) launch_alg1_tb(pdr_tb_args(L, p, T, cur, kk), p.beta > 0, T.nt, s);
        else launch_pdr_tb(pdr_tb_args(L, p, T, cur, kk), p.beta > 0, T.nt, s);
        if (launches) ++*launches;
        cur ^= 1;
        t += kk;
    }
    return cur;
}

// Everything after the level-0 frames are in the pyramid: pyramid, levels, warps, iterations,
// final energy.  `timers` (may be null) receives events around each warp's iteration block.
flow_status enqueue_core(std::vector<LevelPlanes>& Ls, const flow_params& p, Scratch& sc, hipStream_t s,
                         WarpTimers* timers, StopTest* stop, const SolvePlan* plan) {
    const bool f16 = p.storage == FLOW_STORE_F16;
    const bool pdr = pd_state(p);      // pDR or ALG1: state (X, X bar, y)
    const bool hw = p.beta > 0;
    const int nl = (int)Ls.size();
    for (int l = 0; l < nl; ++l) {
        LevelPlanes& L = Ls[l];
        if (l > 0) {
            const LevelPlanes& F = Ls[l - 1];
            launch_downsample(F.I0, F.H, F.W, F.ld, L.I0, L.ld, f16, s, F.I0lo, L.I0lo);
            launch_downsample(F.I1, F.H, F.W, F.ld, L.I1, L.ld, f16, s, F.I1lo, L.I1lo);
        }
        launch_derivatives(L.I1, L.H, L.W, L.ld, L.Dx, L.Dy, L.ld, f16, s, L.I1lo);
    }
    int cur_coarse = 0;
    for (int l = nl - 1; l >= 0; --l) {
        LevelPlanes& L = Ls[l];
        const LevelTbPlan* P = (plan && !pdr && l < (int)plan->levels.size() && plan->levels[l].tb)
                                   ? &plan->levels[l] : nullptr;
        const int rows_hint = (plan && !pdr && l < (int)plan->levels.size()) ? plan->levels[l].rows : 0;
        // level start: upsample flow from level l+1 (or zero), clear duals
        LevelInitArgs ia{};
        ia.H = L.H; ia.W = L.W; ia.ld = L.ld;
        if (l < nl - 1) {
            const LevelPlanes& C = Ls[l + 1];
            ia.uc = level_flow(C, p, 1, cur_coarse);
            ia.vc = level_flow(C, p, 2, cur_coarse);
            ia.ucd = level_inc(C, p, 1, cur_coarse);
            ia.vcd = level_inc(C, p, 2, cur_coarse);
            ia.wc = hw ? level_flow(C, p, 0, cur_coarse) : nullptr;
            ia.Hc = C.H; ia.Wc = C.W; ia.ldc = C.ld;
        }
        if (!pdr) {
            ia.set_flow[0] = hw ? L.st[0][0] : nullptr;
            ia.set_flow[1] = L.U0[0];
            ia.set_flow[2] = L.U0[1];
            int nz = 0;
            for (int k = 3; k < 10; ++k)
                if (L.st[0][k]) ia.zero[nz++] = L.st[0][k];
            ia.nzero = nz;
        } else {
            ia.set_flow[0] = hw ? L.Xs[0][0] : nullptr;
            ia.set_flow[1] = L.Xs[0][1];
            ia.set_flow[2] = L.Xs[0][2];
            ia.copy_flow[0] = hw ? L.Xbs[0][0] : nullptr;
            ia.copy_flow[1] = L.Xbs[0][1];
            ia.copy_flow[2] = L.Xbs[0][2];
            int nz = 0;
            for (int k = 0; k < 6; ++k)
                if (L.ybs[0][k]) ia.zero[nz++] = L.ybs[0][k];
            ia.zero[nz++] = L.s_out;
            ia.nzero = nz;
        }
        ia.clear_scalar = sc.at;     // a~ slot of the level's first warp
        launch_level_init(ia, s);

        int cur = 0;                 // ADMM: state buffer holding the current iterate
        for (int wp = 0; wp < p.warps; ++wp) {
            // warp start: linearise around the current flow with I_t relative to it; the ADMM
            // increment (du, dv) restarts at zero, pDR keeps a copy of the linearisation point
            LinArgs la{};
            la.I0 = L.I0; la.I1 = L.I1; la.Dx = L.Dx; la.Dy = L.Dy;
            la.I0lo = L.I0lo; la.I1lo = L.I1lo;
            la.u0 = const_cast<float*>(level_flow(L, p, 1, cur));
            la.v0 = const_cast<float*>(level_flow(L, p, 2, cur));
            if (wp > 0) {                // commit the previous warp's increment on the way
                la.pend_u = level_inc(L, p, 1, cur);
                la.pend_v = level_inc(L, p, 2, cur);
            }
            la.Ix = L.Ix; la.Iy = L.Iy; la.It = L.It;
            la.at = sc.at + (wp & 1);
            la.at_clear = sc.at + ((wp + 1) & 1);
            la.H = L.H; la.W = L.W; la.ld = L.ld;
            la.kappa = (float)p.intensity_scale; la.beta = (float)p.beta;
            la.rel = 1;
            if (!pdr) {
                la.zero_u = L.st[cur][1];
                la.zero_v = L.st[cur][2];
            } else {
                la.keep_u = L.U0[0];
                la.keep_v = L.U0[1];
            }
            launch_linearize(la, f16, s);
            if (timers) timers->begin(l, s);
            int64_t k = 0;
            while (k < p.iters) {
                int64_t chunk = p.iters - k;
                if (stop && p.tol > 0) chunk = std::min<int64_t>(chunk, p.check_every);
                int64_t nk = 0;
                if (pdr) {
                    const PdrTbPlan* T = (plan && l < (int)plan->pdr.size() && plan->pdr[l].tb) ? &plan->pdr[l]
                                                                                                  : nullptr;
                    if (T) {
                        cur = enqueue_pdr_tiles(L, p, *T, cur, chunk, s, &nk);
                    } else if (p.scheme == FLOW_ALG1) {
                        return fail(FLOW_E_INVAL, "no ALG1 tile plan for this level");
                    } else {
                        for (int64_t t = 0; t < chunk; ++t) enqueue_pdr_iter(pdr_args(L, p, cur), p.gs_sweeps, hw, s);
                        nk = chunk * (2 * p.gs_sweeps + 1);
                    }
                } else {
                    cur = enqueue_admm_iters(L, p, P, rows_hint, cur, chunk, wp & 1, sc.at, s, &nk);
                }
                k += chunk;
                if (timers) timers->count(l, chunk, nk);
                if (stop && p.tol > 0 && k < p.iters) {
                    launch_energy(energy_args(L, p, cur, sc), s);
                    bool converged = false;
                    flow_status st = stop->check(sc, s, &converged);
                    if (st != FLOW_OK) return st;
                    if (converged) break;
                }
            }
            if (timers) timers->end(l, s);
            const bool last = l == 0 && wp == p.warps - 1;
            if (last) launch_energy(energy_args(L, p, cur, sc), s);
            // the warp's increment stays pending in st[cur]: the next linearisation, the next level's
            // upsampling or the export adds it (ADMM family)
        }
        cur_coarse = cur;
        if (l == 0) sc.final_buf = cur;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return FLOW_OK;
}

}  // namespace flowmi

using namespace flowmi;

// =============================================================================================
// C ABI
// =============================================================================================
extern "C" {

flow_status flow_params_default(flow_params* p) {
    if (!p) return fail(FLOW_E_INVAL, "params is NULL");
    std::memset(p, 0, sizeof(*p));
    p->struct_size = sizeof(flow_params);
    p->scheme = FLOW_PADMM;
    p->lambda = 0.05;
    p->beta = 0.0;
    p->c = 0.05;
    p->relax = 1.0;
    p->sigma = 2.0;
    p->tau = 0.4;
    p->gs_sweeps = 1;
    p->intensity_scale = 255.0;
    p->levels = 5;
    p->warps = 5;
    p->iters = 50;
    p->alg1_tau = 0.1;
    p->alg1_sigma = 1.25;
    p->storage = FLOW_STORE_F32;
    p->use_graph = 1;
    p->tol = 0.0;
    p->check_every = 10;
    return FLOW_OK;
}

const char* flow_last_error(void) { return g_last_error.c_str(); }

flow_status flow_tune_set(const char* key, int64_t value) {
    if (!key) return fail(FLOW_E_INVAL, "key is NULL");
    if (std::strcmp(key, "admm_rows") == 0) {
        if (value != 0 && value != 2 && value != 4 && value != 8) return fail(FLOW_E_INVAL, "admm_rows: 0, 2, 4 or 8");
        g_admm_rows_override = (int)value;
        return FLOW_OK;
    }
    if (std::strcmp(key, "tb_mode") == 0) {
        if (value < 0 || value > 14 || value == 5 || value == 10 || value == 11)
            return fail(FLOW_E_INVAL, "tb_mode: 0 built-in, 1 one-pass, 2 tiles/256, 3 tiles/1024, 4 / 7 / 6 small "
                                      "tiles of 1024 / 512 / 256 threads, 8 / 9 one-pixel tiles of 1024 / 512 threads, "
                                      "12 / 13 / 14 wave-row tiles of 32 / 48 / 64 rows");
        g_tb_mode = (int)value;
        return FLOW_OK;
    }
    if (std::strcmp(key, "tb_k") == 0) {
        if (value < 0 || value > 64) return fail(FLOW_E_INVAL, "tb_k: 0 (default) .. 64");
        g_tb_k = (int)value;
        return FLOW_OK;
    }
    if (std::strcmp(key, "pdr_mode") == 0) {
        if (value != 0 && value != 1 && value != 5 && value != 6 && (value < 10 || value > 15))
            return fail(FLOW_E_INVAL, "pdr_mode: 0 built-in, 1 three-pass, 5 tiles of 1024 threads, 6 of 512, "
                                      "10 / 11 tiles of 1024 / 512 threads with two cells of each colour per "
                                      "thread (beta = 0; 5 / 6 otherwise), 12 / 13 wave-row tiles of 128 x 32 / "
                                      "128 x 48 cells (13: beta = 0; 12 otherwise), 14 / 15 wave-row tiles of "
                                      "64 x 48 / 64 x 32 cells (14: beta = 0; 15 otherwise)");
        g_pdr_mode = (int)value;
        return FLOW_OK;
    }
    if (std::strcmp(key, "pdr_k") == 0) {
        if (value < 0 || value > 64) return fail(FLOW_E_INVAL, "pdr_k: 0 (built-in) .. 64");
        g_pdr_k = (int)value;
        return FLOW_OK;
    }
    if (std::strcmp(key, "batch_order") == 0) {
        if (value < -1 || value > 1) return fail(FLOW_E_INVAL, "batch_order: -1 tuned / built-in, 0 table, 1 queue");
        g_batch_order = (int)value;
        return FLOW_OK;
    }
    if (std::strcmp(key, "batch_k") == 0) {
        if (value < 0 || value > 64) return fail(FLOW_E_INVAL, "batch_k: 0 (tuned / built-in) .. 64");
        g_batch_k = (int)value;
        return FLOW_OK;
    }
    if (std::strcmp(key, "serve_graph") == 0) {
        if (value != 0 && value != 1) return fail(FLOW_E_INVAL, "serve_graph: 0 direct launches, 1 graph replay");
        g_serve_graph = (int)value;
        return FLOW_OK;
    }
    if (std::strcmp(key, "batch_nt") == 0) {
        if (value != 0 && value != 1025 && !is_rows_code((int)value))
            return fail(FLOW_E_INVAL, "batch_nt: 0 (tuned / built-in), 1025 (general tiles) or a wave-row code "
                                      "2049 / 3073 / 4097");
        g_batch_nt = (int)value;
        return FLOW_OK;
    }
    if (std::strcmp(key, "batch_ew") == 0) {
        if (value != 0 && (value < 16 || value > 512)) return fail(FLOW_E_INVAL, "batch_ew: 0 (tuned / built-in) or 16 .. 512");
        g_batch_ew = (int)value;
        return FLOW_OK;
    }
    return fail(FLOW_E_INVAL, std::string("unknown tuning key ") + key);
}

flow_status flow_create(flow_ctx** out, int device, size_t budget) {
    if (!out) return fail(FLOW_E_INVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(FLOW_E_INVAL, "no such device");
    HIP_TRY(hipSetDevice(device));
    std::unique_ptr<flow_ctx> c(new flow_ctx());
    c->device = device;
    c->budget = budget;
    flow_status st = c->init_scratch();
    if (st != FLOW_OK) return st;
    *out = c.release();
    return FLOW_OK;
}

flow_status flow_destroy(flow_ctx* ctx) {
    if (!ctx) return FLOW_OK;
    hipSetDevice(ctx->device);
    delete ctx;
    return FLOW_OK;
}

flow_status flow_set_stats(flow_ctx* ctx, int32_t enable) {
    if (!ctx) return fail(FLOW_E_INVAL, "ctx is NULL");
    ctx->stats_enabled = enable != 0;
    return FLOW_OK;
}

flow_status flow_get_stats(const flow_ctx* ctx, flow_stats* out) {
    if (!ctx || !out) return fail(FLOW_E_INVAL, "NULL argument");
    *out = ctx->last_stats;
    return FLOW_OK;
}

flow_status flow_memory_in_use(const flow_ctx* ctx, size_t* bytes) {
    if (!ctx || !bytes) return fail(FLOW_E_INVAL, "NULL argument");
    *bytes = ctx->bytes_in_use();
    return FLOW_OK;
}

flow_status flow_solve(flow_ctx* ctx, const float* I0, const float* I1, int32_t H, int32_t W, int64_t ld,
                       const flow_params* p, float* u, float* v, int64_t ld_uv, flow_result* res, void* stream) {
    if (!ctx) return fail(FLOW_E_INVAL, "ctx is NULL");
    if (!I0 || !I1 || !u || !v) return fail(FLOW_E_INVAL, "NULL device pointer");
    flow_status st = validate(p);
    if (st != FLOW_OK) return st;
    st = validate_shape(H, W, ld, p->levels);
    if (st != FLOW_OK) return st;
    if (ld_uv < W) return fail(FLOW_E_INVAL, "ld_uv smaller than W");
    HIP_TRY(hipSetDevice(ctx->device));
    for (auto [ptr, l, name] : {std::make_tuple((const void*)I0, ld, "I0"), std::make_tuple((const void*)I1, ld, "I1"),
                                std::make_tuple((const void*)u, ld_uv, "u"), std::make_tuple((const void*)v, ld_uv, "v")}) {
        st = check_extent(ptr, H, W, l, sizeof(float), name);
        if (st != FLOW_OK) return st;
    }
    return ctx->solve(I0, I1, H, W, ld, *p, u, v, ld_uv, res, (hipStream_t)stream);
}

// ------------------------------- operator-level entry points ---------------------------------
#define EXTENT(ptr, h, w, ld, name)                                                   \
    do {                                                                              \
        flow_status _s = check_extent((ptr), (h), (w), (ld), sizeof(float), (name));  \
        if (_s != FLOW_OK) return _s;                                                 \
    } while (0)

flow_status flow_op_downsample(const float* src, int32_t H, int32_t W, int64_t ld, float* dst, int64_t ldd,
                               void* stream) {
    if (!src || !dst) return fail(FLOW_E_INVAL, "NULL pointer");
    if (H < 1 || W < 1 || ld < W || ldd < (W + 1) / 2) return fail(FLOW_E_INVAL, "bad shape");
    EXTENT(src, H, W, ld, "src");
    EXTENT(dst, (H + 1) / 2, (W + 1) / 2, ldd, "dst");
    launch_downsample(src, H, W, ld, dst, ldd, false, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return FLOW_OK;
}

flow_status flow_op_derivatives(const float* I, int32_t H, int32_t W, int64_t ld, float* Dx, float* Dy,
                                void* stream) {
    if (!I || !Dx || !Dy) return fail(FLOW_E_INVAL, "NULL pointer");
    if (H < 1 || W < 1 || ld < W) return fail(FLOW_E_INVAL, "bad shape");
    EXTENT(I, H, W, ld, "I");
    EXTENT(Dx, H, W, ld, "Dx");
    EXTENT(Dy, H, W, ld, "Dy");
    launch_derivatives(I, H, W, ld, Dx, Dy, ld, false, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return FLOW_OK;
}

flow_status flow_op_linearize(const float* I0, const float* I1, const float* DxI1, const float* DyI1,
                              const float* u0, const float* v0, int32_t H, int32_t W, int64_t ld, double kappa,
                              double beta, float* Ix, float* Iy, float* It, float* at_out, void* stream) {
    if (!I0 || !I1 || !DxI1 || !DyI1 || !u0 || !v0 || !Ix || !Iy || !It || !at_out)
        return fail(FLOW_E_INVAL, "NULL pointer");
    if (H < 2 || W < 2 || ld < W) return fail(FLOW_E_INVAL, "bad shape");
    EXTENT(I0, H, W, ld, "I0"); EXTENT(I1, H, W, ld, "I1"); EXTENT(DxI1, H, W, ld, "DxI1");
    EXTENT(DyI1, H, W, ld, "DyI1"); EXTENT(u0, H, W, ld, "u0"); EXTENT(v0, H, W, ld, "v0");
    EXTENT(Ix, H, W, ld, "Ix"); EXTENT(Iy, H, W, ld, "Iy"); EXTENT(It, H, W, ld, "It");
    EXTENT(at_out, 1, 1, 1, "at_out");
    HIP_TRY(hipMemsetAsync(at_out, 0, sizeof(float), (hipStream_t)stream));
    LinArgs a{};
    a.I0 = I0; a.I1 = I1; a.Dx = DxI1; a.Dy = DyI1; a.u0 = const_cast<float*>(u0); a.v0 = const_cast<float*>(v0);   // read only: no pending increment
    a.Ix = Ix; a.Iy = Iy; a.It = It; a.at = at_out;
    a.H = H; a.W = W; a.ld = ld; a.kappa = (float)kappa; a.beta = (float)beta;
    launch_linearize(a, false, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return FLOW_OK;
}

flow_status flow_op_upsample(const float* coarse, int64_t ldc, float* fine, int32_t Hf, int32_t Wf, int64_t ldf,
                             double scale, void* stream) {
    if (!coarse || !fine) return fail(FLOW_E_INVAL, "NULL pointer");
    if (Hf < 3 || Wf < 3 || ldf < Wf || ldc < (Wf + 1) / 2) return fail(FLOW_E_INVAL, "bad shape");
    EXTENT(coarse, (Hf + 1) / 2, (Wf + 1) / 2, ldc, "coarse");
    EXTENT(fine, Hf, Wf, ldf, "fine");
    launch_upsample(coarse, ldc, fine, Hf, Wf, ldf, (float)scale, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return FLOW_OK;
}

flow_status flow_op_admm_iter(const flow_admm_state* in, const flow_admm_state* out, const float* Ix,
                              const float* Iy, const float* It, const float* at, int32_t H, int32_t W, int64_t ld,
                              const flow_params* p, void* stream) {
    flow_status st = validate(p);
    if (st != FLOW_OK) return st;
    if (p->scheme == FLOW_PDR) return fail(FLOW_E_INVAL, "flow_op_admm_iter needs an ADMM scheme");
    if (!in || !out || !Ix || !Iy || !It || !at) return fail(FLOW_E_INVAL, "NULL pointer");
    const bool hw = p->beta > 0;
    const float* ins[10] = {in->w, in->u, in->v, in->px, in->py, in->q1x, in->q1y, in->q2x, in->q2y, in->s};
    float* outs[10] = {out->w, out->u, out->v, out->px, out->py, out->q1x, out->q1y, out->q2x, out->q2y, out->s};
    for (int k = 0; k < 10; ++k) {
        const bool wk = k == 0 || k == 3 || k == 4;
        if ((!wk || hw) && (!ins[k] || !outs[k])) return fail(FLOW_E_INVAL, "NULL state plane");
        if ((!wk || hw) && ins[k] == outs[k]) return fail(FLOW_E_INVAL, "in and out planes must differ");
    }
    if (H < 2 || W < 2 || ld < W) return fail(FLOW_E_INVAL, "bad shape");
    for (int k = 0; k < 10; ++k) {
        const bool wk = k == 0 || k == 3 || k == 4;
        if (wk && !hw) continue;
        EXTENT(ins[k], H, W, ld, "state in");
        EXTENT(outs[k], H, W, ld, "state out");
    }
    EXTENT(Ix, H, W, ld, "Ix"); EXTENT(Iy, H, W, ld, "Iy"); EXTENT(It, H, W, ld, "It");
    EXTENT(at, 1, 1, 1, "at");
    AdmmIterArgs a{};
    a.w = ins[0]; a.u = ins[1]; a.v = ins[2]; a.px = ins[3]; a.py = ins[4];
    a.q1x = ins[5]; a.q1y = ins[6]; a.q2x = ins[7]; a.q2y = ins[8]; a.s = ins[9];
    a.wo = outs[0]; a.uo = outs[1]; a.vo = outs[2]; a.pxo = outs[3]; a.pyo = outs[4];
    a.q1xo = outs[5]; a.q1yo = outs[6]; a.q2xo = outs[7]; a.q2yo = outs[8]; a.so = outs[9];
    a.Ix = Ix; a.Iy = Iy; a.It = It; a.at = at; a.H = H; a.W = W; a.ld = ld;
    if ((in->u0 == nullptr) != (in->v0 == nullptr)) return fail(FLOW_E_INVAL, "u0 and v0 go together");
    if (in->u0) {
        EXTENT(in->u0, H, W, ld, "u0");
        EXTENT(in->v0, H, W, ld, "v0");
        a.u0 = in->u0;
        a.v0 = in->v0;
    }
    fill_admm_coeffs(a, *p);
    launch_admm_iter(a, hw, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return FLOW_OK;
}

flow_status flow_op_admm_tb(const flow_admm_state* in, const flow_admm_state* out, const float* Ix, const float* Iy,
                            const float* It, const float* at, int32_t H, int32_t W, int64_t ld, const flow_params* p,
                            int32_t iters, int32_t threads, int32_t tile_h, int32_t tile_w, int32_t order,
                            void* stream) {
    flow_status st = validate(p);
    if (st != FLOW_OK) return st;
    if (p->scheme == FLOW_PDR) return fail(FLOW_E_INVAL, "flow_op_admm_tb needs an ADMM scheme");
    if (!in || !out || !Ix || !Iy || !It || !at) return fail(FLOW_E_INVAL, "NULL pointer");
    if (!in->u0 || !in->v0) return fail(FLOW_E_INVAL, "the tile kernel runs the increment form: u0, v0 required");
    if (H < 2 || W < 2 || ld < W) return fail(FLOW_E_INVAL, "bad shape");
    if (threads != 256 && threads != 1024 && threads != 1025 && threads != 513 && threads != 257 && threads != 1026 &&
        threads != 514 && !is_rows_code(threads))
        return fail(FLOW_E_INVAL, "threads must be 256, 1024, a small-tile code 1025 / 513 / 257 / 1026 / 514 or a "
                                  "wave-row code 2049 / 3073 / 4097");
    if (iters < 1 || tile_h < 1 || tile_w < 1) return fail(FLOW_E_INVAL, "iters, tile_h, tile_w must be >= 1");
    if (order < 0 || order > 3) return fail(FLOW_E_INVAL, "order must be 0, 1, 2 or 3");
    if ((threads == 513 || threads == 257 || threads == 1026 || threads == 514) && order != 0)
        return fail(FLOW_E_INVAL, "work-group codes 513, 257, 1026 and 514 run with direct tiling (order 0) only");
    if (is_rows_code(threads) && order != 0 && order != 3)
        return fail(FLOW_E_INVAL, "wave-row codes run with direct tiling or table order (0 or 3) only");
    const bool hw = p->beta > 0;
    const int64_t halo = (int64_t)tb_halo_lo(iters) + tb_halo_hi(iters);
    if (!tb_fits(hw, threads, std::min<int64_t>(H, tile_h + halo), std::min<int64_t>(W, tile_w + halo)))
        return fail(FLOW_E_INVAL, "tile plus halo exceeds the tile kernel's capacity");
    const float* ins[10] = {in->w, in->u, in->v, in->px, in->py, in->q1x, in->q1y, in->q2x, in->q2y, in->s};
    float* outs[10] = {out->w, out->u, out->v, out->px, out->py, out->q1x, out->q1y, out->q2x, out->q2y, out->s};
    for (int k = 0; k < 10; ++k) {
        const bool wk = k == 0 || k == 3 || k == 4;
        if (wk && !hw) continue;
        if (!ins[k] || !outs[k] || ins[k] == outs[k]) return fail(FLOW_E_INVAL, "bad state plane");
        EXTENT(ins[k], H, W, ld, "state in");
        EXTENT(outs[k], H, W, ld, "state out");
    }
    EXTENT(Ix, H, W, ld, "Ix"); EXTENT(Iy, H, W, ld, "Iy"); EXTENT(It, H, W, ld, "It");
    EXTENT(in->u0, H, W, ld, "u0"); EXTENT(in->v0, H, W, ld, "v0"); EXTENT(at, 1, 1, 1, "at");
    LevelTbPlan P;
    P.tb = true;
    P.nt = threads;
    P.K = iters;
    P.th = tile_h;
    P.tw = tile_w;
    std::vector<TbTile> tiles;
    append_tiles(P, 0, H, W, tiles);
    P.ntiles = (int)tiles.size();
    std::vector<TbLevel> descs(2);
    for (int k = 0; k < 10; ++k) {
        descs[0].in[k] = ins[k];
        descs[0].out[k] = outs[k];
    }
    descs[0].Ix = Ix; descs[0].Iy = Iy; descs[0].It = It; descs[0].u0 = in->u0; descs[0].v0 = in->v0;
    descs[0].at = at; descs[0].H = H; descs[0].W = W; descs[0].ld = ld;
    descs[1] = descs[0];
    TbTables tab;
    st = tab.upload(tiles, descs);
    if (st != FLOW_OK) return st;
    unsigned* q = nullptr;
    HIP_TRY(hipMalloc(&q, 256));
    hipStream_t s = (hipStream_t)stream;
    launch_reset_u32(q, 8, s);
    const bool use_queue = order == 1 || order == 2;
    const int grid = use_queue ? tb_grid(P, P.ntiles) : P.ntiles;
    AdmmIterArgs co{};
    fill_admm_coeffs(co, *p);
    TbArgs a{};
    a.tiles = order == 0 ? nullptr : tab.d_tiles;
    a.ntiles = P.ntiles; a.levels = tab.d_levels; a.dir = 0; a.K = iters; a.at_slot = 0;
    a.queue = use_queue ? q : nullptr; a.queue_base = 0;
    a.nq = order == 2 ? std::min(8, grid) : 1;
    a.c = co.c; a.lam = co.lam; a.beta = co.beta; a.inv_ac = co.inv_ac; a.c_rho_s = co.c_rho_s;
    a.cA = co.cA; a.cB = co.cB; a.cC = co.cC;
    a.lvl = descs[0];
    a.th = tile_h;
    a.tw = tile_w;
    a.ntx = (W + tile_w - 1) / tile_w;
    launch_admm_tb(a, hw, threads, grid, s);
    hipError_t e = hipGetLastError();
    hipError_t e2 = hipStreamSynchronize(s);
    hipFree(q);
    if (e != hipSuccess) return hip_fail(e, "tile kernel launch");
    if (e2 != hipSuccess) return hip_fail(e2, "tile kernel");
    return FLOW_OK;
}

flow_status flow_op_pdr_iter(const flow_pdr_state* st, float* work0, float* work1, float* work2, float* s_out,
                             const float* Ix, const float* Iy, const float* It, int32_t H, int32_t W, int64_t ld,
                             const flow_params* p, void* stream) {
    flow_status v = validate(p);
    if (v != FLOW_OK) return v;
    if (!st || !work1 || !work2 || !Ix || !Iy || !It) return fail(FLOW_E_INVAL, "NULL pointer");
    const bool hw = p->beta > 0;
    if (!st->u || !st->v || !st->ub || !st->vb || !st->qb1x || !st->qb1y || !st->qb2x || !st->qb2y)
        return fail(FLOW_E_INVAL, "NULL state plane");
    if (hw && (!st->w || !st->wb || !st->pbx || !st->pby || !work0)) return fail(FLOW_E_INVAL, "NULL w-block plane");
    if (H < 2 || W < 2 || ld < W) return fail(FLOW_E_INVAL, "bad shape");
    {
        const float* planes[] = {st->u, st->v, st->ub, st->vb, st->qb1x, st->qb1y, st->qb2x, st->qb2y, work1, work2,
                                 Ix, Iy, It};
        for (const float* q : planes) EXTENT(q, H, W, ld, "pDR plane");
        if (hw) {
            const float* wp[] = {st->w, st->wb, st->pbx, st->pby, work0};
            for (const float* q : wp) EXTENT(q, H, W, ld, "pDR w-block plane");
        }
        if (s_out) EXTENT(s_out, H, W, ld, "s_out");
    }
    PdrArgs a{};
    a.w = st->w; a.u = st->u; a.v = st->v; a.wb = st->wb; a.ub = st->ub; a.vb = st->vb;
    a.pbx = st->pbx; a.pby = st->pby; a.qb1x = st->qb1x; a.qb1y = st->qb1y; a.qb2x = st->qb2x; a.qb2y = st->qb2y;
    a.bw = work0; a.bu = work1; a.bv = work2; a.s_out = s_out;
    a.Ix = Ix; a.Iy = Iy; a.It = It; a.H = H; a.W = W; a.ld = ld;
    a.sigma = (float)p->sigma; a.tau = (float)p->tau; a.stt = (float)(p->sigma * p->tau);
    a.lam = (float)p->lambda; a.beta = (float)p->beta;
    enqueue_pdr_iter(a, p->gs_sweeps, hw, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return FLOW_OK;
}

}  // extern "C"

// K iterations of the pDR or ALG1 tile kernel (per pp.scheme) from `in` to `out` for the operator entries.
static flow_status op_pd_tb(const flow_pdr_state* in, const flow_pdr_state* out, float* s_out, const float* Ix,
                            const float* Iy, const float* It, const float* u0, const float* v0, int32_t H, int32_t W,
                            int64_t ld, const flow_params* p, int32_t iters, int32_t tile_h, int32_t tile_w,
                            void* stream) {
    flow_status v = validate(p);
    if (v != FLOW_OK) return v;
    if (!in || !out || !s_out || !Ix || !Iy || !It || !u0 || !v0) return fail(FLOW_E_INVAL, "NULL pointer");
    if (H < 2 || W < 2 || ld < W) return fail(FLOW_E_INVAL, "bad shape");
    if (iters < 1 || tile_h < 1 || tile_w < 1) return fail(FLOW_E_INVAL, "iters, tile_h, tile_w must be >= 1");
    const bool hw = p->beta > 0;
    const int64_t halo = pd_halo(*p, iters);
    const int64_t region = std::min<int64_t>(H, tile_h + halo) * std::min<int64_t>(W, tile_w + halo);
    // regions above the 1024-thread kernel's capacity run the large pDR tiles (beta = 0); with the
    // pdr_mode knob at 12 / 13 / 14 / 15, pDR runs the wave-row tiles of 128 x 32 / 128 x 48 / 64 x 48
    // / 64 x 32 cells, and at 14 / 15 ALG1 its wave-row tiles of 64 x 48 / 64 x 32 cells
    const bool large = p->scheme == FLOW_PDR && !hw && region > pdr_tb_capacity(hw, 1024);
    int nt = large ? 2048 : 1024;
    if (p->scheme == FLOW_PDR && (g_pdr_mode == 12 || g_pdr_mode == 13)) nt = g_pdr_mode == 13 && !hw ? 6145 : 4098;
    if (g_pdr_mode == 14 || g_pdr_mode == 15) nt = g_pdr_mode == 14 && !hw ? 3074 : 2050;   // pDR and ALG1
    if (!pd_fits(hw, nt, std::min<int64_t>(H, tile_h + halo), std::min<int64_t>(W, tile_w + halo)))
        return fail(FLOW_E_INVAL, "tile plus halo exceeds the tile kernel's capacity");
    const float* ins[12] = {in->w, in->u, in->v, in->wb, in->ub, in->vb, in->pbx, in->pby,
                            in->qb1x, in->qb1y, in->qb2x, in->qb2y};
    const float* outs[12] = {out->w, out->u, out->v, out->wb, out->ub, out->vb, out->pbx, out->pby,
                             out->qb1x, out->qb1y, out->qb2x, out->qb2y};
    for (int k = 0; k < 12; ++k) {
        const bool wk = k == 0 || k == 3 || k == 6 || k == 7;
        if (wk && !hw) continue;
        if (!ins[k] || !outs[k] || ins[k] == outs[k]) return fail(FLOW_E_INVAL, "bad pDR state plane");
        EXTENT(ins[k], H, W, ld, "pDR state in");
        EXTENT(outs[k], H, W, ld, "pDR state out");
    }
    EXTENT(Ix, H, W, ld, "Ix"); EXTENT(Iy, H, W, ld, "Iy"); EXTENT(It, H, W, ld, "It");
    EXTENT(u0, H, W, ld, "u0"); EXTENT(v0, H, W, ld, "v0"); EXTENT(s_out, H, W, ld, "s_out");
    LevelPlanes L{};
    L.H = H; L.W = W; L.ld = ld;
    for (int c = 0; c < 3; ++c) {
        L.Xs[0][c] = const_cast<float*>(ins[c]);
        L.Xbs[0][c] = const_cast<float*>(ins[3 + c]);
        L.Xs[1][c] = const_cast<float*>(outs[c]);
        L.Xbs[1][c] = const_cast<float*>(outs[3 + c]);
    }
    for (int c = 0; c < 6; ++c) {
        L.ybs[0][c] = const_cast<float*>(ins[6 + c]);
        L.ybs[1][c] = const_cast<float*>(outs[6 + c]);
    }
    L.Ix = const_cast<float*>(Ix); L.Iy = const_cast<float*>(Iy); L.It = const_cast<float*>(It);
    L.U0[0] = const_cast<float*>(u0); L.U0[1] = const_cast<float*>(v0);
    L.s_out = s_out;
    PdrTbPlan T;
    T.tb = true;
    T.K = iters;
    T.th = tile_h;
    T.tw = tile_w;
    hipStream_t s = (hipStream_t)stream;
    // reads set 0 (in), writes set 1 (out)
    if (p->scheme == FLOW_ALG1) launch_alg1_tb(pdr_tb_args(L, *p, T, 0, iters), hw, nt, s);
    else launch_pdr_tb(pdr_tb_args(L, *p, T, 0, iters), hw, nt, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return FLOW_OK;
}

extern "C" {

flow_status flow_op_pdr_tb(const flow_pdr_state* in, const flow_pdr_state* out, float* s_out, const float* Ix,
                           const float* Iy, const float* It, const float* u0, const float* v0, int32_t H, int32_t W,
                           int64_t ld, const flow_params* p, int32_t iters, int32_t tile_h, int32_t tile_w,
                           void* stream) {
    if (!p) return fail(FLOW_E_INVAL, "params is NULL");
    flow_params q = *p;
    q.scheme = FLOW_PDR;
    return op_pd_tb(in, out, s_out, Ix, Iy, It, u0, v0, H, W, ld, &q, iters, tile_h, tile_w, stream);
}

flow_status flow_op_alg1_tb(const flow_pdr_state* in, const flow_pdr_state* out, float* s_out, const float* Ix,
                            const float* Iy, const float* It, const float* u0, const float* v0, int32_t H, int32_t W,
                            int64_t ld, const flow_params* p, int32_t iters, int32_t tile_h, int32_t tile_w,
                            void* stream) {
    if (!p) return fail(FLOW_E_INVAL, "params is NULL");
    flow_params q = *p;
    q.scheme = FLOW_ALG1;
    return op_pd_tb(in, out, s_out, Ix, Iy, It, u0, v0, H, W, ld, &q, iters, tile_h, tile_w, stream);
}

flow_status flow_op_energy(const flow_admm_state* st, const float* Ix, const float* Iy, const float* It,
                           int32_t H, int32_t W, int64_t ld, double lambda, double beta, flow_result* res,
                           void* stream) {
    if (!st || !Ix || !Iy || !It || !res) return fail(FLOW_E_INVAL, "NULL pointer");
    if (!st->u || !st->v || !st->q1x || !st->q1y || !st->q2x || !st->q2y || !st->s)
        return fail(FLOW_E_INVAL, "NULL state plane");
    if (beta > 0 && (!st->w || !st->px || !st->py)) return fail(FLOW_E_INVAL, "NULL w-block plane");
    if (H < 2 || W < 2 || ld < W) return fail(FLOW_E_INVAL, "bad shape");
    {
        const float* planes[] = {st->u, st->v, st->q1x, st->q1y, st->q2x, st->q2y, st->s, Ix, Iy, It};
        for (const float* q : planes) EXTENT(q, H, W, ld, "energy plane");
        if (beta > 0) {
            const float* wp[] = {st->w, st->px, st->py};
            for (const float* q : wp) EXTENT(q, H, W, ld, "energy w-block plane");
        }
    }
    OpScratch& os = op_scratch();
    flow_status s2 = os.ensure();
    if (s2 != FLOW_OK) return s2;
    EnergyArgs e{};
    e.w = st->w; e.u = st->u; e.v = st->v; e.px = st->px; e.py = st->py;
    e.q1x = st->q1x; e.q1y = st->q1y; e.q2x = st->q2x; e.q2y = st->q2y; e.s = st->s;
    e.Ix = Ix; e.Iy = Iy; e.It = It; e.H = H; e.W = W; e.ld = ld;
    e.lam = (float)lambda; e.beta = (float)beta; e.pdr_tau = 0.f;
    e.partial = os.e_partial; e.out = os.e_out;
    hipStream_t s = (hipStream_t)stream;
    launch_energy(e, s);
    HIP_TRY(hipGetLastError());
    double h[kEnergyTerms];
    HIP_TRY(hipMemcpyAsync(h, os.e_out, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    fill_result(h, res);
    return FLOW_OK;
}

}  // extern "C"
