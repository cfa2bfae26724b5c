// Autotuner: for every level shape of a pair, time each iteration-kernel choice (one-pass kernel
// with strip heights 2 / 4 / 8; K-iteration tiles of 256, 1024 and small 1024-thread work-groups
// with every K up to 16 that is the smallest for its number of launches per warp; a resident tile
// where the level fits) over one warp's worth of iterations with HIP events, and keep the fastest.  Every choice computes the same iteration, so the choice
// changes speed only (results agree to rounding); later solves of the context use the table.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <sstream>

#include "runtime.hpp"

namespace flowmi {

#define HIP_TRY(expr)                                           \
    do {                                                        \
        hipError_t _e = (expr);                                 \
        if (_e != hipSuccess) return hip_fail(_e, #expr);       \
    } while (0)

// The level's state starts at zero and its linearisation (I_x, I_y, I_t and the point u0, v0) is
// deterministic noise at the scale of image gradients and flows.  Timed on zeros, where no operand
// changes, the ranking of launch shapes differed from the one in solves of images (at 1920 x 1080,
// level 0, a choice 0.3% faster on zeros was 10% slower in the solve); on noise the two agree.
std::vector<int> launch_ks(int iters, int kmin, int kmax) {
    std::vector<int> ks;
    for (int n = iters; n >= 1; --n) {
        const int K = (iters + n - 1) / n;
        if (K >= kmin && K <= kmax && (ks.empty() || ks.back() != K)) ks.push_back(K);
    }
    if (ks.empty()) ks.push_back(kmin);
    return ks;
}

static flow_status prepare_level(const LevelPlanes& L, hipStream_t s) {
    const size_t plane = (size_t)L.H * L.ld * sizeof(float);
    for (int b = 0; b < 2; ++b) {
        for (int k = 0; k < 10; ++k)
            if (L.st[b][k]) HIP_TRY(hipMemsetAsync(L.st[b][k], 0, plane, s));
        for (int k = 0; k < 3; ++k) {
            if (L.Xs[b][k]) HIP_TRY(hipMemsetAsync(L.Xs[b][k], 0, plane, s));
            if (L.Xbs[b][k]) HIP_TRY(hipMemsetAsync(L.Xbs[b][k], 0, plane, s));
        }
        for (int k = 0; k < 6; ++k)
            if (L.ybs[b][k]) HIP_TRY(hipMemsetAsync(L.ybs[b][k], 0, plane, s));
    }
    if (L.s_out) HIP_TRY(hipMemsetAsync(L.s_out, 0, plane, s));
    for (float* q : L.b)
        if (q) HIP_TRY(hipMemsetAsync(q, 0, plane, s));
    float* lin[5] = {L.Ix, L.Iy, L.It, L.U0[0], L.U0[1]};
    const float scale[5] = {0.1f, 0.1f, 0.05f, 2.f, 2.f};
    for (int k = 0; k < 5; ++k) launch_fill_noise(lin[k], L.H, L.W, L.ld, 0x51u + 977u * k, scale[k], s);
    HIP_TRY(hipGetLastError());
    return FLOW_OK;
}

}  // namespace flowmi

using namespace flowmi;

extern "C" flow_status flow_autotune(flow_ctx* ctx, int32_t H, int32_t W, const flow_params* p, void* stream) {
    if (!ctx) return fail(FLOW_E_INVAL, "ctx is NULL");
    flow_status st = validate(p);
    if (st != FLOW_OK) return st;
    st = validate_shape(H, W, W, p->levels);
    if (st != FLOW_OK) return st;
    if (p->iters < 1) return FLOW_OK;     // nothing to choose
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    st = ctx->ensure_arena(layout_bytes(H, W, *p));
    if (st != FLOW_OK) return st;
    std::vector<LevelPlanes> Ls;
    st = build_layout(ctx->arena, H, W, *p, Ls);
    if (st != FLOW_OK) return st;
    const bool hw = p->beta > 0;
    const float ones[2] = {1.f, 1.f};
    HIP_TRY(hipMemcpyAsync(ctx->scratch.at, ones, sizeof(ones), hipMemcpyHostToDevice, s));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    std::ostringstream rep;
    rep << "{";
    bool first_level = true;
    for (const LevelPlanes& L : Ls) {
        st = prepare_level(L, s);
        if (st != FLOW_OK) break;
        if (pd_state(*p)) {
            // pDR: the three-pass iteration, or tiles with K = 1, 2, 3, 4, or a resident level;
            // ALG1: tiles with the launch-count K values up to 10, or a resident level
            const bool alg1 = p->scheme == FLOW_ALG1;
            struct PCand { TunedChoice c; PdrTbPlan T; };
            std::vector<PCand> cands;
            if (!alg1) {
                PCand three{};
                three.c.mode = 1;
                cands.push_back(three);
            }
            bool resident_done = false;
            const std::vector<int> ks = alg1 ? launch_ks(p->iters, 1, 10) : std::vector<int>{1, 2, 3, 4};
            for (int nt : {1024, 512, 2048, 513, 4098, 6145, 3074, 2050})
            for (int K : ks) {
                if ((nt == 2048 || nt == 513 || nt == 6145) && (alg1 || hw)) continue;   // pDR, no w
                if (nt == 3074 && hw) continue;                                          // no w
                if (nt == 4098 && alg1) continue;                                        // pDR
                PdrTbPlan T = plan_pd_tiles(L.H, L.W, hw, pd_halo(*p, K), K, 0, nt);
                if (!T.tb) continue;
                if (T.resident) {
                    if (resident_done) continue;
                    resident_done = true;
                    T.K = p->iters;
                }
                PCand c{};
                c.c.mode = nt == 512 ? 6 : nt == 2048 ? 10 : nt == 513 ? 11 : nt == 4098 ? 12 : nt == 6145 ? 13
                         : nt == 3074 ? 14 : nt == 2050 ? 15 : 5;
                c.c.K = T.resident ? 0 : K;
                c.T = T;
                cands.push_back(c);
            }
            double best = 1e30;
            TunedChoice bestc;
            std::ostringstream lv;
            for (PCand& c : cands) {
                float ms_best = 1e30f;
                for (int rep_i = 0; rep_i < 4; ++rep_i) {      // the first run is a warm-up
                    HIP_TRY(hipEventRecord(e0, s));
                    if (c.c.mode == 1) {
                        for (int t = 0; t < p->iters; ++t) enqueue_pdr_iter(pdr_args(L, *p, 0), p->gs_sweeps, hw, s);
                    } else {
                        enqueue_pdr_tiles(L, *p, c.T, 0, p->iters, s, nullptr);
                    }
                    HIP_TRY(hipEventRecord(e1, s));
                    HIP_TRY(hipEventSynchronize(e1));
                    float ms = 0.f;
                    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                    if (rep_i > 0) ms_best = std::min(ms_best, ms);
                }
                HIP_TRY(hipGetLastError());
                c.c.us_per_iter = 1e3 * ms_best / p->iters;
                lv << (lv.tellp() > 0 ? ", " : "") << "\"m" << c.c.mode << "k" << c.c.K << "\": " << c.c.us_per_iter;
                if (c.c.us_per_iter < best) {
                    best = c.c.us_per_iter;
                    bestc = c.c;
                }
            }
            const std::string key = pd_tune_key(L.H, L.W, *p);
            ctx->tuned[key] = bestc;
            rep << (first_level ? "" : ", ") << "\"" << key << "\": {\"choice\": {\"mode\": " << bestc.mode
                << ", \"K\": " << bestc.K << ", \"rows\": 0, \"us_per_iter\": " << bestc.us_per_iter
                << "}, \"candidates\": {" << lv.str() << "}}";
            first_level = false;
            continue;
        }
        struct Cand { TunedChoice c; LevelTbPlan P; bool tb; };
        std::vector<Cand> cands;
        for (int rows : {0, 2, 4, 8}) {
            Cand c{};
            c.c.mode = 1;
            c.c.rows = rows;
            c.tb = false;
            cands.push_back(c);
        }
        // iterations per launch: every launch pays a fixed cost (loads, stores, dispatch), so each
        // launch count matters (50 iterations: 7 launches at K = 8, 6 at K = 9, 5 at K = 10)
        const std::vector<int> ks = launch_ks(p->iters, 2, 16);
        for (int mode : {2, 4, 3, 7, 6, 8, 9, 12, 13, 14})
            for (int K : ks)
                for (int ew : {0, 32, 48, 64, 96}) {             // extended tile width (0: built-in)
                    LevelTbPlan P = plan_level(L.H, L.W, hw, p->iters, mode, K, ew);
                    if (!P.tb) continue;
                    if (P.resident && (K != ks.front() || ew != 0)) continue;   // one resident candidate per size
                    if (!P.resident && P.K != K) continue;              // capacity lowered K: a duplicate
                    bool dup = false;                                   // the same tiling under another width
                    for (const Cand& o : cands)
                        dup = dup || (o.tb && o.c.mode == mode && o.P.K == P.K && o.P.th == P.th && o.P.tw == P.tw);
                    if (dup) continue;
                    std::vector<TbTile> tiles;
                    append_tiles(P, 0, L.H, L.W, tiles);
                    P.ntiles = (int)tiles.size();
                    Cand c{};
                    c.c.mode = mode;
                    c.c.K = P.resident ? 0 : K;
                    c.c.rows = P.resident ? 0 : ew;
                    c.P = P;
                    c.tb = true;
                    cands.push_back(c);
                }
        double best = 1e30;
        TunedChoice bestc;
        std::ostringstream lv;
        for (Cand& c : cands) {
            const LevelTbPlan* P = c.tb ? &c.P : nullptr;
            enqueue_admm_iters(L, *p, P, c.c.rows, 0, p->iters, 0, ctx->scratch.at, s);    // warm-up
            float ms_best = 1e30f;
            for (int rep_i = 0; rep_i < 3; ++rep_i) {
                HIP_TRY(hipEventRecord(e0, s));
                enqueue_admm_iters(L, *p, P, c.c.rows, 0, p->iters, 0, ctx->scratch.at, s);
                HIP_TRY(hipEventRecord(e1, s));
                HIP_TRY(hipEventSynchronize(e1));
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                ms_best = std::min(ms_best, ms);
            }
            HIP_TRY(hipGetLastError());
            c.c.us_per_iter = 1e3 * ms_best / p->iters;
            lv << (lv.tellp() > 0 ? ", " : "") << "\"m" << c.c.mode << "k" << c.c.K << "r" << c.c.rows
               << "\": " << c.c.us_per_iter;
            if (c.c.us_per_iter < best) {
                best = c.c.us_per_iter;
                bestc = c.c;
            }
        }
        ctx->tuned[tune_key(L.H, L.W, hw, p->iters)] = bestc;
        rep << (first_level ? "" : ", ") << "\"" << tune_key(L.H, L.W, hw, p->iters) << "\": {\"choice\": {\"mode\": "
            << bestc.mode << ", \"K\": " << bestc.K << ", \"rows\": " << bestc.rows << ", \"us_per_iter\": "
            << bestc.us_per_iter << "}, \"candidates\": {" << lv.str() << "}}";
        first_level = false;
    }
    rep << "}";
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st != FLOW_OK) return st;
    ctx->tune_report = rep.str();
    ctx->tune_epoch++;
    ctx->drop_graphs();
    return FLOW_OK;
}

extern "C" flow_status flow_get_tuning(const flow_ctx* ctx, char* buf, size_t cap) {
    if (!ctx || !buf || cap == 0) return fail(FLOW_E_INVAL, "NULL argument");
    const std::string& r = ctx->tune_report;
    if (r.size() + 1 > cap) return fail(FLOW_E_INVAL, "buffer too small for the tuning report");
    std::memcpy(buf, r.c_str(), r.size() + 1);
    return FLOW_OK;
}

extern "C" flow_status flow_tune_choice(flow_ctx* ctx, int32_t H, int32_t W, int32_t has_w, int32_t iters,
                                        int32_t pdr_sweeps, int32_t mode, int32_t K, int32_t rows) {
    if (!ctx) return fail(FLOW_E_INVAL, "ctx is NULL");
    if (H < 2 || W < 2 || iters < 1) return fail(FLOW_E_INVAL, "H, W must be >= 2 and iters >= 1");
    if (mode < 1 || mode > 15)
        return fail(FLOW_E_INVAL, "mode must be 1 (one-pass / three-pass), 2..4, 6..9, 12..14 (tiles) or 5 / 10 / 11 "
                                  "(pDR tiles)");
    if (K < 0 || K > 64) return fail(FLOW_E_INVAL, "K must be in [0, 64] (0 = resident or built-in)");
    if (mode == 1 && rows != 0 && rows != 2 && rows != 4 && rows != 8)
        return fail(FLOW_E_INVAL, "rows (one-pass strip height) must be 0, 2, 4 or 8");
    if (mode != 1 && rows != 0 && (rows < 16 || rows > 512))
        return fail(FLOW_E_INVAL, "rows (tile modes: extended tile width) must be 0 or in [16, 512]");
    if (pdr_sweeps < -1) return fail(FLOW_E_INVAL, "pdr_sweeps must be >= -1 (-1: ALG1)");
    if (pdr_sweeps == -1 && mode != 5 && mode != 6 && mode != 14 && mode != 15)
        return fail(FLOW_E_INVAL, "ALG1 modes: 5 / 6 (tiles of 1024 / 512 threads), 14 / 15 (wave-row tiles of 64 x 48 "
                                  "/ 64 x 32 cells)");
    if (pdr_sweeps == -1 && mode == 14 && has_w) return fail(FLOW_E_INVAL, "ALG1 mode 14 needs beta = 0");
    if (pdr_sweeps > 0 && mode != 1 && mode != 5 && mode != 6 && mode < 10)
        return fail(FLOW_E_INVAL, "pDR modes: 1 (three-pass), 5 / 6 (tiles of 1024 / 512 threads), 10 / 11 (the same "
                                  "with two cells of each colour per thread), 12 / 13 (wave-row tiles of 128 x 32 / "
                                  "128 x 48 cells), 14 / 15 (wave-row tiles of 64 x 48 / 64 x 32 cells)");
    if (pdr_sweeps > 0 && (mode == 10 || mode == 11 || mode == 13 || mode == 14) && has_w)
        return fail(FLOW_E_INVAL, "pDR modes 10, 11, 13 and 14 need beta = 0");
    if (pdr_sweeps == 0 && (mode == 5 || mode == 10 || mode == 11 || mode == 15))
        return fail(FLOW_E_INVAL, "modes 5, 10, 11 and 15 are pDR modes");
    if (pdr_sweeps != 0 && mode > 6 && mode < 10) return fail(FLOW_E_INVAL, "modes 7, 8 and 9 are ADMM modes");
    TunedChoice c;
    c.mode = mode;
    c.K = K;
    c.rows = rows;
    std::string key = tune_key(H, W, has_w != 0, iters);
    if (pdr_sweeps > 0) key += "p" + std::to_string(pdr_sweeps);
    if (pdr_sweeps < 0) key += "a";
    ctx->tuned[key] = c;
    ctx->tune_epoch++;
    ctx->drop_graphs();
    return FLOW_OK;
}
