// Shared pieces of the multi-pair paths (batched solves and serving); see multi.hpp.
#include "multi.hpp"

namespace flowmi {

flow_status DevBuf::ensure(size_t need, const char* what) {
    if (need <= bytes) return FLOW_OK;
    if (d) {
        hipDeviceSynchronize();
        hipFree(d);
        d = nullptr;
        bytes = 0;
    }
    hipError_t e = hipMalloc((void**)&d, need);
    if (e != hipSuccess) return fail(FLOW_E_NOMEM, std::string("hipMalloc(") + what + "): " + hipGetErrorString(e));
    bytes = need;
    return FLOW_OK;
}

void DevBuf::release() {
    if (d) hipFree(d);
    d = nullptr;
    bytes = 0;
}

flow_status PinnedBuf::ensure(size_t need) {
    if (need <= bytes) return FLOW_OK;
    if (h) {
        hipDeviceSynchronize();
        hipHostFree(h);
    }
    h = nullptr;
    bytes = 0;
    hipError_t e = hipHostMalloc((void**)&h, need, hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e, "hipHostMalloc");
    bytes = need;
    return FLOW_OK;
}

void PinnedBuf::release() {
    if (h) hipHostFree(h);
    h = nullptr;
    bytes = 0;
}

bool shapes_fit(const Shapes& s, bool hw, int K, int ew, int nt) {
    for (auto& x : s) {
        const LevelTbPlan T = plan_tiles(x.first, x.second, hw, nt, std::min(K, 64), ew);
        if (!T.tb) return false;
        if (!T.resident && T.K != K) return false;
    }
    return true;
}

bool shapes_all_resident(const Shapes& s, bool hw, int nt) {
    for (auto& x : s)
        if (!tb_fits(hw, nt, x.first, x.second)) return false;
    return true;
}

StageChoice fit_stage_choice(StageChoice c, const Shapes& s, bool hw) {
    if (c.K < 1) c.K = 1;
    if (is_rows_code(c.tnt)) {
        c.order = ORDER_TABLE;
        if (c.ew > kWave) c.ew = kWave;
        if (!shapes_fit(s, hw, 1, c.ew, c.tnt)) c.tnt = kBatchNt;
    }
    while (c.K > 1 && !shapes_fit(s, hw, c.K, c.ew, c.tnt)) --c.K;
    if (!shapes_fit(s, hw, c.K, c.ew, c.tnt)) {
        c.ew = 64;
        while (c.K > 1 && !shapes_fit(s, hw, c.K, c.ew, c.tnt)) --c.K;
    }
    return c;
}

StageChoice default_stage_choice(const Shapes& s, bool hw, int iters) {
    StageChoice c;
    c.order = ORDER_TABLE;
    c.ew = 64;
    if (shapes_all_resident(s, hw, c.tnt)) {
        c.K = std::max(1, iters);
        return c;
    }
    int64_t px = 0;
    for (auto& x : s) px += (int64_t)x.first * x.second;
    c.tnt = px >= 1000000 ? 3073 : 2049;
    c.K = px >= 1000000 ? 9 : 8;
    return fit_stage_choice(c, s, hw);
}

void level_tiles(int H, int W, bool hw, const StageChoice& ch, int desc, std::vector<TbTile>& out) {
    const LevelTbPlan T = plan_tiles(H, W, hw, ch.tnt, std::min(ch.K, 64), ch.ew);
    append_tiles(T, desc, H, W, out);
}

int tile_grid(const StageChoice& ch, int ntiles) {
    if (ch.order == ORDER_QUEUE) return std::max(1, std::min(ntiles, 256 * 2));   // 2 work-groups of 1024 per CU
    return ntiles;
}

int enqueue_tile_warp(const TbTile* tiles, int ntiles, int grid, const TbLevel* descs, const StageChoice& ch,
                      const flow_params& p, int at_slot, int dir0, unsigned* counters, hipStream_t s,
                      const int* ntiles_dev) {
    const bool hw = p.beta > 0;
    AdmmIterArgs co{};
    fill_admm_coeffs(co, p);
    TbArgs a{};
    a.tiles = tiles;
    a.ntiles = ntiles;
    a.ntiles_dev = ntiles_dev;
    a.levels = descs;
    a.at_slot = at_slot;
    a.c = co.c; a.lam = co.lam; a.beta = co.beta; a.inv_ac = co.inv_ac; a.c_rho_s = co.c_rho_s;
    a.cA = co.cA; a.cB = co.cB; a.cC = co.cC;
    int dir = dir0, k = 0, li = 0;
    while (k < p.iters) {
        const int kk = std::min(ch.K, p.iters - k);
        a.dir = dir;
        a.K = kk;
        if (ch.order == ORDER_QUEUE) {
            a.queue = counters + li * kNq;
            a.queue_base = 0;
            a.nq = std::min(kNq, grid);
        } else {
            a.queue = nullptr;
            a.nq = 1;
        }
        if (ntiles > 0 || ntiles_dev) launch_admm_tb(a, hw, ch.tnt, grid, s);
        dir ^= 1;
        k += kk;
        ++li;
    }
    return dir;
}

bool pd_pair_tileable(int H, int W, int levels, const flow_params& p) {
    for (auto& x : level_shapes(H, W, levels))
        if (!plan_pd_tiles(x.first, x.second, p.beta > 0, pd_halo(p, 1), 1, 0, 1024).tb) return false;
    return true;
}

int pd_shared_k(const Shapes& s, const flow_params& p) {
    const bool hw = p.beta > 0;
    bool resident = true;
    for (auto& x : s) resident = resident && (int64_t)x.first * x.second <= pdr_tb_capacity(hw, 1024);
    if (resident) return std::max(1, p.iters);
    for (int K = p.scheme == FLOW_ALG1 ? kAlg1DefaultK : kPdrDefaultK; K >= 1; --K) {
        bool fits = true;
        for (auto& x : s) fits = fits && plan_pd_tiles(x.first, x.second, hw, pd_halo(p, K), K, 0, 1024).tb;
        if (fits) return K;
    }
    return 0;
}

flow_status validate_pair(const flow_pair& q, const flow_params& p, const std::string& who) {
    if (q.levels < 0 || q.levels > FLOW_MAX_LEVELS) return fail(FLOW_E_INVAL, who + "levels out of range");
    const int lv = q.levels > 0 ? q.levels : p.levels;
    flow_status st = validate_shape(q.H, q.W, q.ld, lv);
    if (st != FLOW_OK) return fail(st, who + flow_last_error());
    if (q.ld_uv < q.W) return fail(FLOW_E_INVAL, who + "ld_uv smaller than W");
    if (!q.I0 || !q.I1 || !q.u || !q.v) return fail(FLOW_E_INVAL, who + "NULL device pointer");
    const struct { const void* ptr; int64_t ld; const char* name; } planes[4] = {
        {q.I0, q.ld, "I0"}, {q.I1, q.ld, "I1"}, {q.u, q.ld_uv, "u"}, {q.v, q.ld_uv, "v"}};
    for (auto& pl : planes) {
        st = check_extent(pl.ptr, q.H, q.W, pl.ld, sizeof(float), pl.name);
        if (st != FLOW_OK) return fail(st, who + flow_last_error());
    }
    return FLOW_OK;
}

}  // namespace flowmi
