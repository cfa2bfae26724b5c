// Planning of temporally blocked iterations: per level, whether the fused one-pass kernel or the
// K-iteration tile kernel runs, with which work-group size, K and output tile; and the device
// tables (tiles, level descriptors) the tile kernel reads.
#include <algorithm>
#include <cstring>

#include "runtime.hpp"

namespace flowmi {

int g_tb_mode = 0;   // 0 built-in, 1 one-pass only, 2 tiles of 256 threads, 3 of 1024, 4 / 7 / 6 small tiles
                     // of 1024 / 512 / 256 threads, 8 / 9 one-pixel tiles of 1024 / 512 threads, 12 / 13 / 14
                     // wave-row tiles of 32 / 48 / 64 rows
int g_tb_k = 0;      // iterations per launch of tiled levels (0 = default)

constexpr int kDefaultK = 4;

static bool fit_tile(int H, int W, bool hw, int nt, int K, int ew_target, int& th, int& tw) {
    // output tile th x tw whose extended region (halo K + 1 and K per axis, clipped to the image) fits
    const int halo = tb_halo_lo(K) + tb_halo_hi(K);
    const int cap = tb_capacity(hw, nt);
    const int ew = std::min(W, ew_target);
    tw = (ew >= W) ? W : ew - halo;
    const int ext_w = std::min(W, tw + halo);
    int eh = cap / ext_w;
    if (is_rows_code(nt)) eh = std::min(eh, cap / kWave);  // wave-row tiles: rows of one wavefront
    th = (eh >= H) ? H : eh - halo;
    // tiles at least 8 wide, or as wide as a level narrower than that (no side halo then)
    return (tw >= 8 || tw == W) && th >= 2 && tb_fits(hw, nt, std::min(H, th + halo), std::min(W, tw + halo));
}

LevelTbPlan plan_tiles(int H, int W, bool hw, int nt, int K, int ew_target) {
    LevelTbPlan P;
    P.nt = nt;
    if (tb_fits(hw, nt, H, W)) {                             // one tile covers the level, no halo
        P.tb = true;
        P.resident = true;
        P.K = K;
        P.th = H;
        P.tw = W;
        return P;
    }
    if (ew_target <= 0 || (is_rows_code(nt) && ew_target > kWave))
        ew_target = is_rows_code(nt) ? kWave
                  : nt == 1024 ? (hw ? 80 : 96)
                  : nt == 1025 ? 64
                  : (nt == 513 || nt == 257 || nt == 1026) ? 32
                  : nt == 514 ? 24
                  : (hw ? 32 : 48);
    int th = 0, tw = 0;
    while (K > 0 && !fit_tile(H, W, hw, nt, K, ew_target, th, tw)) --K;
    if (K < 1) return P;
    P.tb = true;
    P.K = K;
    P.th = th;
    P.tw = tw;
    return P;
}

// Work-groups of a tile shape that one CU holds at once, set by each kernel's registers (64 VGPRs
// or fewer allow 8 wavefronts per SIMD) and the 8-wavefront limit per SIMD.
static int tb_wgs_per_cu(int nt, bool hw) {
    switch (nt) {
    case 1025: return hw ? 1 : 2;    // 1024 threads, 64 / 81 VGPRs
    case 1026: return 2;             // 1024 threads, one pixel
    case 513: return hw ? 3 : 4;
    case 514: return 4;
    case 257: return hw ? 6 : 8;
    case 1024: return 1;             // 1024 threads, 3-4 pixels
    case 2049: return 2;             // wave-row tiles of 1024 threads: 46 / 54 VGPRs
    case 3073: return hw ? 1 : 2;    // 62 / 74
    case 4097: return 1;             // 78 / 94
    default: return 3;               // 256 threads, 4-6 pixels
    }
}

// A level whose full-height tiles fit in one round of work-groups (one per CU, else as many per CU as
// fit) gets tiles just short enough to fill that round: the launch takes as long as its busiest CU,
// so shorter tiles spread the same level over more CUs, or even it out, with less work each.
// Returns the balanced tile height.
static int balanced_height(int H, int W, int th, int tw, int wgs_per_cu) {
    constexpr int kCUs = 256;
    const int ntx = (W + tw - 1) / tw;
    const int n = ntx * ((H + th - 1) / th);
    for (const int per : {1, wgs_per_cu}) {
        const int slots = kCUs * per;
        if (n > slots) continue;
        const int rows = slots / ntx;                // tile rows that one round holds
        return rows >= 1 ? std::min(th, std::max(2, (H + rows - 1) / rows)) : th;
    }
    return th;
}

static void balance_tiles(LevelTbPlan& P, int H, int W, bool hw) {
    if (P.tb && !P.resident) P.th = balanced_height(H, W, P.th, P.tw, tb_wgs_per_cu(P.nt, hw));
}

LevelTbPlan plan_level(int H, int W, bool hw, int iters, int mode, int kreq, int ew) {
    LevelTbPlan P;
    if (mode == 1 || iters < 2) return P;                    // one-pass kernel
    if (mode == 0) {
        // built-in choice: a level that fits one 1024-thread tile stays resident for a whole warp
        // (one launch instead of `iters`); larger levels take wave-row tiles, 48 rows high and 8
        // iterations per launch from a million pixels on, else 32 rows and 10 iterations (more and
        // shorter tiles for a level that fills fewer CUs); the one-pass kernel where neither fits
        if ((int64_t)H * W <= tb_capacity(hw, 1024)) {
            P.tb = P.resident = true;
            P.nt = 1024;
            P.K = iters;
            P.th = H;
            P.tw = W;
            return P;
        }
        const bool big = (int64_t)H * W >= 1000000;
        P = plan_tiles(H, W, hw, big ? 3073 : 2049, big ? 8 : 10, 0);
        balance_tiles(P, H, W, hw);
        return P;
    }
    const int nt = mode == 3 ? 1024 : mode == 4 ? 1025 : mode == 6 ? 257 : mode == 7 ? 513
                 : mode == 8 ? 1026 : mode == 9 ? 514 : mode == 12 ? 2049 : mode == 13 ? 3073 : mode == 14 ? 4097
                 : 256;
    P = plan_tiles(H, W, hw, nt, kreq > 0 ? kreq : kDefaultK, ew);
    if (P.resident) P.K = iters;                             // the whole warp in one launch
    balance_tiles(P, H, W, hw);
    return P;
}

PdrTbPlan plan_pd_tiles(int H, int W, bool hw, int halo, int K, int ew_target, int nt) {
    // output tile th x tw whose extended region (`halo` = both sides of an axis at K iterations per
    // launch, clipped to the image) fits the kernel's capacity; the whole level if it fits
    PdrTbPlan P;
    P.nt = nt;
    const int cap = pdr_tb_capacity(hw, nt);
    const bool rows = is_pd_rows_code(nt);
    if (pd_fits(hw, nt, H, W)) {
        P.tb = P.resident = true;
        P.K = K;
        P.th = H;
        P.tw = W;
        return P;
    }
    // 32 x 32, 64 x 32 or 64 x 64 regions; the wave-row tiles 128 or 64 columns wide
    if (ew_target <= 0 || (rows && ew_target > pd_rows_width(nt))) ew_target = rows ? pd_rows_width(nt) : nt == 512 ? 32 : 64;
    const int ew = std::min(W, std::max(ew_target, halo + 8));
    const int tw = (ew >= W) ? W : ew - halo;
    const int ext_w = std::min(W, tw + halo);
    const int eh = rows ? std::min(cap / ext_w, cap / pd_rows_width(nt)) : cap / ext_w;
    const int th = (eh >= H) ? H : eh - halo;
    if ((tw < 8 && tw != W) || th < 2 || !pd_fits(hw, nt, std::min(H, th + halo), ext_w)) return P;
    P.tb = true;
    P.K = K;
    // pDR and ALG1 tiles (70 / 67 VGPRs, 80 / 82 with w; two cells of each colour per thread: 128;
    // wave-row tiles with a cell pair per lane: 104 / 128, with one cell per lane: 51 / 64): one
    // 1024-thread work-group per CU (two of the one-cell wave-row tiles), two or three of 512 threads
    P.th = balanced_height(H, W, th, tw, nt == 512 ? (hw ? 2 : 3) : (nt == 513 || nt == 2050 || nt == 3074) ? 2 : 1);
    P.tw = tw;
    return P;
}

std::string tune_key(int H, int W, bool hw, int iters) {
    return std::to_string(H) + "x" + std::to_string(W) + (hw ? "w" : "") + "i" + std::to_string(iters);
}

LevelTbPlan plan_level_tuned(int H, int W, bool hw, int iters, const std::map<std::string, TunedChoice>* tuned) {
    if (g_tb_mode == 0 && tuned) {
        auto it = tuned->find(tune_key(H, W, hw, iters));
        if (it != tuned->end()) {
            // `rows`: the one-pass kernel's strip height, or the tiles' extended width target
            const TunedChoice& c = it->second;
            LevelTbPlan P = plan_level(H, W, hw, iters, c.mode, c.K, c.mode == 1 ? 0 : c.rows);
            P.rows = c.mode == 1 ? c.rows : 0;
            return P;
        }
    }
    return plan_level(H, W, hw, iters, g_tb_mode, g_tb_k);
}

void append_tiles(const LevelTbPlan& P, int level_id, int H, int W, std::vector<TbTile>& out) {
    if (!P.tb || P.th < 1 || P.tw < 1) return;      // no tile plan: no tiles (callers check the plan)
    for (int y = 0; y < H; y += P.th)
        for (int x = 0; x < W; x += P.tw) {
            TbTile t;
            t.level = level_id;
            t.y0 = y;
            t.x0 = x;
            t.th = std::min(P.th, H - y);
            t.tw = std::min(P.tw, W - x);
            out.push_back(t);
        }
}

void fill_tb_level(TbLevel* d, const LevelPlanes& L, const float* at2) {
    for (int dir = 0; dir < 2; ++dir) {
        TbLevel& x = d[dir];
        std::memset(&x, 0, sizeof(x));
        for (int k = 0; k < 10; ++k) {
            x.in[k] = L.st[dir][k];
            x.out[k] = L.st[dir ^ 1][k];
        }
        x.Ix = L.Ix;
        x.Iy = L.Iy;
        x.It = L.It;
        x.u0 = L.U0[0];
        x.v0 = L.U0[1];
        x.at = at2;
        x.H = L.H;
        x.W = L.W;
        x.ld = L.ld;
    }
}

int tb_grid(const LevelTbPlan& P, int ntiles) {
    const int per_cu = (P.nt == 1024 || P.nt == 4097) ? 1 : (P.nt == 1025 || P.nt == 1026 || P.nt == 2049 || P.nt == 3073) ? 2
                     : (P.nt == 513 || P.nt == 514) ? 4 : P.nt == 257 ? 8 : 4;   // residency
    return std::max(1, std::min(ntiles, 256 * per_cu));
}

flow_status TbTables::upload(const std::vector<TbTile>& tiles, const std::vector<TbLevel>& levels) {
    release();
    const size_t bt = sizeof(TbTile) * std::max<size_t>(1, tiles.size());
    const size_t bl = sizeof(TbLevel) * std::max<size_t>(1, levels.size());
    hipError_t e = hipMalloc(&d_tiles, bt);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(tiles)");
    e = hipMalloc(&d_levels, bl);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(levels)");
    if (!tiles.empty()) {
        e = hipMemcpy(d_tiles, tiles.data(), sizeof(TbTile) * tiles.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(tiles)");
    }
    if (!levels.empty()) {
        e = hipMemcpy(d_levels, levels.data(), sizeof(TbLevel) * levels.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(levels)");
    }
    bytes = bt + bl;
    return FLOW_OK;
}

void TbTables::release() {
    if (d_tiles) hipFree(d_tiles);
    if (d_levels) hipFree(d_levels);
    d_tiles = nullptr;
    d_levels = nullptr;
    bytes = 0;
}

}  // namespace flowmi
