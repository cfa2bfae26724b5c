// Host-side launch geometry of the kernels: tile capacities, block counts and the one-pass
// kernel's strip shape.  Pure arithmetic on sizes, shared by the launchers, the planners and the
// tables (and built by the CPU test of the host logic without any device code).
#include "kernels.hpp"

namespace flowmi {

int g_admm_rows_override = 0;

AdmmGeometry admm_geometry(int H, int W, int rows_hint) {
    AdmmGeometry g;
    g.strips = (W + kStrip - 1) / kStrip;
    auto waves = [&](int r) { return (long long)g.strips * ((H + r - 1) / r); };
    // Tall strips amortise the 3-row halo; short ones give more wavefronts to hide latency.
    int rows = 2;
    if (waves(8) >= 4096) rows = 8;
    else if (waves(4) >= 1024) rows = 4;
    if (g_admm_rows_override == 2 || g_admm_rows_override == 4 || g_admm_rows_override == 8)
        rows = g_admm_rows_override;
    else if (rows_hint == 2 || rows_hint == 4 || rows_hint == 8)
        rows = rows_hint;
    g.rows = rows;
    g.segs = (H + g.rows - 1) / g.rows;
    long long blocks = (waves(rows) + 3) / 4;
    blocks = (blocks + 7) / 8 * 8;
    g.blocks = (int)blocks;
    return g;
}

bool is_rows_code(int nt) { return nt == 2049 || nt == 3073 || nt == 4097; }

int tb_capacity(bool has_w, int nt) {
    if (is_rows_code(nt)) return nt - 1;          // 64 columns x 32, 48 or 64 rows
    if (nt == 1024) return 1024 * (has_w ? kTbPptLW : kTbPptL);
    if (nt == 1025) return 1024 * kTbPptSmall;   // 1024 threads, small tiles
    if (nt == 513) return 512 * kTbPptSmall;     // 512 threads, small tiles
    if (nt == 257) return 256 * kTbPptSmall;     // 256 threads, small tiles
    if (nt == 1026) return 1024;                  // 1024 threads, one pixel each
    if (nt == 514) return 512;                    // 512 threads, one pixel each
    return 256 * (has_w ? kTbPptW : kTbPpt);
}

bool tb_fits(bool has_w, int nt, int64_t eh, int64_t ew) {
    if (is_rows_code(nt)) return ew <= kWave && eh * kWave <= nt - 1;
    return eh * ew <= tb_capacity(has_w, nt);
}

// pDR / ALG1 tiles: work-group codes 512 / 1024 (one red and one black cell per thread), 2048 (1024
// threads with two cells of each colour), 513 (512 threads with two of each), and the pDR wave-row
// codes (1024 threads): 4098 / 6145 with a cell pair per lane (regions of at most 128 columns and
// 32 / 48 rows) and 2050 / 3074 with one cell per lane (at most 64 columns and 32 / 48 rows)
bool is_pd_rows_code(int nt) { return nt == 4098 || nt == 6145 || nt == 2050 || nt == 3074; }
int pd_rows_width(int nt) { return (nt == 2050 || nt == 3074) ? kWave : 2 * kWave; }

int pdr_tb_capacity(bool, int nt) {
    if (is_pd_rows_code(nt)) return nt - (nt & 3);   // 4096, 6144, 2048, 3072
    return nt == 513 ? 2048 : 2 * nt;
}

bool pd_fits(bool has_w, int nt, int64_t eh, int64_t ew) {
    if (is_pd_rows_code(nt)) return ew <= pd_rows_width(nt) && eh * pd_rows_width(nt) <= pdr_tb_capacity(has_w, nt);
    return eh * ew <= pdr_tb_capacity(has_w, nt);
}

int blocks_of(int H, int W) { return ((W + 63) / 64) * ((H + 3) / 4); }
int lin_blocks_of(int H, int W) { return ((W + 63) / 64) * ((H + kLinRows - 1) / kLinRows); }

int energy_blocks(int H, int W) {
    const int64_t npix = (int64_t)H * W;
    int blocks = (int)((npix + 255) / 256);
    if (blocks > kEnergyBlocks) blocks = kEnergyBlocks;
    if (blocks < 1) blocks = 1;
    return blocks;
}

}  // namespace flowmi
