// Argument blocks and launchers of the ADMM iteration kernels (fused one-pass and K-iteration
// tiles).  Planes are row-major FP32 with a pitch `ld` in elements.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace flowmi {

constexpr int kWave = 64;
constexpr int kStrip = kWave - 3;   // output columns per wavefront in the streaming iteration kernels

// One iteration of the ADMM family (rpADMMI / rpADMMII), fused into one pass.
struct AdmmIterArgs {
    const float *w, *u, *v, *px, *py, *q1x, *q1y, *q2x, *q2y, *s;   // iterate k
    float *wo, *uo, *vo, *pxo, *pyo, *q1xo, *q1yo, *q2xo, *q2yo, *so; // iterate k + 1
    const float *Ix, *Iy, *It;
    const float *u0, *v0;   // linearisation point (increment form: u, v hold u - u0, It is relative)
    const float* at;        // device scalar a~
    int H, W;
    int64_t ld;
    float c, lam, beta;
    float inv_ac;           // 1 / (a c), a = 8
    float c_rho_s;          // c * rho_s (rho_s = 1 for rpADMMI, rho for rpADMMII)
    float cA, cB, cC;       // Lambda+ = Lambda + cA div y+ - A (cB s+ - cC s)
    int rows;               // output rows per wavefront (caller: 0 = built-in choice, or 2 / 4 / 8)
    int strips, segs;       // wavefront grid: strips along x, segments along y
};

struct AdmmGeometry { int rows, strips, segs, blocks; };
AdmmGeometry admm_geometry(int H, int W, int rows_hint);
extern int g_admm_rows_override;   // 0 = heuristic; 2, 4 or 8 force the strip height
void launch_admm_iter(const AdmmIterArgs& a, bool has_w, hipStream_t s);

// Temporally blocked iterations: K iterations of one output tile per work-group launch.
constexpr int kTbPpt = 6;            // pixels per thread, 256 threads (beta = 0): LDS q1x..q2y, gu, gv
constexpr int kTbPptW = 4;           // with the w / p block
constexpr int kTbPptL = 4;           // 1024 threads (at most 128 VGPRs per thread)
constexpr int kTbPptLW = 3;
constexpr int kTbPptSmall = 2;       // 1024 threads on small tiles (work-group size code 1025)
// Work-group size codes 1026 / 514: 1024 / 512 threads with one pixel each, for latency-bound levels
// (twice the wavefronts of codes 513 / 257 on the same extended region).
// Halo of a K-iteration tile: per iteration the dual field q reaches one cell further in every
// direction and the multipliers follow q's divergence (left / above) at the end of the iteration,
// so after K iterations the iterate of an output pixel depends on the launch's input within K + 1
// rows / columns above and to the left and K below and to the right.
constexpr int tb_halo_lo(int K) { return K + 1; }
constexpr int tb_halo_hi(int K) { return K; }
struct TbTile {
    int level;                       // index of the (pair, level) descriptor
    int y0, x0, th, tw;              // output tile
};
struct TbLevel {
    const float* in[10];             // iterate k: w, du, dv, px, py, q1x, q1y, q2x, q2y, s
    float* out[10];                  // iterate k + K
    const float *Ix, *Iy, *It, *u0, *v0;
    const float* at;                 // the pair's two a~ slots
    int H, W;
    int64_t ld;
};
struct TbArgs {
    const TbTile* tiles;
    int ntiles;
    const int* ntiles_dev;           // table / queue order: if set, the tile count is read from device
                                     // memory (a launch replayed from a graph over tables that change)
    const TbLevel* levels;           // two descriptors per (pair, level): [2 * id + dir]
    int dir;                         // which ping-pong direction this launch uses
    int K;                           // iterations of this launch (halo K + 1 top/left, K bottom/right)
    int at_slot;                     // a~ slot of the current warp
    unsigned* queue;                 // work counters (nullptr: tiles from the work-group index)
    unsigned queue_base;             // counter value at the start of this launch
    int nq;                          // sub-queues: work-group b drains tiles [ntiles*x/nq, ntiles*(x+1)/nq)
                                     // of sub-queue x = b % nq with counter queue[x] (nq <= grid)
    float c, lam, beta, inv_ac, c_rho_s, cA, cB, cC;
    // tiles == nullptr: direct mode (one level, regular tiles): descriptor of this launch's
    // direction and tiling; tiles != nullptr and queue == nullptr: tile k of the table per work-group
    TbLevel lvl;
    int th, tw, ntx;
};
// nt: 256, 1024, or the small-tile codes 1025 / 513 / 257 (1024 / 512 / 256 threads, 2 pixels each;
// 513 and 257 only with direct tiling), or the wave-row codes 2049 / 3073 / 4097 (1024 threads; an
// extended region of at most 64 columns and 32 / 48 / 64 rows, held in registers one wavefront-wide
// row per thread and row; direct or table order)
int tb_capacity(bool has_w, int nt);
bool is_rows_code(int nt);
// an extended region of eh x ew pixels fits the tile kernel of work-group code nt
bool tb_fits(bool has_w, int nt, int64_t eh, int64_t ew);
void launch_admm_tb(const TbArgs& a, bool has_w, int nt, int grid, hipStream_t s);
void launch_admm_rows(const TbArgs& a, bool has_w, int nt, int grid, hipStream_t s);
void launch_reset_u32(unsigned* p, int n, hipStream_t s);

}  // namespace flowmi
