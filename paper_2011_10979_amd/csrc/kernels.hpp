// Kernel argument blocks and host-side launchers shared by the HIP kernels and the C-ABI runtime.
// Planes are row-major FP32 (or FP16 for stored pyramids) with a pitch `ld` in elements.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <cstdint>

#include "admm_args.hpp"

namespace flowmi {

// Warp + linearise + a~ (max of M_s, one atomic max per work-group on the float bits).
struct LinArgs {
    const void *I0, *I1, *Dx, *Dy;   // float or __half, pitch ld
    const float *I0lo, *I1lo;        // optional low parts of float-float image levels (FP32 storage)
    float *u0, *v0;                  // pitch ld: the linearisation point (written when pend_u is set)
    const float *pend_u, *pend_v;    // optional pending increment of the previous warp: the point is
                                     // u0 + pend_u, committed into u0 here (in place, own pixel only)
    float *Ix, *Iy, *It;             // pitch ld
    float* at;                       // device scalar: max of M_s accumulated here (zero on entry)
    float* at_clear;                 // optional scalar cleared for the next warp (the other slot)
    int H, W;
    int64_t ld;
    float kappa, beta;
    int rel;                         // 1: It = kappa (I1w - I0), relative to the linearisation point
    float *zero_u, *zero_v;          // optional planes cleared at the same time (increment state)
    float *keep_u, *keep_v;          // optional planes receiving a copy of (u0, v0)
};
void launch_linearize(const LinArgs& a, bool f16, hipStream_t s);

// Argument blocks of the elementwise pyramid / bookkeeping kernels (also the items of batched launches).
// FP32 image levels below the finest are float-float (hi + lo planes, both pitch ld): a 2x2 mean
// needs two more significand bits per level than its inputs, and FP32 rounding of the coarse images
// moves ill-conditioned pixels of the final flow by up to a few 1e-4 px, while with hi + lo the
// levels are exact.  src_lo / dst_lo / I_lo are nullptr for the finest level and for FP16 storage.
struct DownArgs {
    const void* src; int H, W; int64_t ld; void* dst; int64_t ldd;   // output ceil(H/2) x ceil(W/2)
    const float* src_lo; float* dst_lo;
};
struct DerivArgs { const void* I; int H, W; int64_t ld; void* Dx; void* Dy; int64_t ldd; const float* I_lo; };
// FP32 -> FP32 or FP16 plane copy, dst = src (+ add) - offset.  Frames imported into FP16 pyramids are
// stored centred (offset kFrameOffsetF16): every pyramid step is linear and I_t is a difference, so
// the offset cancels, while FP16 spacing over [-1/2, 1/2] is half of that over [1/2, 1].
struct CopyArgs {
    const float* src; int H, W; int64_t lds; void* dst; int64_t ldd; float offset;
    const float* add;                // optional plane (pitch lds) added to src: dst = src + add - offset
};
constexpr float kFrameOffsetF16 = 0.5f;

// Batched launches of one body over many items (one work-group grid per item, prefix offsets).
enum class BatchOp { Downsample, Derivatives, Copy, Linearize, LevelInit };
int blocks_of(int H, int W);   // 64 x 4 blocks covering an H x W plane
// The linearisation's work-groups have 1024 threads and cover 64 x 16 pixels, one per thread: a~ is
// one atomic max per work-group on one word, and same-word atomics serialise, so a work-group of
// 256 threads per 256 pixels spent longer on them than on its memory traffic.
constexpr int kLinThreads = 1024;
constexpr int kLinRows = kLinThreads / 64;
int lin_blocks_of(int H, int W);
void launch_batched(BatchOp op, const void* items, const int* off, int n, int total_blocks, bool f16, hipStream_t s);

// Pyramid: 2x2 box average with edge replication, central differences, format conversion.
void launch_downsample(const void* src, int H, int W, int64_t ld, void* dst, int64_t ldd, bool f16, hipStream_t s,
                       const float* src_lo = nullptr, float* dst_lo = nullptr);
void launch_derivatives(const void* I, int H, int W, int64_t ld, void* Dx, void* Dy, int64_t ldd, bool f16,
                        hipStream_t s, const float* I_lo = nullptr);
void launch_import(const float* src, int H, int W, int64_t lds, void* dst, int64_t ldd, bool f16, hipStream_t s);
void launch_copy2d(const float* src, int H, int W, int64_t lds, float* dst, int64_t ldd, hipStream_t s,
                   const float* add = nullptr);
// Deterministic pseudo-random plane in [-scale, scale) (timing runs).
void launch_fill_noise(float* p, int H, int W, int64_t ld, uint32_t seed, float scale, hipStream_t s);

// Level start: upsample (or zero) the flow and clear / set the scheme's auxiliary planes.
struct LevelInitArgs {
    const float *uc, *vc, *wc;       // coarse flow (nullptr at the coarsest level -> zeros)
    const float *ucd, *vcd;          // optional pending increment of the coarse flow (sampled as uc + ucd)
    int Hc, Wc;
    int64_t ldc;
    float* set_flow[3];              // w, u, v targets (w may be nullptr)
    float* copy_flow[3];             // pDR X bar: copies of w, u, v (may be nullptr)
    float* zero[8];                  // planes to clear (first nzero entries)
    int nzero;
    float* clear_scalar;             // optional device scalar set to 0 (the first warp's a~ slot)
    int H, W;
    int64_t ld;
};
void launch_level_init(const LevelInitArgs& a, hipStream_t s);
void launch_upsample(const float* coarse, int64_t ldc, float* fine, int Hf, int Wf, int64_t ldf, float scale,
                     hipStream_t s);
// End of a warp in increment form: u0 += du, v0 += dv.

// pDR: three passes per symmetric sweep set (b + red, black, [red, black]*, final red + prox + dual).
struct PdrArgs {
    float *w, *u, *v;                // X, updated in place by the sweeps
    float *wb, *ub, *vb;             // X bar
    float *pbx, *pby, *qb1x, *qb1y, *qb2x, *qb2y;   // y bar
    float *bw, *bu, *bv;             // right-hand sides b = X bar + sigma div y bar
    float* s_out;                    // Theta (may be nullptr)
    const float *Ix, *Iy, *It;
    const float *u0, *v0;            // linearisation point when It is relative (else nullptr)
    int H, W;
    int64_t ld;
    float sigma, tau, stt, lam, beta;
    int colour;                      // for the plain colour sweep: 0 red, 1 black
};
// Temporally blocked pDR: K iterations of one tile per work-group launch (direct tiling of one
// level).  Component order: x / x bar (u, v, w), y (q1x, q1y, q2x, q2y, p_x, p_y).
constexpr int kPdrPpt = 2;           // pixels per thread (1024 or 512 threads)
constexpr int kPdrPptW = 2;
// Halo of a K-iteration pDR tile with n symmetric sweeps: each of the 2n + 1 half sweeps reaches one
// cell in every direction, b takes div y bar (left / above) before them and the dual update grad X+
// (right / below) after them, so X and X bar depend on the launch's input within (2n + 1) K cells
// on every side and y bar one cell further below and to the right.
constexpr int pdr_halo_lo(int n, int K) { return (2 * n + 1) * K; }
constexpr int pdr_halo_hi(int n, int K) { return (2 * n + 1) * K + 1; }
// ALG1: y+ reads X bar to the right / below, X+ reads y+ to the left / above: K cells on every side.
constexpr int alg1_halo(int K) { return K; }
struct PdrTbLevel {
    const float* x_in[3]; const float* xb_in[3]; const float* y_in[6];
    float* x_out[3]; float* xb_out[3]; float* y_out[6];
    const float *Ix, *Iy, *It, *u0, *v0;
    float* s_out;
    int H, W;
    int64_t ld;
};
struct PdrTbArgs {
    PdrTbLevel lvl;
    int K, sweeps;                   // iterations of this launch; symmetric sweeps per iteration
    int th, tw, ntx, ntiles;         // output tiling
    float sigma, tau, stt, lam, beta;
    // table order (batched pairs): with tiles set, work-groups take the ntiles entries of the tile
    // table in XCD order (8 contiguous runs, one per XCD) and each entry names its level descriptor
    // levels[2 * tile.level + dir]; lvl, th, tw and ntx are then unused
    const TbTile* tiles;
    const PdrTbLevel* levels;
    int dir;
};
int pdr_tb_capacity(bool has_w, int nt);                  // nt: 1024 or 512 threads; 2048 / 513: 1024 /
                                                          // 512 threads with two cells of each colour
                                                          // (pDR, beta = 0); 4098 / 6145: pDR wave-row
                                                          // tiles of 128 x 32 / 128 x 48 cells (6145:
                                                          // beta = 0)
bool is_pd_rows_code(int nt);
int pd_rows_width(int nt);                                // widest region of a pDR wave-row code
// an extended region of eh x ew cells fits the pDR / ALG1 tile kernel of work-group code nt
bool pd_fits(bool has_w, int nt, int64_t eh, int64_t ew);
void launch_pdr_tb(const PdrTbArgs& a, bool has_w, int nt, hipStream_t s);
void launch_pdr_rows(const PdrTbArgs& a, bool has_w, int nt, hipStream_t s);
// ALG1 on the one-cell wave-row tiles: 3074 (64 x 48 cells, beta = 0) or 2050 (64 x 32)
void launch_alg1_rows(const PdrTbArgs& a, bool has_w, int nt, hipStream_t s);
// ALG1 (primal-dual) tiles on the same argument block: sigma / tau are its primal / dual steps
void launch_alg1_tb(const PdrTbArgs& a, bool has_w, int nt, hipStream_t s);

void launch_pdr_rhs_red(const PdrArgs& a, bool has_w, hipStream_t s);
void launch_pdr_colour(const PdrArgs& a, bool has_w, hipStream_t s);
void launch_pdr_final(const PdrArgs& a, bool has_w, hipStream_t s);

// FP64 energy / dual / gap / residual with deterministic two-level reduction.
struct EnergyArgs {
    const float *w, *u, *v, *px, *py, *q1x, *q1y, *q2x, *q2y, *s;
    const float *Ix, *Iy, *It;
    int H, W;
    int64_t ld;
    float lam, beta;
    float pdr_tau;                   // > 0: duals are y bar, use q = y bar + tau grad X
    const float *du, *dv;            // increment form: flow = u + du, rho uses du (It relative)
    const float *lu0, *lv0;          // or: rho uses u - lu0, v - lv0 (It relative)
    double* partial;                 // kEnergyTerms doubles per block
    double* out;                     // kEnergyTerms doubles
};
constexpr int kEnergyTerms = 8;      // tv, data, dual, residual^2, g_tv, g_data, lam_r, nonfinite
constexpr int kEnergyBlocks = 1024;
void launch_energy(const EnergyArgs& a, hipStream_t s);
int energy_blocks(int H, int W);     // work-groups of the first energy kernel for an H x W level
// items[k] owns work-groups [off[k], off[k+1]) (off[k+1] - off[k] = energy_blocks of its level);
// each item has its own partial (that many x kEnergyTerms doubles) and out buffers
void launch_energy_batched(const EnergyArgs* items, const int* off, int n, int total_blocks, hipStream_t s);

}  // namespace flowmi
