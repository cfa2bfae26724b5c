// Kernel argument blocks and host-side launchers shared by the HIP kernels and the C-ABI runtime.
// Planes are row-major FP32 (or FP16 for stored pyramids) with a pitch `ld` in elements.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
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
constexpr int kTbPpt = 6;            // pixels per thread (beta = 0): LDS q1x..q2y, gu, gv
constexpr int kTbPptW = 4;           // with the w / p block
constexpr int kTbPptSmall = 2;       // 1024 threads on small tiles (work-group size code 1025)
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
    const TbLevel* levels;           // two descriptors per (pair, level): [2 * id + dir]
    int dir;                         // which ping-pong direction this launch uses
    int K;                           // iterations of this launch (halo = 2K top/left, K bottom/right)
    int at_slot;                     // a~ slot of the current warp
    unsigned* queue;                 // work counter, monotone within a solve (nullptr: direct mode)
    unsigned queue_base;             // counter value at the start of this launch
    float c, lam, beta, inv_ac, c_rho_s, cA, cB, cC;
    // direct mode (one level, regular tiles): descriptor of this launch's direction and tiling
    TbLevel lvl;
    int th, tw, ntx;
};
int tb_capacity(bool has_w, int nt);   // nt: 256, 1024, or 1025 (1024 threads, small tiles)
void launch_admm_tb(const TbArgs& a, bool has_w, int nt, int grid, hipStream_t s);
void launch_reset_u32(unsigned* p, int n, hipStream_t s);

// Warp + linearise + a~ (max of M_s) with a last-block finalisation.
struct LinArgs {
    const void *I0, *I1, *Dx, *Dy;   // float or __half, pitch ld
    const float *u0, *v0;            // pitch ld
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

// Pyramid: 2x2 box average with edge replication, central differences, format conversion.
void launch_downsample(const void* src, int H, int W, int64_t ld, void* dst, int64_t ldd, bool f16, hipStream_t s);
void launch_derivatives(const void* I, int H, int W, int64_t ld, void* Dx, void* Dy, int64_t ldd, bool f16,
                        hipStream_t s);
void launch_import(const float* src, int H, int W, int64_t lds, void* dst, int64_t ldd, bool f16, hipStream_t s);
void launch_copy2d(const float* src, int H, int W, int64_t lds, float* dst, int64_t ldd, hipStream_t s);

// Level start: upsample (or zero) the flow and clear / set the scheme's auxiliary planes.
struct LevelInitArgs {
    const float *uc, *vc, *wc;       // coarse flow (nullptr at the coarsest level -> zeros)
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
void launch_commit(float* u0, float* v0, const float* du, const float* dv, int H, int W, int64_t ld, hipStream_t s);

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
constexpr int kEnergyBlocks = 512;
void launch_energy(const EnergyArgs& a, hipStream_t s);

}  // namespace flowmi
