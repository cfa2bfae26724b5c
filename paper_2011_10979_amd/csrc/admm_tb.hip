// Temporally blocked iterations of the preconditioned dual ADMM family (Sec. 3.1.1) on gfx950.
//
// One work-group owns an output tile of one pyramid level (of one pair) and advances it by K
// iterations in a single launch.  g needs q to the left and above, y+ needs g to the right and
// below, and the multipliers need div y+ (left and above), which is also the divergence the next
// g takes.  So the new q depends on the previous iterate within one cell in every direction, and
// the multipliers one cell further to the left and above: after K iterations the valid region has
// shrunk by K + 1 rows / columns at the top and left and K at the bottom and right, and the tile
// is loaded with that halo; on sides where the tile meets the image border there is no halo and
// the discrete boundary rules of Sec. 2.2 apply exactly.  Halo pixels are recomputed by the
// neighbouring tiles; their values here only feed other halo pixels.
//
// Placement: q (and p), whose neighbours the divergence reads, and g, whose neighbours the
// gradient reads, live in LDS; everything only read at its own pixel (the increment du, dv, s,
// w and the linearisation I_x, I_y, I_t, u0, v0) lives in registers of the thread that owns the
// pixel for the whole launch.  Per iteration:  A: g from q (LDS) -> LDS;  barrier;  B: y+ from
// g (LDS), written over q;  barrier;  C: div y+, s+, multipliers (registers), then A of the next
// iteration from the divergence C has just taken (C only reads y+, A only writes g, so they need
// no barrier between them).
//
// Work distribution: one work-group per tile of one level (direct), per entry of a tile table
// (batched pairs: each tile names its pair-level descriptor), or a persistent grid that pulls
// tile indices from device counters.  Tiles of one launch read one state buffer and write the
// other, so they never depend on each other, and every work-group of the persistent grid exits
// once its counter passes the end of its run of tiles.
#include <type_traits>

#include "kernels.hpp"

namespace flowmi {

namespace {

template <bool HAS_W, int NT, int PPT>
struct TileLds {
    static constexpr int CAP = NT * PPT;
    float sq1x[CAP], sq1y[CAP], sq2x[CAP], sq2y[CAP], sgu[CAP], sgv[CAP];
    float spx[HAS_W ? CAP : 1], spy[HAS_W ? CAP : 1], sgw[HAS_W ? CAP : 1];
};

// K iterations of output tile T of level L by the calling work-group.
//
// Control flow is wavefront-uniform: a wavefront skips a slot only when none of its lanes holds a
// pixel of the extended region; otherwise every lane runs it (lanes past the region hold zeros and
// compute values nobody uses).  Neighbour values are read from LDS at indices clamped into the
// array and weighted by the operators' coefficients, so no read sits behind a branch and the reads
// of a phase issue together.
template <bool HAS_W, int NT, int PPT, bool BAND>
__device__ __forceinline__ void process_tile(const TbArgs& a, const TbTile& T, const TbLevel& L,
                                             TileLds<HAS_W, NT, PPT>& S) {
    constexpr int CAP = NT * PPT;
    float* sq1x = S.sq1x; float* sq1y = S.sq1y; float* sq2x = S.sq2x; float* sq2y = S.sq2y;
    float* sgu = S.sgu; float* sgv = S.sgv; float* spx = S.spx; float* spy = S.spy; float* sgw = S.sgw;
    const int tid = threadIdx.x;
    const float c = a.c, inv_ac = a.inv_ac, beta = a.beta, crs = a.c_rho_s;
    {
        const int H = L.H, W = L.W;
        const int64_t ld = L.ld;
        const int K = a.K;
        // extended region: output tile plus halo, clipped to the image
        const int ey0 = max(T.y0 - tb_halo_lo(K), 0), ex0 = max(T.x0 - tb_halo_lo(K), 0);
        const int ey1 = min(T.y0 + T.th + K, H), ex1 = min(T.x0 + T.tw + K, W);
        const int EW = ex1 - ex0, EN = (ey1 - ey0) * EW;
        const float inv_atc = 1.f / (fmaxf(L.at[a.at_slot], 1e-12f) * c);   // a~ >= ||M_s||, floored

        float du[PPT], dv[PPT], ss[PPT], Ix[PPT], Iy[PPT], It[PPT], u0[PPT], v0[PPT], ww[PPT];
        // the thread's own dual values (q1x, q1y, q2x, q2y[, p_x, p_y]) and g (u, v[, w]): only the
        // owner writes them, so with two pixels per thread they stay in registers and LDS serves the
        // neighbours' reads (larger shapes would spill and read their own values from LDS)
        constexpr int NQ = HAS_W ? 6 : 4, NG = HAS_W ? 3 : 2;
        constexpr bool OWN = PPT <= 2;
        float qo[NQ][PPT], go[NG][PPT];
        float* const sqa[6] = {sq1x, sq1y, sq2x, sq2y, spx, spy};
        float* const sga[3] = {sgu, sgv, sgw};
        // Shrinking band: after iteration m only the region shrunk by m rows on each side with a
        // halo (a side that is not the image border) can still reach the output tile, so a
        // wavefront all of whose rows lie outside it skips the iteration.  Its stale values are as
        // harmless as any other value outside the valid region.  With several pixels per thread a
        // tile that shrinks lays its slots out so that a wavefront covers consecutive rows (its PPT
        // slots are PPT consecutive runs of 64 in the extended region's row-major order); any other
        // tile strides them by the work-group size, which spreads a partly filled region evenly over
        // the wavefronts.  With one pixel per thread both layouts coincide, and the skip costs more
        // than it saves (the iteration is bound by the LDS round trips and barriers, not by issue).
        const int EH = ey1 - ey0;
        const int shr_top = ey0 > 0, shr_bot = ey1 < H;
        const bool band = BAND && PPT > 1 && (shr_top || shr_bot);
        const int wave0 = __builtin_amdgcn_readfirstlane(tid & ~63);
        const int wbase = band ? wave0 * PPT : wave0, stride = band ? 64 : NT;
        const int sbase = wbase + (tid & 63);
        auto slot = [&](int k) { return sbase + k * stride; };
        auto qown = [&](int f, int k) { return OWN ? qo[f][k] : sqa[f][slot(k)]; };
        auto gown = [&](int f, int k) { return OWN ? go[f][k] : sga[f][slot(k)]; };
        // Per-slot neighbour structure, fixed for the launch: in-array neighbour indices clamped into
        // the array, and the operators' coefficients of Sec. 2.2 -- the forward difference exists in
        // the image (fx, fy; folded with 1 / (a c) into cx, cy for the dual step) and the divergence's
        // left / upper term exists (fl, fu).  Only the image border decides a coefficient: at the edge
        // of the extended region a neighbour index may land on an unrelated slot, which only changes
        // halo pixels that are no longer valid (the halo accounts for them).  Every LDS slot holds a
        // finite value, so a zero coefficient times such a read is exactly zero.
        int ei[PPT], ej[PPT], iL[PPT], iU[PPT], iR[PPT], iD[PPT];
        float fx[PPT], fy[PPT], fl[PPT], fu[PPT], cx[PPT], cy[PPT];
        // slot k of this wavefront holds any pixel of the extended region (wave-uniform, scalar branch)
        auto live = [&](int k) { return wbase + k * stride < EN; };
        // first and last row of the wavefront's pixels in the band layout (wave-uniform)
        const int wr0 = __builtin_amdgcn_readfirstlane(min(wbase, EN - 1) / EW);
        const int wr1 = __builtin_amdgcn_readfirstlane(min(wbase + 64 * PPT - 1, EN - 1) / EW);
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int e = slot(k);
            ei[k] = e / EW;
            ej[k] = e - ei[k] * EW;
            const int gi = ey0 + ei[k], gj = ex0 + ej[k];
            iL[k] = max(e - 1, 0);
            iU[k] = max(e - EW, 0);
            iR[k] = min(e + 1, CAP - 1);
            iD[k] = min(e + EW, CAP - 1);
            fx[k] = gj < W - 1 ? 1.f : 0.f;
            fy[k] = gi < H - 1 ? 1.f : 0.f;
            fl[k] = gj > 0 ? 1.f : 0.f;
            fu[k] = gi > 0 ? 1.f : 0.f;
            cx[k] = fx[k] * inv_ac;
            cy[k] = fy[k] * inv_ac;
            du[k] = dv[k] = ss[k] = Ix[k] = Iy[k] = It[k] = u0[k] = v0[k] = ww[k] = 0.f;
            float q1x = 0.f, q1y = 0.f, q2x = 0.f, q2y = 0.f, px = 0.f, py = 0.f;
            if (e < EN) {
                const int64_t o = (int64_t)gi * ld + gj;
                q1x = L.in[5][o];
                q1y = L.in[6][o];
                q2x = L.in[7][o];
                q2y = L.in[8][o];
                du[k] = L.in[1][o];
                dv[k] = L.in[2][o];
                ss[k] = L.in[9][o];
                Ix[k] = L.Ix[o];
                Iy[k] = L.Iy[o];
                It[k] = L.It[o];
                u0[k] = L.u0[o];
                v0[k] = L.v0[o];
                if constexpr (HAS_W) {
                    px = L.in[3][o];
                    py = L.in[4][o];
                    ww[k] = L.in[0][o];
                }
            }
            sq1x[e] = qo[0][k] = q1x;
            sq1y[e] = qo[1][k] = q1y;
            sq2x[e] = qo[2][k] = q2x;
            sq2y[e] = qo[3][k] = q2y;
            if constexpr (HAS_W) {
                spx[e] = qo[4][k] = px;
                spy[e] = qo[5][k] = py;
            }
        }
        __syncthreads();

        // divergence of a dual field at slot k from its own, left and upper values:
        // [j < W-1] ax(i,j) - [j > 0] ax(i,j-1) + [i < H-1] ay(i,j) - [i > 0] ay(i-1,j)
        auto divv = [&](int k, float ax, float al, float ay, float au) {
            float d = fmaf(fx[k], ax, -(fl[k] * al));
            d = fmaf(fy[k], ay, d);
            return fmaf(-fu[k], au, d);
        };
        // divergence of dual field f (0: q1, 1: q2, 2: p) at slot k, own values from registers
        auto divf = [&](int f, int k) {
            const float* sx[3] = {sq1x, sq2x, spx};
            const float* sy[3] = {sq1y, sq2y, spy};
            return divv(k, qown(2 * f, k), sx[f][iL[k]], qown(2 * f + 1, k), sy[f][iU[k]]);
        };
        // phase A (g) for slot k from the divergences of the current dual field
        auto g_out = [&](int k, int e, float dq1, float dq2, float dp) {
            sgu[e] = go[0][k] = u0[k] + (du[k] + c * (dq1 - Ix[k] * ss[k]));
            sgv[e] = go[1][k] = v0[k] + (dv[k] + c * (dq2 - Iy[k] * ss[k]));
            if constexpr (HAS_W) sgw[e] = go[2][k] = ww[k] + c * (dp - beta * ss[k]);
        };
        // Each phase reads the operands of a group of GS slots before it writes LDS, so the reads of
        // the group issue together (the compiler cannot move LDS reads at computed indices past
        // writes); groups of two keep the larger work-group shapes within their register budget.
        constexpr int GS = 2;
        // phase B: y+ = P(y + grad g / (a c)), in place over q (B reads q only at its own slot)
        auto phase_b = [&](auto all_live) {
            constexpr bool AL = decltype(all_live)::value;
            float* sg[3] = {sgu, sgv, sgw};
#pragma unroll
            for (int k0 = 0; k0 < PPT; k0 += GS) {
                float gr[NG][GS], gd[NG][GS];
#pragma unroll
                for (int j = 0; j < GS; ++j) {
                    const int k = k0 + j;
                    if (k >= PPT || (!AL && !live(k))) continue;
#pragma unroll
                    for (int f = 0; f < NG; ++f) {
                        gr[f][j] = sg[f][iR[k]];
                        gd[f][j] = sg[f][iD[k]];
                    }
                }
#pragma unroll
                for (int j = 0; j < GS; ++j) {
                    const int k = k0 + j;
                    if (k >= PPT || (!AL && !live(k))) continue;
                    const int e = slot(k);
                    const float t1x = fmaf(gr[0][j] - gown(0, k), cx[k], qown(0, k));
                    const float t1y = fmaf(gd[0][j] - gown(0, k), cy[k], qown(1, k));
                    const float t2x = fmaf(gr[1][j] - gown(1, k), cx[k], qown(2, k));
                    const float t2y = fmaf(gd[1][j] - gown(1, k), cy[k], qown(3, k));
                    // sums of products as explicit FMA chains: every tile kernel rounds them alike
                    const float nq = fmaf(t2y, t2y, fmaf(t2x, t2x, fmaf(t1y, t1y, t1x * t1x)));
                    // projection scale min(1, 1/|t|): the hardware reciprocal square root is at
                    // least 1 (or infinite) wherever |t| <= 1, so the min alone selects
                    const float sc = fminf(1.f, __builtin_amdgcn_rsqf(nq));
                    sq1x[e] = qo[0][k] = t1x * sc;
                    sq1y[e] = qo[1][k] = t1y * sc;
                    sq2x[e] = qo[2][k] = t2x * sc;
                    sq2y[e] = qo[3][k] = t2y * sc;
                    if constexpr (HAS_W) {
                        const float tpx = fmaf(gr[NG - 1][j] - gown(NG - 1, k), cx[k], qown(4, k));
                        const float tpy = fmaf(gd[NG - 1][j] - gown(NG - 1, k), cy[k], qown(5, k));
                        const float np2 = fmaf(tpy, tpy, tpx * tpx);
                        const float sp = fminf(1.f, __builtin_amdgcn_rsqf(np2));
                        spx[e] = qo[4][k] = tpx * sp;
                        spy[e] = qo[5][k] = tpy * sp;
                    }
                }
            }
        };
        // phase C: div y+, s+, multipliers (own slots, registers), then phase A of the next iteration
        // from the same divergences (C only reads y+, A only writes g: no barrier between them)
        auto phase_c = [&](auto all_live, bool next) {
            constexpr bool AL = decltype(all_live)::value;
            constexpr int ND = HAS_W ? 3 : 2;
#pragma unroll
            for (int k0 = 0; k0 < PPT; k0 += GS) {
                float dn[ND][GS];
#pragma unroll
                for (int j = 0; j < GS; ++j) {
                    const int k = k0 + j;
                    if (k >= PPT || (!AL && !live(k))) continue;
#pragma unroll
                    for (int f = 0; f < ND; ++f) dn[f][j] = divf(f, k);
                }
#pragma unroll
                for (int j = 0; j < GS; ++j) {
                    const int k = k0 + j;
                    if (k >= PPT || (!AL && !live(k))) continue;
                    const int e = slot(k);
                    const float dn1 = dn[0][j], dn2 = dn[1][j];
                    const float hu_ = du[k] + crs * (dn1 - Ix[k] * ss[k]);
                    const float hv_ = dv[k] + crs * (dn2 - Iy[k] * ss[k]);
                    float acc = It[k] + Ix[k] * hu_ + Iy[k] * hv_;
                    float dnp = 0.f;
                    if constexpr (HAS_W) {
                        dnp = dn[ND - 1][j];
                        acc += beta * (ww[k] + crs * (dnp - beta * ss[k]));
                    }
                    float sn = ss[k] + acc * inv_atc;
                    sn = __builtin_amdgcn_fmed3f(sn, -a.lam, a.lam);
                    const float ms = fmaf(a.cB, sn, -(a.cC * ss[k]));
                    du[k] = du[k] + a.cA * dn1 - Ix[k] * ms;
                    dv[k] = dv[k] + a.cA * dn2 - Iy[k] * ms;
                    if constexpr (HAS_W) ww[k] = ww[k] + a.cA * dnp - beta * ms;
                    ss[k] = sn;
                    if (next) g_out(k, e, dn1, dn2, dnp);
                }
            }
        };

        // phase A at the start: every slot, so that every g slot in LDS holds a finite value
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int e = slot(k);
            float dp = 0.f;
            if constexpr (HAS_W) dp = divf(2, k);
            g_out(k, e, divf(0, k), divf(1, k), dp);
        }
        // a wavefront whose last slot holds a pixel of the region runs every slot without branches,
        // so the LDS reads of all its slots issue together
        const bool all_live = live(PPT - 1);
        for (int it = 0; it < K; ++it) {
            const int band_lo = shr_top * (it + 1), band_hi = EH - shr_bot * (it + 1);
            const bool run = !band || __builtin_amdgcn_readfirstlane(live(0) && wr1 >= band_lo && wr0 < band_hi);
            __syncthreads();
            if (run) {
                if (all_live) phase_b(std::true_type{});
                else phase_b(std::false_type{});
            }
            __syncthreads();
            if (run) {
                if (all_live) phase_c(std::true_type{}, it + 1 < K);
                else phase_c(std::false_type{}, it + 1 < K);
            }
        }

        // write the output tile
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int e = slot(k);
            if (e >= EN) continue;
            const int ei = e / EW, ej = e - ei * EW;
            const int gi = ey0 + ei, gj = ex0 + ej;
            if (gi < T.y0 || gi >= T.y0 + T.th || gj < T.x0 || gj >= T.x0 + T.tw) continue;
            const int64_t o = (int64_t)gi * ld + gj;
            L.out[1][o] = du[k];
            L.out[2][o] = dv[k];
            L.out[9][o] = ss[k];
            L.out[5][o] = qown(0, k);
            L.out[6][o] = qown(1, k);
            L.out[7][o] = qown(2, k);
            L.out[8][o] = qown(3, k);
            if constexpr (HAS_W) {
                L.out[0][o] = ww[k];
                L.out[3][o] = qown(4, k);
                L.out[4][o] = qown(5, k);
            }
        }
    }
}

// Minimum wavefronts per SIMD each kernel shape asks the register allocator to allow: with two
// pixels per thread, no w and the shrinking band, 64 VGPRs give 8 wavefronts per SIMD (two
// 1024-thread work-groups, or four of 512, per CU), which hide each other's barriers and loads;
// other shapes leave the allocator free.  BAND = false: the kernel is only launched on a level
// that one tile covers (nothing shrinks), without the band's per-iteration test.
template <bool HAS_W, int NT, int PPT, bool BAND>
constexpr int tb_waves_per_simd() { return (!HAS_W && PPT == 2 && BAND) ? 8 : 1; }

__device__ __forceinline__ int xcd_tile(int b, int nb) {
    // work-groups are dealt round-robin to the 8 XCDs; neighbouring tiles (which re-read each
    // other's halo) go to the same XCD's L2
    const int per = nb >> 3;   // host pads the grid to a multiple of 8
    return (b & 7) * per + (b >> 3);
}

// One level, regular tiling: the tile comes from the work-group index, the level descriptor from
// the kernel arguments (no table reads, no counter).
template <bool HAS_W, int NT, int PPT, bool BAND>
__global__ __launch_bounds__(NT, (tb_waves_per_simd<HAS_W, NT, PPT, BAND>())) void admm_tb_direct_kernel(TbArgs a) {
    __shared__ TileLds<HAS_W, NT, PPT> S;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    if (t >= a.ntiles) return;
    TbTile T;
    T.level = 0;
    const int ty = t / a.ntx, tx = t - ty * a.ntx;
    T.y0 = ty * a.th;
    T.x0 = tx * a.tw;
    T.th = min(a.th, a.lvl.H - T.y0);
    T.tw = min(a.tw, a.lvl.W - T.x0);
    process_tile<HAS_W, NT, PPT, BAND>(a, T, a.lvl, S);
}

// Many levels (batched pairs), table order: one tile per work-group.  The n tiles are split into 8
// contiguous runs, one per XCD (work-groups are dealt to the XCDs round-robin, so XCD x holds
// work-groups b = x (mod 8)): neighbouring tiles, which re-read each other's halo, share its L2,
// and a grid larger than the table (a launch replayed from a graph over changing tables) still
// spreads a small table over every XCD.  The grid is a multiple of 8 of at least n.
template <bool HAS_W, int NT, int PPT>
__global__ __launch_bounds__(NT, (tb_waves_per_simd<HAS_W, NT, PPT, true>())) void admm_tb_table_kernel(TbArgs a) {
    __shared__ TileLds<HAS_W, NT, PPT> S;
    const int n = a.ntiles_dev ? *a.ntiles_dev : a.ntiles;
    const int per = (n + 7) >> 3;                      // tiles per XCD
    const int x = blockIdx.x & 7, y = blockIdx.x >> 3;
    const int t = x * per + y;
    if (y >= per || t >= n) return;
    const TbTile T = a.tiles[t];
    process_tile<HAS_W, NT, PPT, true>(a, T, a.levels[2 * T.level + a.dir], S);
}

// Many levels (batched pairs), work queue: a persistent grid pulls (level, tile) items from nq
// counters; sub-queue x owns a contiguous run of the table and is drained by the work-groups
// b = x (mod nq), which the dispatcher places on one XCD when nq = 8.
template <bool HAS_W, int NT, int PPT>
__global__ __launch_bounds__(NT, (tb_waves_per_simd<HAS_W, NT, PPT, true>())) void admm_tb_queue_kernel(TbArgs a) {
    __shared__ TileLds<HAS_W, NT, PPT> S;
    __shared__ int s_tile;
    const int n = a.ntiles_dev ? *a.ntiles_dev : a.ntiles;
    const int x = blockIdx.x % a.nq;
    const int lo = (int)((int64_t)n * x / a.nq);
    const int hi = (int)((int64_t)n * (x + 1) / a.nq);
    for (;;) {
        if (threadIdx.x == 0) s_tile = lo + (int)(atomicAdd(a.queue + x, 1u) - a.queue_base);
        __syncthreads();
        const int t = s_tile;
        __syncthreads();                  // everyone has read s_tile before it is overwritten
        if (t >= hi) break;               // uniform: the whole work-group leaves together
        const TbTile T = a.tiles[t];
        process_tile<HAS_W, NT, PPT, true>(a, T, a.levels[2 * T.level + a.dir], S);
        __syncthreads();                  // LDS is reused by the next tile
    }
}

__global__ void reset_u32_kernel(unsigned* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

}  // namespace

void launch_reset_u32(unsigned* p, int n, hipStream_t s) {
    hipLaunchKernelGGL(reset_u32_kernel, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
}


// direct tiling; a level that one tile covers runs the instance without the shrinking band
template <bool HAS_W, int NT, int PPT>
static void launch_direct(const TbArgs& a, int grid, hipStream_t s) {
    if constexpr (PPT > 1) {
        const bool whole = a.ntiles == 1 && a.th >= a.lvl.H && a.tw >= a.lvl.W;
        if (!whole) {
            hipLaunchKernelGGL((admm_tb_direct_kernel<HAS_W, NT, PPT, true>), dim3(grid), dim3(NT), 0, s, a);
            return;
        }
    }
    hipLaunchKernelGGL((admm_tb_direct_kernel<HAS_W, NT, PPT, false>), dim3(grid), dim3(NT), 0, s, a);
}

template <bool HAS_W, int NT, int PPT>
static void launch_one(const TbArgs& a, int grid, hipStream_t s) {
    if (a.queue) hipLaunchKernelGGL((admm_tb_queue_kernel<HAS_W, NT, PPT>), dim3(grid), dim3(NT), 0, s, a);
    else if (a.tiles) hipLaunchKernelGGL((admm_tb_table_kernel<HAS_W, NT, PPT>), dim3(grid), dim3(NT), 0, s, a);
    else launch_direct<HAS_W, NT, PPT>(a, grid, s);
}

void launch_admm_tb(const TbArgs& a, bool has_w, int nt, int grid, hipStream_t s) {
    if (is_rows_code(nt)) {                     // direct or table order (callers never pass a queue)
        if (!a.queue) launch_admm_rows(a, has_w, nt, grid, s);
        return;
    }
    if (!a.queue) grid = (grid + 7) / 8 * 8;     // direct / table order: the XCD remap wants a multiple of 8
    if (nt == 1024) {
        if (has_w) launch_one<true, 1024, kTbPptLW>(a, grid, s);
        else launch_one<false, 1024, kTbPptL>(a, grid, s);
    } else if (nt == 1025) {
        if (has_w) launch_one<true, 1024, kTbPptSmall>(a, grid, s);
        else launch_one<false, 1024, kTbPptSmall>(a, grid, s);
    } else if (nt == 1026 || nt == 514) {
        // one pixel per thread, for latency-bound levels: direct tiling only
        if (nt == 1026) {
            if (has_w) launch_direct<true, 1024, 1>(a, grid, s);
            else launch_direct<false, 1024, 1>(a, grid, s);
        } else {
            if (has_w) launch_direct<true, 512, 1>(a, grid, s);
            else launch_direct<false, 512, 1>(a, grid, s);
        }
    } else if (nt == 513 || nt == 257) {
        // small work-groups for latency-bound levels: direct tiling only
        if (nt == 513) {
            if (has_w) launch_direct<true, 512, kTbPptSmall>(a, grid, s);
            else launch_direct<false, 512, kTbPptSmall>(a, grid, s);
        } else {
            if (has_w) launch_direct<true, 256, kTbPptSmall>(a, grid, s);
            else launch_direct<false, 256, kTbPptSmall>(a, grid, s);
        }
    } else {
        if (has_w) launch_one<true, 256, kTbPptW>(a, grid, s);
        else launch_one<false, 256, kTbPpt>(a, grid, s);
    }
}

}  // namespace flowmi
