// Temporally blocked iterations of ALG1, the first-order primal-dual method that Sec. 4 compares the
// preconditioned schemes against, on the saddle form eq:primal-dual:optical:o (K = diag(grad, grad),
// F the data term, unit balls for p and the coupled q), extrapolation weight 1:
//   [Y]  y+     = P(y + tau grad X bar)                   (reads X bar at the right / lower neighbour)
//   [X]  X+     = (I + sigma dF)^{-1}(X + sigma div y+)   (eq:resolvent; reads y+ left / above)
//        X bar+ = 2 X+ - X
// with a barrier after each phase.  A value reaches one cell in every direction per iteration, so a
// tile is loaded with a halo of K on each side (none where it meets the image border, where the
// boundary rules of Sec. 2.2 apply exactly).  X bar and y, whose neighbours are read, live in LDS;
// X and the linearisation live in registers.  Reads and writes go to different state sets, so the
// tiles of one launch are independent.  Neighbour reads are unconditional LDS reads at indices
// clamped into the array, weighted by the operators' coefficients.
#include <type_traits>

#include "kernels.hpp"

namespace flowmi {

namespace {

template <bool HAS_W, int NT, int PPT>
struct Alg1Lds {
    static constexpr int CAP = NT * PPT;
    static constexpr int NX = HAS_W ? 3 : 2;
    static constexpr int NY = HAS_W ? 6 : 4;
    float xb[NX][CAP];
    float y[NY][CAP];
};

template <bool HAS_W, int NT, int PPT>
__device__ __forceinline__ void alg1_tile(const PdrTbArgs& a, const PdrTbLevel& L, int y0, int x0, int th, int tw,
                                          Alg1Lds<HAS_W, NT, PPT>& S) {
    constexpr int CAP = NT * PPT;
    constexpr int NX = Alg1Lds<HAS_W, NT, PPT>::NX;
    constexpr int NY = Alg1Lds<HAS_W, NT, PPT>::NY;
    const int tid = threadIdx.x;
    const int H = L.H, W = L.W;
    const int64_t ld = L.ld;
    const int K = a.K;
    const int hk = alg1_halo(K);
    const int ey0 = max(y0 - hk, 0), ex0 = max(x0 - hk, 0);
    const int ey1 = min(y0 + th + hk, H), ex1 = min(x0 + tw + hk, W);
    const int EW = ex1 - ex0, EN = (ey1 - ey0) * EW;
    const float sigma = a.sigma, tau = a.tau, lam = a.lam, beta = a.beta;
    const float sl = sigma * lam, inv_sigma = 1.f / sigma;
    const int wave0 = __builtin_amdgcn_readfirstlane(tid & ~63);
    auto live = [&](int k) { return wave0 + k * NT < EN; };

    // Per-slot neighbour structure, fixed for the launch: neighbour indices clamped into the array
    // and the operators' coefficients of Sec. 2.2 (the forward difference exists in the image: fx,
    // fy, folded with tau into cx, cy; the divergence's left / upper term exists: fl, fu).  Only the
    // image border decides a coefficient; at the edge of the extended region an index may land on
    // an unrelated slot, which only changes halo pixels the halo accounts for.  Every LDS slot holds
    // a finite value, so a zero coefficient times such a read is exactly zero.
    // components: x / x bar (u, v, w); y (q1x, q1y, q2x, q2y, p_x, p_y)
    int ei[PPT], ej[PPT], iL[PPT], iU[PPT], iR[PPT], iD[PPT];
    float fx[PPT], fy[PPT], fl[PPT], fu[PPT], cx[PPT], cy[PPT];
    float x[NX][PPT], Ix[PPT], Iy[PPT], It[PPT], u0[PPT], v0[PPT], th_s[PPT];
    // the thread's own X bar and y: only the owner writes them, so they stay in registers and LDS
    // serves the neighbours' reads
    float xbo[NX][PPT], yow[NY][PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int e = tid + k * NT;
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
        cx[k] = fx[k] * tau;
        cy[k] = fy[k] * tau;
        float xbv[NX], yv[NY];
#pragma unroll
        for (int c = 0; c < NX; ++c) x[c][k] = xbv[c] = 0.f;
#pragma unroll
        for (int c = 0; c < NY; ++c) yv[c] = 0.f;
        Ix[k] = Iy[k] = It[k] = u0[k] = v0[k] = th_s[k] = 0.f;
        if (e < EN) {
            const int64_t o = (int64_t)gi * ld + gj;
#pragma unroll
            for (int c = 0; c < NX; ++c) {
                x[c][k] = L.x_in[c][o];
                xbv[c] = L.xb_in[c][o];
            }
#pragma unroll
            for (int c = 0; c < NY; ++c) yv[c] = L.y_in[c][o];
            Ix[k] = L.Ix[o];
            Iy[k] = L.Iy[o];
            It[k] = L.It[o];
            u0[k] = L.u0[o];
            v0[k] = L.v0[o];
        }
#pragma unroll
        for (int c = 0; c < NX; ++c) S.xb[c][e] = xbo[c][k] = xbv[c];
#pragma unroll
        for (int c = 0; c < NY; ++c) S.y[c][e] = yow[c][k] = yv[c];
    }
    __syncthreads();

    // Each phase reads the operands of a group of GS slots before it writes LDS, so the reads of
    // the group issue together (the compiler cannot move LDS reads at computed indices past writes).
    constexpr int GS = 2;
    // [Y]: dual ascent from the forward differences of X bar, projected (joint q ball, p ball)
    auto phase_y = [&](auto all_live) {
        constexpr bool AL = decltype(all_live)::value;
#pragma unroll
        for (int k0 = 0; k0 < PPT; k0 += GS) {
            float xr[NX][GS], xd[NX][GS];
#pragma unroll
            for (int j = 0; j < GS; ++j) {
                const int k = k0 + j;
                if (k >= PPT || (!AL && !live(k))) continue;
#pragma unroll
                for (int c = 0; c < NX; ++c) {
                    xr[c][j] = S.xb[c][iR[k]];
                    xd[c][j] = S.xb[c][iD[k]];
                }
            }
#pragma unroll
            for (int j = 0; j < GS; ++j) {
                const int k = k0 + j;
                if (k >= PPT || (!AL && !live(k))) continue;
                const int e = tid + k * NT;
                const float a1x = fmaf(cx[k], xr[0][j] - xbo[0][k], yow[0][k]);
                const float a1y = fmaf(cy[k], xd[0][j] - xbo[0][k], yow[1][k]);
                const float a2x = fmaf(cx[k], xr[1][j] - xbo[1][k], yow[2][k]);
                const float a2y = fmaf(cy[k], xd[1][j] - xbo[1][k], yow[3][k]);
                // sums of products as explicit FMA chains: every ALG1 tile kernel rounds them alike
                const float nq = fmaf(a2y, a2y, fmaf(a2x, a2x, fmaf(a1y, a1y, a1x * a1x)));
                const float sq = fminf(1.f, __builtin_amdgcn_rsqf(nq));
                S.y[0][e] = yow[0][k] = a1x * sq;
                S.y[1][e] = yow[1][k] = a1y * sq;
                S.y[2][e] = yow[2][k] = a2x * sq;
                S.y[3][e] = yow[3][k] = a2y * sq;
                if constexpr (HAS_W) {
                    const float bx = fmaf(cx[k], xr[2][j] - xbo[2][k], yow[4][k]);
                    const float by = fmaf(cy[k], xd[2][j] - xbo[2][k], yow[5][k]);
                    const float np2 = fmaf(by, by, bx * bx);
                    const float sp = fminf(1.f, __builtin_amdgcn_rsqf(np2));
                    S.y[4][e] = yow[4][k] = bx * sp;
                    S.y[5][e] = yow[5][k] = by * sp;
                }
            }
        }
    };
    // [X]: primal proximal descent X+ = J(X + sigma div y+), extrapolation X bar+ = 2 X+ - X
    auto phase_x = [&](auto all_live) {
        constexpr bool AL = decltype(all_live)::value;
#pragma unroll
        for (int k0 = 0; k0 < PPT; k0 += GS) {
            float dvv[NX][GS];
#pragma unroll
            for (int j = 0; j < GS; ++j) {
                const int k = k0 + j;
                if (k >= PPT || (!AL && !live(k))) continue;
                // [j < W-1] y_x - [j > 0] y_x(left) + [i < H-1] y_y - [i > 0] y_y(up)
#pragma unroll
                for (int c = 0; c < NX; ++c) {
                    float d = fmaf(fx[k], yow[2 * c][k], -(fl[k] * S.y[2 * c][iL[k]]));
                    d = fmaf(fy[k], yow[2 * c + 1][k], d);
                    dvv[c][j] = fmaf(-fu[k], S.y[2 * c + 1][iU[k]], d);
                }
            }
#pragma unroll
            for (int j = 0; j < GS; ++j) {
                const int k = k0 + j;
                if (k >= PPT || (!AL && !live(k))) continue;
                const int e = tid + k * NT;
                const float ut = x[0][k] + sigma * dvv[0][j];
                const float vt = x[1][k] + sigma * dvv[1][j];
                float wt = 0.f;
                if constexpr (HAS_W) wt = x[2][k] + sigma * dvv[NX - 1][j];
                const float e2 = fmaf(Iy[k], Iy[k], fmaf(Ix[k], Ix[k], beta * beta));
                const float rho = fmaf(Iy[k], vt - v0[k], fmaf(Ix[k], ut - u0[k], fmaf(beta, wt, It[k])));
                // eq:resolvent with step sigma: -rho / |e|^2 clamped to [-sigma lam, sigma lam], and
                // Theta = clamp(rho / (sigma |e|^2), -lam, lam) = -step / sigma (both 0 where e = 0);
                // 1 / |e|^2 is the hardware reciprocal (within 1 ulp)
                float step = 0.f, theta = 0.f;
                if (e2 > 0.f) {
                    step = __builtin_amdgcn_fmed3f(-rho * __builtin_amdgcn_rcpf(e2), -sl, sl);
                    theta = -step * inv_sigma;
                }
                const float un = ut + step * Ix[k], vn = vt + step * Iy[k];
                S.xb[0][e] = xbo[0][k] = 2.f * un - x[0][k];
                S.xb[1][e] = xbo[1][k] = 2.f * vn - x[1][k];
                x[0][k] = un;
                x[1][k] = vn;
                if constexpr (HAS_W) {
                    const float wn = wt + step * beta;
                    S.xb[2][e] = xbo[2][k] = 2.f * wn - x[2][k];
                    x[2][k] = wn;
                }
                th_s[k] = theta;
            }
        }
    };

    // a wavefront whose last slot holds a pixel of the region runs every slot without branches
    const bool all_live = live(PPT - 1);
    for (int it = 0; it < K; ++it) {
        if (all_live) phase_y(std::true_type{});
        else phase_y(std::false_type{});
        __syncthreads();
        if (all_live) phase_x(std::true_type{});
        else phase_x(std::false_type{});
        __syncthreads();
    }

    // write the output tile
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int e = tid + k * NT;
        if (e >= EN) continue;
        const int gi = ey0 + ei[k], gj = ex0 + ej[k];
        if (gi < y0 || gi >= y0 + th || gj < x0 || gj >= x0 + tw) continue;
        const int64_t o = (int64_t)gi * ld + gj;
#pragma unroll
        for (int c = 0; c < NX; ++c) {
            L.x_out[c][o] = x[c][k];
            L.xb_out[c][o] = xbo[c][k];
        }
#pragma unroll
        for (int c = 0; c < NY; ++c) L.y_out[c][o] = yow[c][k];
        L.s_out[o] = th_s[k];
    }
}

__device__ __forceinline__ int xcd_tile_a(int b, int nb) {
    const int per = nb >> 3;   // host pads the grid to a multiple of 8
    return (b & 7) * per + (b >> 3);
}

template <bool HAS_W, int NT, int PPT>
__global__ __launch_bounds__(NT) void alg1_tb_kernel(PdrTbArgs a) {
    __shared__ Alg1Lds<HAS_W, NT, PPT> S;
    const int t = xcd_tile_a(blockIdx.x, gridDim.x);
    if (t >= a.ntiles) return;
    const int ty = t / a.ntx, tx = t - ty * a.ntx;
    const int y0 = ty * a.th, x0 = tx * a.tw;
    alg1_tile<HAS_W, NT, PPT>(a, a.lvl, y0, x0, min(a.th, a.lvl.H - y0), min(a.tw, a.lvl.W - x0), S);
}

// Many levels (batched pairs): tile entries of a table in XCD order (as the pDR table kernel).
template <bool HAS_W, int NT, int PPT>
__global__ __launch_bounds__(NT) void alg1_tb_table_kernel(PdrTbArgs a) {
    __shared__ Alg1Lds<HAS_W, NT, PPT> S;
    const int per = (a.ntiles + 7) >> 3;
    const int x = blockIdx.x & 7, y = blockIdx.x >> 3;
    const int t = x * per + y;
    if (y >= per || t >= a.ntiles) return;
    const TbTile T = a.tiles[t];
    alg1_tile<HAS_W, NT, PPT>(a, a.levels[2 * T.level + a.dir], T.y0, T.x0, T.th, T.tw, S);
}

}  // namespace

template <bool HAS_W, int NT, int PPT>
static void launch_alg1_shape(const PdrTbArgs& a, int grid, hipStream_t s) {
    if (a.tiles) hipLaunchKernelGGL((alg1_tb_table_kernel<HAS_W, NT, PPT>), dim3(grid), dim3(NT), 0, s, a);
    else hipLaunchKernelGGL((alg1_tb_kernel<HAS_W, NT, PPT>), dim3(grid), dim3(NT), 0, s, a);
}

void launch_alg1_tb(const PdrTbArgs& a, bool has_w, int nt, hipStream_t s) {
    const int grid = (a.ntiles + 7) / 8 * 8;
    if (a.ntiles < 1) return;
    if (nt == 3074 || nt == 2050) {            // wave-row tiles, one cell per lane (3074 without w only)
        launch_alg1_rows(a, has_w, nt, s);
        return;
    }
    if (nt == 512) {
        if (has_w) launch_alg1_shape<true, 512, kPdrPptW>(a, grid, s);
        else launch_alg1_shape<false, 512, kPdrPpt>(a, grid, s);
    } else {
        if (has_w) launch_alg1_shape<true, 1024, kPdrPptW>(a, grid, s);
        else launch_alg1_shape<false, 1024, kPdrPpt>(a, grid, s);
    }
}

}  // namespace flowmi
