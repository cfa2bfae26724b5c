// Temporally blocked ALG1 iterations (the first-order primal-dual method Sec. 4 compares against, on
// eq:primal-dual:optical:o) on tiles one wavefront wide: the register-resident form of the ALG1 tiles.
//
// The extended region (output tile plus a halo of K rows / columns on every side, clipped to the
// image) is at most 64 columns wide and NW * R rows high.  Wavefront w holds rows w R .. w R + R - 1
// of it, lane l column l, one cell per lane and row, with every field of its cells in registers for
// the whole launch.  The discrete operators of Sec. 2.2 find their neighbours without memory: left /
// right in the adjacent lane (a whole-wavefront DPP shift), up / down in the thread's neighbouring
// row, and across the boundary between two wavefronts in LDS, which holds one row of X bar (each
// wavefront's top row, read by the wavefront above for its forward difference) and one row of the
// dual's y components (each wavefront's bottom row, read by the wavefront below for its divergence).
//
// The iteration is the one of the general ALG1 tiles, with the same operations in the same order, so
// the two give bitwise the same iterates:  [Y] y+ = P(y + tau grad X bar);  barrier;  [X] X+ = the
// resolvent at X + sigma div y+, X bar+ = 2 X+ - X;  barrier.  A neighbour outside the extended
// region reads zero or an unrelated finite value, which only changes halo cells the halo accounts
// for.  After iteration m of the launch only the region shrunk by m rows on each side with a halo
// can still reach the output tile, so the rows outside that band skip the iteration.
#include "rows_dev.hpp"

namespace flowmi {

namespace {

template <bool HAS_W, int NW>
struct Alg1RowLds {
    static constexpr int NX = HAS_W ? 3 : 2;
    // [c][w + 1][lane]: component c of X bar in wavefront w's top row / of the y components (q1y,
    // q2y, p_y) in its bottom row; entries 0 and NW + 1 stand for rows beyond the work-group, zero
    float xbtop[NX][NW + 2][64];
    float ybot[NX][NW + 2][64];
};

// IN: the extended region holds no image edge, so every neighbour-exists coefficient is 1 and its
// products drop out (the same arithmetic: a product by 1 is exact)
template <bool HAS_W, int NW, int R, bool IN>
__device__ __forceinline__ void alg1_rows(const PdrTbArgs& a, const PdrTbLevel& L, int y0, int x0, int th, int tw,
                                          Alg1RowLds<HAS_W, NW>& S) {
    constexpr int NX = HAS_W ? 3 : 2, NY = 2 * NX;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int H = L.H, W = L.W;
    const int64_t ld = L.ld;
    const int K = a.K;
    const int hk = alg1_halo(K);
    const int ey0 = max(y0 - hk, 0), ex0 = max(x0 - hk, 0);
    const int ey1 = min(y0 + th + hk, H), ex1 = min(x0 + tw + hk, W);
    const int EW = ex1 - ex0, EH = ey1 - ey0;          // at most 64 and NW R (the planners' bound)
    const float sigma = a.sigma, tau = a.tau, lam = a.lam, beta = a.beta;
    const float sl = sigma * lam, inv_sigma = 1.f / sigma;
    const int gj = ex0 + lane;
    const float fx = IN || gj < W - 1 ? 1.f : 0.f, fl = IN || gj > 0 ? 1.f : 0.f;
    const float cx = IN ? tau : fx * tau;
    const int shr_top = ey0 > 0, shr_bot = ey1 < H;

    // components: X / X bar (u, v, w); y (q1x, q1y, q2x, q2y, p_x, p_y)
    float x[NX][R], xb[NX][R], y[NY][R], Ix[R], Iy[R], It[R], u0[R], v0[R], th_s[R];
    float fy[R], fu[R], cy[R];                          // wavefront-uniform
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = wv * R + k, gi = ey0 + r;
        fy[k] = IN || gi < H - 1 ? 1.f : 0.f;
        fu[k] = IN || gi > 0 ? 1.f : 0.f;
        cy[k] = IN ? tau : fy[k] * tau;
#pragma unroll
        for (int c = 0; c < NX; ++c) x[c][k] = xb[c][k] = 0.f;
#pragma unroll
        for (int c = 0; c < NY; ++c) y[c][k] = 0.f;
        Ix[k] = Iy[k] = It[k] = u0[k] = v0[k] = th_s[k] = 0.f;
        if (r < EH && lane < EW) {
            const int64_t o = (int64_t)gi * ld + gj;
#pragma unroll
            for (int c = 0; c < NX; ++c) {
                x[c][k] = gload(L.x_in[c], o);
                xb[c][k] = gload(L.xb_in[c], o);
            }
#pragma unroll
            for (int c = 0; c < NY; ++c) y[c][k] = gload(L.y_in[c], o);
            Ix[k] = gload(L.Ix, o);
            Iy[k] = gload(L.Iy, o);
            It[k] = gload(L.It, o);
            u0[k] = gload(L.u0, o);
            v0[k] = gload(L.v0, o);
        }
    }
#pragma unroll
    for (int c = 0; c < NX; ++c) {
        S.xbtop[c][wv + 1][lane] = xb[c][0];
        S.ybot[c][wv + 1][lane] = y[2 * c + 1][R - 1];
    }
    if (wv == 0) {
#pragma unroll
        for (int c = 0; c < NX; ++c) {
            S.xbtop[c][0][lane] = S.xbtop[c][NW + 1][lane] = 0.f;
            S.ybot[c][0][lane] = S.ybot[c][NW + 1][lane] = 0.f;
        }
    }
    __syncthreads();

    // [Y] at row k: dual ascent from the forward differences of X bar, projected (joint q ball, p ball)
    auto phase_y = [&](int k) {
        float xr[NX], xd[NX];
#pragma unroll
        for (int c = 0; c < NX; ++c) {
            xr[c] = from_right(xb[c][k]);
            xd[c] = k + 1 < R ? xb[c][k + 1 < R ? k + 1 : k] : S.xbtop[c][wv + 2][lane];
        }
        const float a1x = fmaf(cx, xr[0] - xb[0][k], y[0][k]);
        const float a1y = fmaf(cy[k], xd[0] - xb[0][k], y[1][k]);
        const float a2x = fmaf(cx, xr[1] - xb[1][k], y[2][k]);
        const float a2y = fmaf(cy[k], xd[1] - xb[1][k], y[3][k]);
        // sums of products as explicit FMA chains: every ALG1 tile kernel rounds them alike
        const float nq = fmaf(a2y, a2y, fmaf(a2x, a2x, fmaf(a1y, a1y, a1x * a1x)));
        const float sq = fminf(1.f, __builtin_amdgcn_rsqf(nq));
        y[0][k] = a1x * sq;
        y[1][k] = a1y * sq;
        y[2][k] = a2x * sq;
        y[3][k] = a2y * sq;
        if constexpr (HAS_W) {
            const float bx = fmaf(cx, xr[2] - xb[2][k], y[4][k]);
            const float by = fmaf(cy[k], xd[2] - xb[2][k], y[5][k]);
            const float np2 = fmaf(by, by, bx * bx);
            const float sp = fminf(1.f, __builtin_amdgcn_rsqf(np2));
            y[4][k] = bx * sp;
            y[5][k] = by * sp;
        }
        if (k == R - 1) {
#pragma unroll
            for (int c = 0; c < NX; ++c) S.ybot[c][wv + 1][lane] = y[2 * c + 1][R - 1];
        }
    };
    // [X] at row k: primal proximal descent X+ = J(X + sigma div y+), extrapolation X bar+ = 2 X+ - X
    auto phase_x = [&](int k) {
        float dv[NX];
#pragma unroll
        for (int c = 0; c < NX; ++c) {
            // [j < W-1] y_x - [j > 0] y_x(left) + [i < H-1] y_y - [i > 0] y_y(up)
            const float yl = from_left(y[2 * c][k]);
            const float yu = k > 0 ? y[2 * c + 1][k > 0 ? k - 1 : 0] : S.ybot[c][wv][lane];
            float d = fmaf(fx, y[2 * c][k], -(fl * yl));
            d = fmaf(fy[k], y[2 * c + 1][k], d);
            dv[c] = fmaf(-fu[k], yu, d);
        }
        const float ut = x[0][k] + sigma * dv[0];
        const float vt = x[1][k] + sigma * dv[1];
        float wt = 0.f;
        if constexpr (HAS_W) wt = x[2][k] + sigma * dv[NX - 1];
        const float e2 = fmaf(Iy[k], Iy[k], fmaf(Ix[k], Ix[k], beta * beta));
        const float rho = fmaf(Iy[k], vt - v0[k], fmaf(Ix[k], ut - u0[k], fmaf(beta, wt, It[k])));
        // eq:resolvent with step sigma (as the general ALG1 tiles)
        float step = 0.f, theta = 0.f;
        if (e2 > 0.f) {
            step = __builtin_amdgcn_fmed3f(-rho * __builtin_amdgcn_rcpf(e2), -sl, sl);
            theta = -step * inv_sigma;
        }
        const float un = ut + step * Ix[k], vn = vt + step * Iy[k];
        xb[0][k] = 2.f * un - x[0][k];
        xb[1][k] = 2.f * vn - x[1][k];
        x[0][k] = un;
        x[1][k] = vn;
        if constexpr (HAS_W) {
            const float wn = wt + step * beta;
            xb[2][k] = 2.f * wn - x[2][k];
            x[2][k] = wn;
        }
        th_s[k] = theta;
        if (k == 0) {
#pragma unroll
            for (int c = 0; c < NX; ++c) S.xbtop[c][wv + 1][lane] = xb[c][0];
        }
    };

    for (int it = 0; it < K; ++it) {
        // rows that can still reach the output tile; the bounds are re-read as scalars in each phase
        // (a row condition kept across a barrier would live as a lane mask)
        const int lo = shr_top * it, hi = EH - shr_bot * it;
        {
            const int lo_s = __builtin_amdgcn_readfirstlane(lo), hi_s = __builtin_amdgcn_readfirstlane(hi);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int r = wv * R + k;
                if (r >= lo_s && r < hi_s) phase_y(k);
            }
        }
        __syncthreads();
        {
            const int lo_s = __builtin_amdgcn_readfirstlane(lo), hi_s = __builtin_amdgcn_readfirstlane(hi);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int r = wv * R + k;
                if (r >= lo_s && r < hi_s) phase_x(k);
            }
        }
        __syncthreads();
    }

    // write the output tile
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = wv * R + k, gi = ey0 + r;
        if (r >= EH || gi < y0 || gi >= y0 + th) continue;
        if (lane >= EW || gj < x0 || gj >= x0 + tw) continue;
        const int64_t o = (int64_t)gi * ld + gj;
#pragma unroll
        for (int c = 0; c < NX; ++c) {
            gstore(L.x_out[c], o, x[c][k]);
            gstore(L.xb_out[c], o, xb[c][k]);
        }
#pragma unroll
        for (int c = 0; c < NY; ++c) gstore(L.y_out[c], o, y[c][k]);
        gstore(L.s_out, o, th_s[k]);
    }
}

template <bool HAS_W, int NW, int R>
__device__ __forceinline__ void alg1_rows_any(const PdrTbArgs& a, const PdrTbLevel& L, int y0, int x0, int th, int tw,
                                              Alg1RowLds<HAS_W, NW>& S) {
    const int hk = alg1_halo(a.K);
    if (y0 - hk > 0 && x0 - hk > 0 && y0 + th + hk < L.H && x0 + tw + hk < L.W)
        alg1_rows<HAS_W, NW, R, true>(a, L, y0, x0, th, tw, S);
    else
        alg1_rows<HAS_W, NW, R, false>(a, L, y0, x0, th, tw, S);
}

__device__ __forceinline__ int xcd_tile_ar(int b, int nb) {
    const int per = nb >> 3;   // host pads the grid to a multiple of 8
    return (b & 7) * per + (b >> 3);
}

template <bool HAS_W, int NW, int R>
__global__ __launch_bounds__(NW * 64, 8) void alg1_rows_kernel(PdrTbArgs a) {
    __shared__ Alg1RowLds<HAS_W, NW> S;
    const int t = xcd_tile_ar(blockIdx.x, gridDim.x);
    if (t >= a.ntiles) return;
    const int ty = t / a.ntx, tx = t - ty * a.ntx;
    const int y0 = ty * a.th, x0 = tx * a.tw;
    alg1_rows_any<HAS_W, NW, R>(a, a.lvl, y0, x0, min(a.th, a.lvl.H - y0), min(a.tw, a.lvl.W - x0), S);
}

// Many levels (batched pairs): tile entries of a table in XCD order
template <bool HAS_W, int NW, int R>
__global__ __launch_bounds__(NW * 64, 8) void alg1_rows_table_kernel(PdrTbArgs a) {
    __shared__ Alg1RowLds<HAS_W, NW> S;
    const int per = (a.ntiles + 7) >> 3;
    const int x = blockIdx.x & 7, y = blockIdx.x >> 3;
    const int t = x * per + y;
    if (y >= per || t >= a.ntiles) return;
    const TbTile T = a.tiles[t];
    const PdrTbLevel L = pdr_level_scalar(a.levels + (2 * T.level + a.dir));
    alg1_rows_any<HAS_W, NW, R>(a, L, T.y0, T.x0, T.th, T.tw, S);
}

template <bool HAS_W, int NW, int R>
void launch_alg1_rows_shape(const PdrTbArgs& a, int grid, hipStream_t s) {
    if (a.tiles) hipLaunchKernelGGL((alg1_rows_table_kernel<HAS_W, NW, R>), dim3(grid), dim3(NW * 64), 0, s, a);
    else hipLaunchKernelGGL((alg1_rows_kernel<HAS_W, NW, R>), dim3(grid), dim3(NW * 64), 0, s, a);
}

}  // namespace

// 3074: 64 x 48 cells (three rows per lane, beta = 0); 2050: 64 x 32 (two rows per lane)
void launch_alg1_rows(const PdrTbArgs& a, bool has_w, int nt, hipStream_t s) {
    if (a.ntiles < 1) return;
    const int grid = (a.ntiles + 7) / 8 * 8;
    if (nt == 3074 && !has_w) launch_alg1_rows_shape<false, 16, 3>(a, grid, s);
    else if (has_w) launch_alg1_rows_shape<true, 16, 2>(a, grid, s);
    else launch_alg1_rows_shape<false, 16, 2>(a, grid, s);
}

}  // namespace flowmi
