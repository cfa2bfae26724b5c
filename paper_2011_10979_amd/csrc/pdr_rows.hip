// Temporally blocked pDR iterations (Sec. 3.1.2, tag pDR, with the symmetric red-black Gauss-Seidel
// preconditioner of eq. neumann:boudary) on tiles one wavefront of cell pairs wide: the
// register-resident form of the pDR tiles.
//
// The extended region (output tile plus the halo of (2n + 1) K cells above and to the left and one
// more below and to the right, clipped to the image) is at most 128 columns wide and NW R rows
// high.  Wavefront w holds rows w R .. w R + R - 1; lane l holds the cells of columns 2l and 2l + 1
// of each of its rows, which always have opposite colours, so a half sweep updates one cell in
// every lane.  Every field of the thread's cells stays in registers for the whole launch, and a
// cell's neighbours are found without memory: the horizontal ones in the lane's other cell or in
// the adjacent lane (a whole-wavefront DPP shift), the vertical ones in the thread's neighbouring
// rows, and only across the boundary between two wavefronts in LDS (each wavefront's top and
// bottom row of X, and its bottom row of the y components of y bar).  A cell's vertical neighbours
// have the same position in the pair and the other colour, so the colour that a half sweep writes
// is never read by it.
//
// The iteration is the one of the general pDR tiles, with the same operations in the same order,
// so the two give bitwise the same iterates: [b + R] | ([B] | [R]) x n | [D] with a barrier after
// each phase.  A neighbour outside the extended region reads zero or an unrelated finite value,
// which only changes halo cells the halo accounts for.
#include <type_traits>

#include "rows_dev.hpp"

namespace flowmi {

namespace {

template <bool HAS_W, int NW, int R>
struct PdrRowLds {
    static constexpr int NX = HAS_W ? 3 : 2;
    // I_t, u0, v0 of every cell ([field][row][cell of the pair][lane]): read once per iteration, by
    // the resolvent, so they wait in LDS rather than in registers
    float lin[3][NW * R][2][64];
    // [component][cell of the pair][w + 1][lane]: wavefront w's top / bottom row of X and the y
    // components (q1y, q2y[, p_y]) of its bottom row; entries 0 and NW + 1 stand for the rows beyond
    // the work-group and stay zero
    float xtop[NX][2][NW + 2][64];
    float xbot[NX][2][NW + 2][64];
    float ybot[NX][2][NW + 2][64];
};

template <int C>
using cell_t = std::integral_constant<int, C>;

template <bool HAS_W, int NW, int R>
__device__ __forceinline__ void pdr_rows(const PdrTbArgs& a, const PdrTbLevel& L, int y0, int x0, int th, int tw,
                                         PdrRowLds<HAS_W, NW, R>& S) {
    constexpr int NX = HAS_W ? 3 : 2, NY = 2 * NX;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int H = L.H, W = L.W;
    const int64_t ld = L.ld;
    const int K = a.K, n = a.sweeps;
    const int hlu = pdr_halo_lo(n, K), hrd = pdr_halo_hi(n, K);
    const int ey0 = max(y0 - hlu, 0), ex0 = max(x0 - hlu, 0);
    const int ey1 = min(y0 + th + hrd, H), ex1 = min(x0 + tw + hrd, W);
    const int EW = ex1 - ex0, EH = ey1 - ey0;          // at most 128 and NW R (the planners' bound)
    const float sigma = a.sigma, tau = a.tau, stt = a.stt, lam = a.lam, beta = a.beta;
    const float sl = sigma * lam, inv_sigma = 1.f / sigma;

    float fl[2], fr[2];                                 // the left / right neighbour exists in the image
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int gj = ex0 + 2 * lane + c;
        fl[c] = gj > 0 ? 1.f : 0.f;
        fr[c] = gj < W - 1 ? 1.f : 0.f;
    }
    float x[NX][R][2], xb[NX][R][2], y[NY][R][2], bb[NX][R][2];
    float Ix[R][2], Iy[R][2], rden[R][2];
    float fu[R], fd[R];                                 // wavefront-uniform
    int par[R];                                         // parity of the row's first column: its red cell
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = wv * R + k, gi = ey0 + r;
        fu[k] = gi > 0 ? 1.f : 0.f;
        fd[k] = gi < H - 1 ? 1.f : 0.f;
        par[k] = (gi + ex0) & 1;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            rden[k][c] = 1.f / (1.f + stt * (((fl[c] + fr[c]) + fu[k]) + fd[k]));
#pragma unroll
            for (int f = 0; f < NX; ++f) x[f][k][c] = xb[f][k][c] = bb[f][k][c] = 0.f;
#pragma unroll
            for (int f = 0; f < NY; ++f) y[f][k][c] = 0.f;
            Ix[k][c] = Iy[k][c] = 0.f;
            float lt = 0.f, lu = 0.f, lv = 0.f;
            if (r < EH && 2 * lane + c < EW) {
                const int64_t o = (int64_t)gi * ld + ex0 + 2 * lane + c;
#pragma unroll
                for (int f = 0; f < NX; ++f) {
                    x[f][k][c] = gload(L.x_in[f], o);
                    xb[f][k][c] = gload(L.xb_in[f], o);
                }
#pragma unroll
                for (int f = 0; f < NY; ++f) y[f][k][c] = gload(L.y_in[f], o);
                Ix[k][c] = gload(L.Ix, o);
                Iy[k][c] = gload(L.Iy, o);
                lt = gload(L.It, o);
                lu = gload(L.u0, o);
                lv = gload(L.v0, o);
            }
            S.lin[0][r][c][lane] = lt;
            S.lin[1][r][c][lane] = lu;
            S.lin[2][r][c][lane] = lv;
        }
    }
#pragma unroll
    for (int f = 0; f < NX; ++f)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            S.xtop[f][c][wv + 1][lane] = x[f][0][c];
            S.xbot[f][c][wv + 1][lane] = x[f][R - 1][c];
            S.ybot[f][c][wv + 1][lane] = y[2 * f + 1][R - 1][c];
            if (wv == 0) {
                S.xtop[f][c][0][lane] = S.xtop[f][c][NW + 1][lane] = 0.f;
                S.xbot[f][c][0][lane] = S.xbot[f][c][NW + 1][lane] = 0.f;
                S.ybot[f][c][0][lane] = S.ybot[f][c][NW + 1][lane] = 0.f;
            }
        }
    __syncthreads();

    // neighbours of cell c of row k in component f of X: left, right, up, down
    auto xl = [&](int f, int k, auto cc) {
        constexpr int c = decltype(cc)::value;
        return c == 1 ? x[f][k][0] : from_left(x[f][k][1]);
    };
    auto xr = [&](int f, int k, auto cc) {
        constexpr int c = decltype(cc)::value;
        return c == 0 ? x[f][k][1] : from_right(x[f][k][0]);
    };
    auto xu = [&](int f, int k, auto cc) {
        constexpr int c = decltype(cc)::value;
        return k > 0 ? x[f][k > 0 ? k - 1 : 0][c] : S.xbot[f][c][wv][lane];
    };
    auto xd = [&](int f, int k, auto cc) {
        constexpr int c = decltype(cc)::value;
        return k + 1 < R ? x[f][k + 1 < R ? k + 1 : k][c] : S.xtop[f][c][wv + 2][lane];
    };

    // one Gauss-Seidel update of cell c of row k: x = (b + st sum of in-image neighbours) / (1 + st #),
    // evaluated as x + ((b - x) + st sum of (neighbour - x)) / (1 + st #), summed left, right, up,
    // down (the flows cancel in the differences before any rounding)
    auto update = [&](int k, auto cc) {
        constexpr int c = decltype(cc)::value;
        float nl[NX], nr[NX], nu[NX], nd[NX];
#pragma unroll
        for (int f = 0; f < NX; ++f) {
            nl[f] = xl(f, k, cc);
            nr[f] = xr(f, k, cc);
            nu[f] = xu(f, k, cc);
            nd[f] = xd(f, k, cc);
        }
#pragma unroll
        for (int f = 0; f < NX; ++f) {
            const float xo = x[f][k][c];
            float sm = fl[c] * (nl[f] - xo);
            sm = fmaf(fr[c], nr[f] - xo, sm);
            sm = fmaf(fu[k], nu[f] - xo, sm);
            sm = fmaf(fd[k], nd[f] - xo, sm);
            x[f][k][c] = fmaf(fmaf(stt, sm, bb[f][k][c] - xo), rden[k][c], xo);
        }
        if (k == 0) {
#pragma unroll
            for (int f = 0; f < NX; ++f) S.xtop[f][c][wv + 1][lane] = x[f][0][c];
        }
        if (k == R - 1) {
#pragma unroll
            for (int f = 0; f < NX; ++f) S.xbot[f][c][wv + 1][lane] = x[f][R - 1][c];
        }
    };
    // half sweep over colour col (0 red, 1 black): in row k that is cell par[k] ^ col of each pair
    auto half_sweep = [&](int col, int lo, int hi) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (wv * R + k < lo || wv * R + k >= hi) continue;
            if ((par[k] ^ col) == 0) update(k, cell_t<0>{});
            else update(k, cell_t<1>{});
        }
    };
    // b = X bar + sigma div y bar for cell c of row k:
    // [j < W-1] y_x - [j > 0] y_x left + [i < H-1] y_y - [i > 0] y_y up
    auto rhs = [&](int k, auto cc) {
        constexpr int c = decltype(cc)::value;
#pragma unroll
        for (int f = 0; f < NX; ++f) {
            const float yox = y[2 * f][k][c], yoy = y[2 * f + 1][k][c];
            const float ynx = c == 1 ? y[2 * f][k][0] : from_left(y[2 * f][k][1]);
            const float yny = k > 0 ? y[2 * f + 1][k > 0 ? k - 1 : 0][c] : S.ybot[f][c][wv][lane];
            float d = fr[c] * yox;
            d = fmaf(-fl[c], ynx, d);
            d = fmaf(fd[k], yoy, d);
            d = fmaf(-fu[k], yny, d);
            bb[f][k][c] = fmaf(sigma, d, xb[f][k][c]);
        }
    };
    // [D] for cell c of row k: resolvent at X~ = 2 X+ - X bar, dual update from grad X+
    auto dual = [&](int k, auto cc, bool last) {
        constexpr int c = decltype(cc)::value;
        const int r = wv * R + k;
        float xo[NX], gx[NX], gy[NX];
#pragma unroll
        for (int f = 0; f < NX; ++f) {
            xo[f] = x[f][k][c];
            gx[f] = fr[c] * (xr(f, k, cc) - xo[f]);
            gy[f] = fd[k] * (xd(f, k, cc) - xo[f]);
        }
        const float u = xo[0], v = xo[1];
        const float ut = 2.f * u - xb[0][k][c], vt = 2.f * v - xb[1][k][c];
        float w = 0.f, wt = 0.f;
        if constexpr (HAS_W) { w = xo[2]; wt = 2.f * w - xb[2][k][c]; }
        const float ix = Ix[k][c], iy = Iy[k][c];
        // sums of products as explicit FMA chains: every pDR tile kernel rounds them alike
        const float e2 = fmaf(iy, iy, fmaf(ix, ix, beta * beta));
        const float rho = fmaf(iy, vt - S.lin[2][r][c][lane], fmaf(ix, ut - S.lin[1][r][c][lane],
                                                                  fmaf(beta, wt, S.lin[0][r][c][lane])));
        // eq:resolvent: the step along e is -rho / |e|^2 clamped to [-sigma lam, sigma lam], and
        // Theta = -step / sigma (both 0 where e = 0); 1 / |e|^2 is the hardware reciprocal (within
        // 1 ulp), as in every pDR kernel
        float step = 0.f, theta = 0.f;
        if (e2 > 0.f) {
            step = __builtin_amdgcn_fmed3f(-rho * __builtin_amdgcn_rcpf(e2), -sl, sl);
            theta = -step * inv_sigma;
        }
        xb[0][k][c] = fmaf(step, ix, u);
        xb[1][k][c] = fmaf(step, iy, v);
        if constexpr (HAS_W) xb[2][k][c] = fmaf(step, beta, w);
        if (last) {                                     // Theta of an output cell: the data dual for the gap
            const int gi = ey0 + r, j = 2 * lane + c, gj = ex0 + j;
            if (gi >= y0 && gi < y0 + th && j < EW && gj >= x0 && gj < x0 + tw)
                gstore(L.s_out, (int64_t)gi * ld + gj, theta);
        }
        const float t2 = 2.f * tau;
        const float a1x = fmaf(t2, gx[0], y[0][k][c]), a1y = fmaf(t2, gy[0], y[1][k][c]);
        const float a2x = fmaf(t2, gx[1], y[2][k][c]), a2y = fmaf(t2, gy[1], y[3][k][c]);
        const float nq = fmaf(a2y, a2y, fmaf(a2x, a2x, fmaf(a1y, a1y, a1x * a1x)));
        const float sq = fminf(1.f, __builtin_amdgcn_rsqf(nq));
        y[0][k][c] = fmaf(a1x, sq, -(tau * gx[0]));
        y[1][k][c] = fmaf(a1y, sq, -(tau * gy[0]));
        y[2][k][c] = fmaf(a2x, sq, -(tau * gx[1]));
        y[3][k][c] = fmaf(a2y, sq, -(tau * gy[1]));
        if constexpr (HAS_W) {
            const float bx = fmaf(t2, gx[2], y[4][k][c]), by = fmaf(t2, gy[2], y[5][k][c]);
            const float np2 = fmaf(by, by, bx * bx);
            const float sp = fminf(1.f, __builtin_amdgcn_rsqf(np2));
            y[4][k][c] = fmaf(bx, sp, -(tau * gx[2]));
            y[5][k][c] = fmaf(by, sp, -(tau * gy[2]));
        }
        if (k == R - 1) {
#pragma unroll
            for (int f = 0; f < NX; ++f) S.ybot[f][c][wv + 1][lane] = y[2 * f + 1][R - 1][c];
        }
    };

    // Shrinking band: at iteration it only the rows of the region shrunk by (2n + 1) it + 1 rows on
    // each side with a halo can still reach the output tile; the others skip every phase and keep
    // their state (the halo accounts for what their neighbours then read)
    const int shr_top = ey0 > 0, shr_bot = ey1 < H;
    for (int it = 0; it < K; ++it) {
        const int lo = shr_top * ((2 * n + 1) * it + 1), hi = EH - shr_bot * ((2 * n + 1) * it + 1);
        // [b + R]
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (wv * R + k < lo || wv * R + k >= hi) continue;
            rhs(k, cell_t<0>{});
            rhs(k, cell_t<1>{});
        }
        half_sweep(0, lo, hi);
        for (int sw = 0; sw < n; ++sw) {
            __syncthreads();
            half_sweep(1, lo, hi);
            __syncthreads();
            half_sweep(0, lo, hi);
        }
        __syncthreads();
        // [D]
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (wv * R + k < lo || wv * R + k >= hi) continue;
            dual(k, cell_t<0>{}, it + 1 == K);
            dual(k, cell_t<1>{}, it + 1 == K);
        }
        __syncthreads();
    }

    // write the output tile
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = wv * R + k, gi = ey0 + r;
        if (r >= EH || gi < y0 || gi >= y0 + th) continue;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int j = 2 * lane + c, gj = ex0 + j;
            if (j >= EW || gj < x0 || gj >= x0 + tw) continue;
            const int64_t o = (int64_t)gi * ld + gj;
#pragma unroll
            for (int f = 0; f < NX; ++f) {
                gstore(L.x_out[f], o, x[f][k][c]);
                gstore(L.xb_out[f], o, xb[f][k][c]);
            }
#pragma unroll
            for (int f = 0; f < NY; ++f) gstore(L.y_out[f], o, y[f][k][c]);
        }
    }
}

__device__ __forceinline__ int xcd_tile_pr(int b, int nb) {
    const int per = nb >> 3;   // host pads the grid to a multiple of 8
    return (b & 7) * per + (b >> 3);
}

template <bool HAS_W, int NW, int R>
__global__ __launch_bounds__(NW * 64) void pdr_rows_kernel(PdrTbArgs a) {
    __shared__ PdrRowLds<HAS_W, NW, R> S;
    const int t = xcd_tile_pr(blockIdx.x, gridDim.x);
    if (t >= a.ntiles) return;
    const int ty = t / a.ntx, tx = t - ty * a.ntx;
    const int y0 = ty * a.th, x0 = tx * a.tw;
    pdr_rows<HAS_W, NW, R>(a, a.lvl, y0, x0, min(a.th, a.lvl.H - y0), min(a.tw, a.lvl.W - x0), S);
}

// Many levels (batched pairs): tile entries of a table in XCD order
template <bool HAS_W, int NW, int R>
__global__ __launch_bounds__(NW * 64) void pdr_rows_table_kernel(PdrTbArgs a) {
    __shared__ PdrRowLds<HAS_W, NW, R> S;
    const int per = (a.ntiles + 7) >> 3;
    const int x = blockIdx.x & 7, y = blockIdx.x >> 3;
    const int t = x * per + y;
    if (y >= per || t >= a.ntiles) return;
    const TbTile T = a.tiles[t];
    pdr_rows<HAS_W, NW, R>(a, a.levels[2 * T.level + a.dir], T.y0, T.x0, T.th, T.tw, S);
}

template <bool HAS_W, int NW, int R>
void launch_rows_shape(const PdrTbArgs& a, int grid, hipStream_t s) {
    if (a.tiles) hipLaunchKernelGGL((pdr_rows_table_kernel<HAS_W, NW, R>), dim3(grid), dim3(NW * 64), 0, s, a);
    else hipLaunchKernelGGL((pdr_rows_kernel<HAS_W, NW, R>), dim3(grid), dim3(NW * 64), 0, s, a);
}

// The same iteration on regions of at most 64 columns, one cell per lane and row: lanes alternate
// in colour, so a half sweep computes every lane and keeps the update only in the lanes of its
// colour.  Half the lanes idle in the sweeps, but 12 values per cell in registers (I_t, u0, v0 and
// I_x in LDS, read once per iteration) let three rows per lane fit 64 VGPRs, two 1024-thread
// work-groups per CU.
template <bool HAS_W, int NW, int R>
struct PdrRow1Lds {
    static constexpr int NX = HAS_W ? 3 : 2;
    float lin[4][NW * R][64];                           // I_t, u0, v0, I_x
    float xtop[NX][NW + 2][64];                         // [w + 1]: wavefront w's top / bottom row of X
    float xbot[NX][NW + 2][64];
    float ybot[NX][NW + 2][64];                         // y components of wavefront w's bottom row
};

// IN: the extended region holds no image edge, so every neighbour-exists coefficient is 1 and its
// products drop out (the same arithmetic: a product by 1 is exact)
template <bool HAS_W, int NW, int R, bool IN>
__device__ __forceinline__ void pdr_rows1(const PdrTbArgs& a, const PdrTbLevel& L, int y0, int x0, int th, int tw,
                                          PdrRow1Lds<HAS_W, NW, R>& S) {
    constexpr int NX = HAS_W ? 3 : 2, NY = 2 * NX;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int H = L.H, W = L.W;
    const int64_t ld = L.ld;
    const int K = a.K, n = a.sweeps;
    const int hlu = pdr_halo_lo(n, K), hrd = pdr_halo_hi(n, K);
    const int ey0 = max(y0 - hlu, 0), ex0 = max(x0 - hlu, 0);
    const int ey1 = min(y0 + th + hrd, H), ex1 = min(x0 + tw + hrd, W);
    const int EW = ex1 - ex0, EH = ey1 - ey0;          // at most 64 and NW R (the planners' bound)
    const float sigma = a.sigma, tau = a.tau, stt = a.stt, lam = a.lam, beta = a.beta;
    const float sl = sigma * lam, inv_sigma = 1.f / sigma;
    const int gj = ex0 + lane;
    const float fl = IN || gj > 0 ? 1.f : 0.f, fr = IN || gj < W - 1 ? 1.f : 0.f;

    float x[NX][R], xb[NX][R], y[NY][R], bb[NX][R], Iy[R], rden[R];
    float fu[R], fd[R];                                 // wavefront-uniform
    int par[R];                                         // colour of lane 0 of the row (0 red)
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = wv * R + k, gi = ey0 + r;
        fu[k] = IN || gi > 0 ? 1.f : 0.f;
        fd[k] = IN || gi < H - 1 ? 1.f : 0.f;
        par[k] = (gi + ex0) & 1;
        rden[k] = 1.f / (1.f + stt * (((fl + fr) + fu[k]) + fd[k]));
#pragma unroll
        for (int f = 0; f < NX; ++f) x[f][k] = xb[f][k] = bb[f][k] = 0.f;
#pragma unroll
        for (int f = 0; f < NY; ++f) y[f][k] = 0.f;
        Iy[k] = 0.f;
        float lt = 0.f, lu = 0.f, lv = 0.f, lx = 0.f;
        if (r < EH && lane < EW) {
            const int64_t o = (int64_t)gi * ld + gj;
#pragma unroll
            for (int f = 0; f < NX; ++f) {
                x[f][k] = gload(L.x_in[f], o);
                xb[f][k] = gload(L.xb_in[f], o);
            }
#pragma unroll
            for (int f = 0; f < NY; ++f) y[f][k] = gload(L.y_in[f], o);
            lx = gload(L.Ix, o);
            Iy[k] = gload(L.Iy, o);
            lt = gload(L.It, o);
            lu = gload(L.u0, o);
            lv = gload(L.v0, o);
        }
        S.lin[0][r][lane] = lt;
        S.lin[1][r][lane] = lu;
        S.lin[2][r][lane] = lv;
        S.lin[3][r][lane] = lx;
    }
#pragma unroll
    for (int f = 0; f < NX; ++f) {
        S.xtop[f][wv + 1][lane] = x[f][0];
        S.xbot[f][wv + 1][lane] = x[f][R - 1];
        S.ybot[f][wv + 1][lane] = y[2 * f + 1][R - 1];
        if (wv == 0) {
            S.xtop[f][0][lane] = S.xtop[f][NW + 1][lane] = 0.f;
            S.xbot[f][0][lane] = S.xbot[f][NW + 1][lane] = 0.f;
            S.ybot[f][0][lane] = S.ybot[f][NW + 1][lane] = 0.f;
        }
    }
    __syncthreads();

    auto xu = [&](int f, int k) { return k > 0 ? x[f][k > 0 ? k - 1 : 0] : S.xbot[f][wv][lane]; };
    auto xd = [&](int f, int k) { return k + 1 < R ? x[f][k + 1 < R ? k + 1 : k] : S.xtop[f][wv + 2][lane]; };
    // half sweep over colour col (0 red, 1 black): every lane computes the update of its cell, the
    // lanes of that colour keep it
    auto half_sweep = [&](int col, int lo_, int hi_) {
        // bounds re-read as scalars: a row condition kept across a barrier would live as a lane
        // mask and cost vector instructions per row
        const int lo = __builtin_amdgcn_readfirstlane(lo_), hi = __builtin_amdgcn_readfirstlane(hi_);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (wv * R + k < lo || wv * R + k >= hi) continue;
            const bool mine = ((par[k] + lane) & 1) == col;
            float nl[NX], nr[NX], nu[NX], nd[NX];
#pragma unroll
            for (int f = 0; f < NX; ++f) {
                nl[f] = from_left(x[f][k]);
                nr[f] = from_right(x[f][k]);
                nu[f] = xu(f, k);
                nd[f] = xd(f, k);
            }
#pragma unroll
            for (int f = 0; f < NX; ++f) {
                const float xo = x[f][k];
                float sm = fl * (nl[f] - xo);
                sm = fmaf(fr, nr[f] - xo, sm);
                sm = fmaf(fu[k], nu[f] - xo, sm);
                sm = fmaf(fd[k], nd[f] - xo, sm);
                const float upd = fmaf(fmaf(stt, sm, bb[f][k] - xo), rden[k], xo);
                x[f][k] = mine ? upd : xo;
            }
            if (k == 0) {
#pragma unroll
                for (int f = 0; f < NX; ++f) S.xtop[f][wv + 1][lane] = x[f][0];
            }
            if (k == R - 1) {
#pragma unroll
                for (int f = 0; f < NX; ++f) S.xbot[f][wv + 1][lane] = x[f][R - 1];
            }
        }
    };

    // Shrinking band: at iteration it only the rows of the region shrunk by (2n + 1) it + 1 rows on
    // each side with a halo can still reach the output tile; the others skip every phase and keep
    // their state (the halo accounts for what their neighbours then read)
    const int shr_top = ey0 > 0, shr_bot = ey1 < H;
    for (int it = 0; it < K; ++it) {
        const int lo = shr_top * ((2 * n + 1) * it + 1), hi = EH - shr_bot * ((2 * n + 1) * it + 1);
        // [b + R]: b = X bar + sigma div y bar
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (wv * R + k < lo || wv * R + k >= hi) continue;
#pragma unroll
            for (int f = 0; f < NX; ++f) {
                const float yox = y[2 * f][k], yoy = y[2 * f + 1][k];
                const float ynx = from_left(yox);
                const float yny = k > 0 ? y[2 * f + 1][k > 0 ? k - 1 : 0] : S.ybot[f][wv][lane];
                float d = fr * yox;
                d = fmaf(-fl, ynx, d);
                d = fmaf(fd[k], yoy, d);
                d = fmaf(-fu[k], yny, d);
                bb[f][k] = fmaf(sigma, d, xb[f][k]);
            }
        }
        half_sweep(0, lo, hi);
        for (int sw = 0; sw < n; ++sw) {
            __syncthreads();
            half_sweep(1, lo, hi);
            __syncthreads();
            half_sweep(0, lo, hi);
        }
        __syncthreads();
        // [D]: resolvent at X~ = 2 X+ - X bar, dual update from grad X+ (right / down neighbours)
        const int lo_d = __builtin_amdgcn_readfirstlane(lo), hi_d = __builtin_amdgcn_readfirstlane(hi);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int r = wv * R + k;
            if (r < lo_d || r >= hi_d) continue;
            float xo[NX], gx[NX], gy[NX];
#pragma unroll
            for (int f = 0; f < NX; ++f) {
                xo[f] = x[f][k];
                gx[f] = fr * (from_right(xo[f]) - xo[f]);
                gy[f] = fd[k] * (xd(f, k) - xo[f]);
            }
            const float u = xo[0], v = xo[1];
            const float ut = 2.f * u - xb[0][k], vt = 2.f * v - xb[1][k];
            float w = 0.f, wt = 0.f;
            if constexpr (HAS_W) { w = xo[2]; wt = 2.f * w - xb[2][k]; }
            const float ix = S.lin[3][r][lane], iy = Iy[k];
            const float e2 = fmaf(iy, iy, fmaf(ix, ix, beta * beta));
            const float rho = fmaf(iy, vt - S.lin[2][r][lane], fmaf(ix, ut - S.lin[1][r][lane],
                                                                    fmaf(beta, wt, S.lin[0][r][lane])));
            float step = 0.f, theta = 0.f;
            if (e2 > 0.f) {
                step = __builtin_amdgcn_fmed3f(-rho * __builtin_amdgcn_rcpf(e2), -sl, sl);
                theta = -step * inv_sigma;
            }
            xb[0][k] = fmaf(step, ix, u);
            xb[1][k] = fmaf(step, iy, v);
            if constexpr (HAS_W) xb[2][k] = fmaf(step, beta, w);
            if (it + 1 == K) {                          // Theta of an output cell: the data dual for the gap
                const int gi = ey0 + r;
                if (gi >= y0 && gi < y0 + th && lane < EW && gj >= x0 && gj < x0 + tw)
                    gstore(L.s_out, (int64_t)gi * ld + gj, theta);
            }
            const float t2 = 2.f * tau;
            const float a1x = fmaf(t2, gx[0], y[0][k]), a1y = fmaf(t2, gy[0], y[1][k]);
            const float a2x = fmaf(t2, gx[1], y[2][k]), a2y = fmaf(t2, gy[1], y[3][k]);
            const float nq = fmaf(a2y, a2y, fmaf(a2x, a2x, fmaf(a1y, a1y, a1x * a1x)));
            const float sq = fminf(1.f, __builtin_amdgcn_rsqf(nq));
            y[0][k] = fmaf(a1x, sq, -(tau * gx[0]));
            y[1][k] = fmaf(a1y, sq, -(tau * gy[0]));
            y[2][k] = fmaf(a2x, sq, -(tau * gx[1]));
            y[3][k] = fmaf(a2y, sq, -(tau * gy[1]));
            if constexpr (HAS_W) {
                const float bx = fmaf(t2, gx[2], y[4][k]), by = fmaf(t2, gy[2], y[5][k]);
                const float np2 = fmaf(by, by, bx * bx);
                const float sp = fminf(1.f, __builtin_amdgcn_rsqf(np2));
                y[4][k] = fmaf(bx, sp, -(tau * gx[2]));
                y[5][k] = fmaf(by, sp, -(tau * gy[2]));
            }
            if (k == R - 1) {
#pragma unroll
                for (int f = 0; f < NX; ++f) S.ybot[f][wv + 1][lane] = y[2 * f + 1][R - 1];
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
        for (int f = 0; f < NX; ++f) {
            gstore(L.x_out[f], o, x[f][k]);
            gstore(L.xb_out[f], o, xb[f][k]);
        }
#pragma unroll
        for (int f = 0; f < NY; ++f) gstore(L.y_out[f], o, y[f][k]);
    }
}

// the tile's extended region, as pdr_rows1 clips it, holds no image edge
template <bool HAS_W, int NW, int R>
__device__ __forceinline__ void pdr_rows1_any(const PdrTbArgs& a, const PdrTbLevel& L, int y0, int x0, int th, int tw,
                                              PdrRow1Lds<HAS_W, NW, R>& S) {
    const int hlu = pdr_halo_lo(a.sweeps, a.K), hrd = pdr_halo_hi(a.sweeps, a.K);
    if (y0 - hlu > 0 && x0 - hlu > 0 && y0 + th + hrd < L.H && x0 + tw + hrd < L.W)
        pdr_rows1<HAS_W, NW, R, true>(a, L, y0, x0, th, tw, S);
    else
        pdr_rows1<HAS_W, NW, R, false>(a, L, y0, x0, th, tw, S);
}

template <bool HAS_W, int NW, int R>
__global__ __launch_bounds__(NW * 64, 8) void pdr_rows1_kernel(PdrTbArgs a) {
    __shared__ PdrRow1Lds<HAS_W, NW, R> S;
    const int t = xcd_tile_pr(blockIdx.x, gridDim.x);
    if (t >= a.ntiles) return;
    const int ty = t / a.ntx, tx = t - ty * a.ntx;
    const int y0 = ty * a.th, x0 = tx * a.tw;
    pdr_rows1_any<HAS_W, NW, R>(a, a.lvl, y0, x0, min(a.th, a.lvl.H - y0), min(a.tw, a.lvl.W - x0), S);
}

template <bool HAS_W, int NW, int R>
__global__ __launch_bounds__(NW * 64, 8) void pdr_rows1_table_kernel(PdrTbArgs a) {
    __shared__ PdrRow1Lds<HAS_W, NW, R> S;
    const int per = (a.ntiles + 7) >> 3;
    const int x = blockIdx.x & 7, y = blockIdx.x >> 3;
    const int t = x * per + y;
    if (y >= per || t >= a.ntiles) return;
    const TbTile T = a.tiles[t];
    const PdrTbLevel L = pdr_level_scalar(a.levels + (2 * T.level + a.dir));
    pdr_rows1_any<HAS_W, NW, R>(a, L, T.y0, T.x0, T.th, T.tw, S);
}

template <bool HAS_W, int NW, int R>
void launch_rows1_shape(const PdrTbArgs& a, int grid, hipStream_t s) {
    if (a.tiles) hipLaunchKernelGGL((pdr_rows1_table_kernel<HAS_W, NW, R>), dim3(grid), dim3(NW * 64), 0, s, a);
    else hipLaunchKernelGGL((pdr_rows1_kernel<HAS_W, NW, R>), dim3(grid), dim3(NW * 64), 0, s, a);
}

}  // namespace

void launch_pdr_rows(const PdrTbArgs& a, bool has_w, int nt, hipStream_t s) {
    const int grid = (a.ntiles + 7) / 8 * 8;
    if (a.ntiles < 1) return;
    if (nt == 6145) {                        // 128 x 48 cells, beta = 0 only (the w block would spill)
        if (!has_w) launch_rows_shape<false, 16, 3>(a, grid, s);
    } else if (nt == 4098) {                 // 128 x 32 cells
        if (has_w) launch_rows_shape<true, 16, 2>(a, grid, s);
        else launch_rows_shape<false, 16, 2>(a, grid, s);
    } else if (nt == 3074) {                 // 64 x 48 cells, one per lane and row, beta = 0 only
        if (!has_w) launch_rows1_shape<false, 16, 3>(a, grid, s);
    } else if (nt == 2050) {                 // 64 x 32 cells, one per lane and row
        if (has_w) launch_rows1_shape<true, 16, 2>(a, grid, s);
        else launch_rows1_shape<false, 16, 2>(a, grid, s);
    }
}

}  // namespace flowmi
