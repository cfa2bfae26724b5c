// Temporally blocked iterations of the preconditioned Douglas-Rachford scheme (Sec. 3.1.2, tag
// pDR, with the symmetric red-black Gauss-Seidel preconditioner of eq. neumann:boudary) on gfx950.
//
// One work-group owns an output tile of one level and advances it by K iterations in one launch.
// Per iteration and cell (X = (w, u, v), X bar, y bar = (p bar, q bar), n sweeps):
//   [b + R]   b = X bar + sigma div y bar; first red half sweep
//   [B] [R]   n black / red half sweep pairs (x = (b + st sum_nb x) / (1 + st #nb), st = sigma tau)
//   [D]       X+ = x; X bar+ = X bar + J(2 X+ - X bar) - X+ = X+ + step e (eq:resolvent: J moves
//             its argument by a step along e = (beta, I_x, I_y));
//             y bar+ = P(y bar + 2 tau grad X+) - tau grad X+
// with a barrier between phases.  Each half sweep reaches one cell further in every direction; b
// takes div y bar (left / up) and the dual update grad X+ (right / down), so after K iterations
// X and X bar depend on the launch's input within (2n + 1) K cells on every side and y bar one
// more below and to the right.  The tile is loaded with that halo; where it meets the image border
// there is no halo and the boundary rules of Sec. 2.2 apply exactly.
//
// Layout by colour: thread t owns the t-th red and the t-th black cell of the extended region (in
// row-major order), and LDS holds X and y bar per colour, indexed by a cell's rank within its
// colour.  A half sweep then runs one cell per thread with every lane busy, and every neighbour of
// a cell lies in the other colour's arrays.  X bar, b and the linearisation are read at their own
// cell only and live in registers.  Neighbour ranks and the operators' coefficients (the
// neighbour exists in the image, the Gauss-Seidel denominator) are fixed for the launch; a
// neighbour outside the extended region reads an unrelated finite value with a non-zero
// coefficient, which only changes halo cells the halo accounts for.  Reads and writes go to
// different state buffers, so tiles of one launch are independent.
#include "kernels.hpp"

namespace flowmi {

namespace {

template <bool HAS_W, int NC>
struct PdrLds {
    static constexpr int NX = HAS_W ? 3 : 2;   // x components held: (u, v) or (u, v, w)
    static constexpr int NY = HAS_W ? 6 : 4;
    // [colour][component][1 + rank]: one spare slot at each end, so that the ranks of a cell's left and
    // right neighbours (always consecutive within a row of the other colour) both index the array
    float x[2][NX][NC + 2];
    float y[2][NY][NC + 2];
};

// NT threads, CPC cells of each colour per thread (ranks tid, tid + NT, ...): NC = NT * CPC cells of
// each colour per tile.
template <bool HAS_W, int NT, int CPC>
__device__ __forceinline__ void pdr_tile(const PdrTbArgs& a, const PdrTbLevel& L, int y0, int x0, int th, int tw,
                                         PdrLds<HAS_W, NT * CPC>& S) {
    constexpr int NC = NT * CPC;
    constexpr int NX = PdrLds<HAS_W, NC>::NX;
    constexpr int NY = PdrLds<HAS_W, NC>::NY;
    const int tid = threadIdx.x;
    const int H = L.H, W = L.W;
    const int64_t ld = L.ld;
    const int K = a.K, n = a.sweeps;
    const int hlu = pdr_halo_lo(n, K), hrd = pdr_halo_hi(n, K);
    const int ey0 = max(y0 - hlu, 0), ex0 = max(x0 - hlu, 0);
    const int ey1 = min(y0 + th + hrd, H), ex1 = min(x0 + tw + hrd, W);
    const int EW = ex1 - ex0, EH = ey1 - ey0;
    const float sigma = a.sigma, tau = a.tau, stt = a.stt, lam = a.lam, beta = a.beta;
    const float sl = sigma * lam, inv_sigma = 1.f / sigma;
    const int wave0 = __builtin_amdgcn_readfirstlane(tid & ~63);

    // colour c (0 red, 1 black) of local cell (i, j): red iff (p0 + i + j) is even, p0 the parity of
    // the region's corner in image coordinates.  Row i holds its colour-c cells at columns of parity
    // (p0 + i + c) & 1; two consecutive rows hold EW cells of each colour.
    const int p0 = (ey0 + ex0) & 1;
    auto row_count = [&](int c, int i) { return (EW - ((p0 + i + c) & 1) + 1) >> 1; };
    auto rank_of = [&](int c, int i, int j) { return (i >> 1) * EW + ((i & 1) ? row_count(c, 0) : 0) + (j >> 1); };
    int ncol[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) ncol[c] = rank_of(c, EH, 0);
    // slot k of colour c: the thread's cell of rank tid + k NT (a cell of the region iff own(c, k));
    // live: some lane of the wavefront holds a cell (wave-uniform)
    auto live = [&](int c, int k) { return wave0 + k * NT < ncol[c]; };
    auto own = [&](int c, int k) { return tid + k * NT < ncol[c]; };
    auto cell = [&](int c, int k, int& i, int& j) {
        const int r = tid + k * NT;
        const int m = r / EW, rem = r - m * EW, rc0 = row_count(c, 0);
        i = rem < rc0 ? 2 * m : 2 * m + 1;
        j = ((p0 + i + c) & 1) + 2 * (rem < rc0 ? rem : rem - rc0);
    };
    // LDS positions (1 + rank, in the other colour's arrays) of the left, upper and lower neighbours;
    // the right neighbour sits at nL + 1.  Outside the region: a spare or unrelated finite slot.
    int nL[2][CPC], nU[2][CPC], nD[2][CPC];
    float fl[2][CPC], fr[2][CPC], fu[2][CPC], fd[2][CPC], rden[2][CPC];
    float xb[NX][2][CPC], bb[NX][2][CPC], Ix[2][CPC], Iy[2][CPC], It[2][CPC], u0[2][CPC], v0[2][CPC];
    float th_s[2][CPC];
    if (tid == 0) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
#pragma unroll
            for (int f = 0; f < NX; ++f) S.x[c][f][0] = S.x[c][f][NC + 1] = 0.f;
#pragma unroll
            for (int f = 0; f < NY; ++f) S.y[c][f][0] = S.y[c][f][NC + 1] = 0.f;
        }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int k = 0; k < CPC; ++k) {
        int i, j;
        cell(c, k, i, j);
        const int gi = ey0 + i, gj = ex0 + j;
        const int oc = 1 - c;                       // every neighbour has the other colour
        const bool mine = own(c, k);
        nL[c][k] = mine ? 1 + rank_of(oc, i, j - 1) : 0;   // j - 1 = -1 gives rank - 1: the spare slot
        nU[c][k] = (mine && i > 0) ? 1 + rank_of(oc, i - 1, j) : 0;
        nD[c][k] = (mine && i + 1 < EH) ? 1 + rank_of(oc, i + 1, j) : 0;
        fl[c][k] = gj > 0 ? 1.f : 0.f;
        fr[c][k] = gj < W - 1 ? 1.f : 0.f;
        fu[c][k] = gi > 0 ? 1.f : 0.f;
        fd[c][k] = gi < H - 1 ? 1.f : 0.f;
        rden[c][k] = 1.f / (1.f + stt * (((fl[c][k] + fr[c][k]) + fu[c][k]) + fd[c][k]));
        float xv[NX], yv[NY];
#pragma unroll
        for (int f = 0; f < NX; ++f) xv[f] = xb[f][c][k] = bb[f][c][k] = 0.f;
#pragma unroll
        for (int f = 0; f < NY; ++f) yv[f] = 0.f;
        Ix[c][k] = Iy[c][k] = It[c][k] = u0[c][k] = v0[c][k] = th_s[c][k] = 0.f;
        if (mine) {
            const int64_t o = (int64_t)gi * ld + gj;
#pragma unroll
            for (int f = 0; f < NX; ++f) {
                xv[f] = L.x_in[f][o];
                xb[f][c][k] = L.xb_in[f][o];
            }
#pragma unroll
            for (int f = 0; f < NY; ++f) yv[f] = L.y_in[f][o];
            Ix[c][k] = L.Ix[o];
            Iy[c][k] = L.Iy[o];
            It[c][k] = L.It[o];
            u0[c][k] = L.u0[o];
            v0[c][k] = L.v0[o];
        }
        const int e = 1 + tid + k * NT;
#pragma unroll
        for (int f = 0; f < NX; ++f) S.x[c][f][e] = xv[f];
#pragma unroll
        for (int f = 0; f < NY; ++f) S.y[c][f][e] = yv[f];
    }
    __syncthreads();

    // one half sweep over the cells of colour c: x = (b + st sum of in-image neighbours) / (1 + st #),
    // evaluated as x + ((b - x) + st sum of (neighbour - x)) / (1 + st #), summed left, right, up,
    // down: the flows cancel in the differences before any rounding, so FP32 rounds only the small
    // correction and the final sum.  A thread's slots of one colour have no neighbour in common
    // colour, so the slots of one half sweep are independent.
    auto half_sweep = [&](int c) {
        const int oc = 1 - c;
#pragma unroll
        for (int k = 0; k < CPC; ++k) {
            if (!live(c, k)) continue;
            const int e = 1 + tid + k * NT;
            float nb[NX][4], xo[NX];
#pragma unroll
            for (int f = 0; f < NX; ++f) {
                nb[f][0] = S.x[oc][f][nL[c][k]];
                nb[f][1] = S.x[oc][f][nL[c][k] + 1];
                nb[f][2] = S.x[oc][f][nU[c][k]];
                nb[f][3] = S.x[oc][f][nD[c][k]];
                xo[f] = S.x[c][f][e];
            }
#pragma unroll
            for (int f = 0; f < NX; ++f) {
                float sm = fl[c][k] * (nb[f][0] - xo[f]);
                sm = fmaf(fr[c][k], nb[f][1] - xo[f], sm);
                sm = fmaf(fu[c][k], nb[f][2] - xo[f], sm);
                sm = fmaf(fd[c][k], nb[f][3] - xo[f], sm);
                S.x[c][f][e] = fmaf((bb[f][c][k] - xo[f]) + stt * sm, rden[c][k], xo[f]);
            }
        }
    };

    for (int it = 0; it < K; ++it) {
        // [b + R]: b from div y bar ([j < W-1] y_x - [j > 0] y_x left + [i < H-1] y_y - [i > 0] y_y up),
        // then the first red half sweep (reads only black cells, writes only red ones)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int k = 0; k < CPC; ++k) {
            if (!live(c, k)) continue;
            const int e = 1 + tid + k * NT;
            float yo[NX][2], yn[NX][2];
#pragma unroll
            for (int f = 0; f < NX; ++f) {
                yo[f][0] = S.y[c][2 * f][e];
                yo[f][1] = S.y[c][2 * f + 1][e];
                yn[f][0] = S.y[1 - c][2 * f][nL[c][k]];
                yn[f][1] = S.y[1 - c][2 * f + 1][nU[c][k]];
            }
#pragma unroll
            for (int f = 0; f < NX; ++f) {
                float d = fr[c][k] * yo[f][0];
                d = fmaf(-fl[c][k], yn[f][0], d);
                d = fmaf(fd[c][k], yo[f][1], d);
                d = fmaf(-fu[c][k], yn[f][1], d);
                bb[f][c][k] = xb[f][c][k] + sigma * d;
            }
        }
        half_sweep(0);
        for (int sw = 0; sw < n; ++sw) {
            __syncthreads();
            half_sweep(1);
            __syncthreads();
            half_sweep(0);
        }
        __syncthreads();
        // [D]: resolvent at X~ = 2 X+ - X bar, dual update from grad X+ (right / down neighbours)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int k = 0; k < CPC; ++k) {
            if (!live(c, k)) continue;
            const int e = 1 + tid + k * NT;
            float xo[NX], xr[NX], xd[NX], yo[NY];
#pragma unroll
            for (int f = 0; f < NX; ++f) {
                xo[f] = S.x[c][f][e];
                xr[f] = S.x[1 - c][f][nL[c][k] + 1];
                xd[f] = S.x[1 - c][f][nD[c][k]];
            }
#pragma unroll
            for (int f = 0; f < NY; ++f) yo[f] = S.y[c][f][e];
            float gx[NX], gy[NX];
#pragma unroll
            for (int f = 0; f < NX; ++f) {
                gx[f] = fr[c][k] * (xr[f] - xo[f]);
                gy[f] = fd[c][k] * (xd[f] - xo[f]);
            }
            const float u = xo[0], v = xo[1];
            const float ub = xb[0][c][k], vbv = xb[1][c][k];
            const float ut = 2.f * u - ub, vt = 2.f * v - vbv;
            float w = 0.f, wbv = 0.f, wt = 0.f;
            if constexpr (HAS_W) { w = xo[2]; wbv = xb[2][c][k]; wt = 2.f * w - wbv; }
            const float ix = Ix[c][k], iy = Iy[c][k];
            // sums of products as explicit FMA chains: every pDR tile kernel rounds them alike
            const float e2 = fmaf(iy, iy, fmaf(ix, ix, beta * beta));
            const float rho = fmaf(iy, vt - v0[c][k], fmaf(ix, ut - u0[c][k], fmaf(beta, wt, It[c][k])));
            // eq:resolvent: the step along e is -rho / |e|^2 clamped to [-sigma lam, sigma lam], and
            // Theta = clamp(rho / (sigma |e|^2), -lam, lam) = -step / sigma (both 0 where e = 0);
            // 1 / |e|^2 is the hardware reciprocal (within 1 ulp): the same in every pDR kernel
            float step = 0.f, theta = 0.f;
            if (e2 > 0.f) {
                step = __builtin_amdgcn_fmed3f(-rho * __builtin_amdgcn_rcpf(e2), -sl, sl);
                theta = -step * inv_sigma;
            }
            // X bar + J(X~) - X+ with J(X~) = X~ + step e, X~ = 2 X+ - X bar: X+ + step e
            xb[0][c][k] = fmaf(step, ix, u);
            xb[1][c][k] = fmaf(step, iy, v);
            if constexpr (HAS_W) xb[2][c][k] = fmaf(step, beta, w);
            th_s[c][k] = theta;
            const float t2 = 2.f * tau;
            const float a1x = yo[0] + t2 * gx[0], a1y = yo[1] + t2 * gy[0];
            const float a2x = yo[2] + t2 * gx[1], a2y = yo[3] + t2 * gy[1];
            const float nq = fmaf(a2y, a2y, fmaf(a2x, a2x, fmaf(a1y, a1y, a1x * a1x)));
            const float sq = fminf(1.f, __builtin_amdgcn_rsqf(nq));
            S.y[c][0][e] = fmaf(a1x, sq, -(tau * gx[0]));
            S.y[c][1][e] = fmaf(a1y, sq, -(tau * gy[0]));
            S.y[c][2][e] = fmaf(a2x, sq, -(tau * gx[1]));
            S.y[c][3][e] = fmaf(a2y, sq, -(tau * gy[1]));
            if constexpr (HAS_W) {
                const float bx = yo[4] + t2 * gx[2], by = yo[5] + t2 * gy[2];
                const float np2 = fmaf(by, by, bx * bx);
                const float sp = fminf(1.f, __builtin_amdgcn_rsqf(np2));
                S.y[c][4][e] = fmaf(bx, sp, -(tau * gx[2]));
                S.y[c][5][e] = fmaf(by, sp, -(tau * gy[2]));
            }
        }
        __syncthreads();
    }

    // write the output tile
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int k = 0; k < CPC; ++k) {
        if (!own(c, k)) continue;
        int i, j;
        cell(c, k, i, j);
        const int gi = ey0 + i, gj = ex0 + j;
        if (gi < y0 || gi >= y0 + th || gj < x0 || gj >= x0 + tw) continue;
        const int64_t o = (int64_t)gi * ld + gj;
        const int e = 1 + tid + k * NT;
#pragma unroll
        for (int f = 0; f < NX; ++f) {
            L.x_out[f][o] = S.x[c][f][e];
            L.xb_out[f][o] = xb[f][c][k];
        }
#pragma unroll
        for (int f = 0; f < NY; ++f) L.y_out[f][o] = S.y[c][f][e];
        L.s_out[o] = th_s[c][k];
    }
}

__device__ __forceinline__ int xcd_tile_p(int b, int nb) {
    const int per = nb >> 3;   // host pads the grid to a multiple of 8
    return (b & 7) * per + (b >> 3);
}

template <bool HAS_W, int NT, int CPC>
__global__ __launch_bounds__(NT) void pdr_tb_kernel(PdrTbArgs a) {
    __shared__ PdrLds<HAS_W, NT * CPC> S;
    const int t = xcd_tile_p(blockIdx.x, gridDim.x);
    if (t >= a.ntiles) return;
    const int ty = t / a.ntx, tx = t - ty * a.ntx;
    const int y0 = ty * a.th, x0 = tx * a.tw;
    pdr_tile<HAS_W, NT, CPC>(a, a.lvl, y0, x0, min(a.th, a.lvl.H - y0), min(a.tw, a.lvl.W - x0), S);
}

// Many levels (batched pairs): tile entries of a table in XCD order; neighbouring tiles of a level,
// which re-read each other's halo, share one XCD's L2.  The grid is a multiple of 8 of at least
// ntiles.
template <bool HAS_W, int NT, int CPC>
__global__ __launch_bounds__(NT) void pdr_tb_table_kernel(PdrTbArgs a) {
    __shared__ PdrLds<HAS_W, NT * CPC> S;
    const int per = (a.ntiles + 7) >> 3;             // tiles per XCD
    const int x = blockIdx.x & 7, y = blockIdx.x >> 3;
    const int t = x * per + y;
    if (y >= per || t >= a.ntiles) return;
    const TbTile T = a.tiles[t];
    pdr_tile<HAS_W, NT, CPC>(a, a.levels[2 * T.level + a.dir], T.y0, T.x0, T.th, T.tw, S);
}

}  // namespace


template <bool HAS_W, int NT, int CPC>
static void launch_pdr_shape(const PdrTbArgs& a, int grid, hipStream_t s) {
    if (a.tiles) hipLaunchKernelGGL((pdr_tb_table_kernel<HAS_W, NT, CPC>), dim3(grid), dim3(NT), 0, s, a);
    else hipLaunchKernelGGL((pdr_tb_kernel<HAS_W, NT, CPC>), dim3(grid), dim3(NT), 0, s, a);
}

void launch_pdr_tb(const PdrTbArgs& a, bool has_w, int nt, hipStream_t s) {
    const int grid = (a.ntiles + 7) / 8 * 8;
    if (a.ntiles < 1) return;
    if (is_pd_rows_code(nt)) {               // wave-row tiles (6145 without the w block only)
        launch_pdr_rows(a, has_w, nt, s);
        return;
    }
    // two cells of each colour per thread exist for beta = 0 only (with the w block they would need
    // more than 128 VGPRs); the planners never pair them with w, and a tile sized for them must not
    // reach the other kernels' LDS
    if ((nt == 2048 || nt == 513) && has_w) return;
    if (nt == 512) {
        if (has_w) launch_pdr_shape<true, 512, 1>(a, grid, s);
        else launch_pdr_shape<false, 512, 1>(a, grid, s);
    } else if (nt == 2048) {                 // 1024 threads, two cells of each colour per thread
        launch_pdr_shape<false, 1024, 2>(a, grid, s);
    } else if (nt == 513) {                  // 512 threads, two cells of each colour per thread
        launch_pdr_shape<false, 512, 2>(a, grid, s);
    } else {
        if (has_w) launch_pdr_shape<true, 1024, 1>(a, grid, s);
        else launch_pdr_shape<false, 1024, 1>(a, grid, s);
    }
}

}  // namespace flowmi
