// Temporally blocked iterations of the preconditioned Douglas-Rachford scheme (Sec. 3.1.2, tag
// pDR, with the symmetric red-black Gauss-Seidel preconditioner of eq. neumann:boudary) on gfx950.
//
// One work-group owns an output tile of one level and advances it by K iterations in one launch.
// Per iteration and cell (X = (w, u, v), X bar, y bar = (p bar, q bar), n sweeps):
//   [b + R]   b = X bar + sigma div y bar; first red half sweep
//   [B] [R]   n black / red half sweep pairs (x = (b + st sum_nb x) / (1 + st #nb), st = sigma tau)
//   [D]       X+ = x; X bar+ = X bar + J(2 X+ - X bar) - X+ (eq:resolvent);
//             y bar+ = P(y bar + 2 tau grad X+) - tau grad X+
// with a barrier between phases.  Each half sweep reaches one cell further in every direction; b
// takes div y bar (left / up) and the dual update grad X+ (right / down), so after K iterations
// X and X bar depend on the launch's input within (2n + 1) K cells on every side and y bar one
// more below and to the right.  The tile is loaded with that halo; where it meets the image border
// there is no halo and the boundary rules of Sec. 2.2 apply exactly.  X and y bar, whose neighbours are read, live in LDS; X bar, b and the
// linearisation are read at their own cell only and live in registers.  Reads and writes go to
// different state buffers, so tiles of one launch are independent.  Every neighbour read is an
// unconditional LDS read at an index clamped into the array followed by a select, in the same
// summation order as the three-pass kernels.
#include "kernels.hpp"

namespace flowmi {

namespace {

template <bool HAS_W, int NT, int PPT>
struct PdrLds {
    static constexpr int CAP = NT * PPT;
    static constexpr int NX = HAS_W ? 3 : 2;   // x components held: (u, v) or (w, u, v)
    static constexpr int NY = HAS_W ? 6 : 4;
    float x[NX][CAP];
    float y[NY][CAP];
};

template <bool HAS_W, int NT, int PPT>
__device__ __forceinline__ void pdr_tile(const PdrTbArgs& a, int y0, int x0, int th, int tw,
                                         PdrLds<HAS_W, NT, PPT>& S) {
    constexpr int CAP = NT * PPT;
    constexpr int NX = PdrLds<HAS_W, NT, PPT>::NX;
    constexpr int NY = PdrLds<HAS_W, NT, PPT>::NY;
    const PdrTbLevel& L = a.lvl;
    const int tid = threadIdx.x;
    const int H = L.H, W = L.W;
    const int64_t ld = L.ld;
    const int K = a.K, n = a.sweeps;
    const int hlu = pdr_halo_lo(n, K), hrd = pdr_halo_hi(n, K);
    const int ey0 = max(y0 - hlu, 0), ex0 = max(x0 - hlu, 0);
    const int ey1 = min(y0 + th + hrd, H), ex1 = min(x0 + tw + hrd, W);
    const int EW = ex1 - ex0, EN = (ey1 - ey0) * EW;
    const float sigma = a.sigma, tau = a.tau, stt = a.stt, lam = a.lam, beta = a.beta;
    const int wave0 = __builtin_amdgcn_readfirstlane(tid & ~63);
    auto live = [&](int k) { return wave0 + k * NT < EN; };

    // component c of x / X bar: 0 -> u, 1 -> v, 2 -> w; y planes: q1x q1y q2x q2y (p_x p_y)
    int ei[PPT], ej[PPT];
    float xb[NX][PPT], bb[NX][PPT], Ix[PPT], Iy[PPT], It[PPT], u0[PPT], v0[PPT], th_s[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int e = tid + k * NT;
        ei[k] = e / EW;
        ej[k] = e - ei[k] * EW;
        const int gi = ey0 + ei[k], gj = ex0 + ej[k];
        float xv[NX], yv[NY];
#pragma unroll
        for (int c = 0; c < NX; ++c) xv[c] = xb[c][k] = bb[c][k] = 0.f;
#pragma unroll
        for (int c = 0; c < NY; ++c) yv[c] = 0.f;
        Ix[k] = Iy[k] = It[k] = u0[k] = v0[k] = th_s[k] = 0.f;
        if (e < EN) {
            const int64_t o = (int64_t)gi * ld + gj;
#pragma unroll
            for (int c = 0; c < NX; ++c) {
                xv[c] = L.x_in[c][o];
                xb[c][k] = L.xb_in[c][o];
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
        for (int c = 0; c < NX; ++c) S.x[c][e] = xv[c];
#pragma unroll
        for (int c = 0; c < NY; ++c) S.y[c][e] = yv[c];
    }
    __syncthreads();

    // red = (i + j) even, in image coordinates
    auto is_red = [&](int k) { return ((ey0 + ei[k] + ex0 + ej[k]) & 1) == 0; };
    // x = (b + st sum of in-image neighbours) / (1 + st #neighbours), summed left, right, up, down
    auto gs = [&](const float* X, float b, int k) {
        const int e = tid + k * NT;
        const int gi = ey0 + ei[k], gj = ex0 + ej[k];
        const float xl = X[max(e - 1, 0)], xr = X[min(e + 1, CAP - 1)];
        const float xu = X[max(e - EW, 0)], xd = X[min(e + EW, CAP - 1)];
        float s = 0.f, cnt = 0.f;
        if (gj > 0) { s += xl; cnt += 1.f; }
        if (gj < W - 1) { s += xr; cnt += 1.f; }
        if (gi > 0) { s += xu; cnt += 1.f; }
        if (gi < H - 1) { s += xd; cnt += 1.f; }
        return (b + stt * s) / (1.f + stt * cnt);
    };
    // [j < W-1] fx(i,j) - [j > 0] fx(i,j-1) + [i < H-1] fy(i,j) - [i > 0] fy(i-1,j)
    auto dv = [&](const float* fx, const float* fy, int k) {
        const int e = tid + k * NT;
        const int gi = ey0 + ei[k], gj = ex0 + ej[k];
        const float l = fx[max(e - 1, 0)], u = fy[max(e - EW, 0)];
        float d = 0.f;
        if (gj < W - 1) d += fx[e];
        if (gj > 0) d -= l;
        if (gi < H - 1) d += fy[e];
        if (gi > 0) d -= u;
        return d;
    };
    auto half_sweep = [&](bool red) {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (!live(k)) continue;
            if (is_red(k) != red) continue;
            const int e = tid + k * NT;
#pragma unroll
            for (int c = 0; c < NX; ++c) {
                const float xn = gs(S.x[c], bb[c][k], k);
                S.x[c][e] = xn;
            }
        }
    };

    for (int it = 0; it < K; ++it) {
        // [b + R]: b from y bar (left / up neighbours), then the first red half sweep (reads only
        // black neighbours, writes only red cells)
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (!live(k)) continue;
            bb[0][k] = xb[0][k] + sigma * dv(S.y[0], S.y[1], k);     // u from q1
            bb[1][k] = xb[1][k] + sigma * dv(S.y[2], S.y[3], k);     // v from q2
            if constexpr (HAS_W) bb[2][k] = xb[2][k] + sigma * dv(S.y[4], S.y[5], k);   // w from p
        }
        half_sweep(true);
        for (int sw = 0; sw < n; ++sw) {
            __syncthreads();
            half_sweep(false);
            __syncthreads();
            half_sweep(true);
        }
        __syncthreads();
        // [D]: resolvent at X~ = 2 X+ - X bar, dual update from grad X+ (right / down neighbours)
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (!live(k)) continue;
            const int e = tid + k * NT;
            const int gi = ey0 + ei[k], gj = ex0 + ej[k];
            const bool hasr = gj < W - 1, hasd = gi < H - 1;
            const int er = min(e + 1, CAP - 1), ed = min(e + EW, CAP - 1);
            const float u = S.x[0][e], v = S.x[1][e];
            const float ur = S.x[0][er], ud = S.x[0][ed], vr = S.x[1][er], vd = S.x[1][ed];
            const float ux = hasr ? ur - u : 0.f, uy = hasd ? ud - u : 0.f;
            const float vx = hasr ? vr - v : 0.f, vy = hasd ? vd - v : 0.f;
            float w = 0.f, wx = 0.f, wy = 0.f;
            if constexpr (HAS_W) {
                w = S.x[2][e];
                const float wr = S.x[2][er], wd = S.x[2][ed];
                wx = hasr ? wr - w : 0.f;
                wy = hasd ? wd - w : 0.f;
            }
            const float ub = xb[0][k], vbv = xb[1][k];
            const float ut = 2.f * u - ub, vt = 2.f * v - vbv;
            float wbv = 0.f, wt = 0.f;
            if constexpr (HAS_W) { wbv = xb[2][k]; wt = 2.f * w - wbv; }
            const float e2 = beta * beta + Ix[k] * Ix[k] + Iy[k] * Iy[k];
            const float rho = It[k] + beta * wt + Ix[k] * (ut - u0[k]) + Iy[k] * (vt - v0[k]);
            const float thr = sigma * lam * e2;
            float step, theta;
            if (e2 > 0.f) {
                if (rho < -thr) step = sigma * lam;
                else if (rho > thr) step = -sigma * lam;
                else step = -rho / e2;
                theta = fminf(fmaxf(rho / (sigma * e2), -lam), lam);
            } else {
                step = 0.f;
                theta = 0.f;
            }
            xb[0][k] = ub + (ut + step * Ix[k]) - u;
            xb[1][k] = vbv + (vt + step * Iy[k]) - v;
            if constexpr (HAS_W) xb[2][k] = wbv + (wt + step * beta) - w;
            th_s[k] = theta;
            const float t2 = 2.f * tau;
            const float a1x = S.y[0][e] + t2 * ux, a1y = S.y[1][e] + t2 * uy;
            const float a2x = S.y[2][e] + t2 * vx, a2y = S.y[3][e] + t2 * vy;
            const float nq = a1x * a1x + a1y * a1y + a2x * a2x + a2y * a2y;
            const float sq = nq > 1.f ? rsqrtf(nq) : 1.f;
            S.y[0][e] = a1x * sq - tau * ux;
            S.y[1][e] = a1y * sq - tau * uy;
            S.y[2][e] = a2x * sq - tau * vx;
            S.y[3][e] = a2y * sq - tau * vy;
            if constexpr (HAS_W) {
                const float bx = S.y[4][e] + t2 * wx, by = S.y[5][e] + t2 * wy;
                const float np2 = bx * bx + by * by;
                const float sp = np2 > 1.f ? rsqrtf(np2) : 1.f;
                S.y[4][e] = bx * sp - tau * wx;
                S.y[5][e] = by * sp - tau * wy;
            }
        }
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
            L.x_out[c][o] = S.x[c][e];
            L.xb_out[c][o] = xb[c][k];
        }
#pragma unroll
        for (int c = 0; c < NY; ++c) L.y_out[c][o] = S.y[c][e];
        L.s_out[o] = th_s[k];
    }
}

__device__ __forceinline__ int xcd_tile_p(int b, int nb) {
    const int per = nb >> 3;   // host pads the grid to a multiple of 8
    return (b & 7) * per + (b >> 3);
}

template <bool HAS_W, int NT, int PPT>
__global__ __launch_bounds__(NT) void pdr_tb_kernel(PdrTbArgs a) {
    __shared__ PdrLds<HAS_W, NT, PPT> S;
    const int t = xcd_tile_p(blockIdx.x, gridDim.x);
    if (t >= a.ntiles) return;
    const int ty = t / a.ntx, tx = t - ty * a.ntx;
    const int y0 = ty * a.th, x0 = tx * a.tw;
    pdr_tile<HAS_W, NT, PPT>(a, y0, x0, min(a.th, a.lvl.H - y0), min(a.tw, a.lvl.W - x0), S);
}

}  // namespace

int pdr_tb_capacity(bool has_w, int nt) { return nt * (has_w ? kPdrPptW : kPdrPpt); }

void launch_pdr_tb(const PdrTbArgs& a, bool has_w, int nt, hipStream_t s) {
    const int grid = (a.ntiles + 7) / 8 * 8;
    if (nt == 512) {
        if (has_w) hipLaunchKernelGGL((pdr_tb_kernel<true, 512, kPdrPptW>), dim3(grid), dim3(512), 0, s, a);
        else hipLaunchKernelGGL((pdr_tb_kernel<false, 512, kPdrPpt>), dim3(grid), dim3(512), 0, s, a);
    } else {
        if (has_w) hipLaunchKernelGGL((pdr_tb_kernel<true, 1024, kPdrPptW>), dim3(grid), dim3(1024), 0, s, a);
        else hipLaunchKernelGGL((pdr_tb_kernel<false, 1024, kPdrPpt>), dim3(grid), dim3(1024), 0, s, a);
    }
}

}  // namespace flowmi
