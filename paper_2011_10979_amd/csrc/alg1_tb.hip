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
// clamped into the array, followed by selects.
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
__device__ __forceinline__ void alg1_tile(const PdrTbArgs& a, int y0, int x0, int th, int tw,
                                          Alg1Lds<HAS_W, NT, PPT>& S) {
    constexpr int CAP = NT * PPT;
    constexpr int NX = Alg1Lds<HAS_W, NT, PPT>::NX;
    constexpr int NY = Alg1Lds<HAS_W, NT, PPT>::NY;
    const PdrTbLevel& L = a.lvl;
    const int tid = threadIdx.x;
    const int H = L.H, W = L.W;
    const int64_t ld = L.ld;
    const int K = a.K;
    const int hk = alg1_halo(K);
    const int ey0 = max(y0 - hk, 0), ex0 = max(x0 - hk, 0);
    const int ey1 = min(y0 + th + hk, H), ex1 = min(x0 + tw + hk, W);
    const int EW = ex1 - ex0, EN = (ey1 - ey0) * EW;
    const float sigma = a.sigma, tau = a.tau, lam = a.lam, beta = a.beta;
    const int wave0 = __builtin_amdgcn_readfirstlane(tid & ~63);
    auto live = [&](int k) { return wave0 + k * NT < EN; };

    // components: x / x bar (u, v, w); y (q1x, q1y, q2x, q2y, p_x, p_y)
    int ei[PPT], ej[PPT];
    float x[NX][PPT], Ix[PPT], Iy[PPT], It[PPT], u0[PPT], v0[PPT], th_s[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int e = tid + k * NT;
        ei[k] = e / EW;
        ej[k] = e - ei[k] * EW;
        const int gi = ey0 + ei[k], gj = ex0 + ej[k];
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
        for (int c = 0; c < NX; ++c) S.xb[c][e] = xbv[c];
#pragma unroll
        for (int c = 0; c < NY; ++c) S.y[c][e] = yv[c];
    }
    __syncthreads();

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

    for (int it = 0; it < K; ++it) {
        // [Y]: dual ascent from the forward differences of X bar, projected (joint q ball, p ball)
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (!live(k)) continue;
            const int e = tid + k * NT;
            const int gi = ey0 + ei[k], gj = ex0 + ej[k];
            const bool hasr = gj < W - 1, hasd = gi < H - 1;
            const int er = min(e + 1, CAP - 1), ed = min(e + EW, CAP - 1);
            float g[NX][2];
#pragma unroll
            for (int c = 0; c < NX; ++c) {
                const float xc = S.xb[c][e], xr = S.xb[c][er], xd = S.xb[c][ed];
                g[c][0] = hasr ? xr - xc : 0.f;
                g[c][1] = hasd ? xd - xc : 0.f;
            }
            const float a1x = S.y[0][e] + tau * g[0][0], a1y = S.y[1][e] + tau * g[0][1];
            const float a2x = S.y[2][e] + tau * g[1][0], a2y = S.y[3][e] + tau * g[1][1];
            const float nq = a1x * a1x + a1y * a1y + a2x * a2x + a2y * a2y;
            const float sq = nq > 1.f ? rsqrtf(nq) : 1.f;
            float pxn = 0.f, pyn = 0.f;
            if constexpr (HAS_W) {
                const float bx = S.y[4][e] + tau * g[2][0], by = S.y[5][e] + tau * g[2][1];
                const float np2 = bx * bx + by * by;
                const float sp = np2 > 1.f ? rsqrtf(np2) : 1.f;
                pxn = bx * sp;
                pyn = by * sp;
            }
            // every thread has read its neighbours' X bar; y is only read at its own cell here
            S.y[0][e] = a1x * sq;
            S.y[1][e] = a1y * sq;
            S.y[2][e] = a2x * sq;
            S.y[3][e] = a2y * sq;
            if constexpr (HAS_W) {
                S.y[4][e] = pxn;
                S.y[5][e] = pyn;
            }
        }
        __syncthreads();
        // [X]: primal proximal descent X+ = J(X + sigma div y+), extrapolation X bar+ = 2 X+ - X
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (!live(k)) continue;
            const int e = tid + k * NT;
            const float ut = x[0][k] + sigma * dv(S.y[0], S.y[1], k);
            const float vt = x[1][k] + sigma * dv(S.y[2], S.y[3], k);
            float wt = 0.f;
            if constexpr (HAS_W) wt = x[2][k] + sigma * dv(S.y[4], S.y[5], k);
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
            const float un = ut + step * Ix[k], vn = vt + step * Iy[k];
            S.xb[0][e] = 2.f * un - x[0][k];
            S.xb[1][e] = 2.f * vn - x[1][k];
            x[0][k] = un;
            x[1][k] = vn;
            if constexpr (HAS_W) {
                const float wn = wt + step * beta;
                S.xb[2][e] = 2.f * wn - x[2][k];
                x[2][k] = wn;
            }
            th_s[k] = theta;
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
            L.x_out[c][o] = x[c][k];
            L.xb_out[c][o] = S.xb[c][e];
        }
#pragma unroll
        for (int c = 0; c < NY; ++c) L.y_out[c][o] = S.y[c][e];
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
    alg1_tile<HAS_W, NT, PPT>(a, y0, x0, min(a.th, a.lvl.H - y0), min(a.tw, a.lvl.W - x0), S);
}

}  // namespace

void launch_alg1_tb(const PdrTbArgs& a, bool has_w, int nt, hipStream_t s) {
    const int grid = (a.ntiles + 7) / 8 * 8;
    if (nt == 512) {
        if (has_w) hipLaunchKernelGGL((alg1_tb_kernel<true, 512, kPdrPptW>), dim3(grid), dim3(512), 0, s, a);
        else hipLaunchKernelGGL((alg1_tb_kernel<false, 512, kPdrPpt>), dim3(grid), dim3(512), 0, s, a);
    } else {
        if (has_w) hipLaunchKernelGGL((alg1_tb_kernel<true, 1024, kPdrPptW>), dim3(grid), dim3(1024), 0, s, a);
        else hipLaunchKernelGGL((alg1_tb_kernel<false, 1024, kPdrPpt>), dim3(grid), dim3(1024), 0, s, a);
    }
}

}  // namespace flowmi
