// Preconditioned Douglas-Rachford iteration (Sec. 3.1.2, tag pDR) on gfx950.
//
//   b      = X bar + sigma div y bar                                  (per component w, u, v)
//   X+     = X + M^{-1}(b - T X),  T = I - sigma tau Delta (Neumann),  M = n symmetric red-black
//            Gauss-Seidel sweeps (eq. neumann:boudary)
//   X bar+ = X bar + J(2 X+ - X bar) - X+,  J = (I + sigma dF)^{-1} (eq:resolvent); J moves its
//            argument by a step along e = (beta, I_x, I_y), so this is X+ + step e
//   y bar+ = P(y bar + 2 tau grad X+) - tau grad X+                   (P_p on p, joint P_q on q)
//
// A red (i + j even) or black cell update only reads cells of the other colour, so every half
// sweep runs in place and in parallel.  One symmetric sweep (red, black, black, red) equals red,
// black, red because the repeated black half sweep changes nothing; n sweeps are the 2n + 1
// half sweeps R B R B ... R.  Passes:
//   rhs_red   b for all cells, first red half sweep
//   colour    one black or red half sweep (2n - 1 of them, alternating, starting with black)
//   final     the last red half sweep fused with the resolvent and the dual update: each cell
//             re-derives X+ at itself and at its right / lower neighbours from black values
//             (which no pass writes any more), so no cell reads a value written in the pass.
#include "kernels.hpp"

namespace flowmi {

namespace {

dim3 grid2d(int H, int W) { return dim3((W + 63) / 64, (H + 3) / 4); }

// GS update of one cell, (b + st * sum of in-frame neighbours) / (1 + st * count), evaluated as
// the cell's value plus its correction ((b - x) + st * sum of (neighbour - x)) / (1 + st * count):
// the same value, but the flows (several pixels) cancel in the differences before any rounding,
// so FP32 rounds only the small correction and the final sum
__device__ __forceinline__ float gs_cell(const float* x, const float* b, int i, int j, int H, int W, int64_t ld,
                                         float stt) {
    const int64_t o = (int64_t)i * ld + j;
    const float xo = x[o];
    float s = 0.f, n = 0.f;
    if (j > 0) { s += x[o - 1] - xo; n += 1.f; }
    if (j < W - 1) { s += x[o + 1] - xo; n += 1.f; }
    if (i > 0) { s += x[o - ld] - xo; n += 1.f; }
    if (i < H - 1) { s += x[o + ld] - xo; n += 1.f; }
    return xo + ((b[o] - xo) + stt * s) / (1.f + stt * n);
}

__device__ __forceinline__ float div_at(const float* px, const float* py, int i, int j, int H, int W, int64_t ld) {
    const int64_t o = (int64_t)i * ld + j;
    float d = 0.f;
    if (j < W - 1) d += px[o];
    if (j > 0) d -= px[o - 1];
    if (i < H - 1) d += py[o];
    if (i > 0) d -= py[o - ld];
    return d;
}

template <bool HAS_W>
__global__ __launch_bounds__(256) void pdr_rhs_red_kernel(PdrArgs a) {
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= a.H || j >= a.W) return;
    const int64_t o = (int64_t)i * a.ld + j;
    const float bu = a.ub[o] + a.sigma * div_at(a.qb1x, a.qb1y, i, j, a.H, a.W, a.ld);
    const float bv = a.vb[o] + a.sigma * div_at(a.qb2x, a.qb2y, i, j, a.H, a.W, a.ld);
    a.bu[o] = bu;
    a.bv[o] = bv;
    float bw = 0.f;
    if constexpr (HAS_W) {
        bw = a.wb[o] + a.sigma * div_at(a.pbx, a.pby, i, j, a.H, a.W, a.ld);
        a.bw[o] = bw;
    }
    if (((i + j) & 1) == 0) {
        a.u[o] = gs_cell(a.u, a.bu, i, j, a.H, a.W, a.ld, a.stt);
        a.v[o] = gs_cell(a.v, a.bv, i, j, a.H, a.W, a.ld, a.stt);
        if constexpr (HAS_W) a.w[o] = gs_cell(a.w, a.bw, i, j, a.H, a.W, a.ld, a.stt);
    }
}

template <bool HAS_W>
__global__ __launch_bounds__(256) void pdr_colour_kernel(PdrArgs a) {
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= a.H || j >= a.W) return;
    if (((i + j) & 1) != a.colour) return;
    const int64_t o = (int64_t)i * a.ld + j;
    a.u[o] = gs_cell(a.u, a.bu, i, j, a.H, a.W, a.ld, a.stt);
    a.v[o] = gs_cell(a.v, a.bv, i, j, a.H, a.W, a.ld, a.stt);
    if constexpr (HAS_W) a.w[o] = gs_cell(a.w, a.bw, i, j, a.H, a.W, a.ld, a.stt);
}

// X+ at (i, j) after the last red half sweep: red cells are re-derived from their (final) black
// neighbours, black cells are final already.
__device__ __forceinline__ float final_x(const float* x, const float* b, int i, int j, int H, int W, int64_t ld,
                                         float stt) {
    if (((i + j) & 1) == 0) return gs_cell(x, b, i, j, H, W, ld, stt);
    return x[(int64_t)i * ld + j];
}

template <bool HAS_W>
__global__ __launch_bounds__(256) void pdr_final_kernel(PdrArgs a) {
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= a.H || j >= a.W) return;
    const int64_t o = (int64_t)i * a.ld + j;
    const bool red = ((i + j) & 1) == 0;
    const bool hasr = j < a.W - 1, hasd = i < a.H - 1;

    const float u = final_x(a.u, a.bu, i, j, a.H, a.W, a.ld, a.stt);
    const float v = final_x(a.v, a.bv, i, j, a.H, a.W, a.ld, a.stt);
    const float ux = hasr ? final_x(a.u, a.bu, i, j + 1, a.H, a.W, a.ld, a.stt) - u : 0.f;
    const float uy = hasd ? final_x(a.u, a.bu, i + 1, j, a.H, a.W, a.ld, a.stt) - u : 0.f;
    const float vx = hasr ? final_x(a.v, a.bv, i, j + 1, a.H, a.W, a.ld, a.stt) - v : 0.f;
    const float vy = hasd ? final_x(a.v, a.bv, i + 1, j, a.H, a.W, a.ld, a.stt) - v : 0.f;
    float w = 0.f, wx = 0.f, wy = 0.f;
    if constexpr (HAS_W) {
        w = final_x(a.w, a.bw, i, j, a.H, a.W, a.ld, a.stt);
        wx = hasr ? final_x(a.w, a.bw, i, j + 1, a.H, a.W, a.ld, a.stt) - w : 0.f;
        wy = hasd ? final_x(a.w, a.bw, i + 1, j, a.H, a.W, a.ld, a.stt) - w : 0.f;
    }

    // data-term resolvent at X~ = 2 X+ - X bar (eq:resolvent)
    const float ub = a.ub[o], vb = a.vb[o];
    const float ut = 2.f * u - ub, vt = 2.f * v - vb;
    const float Ix = a.Ix[o], Iy = a.Iy[o], It = a.It[o];
    float wbv = 0.f, wt = 0.f;
    if constexpr (HAS_W) { wbv = a.wb[o]; wt = 2.f * w - wbv; }
    const float e2 = a.beta * a.beta + Ix * Ix + Iy * Iy;
    // with a relative I_t the residual is formed from the displacement relative to the
    // linearisation point, which keeps FP32 cancellation out of rho
    const float du0 = a.u0 ? ut - a.u0[o] : ut;
    const float dv0 = a.v0 ? vt - a.v0[o] : vt;
    const float rho = It + a.beta * wt + Ix * du0 + Iy * dv0;
    // eq:resolvent: the step along e is -rho / |e|^2 clamped to [-sigma lam, sigma lam], and
    // Theta = clamp(rho / (sigma |e|^2), -lam, lam) = -step / sigma (both 0 where e = 0);
    // 1 / |e|^2 is the hardware reciprocal (within 1 ulp): the same in every pDR kernel
    const float sl = a.sigma * a.lam;
    float step = 0.f, theta = 0.f;
    if (e2 > 0.f) {
        step = __builtin_amdgcn_fmed3f(-rho * __builtin_amdgcn_rcpf(e2), -sl, sl);
        theta = -step * (1.f / a.sigma);
    }
    // X bar + J(X~) - X+ with J(X~) = X~ + step e and X~ = 2 X+ - X bar is X+ + step e (one rounding)
    a.ub[o] = u + step * Ix;
    a.vb[o] = v + step * Iy;
    if constexpr (HAS_W) a.wb[o] = w + step * a.beta;
    if (a.s_out) a.s_out[o] = theta;

    // dual: y bar+ = P(y bar + 2 tau grad X+) - tau grad X+
    const float t2 = 2.f * a.tau;
    const float a1x = a.qb1x[o] + t2 * ux, a1y = a.qb1y[o] + t2 * uy;
    const float a2x = a.qb2x[o] + t2 * vx, a2y = a.qb2y[o] + t2 * vy;
    const float nq = a1x * a1x + a1y * a1y + a2x * a2x + a2y * a2y;
    const float sq = nq > 1.f ? rsqrtf(nq) : 1.f;
    a.qb1x[o] = a1x * sq - a.tau * ux;
    a.qb1y[o] = a1y * sq - a.tau * uy;
    a.qb2x[o] = a2x * sq - a.tau * vx;
    a.qb2y[o] = a2y * sq - a.tau * vy;
    if constexpr (HAS_W) {
        const float bx = a.pbx[o] + t2 * wx, by = a.pby[o] + t2 * wy;
        const float np2 = bx * bx + by * by;
        const float sp = np2 > 1.f ? rsqrtf(np2) : 1.f;
        a.pbx[o] = bx * sp - a.tau * wx;
        a.pby[o] = by * sp - a.tau * wy;
    }
    if (red) {
        a.u[o] = u;
        a.v[o] = v;
        if constexpr (HAS_W) a.w[o] = w;
    }
}

}  // namespace

void launch_pdr_rhs_red(const PdrArgs& a, bool has_w, hipStream_t s) {
    if (has_w) hipLaunchKernelGGL(pdr_rhs_red_kernel<true>, grid2d(a.H, a.W), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(pdr_rhs_red_kernel<false>, grid2d(a.H, a.W), dim3(256), 0, s, a);
}

void launch_pdr_colour(const PdrArgs& a, bool has_w, hipStream_t s) {
    if (has_w) hipLaunchKernelGGL(pdr_colour_kernel<true>, grid2d(a.H, a.W), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(pdr_colour_kernel<false>, grid2d(a.H, a.W), dim3(256), 0, s, a);
}

void launch_pdr_final(const PdrArgs& a, bool has_w, hipStream_t s) {
    if (has_w) hipLaunchKernelGGL(pdr_final_kernel<true>, grid2d(a.H, a.W), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(pdr_final_kernel<false>, grid2d(a.H, a.W), dim3(256), 0, s, a);
}

}  // namespace flowmi
