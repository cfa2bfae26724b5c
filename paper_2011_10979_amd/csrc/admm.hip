// One fused iteration of the preconditioned dual ADMM family (rpADMMI, pADMM, Zach-pADMM,
// rpADMMII; Sec. 3.1.1) on gfx950.
//
// The paper's component form is evaluated in the equivalent "g / h" arrangement
//   g   = Lambda + c (div y - A s)                         (iterate k)
//   y+  = P(y + grad g / (a c))                            (P_p on p, joint P_q on (q1, q2))
//   h   = Lambda + c rho_s (div y+ - A s)
//   s+  = clamp(s + (I_t + beta h_w + I_x h_u + I_y h_v) / (a~ c), -lambda, lambda)
//   Lambda+ = Lambda + cA div y+ - A (cB s+ - cC s)
// which follows from (I - grad grad^*/a) y = y + grad div y / a and from absorbing the
// -(rho_s/a~) M_s s term into h.  rpADMMI: rho_s = 1, cA = cB = r c, cC = 0.  rpADMMII:
// rho_s = rho, cA = rho c, cB = c, cC = (1 - rho) c.
//
// Increment form (used by the solver): within a warp the multipliers are stored as u - u0 with
// u0 the linearisation point and I_t relative to it (I_t = kappa (I1(x + d0) - I0)), so the long
// running sum of multiplier updates and the data residual rho = I_t + I_x u + I_y v never carry the
// O(|grad I| |d0|) terms that FP32 would round; only g needs u0 (its gradient feeds the dual step).
//
// Data flow: HBM-bound (about 0.9 flop per byte), so one pass reads the iterate and the
// linearisation once and writes the next iterate once.  Each 64-lane wavefront owns a strip of
// 61 output columns (lane l <-> column x0 - 2 + l) and a short segment of R rows (R = 2, 4 or 8).  Horizontal
// neighbours come from lane shuffles, vertical ones from registers carried between rows, so no
// LDS and no barriers are needed.  Per row step r the wave computes g at row r, y+ at row r - 1
// and the output at row r - 1; all R + 3 input rows of the strip are loaded up front.
// Boundary masks follow the discrete gradient / divergence of Sec. 2.2 exactly (forward
// differences, the last column / row of a dual field does not enter div).
#include "kernels.hpp"

namespace flowmi {

namespace {

template <bool HAS_W>
struct Row {
    float q1x, q1y, q2x, q2y, u, v, s, Ix, Iy, It;
    float w, px, py;
    float u0, v0;
};

template <bool HAS_W, bool REL>
__device__ __forceinline__ void load_row(const AdmmIterArgs& a, int r, int j, bool cv, int y0, int y1,
                                         Row<HAS_W>& R) {
    const bool ok = cv && r >= 0 && r < a.H;
    const int64_t off = (int64_t)r * a.ld + j;
    R.q1x = ok ? a.q1x[off] : 0.f;
    R.q1y = ok ? a.q1y[off] : 0.f;
    R.q2x = ok ? a.q2x[off] : 0.f;
    R.q2y = ok ? a.q2y[off] : 0.f;
    const bool ok2 = ok && r >= y0 - 1;
    R.u = ok2 ? a.u[off] : 0.f;
    R.v = ok2 ? a.v[off] : 0.f;
    R.s = ok2 ? a.s[off] : 0.f;
    R.Ix = ok2 ? a.Ix[off] : 0.f;
    R.Iy = ok2 ? a.Iy[off] : 0.f;
    if constexpr (REL) {
        R.u0 = ok2 ? a.u0[off] : 0.f;
        R.v0 = ok2 ? a.v0[off] : 0.f;
    } else {
        R.u0 = R.v0 = 0.f;
    }
    const bool ok3 = ok && r >= y0 && r < y1;
    R.It = ok3 ? a.It[off] : 0.f;
    if constexpr (HAS_W) {
        R.px = ok ? a.px[off] : 0.f;
        R.py = ok ? a.py[off] : 0.f;
        R.w = ok2 ? a.w[off] : 0.f;
    } else {
        R.px = R.py = R.w = 0.f;
    }
}

__device__ __forceinline__ int xcd_tile(int b, int nb) {
    // Work-groups are dealt round-robin to the 8 XCDs; give each XCD a contiguous run of tiles so
    // the halo rows / columns that neighbouring waves re-read stay in that XCD's L2.
    const int per = nb >> 3;   // host pads the grid to a multiple of 8
    return (b & 7) * per + (b >> 3);
}

template <bool HAS_W, bool REL, int R>
__global__ __launch_bounds__(256) void admm_iter_kernel(AdmmIterArgs a) {
    const int lane = threadIdx.x & 63;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int wave = tile * 4 + (threadIdx.x >> 6);
    if (wave >= a.strips * a.segs) return;              // whole wavefront leaves together
    const int strip = wave % a.strips;
    const int seg = wave / a.strips;
    const int j = strip * kStrip - 2 + lane;
    const bool cv = j >= 0 && j < a.W;
    const float mx = (j < a.W - 1) ? 1.f : 0.f;          // [j < W-1]
    const float mxl = (j > 0) ? 1.f : 0.f;               // [j > 0]
    const bool store_col = cv && lane >= 2 && lane <= 62;
    const int y0 = seg * R;
    const int y1 = min(y0 + R, a.H);
    const float inv_atc = 1.f / (fmaxf(*a.at, 1e-12f) * a.c);   // a~ >= ||M_s|| (Prop. 3.1), floored
    const float c = a.c, inv_ac = a.inv_ac, beta = a.beta;

    // values of row r - 1 (and y+ of row r - 2) carried between steps
    float q1x_p = 0.f, q1y_p = 0.f, q2x_p = 0.f, q2y_p = 0.f, gu_p = 0.f, gv_p = 0.f;
    float u_p = 0.f, v_p = 0.f, s_p = 0.f, Ix_p = 0.f, Iy_p = 0.f, It_p = 0.f;
    float n1y_pp = 0.f, n2y_pp = 0.f;
    float px_p = 0.f, py_p = 0.f, gw_p = 0.f, w_p = 0.f, npy_pp = 0.f;

    // every row the strip needs (y0 - 2 .. y0 + R) is loaded before any arithmetic, so a strip
    // costs one memory round trip instead of one per row
    Row<HAS_W> rows[R + 3];
#pragma unroll
    for (int k = 0; k < R + 3; ++k) load_row<HAS_W, REL>(a, y0 - 2 + k, j, cv, y0, y1, rows[k]);
#pragma unroll
    for (int k = 0; k < R + 3; ++k) {
        const int r = y0 - 2 + k;
        const Row<HAS_W>& cur = rows[k];
        const float my = (r < a.H - 1) ? 1.f : 0.f;
        const float myl = (r > 0) ? 1.f : 0.f;

        // g at row r
        const float q1x_l = __shfl_up(cur.q1x, 1);
        const float q2x_l = __shfl_up(cur.q2x, 1);
        const float dq1 = mx * cur.q1x - mxl * q1x_l + my * cur.q1y - myl * q1y_p;
        const float dq2 = mx * cur.q2x - mxl * q2x_l + my * cur.q2y - myl * q2y_p;
        // increment form: the multiplier is u0 + u, and only its gradient enters the dual step
        float gu = cur.u + c * (dq1 - cur.Ix * cur.s);
        float gv = cur.v + c * (dq2 - cur.Iy * cur.s);
        if constexpr (REL) {
            gu += cur.u0;
            gv += cur.v0;
        }
        float gw = 0.f;
        if constexpr (HAS_W) {
            const float px_l = __shfl_up(cur.px, 1);
            const float dp = mx * cur.px - mxl * px_l + my * cur.py - myl * py_p;
            gw = cur.w + c * (dp - beta * cur.s);
        }

        if (r >= y0) {
            // y+ at row r - 1
            const int rm = r - 1;
            const float my1 = (rm < a.H - 1) ? 1.f : 0.f;
            const float gu_r = __shfl_down(gu_p, 1);
            const float gv_r = __shfl_down(gv_p, 1);
            const float t1x = q1x_p + mx * (gu_r - gu_p) * inv_ac;
            const float t1y = q1y_p + my1 * (gu - gu_p) * inv_ac;
            const float t2x = q2x_p + mx * (gv_r - gv_p) * inv_ac;
            const float t2y = q2y_p + my1 * (gv - gv_p) * inv_ac;
            const float nq = t1x * t1x + t1y * t1y + t2x * t2x + t2y * t2y;
            const float sq = nq > 1.f ? rsqrtf(nq) : 1.f;
            const float n1x = t1x * sq, n1y = t1y * sq, n2x = t2x * sq, n2y = t2y * sq;
            float npx = 0.f, npy = 0.f;
            if constexpr (HAS_W) {
                const float gw_r = __shfl_down(gw_p, 1);
                const float tpx = px_p + mx * (gw_r - gw_p) * inv_ac;
                const float tpy = py_p + my1 * (gw - gw_p) * inv_ac;
                const float np2 = tpx * tpx + tpy * tpy;
                const float sp = np2 > 1.f ? rsqrtf(np2) : 1.f;
                npx = tpx * sp;
                npy = tpy * sp;
            }
            const float n1x_l = __shfl_up(n1x, 1);
            const float n2x_l = __shfl_up(n2x, 1);
            float npx_l = 0.f;
            if constexpr (HAS_W) npx_l = __shfl_up(npx, 1);
            if (r >= y0 + 1 && rm < y1) {
                // output at row r - 1 (all inputs of that row are in the *_p registers)
                const float myl1 = (rm > 0) ? 1.f : 0.f;
                const float dn1 = mx * n1x - mxl * n1x_l + my1 * n1y - myl1 * n1y_pp;
                const float dn2 = mx * n2x - mxl * n2x_l + my1 * n2y - myl1 * n2y_pp;
                const float hu = u_p + a.c_rho_s * (dn1 - Ix_p * s_p);
                const float hv = v_p + a.c_rho_s * (dn2 - Iy_p * s_p);
                float acc = It_p + Ix_p * hu + Iy_p * hv;
                float dnp = 0.f;
                if constexpr (HAS_W) {
                    dnp = mx * npx - mxl * npx_l + my1 * npy - myl1 * npy_pp;
                    const float hw = w_p + a.c_rho_s * (dnp - beta * s_p);
                    acc += beta * hw;
                }
                float sn = s_p + acc * inv_atc;
                sn = fminf(fmaxf(sn, -a.lam), a.lam);
                const float ms = a.cB * sn - a.cC * s_p;
                const float un = u_p + a.cA * dn1 - Ix_p * ms;
                const float vn = v_p + a.cA * dn2 - Iy_p * ms;
                if (store_col) {
                    const int64_t off = (int64_t)rm * a.ld + j;
                    a.uo[off] = un;
                    a.vo[off] = vn;
                    a.so[off] = sn;
                    a.q1xo[off] = n1x;
                    a.q1yo[off] = n1y;
                    a.q2xo[off] = n2x;
                    a.q2yo[off] = n2y;
                    if constexpr (HAS_W) {
                        a.wo[off] = w_p + a.cA * dnp - beta * ms;
                        a.pxo[off] = npx;
                        a.pyo[off] = npy;
                    }
                }
            }
            n1y_pp = n1y;
            n2y_pp = n2y;
            npy_pp = npy;
        }
        q1x_p = cur.q1x; q1y_p = cur.q1y; q2x_p = cur.q2x; q2y_p = cur.q2y;
        gu_p = gu; gv_p = gv;
        u_p = cur.u; v_p = cur.v; s_p = cur.s; Ix_p = cur.Ix; Iy_p = cur.Iy; It_p = cur.It;
        if constexpr (HAS_W) { px_p = cur.px; py_p = cur.py; gw_p = gw; w_p = cur.w; }
    }
}

}  // namespace



template <int R>
static void launch_rows(const AdmmIterArgs& b, const AdmmGeometry& g, bool has_w, bool rel, hipStream_t s) {
    if (has_w && rel) hipLaunchKernelGGL((admm_iter_kernel<true, true, R>), dim3(g.blocks), dim3(256), 0, s, b);
    else if (has_w) hipLaunchKernelGGL((admm_iter_kernel<true, false, R>), dim3(g.blocks), dim3(256), 0, s, b);
    else if (rel) hipLaunchKernelGGL((admm_iter_kernel<false, true, R>), dim3(g.blocks), dim3(256), 0, s, b);
    else hipLaunchKernelGGL((admm_iter_kernel<false, false, R>), dim3(g.blocks), dim3(256), 0, s, b);
}

void launch_admm_iter(const AdmmIterArgs& a, bool has_w, hipStream_t s) {
    const AdmmGeometry g = admm_geometry(a.H, a.W, a.rows);
    AdmmIterArgs b = a;
    b.rows = g.rows;
    b.strips = g.strips;
    b.segs = g.segs;
    const bool rel = a.u0 != nullptr;
    if (g.rows == 8) launch_rows<8>(b, g, has_w, rel, s);
    else if (g.rows == 4) launch_rows<4>(b, g, has_w, rel, s);
    else launch_rows<2>(b, g, has_w, rel, s);
}

}  // namespace flowmi
