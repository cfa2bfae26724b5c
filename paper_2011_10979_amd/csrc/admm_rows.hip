// Temporally blocked iterations of the preconditioned dual ADMM family (Sec. 3.1.1) on tiles one
// wavefront wide: the register-resident form of the K-iteration tiles.
//
// The extended region (output tile plus the halo of K + 1 rows / columns above and to the left and
// K below and to the right, clipped to the image) is at most 64 columns wide and NW * R rows high.
// Wavefront w of the work-group holds rows w R .. w R + R - 1 of it, lane l column l, and keeps every
// field of its R pixels per lane in registers for the whole launch.  The discrete operators of
// Sec. 2.2 then find their neighbours without memory: left / right in the adjacent lane (a whole-
// wavefront DPP shift), up / down in the thread's neighbouring row, and only across the boundary
// between two wavefronts in LDS, which holds one row of g (each wavefront's top row, read by the
// wavefront above for its gradient) and one row of the dual's y components (each wavefront's bottom
// row, read by the wavefront below for its divergence).
//
// The iteration is the one of the general tile kernels, with the same operations in the same order,
// so the two give bitwise the same iterates:  A: g from div q;  barrier;  B: y+ = P(y + grad g /
// (a c));  barrier;  C: div y+, s+, multipliers, then A of the next iteration.  The coefficients of
// Sec. 2.2 (a neighbour exists in the image) are per lane for the horizontal differences and per row,
// so wavefront-uniform, for the vertical ones.  A neighbour outside the extended region reads zero or
// an unrelated finite value, which only changes halo pixels the halo accounts for, and a row outside
// the band that can still reach the output tile skips the iteration, as in the general kernels.
#include "kernels.hpp"

namespace flowmi {

namespace {

// lane l receives lane l + 1's value (lane 63: 0), and lane l - 1's (lane 0: 0)
__device__ __forceinline__ float from_right(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_left(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x138, 0xf, 0xf, false));
}

// the planes live in global memory: loads and stores through the global address space (pointers read
// from a descriptor table would otherwise be flat, whose loads also hold the LDS counter)
using gfloat = __attribute__((address_space(1))) float;
__device__ __forceinline__ float gload(const float* p, int64_t o) { return ((const gfloat*)p)[o]; }
__device__ __forceinline__ void gstore(float* p, int64_t o, float v) { ((gfloat*)p)[o] = v; }

// a level descriptor of the tile table, read through the constant address space: the table does
// not change while a launch runs, so its pointers load into scalar registers (read as ordinary
// global memory they would be vector loads, their values held in vector registers)
__device__ __forceinline__ TbLevel level_scalar(const TbLevel* p) {
    using CL = const __attribute__((address_space(4))) TbLevel;
    CL* q = (CL*)p;
    TbLevel L;
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        L.in[i] = q->in[i];
        L.out[i] = q->out[i];
    }
    L.Ix = q->Ix;
    L.Iy = q->Iy;
    L.It = q->It;
    L.u0 = q->u0;
    L.v0 = q->v0;
    L.at = q->at;
    L.H = q->H;
    L.W = q->W;
    L.ld = q->ld;
    return L;
}

template <bool HAS_W, int NW>
struct RowLds {
    static constexpr int NG = HAS_W ? 3 : 2;
    // [f][w + 1][lane]: g_f of wavefront w's top row / y component f (q1y, q2y, p_y) of its bottom row;
    // entries 0 and NW + 1 stand for the rows beyond the work-group and stay zero
    float gtop[NG][NW + 2][64];
    float ybot[NG][NW + 2][64];
};

// IN: the extended region lies inside the image's interior (no image edge in it), so every
// neighbour-exists coefficient of the discrete operators is 1 and their products drop out (the same
// arithmetic: a product by 1 is exact)
template <bool HAS_W, int NW, int R, bool BAND, bool IN>
__device__ __forceinline__ void process_rows(const TbArgs& a, const TbTile& T, const TbLevel& L, RowLds<HAS_W, NW>& S) {
    constexpr int NG = HAS_W ? 3 : 2, NQ = HAS_W ? 6 : 4;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const float c = a.c, inv_ac = a.inv_ac, beta = a.beta, crs = a.c_rho_s;
    const int H = L.H, W = L.W;
    const int64_t ld = L.ld;
    const int K = a.K;
    const int ey0 = max(T.y0 - tb_halo_lo(K), 0), ex0 = max(T.x0 - tb_halo_lo(K), 0);
    const int ey1 = min(T.y0 + T.th + K, H), ex1 = min(T.x0 + T.tw + K, W);
    const int EW = ex1 - ex0, EH = ey1 - ey0;          // at most 64 and NW R (the planners' bound)
    const float inv_atc = 1.f / (fmaxf(gload(L.at, a.at_slot), 1e-12f) * c);
    const int gj = ex0 + lane;
    const float fx = IN || gj < W - 1 ? 1.f : 0.f, fl = IN || gj > 0 ? 1.f : 0.f;
    const float cx = IN ? inv_ac : fx * inv_ac;
    const int shr_top = ey0 > 0, shr_bot = ey1 < H;
    const bool band = BAND && (shr_top || shr_bot);

    float du[R], dv[R], ss[R], Ix[R], Iy[R], It[R], u0[R], v0[R], ww[R];
    float qo[NQ][R], go[NG][R];
    float fy[R], fu[R], cy[R];                          // wavefront-uniform
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = wv * R + k, gi = ey0 + r;
        fy[k] = IN || gi < H - 1 ? 1.f : 0.f;
        fu[k] = IN || gi > 0 ? 1.f : 0.f;
        cy[k] = IN ? inv_ac : fy[k] * inv_ac;
        du[k] = dv[k] = ss[k] = Ix[k] = Iy[k] = It[k] = u0[k] = v0[k] = ww[k] = 0.f;
#pragma unroll
        for (int f = 0; f < NQ; ++f) qo[f][k] = 0.f;
#pragma unroll
        for (int f = 0; f < NG; ++f) go[f][k] = 0.f;
        if (r < EH && lane < EW) {
            const int64_t o = (int64_t)gi * ld + gj;
            qo[0][k] = gload(L.in[5], o);
            qo[1][k] = gload(L.in[6], o);
            qo[2][k] = gload(L.in[7], o);
            qo[3][k] = gload(L.in[8], o);
            du[k] = gload(L.in[1], o);
            dv[k] = gload(L.in[2], o);
            ss[k] = gload(L.in[9], o);
            Ix[k] = gload(L.Ix, o);
            Iy[k] = gload(L.Iy, o);
            It[k] = gload(L.It, o);
            u0[k] = gload(L.u0, o);
            v0[k] = gload(L.v0, o);
            if constexpr (HAS_W) {
                qo[4][k] = gload(L.in[3], o);
                qo[5][k] = gload(L.in[4], o);
                ww[k] = gload(L.in[0], o);
            }
        }
    }
#pragma unroll
    for (int f = 0; f < NG; ++f) S.ybot[f][wv + 1][lane] = qo[2 * f + 1][R - 1];
    if (wv == 0) {
#pragma unroll
        for (int f = 0; f < NG; ++f) {
            S.gtop[f][0][lane] = S.gtop[f][NW + 1][lane] = 0.f;
            S.ybot[f][0][lane] = S.ybot[f][NW + 1][lane] = 0.f;
        }
    }
    __syncthreads();

    // divergence of dual field f (0: q1, 1: q2, 2: p) at row k:
    // [j < W-1] ax(i,j) - [j > 0] ax(i,j-1) + [i < H-1] ay(i,j) - [i > 0] ay(i-1,j)
    auto divf = [&](int f, int k) {
        const float ax = qo[2 * f][k], ay = qo[2 * f + 1][k];
        const float al = from_left(ax);
        const float au = k > 0 ? qo[2 * f + 1][k > 0 ? k - 1 : 0] : S.ybot[f][wv][lane];
        float d = fmaf(fx, ax, -(fl * al));
        d = fmaf(fy[k], ay, d);
        return fmaf(-fu[k], au, d);
    };
    auto g_out = [&](int k, float dq1, float dq2, float dp) {
        go[0][k] = u0[k] + (du[k] + c * (dq1 - Ix[k] * ss[k]));
        go[1][k] = v0[k] + (dv[k] + c * (dq2 - Iy[k] * ss[k]));
        if constexpr (HAS_W) go[2][k] = ww[k] + c * (dp - beta * ss[k]);
        if (k == 0) {
#pragma unroll
            for (int f = 0; f < NG; ++f) S.gtop[f][wv + 1][lane] = go[f][0];
        }
    };
    // phase B at row k: y+ = P(y + grad g / (a c))
    auto phase_b = [&](int k) {
        float gr[NG], gd[NG];
#pragma unroll
        for (int f = 0; f < NG; ++f) {
            gr[f] = from_right(go[f][k]);
            gd[f] = k + 1 < R ? go[f][k + 1 < R ? k + 1 : k] : S.gtop[f][wv + 2][lane];
        }
        const float t1x = fmaf(gr[0] - go[0][k], cx, qo[0][k]);
        const float t1y = fmaf(gd[0] - go[0][k], cy[k], qo[1][k]);
        const float t2x = fmaf(gr[1] - go[1][k], cx, qo[2][k]);
        const float t2y = fmaf(gd[1] - go[1][k], cy[k], qo[3][k]);
        // sums of products as explicit FMA chains: every tile kernel rounds them alike
        const float nq = fmaf(t2y, t2y, fmaf(t2x, t2x, fmaf(t1y, t1y, t1x * t1x)));
        // projection scale min(1, 1/|t|): the hardware reciprocal square root is at least 1 (or
        // infinite) wherever |t| <= 1, so the min alone selects
        const float sc = fminf(1.f, __builtin_amdgcn_rsqf(nq));
        qo[0][k] = t1x * sc;
        qo[1][k] = t1y * sc;
        qo[2][k] = t2x * sc;
        qo[3][k] = t2y * sc;
        if constexpr (HAS_W) {
            const float tpx = fmaf(gr[NG - 1] - go[NG - 1][k], cx, qo[4][k]);
            const float tpy = fmaf(gd[NG - 1] - go[NG - 1][k], cy[k], qo[5][k]);
            const float np2 = fmaf(tpy, tpy, tpx * tpx);
            const float sp = fminf(1.f, __builtin_amdgcn_rsqf(np2));
            qo[4][k] = tpx * sp;
            qo[5][k] = tpy * sp;
        }
        if (k == R - 1) {
#pragma unroll
            for (int f = 0; f < NG; ++f) S.ybot[f][wv + 1][lane] = qo[2 * f + 1][k];
        }
    };
    // phase C at row k: div y+, s+, multipliers, then phase A of the next iteration
    auto phase_c = [&](int k, bool next) {
        const float dn1 = divf(0, k), dn2 = divf(1, k);
        const float hu_ = du[k] + crs * (dn1 - Ix[k] * ss[k]);
        const float hv_ = dv[k] + crs * (dn2 - Iy[k] * ss[k]);
        float acc = It[k] + Ix[k] * hu_ + Iy[k] * hv_;
        float dnp = 0.f;
        if constexpr (HAS_W) {
            dnp = divf(2, k);
            acc += beta * (ww[k] + crs * (dnp - beta * ss[k]));
        }
        float sn = ss[k] + acc * inv_atc;
        sn = __builtin_amdgcn_fmed3f(sn, -a.lam, a.lam);
        const float ms = fmaf(a.cB, sn, -(a.cC * ss[k]));
        du[k] = du[k] + a.cA * dn1 - Ix[k] * ms;
        dv[k] = dv[k] + a.cA * dn2 - Iy[k] * ms;
        if constexpr (HAS_W) ww[k] = ww[k] + a.cA * dnp - beta * ms;
        ss[k] = sn;
        if (next) g_out(k, dn1, dn2, dnp);
    };

    // phase A at the start, every row
#pragma unroll
    for (int k = 0; k < R; ++k) {
        float dp = 0.f;
        if constexpr (HAS_W) dp = divf(2, k);
        g_out(k, divf(0, k), divf(1, k), dp);
    }
    // one iteration; the last one (NEXT false) is its own copy, so that no select on "is there a next
    // iteration" runs per row in the others
    auto iteration = [&](int it, auto next) {
        // rows that can still reach the output tile (all rows of the region without the band)
        const int lo = band ? shr_top * (it + 1) : 0, hi = band ? EH - shr_bot * (it + 1) : EH;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int r = wv * R + k;
            if (r >= lo && r < hi) phase_b(k);
        }
        __syncthreads();
        // the same rows, from bounds re-read as scalars: a row condition kept across the barrier
        // would live as a lane mask and cost vector instructions per row
        const int lo_c = __builtin_amdgcn_readfirstlane(lo), hi_c = __builtin_amdgcn_readfirstlane(hi);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int r = wv * R + k;
            if (r >= lo_c && r < hi_c) phase_c(k, decltype(next)::value);
        }
    };
    for (int it = 0; it + 1 < K; ++it) iteration(it, std::true_type{});
    if (K > 0) iteration(K - 1, std::false_type{});

    // write the output tile
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = wv * R + k, gi = ey0 + r;
        if (r >= EH || gi < T.y0 || gi >= T.y0 + T.th) continue;
        if (lane >= EW || gj < T.x0 || gj >= T.x0 + T.tw) continue;
        const int64_t o = (int64_t)gi * ld + gj;
        gstore(L.out[1], o, du[k]);
        gstore(L.out[2], o, dv[k]);
        gstore(L.out[9], o, ss[k]);
        gstore(L.out[5], o, qo[0][k]);
        gstore(L.out[6], o, qo[1][k]);
        gstore(L.out[7], o, qo[2][k]);
        gstore(L.out[8], o, qo[3][k]);
        if constexpr (HAS_W) {
            gstore(L.out[0], o, ww[k]);
            gstore(L.out[3], o, qo[4][k]);
            gstore(L.out[4], o, qo[5][k]);
        }
    }
}

// the tile's extended region, as process_rows clips it, holds no image edge
__device__ __forceinline__ bool region_interior(const TbArgs& a, const TbTile& T, const TbLevel& L) {
    return T.y0 - tb_halo_lo(a.K) > 0 && T.x0 - tb_halo_lo(a.K) > 0 && T.y0 + T.th + a.K < L.H && T.x0 + T.tw + a.K < L.W;
}

template <bool HAS_W, int NW, int R>
__device__ __forceinline__ void process_rows_banded(const TbArgs& a, const TbTile& T, const TbLevel& L, RowLds<HAS_W, NW>& S) {
    if (region_interior(a, T, L)) process_rows<HAS_W, NW, R, true, true>(a, T, L, S);
    else process_rows<HAS_W, NW, R, true, false>(a, T, L, S);
}

// Wavefronts per SIMD each shape asks the register allocator to allow: 8 (64 VGPRs, two 1024-thread
// work-groups per CU) where the rows fit, else 4.
template <bool HAS_W, int R>
constexpr int rows_waves_per_simd() { return (!HAS_W && R <= 3) ? 8 : 4; }

__device__ __forceinline__ int xcd_tile_r(int b, int nb) {
    const int per = nb >> 3;   // host pads the grid to a multiple of 8
    return (b & 7) * per + (b >> 3);
}

template <bool HAS_W, int NW, int R, bool BAND>
__global__ __launch_bounds__(NW * 64, (rows_waves_per_simd<HAS_W, R>())) void admm_rows_direct_kernel(TbArgs a) {
    __shared__ RowLds<HAS_W, NW> S;
    const int t = xcd_tile_r(blockIdx.x, gridDim.x);
    if (t >= a.ntiles) return;
    TbTile T;
    T.level = 0;
    const int ty = t / a.ntx, tx = t - ty * a.ntx;
    T.y0 = ty * a.th;
    T.x0 = tx * a.tw;
    T.th = min(a.th, a.lvl.H - T.y0);
    T.tw = min(a.tw, a.lvl.W - T.x0);
    if constexpr (BAND) process_rows_banded<HAS_W, NW, R>(a, T, a.lvl, S);
    else process_rows<HAS_W, NW, R, false, false>(a, T, a.lvl, S);
}

// Many levels (batched pairs), table order: tile entries split into 8 contiguous runs, one per XCD.
template <bool HAS_W, int NW, int R>
__global__ __launch_bounds__(NW * 64, (rows_waves_per_simd<HAS_W, R>())) void admm_rows_table_kernel(TbArgs a) {
    __shared__ RowLds<HAS_W, NW> S;
    const int n = a.ntiles_dev ? *a.ntiles_dev : a.ntiles;
    const int per = (n + 7) >> 3;
    const int x = blockIdx.x & 7, y = blockIdx.x >> 3;
    const int t = x * per + y;
    if (y >= per || t >= n) return;
    const TbTile T = a.tiles[t];
    const TbLevel L = level_scalar(a.levels + (2 * T.level + a.dir));
    process_rows_banded<HAS_W, NW, R>(a, T, L, S);
}

template <bool HAS_W, int NW, int R>
void launch_rows_shape(const TbArgs& a, int grid, hipStream_t s) {
    if (a.tiles) {
        hipLaunchKernelGGL((admm_rows_table_kernel<HAS_W, NW, R>), dim3(grid), dim3(NW * 64), 0, s, a);
    } else if (a.ntiles == 1 && a.th >= a.lvl.H && a.tw >= a.lvl.W) {
        hipLaunchKernelGGL((admm_rows_direct_kernel<HAS_W, NW, R, false>), dim3(grid), dim3(NW * 64), 0, s, a);
    } else {
        hipLaunchKernelGGL((admm_rows_direct_kernel<HAS_W, NW, R, true>), dim3(grid), dim3(NW * 64), 0, s, a);
    }
}

}  // namespace

void launch_admm_rows(const TbArgs& a, bool has_w, int nt, int grid, hipStream_t s) {
    grid = (grid + 7) / 8 * 8;
    if (nt == 2049) {
        if (has_w) launch_rows_shape<true, 16, 2>(a, grid, s);
        else launch_rows_shape<false, 16, 2>(a, grid, s);
    } else if (nt == 3073) {
        if (has_w) launch_rows_shape<true, 16, 3>(a, grid, s);
        else launch_rows_shape<false, 16, 3>(a, grid, s);
    } else if (nt == 4097) {
        if (has_w) launch_rows_shape<true, 16, 4>(a, grid, s);
        else launch_rows_shape<false, 16, 4>(a, grid, s);
    }
}

}  // namespace flowmi
