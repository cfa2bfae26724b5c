// FP64 energy, dual objective, dual gap and feasibility residual of one warp's linearised problem.
//
//   E = sum |grad d| (4-component, coupled) [+ sum |grad w|] + lambda sum |rho|   (eq:l1:finite)
//   D = sum I_t s                                                               (eq:dual:l1:flow:cons)
//   r = A s + B y = (beta s - div p, I_x s - div q1, I_y s - div q2)           (eq:dual:l1:flow:constaint)
// plus G_TV = sum(|grad d| - <grad d, q>), G_data = sum(lambda |rho| - rho s) and <Lambda, r>, whose
// sum equals E - D.  Per-pixel terms are formed in FP32 and accumulated in FP64: per thread over a
// fixed grid-stride set of pixels, across the wavefront with lane shuffles, across the block in
// LDS, and over blocks by a second one-block kernel in a fixed order, so the result is bitwise
// reproducible for a given shape.
#include "kernels.hpp"

namespace flowmi {

namespace {

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Partial sums of work-group `blk` of `nblk` (grid-stride over the pixels) into a.partial[blk].
__device__ __forceinline__ void energy_body(const EnergyArgs& a, int blk, int nblk) {
    double acc[kEnergyTerms];
#pragma unroll
    for (int k = 0; k < kEnergyTerms; ++k) acc[k] = 0.0;
    const bool has_w = a.beta != 0.f;
    const int64_t npix = (int64_t)a.H * a.W;
    const float tau = a.pdr_tau;
    const bool small = npix < ((int64_t)1 << 31);   // 32-bit index arithmetic (64-bit division is slow)
    for (int64_t idx = (int64_t)blk * 256 + threadIdx.x; idx < npix; idx += (int64_t)nblk * 256) {
        int i, j;
        if (small) {
            i = (int)((uint32_t)idx / (uint32_t)a.W);
            j = (int)idx - i * a.W;
        } else {
            i = (int)(idx / a.W);
            j = (int)(idx % a.W);
        }
        const int64_t o = (int64_t)i * a.ld + j;
        const bool hr = j < a.W - 1, hd = i < a.H - 1, hl = j > 0, hu = i > 0;
        // flow value at a cell: u, or u + du when the flow is given as base + increment
        auto U = [&](int64_t oo) { return a.du ? a.u[oo] + a.du[oo] : a.u[oo]; };
        auto V = [&](int64_t oo) { return a.dv ? a.v[oo] + a.dv[oo] : a.v[oo]; };
        auto W = [&](int64_t oo) { return a.w[oo]; };
        // forward differences of a field at (i, j), (i, j-1) [x part] and (i-1, j) [y part]
        auto gx = [&](auto f, int64_t oo, bool ok) { return ok ? f(oo + 1) - f(oo) : 0.f; };
        auto gy = [&](auto f, int64_t oo, bool ok) { return ok ? f(oo + a.ld) - f(oo) : 0.f; };
        // dual value at a cell: q itself, or y bar + tau grad X for pDR
        auto dual_x = [&](const float* qx, auto f, int64_t oo, bool ok_r) {
            return tau > 0.f ? qx[oo] + tau * gx(f, oo, ok_r) : qx[oo];
        };
        auto dual_y = [&](const float* qy, auto f, int64_t oo, bool ok_d) {
            return tau > 0.f ? qy[oo] + tau * gy(f, oo, ok_d) : qy[oo];
        };
        const float u = U(o), v = V(o), s = a.s[o];
        const float ux = gx(U, o, hr), uy = gy(U, o, hd), vx = gx(V, o, hr), vy = gy(V, o, hd);
        const float q1x = dual_x(a.q1x, U, o, hr), q1y = dual_y(a.q1y, U, o, hd);
        const float q2x = dual_x(a.q2x, V, o, hr), q2y = dual_y(a.q2y, V, o, hd);
        // div q at (i, j): [j<W-1] qx(i,j) - [j>0] qx(i,j-1) + [i<H-1] qy(i,j) - [i>0] qy(i-1,j)
        const float q1x_l = hl ? dual_x(a.q1x, U, o - 1, true) : 0.f;
        const float q2x_l = hl ? dual_x(a.q2x, V, o - 1, true) : 0.f;
        const float q1y_u = hu ? dual_y(a.q1y, U, o - a.ld, true) : 0.f;
        const float q2y_u = hu ? dual_y(a.q2y, V, o - a.ld, true) : 0.f;
        const float dq1 = (hr ? q1x : 0.f) - q1x_l + (hd ? q1y : 0.f) - q1y_u;
        const float dq2 = (hr ? q2x : 0.f) - q2x_l + (hd ? q2y : 0.f) - q2y_u;
        const float Ix = a.Ix[o], Iy = a.Iy[o], It = a.It[o];
        const float nd = sqrtf(ux * ux + uy * uy + vx * vx + vy * vy);
        float tv = nd;
        float gtv = nd - (ux * q1x + uy * q1y + vx * q2x + vy * q2y);
        float w = 0.f;
        float rw = 0.f;
        if (has_w) {
            w = a.w[o];
            const float wx = gx(W, o, hr), wy = gy(W, o, hd);
            const float pxv = dual_x(a.px, W, o, hr), pyv = dual_y(a.py, W, o, hd);
            const float px_l = hl ? dual_x(a.px, W, o - 1, true) : 0.f;
            const float py_u = hu ? dual_y(a.py, W, o - a.ld, true) : 0.f;
            const float dp = (hr ? pxv : 0.f) - px_l + (hd ? pyv : 0.f) - py_u;
            const float nw = sqrtf(wx * wx + wy * wy);
            tv += nw;
            gtv += nw - (wx * pxv + wy * pyv);
            rw = a.beta * s - dp;
        }
        float du = u, dv = v;                 // displacement entering rho (relative I_t: from d0)
        if (a.du) { du = a.du[o]; dv = a.dv[o]; }
        else if (a.lu0) { du = u - a.lu0[o]; dv = v - a.lv0[o]; }
        const float rho = It + a.beta * w + Ix * du + Iy * dv;
        const float data = a.lam * fabsf(rho);
        const float ru = Ix * s - dq1, rv = Iy * s - dq2;
        acc[0] += (double)tv;
        acc[1] += (double)data;
        // the dual objective takes the absolute I_t of the warp's linearised problem
        double It_abs = (double)It;
        if (a.du) It_abs -= (double)Ix * a.u[o] + (double)Iy * a.v[o];
        else if (a.lu0) It_abs -= (double)Ix * a.lu0[o] + (double)Iy * a.lv0[o];
        acc[2] += It_abs * (double)s;
        acc[3] += (double)ru * ru + (double)rv * rv + (double)rw * rw;
        acc[4] += (double)gtv;
        acc[5] += (double)data - (double)rho * (double)s;
        acc[6] += (double)u * ru + (double)v * rv + (double)w * rw;
        const float chk = tv + data + rho + s + u + v + w;
        if (!isfinite(chk)) acc[7] += 1.0;
    }
    __shared__ double sm[4][kEnergyTerms];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kEnergyTerms; ++k) {
        const double t = wave_sum(acc[k]);
        if (lane == 0) sm[wid][k] = t;
    }
    __syncthreads();
    if (threadIdx.x < kEnergyTerms) {
        const int k = threadIdx.x;
        a.partial[blk * kEnergyTerms + k] = ((sm[0][k] + sm[1][k]) + sm[2][k]) + sm[3][k];
    }
}

__global__ __launch_bounds__(256) void energy_kernel(EnergyArgs a) { energy_body(a, blockIdx.x, gridDim.x); }

// Sum of the per-block partials (a separate launch: the kernel boundary makes the partials
// visible without any fence).  Thread t adds partials t, t + 256, ... in order, then a fixed
// pairwise tree in LDS combines the 256 sums, so the result is reproducible bit for bit.
__device__ __forceinline__ void energy_final_body(const double* __restrict__ partial, int nblocks,
                                                  double* __restrict__ out) {
    // every term at once: thread t adds the partials of blocks t, t + 256, ... in order, then one
    // fixed pairwise tree over the threads (the same order for every term)
    __shared__ double sm[kEnergyTerms][256];
    double t[kEnergyTerms];
#pragma unroll
    for (int k = 0; k < kEnergyTerms; ++k) t[k] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) {
#pragma unroll
        for (int k = 0; k < kEnergyTerms; ++k) t[k] += partial[b * kEnergyTerms + k];
    }
#pragma unroll
    for (int k = 0; k < kEnergyTerms; ++k) sm[k][threadIdx.x] = t[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int k = 0; k < kEnergyTerms; ++k) sm[k][threadIdx.x] += sm[k][threadIdx.x + w];
        }
        __syncthreads();
    }
    if ((int)threadIdx.x < kEnergyTerms) out[threadIdx.x] = sm[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void energy_final_kernel(const double* __restrict__ partial, int nblocks,
                                                          double* __restrict__ out) {
    energy_final_body(partial, nblocks, out);
}

// Batched: item k owns work-groups [off[k], off[k+1]) of the first kernel (as many as its own
// single launch would use, so each pair's sums are formed in the same order as in a plain solve)
// and work-group k of the second.
__device__ __forceinline__ int find_item_e(const int* __restrict__ off, int n, int b) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void energy_batched_kernel(const EnergyArgs* __restrict__ items,
                                                            const int* __restrict__ off, int n) {
    const int k = find_item_e(off, n, blockIdx.x);
    const EnergyArgs a = items[k];
    energy_body(a, blockIdx.x - off[k], off[k + 1] - off[k]);
}

__global__ __launch_bounds__(256) void energy_final_batched_kernel(const EnergyArgs* __restrict__ items,
                                                                  const int* __restrict__ off) {
    const int k = blockIdx.x;
    energy_final_body(items[k].partial, off[k + 1] - off[k], items[k].out);
}

}  // namespace


void launch_energy(const EnergyArgs& a, hipStream_t s) {
    const int blocks = energy_blocks(a.H, a.W);
    hipLaunchKernelGGL(energy_kernel, dim3(blocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(energy_final_kernel, dim3(1), dim3(256), 0, s, (const double*)a.partial, blocks, a.out);
}

void launch_energy_batched(const EnergyArgs* items, const int* off, int n, int total_blocks, hipStream_t s) {
    if (n <= 0 || total_blocks <= 0) return;
    hipLaunchKernelGGL(energy_batched_kernel, dim3(total_blocks), dim3(256), 0, s, items, off, n);
    hipLaunchKernelGGL(energy_final_batched_kernel, dim3(n), dim3(256), 0, s, items, off);
}

}  // namespace flowmi
