// Coarse-to-fine framework kernels (Sec. 4 runs the solvers inside a standard coarse-to-fine
// warping pyramid; the filters below are this library's choice, the paper names none):
//   downsample   2x2 box mean with edge replication, ceil sizes (factor 1/2)
//   derivatives  central differences with replicated neighbours
//   linearize    bilinear warp of I1, D_x I1, D_y I1 at x + d0 and the linearisation
//                rho(d) = I_x u + I_y v + I_t (Sec. 1), plus a~ = max M_s (Prop. 3.1); it first
//                commits the previous warp's flow increment (u0 += du) at its own pixel
//   level_init   centre-aligned bilinear x2 upsampling of the flow, dual reset
//   copy         plane copies with format conversion (frame import, flow export)
// All are elementwise or gather kernels: one thread per output pixel, 64-wide rows per wavefront
// so that every plane access is a coalesced row segment.  Each body is written once and launched
// either for one plane set (grid = the plane's blocks) or batched over many plane sets in one launch,
// where a block-offset prefix maps each work-group to its item (no work-group is wasted).
#include "kernels.hpp"

namespace flowmi {

namespace {

template <typename T> __device__ __forceinline__ float ldv(const T* p, int64_t i);
template <> __device__ __forceinline__ float ldv<float>(const float* p, int64_t i) { return p[i]; }
template <> __device__ __forceinline__ float ldv<__half>(const __half* p, int64_t i) { return __half2float(p[i]); }
template <typename T> __device__ __forceinline__ void stv(T* p, int64_t i, float x);
template <> __device__ __forceinline__ void stv<float>(float* p, int64_t i, float x) { p[i] = x; }
template <> __device__ __forceinline__ void stv<__half>(__half* p, int64_t i, float x) { p[i] = __float2half(x); }

dim3 grid2d(int H, int W) { return dim3((W + 63) / 64, (H + 3) / 4); }

// ---------------------------------------------------------------------------------------------
// bodies: (bx, by) is the work-group's position in the item's grid of 64 x 4 blocks
// ---------------------------------------------------------------------------------------------
// Error-free sum of two floats (Knuth's TwoSum): s + e == a + b exactly, s = fl(a + b).
__device__ __forceinline__ float two_sum(float a, float b, float& e) {
    const float s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
    return s;
}

template <typename T>
__device__ __forceinline__ void downsample_body(const DownArgs& a, int bx, int by) {
    const int Hc = (a.H + 1) / 2, Wc = (a.W + 1) / 2;
    const int b = bx * 64 + (threadIdx.x & 63);
    const int r = by * 4 + (threadIdx.x >> 6);
    if (r >= Hc || b >= Wc) return;
    const T* src = (const T*)a.src;
    const int r0 = 2 * r, r1 = min(2 * r + 1, a.H - 1);
    const int c0 = 2 * b, c1 = min(2 * b + 1, a.W - 1);
    const int64_t o[4] = {(int64_t)r0 * a.ld + c0, (int64_t)r0 * a.ld + c1, (int64_t)r1 * a.ld + c0,
                          (int64_t)r1 * a.ld + c1};
    const int64_t od = (int64_t)r * a.ldd + b;
    if (a.dst_lo) {
        // float-float mean: the four high parts summed without error, the rounding errors and the
        // low parts collected in a second float, renormalised; the factor 1/4 is exact
        float e1, e2, e3;
        float hi = two_sum(ldv(src, o[0]), ldv(src, o[1]), e1);
        hi = two_sum(hi, ldv(src, o[2]), e2);
        hi = two_sum(hi, ldv(src, o[3]), e3);
        float lo = (e1 + e2) + e3;
        if (a.src_lo) lo += (a.src_lo[o[0]] + a.src_lo[o[1]]) + (a.src_lo[o[2]] + a.src_lo[o[3]]);
        float l;
        const float h = two_sum(hi, lo, l);
        stv((T*)a.dst, od, 0.25f * h);
        a.dst_lo[od] = 0.25f * l;
        return;
    }
    const float s = ldv(src, o[0]) + ldv(src, o[1]) + ldv(src, o[2]) + ldv(src, o[3]);
    stv((T*)a.dst, od, 0.25f * s);
}

template <typename T>
__device__ __forceinline__ void derivatives_body(const DerivArgs& a, int bx, int by) {
    const int j = bx * 64 + (threadIdx.x & 63);
    const int i = by * 4 + (threadIdx.x >> 6);
    if (i >= a.H || j >= a.W) return;
    const T* I = (const T*)a.I;
    const int64_t row = (int64_t)i * a.ld;
    const int W = a.W, H = a.H;
    const int64_t xr = row + min(j + 1, W - 1), xl = row + max(j - 1, 0);
    const int64_t yd = (int64_t)min(i + 1, H - 1) * a.ld + j, yu = (int64_t)max(i - 1, 0) * a.ld + j;
    float dx = ldv(I, xr) - ldv(I, xl);
    float dy = ldv(I, yd) - ldv(I, yu);
    if (a.I_lo) {   // float-float level: the low parts' difference completes the high parts'
        dx += a.I_lo[xr] - a.I_lo[xl];
        dy += a.I_lo[yd] - a.I_lo[yu];
    }
    dx *= 0.5f;
    dy *= 0.5f;
    stv((T*)a.Dx, (int64_t)i * a.ldd + j, dx);
    stv((T*)a.Dy, (int64_t)i * a.ldd + j, dy);
}

template <typename T>
__device__ __forceinline__ void copy_body(const CopyArgs& a, int bx, int by) {
    const int j = bx * 64 + (threadIdx.x & 63);
    const int i = by * 4 + (threadIdx.x >> 6);
    if (i >= a.H || j >= a.W) return;
    const int64_t o = (int64_t)i * a.lds + j;
    const float x = a.add ? a.src[o] + a.add[o] : a.src[o];
    stv((T*)a.dst, (int64_t)i * a.ldd + j, x - a.offset);
}

// Integer / fraction split of the sample position p + d clamped into [0, n-1]; keeps the
// fraction exact where p + d in FP32 would lose bits (|p| up to 2^11, ulp 1e-4 px).  The whole
// part is clamped to [-n, n] before the conversion, so a displacement that is NaN (max of NaN and
// -n is -n) or beyond the level converts to a defined integer and samples the border.  A NaN flow
// still reaches I_t (through -I_x u0 - I_y v0) and the state, and the energy check reports it.
__device__ __forceinline__ void split_pos(int p, float d, int n, int& i0, float& t) {
    const float fl = fminf(fmaxf(floorf(d), -(float)n), (float)n);
    t = d - fl;
    int ii = p + (int)fl;
    if (ii < 0) { ii = 0; t = 0.f; }
    else if (ii >= n - 1) { ii = n - 2; t = 1.f; }
    i0 = ii;
}

template <typename T>
__device__ __forceinline__ float bilin(const T* F, int64_t o00, int64_t ld, float ty, float tx) {
    const float f00 = ldv(F, o00), f01 = ldv(F, o00 + 1), f10 = ldv(F, o00 + ld), f11 = ldv(F, o00 + ld + 1);
    return (1.f - ty) * ((1.f - tx) * f00 + tx * f01) + ty * ((1.f - tx) * f10 + tx * f11);
}

__device__ __forceinline__ float wave_max(float x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o));
    return x;
}

template <typename T>
__device__ __forceinline__ void linearize_body(const LinArgs& a, int bx, int by) {
    const int j = bx * 64 + (threadIdx.x & 63);
    const T* I0 = (const T*)a.I0;
    const T* I1 = (const T*)a.I1;
    const T* Dx = (const T*)a.Dx;
    const T* Dy = (const T*)a.Dy;
    float ms = 0.f;
    const int i = by * kLinRows + (threadIdx.x >> 6);
    if (i < a.H && j < a.W) {
        const int64_t off = (int64_t)i * a.ld + j;
        float u0 = a.u0[off], v0 = a.v0[off];
        if (a.pend_u) {                       // commit the previous warp's increment
            u0 += a.pend_u[off];
            v0 += a.pend_v[off];
            a.u0[off] = u0;
            a.v0[off] = v0;
        }
        int iy, jx;
        float ty, tx;
        split_pos(i, v0, a.H, iy, ty);
        split_pos(j, u0, a.W, jx, tx);
        const int64_t o00 = (int64_t)iy * a.ld + jx;
        const float Ix = a.kappa * bilin(Dx, o00, a.ld, ty, tx);
        const float Iy = a.kappa * bilin(Dy, o00, a.ld, ty, tx);
        // I1(x + d0) - I0(x) as the bilinear mean of the four taps' differences to I0 (the weights
        // sum to one): the differences are small and formed before any rounding of a weighted sum
        // of values near 1/2, and on float-float levels they include the low parts
        const float i0 = ldv(I0, off);
        const int64_t ot[4] = {o00, o00 + 1, o00 + a.ld, o00 + a.ld + 1};
        float dt[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) dt[k] = ldv(I1, ot[k]) - i0;
        if (a.I1lo) {
            const float l0 = a.I0lo[off];
#pragma unroll
            for (int k = 0; k < 4; ++k) dt[k] += a.I1lo[ot[k]] - l0;
        }
        const float Ir = a.kappa * ((1.f - ty) * ((1.f - tx) * dt[0] + tx * dt[1]) + ty * ((1.f - tx) * dt[2] + tx * dt[3]));
        a.Ix[off] = Ix;
        a.Iy[off] = Iy;
        a.It[off] = a.rel ? Ir : Ir - Ix * u0 - Iy * v0;
        if (a.zero_u) { a.zero_u[off] = 0.f; a.zero_v[off] = 0.f; }
        if (a.keep_u) { a.keep_u[off] = u0; a.keep_v[off] = v0; }
        ms = a.beta * a.beta + Ix * Ix + Iy * Iy;
    }
    // a~ = max M_s: wave -> block -> one atomic max per block on the float's bit pattern (exact
    // and order-independent for non-negative values); the consumer applies the 1e-12 floor.
    __shared__ float smax[kLinRows];
    ms = wave_max(ms);
    if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = ms;
    __syncthreads();
    if (threadIdx.x == 0) {
        float bm = smax[0];
#pragma unroll
        for (int w = 1; w < kLinRows; ++w) bm = fmaxf(bm, smax[w]);
        atomicMax((unsigned int*)a.at, __float_as_uint(bm));
        if (a.at_clear && bx == 0 && by == 0) *a.at_clear = 0.f;
    }
}

// centre-aligned bilinear sample of a coarse plane (plus an optional increment plane D, added at
// each tap) at fine pixel (i, j): coarse coordinate i/2 - 1/4
__device__ __forceinline__ float up_sample(const float* F, int Hc, int Wc, int64_t ldc, int i, int j,
                                           const float* D = nullptr) {
    float y = 0.5f * (float)i - 0.25f;
    float x = 0.5f * (float)j - 0.25f;
    y = fminf(fmaxf(y, 0.f), (float)(Hc - 1));
    x = fminf(fmaxf(x, 0.f), (float)(Wc - 1));
    const int i0 = min((int)floorf(y), Hc - 2);
    const int j0 = min((int)floorf(x), Wc - 2);
    const float ty = y - (float)i0, tx = x - (float)j0;
    const int64_t o = (int64_t)i0 * ldc + j0;
    float f00 = F[o], f01 = F[o + 1], f10 = F[o + ldc], f11 = F[o + ldc + 1];
    if (D) {
        f00 += D[o];
        f01 += D[o + 1];
        f10 += D[o + ldc];
        f11 += D[o + ldc + 1];
    }
    return (1.f - ty) * ((1.f - tx) * f00 + tx * f01) + ty * ((1.f - tx) * f10 + tx * f11);
}

__device__ __forceinline__ void level_init_body(const LevelInitArgs& a, int bx, int by) {
    const int j = bx * 64 + (threadIdx.x & 63);
    const int i = by * 4 + (threadIdx.x >> 6);
    if (i >= a.H || j >= a.W) return;
    const int64_t off = (int64_t)i * a.ld + j;
    // target order (w, u, v): illumination keeps its scale, flow components double
    const float* src[3] = {a.wc, a.uc, a.vc};
    const float* inc[3] = {nullptr, a.ucd, a.vcd};
    const float scale[3] = {1.f, 2.f, 2.f};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (!a.set_flow[k]) continue;
        const float val = src[k] ? scale[k] * up_sample(src[k], a.Hc, a.Wc, a.ldc, i, j, inc[k]) : 0.f;
        a.set_flow[k][off] = val;
        if (a.copy_flow[k]) a.copy_flow[k][off] = val;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)   // constant indices keep the argument block out of scratch
        if (k < a.nzero) a.zero[k][off] = 0.f;
    if (a.clear_scalar && i == 0 && j == 0) *a.clear_scalar = 0.f;
}

// ---------------------------------------------------------------------------------------------
// single launches: the grid is the item's own block grid
// ---------------------------------------------------------------------------------------------
template <typename T> __global__ __launch_bounds__(256) void downsample_kernel(DownArgs a) {
    downsample_body<T>(a, blockIdx.x, blockIdx.y);
}
template <typename T> __global__ __launch_bounds__(256) void derivatives_kernel(DerivArgs a) {
    derivatives_body<T>(a, blockIdx.x, blockIdx.y);
}
template <typename T> __global__ __launch_bounds__(256) void copy_kernel(CopyArgs a) {
    copy_body<T>(a, blockIdx.x, blockIdx.y);
}
// Deterministic noise in [-scale, scale) from the "lowbias32" integer mixer of C. Wellons' hash
// prospector, applied to seed ^ (row * 0x9E3779B9 + column): operands for timing runs that vary
// from pixel to pixel as those of real images do.
__global__ __launch_bounds__(256) void noise_kernel(float* p, int H, int W, int64_t ld, uint32_t seed, float scale) {
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= H || j >= W) return;
    uint32_t x = seed ^ ((uint32_t)i * 0x9E3779B9u + (uint32_t)j);
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    p[(int64_t)i * ld + j] = scale * fmaf((float)(x >> 8), 2.f / 16777216.f, -1.f);
}
template <typename T> __global__ __launch_bounds__(kLinThreads) void linearize_kernel(LinArgs a) {
    linearize_body<T>(a, blockIdx.x, blockIdx.y);
}
__global__ __launch_bounds__(256) void level_init_kernel(LevelInitArgs a) {
    level_init_body(a, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(256) void upsample_kernel(const float* __restrict__ F, int Hc, int Wc, int64_t ldc,
                                                       float* __restrict__ out, int Hf, int Wf, int64_t ldf,
                                                       float scale) {
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= Hf || j >= Wf) return;
    out[(int64_t)i * ldf + j] = scale * up_sample(F, Hc, Wc, ldc, i, j);
}

// ---------------------------------------------------------------------------------------------
// batched launches: item k owns work-groups [off[k], off[k+1]), row-major over its block grid
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ int find_item(const int* __restrict__ off, int n, int b) {
    int lo = 0, hi = n;   // invariant off[lo] <= b < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <typename A> __device__ __forceinline__ int grid_w(const A& a) { return (a.W + 63) / 64; }
template <> __device__ __forceinline__ int grid_w<DownArgs>(const DownArgs& a) { return ((a.W + 1) / 2 + 63) / 64; }

template <typename A, void (*BODY)(const A&, int, int), int NT = 256>
__global__ __launch_bounds__(NT) void batched_kernel(const A* __restrict__ items, const int* __restrict__ off, int n) {
    const int k = find_item(off, n, blockIdx.x);
    const A a = items[k];
    const int local = blockIdx.x - off[k];
    const int gx = grid_w(a);
    BODY(a, local % gx, local / gx);
}

template <typename A, void (*BODY)(const A&, int, int), int NT = 256>
void launch_b(const void* items, const int* off, int n, int total, hipStream_t s) {
    hipLaunchKernelGGL((batched_kernel<A, BODY, NT>), dim3(total), dim3(NT), 0, s, (const A*)items, off, n);
}

}  // namespace

// ----------------------------------- host launchers --------------------------------------------
void launch_downsample(const void* src, int H, int W, int64_t ld, void* dst, int64_t ldd, bool f16, hipStream_t s,
                       const float* src_lo, float* dst_lo) {
    const DownArgs a{src, H, W, ld, dst, ldd, f16 ? nullptr : src_lo, f16 ? nullptr : dst_lo};
    const dim3 g = grid2d((H + 1) / 2, (W + 1) / 2);
    if (f16) hipLaunchKernelGGL(downsample_kernel<__half>, g, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(downsample_kernel<float>, g, dim3(256), 0, s, a);
}

void launch_derivatives(const void* I, int H, int W, int64_t ld, void* Dx, void* Dy, int64_t ldd, bool f16,
                        hipStream_t s, const float* I_lo) {
    const DerivArgs a{I, H, W, ld, Dx, Dy, ldd, f16 ? nullptr : I_lo};
    if (f16) hipLaunchKernelGGL(derivatives_kernel<__half>, grid2d(H, W), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(derivatives_kernel<float>, grid2d(H, W), dim3(256), 0, s, a);
}

void launch_import(const float* src, int H, int W, int64_t lds, void* dst, int64_t ldd, bool f16, hipStream_t s) {
    const CopyArgs a{src, H, W, lds, dst, ldd, f16 ? kFrameOffsetF16 : 0.f};
    if (f16) hipLaunchKernelGGL(copy_kernel<__half>, grid2d(H, W), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(copy_kernel<float>, grid2d(H, W), dim3(256), 0, s, a);
}

void launch_copy2d(const float* src, int H, int W, int64_t lds, float* dst, int64_t ldd, hipStream_t s,
                   const float* add) {
    const CopyArgs a{src, H, W, lds, dst, ldd, 0.f, add};
    hipLaunchKernelGGL(copy_kernel<float>, grid2d(H, W), dim3(256), 0, s, a);
}

void launch_fill_noise(float* p, int H, int W, int64_t ld, uint32_t seed, float scale, hipStream_t s) {
    hipLaunchKernelGGL(noise_kernel, grid2d(H, W), dim3(256), 0, s, p, H, W, ld, seed, scale);
}

void launch_linearize(const LinArgs& a, bool f16, hipStream_t s) {
    const dim3 g((a.W + 63) / 64, (a.H + kLinRows - 1) / kLinRows);
    if (f16) hipLaunchKernelGGL(linearize_kernel<__half>, g, dim3(kLinThreads), 0, s, a);
    else hipLaunchKernelGGL(linearize_kernel<float>, g, dim3(kLinThreads), 0, s, a);
}

void launch_level_init(const LevelInitArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(level_init_kernel, grid2d(a.H, a.W), dim3(256), 0, s, a);
}

void launch_upsample(const float* coarse, int64_t ldc, float* fine, int Hf, int Wf, int64_t ldf, float scale,
                     hipStream_t s) {
    hipLaunchKernelGGL(upsample_kernel, grid2d(Hf, Wf), dim3(256), 0, s, coarse, (Hf + 1) / 2, (Wf + 1) / 2, ldc,
                       fine, Hf, Wf, ldf, scale);
}


void launch_batched(BatchOp op, const void* items, const int* off, int n, int total, bool f16, hipStream_t s) {
    if (n <= 0 || total <= 0) return;
    switch (op) {
        case BatchOp::Downsample:
            if (f16) launch_b<DownArgs, downsample_body<__half>>(items, off, n, total, s);
            else launch_b<DownArgs, downsample_body<float>>(items, off, n, total, s);
            break;
        case BatchOp::Derivatives:
            if (f16) launch_b<DerivArgs, derivatives_body<__half>>(items, off, n, total, s);
            else launch_b<DerivArgs, derivatives_body<float>>(items, off, n, total, s);
            break;
        case BatchOp::Copy:
            if (f16) launch_b<CopyArgs, copy_body<__half>>(items, off, n, total, s);
            else launch_b<CopyArgs, copy_body<float>>(items, off, n, total, s);
            break;
        case BatchOp::Linearize:
            if (f16) launch_b<LinArgs, linearize_body<__half>, kLinThreads>(items, off, n, total, s);
            else launch_b<LinArgs, linearize_body<float>, kLinThreads>(items, off, n, total, s);
            break;
        case BatchOp::LevelInit: launch_b<LevelInitArgs, level_init_body>(items, off, n, total, s); break;
    }
}

}  // namespace flowmi
