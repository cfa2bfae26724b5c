// Coarse-to-fine framework kernels (Sec. 4 runs the solvers inside a standard coarse-to-fine
// warping pyramid; the filters below are this library's choice, the paper names none):
//   downsample   2x2 box mean with edge replication, ceil sizes (factor 1/2)
//   derivatives  central differences with replicated neighbours
//   linearize    bilinear warp of I1, D_x I1, D_y I1 at x + d0 and the linearisation
//                rho(d) = I_x u + I_y v + I_t (Sec. 1), plus a~ = max M_s (Prop. 3.1)
//   level_init   centre-aligned bilinear x2 upsampling of the flow, dual reset
// All are elementwise or gather kernels: one thread per output pixel, 64-wide rows per wavefront
// so that every plane access is a coalesced row segment.
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

template <typename T>
__global__ __launch_bounds__(256) void downsample_kernel(const T* __restrict__ src, int H, int W, int64_t ld,
                                                         T* __restrict__ dst, int Hc, int Wc, int64_t ldd) {
    const int b = blockIdx.x * 64 + (threadIdx.x & 63);
    const int a = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (a >= Hc || b >= Wc) return;
    const int r0 = 2 * a, r1 = min(2 * a + 1, H - 1);
    const int c0 = 2 * b, c1 = min(2 * b + 1, W - 1);
    const float s = ldv(src, (int64_t)r0 * ld + c0) + ldv(src, (int64_t)r0 * ld + c1) +
                    ldv(src, (int64_t)r1 * ld + c0) + ldv(src, (int64_t)r1 * ld + c1);
    stv(dst, (int64_t)a * ldd + b, 0.25f * s);
}

template <typename T>
__global__ __launch_bounds__(256) void derivatives_kernel(const T* __restrict__ I, int H, int W, int64_t ld,
                                                          T* __restrict__ Dx, T* __restrict__ Dy, int64_t ldd) {
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= H || j >= W) return;
    const int64_t row = (int64_t)i * ld;
    const float dx = 0.5f * (ldv(I, row + min(j + 1, W - 1)) - ldv(I, row + max(j - 1, 0)));
    const float dy = 0.5f * (ldv(I, (int64_t)min(i + 1, H - 1) * ld + j) - ldv(I, (int64_t)max(i - 1, 0) * ld + j));
    stv(Dx, (int64_t)i * ldd + j, dx);
    stv(Dy, (int64_t)i * ldd + j, dy);
}

template <typename T>
__global__ __launch_bounds__(256) void import_kernel(const float* __restrict__ src, int H, int W, int64_t lds,
                                                     T* __restrict__ dst, int64_t ldd) {
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= H || j >= W) return;
    stv(dst, (int64_t)i * ldd + j, src[(int64_t)i * lds + j]);
}

// Integer / fraction split of the sample position p + d clamped into [0, n-1]; keeps the
// fraction exact where p + d in FP32 would lose bits (|p| up to 2^11, ulp 1e-4 px).
__device__ __forceinline__ void split_pos(int p, float d, int n, int& i0, float& t) {
    const float fl = floorf(d);
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
__global__ __launch_bounds__(256) void linearize_kernel(LinArgs a) {
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    const T* I0 = (const T*)a.I0;
    const T* I1 = (const T*)a.I1;
    const T* Dx = (const T*)a.Dx;
    const T* Dy = (const T*)a.Dy;
    float ms = 0.f;
    if (i < a.H && j < a.W) {
        const int64_t off = (int64_t)i * a.ld + j;
        const float u0 = a.u0[off], v0 = a.v0[off];
        int iy, jx;
        float ty, tx;
        split_pos(i, v0, a.H, iy, ty);
        split_pos(j, u0, a.W, jx, tx);
        const int64_t o00 = (int64_t)iy * a.ld + jx;
        const float I1w = bilin(I1, o00, a.ld, ty, tx);
        const float Ix = a.kappa * bilin(Dx, o00, a.ld, ty, tx);
        const float Iy = a.kappa * bilin(Dy, o00, a.ld, ty, tx);
        const float Ir = a.kappa * (I1w - ldv(I0, off));
        a.Ix[off] = Ix;
        a.Iy[off] = Iy;
        a.It[off] = a.rel ? Ir : Ir - Ix * u0 - Iy * v0;
        if (a.zero_u) { a.zero_u[off] = 0.f; a.zero_v[off] = 0.f; }
        if (a.keep_u) { a.keep_u[off] = u0; a.keep_v[off] = v0; }
        ms = a.beta * a.beta + Ix * Ix + Iy * Iy;
    }
    // a~ = max M_s: wave -> block -> one atomic max per block on the float's bit pattern (exact
    // and order-independent for non-negative values); the consumer applies the 1e-12 floor.
    __shared__ float smax[4];
    ms = wave_max(ms);
    if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = ms;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float bm = fmaxf(fmaxf(smax[0], smax[1]), fmaxf(smax[2], smax[3]));
        atomicMax((unsigned int*)a.at, __float_as_uint(bm));
        if (a.at_clear && blockIdx.x == 0 && blockIdx.y == 0) *a.at_clear = 0.f;
    }
}

// centre-aligned bilinear sample of a coarse plane at fine pixel (i, j): coarse coordinate i/2 - 1/4
__device__ __forceinline__ float up_sample(const float* F, int Hc, int Wc, int64_t ldc, int i, int j) {
    float y = 0.5f * (float)i - 0.25f;
    float x = 0.5f * (float)j - 0.25f;
    y = fminf(fmaxf(y, 0.f), (float)(Hc - 1));
    x = fminf(fmaxf(x, 0.f), (float)(Wc - 1));
    const int i0 = min((int)floorf(y), Hc - 2);
    const int j0 = min((int)floorf(x), Wc - 2);
    const float ty = y - (float)i0, tx = x - (float)j0;
    const int64_t o = (int64_t)i0 * ldc + j0;
    return (1.f - ty) * ((1.f - tx) * F[o] + tx * F[o + 1]) + ty * ((1.f - tx) * F[o + ldc] + tx * F[o + ldc + 1]);
}

__global__ __launch_bounds__(256) void level_init_kernel(LevelInitArgs a) {
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= a.H || j >= a.W) return;
    const int64_t off = (int64_t)i * a.ld + j;
    // target order (w, u, v): illumination keeps its scale, flow components double
    const float* src[3] = {a.wc, a.uc, a.vc};
    const float scale[3] = {1.f, 2.f, 2.f};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (!a.set_flow[k]) continue;
        const float val = src[k] ? scale[k] * up_sample(src[k], a.Hc, a.Wc, a.ldc, i, j) : 0.f;
        a.set_flow[k][off] = val;
        if (a.copy_flow[k]) a.copy_flow[k][off] = val;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)   // constant indices keep the argument block out of scratch
        if (k < a.nzero) a.zero[k][off] = 0.f;
    if (a.clear_scalar && i == 0 && j == 0) *a.clear_scalar = 0.f;
}

__global__ __launch_bounds__(256) void upsample_kernel(const float* __restrict__ F, int Hc, int Wc, int64_t ldc,
                                                       float* __restrict__ out, int Hf, int Wf, int64_t ldf,
                                                       float scale) {
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= Hf || j >= Wf) return;
    out[(int64_t)i * ldf + j] = scale * up_sample(F, Hc, Wc, ldc, i, j);
}

__global__ __launch_bounds__(256) void commit_kernel(float* __restrict__ u0, float* __restrict__ v0,
                                                     const float* __restrict__ du, const float* __restrict__ dv,
                                                     int H, int W, int64_t ld) {
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= H || j >= W) return;
    const int64_t o = (int64_t)i * ld + j;
    u0[o] += du[o];
    v0[o] += dv[o];
}

__global__ __launch_bounds__(256) void copy2d_kernel(const float* __restrict__ src, int H, int W, int64_t lds,
                                                     float* __restrict__ dst, int64_t ldd) {
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= H || j >= W) return;
    dst[(int64_t)i * ldd + j] = src[(int64_t)i * lds + j];
}

}  // namespace

void launch_downsample(const void* src, int H, int W, int64_t ld, void* dst, int64_t ldd, bool f16, hipStream_t s) {
    const int Hc = (H + 1) / 2, Wc = (W + 1) / 2;
    if (f16)
        hipLaunchKernelGGL(downsample_kernel<__half>, grid2d(Hc, Wc), dim3(256), 0, s, (const __half*)src, H, W,
                           ld, (__half*)dst, Hc, Wc, ldd);
    else
        hipLaunchKernelGGL(downsample_kernel<float>, grid2d(Hc, Wc), dim3(256), 0, s, (const float*)src, H, W,
                           ld, (float*)dst, Hc, Wc, ldd);
}

void launch_derivatives(const void* I, int H, int W, int64_t ld, void* Dx, void* Dy, int64_t ldd, bool f16,
                        hipStream_t s) {
    if (f16)
        hipLaunchKernelGGL(derivatives_kernel<__half>, grid2d(H, W), dim3(256), 0, s, (const __half*)I, H, W, ld,
                           (__half*)Dx, (__half*)Dy, ldd);
    else
        hipLaunchKernelGGL(derivatives_kernel<float>, grid2d(H, W), dim3(256), 0, s, (const float*)I, H, W, ld,
                           (float*)Dx, (float*)Dy, ldd);
}

void launch_import(const float* src, int H, int W, int64_t lds, void* dst, int64_t ldd, bool f16, hipStream_t s) {
    if (f16)
        hipLaunchKernelGGL(import_kernel<__half>, grid2d(H, W), dim3(256), 0, s, src, H, W, lds, (__half*)dst, ldd);
    else
        hipLaunchKernelGGL(import_kernel<float>, grid2d(H, W), dim3(256), 0, s, src, H, W, lds, (float*)dst, ldd);
}

void launch_commit(float* u0, float* v0, const float* du, const float* dv, int H, int W, int64_t ld, hipStream_t s) {
    hipLaunchKernelGGL(commit_kernel, grid2d(H, W), dim3(256), 0, s, u0, v0, du, dv, H, W, ld);
}

void launch_copy2d(const float* src, int H, int W, int64_t lds, float* dst, int64_t ldd, hipStream_t s) {
    hipLaunchKernelGGL(copy2d_kernel, grid2d(H, W), dim3(256), 0, s, src, H, W, lds, dst, ldd);
}

void launch_linearize(const LinArgs& a, bool f16, hipStream_t s) {
    if (f16)
        hipLaunchKernelGGL(linearize_kernel<__half>, grid2d(a.H, a.W), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(linearize_kernel<float>, grid2d(a.H, a.W), dim3(256), 0, s, a);
}

void launch_level_init(const LevelInitArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(level_init_kernel, grid2d(a.H, a.W), dim3(256), 0, s, a);
}

void launch_upsample(const float* coarse, int64_t ldc, float* fine, int Hf, int Wf, int64_t ldf, float scale,
                     hipStream_t s) {
    hipLaunchKernelGGL(upsample_kernel, grid2d(Hf, Wf), dim3(256), 0, s, coarse, (Hf + 1) / 2, (Wf + 1) / 2, ldc,
                       fine, Hf, Wf, ldf, scale);
}

}  // namespace flowmi
