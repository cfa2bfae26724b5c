// A fake device for the CPU test of the library's host code.
//
// The HIP runtime calls the host sources make are served from host memory: allocations are
// tracked (so pointer-extent checks work) and filled with NaN bytes (a read of memory nobody wrote
// poisons the results); every stream is in order and complete at once; a capturing stream records
// its work into a graph that hipGraphLaunch replays later, reading device memory at replay time
// as a real graph does.
//
// The kernel launchers are replaced by toy kernels with the same memory footprint as the real
// ones (each reads and writes the planes and pixels the real kernel would) but integer arithmetic
// that is exact in FP32: a pair's final flow and energy are a fixed function of its own frames and
// of the sequence of steps the host code applies to its planes.  Any mix-up -- a wrong descriptor,
// an overlapping arena, a missing or repeated tile, a wrong a~ slot or ping-pong direction --
// changes them, and the same pair solved alone, batched or served must give bitwise the same
// numbers.  The iteration toys add K x c per launch of K iterations, c an integer of the pixel's
// linearisation, so any split of a warp into launches gives the same result, as the real tile
// kernels do.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <vector>

#include "kernels.hpp"

struct fake_stream { std::vector<std::function<void()>>* capture = nullptr; };
struct fake_event { int recorded = 0; };
struct fake_graph { std::vector<std::function<void()>> work; };
struct fake_graph_exec { std::vector<std::function<void()>> work; };

namespace {

std::map<uintptr_t, size_t> g_allocs;   // base -> bytes
fake_stream g_null_stream;
long g_launches = 0;

fake_stream* S(hipStream_t s) { return s ? s : &g_null_stream; }

// run now, or record into the capturing stream's graph
void enqueue(hipStream_t s, std::function<void()> f) {
    fake_stream* st = S(s);
    if (st->capture) st->capture->push_back(std::move(f));
    else f();
}

uintptr_t g_hit_lo = 1, g_hit_hi = 0;          // the allocation found last (most accesses repeat it)

bool tracked(const void* p, size_t n) {
    const uintptr_t a = (uintptr_t)p;
    if (a >= g_hit_lo && a + n <= g_hit_hi) return true;
    auto it = g_allocs.upper_bound(a);
    if (it == g_allocs.begin()) return false;
    --it;
    if (!(a >= it->first && a + n <= it->first + it->second)) return false;
    g_hit_lo = it->first;
    g_hit_hi = it->first + it->second;
    return true;
}

void check(bool ok, const char* what) {
    if (!ok) {
        std::fprintf(stderr, "fake device: %s\n", what);
        std::abort();
    }
}

}  // namespace

long fake_device_launches() { return g_launches; }
size_t fake_device_live_allocations() { return g_allocs.size(); }

// ------------------------------------------------------------------ runtime
hipError_t hipMalloc(void** p, size_t n) {
    const size_t m = std::max<size_t>(256, (n + 255) & ~(size_t)255);
    void* q = std::aligned_alloc(256, m);
    if (!q) return hipErrorOutOfMemory;
    std::memset(q, 0xff, m);                  // NaN in every float: reads of unwritten memory show
    g_allocs[(uintptr_t)q] = n;
    *p = q;
    return hipSuccess;
}
hipError_t hipFree(void* p) {
    if (!p) return hipSuccess;
    auto it = g_allocs.find((uintptr_t)p);
    check(it != g_allocs.end(), "hipFree of a pointer hipMalloc did not return");
    g_allocs.erase(it);
    g_hit_lo = 1;
    g_hit_hi = 0;
    std::free(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned) {
    *p = std::calloc(1, std::max<size_t>(1, n));
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* p) {
    std::free(p);
    return hipSuccess;
}
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
    std::memmove(d, s, n);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t st) {
    enqueue(st, [=] { std::memmove(d, s, n); });
    return hipSuccess;
}
hipError_t hipMemset(void* d, int v, size_t n) {
    std::memset(d, v, n);
    return hipSuccess;
}
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t st) {
    enqueue(st, [=] { std::memset(d, v, n); });
    return hipSuccess;
}
hipError_t hipMemGetAddressRange(hipDeviceptr_t* base, size_t* size, hipDeviceptr_t p) {
    const uintptr_t a = (uintptr_t)p;
    auto it = g_allocs.upper_bound(a);
    if (it == g_allocs.begin()) return hipErrorInvalidValue;
    --it;
    if (a >= it->first + it->second) return hipErrorInvalidValue;
    *base = (void*)it->first;
    *size = it->second;
    return hipSuccess;
}
hipError_t hipGetDeviceCount(int* n) { *n = 1; return hipSuccess; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "fake device error"; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = new fake_stream(); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = new fake_event(); return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = new fake_event(); return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    enqueue(s, [=] { e->recorded++; });
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 1e-3f; return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    check(s && !s->capture, "capture on the null stream or twice");
    s->capture = new std::vector<std::function<void()>>();
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
    check(s && s->capture, "end of a capture that did not begin");
    *g = new fake_graph{std::move(*s->capture)};
    delete s->capture;
    s->capture = nullptr;
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, void*, void*, size_t) {
    *e = new fake_graph_exec{g->work};
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s) {
    for (auto& f : e->work) enqueue(s, f);
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t e) { delete e; return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }

// ------------------------------------------------------------------ toy kernels
namespace flowmi {

namespace {

float ldf(const void* p, int64_t o) {
    check(tracked((const float*)p + o, 4), "toy kernel read outside device memory");
    return ((const float*)p)[o];
}
void stf(void* p, int64_t o, float x) {
    check(tracked((float*)p + o, 4), "toy kernel write outside device memory");
    ((float*)p)[o] = x;
}
// a small non-negative integer of a finite integer-valued x, NaN for anything else
float imod(float x, int m) {
    if (!std::isfinite(x) || x != std::floor(x)) return NAN;
    const long long v = (long long)std::fabs(x);
    return (float)(v % m);
}

void copy_body(const CopyArgs& a) {
    for (int i = 0; i < a.H; ++i)
        for (int j = 0; j < a.W; ++j) {
            const int64_t o = (int64_t)i * a.lds + j;
            const float x = ldf(a.src, o) + (a.add ? ldf(a.add, o) : 0.f);
            stf(a.dst, (int64_t)i * a.ldd + j, x - a.offset);
        }
}
// the sum (not the mean) of the 2 x 2 block keeps integer images integer; low parts zero
void down_body(const DownArgs& a) {
    const int Hc = (a.H + 1) / 2, Wc = (a.W + 1) / 2;
    for (int r = 0; r < Hc; ++r)
        for (int b = 0; b < Wc; ++b) {
            const int r0 = 2 * r, r1 = std::min(2 * r + 1, a.H - 1), c0 = 2 * b, c1 = std::min(2 * b + 1, a.W - 1);
            float s = ldf(a.src, (int64_t)r0 * a.ld + c0) + ldf(a.src, (int64_t)r0 * a.ld + c1) +
                      ldf(a.src, (int64_t)r1 * a.ld + c0) + ldf(a.src, (int64_t)r1 * a.ld + c1);
            if (a.src_lo) s += ldf(a.src_lo, (int64_t)r0 * a.ld + c0);
            stf(a.dst, (int64_t)r * a.ldd + b, s);
            if (a.dst_lo) stf(a.dst_lo, (int64_t)r * a.ldd + b, 0.f);
        }
}
void deriv_body(const DerivArgs& a) {
    for (int i = 0; i < a.H; ++i)
        for (int j = 0; j < a.W; ++j) {
            const int64_t row = (int64_t)i * a.ld;
            float dx = ldf(a.I, row + std::min(j + 1, a.W - 1)) - ldf(a.I, row + std::max(j - 1, 0));
            float dy = ldf(a.I, (int64_t)std::min(i + 1, a.H - 1) * a.ld + j) - ldf(a.I, (int64_t)std::max(i - 1, 0) * a.ld + j);
            if (a.I_lo) dx += ldf(a.I_lo, row + j), dy += ldf(a.I_lo, row + j);
            stf(a.Dx, (int64_t)i * a.ldd + j, dx);
            stf(a.Dy, (int64_t)i * a.ldd + j, dy);
        }
}
void lin_body(const LinArgs& a) {
    float ms = 0.f;
    for (int i = 0; i < a.H; ++i)
        for (int j = 0; j < a.W; ++j) {
            const int64_t o = (int64_t)i * a.ld + j;
            float u0 = ldf(a.u0, o), v0 = ldf(a.v0, o);
            if (a.pend_u) {
                u0 += ldf(a.pend_u, o);
                v0 += ldf(a.pend_v, o);
                stf(a.u0, o, u0);
                stf(a.v0, o, v0);
            }
            const float Ix = imod(ldf(a.Dx, o) + u0, 7), Iy = imod(ldf(a.Dy, o) + v0 + (float)i, 5);
            float It = imod(ldf(a.I1, o) - ldf(a.I0, o) + (float)j, 11);
            if (a.I1lo) It += ldf(a.I1lo, o) - ldf(a.I0lo, o);
            stf(a.Ix, o, Ix);
            stf(a.Iy, o, Iy);
            stf(a.It, o, a.rel ? It : It - Ix * u0 - Iy * v0);
            if (a.zero_u) { stf(a.zero_u, o, 0.f); stf(a.zero_v, o, 0.f); }
            if (a.keep_u) { stf(a.keep_u, o, u0); stf(a.keep_v, o, v0); }
            ms = std::max(ms, Ix * Ix + Iy * Iy);
        }
    const float old = ldf(a.at, 0);
    stf(a.at, 0, std::isnan(old) ? old : std::max(old, ms));   // an uncleared slot stays NaN
    if (a.at_clear) stf(a.at_clear, 0, 0.f);
}
void init_body(const LevelInitArgs& a) {
    const float* src[3] = {a.wc, a.uc, a.vc};
    const float* inc[3] = {nullptr, a.ucd, a.vcd};
    const float scale[3] = {1.f, 2.f, 2.f};
    for (int i = 0; i < a.H; ++i)
        for (int j = 0; j < a.W; ++j) {
            const int64_t o = (int64_t)i * a.ld + j;
            for (int k = 0; k < 3; ++k) {
                if (!a.set_flow[k]) continue;
                float val = 0.f;
                if (src[k]) {
                    const int64_t oc = (int64_t)std::min(i / 2, a.Hc - 1) * a.ldc + std::min(j / 2, a.Wc - 1);
                    val = scale[k] * (ldf(src[k], oc) + (inc[k] ? ldf(inc[k], oc) : 0.f));
                }
                stf(a.set_flow[k], o, val);
                if (a.copy_flow[k]) stf(a.copy_flow[k], o, val);
            }
            for (int k = 0; k < a.nzero; ++k) stf(a.zero[k], o, 0.f);
        }
    if (a.clear_scalar) stf(a.clear_scalar, 0, 0.f);
}
// per-iteration increment of state plane k at pixel o
float incr(const float* Ix, const float* It, const float* at, int64_t o, int k) {
    return imod(ldf(Ix, o) + ldf(It, o) + (float)k + ldf(at, 0), 3);
}
void tile_body(const TbLevel& L, const TbTile& T, int K, int slot) {
    check(T.y0 >= 0 && T.x0 >= 0 && T.th > 0 && T.tw > 0 && T.y0 + T.th <= L.H && T.x0 + T.tw <= L.W,
          "tile outside its level");
    for (int i = T.y0; i < T.y0 + T.th; ++i)
        for (int j = T.x0; j < T.x0 + T.tw; ++j) {
            const int64_t o = (int64_t)i * L.ld + j;
            for (int k = 0; k < 10; ++k)
                if (L.in[k]) stf(L.out[k], o, ldf(L.in[k], o) + (float)K * incr(L.Ix, L.It, L.at + slot, o, k));
        }
}
void energy_body(const EnergyArgs& a) {
    double t[kEnergyTerms] = {};
    for (int i = 0; i < a.H; ++i)
        for (int j = 0; j < a.W; ++j) {
            const int64_t o = (int64_t)i * a.ld + j;
            const double u = ldf(a.u, o) + (a.du ? ldf(a.du, o) : 0.f) - (a.lu0 ? ldf(a.lu0, o) : 0.f);
            const double v = ldf(a.v, o) + (a.dv ? ldf(a.dv, o) : 0.f) - (a.lv0 ? ldf(a.lv0, o) : 0.f);
            t[0] += u * (1 + (i + 2 * j) % 5);
            t[1] += v * (1 + (2 * i + j) % 7);
            t[2] += ldf(a.s, o) + ldf(a.q1x, o) + 2.0 * ldf(a.q2y, o) + ldf(a.It, o);
            t[3] += ldf(a.q1y, o) * ldf(a.q2x, o);
        }
    const int nb = energy_blocks(a.H, a.W);
    stf(a.partial, (int64_t)nb * kEnergyTerms - 1, 0.f);        // the last partial the real kernel writes
    bool finite = true;
    for (int k = 0; k < 4; ++k) finite = finite && std::isfinite(t[k]);
    double* out = a.out;
    check(tracked(out, sizeof(double) * kEnergyTerms), "energy output outside device memory");
    out[0] = t[0]; out[1] = t[1]; out[2] = t[2]; out[3] = std::fabs(t[3]);
    out[4] = out[5] = out[6] = 0.0;
    out[7] = finite ? 0.0 : 1.0;
}

template <typename A> void run_items(const void* items, const int* off, int n, int total, void (*body)(const A&)) {
    check(tracked(items, sizeof(A) * n) && tracked(off, sizeof(int) * (n + 1)), "item table outside device memory");
    check(off[0] == 0 && off[n] == total, "item block offsets");
    for (int k = 0; k < n; ++k) {
        check(off[k + 1] >= off[k], "item block offsets decrease");
        body(((const A*)items)[k]);
    }
}

}  // namespace

void launch_import(const float* src, int H, int W, int64_t lds, void* dst, int64_t ldd, bool f16, hipStream_t s) {
    check(!f16, "FP16 storage is not modelled");
    const CopyArgs a{src, H, W, lds, dst, ldd, 0.f, nullptr};
    ++g_launches;
    enqueue(s, [=] { copy_body(a); });
}
void launch_copy2d(const float* src, int H, int W, int64_t lds, float* dst, int64_t ldd, hipStream_t s, const float* add) {
    const CopyArgs a{src, H, W, lds, dst, ldd, 0.f, add};
    ++g_launches;
    enqueue(s, [=] { copy_body(a); });
}
void launch_downsample(const void* src, int H, int W, int64_t ld, void* dst, int64_t ldd, bool f16, hipStream_t s,
                       const float* src_lo, float* dst_lo) {
    check(!f16, "FP16 storage is not modelled");
    const DownArgs a{src, H, W, ld, dst, ldd, src_lo, dst_lo};
    ++g_launches;
    enqueue(s, [=] { down_body(a); });
}
void launch_derivatives(const void* I, int H, int W, int64_t ld, void* Dx, void* Dy, int64_t ldd, bool f16, hipStream_t s,
                        const float* I_lo) {
    check(!f16, "FP16 storage is not modelled");
    const DerivArgs a{I, H, W, ld, Dx, Dy, ldd, I_lo};
    ++g_launches;
    enqueue(s, [=] { deriv_body(a); });
}
void launch_linearize(const LinArgs& a, bool f16, hipStream_t s) {
    check(!f16, "FP16 storage is not modelled");
    ++g_launches;
    enqueue(s, [=] { lin_body(a); });
}
void launch_level_init(const LevelInitArgs& a, hipStream_t s) {
    ++g_launches;
    enqueue(s, [=] { init_body(a); });
}
void launch_upsample(const float* coarse, int64_t ldc, float* fine, int Hf, int Wf, int64_t ldf_, float scale,
                     hipStream_t s) {
    LevelInitArgs a{};
    a.uc = coarse;
    a.Hc = (Hf + 1) / 2;
    a.Wc = (Wf + 1) / 2;
    a.ldc = ldc;
    a.set_flow[1] = fine;
    a.H = Hf;
    a.W = Wf;
    a.ld = ldf_;
    (void)scale;
    ++g_launches;
    enqueue(s, [=] { init_body(a); });
}
void launch_fill_noise(float* p, int H, int W, int64_t ld, uint32_t seed, float, hipStream_t s) {
    ++g_launches;
    enqueue(s, [=] {
        for (int i = 0; i < H; ++i)
            for (int j = 0; j < W; ++j) stf(p, (int64_t)i * ld + j, (float)((seed + 3 * i + 7 * j) % 13));
    });
}
void launch_reset_u32(unsigned* p, int n, hipStream_t s) {
    ++g_launches;
    enqueue(s, [=] {
        check(tracked(p, sizeof(unsigned) * n), "counter reset outside device memory");
        for (int i = 0; i < n; ++i) p[i] = 0u;
    });
}
void launch_batched(BatchOp op, const void* items, const int* off, int n, int total, bool f16, hipStream_t s) {
    if (n <= 0 || total <= 0) return;
    check(!f16, "FP16 storage is not modelled");
    ++g_launches;
    enqueue(s, [=] {
        switch (op) {
            case BatchOp::Downsample: run_items<DownArgs>(items, off, n, total, down_body); break;
            case BatchOp::Derivatives: run_items<DerivArgs>(items, off, n, total, deriv_body); break;
            case BatchOp::Copy: run_items<CopyArgs>(items, off, n, total, copy_body); break;
            case BatchOp::Linearize: run_items<LinArgs>(items, off, n, total, lin_body); break;
            case BatchOp::LevelInit: run_items<LevelInitArgs>(items, off, n, total, init_body); break;
        }
    });
}
void launch_energy(const EnergyArgs& a, hipStream_t s) {
    ++g_launches;
    enqueue(s, [=] { energy_body(a); });
}
void launch_energy_batched(const EnergyArgs* items, const int* off, int n, int total, hipStream_t s) {
    ++g_launches;
    enqueue(s, [=] { run_items<EnergyArgs>(items, off, n, total, energy_body); });
}
void launch_admm_iter(const AdmmIterArgs& a, bool, hipStream_t s) {
    ++g_launches;
    enqueue(s, [=] {
        const float* in[10] = {a.w, a.u, a.v, a.px, a.py, a.q1x, a.q1y, a.q2x, a.q2y, a.s};
        float* out[10] = {a.wo, a.uo, a.vo, a.pxo, a.pyo, a.q1xo, a.q1yo, a.q2xo, a.q2yo, a.so};
        for (int i = 0; i < a.H; ++i)
            for (int j = 0; j < a.W; ++j) {
                const int64_t o = (int64_t)i * a.ld + j;
                for (int k = 0; k < 10; ++k)
                    if (in[k]) stf(out[k], o, ldf(in[k], o) + incr(a.Ix, a.It, a.at, o, k));
            }
    });
}
// the extended region of an ADMM tile (halo K + 1 above / left, K below / right, clipped) fits the
// work-group shape it is launched with: the real kernels index LDS or registers by its cells
static void check_admm_region(const TbLevel& L, const TbTile& T, int K, bool hw, int nt) {
    const int64_t eh = std::min(T.y0 + T.th + K, L.H) - std::max(T.y0 - (K + 1), 0);
    const int64_t ew = std::min(T.x0 + T.tw + K, L.W) - std::max(T.x0 - (K + 1), 0);
    check(tb_fits(hw, nt, eh, ew), "ADMM tile region beyond the kernel's shape");
}
void launch_admm_tb(const TbArgs& a, bool hw, int nt, int grid, hipStream_t s) {
    check(grid > 0 && a.K > 0, "tile launch without work-groups or iterations");
    check(tb_capacity(false, nt) > 0, "tile launch of an unknown work-group shape");
    check(!(is_rows_code(nt) && a.queue), "wave-row tiles launched from work queues");
    ++g_launches;
    enqueue(s, [=] {
        if (!a.tiles) {                                  // direct: regular tiles of one level
            for (int t = 0; t < a.ntiles; ++t) {
                const int ty = t / a.ntx, tx = t - ty * a.ntx;
                TbTile T{0, ty * a.th, tx * a.tw, std::min(a.th, a.lvl.H - ty * a.th), std::min(a.tw, a.lvl.W - tx * a.tw)};
                check_admm_region(a.lvl, T, a.K, hw, nt);
                tile_body(a.lvl, T, a.K, a.at_slot);
            }
            return;
        }
        const int n = a.ntiles_dev ? *a.ntiles_dev : a.ntiles;
        check(tracked(a.tiles, sizeof(TbTile) * std::max(1, n)), "tile table outside device memory");
        auto run = [&](int t) {
            const TbTile& T = a.tiles[t];
            const TbLevel* L = a.levels + 2 * T.level + a.dir;
            check(tracked(L, sizeof(TbLevel)), "level descriptor outside device memory");
            check_admm_region(*L, T, a.K, hw, nt);
            tile_body(*L, T, a.K, a.at_slot);
        };
        if (!a.queue) {
            for (int t = 0; t < n; ++t) run(t);
            return;
        }
        // work queue: every work-group b of sub-queue x = b % nq pulls until its counter passes the
        // end of the sub-queue's run of tiles, exactly as the real kernel counts
        for (int b = 0; b < grid; ++b) {
            const int x = b % a.nq;
            const int lo = (int)((int64_t)n * x / a.nq), hi = (int)((int64_t)n * (x + 1) / a.nq);
            for (;;) {
                check(tracked(a.queue + x, sizeof(unsigned)), "queue counter outside device memory");
                const int t = lo + (int)(a.queue[x]++ - a.queue_base);
                if (t >= hi) break;
                run(t);
            }
        }
    });
}
// every tile's extended region fits the work-group shape it is launched with (the real kernels
// index LDS by the region's cells), and the tiles with two cells of each colour run without the w
// block only
static void check_pd_codes(bool has_w, int nt) {
    check(nt == 512 || nt == 1024 || nt == 2048 || nt == 513 || is_pd_rows_code(nt),
          "pDR / ALG1 tile launch: work-group code");
    check((nt != 2048 && nt != 513 && nt != 6145 && nt != 3074) || !has_w, "pDR tiles for beta = 0 launched with w");
}
static void check_pd_region(const PdrTbLevel& L, int th, int tw, bool has_w, int nt, int halo) {
    const int64_t eh = std::min<int64_t>(L.H, (int64_t)th + halo);
    const int64_t ew = std::min<int64_t>(L.W, (int64_t)tw + halo);
    check(pd_fits(has_w, nt, eh, ew), "pDR / ALG1 tile region beyond the kernel's shape");
}
// toy iteration: X += K on the tile's output cells, X bar and y bar copied, Theta = I_t
static void toy_pd_region(const PdrTbLevel& L, int K, int y0, int x0, int th, int tw) {
    for (int i = y0; i < y0 + th; ++i)
        for (int j = x0; j < x0 + tw; ++j) {
            const int64_t o = (int64_t)i * L.ld + j;
            for (int f = 0; f < 3; ++f)
                if (L.x_in[f]) {
                    stf(L.x_out[f], o, ldf(L.x_in[f], o) + (float)K);
                    stf(L.xb_out[f], o, ldf(L.xb_in[f], o));
                }
            for (int f = 0; f < 6; ++f)
                if (L.y_in[f]) stf(L.y_out[f], o, ldf(L.y_in[f], o));
            stf(L.s_out, o, ldf(L.It, o));
        }
}
static void launch_pd(const PdrTbArgs& a, bool has_w, int nt, int halo, hipStream_t s) {
    check_pd_codes(has_w, nt);
    check(a.K > 0 && a.ntiles > 0, "pDR / ALG1 tile launch without tiles or iterations");
    ++g_launches;
    if (!a.tiles) {                                      // direct: regular tiles of one level
        check_pd_region(a.lvl, a.th, a.tw, has_w, nt, halo);
        enqueue(s, [=] { toy_pd_region(a.lvl, a.K, 0, 0, a.lvl.H, a.lvl.W); });
        return;
    }
    enqueue(s, [=] {                                     // table order: tile entries name their level
        check(tracked(a.tiles, sizeof(TbTile) * a.ntiles), "pDR tile table outside device memory");
        for (int t = 0; t < a.ntiles; ++t) {
            const TbTile& T = a.tiles[t];
            const PdrTbLevel* L = a.levels + 2 * T.level + a.dir;
            check(tracked(L, sizeof(PdrTbLevel)), "pDR level descriptor outside device memory");
            check(T.y0 >= 0 && T.x0 >= 0 && T.th >= 1 && T.tw >= 1 && T.y0 + T.th <= L->H && T.x0 + T.tw <= L->W,
                  "pDR tile outside its level");
            check_pd_region(*L, T.th, T.tw, has_w, nt, halo);
            toy_pd_region(*L, a.K, T.y0, T.x0, T.th, T.tw);
        }
    });
}
void launch_pdr_tb(const PdrTbArgs& a, bool has_w, int nt, hipStream_t s) {
    launch_pd(a, has_w, nt, pdr_halo_lo(a.sweeps, a.K) + pdr_halo_hi(a.sweeps, a.K), s);
}
void launch_alg1_tb(const PdrTbArgs& a, bool has_w, int nt, hipStream_t s) {
    check(nt != 2048 && nt != 513 && nt != 4098 && nt != 6145, "pDR-only tiles launched for ALG1");
    check(nt != 3074 || !has_w, "ALG1 64 x 48 wave-row tiles launched with w");
    launch_pd(a, has_w, nt, 2 * alg1_halo(a.K), s);
}
static void pdr_pass(const PdrArgs& a, bool final_pass) {
    float* x[3] = {a.w, a.u, a.v};
    for (int i = 0; i < a.H; ++i)
        for (int j = 0; j < a.W; ++j) {
            const int64_t o = (int64_t)i * a.ld + j;
            for (int f = 0; f < 3; ++f)
                if (x[f]) stf(x[f], o, ldf(x[f], o) + (final_pass ? 1.f : 0.f));
            if (final_pass && a.s_out) stf(a.s_out, o, ldf(a.It, o));
        }
}
void launch_pdr_rhs_red(const PdrArgs& a, bool, hipStream_t s) { ++g_launches; enqueue(s, [=] { pdr_pass(a, false); }); }
void launch_pdr_colour(const PdrArgs& a, bool, hipStream_t s) { ++g_launches; enqueue(s, [=] { pdr_pass(a, false); }); }
void launch_pdr_final(const PdrArgs& a, bool, hipStream_t s) { ++g_launches; enqueue(s, [=] { pdr_pass(a, true); }); }

}  // namespace flowmi
