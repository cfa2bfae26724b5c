/* A plain C client of the flow library: no Python, no torch.  It builds a synthetic pair whose
 * second frame is the first translated by (0.3, -0.2) px, solves it with flow_solve on device
 * buffers it allocates itself, and checks that the flow it gets back is that translation (mean
 * over the interior, within 0.02 px) and that the energy and the gap are finite.  Exit status 0 on
 * success.  Usage: solve_pair [H W] */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "flow.h"

/* a smooth texture in [0, 1], defined everywhere so the translated frame is exact */
static double texture(double y, double x) {
    double t = 0.5 + 0.18 * sin(0.21 * x + 0.13 * y) + 0.14 * cos(0.17 * x - 0.23 * y);
    t += 0.12 * exp(-((x - 40.0) * (x - 40.0) + (y - 30.0) * (y - 30.0)) / 180.0);
    t -= 0.10 * exp(-((x - 90.0) * (x - 90.0) + (y - 60.0) * (y - 60.0)) / 260.0);
    return t;
}

#define CHECK(call)                                                                    \
    do {                                                                               \
        if ((call) != 0) {                                                             \
            fprintf(stderr, "%s failed: %s\n", #call, flow_last_error());              \
            return 1;                                                                  \
        }                                                                              \
    } while (0)

int main(int argc, char** argv) {
    const int H = argc > 2 ? atoi(argv[1]) : 96, W = argc > 2 ? atoi(argv[2]) : 128;
    const double du = 0.3, dv = -0.2;          /* I1(x + d) = I0(x) */
    const size_t n = (size_t)H * W;
    float* h0 = (float*)malloc(n * sizeof(float));
    float* h1 = (float*)malloc(n * sizeof(float));
    float* hu = (float*)malloc(n * sizeof(float));
    float* hv = (float*)malloc(n * sizeof(float));
    if (!h0 || !h1 || !hu || !hv) return 1;
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            h0[(size_t)i * W + j] = (float)texture(i, j);
            h1[(size_t)i * W + j] = (float)texture(i - dv, j - du);
        }
    float *d0, *d1, *dU, *dV;
    if (hipMalloc((void**)&d0, n * sizeof(float)) || hipMalloc((void**)&d1, n * sizeof(float)) ||
        hipMalloc((void**)&dU, n * sizeof(float)) || hipMalloc((void**)&dV, n * sizeof(float))) {
        fprintf(stderr, "hipMalloc failed\n");
        return 1;
    }
    if (hipMemcpy(d0, h0, n * sizeof(float), hipMemcpyHostToDevice) ||
        hipMemcpy(d1, h1, n * sizeof(float), hipMemcpyHostToDevice)) {
        fprintf(stderr, "hipMemcpy failed\n");
        return 1;
    }
    flow_ctx* ctx = NULL;
    CHECK(flow_create(&ctx, 0, 0));
    flow_params p;
    CHECK(flow_params_default(&p));
    p.levels = 2;
    p.warps = 3;
    p.iters = 100;
    flow_result res;
    CHECK(flow_solve(ctx, d0, d1, H, W, W, &p, dU, dV, W, &res, NULL));
    if (hipMemcpy(hu, dU, n * sizeof(float), hipMemcpyDeviceToHost) ||
        hipMemcpy(hv, dV, n * sizeof(float), hipMemcpyDeviceToHost)) {
        fprintf(stderr, "hipMemcpy failed\n");
        return 1;
    }
    double su = 0.0, sv = 0.0;
    int cnt = 0;
    for (int i = 8; i < H - 8; ++i)
        for (int j = 8; j < W - 8; ++j) {
            su += hu[(size_t)i * W + j];
            sv += hv[(size_t)i * W + j];
            ++cnt;
        }
    const double mu = su / cnt, mv = sv / cnt;
    printf("c_client %dx%d: mean flow (%.4f, %.4f) px, expected (%.1f, %.1f); energy %.4f gap %.4f\n", H, W, mu,
           mv, du, dv, res.energy, res.gap);
    CHECK(flow_destroy(ctx));
    hipFree(d0);
    hipFree(d1);
    hipFree(dU);
    hipFree(dV);
    free(h0);
    free(h1);
    free(hu);
    free(hv);
    const int ok = fabs(mu - du) < 0.02 && fabs(mv - dv) < 0.02 && isfinite(res.energy) && isfinite(res.gap);
    return ok ? 0 : 2;
}
