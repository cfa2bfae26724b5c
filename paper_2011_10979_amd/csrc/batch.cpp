// Batched solve of many pairs (placeholder until the work-queue path lands: plain solves in turn).
#include "runtime.hpp"

namespace flowmi {
struct BatchState {};
void destroy_batch(BatchState* b) { delete b; }
}  // namespace flowmi

using namespace flowmi;

extern "C" flow_status flow_solve_batched(flow_ctx* ctx, int32_t n, const flow_pair* pairs, const flow_params* p,
                                          void* stream) {
    if (!ctx || !pairs || n < 0) return fail(FLOW_E_INVAL, "bad batch arguments");
    for (int32_t k = 0; k < n; ++k) {
        const flow_pair& q = pairs[k];
        flow_status st = flow_solve(ctx, q.I0, q.I1, q.H, q.W, q.ld, p, q.u, q.v, q.ld_uv, q.res, stream);
        if (st != FLOW_OK) return st;
    }
    return FLOW_OK;
}
