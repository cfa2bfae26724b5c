// Device helpers shared by the wave-row pDR and ALG1 tile kernels (one cell per lane and row): the
// whole-wavefront DPP neighbour shifts, loads and stores through the global address space, and
// the scalar read of a tile table's level descriptor.
#pragma once

#include "kernels.hpp"

namespace flowmi {

// lane l receives lane l + 1's value (lane 63: 0), and lane l - 1's (lane 0: 0)
__device__ __forceinline__ float from_right(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_left(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x138, 0xf, 0xf, false));
}

// the planes live in global memory: loads and stores through the global address space (pointers
// read from a descriptor table would otherwise be flat, whose loads also hold the LDS counter)
using gfloat = __attribute__((address_space(1))) float;
__device__ __forceinline__ float gload(const float* p, int64_t o) { return ((const gfloat*)p)[o]; }
__device__ __forceinline__ void gstore(float* p, int64_t o, float v) { ((gfloat*)p)[o] = v; }

// a level descriptor of the tile table, read through the constant address space: the table does
// not change while a launch runs, so its pointers load into scalar registers
__device__ __forceinline__ PdrTbLevel pdr_level_scalar(const PdrTbLevel* p) {
    using CL = const __attribute__((address_space(4))) PdrTbLevel;
    CL* q = (CL*)p;
    PdrTbLevel L;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        L.x_in[i] = q->x_in[i];
        L.xb_in[i] = q->xb_in[i];
        L.x_out[i] = q->x_out[i];
        L.xb_out[i] = q->xb_out[i];
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        L.y_in[i] = q->y_in[i];
        L.y_out[i] = q->y_out[i];
    }
    L.Ix = q->Ix;
    L.Iy = q->Iy;
    L.It = q->It;
    L.u0 = q->u0;
    L.v0 = q->v0;
    L.s_out = q->s_out;
    L.H = q->H;
    L.W = q->W;
    L.ld = q->ld;
    return L;
}

}  // namespace flowmi
