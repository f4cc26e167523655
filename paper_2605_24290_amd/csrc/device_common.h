// Device helpers shared by the forward and backward kernels of librxgs.
#pragma once

#include "rxgs_internal.h"

namespace rxgs {

typedef float floatx16 __attribute__((ext_vector_type(16)));

// Blend exponent of one (pixel, record): log2 of o exp(-q/2), with the record
// holding (-a/2, -b, -c/2) log2(e) and log2(o).  Written with explicit fmaf so
// that the forward and the backward evaluate bit-identical weights.
__device__ __forceinline__ float blend_exponent(float du, float dv, const float4 &r1)
{
    return fmaf(du, fmaf(r1.x, du, r1.y * dv), fmaf(r1.z * dv, dv, r1.w));
}

// Hidden-unit order of the MLP on MFMA.  Lane half h (lanes 0-31 / 32-63) at
// step t (0..31) handles hidden unit hid_of(h, t); the same map gives the rows
// an MFMA 32x32 accumulator leaves in lane half h, register r of block b
// (t = 16 b + r), so layer-2 inputs, layer-2 outputs and the backward's
// layer-1 gradients line up register by register.
__host__ __device__ __forceinline__ int hid_of(int h, int t)
{
    return 8 * ((t & 15) >> 2) + 4 * h + (t & 3) + 32 * (t >> 4);
}
// position of hidden unit d in a row stored in that order (h * 32 + t)
__host__ __device__ __forceinline__ int hid_pos(int d)
{
    const int h = (d & 7) >> 2;
    const int t = 16 * (d >> 5) + 4 * ((d & 31) >> 3) + (d & 3);
    return h * 32 + t;
}

// DPP move (row_shr, row_bcast, ...) with masked-off or out-of-row lanes reading 0
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_shift(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, ROW_MASK,
                                                                 0xf, false));
}

// Sum over each 32-lane half of the wave; lanes 31 and 63 hold the two sums.
__device__ __forceinline__ float half_wave_sum(float x)
{
    x += dpp_shift<0x111, 0xf>(x);   // row_shr:1
    x += dpp_shift<0x112, 0xf>(x);   // row_shr:2
    x += dpp_shift<0x114, 0xf>(x);   // row_shr:4
    x += dpp_shift<0x118, 0xf>(x);   // row_shr:8
    x += dpp_shift<0x142, 0xa>(x);   // row_bcast:15 into rows 1 and 3
    return x;
}

// Sum over the whole wave; lane 63 holds the sum.
__device__ __forceinline__ float wave_sum_last(float x)
{
    x = half_wave_sum(x);
    x += dpp_shift<0x143, 0xc>(x);   // row_bcast:31 into rows 2 and 3
    return x;
}

}  // namespace rxgs
