// Wave-level device helpers shared by the SGD, prediction and loss kernels.
#pragma once

#include "common.hpp"

namespace lshmf {

template <int CTRL, int ROW_MASK, bool BOUND_ZERO>
__device__ inline float dpp_f32(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, ROW_MASK,
                                                                 0xF, BOUND_ZERO));
}

// FP32 -> BF16 with round-to-nearest-even on the dropped 16 bits (NaN stays
// a quiet NaN).
__device__ inline uint16_t to_bf16(float x)
{
    const uint32_t u = __float_as_uint(x);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)0x7FC0u;
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ inline float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Full 64-lane sum with DPP row operations; the total ends in lane 63 and is
// broadcast through a scalar register.  Fixed association order.  The two
// row_bcast steps are single DPP adds (the compiler would emit a move of zero,
// a DPP move and an add for each); rows they leave disabled keep their value,
// which lane 63 never reads.  The s_nop before each gives the DPP read the two
// wait states a VALU result needs (the compiler does not look inside asm).
__device__ inline float wave_sum(float v)
{
    v += dpp_f32<0xB1, 0xF, true>(v);    // quad_perm [1,0,3,2]
    v += dpp_f32<0x4E, 0xF, true>(v);    // quad_perm [2,3,0,1]
    v += dpp_f32<0x141, 0xF, true>(v);   // row_half_mirror
    v += dpp_f32<0x140, 0xF, true>(v);   // row_mirror: every lane holds its row's sum
    asm volatile(
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"  // rows 1, 3 += lane 15, 47
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf"  // rows 2, 3 += lane 31
        : "+v"(v));
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

}  // namespace lshmf
