// BF16-operand matrix-core product with FP32 accumulation, shared by the
// single-problem and the batched matrix-core sweeps.
//
// v_mfma_f32_16x16x16_bf16 takes four consecutive K entries per lane where
// v_mfma_f32_16x16x4_f32 takes one, so the four operands a lane feeds to four
// FP32 steps go to one BF16 instruction.  The K index is then visited in
// another order, the same for A and B, which leaves the contraction
// unchanged.  Operands are rounded to nearest, ties to even, as they enter.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sfr {

typedef float mfma_f32x4 __attribute__((ext_vector_type(4)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float x)
{
    // round to nearest, ties to even (finite inputs)
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

__device__ __forceinline__ mfma_f32x4 mfma_bf16(const float (&a)[4], const float (&b)[4], mfma_f32x4 c)
{
    const bf16x4 av = {to_bf16(a[0]), to_bf16(a[1]), to_bf16(a[2]), to_bf16(a[3])};
    const bf16x4 bv = {to_bf16(b[0]), to_bf16(b[1]), to_bf16(b[2]), to_bf16(b[3])};
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, c, 0, 0, 0);
}

}  // namespace sfr
