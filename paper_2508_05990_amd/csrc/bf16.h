// bfloat16 helpers and the bfloat16 MFMA used by the network kernels.
//
// v_mfma_f32_16x16x16_bf16 takes, per lane L (g = L / 16): A[m = L%16]
// [k = 4g..4g+3], B[k = 4g..4g+3][n = L%16], and returns D[m = 4g+i][n = L%16]
// for i = 0..3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace me {

typedef short v4i16 __attribute__((ext_vector_type(4)));
typedef float v4f32 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// Round to nearest even (gfx950's v_cvt_pk_bf16_f32: two values per
// instruction); NaN stays NaN.
__device__ __forceinline__ uint32_t pack2(float a, float b)
{
    const bf16x2_t v = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

__device__ __forceinline__ v4i16 as_v4(uint2 u)
{
    v4i16 r;
    r.x = (short)(u.x & 0xffff);
    r.y = (short)(u.x >> 16);
    r.z = (short)(u.y & 0xffff);
    r.w = (short)(u.y >> 16);
    return r;
}

__device__ __forceinline__ uint2 pack4(float a, float b, float c, float d) { return make_uint2(pack2(a, b), pack2(c, d)); }

__device__ __forceinline__ float4 unpack4(uint2 u)
{
    return make_float4(bf2f((uint16_t)(u.x & 0xffff)), bf2f((uint16_t)(u.x >> 16)), bf2f((uint16_t)(u.y & 0xffff)),
                       bf2f((uint16_t)(u.y >> 16)));
}

__device__ __forceinline__ v4f32 mfma(v4i16 a, v4i16 b, v4f32 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

}  // namespace me
