// codec.h - layer storage element types (device side).
//
// Wide feature layers may be stored in bfloat16 or in OCP FP8 E4M3 ("fn":
// no infinities, 0x7F/0xFF are NaN, largest finite 448) with a per-channel
// scale; arithmetic is always binary32.  Encoding rounds to nearest even;
// FP8 saturates to +-448 before the scale is applied back.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/mem.h"
#include "mem_internal.h"

namespace memk {

__device__ __forceinline__ float bf16_to_f32(uint16_t b)
{
    return __uint_as_float(((uint32_t)b) << 16);
}

__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x0040u);  // quiet NaN
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

// E4M3 <-> binary32 with the GPU's conversion instructions, which use the
// OCP E4M3 ("fn") format on gfx950.  Decoding is exact.  The encoder rounds
// to nearest even; saturation comes from clamping to +-448 first (the
// instruction itself would turn overflow into NaN), and since the clamp
// turns a NaN into a number, NaN inputs are mapped to 0x7F separately.
// Equal, for all 2^32 binary32 inputs, to the textbook steps (split off the
// binade, scale the significand to [8, 16), round the integer, carry into
// the exponent, saturate), and to them for all 256 codes when decoding.
__device__ __forceinline__ float e4m3_to_f32(uint8_t c)
{
    return __builtin_amdgcn_cvt_f32_fp8((int)c, 0);
}

// Byte k (0..3, a compile-time constant after unrolling) of a word of four
// codes.
__device__ __forceinline__ float e4m3_word_to_f32(uint32_t w, int k)
{
    switch (k) {
    case 0: return __builtin_amdgcn_cvt_f32_fp8((int)w, 0);
    case 1: return __builtin_amdgcn_cvt_f32_fp8((int)w, 1);
    case 2: return __builtin_amdgcn_cvt_f32_fp8((int)w, 2);
    default: return __builtin_amdgcn_cvt_f32_fp8((int)w, 3);
    }
}

__device__ __forceinline__ float e4m3_clamp(float x) { return fminf(fmaxf(x, -448.0f), 448.0f); }

__device__ __forceinline__ uint8_t f32_to_e4m3(float x)
{
    const float y = e4m3_clamp(x);
    const uint32_t c = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(y, y, 0, false) & 0xffu;
    return x != x ? (uint8_t)0x7f : (uint8_t)c;
}

// Four values into one word of codes (value k in byte k).
__device__ __forceinline__ uint32_t f32x4_to_e4m3(float x0, float x1, float x2, float x3)
{
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(e4m3_clamp(x0), e4m3_clamp(x1), 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(e4m3_clamp(x2), e4m3_clamp(x3), w, true);
    uint32_t u = (uint32_t)w;
    if ((x0 != x0) | (x1 != x1) | (x2 != x2) | (x3 != x3)) {
        const float x[4] = {x0, x1, x2, x3};
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (x[k] != x[k]) u = (u & ~(0xffu << (8 * k))) | (0x7fu << (8 * k));
    }
    return u;
}

// v / s for a scale s given with r = 1 / s rounded to binary32: the product
// q0 = v r is within about one ulp of the quotient, the residual v - q0 s is
// exact in one fused multiply-add, and adding it back times r (Markstein's
// correction) gives the correctly rounded quotient.  Checked on the CPU
// (tests/fp8_divide_check.c) for all 2^32 v on 26 scales across
// 2^-60 .. 2^60 (the range scale_rcp_ok admits): equal
// bits wherever |v / s| lies in [2^-12, 2^9]; elsewhere the same sign and
// the same side of the E4M3 range (below half its least subnormal, above
// 448), so the E4M3 code is always that of the correctly rounded quotient.
// A product too large to correct (beyond 2^120, or infinite) saturates to
// +-448 either way and is kept; so is a zero product, which has the
// quotient's sign (the correction would turn -0 into +0); NaN stays NaN.
__device__ __forceinline__ float div_rcp(float v, float s, float r)
{
    const float q0 = v * r;
    if (!(fabsf(q0) <= 0x1p120f) || q0 == 0.0f) return q0;
    const float e = fmaf(-q0, s, v);
    return fmaf(e, r, q0);
}

// Element access by storage type.
template <int S>
struct Store;

template <>
struct Store<MEM_F32> {
    using T = float;
    __device__ __forceinline__ static float load(const void* p, int64_t i, float) { return ((const float*)p)[i]; }
    __device__ __forceinline__ static void store(void* p, int64_t i, float v, float) { ((float*)p)[i] = v; }
};

template <>
struct Store<MEM_BF16> {
    using T = uint16_t;
    __device__ __forceinline__ static float load(const void* p, int64_t i, float)
    {
        return bf16_to_f32(((const uint16_t*)p)[i]);
    }
    __device__ __forceinline__ static void store(void* p, int64_t i, float v, float)
    {
        ((uint16_t*)p)[i] = f32_to_bf16(v);
    }
};

template <>
struct Store<MEM_FP8_E4M3> {
    using T = uint8_t;
    __device__ __forceinline__ static float load(const void* p, int64_t i, float scale)
    {
        return e4m3_to_f32(((const uint8_t*)p)[i]) * scale;
    }
    __device__ __forceinline__ static void store(void* p, int64_t i, float v, float scale)
    {
        ((uint8_t*)p)[i] = f32_to_e4m3(v / scale);
    }
};

}  // namespace memk

namespace memk {

// Runtime-dispatched element access of a user layer (q = channel, for the
// FP8 per-channel scale).
__device__ __forceinline__ float layer_load(const void* val, int storage, const float* scale,
                                            int64_t idx, int q)
{
    switch (storage) {
    case MEM_BF16: return bf16_to_f32(((const uint16_t*)val)[idx]);
    case MEM_FP8_E4M3: return e4m3_to_f32(((const uint8_t*)val)[idx]) * scale[q];
    default: return ((const float*)val)[idx];
    }
}

__device__ __forceinline__ void layer_store(void* val, int storage, const float* scale, int64_t idx,
                                            int q, float v)
{
    switch (storage) {
    case MEM_BF16: ((uint16_t*)val)[idx] = f32_to_bf16(v); break;
    case MEM_FP8_E4M3: ((uint8_t*)val)[idx] = f32_to_e4m3(v / scale[q]); break;
    default: ((float*)val)[idx] = v; break;
    }
}

// Sums v[k] over the workgroup and adds each sum to counter id[k] with one
// atomic per workgroup.  Every thread of the workgroup must call it.
template <int N>
__device__ __forceinline__ void block_stats(unsigned long long* stats, const int (&id)[N], int (&v)[N])
{
    __shared__ int s[N];
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    if (tid < N) s[tid] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; k++) {
        int x = v[k];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if (__lane_id() == 0 && x != 0) atomicAdd(&s[k], x);
    }
    __syncthreads();
    if (tid < N && s[tid] != 0) {
        int slot = (int)((blockIdx.x + gridDim.x * blockIdx.y) % kStatSlots);
        atomicAdd(&stats[id[tid] * kStatSlots + slot], (unsigned long long)s[tid]);
    }
}

}  // namespace memk
