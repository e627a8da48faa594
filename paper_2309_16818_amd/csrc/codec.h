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

__device__ __forceinline__ float e4m3_to_f32(uint8_t c)
{
    uint32_t e = (c >> 3) & 0xfu, m = c & 7u;
    if (e == 0xfu && m == 7u) return __uint_as_float(0x7fc00000u);
    float v = (e == 0) ? (float)m * 0.001953125f  // m * 2^-9
                       : ldexpf(1.0f + (float)m * 0.125f, (int)e - 7);
    return (c & 0x80u) ? -v : v;
}

__device__ __forceinline__ uint8_t f32_to_e4m3(float x)
{
    if (isnan(x)) return 0x7f;
    uint8_t sign = signbit(x) ? 0x80 : 0x00;
    float a = fabsf(x);
    if (a >= 448.0f) return sign | 0x7e;
    if (a < 0.015625f) {  // below 2^-6: quantum 2^-9; m == 8 is the smallest normal
        int m = (int)rintf(a * 512.0f);
        return sign | (uint8_t)m;
    }
    int E;
    frexpf(a, &E);     // a = f 2^E, f in [0.5, 1)
    int e = E - 1;     // a in [2^e, 2^(e+1)), e in [-6, 8]
    float q = ldexpf(a, 3 - e);  // a / 2^(e-3), in [8, 16)
    int m = (int)rintf(q);
    if (m == 16) {
        m = 8;
        e += 1;
    }
    int code = ((e + 7) << 3) | (m - 8);
    if (code > 0x7e) code = 0x7e;
    return sign | (uint8_t)code;
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
