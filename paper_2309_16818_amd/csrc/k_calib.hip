// k_calib.hip - calibration kernels behind the measured peaks of the
// benchmark: a streaming device copy (the HBM bandwidth a kernel can reach,
// and the scale of the profiler's FETCH_SIZE / WRITE_SIZE counters) and
// global atomic adds in the address patterns of the map update (the atomic
// rate a kernel can reach).  They compute nothing of the map update.
//
//   k_copy16     16-byte loads and stores, four per lane, coalesced: a wave
//                moves 4 x 1 KiB per pass; one pass per workgroup, enough
//                workgroups to cover the buffer (no grid-stride loop).
//   k_atomic     n_ops relaxed device-scope atomic adds of 1 (int32 or
//                binary32, no return value used) to buf[addr(i)]:
//                  unique   addr(i) = i              a wave's 64 lanes hit
//                                                    64 consecutive words
//                  scatter  addr(i) = perm(i)        a bijection of [0, n_addr),
//                                                    n_addr a power of two: the
//                                                    flush of a point ingest
//                  shared   addr(i) = i mod n_addr   few addresses, all lanes
//                                                    contend
#include <cstdint>
#include <cstdio>
#include <type_traits>

#include <hip/hip_runtime.h>

#include "mem_calib.h"

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kCopyWG = 256;
constexpr int kCopyPer = 4;  // 16-byte elements per lane

__global__ __launch_bounds__(kCopyWG) void k_copy16(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                   int64_t n)
{
    const int64_t base = (int64_t)blockIdx.x * (kCopyWG * kCopyPer) + threadIdx.x;
    u32x4 v[kCopyPer];
#pragma unroll
    for (int k = 0; k < kCopyPer; k++) {
        const int64_t i = base + (int64_t)k * kCopyWG;
        if (i < n) v[k] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int k = 0; k < kCopyPer; k++) {
        const int64_t i = base + (int64_t)k * kCopyWG;
        if (i < n) __builtin_nontemporal_store(v[k], dst + i);
    }
}

// A bijection of [0, 2^bits): multiplication by an odd constant and a
// xor-shift, both invertible modulo 2^bits.
__device__ __forceinline__ uint32_t scatter(uint32_t i, int bits)
{
    const uint32_t mask = bits >= 32 ? 0xffffffffu : ((1u << bits) - 1u);
    uint32_t x = (i * 2654435761u) & mask;
    x ^= x >> (bits / 2 + 1);
    return (x * 0x9E3779B1u) & mask;
}

template <typename T>
__global__ __launch_bounds__(256) void k_atomic(T* __restrict__ buf, int64_t n_ops, int64_t n_addr, int pattern,
                                                int bits)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_ops) return;
    int64_t a;
    if (pattern == MEM_CALIB_UNIQUE)
        a = i;
    else if (pattern == MEM_CALIB_SCATTER)
        a = scatter((uint32_t)i, bits);
    else
        a = i % n_addr;
    if constexpr (std::is_floating_point<T>::value)
        unsafeAtomicAdd(buf + a, static_cast<T>(1));
    else
        atomicAdd(buf + a, static_cast<T>(1));
}

thread_local char g_err[256];

int calib_fail(int code, const char* msg)
{
    snprintf(g_err, sizeof g_err, "%s", msg);
    return code;
}

}  // namespace

extern "C" {

const char* mem_calib_last_error(void)
{
    return g_err;
}

int mem_calib_copy(const void* src, void* dst, int64_t bytes, void* stream)
{
    if (!src || !dst) return calib_fail(-1, "NULL buffer");
    if (bytes < 0 || bytes % 16 != 0) return calib_fail(-1, "bytes must be a non-negative multiple of 16");
    if (((uintptr_t)src | (uintptr_t)dst) % 16 != 0) return calib_fail(-1, "buffers must be 16-byte aligned");
    const int64_t n = bytes / 16;
    if (n == 0) return 0;
    const int64_t per = (int64_t)kCopyWG * kCopyPer;
    const int64_t blocks = (n + per - 1) / per;
    if (blocks > 0x7fffffff) return calib_fail(-1, "copy too large");
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(kCopyWG), 0, (hipStream_t)stream,
                       static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return calib_fail(-3, hipGetErrorString(e));
    return 0;
}

int mem_calib_atomic(void* buf, int32_t dtype, int32_t pattern, int64_t n_ops, int64_t n_addr, void* stream)
{
    if (!buf) return calib_fail(-1, "NULL buffer");
    if (dtype != MEM_CALIB_I32 && dtype != MEM_CALIB_F32) return calib_fail(-1, "dtype must be I32 or F32");
    if (n_ops < 0 || n_ops > 0x7fffffffll * 256) return calib_fail(-1, "n_ops out of range");
    int bits = 0;
    if (pattern == MEM_CALIB_UNIQUE) {
        if (n_addr < n_ops) return calib_fail(-1, "unique: the buffer must hold n_ops words");
    } else if (pattern == MEM_CALIB_SCATTER) {
        if (n_addr < 1 || n_addr > (1ll << 32) || (n_addr & (n_addr - 1)) != 0)
            return calib_fail(-1, "scatter: n_addr must be a power of two up to 2^32");
        if (n_ops > n_addr) return calib_fail(-1, "scatter: n_ops must not exceed n_addr");
        while ((1ll << bits) < n_addr) bits++;
    } else if (pattern == MEM_CALIB_SHARED) {
        if (n_addr < 1) return calib_fail(-1, "shared: n_addr must be positive");
    } else {
        return calib_fail(-1, "unknown pattern");
    }
    if (n_ops == 0) return 0;
    const dim3 grid((unsigned)((n_ops + 255) / 256));
    hipStream_t s = (hipStream_t)stream;
    if (dtype == MEM_CALIB_I32)
        hipLaunchKernelGGL(k_atomic<int>, grid, dim3(256), 0, s, static_cast<int*>(buf), n_ops, n_addr, pattern, bits);
    else
        hipLaunchKernelGGL(k_atomic<float>, grid, dim3(256), 0, s, static_cast<float*>(buf), n_ops, n_addr, pattern,
                           bits);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return calib_fail(-3, hipGetErrorString(e));
    return 0;
}

}  // extern "C"
