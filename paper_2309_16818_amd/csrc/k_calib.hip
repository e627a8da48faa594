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
//   k_gather     4-byte loads from a small (cache-resident) table, eight in
//                flight per lane, scattered or in per-lane runs of
//                consecutive words: the load rates that bracket a walk over
//                the heights, one cell per lane and load.
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

// Lane i loads per_lane words of the table (2^bits words), eight at a time
// (their addresses computed before any is loaded), and writes the sum of
// what it loaded to out[i]: words scatter(i * per_lane + j) (runs = 0), or
// the run of consecutive words from scatter(i) on, wrapping (runs = 1).
__global__ __launch_bounds__(256) void k_gather(const float* __restrict__ buf, int bits, float* __restrict__ out,
                                                int64_t n_lanes, int per_lane, int runs)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_lanes) return;
    float acc = 0.0f;
    const uint32_t base = (uint32_t)(i * per_lane);
    const uint32_t start = scatter((uint32_t)i, bits), mask = (1u << bits) - 1u;
    for (int j = 0; j < per_lane; j += 8) {
        uint32_t a[8];
#pragma unroll
        for (int u = 0; u < 8; u++)
            a[u] = runs ? (start + (uint32_t)(j + u)) & mask : scatter(base + (uint32_t)(j + u), bits);
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) v[u] = buf[a[u]];
#pragma unroll
        for (int u = 0; u < 8; u++) acc += v[u];
    }
    out[i] = acc;
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

int mem_calib_gather(const float* buf, int64_t n_words, float* out, int64_t n_lanes, int32_t per_lane, int32_t runs,
                     void* stream)
{
    if (runs != 0 && runs != 1) return calib_fail(-1, "runs must be 0 or 1");
    if (!buf || !out) return calib_fail(-1, "NULL buffer");
    if (n_words < 1 || n_words > (1ll << 30) || (n_words & (n_words - 1)) != 0)
        return calib_fail(-1, "n_words must be a power of two up to 2^30");
    if (n_lanes < 0 || n_lanes > 0x7fffffffll * 256) return calib_fail(-1, "n_lanes out of range");
    if (per_lane < 8 || per_lane % 8 != 0 || per_lane > (1 << 20))
        return calib_fail(-1, "per_lane must be a positive multiple of 8 up to 2^20");
    int bits = 0;
    while ((1ll << bits) < n_words) bits++;
    if (n_lanes == 0) return 0;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)((n_lanes + 255) / 256)), dim3(256), 0, (hipStream_t)stream, buf, bits,
                       out, n_lanes, per_lane, runs);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return calib_fail(-3, hipGetErrorString(e));
    return 0;
}
}  // extern "C"
