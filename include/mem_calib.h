/* mem_calib.h - calibration kernels of libmem.so for the measured peaks
 * that the map update's kernels are compared with: the device copy rate
 * (the HBM bandwidth a kernel can reach, and the bytes per unit of the
 * profiler's FETCH_SIZE / WRITE_SIZE counters) and the rate of global
 * atomic adds in the address patterns the point ingest uses.  They compute
 * nothing of the map update.  All pointers are device memory owned by the
 * caller; calls are asynchronous on `stream` (a hipStream_t, NULL = the
 * default stream) and never wait.  Return 0, or -1 for an invalid argument
 * (nothing enqueued) or -3 for a launch error; mem_calib_last_error() holds
 * the message (per thread). */
#ifndef MEM_CALIB_H
#define MEM_CALIB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { MEM_CALIB_I32 = 0, MEM_CALIB_F32 = 1 };
enum { MEM_CALIB_UNIQUE = 0, MEM_CALIB_SCATTER = 1, MEM_CALIB_SHARED = 2 };

/* Copies `bytes` (a multiple of 16; both buffers 16-byte aligned, not
 * overlapping) from src to dst with 16-byte non-temporal loads and stores,
 * four per lane, one pass per workgroup of 256 lanes. */
int mem_calib_copy(const void* src, void* dst, int64_t bytes, void* stream);

/* n_ops relaxed device-scope atomic adds of 1 (dtype MEM_CALIB_I32: int32
 * atomicAdd; MEM_CALIB_F32: binary32 add, no return value) into buf, one
 * per lane, operation i to word
 *   MEM_CALIB_UNIQUE   i                (buf holds n_addr >= n_ops words),
 *   MEM_CALIB_SCATTER  a fixed bijection of [0, n_addr) taken at i
 *                      (n_addr a power of two <= 2^32, n_ops <= n_addr): every
 *                      word at most once, neighbouring lanes far apart,
 *   MEM_CALIB_SHARED   i mod n_addr     (all lanes contend for n_addr words).
 * The caller clears buf beforehand if it checks the counts. */
int mem_calib_atomic(void* buf, int32_t dtype, int32_t pattern, int64_t n_ops, int64_t n_addr, void* stream);

const char* mem_calib_last_error(void);

#ifdef __cplusplus
}
#endif

#endif
