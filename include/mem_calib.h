/* mem_calib.h - calibration kernels of libmem.so for the measured peaks
 * that the map update's kernels are compared with: the device copy rate
 * (the HBM bandwidth a kernel can reach, and the bytes per unit of the
 * profiler's FETCH_SIZE / WRITE_SIZE counters), the rate of global
 * atomic adds in the address patterns the point ingest uses and the rate of
 * scattered loads from a cache-resident table (the clearing walk's loads).  They compute
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

/* n_lanes x per_lane 4-byte loads from buf, a table of n_words floats (a
 * power of two up to 2^30; 2^18 words, 1 MiB, stays in the caches as a
 * map's height copy does): lane i loads, for j = 0 .. per_lane - 1, word
 * perm(i * per_lane + j) (runs = 0; perm the bijection of MEM_CALIB_SCATTER)
 * or word (perm(i) + j) mod n_words (runs = 1: a run of consecutive words
 * per lane), eight loads in flight at a time, and writes the sum of the
 * values it loaded to out[i] (n_lanes floats).  per_lane: a positive
 * multiple of 8 up to 2^20.  The two rates bracket a walk over the heights
 * (one cell per lane and load; a line's cells are neighbours along its
 * major axis). */
int mem_calib_gather(const float* buf, int64_t n_words, float* out, int64_t n_lanes, int32_t per_lane,
                     int32_t runs, void* stream);

const char* mem_calib_last_error(void);

#ifdef __cplusplus
}
#endif

#endif
