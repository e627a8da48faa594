// k_points.hip - point-cloud path of the map update (one map).
//
//   k_zero_accum   clears the per-cloud accumulators (dense, HBM-bound).
//   k_ingest       point transform + cell association (Sec. III-B) and
//                  LDS-binned per-cell sums: a workgroup hashes its 1024
//                  points into an LDS table keyed by cell, reduces equal cells
//                  with LDS atomics, then issues one global atomic per
//                  (cell, field) it saw.
//   k_clear_march  the ray cast of Table I's "height update & ray cast":
//                  one ray per accepted point along Bresenham's line, voting
//                  to clear cells whose height lies above the ray.
//   k_finalize     per-cell information-form Gaussian height fusion, clear
//                  application, and fusion of bound point channels with the
//                  layer's rule (Sec. III-C, Eq. (1), (2), (6)-(7), (12)).
#include "update.h"

namespace memk {

namespace {

constexpr int kWG = 256;
constexpr int kChunk = 1024;             // points per ingest workgroup
constexpr int kSlotsLog2 = 11;
constexpr int kSlots = 1 << kSlotsLog2;  // LDS hash slots (2 x points)
constexpr int kMaxLdsCh = 16;            // bound channels reduced in LDS at most
constexpr size_t kStaticLds = sizeof(int) * 2 * kSlots + sizeof(float) * 2 * kSlots + sizeof(float2) * kSlots;

static_assert(kSlots >= 2 * kChunk, "hash table must never fill");

__global__ __launch_bounds__(256) void k_zero_accum(int HW, int* __restrict__ n,
                                                    float* __restrict__ wsum,
                                                    float* __restrict__ ssum,
                                                    int* __restrict__ clr,
                                                    float* __restrict__ chsum, int Cb)
{
    int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < HW; i += stride) {
        n[i] = 0;
        wsum[i] = 0.0f;
        ssum[i] = 0.0f;
        clr[i] = 0;
        for (int q = 0; q < Cb; q++) chsum[(int64_t)q * HW + i] = 0.0f;
    }
}

__global__ __launch_bounds__(kWG) void k_ingest(Grid g, const float* __restrict__ xyz, int64_t n,
                                                const float* __restrict__ ch, Pose T, float c0,
                                                float c1, float mr2, PointBinds pb, Accum acc,
                                                unsigned long long* __restrict__ stats)
{
    __shared__ int s_key[kSlots];
    __shared__ int s_cnt[kSlots];
    __shared__ float s_w[kSlots];
    __shared__ float s_s[kSlots];
    __shared__ float2 s_first[kSlots];
    extern __shared__ float s_ch[];  // [Cb][kSlots] when the channels fit in LDS
    const IngestLds lds{s_key, s_cnt, s_w, s_s, s_first, s_ch, kSlotsLog2};

    const int64_t begin = (int64_t)blockIdx.x * kChunk;
    const int64_t end = begin + kChunk < n ? begin + kChunk : n;
    PointCounts pc;
    ingest_range(g, xyz, begin, end, ch, T, c0, c1, mr2, pb, acc, lds, pc);
    const int ids[5] = {ST_ACCEPTED, ST_NONFINITE, ST_RANGE, ST_OUTSIDE, ST_POINTS_IN};
    int vals[5] = {pc.acc, pc.nonfinite, pc.range, pc.outside,
                   pc.acc + pc.nonfinite + pc.range + pc.outside};
    block_stats(stats, ids, vals);
}

__global__ __launch_bounds__(256) void k_clear_march(Grid g, const float* __restrict__ xyz,
                                                     int64_t n, Pose T, float mr2, float margin,
                                                     const float* __restrict__ h,
                                                     int* __restrict__ clr,
                                                     unsigned long long* __restrict__ stats)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int visited = (i < n) ? march_point(g, xyz, i, T, mr2, margin, h, clr) : 0;
    const int ids[1] = {ST_RAY_CELLS};
    int vals[1] = {visited};
    block_stats(stats, ids, vals);
}

__global__ __launch_bounds__(256) void k_finalize(Grid g, Accum acc, int clear_min,
                                                  float* __restrict__ h, float* __restrict__ v,
                                                  PointBinds pb,
                                                  unsigned long long* __restrict__ stats)
{
    const int st = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = (st < acc.HW) ? finalize_cell(st, acc, clear_min, h, v, pb) : 0;
    const int ids[2] = {ST_TOUCHED, ST_CLEARED};
    int vals[2] = {r == 1 ? 1 : 0, r == 2 ? 1 : 0};
    block_stats(stats, ids, vals);
}

__global__ __launch_bounds__(256) void k_point_cells(Grid g, const float* __restrict__ xyz,
                                                     int64_t n, Pose T, float mr2,
                                                     int32_t* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float px, py, pz, r2;
    int ix = 0, iy = 0;
    int r = point_cell(g, T, mr2, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], px, py, pz, r2, ix, iy);
    out[i] = (r == 0) ? iy * g.W + ix : r;
}

inline unsigned blocks_for(int64_t n, int per)
{
    return (unsigned)((n + per - 1) / per);
}

}  // namespace

size_t ingest_lds_bytes(int Cb)
{
    return kStaticLds + (Cb > kMaxLdsCh ? (size_t)1 << 30 : sizeof(float) * kSlots * Cb);
}

void launch_zero_accum(hipStream_t s, const Grid& g, int* n, float* wsum, float* ssum, int* clr,
                       float* chsum, int Cb)
{
    int HW = g.W * g.H;
    unsigned b = blocks_for(HW, 256);
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(k_zero_accum, dim3(b), dim3(256), 0, s, HW, n, wsum, ssum, clr, chsum, Cb);
}

void launch_ingest(hipStream_t s, const Grid& g, const float* xyz, int64_t n, const float* ch,
                   const Pose& T, float c0, float c1, float mr2, const PointBinds& pb, int* cnt,
                   float* wsum, float* ssum, float2* stash, float* chsum,
                   unsigned long long* stats)
{
    if (n <= 0) return;
    const Accum acc{cnt, wsum, ssum, stash, nullptr, chsum, g.W * g.H};
    const size_t lds = pb.lds_ch ? sizeof(float) * kSlots * pb.Cb : 0;
    hipLaunchKernelGGL(k_ingest, dim3(blocks_for(n, kChunk)), dim3(kWG), lds, s, g, xyz, n, ch, T,
                       c0, c1, mr2, pb, acc, stats);
}

void launch_clear_march(hipStream_t s, const Grid& g, const float* xyz, int64_t n, const Pose& T,
                        float mr2, float margin, const float* h, int* clr,
                        unsigned long long* stats)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_clear_march, dim3(blocks_for(n, 256)), dim3(256), 0, s, g, xyz, n, T, mr2,
                       margin, h, clr, stats);
}

void launch_finalize(hipStream_t s, const Grid& g, const int* cnt, const float* wsum,
                     const float* ssum, const float2* stash, const int* clr, int clear_min,
                     float* h, float* v, const float* chsum, const PointBinds& pb,
                     unsigned long long* stats)
{
    const int HW = g.W * g.H;
    const Accum acc{const_cast<int*>(cnt), const_cast<float*>(wsum), const_cast<float*>(ssum),
                    const_cast<float2*>(stash), const_cast<int*>(clr), const_cast<float*>(chsum), HW};
    hipLaunchKernelGGL(k_finalize, dim3(blocks_for(HW, 256)), dim3(256), 0, s, g, acc, clear_min, h,
                       v, pb, stats);
}

void launch_point_cells(hipStream_t s, const Grid& g, const float* xyz, int64_t n, const Pose& T,
                        float mr2, int32_t* out)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_point_cells, dim3(blocks_for(n, 256)), dim3(256), 0, s, g, xyz, n, T, mr2,
                       out);
}

}  // namespace memk
