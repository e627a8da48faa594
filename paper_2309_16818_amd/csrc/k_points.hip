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
//                  to clear cells whose height lies above the ray.  Rays of
//                  up to kShortMax intermediate cells are walked one per
//                  lane; longer ones are listed for
//   k_clear_long   which walks each listed ray in segments of kSeg cells,
//                  one segment per lane, so that no lane walks a whole long
//                  ray while the rest of the chip idles.
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
static_assert(kChunk % kWG == 0, "whole points per ingest thread");

constexpr int kShortMax = 64;   // longest ray (intermediate cells) walked by one lane
constexpr int kSeg = 64;        // cells per lane segment of a long ray
constexpr int kLongRays = 64;   // long rays per k_clear_long workgroup
constexpr int kLongGrid = 2048; // k_clear_long workgroups at most
constexpr int kSegTable = 1024; // segments of a k_clear_long batch found by table, not search

// Clears the accumulators (`clr` in any order) and, if `hl` is given,
// copies the heights into logical order for the clearing march.
__global__ __launch_bounds__(256) void k_zero_accum(Grid g, int* __restrict__ n,
                                                    float* __restrict__ wsum,
                                                    float* __restrict__ ssum,
                                                    int* __restrict__ clr,
                                                    float* __restrict__ chsum, int Cb,
                                                    int* __restrict__ zero1,
                                                    const float* __restrict__ h,
                                                    float* __restrict__ hl,
                                                    DriftDev* __restrict__ drift)
{
    const int HW = g.W * g.H;
    if (zero1 && blockIdx.x == 0 && threadIdx.x == 0) *zero1 = 0;
    if (drift && blockIdx.x == 0 && threadIdx.x == 0) *drift = DriftDev{0.0, 0.0, 0, 0.0f};
    int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < HW; i += stride) {
        n[i] = 0;
        wsum[i] = 0.0f;
        ssum[i] = 0.0f;
        clr[i] = 0;
        for (int q = 0; q < Cb; q++) chsum[(int64_t)q * HW + i] = 0.0f;
        if (hl) {
            int ix, iy;
            logical_index(g, i, ix, iy);
            hl[iy * g.W + ix] = h[i];
        }
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
    ingest_range<kChunk / kWG>(g, xyz, begin, end, ch, T, c0, c1, mr2, pb, acc, lds, pc);
    const int ids[6] = {ST_ACCEPTED, ST_NONFINITE, ST_RANGE, ST_OUTSIDE, ST_POINTS_IN, ST_FLUSHES};
    int vals[6] = {pc.acc, pc.nonfinite, pc.range, pc.outside,
                   pc.acc + pc.nonfinite + pc.range + pc.outside, pc.flushed};
    block_stats(stats, ids, vals);
}

// One ray per lane.  Scan order puts rays of very different lengths side by
// side (the beams of one LiDAR firing), and a wave runs as long as its
// longest ray, so the workgroup first orders its 256 rays by length bucket
// (8 cells per bucket; a counting sort in LDS) and each wave walks 64 rays
// of similar length; neighbouring points stay in one workgroup, so the
// walks still share cache lines.  Rays longer than kShortMax cells (the
// last bucket) are appended to `longs` (indices into this launch's points)
// instead: workgroups whose points lie far away would otherwise hold their
// CU long after the rest of the grid has finished.
__global__ __launch_bounds__(256) void k_clear_march(Grid g, Grid gl, const float* __restrict__ hl,
                                                     const float* __restrict__ xyz, int64_t n, Pose T,
                                                     float mr2, float margin, int* __restrict__ clr,
                                                     int* __restrict__ longs,
                                                     int* __restrict__ n_long,
                                                     unsigned long long* __restrict__ stats)
{
    constexpr int kBuckets = kShortMax / 8 + 2;  // none, 1-8, ..., 57-64, long
    static_assert(kShortMax % 8 == 0, "length buckets of 8 cells");
    __shared__ int s_long_base;
    __shared__ int s_off[kBuckets];
    __shared__ int s_order[256];
    __shared__ int s_steps[256];
    __shared__ float4 s_pt[256];
    __shared__ int2 s_cell[256];
    const int t = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * 256 + t;
    float px = 0.f, py = 0.f, pz = 0.f, r2;
    int ix = 0, iy = 0, steps = 0;
    const float sx = T.m[3], sy = T.m[7], sz = T.m[11];
    int ax, ay;
    lattice_cell(g, sx, sy, ax, ay);
    if (i < n && point_cell(g, T, mr2, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], px, py, pz, r2, ix, iy) == 0)
        steps = max(max(abs(ix - ax), abs(iy - ay)) - 1, 0);
    s_steps[t] = steps;
    s_pt[t] = make_float4(px, py, pz, 0.f);
    s_cell[t] = make_int2(ix, iy);
    const int src = order_by_length<kBuckets>(steps, s_off, s_order);
    const int first_long = s_off[kBuckets - 1];  // the long rays are the last lanes
    if (t == 0) {
        const int nl = 256 - first_long;
        s_long_base = nl > 0 ? atomicAdd(n_long, nl) : 0;
    }
    __syncthreads();
    const int my_steps = s_steps[src];
    int visited = 0;
    if (t >= first_long) {
        longs[s_long_base + t - first_long] = (int)((int64_t)blockIdx.x * 256 + src);
    } else if (my_steps > 0) {
        const float4 p = s_pt[src];
        const int2 c = s_cell[src];
        Ray ray(gl, ax, ay, c.x, c.y, sx, sy, sz, p.x, p.y, p.z);
        visited = walk_logical<8>(gl, ray, hl, ClearVoteLogical{clr, g, margin});
    }
    const int ids[2] = {ST_RAY_CELLS, ST_RAY_STEPS};
    int vals[2] = {visited, steps};
    block_stats(stats, ids, vals);
}

// The listed long rays, kLongRays per workgroup: each ray is cut into
// segments of kSeg cells (the last one shorter) and the workgroup's lanes
// take the segments in turn, entering a ray mid-way with the closed-form
// Bresenham jump; the votes are those of walking every ray whole.
__global__ __launch_bounds__(256) void k_clear_long(Grid g, Grid gl, const float* __restrict__ hl,
                                                    const float* __restrict__ xyz, Pose T,
                                                    float mr2, float margin,
                                                    int* __restrict__ clr,
                                                    const int* __restrict__ longs,
                                                    const int* __restrict__ n_long,
                                                    unsigned long long* __restrict__ stats)
{
    __shared__ float4 s_pt[kLongRays];
    __shared__ int2 s_cell[kLongRays];
    __shared__ int s_pre[kLongRays + 1];  // exclusive prefix of the segment counts, then the total
    __shared__ uint16_t s_seg[kSegTable];  // segment q: its ray | (its index within the ray << 6)
    static_assert(kLongRays <= 64 && kSegTable <= 65536, "segment table entries are 16 bits");
    const int t = threadIdx.x;
    const int count = *n_long;
    const float sx = T.m[3], sy = T.m[7], sz = T.m[11];
    int ax, ay;
    lattice_cell(g, sx, sy, ax, ay);
    int visited = 0;
    for (int base = blockIdx.x * kLongRays; base < count; base += gridDim.x * kLongRays) {
        if (t < kLongRays) {  // wave 0 loads the rays and scans their segment counts
            int nseg = 0;
            float px = 0.f, py = 0.f, pz = 0.f, r2;
            int ix = 0, iy = 0;
            if (base + t < count) {
                const int64_t i = longs[base + t];
                if (point_cell(g, T, mr2, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], px, py, pz, r2, ix, iy) == 0)
                    nseg = (max(abs(ix - ax), abs(iy - ay)) - 1 + kSeg - 1) / kSeg;
            }
            s_pt[t] = make_float4(px, py, pz, 0.f);
            s_cell[t] = make_int2(ix, iy);
            int incl = nseg;
#pragma unroll
            for (int o = 1; o < kLongRays; o <<= 1) {
                const int u = __shfl_up(incl, o);
                if (t >= o) incl += u;
            }
            s_pre[t + 1] = incl;
            if (t == 0) s_pre[0] = 0;
            const int pre = incl - nseg;
            for (int k = 0; k < nseg && pre + k < kSegTable; k++) s_seg[pre + k] = (uint16_t)(t | (k << 6));
        }
        __syncthreads();
        const int total = s_pre[kLongRays];
        for (int q = t; q < total; q += 256) {
            int r, k;
            if (q < kSegTable) {
                const int e = s_seg[q];
                r = e & 63;
                k = e >> 6;
            } else {
                r = 0;  // the last ray whose first segment is at or before q
#pragma unroll
                for (int bit = kLongRays / 2; bit > 0; bit >>= 1)
                    if (s_pre[r + bit] <= q) r += bit;
                k = q - s_pre[r];
            }
            const float4 p = s_pt[r];
            const int2 c = s_cell[r];
            Ray ray(gl, ax, ay, c.x, c.y, sx, sy, sz, p.x, p.y, p.z);
            const int first = 1 + k * kSeg;
            const int cnt = min(kSeg, ray.L.steps - first);
            visited += walk_range_logical<8>(gl, ray, hl, first, cnt, ClearVoteLogical{clr, g, margin});
        }
        __syncthreads();  // the next batch overwrites the LDS tables
    }
    const int ids[1] = {ST_RAY_CELLS};
    int vals[1] = {visited};
    block_stats(stats, ids, vals);
}

// Block maxima of the height layer over logical cells: one wave per 8x8
// block (lane = cell), then one wave per 64x64 block over its 8x8 maxima.
__global__ __launch_bounds__(256) void k_tile_max8(Grid g, const float* __restrict__ h, float* __restrict__ t8,
                                                   int tw, int th)
{
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (tile >= tw * th) return;  // whole waves leave together
    const int tx = tile % tw, ty = tile / tw;
    const int x = tx * 8 + (lane & 7), y = ty * 8 + (lane >> 3);
    float v = -__builtin_inff();
    if (x < g.W && y < g.H) v = fmaxf(v, h[storage_index(g, x, y)]);  // NaN (no height) drops out
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    if (lane == 0) t8[tile] = v;
}

__global__ __launch_bounds__(256) void k_tile_max64(const float* __restrict__ t8, int tw8, int th8,
                                                    float* __restrict__ t64, int tw, int th)
{
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (tile >= tw * th) return;
    const int tx = tile % tw, ty = tile / tw;
    const int x = tx * 8 + (lane & 7), y = ty * 8 + (lane >> 3);
    float v = -__builtin_inff();
    if (x < tw8 && y < th8) v = t8[y * tw8 + x];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    if (lane == 0) t64[tile] = v;
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

// LDS of a k_ingest workgroup that reduces Cb channel planes in LDS: the
// kernel's static arrays as the compiler laid them out (the hash table and
// the per-block statistics) plus the dynamic channel sums; more than any
// device offers when Cb exceeds kMaxLdsCh.
size_t ingest_lds_bytes(int Cb)
{
    static const size_t fixed = [] {
        hipFuncAttributes a{};
        const bool ok = hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_ingest)) == hipSuccess;
        (void)hipGetLastError();
        return ok && a.sharedSizeBytes >= kStaticLds ? (size_t)a.sharedSizeBytes : kStaticLds + 1024;
    }();
    return fixed + (Cb > kMaxLdsCh ? (size_t)1 << 30 : sizeof(float) * kSlots * Cb);
}

void launch_zero_accum(hipStream_t s, const Grid& g, int* n, float* wsum, float* ssum, int* clr,
                       float* chsum, int Cb, int* zero1, const float* h, float* hl, DriftDev* drift)
{
    int HW = g.W * g.H;
    unsigned b = blocks_for(HW, 256);
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    hipLaunchKernelGGL(k_zero_accum, dim3(b), dim3(256), 0, s, g, n, wsum, ssum, clr, chsum, Cb, zero1, h, hl,
                       drift);
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

void launch_clear_march(hipStream_t s, const Grid& g_storage, const float* xyz, int64_t n, const Pose& T,
                        float mr2, float margin, const float* hl, int* clr, int* longs, int* n_long,
                        unsigned long long* stats)
{
    // the walks read heights in logical order: the grid without its ring offsets
    const Grid& g = g_storage;
    Grid gl = g_storage;
    gl.rx = 0;
    gl.ry = 0;
    // The long-ray list holds kMarchPass entries: clouds beyond that are
    // marched in passes, each pass clearing the list's counter first (the
    // first pass's counter was cleared with the accumulators).
    for (int64_t b = 0; b < n; b += kMarchPass) {
        const int64_t m = n - b < kMarchPass ? n - b : kMarchPass;
        if (b > 0) launch_zero_int(s, n_long, 1);
        hipLaunchKernelGGL(k_clear_march, dim3(blocks_for(m, 256)), dim3(256), 0, s, g, gl, hl, xyz + 3 * b, m, T,
                           mr2, margin, clr, longs, n_long, stats);
        unsigned grid_long = blocks_for(m, kLongRays);
        if (grid_long > kLongGrid) grid_long = kLongGrid;
        hipLaunchKernelGGL(k_clear_long, dim3(grid_long), dim3(256), 0, s, g, gl, hl, xyz + 3 * b, T, mr2, margin,
                           clr, longs, n_long, stats);
    }
}

TileMax tile_max_dims(const Grid& g, const float* t8, const float* t64)
{
    TileMax tm;
    tm.t8 = t8;
    tm.t64 = t64;
    tm.tw8 = (g.W + 7) / 8;
    tm.th8 = (g.H + 7) / 8;
    tm.tw64 = (g.W + 63) / 64;
    tm.th64 = (g.H + 63) / 64;
    return tm;
}

void launch_tile_max(hipStream_t s, const Grid& g, const float* h, float* t8, float* t64)
{
    const TileMax tm = tile_max_dims(g, t8, t64);
    const int n8 = tm.tw8 * tm.th8, n64 = tm.tw64 * tm.th64;
    hipLaunchKernelGGL(k_tile_max8, dim3((n8 + 3) / 4), dim3(256), 0, s, g, h, t8, tm.tw8, tm.th8);
    hipLaunchKernelGGL(k_tile_max64, dim3((n64 + 3) / 4), dim3(256), 0, s, t8, tm.tw8, tm.th8, t64, tm.tw64,
                       tm.th64);
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
