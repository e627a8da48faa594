// k_points.hip - point-cloud path of the map update (one map).
//
//   k_zero_accum   clears the per-cloud accumulators (dense, HBM-bound).
//   k_ingest       point transform + cell association (Sec. III-B) and
//                  LDS-binned per-cell sums: a workgroup hashes its 1024
//                  points into an LDS table keyed by cell, reduces equal cells
//                  with LDS atomics, then issues one global atomic per
//                  (cell, field) it saw.
//   k_ray_prep     the ray cast of Table I's "height update & ray cast":
//                  one ray per accepted point along Bresenham's line, voting
//                  to clear cells whose height lies above the ray.  Lists
//                  every ray's segments of kSegLen cells, full ones apart
//                  from each ray's shorter last one, for
//   k_ray_walk     which walks one segment per lane, full segments first,
//                  so that the waves walk segments of equal length.
//   k_finalize     per-cell information-form Gaussian height fusion, clear
//                  application, and fusion of bound point channels with the
//                  layer's rule (Sec. III-C, Eq. (1), (2), (6)-(7), (12)).
#include <algorithm>
#include <cmath>

#include "update.h"

namespace memk {

namespace {

constexpr int kWG = 512;              // threads per ingest workgroup (two points each; 256 and 1024 measured slower)
constexpr int kChunk = 1024;             // points per ingest workgroup
constexpr int kSlotsLog2 = 11;
constexpr int kSlots = 1 << kSlotsLog2;  // LDS hash slots (2 x points)
constexpr int kMaxLdsCh = 16;            // bound channels reduced in LDS at most
constexpr size_t kStaticLds = sizeof(int) * 2 * kSlots + sizeof(float) * 2 * kSlots + sizeof(float2) * kSlots;

static_assert(kSlots >= 2 * kChunk, "hash table must never fill");
static_assert(kChunk % kWG == 0, "whole points per ingest thread");

constexpr int kWalkGrid = 1280;  // k_ray_walk workgroups: about five per CU

// Clears the accumulators (`clr` in any order) and, if `hl` is given,
// copies the heights into logical order for the clearing march.
__global__ __launch_bounds__(256) void k_zero_accum(Grid g, int* __restrict__ n,
                                                    float* __restrict__ wsum,
                                                    float* __restrict__ ssum,
                                                    int* __restrict__ clr,
                                                    float* __restrict__ chsum, int Cb,
                                                    int* __restrict__ march_counts,
                                                    const float* __restrict__ h,
                                                    float* __restrict__ hl,
                                                    DriftDev* __restrict__ drift)
{
    const int HW = g.W * g.H;
    if (march_counts && blockIdx.x == 0)
        for (int k = threadIdx.x; k < kSegLists * kSegSubs; k += blockDim.x) march_counts[k] = 0;
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
                                                MarchBufs mb, int march, unsigned long long* __restrict__ stats)
{
    __shared__ int s_march[kMarchLds];
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
    ingest_range<kChunk / kWG>(g, xyz, begin, end, ch, T, c0, c1, mr2, pb, acc, lds, pc, march != 0, mb, s_march);
    const int ids[8] = {ST_ACCEPTED,  ST_NONFINITE, ST_RANGE,     ST_OUTSIDE,
                        ST_POINTS_IN, ST_FLUSHES,   ST_RAY_STEPS, ST_SEGMENTS};
    int vals[8] = {pc.acc,     pc.nonfinite, pc.range,     pc.outside, pc.acc + pc.nonfinite + pc.range + pc.outside,
                   pc.flushed, pc.ray_steps, pc.ray_segs};
    block_stats(stats, ids, vals);
}

// k_ingest over several clouds in one launch (grid row y = cloud): each
// cloud bins into its own sums and ray lists, so the clouds' workgroups
// are independent; a workgroup past its cloud's points leaves at once.
__global__ __launch_bounds__(kWG) void k_ingest_clouds(Grid g, IngestClouds cl, float c0, float c1, float mr2,
                                                       PointBinds pb, unsigned long long* __restrict__ stats)
{
    __shared__ int s_march[kMarchLds];
    __shared__ int s_key[kSlots];
    __shared__ int s_cnt[kSlots];
    __shared__ float s_w[kSlots];
    __shared__ float s_s[kSlots];
    __shared__ float2 s_first[kSlots];
    const IngestLds lds{s_key, s_cnt, s_w, s_s, s_first, nullptr, kSlotsLog2};

    const IngestCloud& C = cl.c[blockIdx.y];
    const int64_t begin = (int64_t)blockIdx.x * kChunk;
    if (begin >= C.n) return;  // the whole workgroup
    const int64_t end = begin + kChunk < C.n ? begin + kChunk : C.n;
    const Accum acc{C.cnt, C.wsum, C.ssum, C.stash, nullptr, nullptr, g.W * g.H};
    PointCounts pc;
    ingest_range<kChunk / kWG>(g, C.xyz, begin, end, nullptr, C.T, c0, c1, mr2, pb, acc, lds, pc, true, C.mb,
                               s_march);
    const int ids[8] = {ST_ACCEPTED,  ST_NONFINITE, ST_RANGE,     ST_OUTSIDE,
                        ST_POINTS_IN, ST_FLUSHES,   ST_RAY_STEPS, ST_SEGMENTS};
    int vals[8] = {pc.acc,     pc.nonfinite, pc.range,     pc.outside, pc.acc + pc.nonfinite + pc.range + pc.outside,
                   pc.flushed, pc.ray_steps, pc.ray_segs};
    block_stats(stats, ids, vals);
}

// The clearing march in two kernels.  k_ray_prep (one lane per point)
// transforms the point, stores the ray's record (its cell, the reciprocal
// of its major extent and its height difference)
// and lists the ray's segments of kSegLen cells: every full segment in the
// full list and the last, shorter segment (if any) in one of four lists by
// its length (for 64-cell segments: 48-63, 32-47, 16-31, 1-15 cells).  Each list is split into
// kSegSubs sub-lists with their own counters (workgroup b appends to
// sub-list b mod kSegSubs, reserving its room with one atomic per list), so
// no counter sees more than 1 / kSegSubs of the workgroups: atomics on one
// address serialise.  k_ray_walk then hands each lane one segment in the
// order full list, then the partial lists from the longest, so the lanes of
// a wave walk segments of nearly equal length, every wave of the grid is
// full, and no wave walks a whole long ray while others idle.  Each lane
// enters its ray mid-way with the closed-form Bresenham jump; the votes are
// those of walking every ray whole (integer atomics, any order).
__global__ __launch_bounds__(256) void k_ray_prep(Grid g, const float* __restrict__ xyz, int64_t n, Pose T,
                                                  float mr2, MarchBufs mb, unsigned long long* __restrict__ stats)
{
    __shared__ int s_march[kMarchLds];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float px = 0.f, py = 0.f, pz = 0.f, r2;
    int ix = 0, iy = 0;
    int ax, ay;
    lattice_cell(g, T.m[3], T.m[7], ax, ay);
    int steps[1] = {0};
    const int ri[1] = {(int)i};  // a pass holds at most kMarchPass points
    if (i < n && point_cell(g, T, mr2, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], px, py, pz, r2, ix, iy) == 0)
        steps[0] = max(max(abs(ix - ax), abs(iy - ay)) - 1, 0);
    if (steps[0] > 0) {
        // the walks need the ray's reciprocal major extent and height
        // difference, computed once here
        const Ray ray(g, ax, ay, ix, iy, T.m[3], T.m[7], T.m[11], px, py, pz);
        mb.rec[i] = make_float4(ray.inv_d, ray.dz, __int_as_float(ix | (iy << 16)), 0.0f);
    }
    march_lists<1>(mb, ri, steps, s_march);
    const int ids[2] = {ST_RAY_STEPS, ST_SEGMENTS};
    int vals[2] = {steps[0], (steps[0] + kSegLen - 1) / kSegLen};
    block_stats(stats, ids, vals);
}

__global__ __launch_bounds__(256) void k_ray_walk(Grid g, Grid gl, const float* __restrict__ hl, Pose T,
                                                  float margin, int* __restrict__ clr, MarchBufs mb,
                                                  unsigned long long* __restrict__ stats)
{
    constexpr int NS = kSegLists * kSegSubs;
    // exclusive prefix of the sub-lists' counts in walk order (list-major)
    __shared__ int s_pre[NS + 1];
    __shared__ int s_wave[4];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    {
        static_assert(NS <= 2 * 256, "two sub-lists per thread");
        // entries t and t + 256 of the list-major order: a workgroup scan of
        // the first 256, then of the rest on top of their total
        // counts clamped to the capacities (which bound them by construction)
        auto count = [&](int e) {
            const int64_t cap = e < kSegSubs ? mb.full_sub : mb.part_sub;
            return e < NS ? (int)min((int64_t)mb.counts[e], cap) : 0;
        };
        const int a = count(t);
        const int b = count(t + 256);
        int incl = a;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(incl, o);
            if (lane >= o) incl += u;
        }
        if (lane == 63) s_wave[w] = incl;
        __syncthreads();
        int base = 0;
        for (int k = 0; k < w; k++) base += s_wave[k];
        const int tot_a = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
        if (t < NS) s_pre[t] = base + incl - a;
        __syncthreads();
        int incl_b = b;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(incl_b, o);
            if (lane >= o) incl_b += u;
        }
        if (lane == 63) s_wave[w] = incl_b;
        __syncthreads();
        int base_b = tot_a;
        for (int k = 0; k < w; k++) base_b += s_wave[k];
        if (t + 256 < NS) s_pre[t + 256] = base_b + incl_b - b;
        if (t == 255) s_pre[NS] = base_b + incl_b;
        __syncthreads();
    }
    const int total = s_pre[NS];
    const float sx = T.m[3], sy = T.m[7], sz = T.m[11];
    int ax, ay;
    lattice_cell(g, sx, sy, ax, ay);
    const int wave = blockIdx.x * 4 + w, nwaves = gridDim.x * 4;
    int visited = 0;
    // wave-sized chunks of the concatenated sub-lists, dealt to the waves in turn
    for (int q0 = wave * 64; q0 < total; q0 += nwaves * 64) {
        const int q = q0 + lane;
        if (q >= total) continue;
        int lo = 0, hi = NS;  // s_pre[lo] <= q < s_pre[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_pre[mid] <= q) lo = mid;
            else hi = mid;
        }
        const int local = q - s_pre[lo];
        const int2 e = lo < kSegSubs ? mb.full[(int64_t)lo * mb.full_sub + local]
                                     : mb.part[(int64_t)(lo - kSegSubs) * mb.part_sub + local];
        const float4 p = mb.rec[e.x];
        const int cell = __float_as_int(p.z);
        Ray ray(gl, ax, ay, cell & 0xffff, cell >> 16, sx, sy, sz, p.x, p.y, 0);
        const int first = 1 + e.y * kSegLen;
        const int cnt = min(kSegLen, ray.L.steps - first);
        visited += walk_votes<8>(gl, ray, hl, first, cnt, ClearVoteLogical{clr, g, margin});
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
                                                  unsigned long long* __restrict__ stats, int clean,
                                                  int* __restrict__ zero_cnt, int* __restrict__ zero_clr,
                                                  float* __restrict__ hl, int* __restrict__ march_counts,
                                                  DriftDev* __restrict__ drift)
{
    const int st = blockIdx.x * blockDim.x + threadIdx.x;
    int r = 0;
    if (st < acc.HW) {
        r = finalize_cell(st, acc, clear_min, h, v, pb);
        if (clean) {
            if (acc.cnt[st] != 0) {  // only cells with points hold nonzero sums
                acc.wsum[st] = 0.0f;
                acc.ssum[st] = 0.0f;
                for (int q = 0; q < pb.Cb; q++) acc.chsum[(int64_t)q * acc.HW + st] = 0.0f;
            }
            if (zero_cnt[st] != 0) zero_cnt[st] = 0;
            if (zero_clr[st] != 0) zero_clr[st] = 0;
            if (hl && r != 0) {
                int ix, iy;
                logical_index(g, st, ix, iy);
                hl[iy * g.W + ix] = h[st];
            }
        }
    }
    if (clean && blockIdx.x == 0) {
        if (march_counts)
            for (int k = threadIdx.x; k < kSegLists * kSegSubs; k += blockDim.x) march_counts[k] = 0;
        if (drift && threadIdx.x == 0) *drift = DriftDev{0.0, 0.0, 0, 0.0f};
    }
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
                       float* chsum, int Cb, int* march_counts, const float* h, float* hl, DriftDev* drift,
                       LaunchEv ev)
{
    int HW = g.W * g.H;
    unsigned b = blocks_for(HW, 256);
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    hipExtLaunchKernelGGL(k_zero_accum, dim3(b), dim3(256), 0, s, ev.start, ev.stop, 0, g, n, wsum, ssum, clr, chsum,
                          Cb, march_counts, h, hl, drift);
}

void launch_ingest(hipStream_t s, const Grid& g, const float* xyz, int64_t n, const float* ch,
                   const Pose& T, float c0, float c1, float mr2, const PointBinds& pb, int* cnt,
                   float* wsum, float* ssum, float2* stash, float* chsum, const MarchBufs* march,
                   unsigned long long* stats, LaunchEv ev)
{
    if (n <= 0) return;
    const Accum acc{cnt, wsum, ssum, stash, nullptr, chsum, g.W * g.H};
    const size_t lds = pb.lds_ch ? sizeof(float) * kSlots * pb.Cb : 0;
    hipExtLaunchKernelGGL(k_ingest, dim3(blocks_for(n, kChunk)), dim3(kWG), (uint32_t)lds, s, ev.start, ev.stop, 0, g,
                          xyz, n, ch, T, c0, c1, mr2, pb, acc, march ? *march : MarchBufs{}, march ? 1 : 0, stats);
}

void launch_ingest_clouds(hipStream_t s, const Grid& g, const IngestClouds& cl, float c0, float c1, float mr2,
                          unsigned long long* stats, LaunchEv ev)
{
    int64_t nmax = 0;
    for (int k = 0; k < cl.n; k++) nmax = std::max(nmax, cl.c[k].n);
    if (cl.n < 1 || nmax <= 0) return;
    PointBinds pb{};
    hipExtLaunchKernelGGL(k_ingest_clouds, dim3(blocks_for(nmax, kChunk), (unsigned)cl.n), dim3(kWG), 0, s, ev.start,
                          ev.stop, 0, g, cl, c0, c1, mr2, pb, stats);
}

void march_pass(float mr2, float res, int64_t n, int64_t* pts, int64_t* full_per_ray)
{
    // a ray's steps lie below range / res + 2 cells (a margin of 0.1 % for
    // the pose's rotation, orthonormal to 1e-4)
    const double lmax = std::ceil(1.001 * std::sqrt((double)mr2) / (double)res) + 2.0;
    const int64_t fpr = (int64_t)std::min(lmax / kSegLen, 1e15);
    int64_t p = fpr > 0 ? kMarchFullCap / fpr : kMarchPass;
    p = std::max<int64_t>(1, std::min<int64_t>(p, kMarchPass));
    *pts = std::min<int64_t>(n, p);
    *full_per_ray = fpr;
}

MarchSizes march_sizes(int64_t pts, int64_t full_per_ray)
{
    // Sub-list s takes the workgroups b = s mod kSegSubs of a pass, which
    // list 256 points each (k_ray_prep) or kChunk (k_ingest): rays per
    // sub-list at most, for either.
    auto rays = [&](int64_t per_wg) {
        const int64_t wgs = (pts + per_wg - 1) / per_wg;
        return (wgs + kSegSubs - 1) / kSegSubs * per_wg;
    };
    const int64_t per_sub = std::max(rays(256), rays(kChunk));
    MarchSizes z;
    z.part_sub = per_sub;
    z.full_sub = per_sub * std::max<int64_t>(full_per_ray, 1);
    return z;
}

void launch_clear_march(hipStream_t s, const Grid& g_storage, const float* xyz, int64_t n, const Pose& T,
                        float mr2, float margin, const float* hl, int* clr, const MarchBufs& mb,
                        bool prepared, unsigned long long* stats, LaunchEv ev)
{
    // the walks read heights in logical order: the grid without its ring offsets
    const Grid& g = g_storage;
    Grid gl = g_storage;
    gl.rx = 0;
    gl.ry = 0;
    // Clouds beyond the buffers' capacity are marched in passes, each pass
    // clearing the lists' counts first (the first pass's counts were cleared
    // with the accumulators).
    for (int64_t b = 0; b < n; b += mb.cap_pts) {
        const int64_t m = n - b < mb.cap_pts ? n - b : mb.cap_pts;
        if (b > 0) launch_zero_int(s, mb.counts, kSegLists * kSegSubs);
        // the events: start on the pass's first kernel, stop on the last pass's walk
        hipEvent_t e0 = b == 0 ? ev.start : nullptr, e1 = b + m >= n ? ev.stop : nullptr;
        if (!(prepared && b == 0)) {
            hipExtLaunchKernelGGL(k_ray_prep, dim3(blocks_for(m, 256)), dim3(256), 0, s, e0, nullptr, 0, g, xyz + 3 * b,
                                  m, T, mr2, mb, stats);
            e0 = nullptr;
        }
        hipExtLaunchKernelGGL(k_ray_walk, dim3(kWalkGrid), dim3(256), 0, s, e0, e1, 0, g, gl, hl, T, margin, clr, mb,
                              stats);
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

void launch_finalize(hipStream_t s, const Grid& g, int* cnt, float* wsum, float* ssum, const float2* stash,
                     int* clr, int clear_min, float* h, float* v, float* chsum, const PointBinds& pb,
                     unsigned long long* stats, bool clean, int* zero_cnt, int* zero_clr, float* hl,
                     int* march_counts, DriftDev* drift, LaunchEv ev)
{
    const int HW = g.W * g.H;
    const Accum acc{cnt, wsum, ssum, const_cast<float2*>(stash), clr, chsum, HW};
    hipExtLaunchKernelGGL(k_finalize, dim3(blocks_for(HW, 256)), dim3(256), 0, s, ev.start, ev.stop, 0, g, acc,
                          clear_min, h, v, pb, stats, clean ? 1 : 0, zero_cnt, zero_clr, hl, march_counts, drift);
}

void launch_point_cells(hipStream_t s, const Grid& g, const float* xyz, int64_t n, const Pose& T,
                        float mr2, int32_t* out)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_point_cells, dim3(blocks_for(n, 256)), dim3(256), 0, s, g, xyz, n, T, mr2,
                       out);
}

}  // namespace memk
