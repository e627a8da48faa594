// k_batch.hip - one step of a batch of independent maps.
//
// Every stage is a persistent kernel: a fixed grid of workgroups pulls work
// items from a device counter (work stealing), so maps of very different
// sizes and point counts share the GPU without a launch per map.  Each item
// runs the same per-item body as the single-map kernels (update.h) on its
// map's slice of the concatenated arrays.
//
//   k_b_prep      zero the work-queue counters and per-map pair counts
//   k_b_reset     cells entering each map's grid (robot motion)
//   k_b_zero      per-cloud accumulators of every cell (dense)
//   k_b_ingest    (map, point chunk) items: LDS-binned aggregation
//   k_b_march     (map, point chunk) items: clearing walks
//   k_b_finalize  every cell (dense): height fusion and clearing
//   k_b_project   (map, tile) items: frustum, pixel, occlusion, pair lists
//   k_b_gather    (map, pair chunk) items: pixel gather and fusion
#include "update.h"

namespace memk {

namespace {

constexpr int kBatchWG = 256;

// Pulls the next item of queue q for the whole workgroup (-1: none left).
__device__ __forceinline__ int next_item(int* qctr, int q, int n, int* s_item)
{
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        int it = atomicAdd(&qctr[q], 1);
        *s_item = it < n ? it : -1;
    }
    __syncthreads();
    return *s_item;
}

// Map of point-chunk item `it` (binary search over the per-map prefix) and
// the item's point range.
__device__ __forceinline__ int chunk_item(const BatchDev& d, int it, int64_t& begin, int64_t& end)
{
    int lo = 0, hi = d.n_maps;  // chunk_start[lo] <= it < chunk_start[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (d.chunk_start[mid] <= it) lo = mid;
        else hi = mid;
    }
    const BatchMap& m = d.maps[lo];
    begin = m.pt_begin + (int64_t)(it - d.chunk_start[lo]) * d.chunk;
    end = begin + d.chunk < m.pt_end ? begin + d.chunk : m.pt_end;
    return lo;
}

__device__ __forceinline__ Accum map_accum(const BatchDev& d, const BatchMap& m)
{
    const int64_t o = m.cell_off;
    return Accum{d.cnt + o, d.wsum + o, d.ssum + o, d.stash + o, d.clr + o, nullptr, m.g.W * m.g.H};
}

struct BatchLayers {
    LayerDev L[32];
    int n;
};

__global__ void k_b_prep(BatchDev d)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kQueues) d.qctr[i] = 0;
    if (i < d.n_maps) d.pair_count[i] = 0;
}

__global__ __launch_bounds__(kBatchWG) void k_b_reset(BatchDev d, BatchLayers ls)
{
    __shared__ int s_item;
    const int n = d.n_items[0];
    for (int r = next_item(d.qctr, 0, n, &s_item); r >= 0; r = next_item(d.qctr, 0, n, &s_item)) {
        const BatchRect R = d.rects[r];
        const BatchMap& m = d.maps[R.map];
        const int w = R.x1 - R.x0;
        const int total = w * (R.y1 - R.y0);
        for (int k = threadIdx.x; k < total; k += blockDim.x) {
            // the concatenated arrays are indexed by the global cell index
            const int st = (int)m.cell_off + storage_index(m.g, R.x0 + k % w, R.y0 + k / w);
            reset_cell(st, d.h, d.v, d.cnt, d.clr, ls.L, ls.n);
        }
    }
}

__global__ __launch_bounds__(256) void k_b_zero(BatchDev d)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d.total_cells;
         i += (int64_t)gridDim.x * blockDim.x) {
        d.cnt[i] = 0;
        d.wsum[i] = 0.0f;
        d.ssum[i] = 0.0f;
        d.clr[i] = 0;
    }
}

__global__ __launch_bounds__(kBatchWG) void k_b_ingest(BatchDev d, const float* __restrict__ xyz,
                                                       float c0, float c1, float mr2,
                                                       int slots_log2)
{
    extern __shared__ char s_raw[];
    const int slots = 1 << slots_log2;
    const IngestLds lds{(int*)s_raw, (int*)s_raw + slots, (float*)s_raw + 2 * slots,
                        (float*)s_raw + 3 * slots, (float2*)((float*)s_raw + 4 * slots), nullptr,
                        slots_log2};
    __shared__ int s_item;
    PointBinds pb{};
    PointCounts pc;
    const int n = d.n_items[1];
    for (int it = next_item(d.qctr, 1, n, &s_item); it >= 0; it = next_item(d.qctr, 1, n, &s_item)) {
        int64_t b0, b1;
        const BatchMap& m = d.maps[chunk_item(d, it, b0, b1)];
        ingest_range(m.g, xyz, b0, b1, nullptr, m.T, c0, c1, mr2, pb, map_accum(d, m), lds, pc);
    }
    const int ids[5] = {ST_ACCEPTED, ST_NONFINITE, ST_RANGE, ST_OUTSIDE, ST_POINTS_IN};
    int vals[5] = {pc.acc, pc.nonfinite, pc.range, pc.outside,
                   pc.acc + pc.nonfinite + pc.range + pc.outside};
    block_stats(d.stats, ids, vals);
}

__global__ __launch_bounds__(kBatchWG) void k_b_march(BatchDev d, const float* __restrict__ xyz,
                                                      float mr2, float margin)
{
    __shared__ int s_item;
    int visited = 0;
    const int n = d.n_items[1];
    for (int it = next_item(d.qctr, 2, n, &s_item); it >= 0; it = next_item(d.qctr, 2, n, &s_item)) {
        int64_t b0, b1;
        const BatchMap& m = d.maps[chunk_item(d, it, b0, b1)];
        for (int64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x)
            visited += march_point(m.g, xyz, i, m.T, mr2, margin, d.h + m.cell_off, d.clr + m.cell_off);
    }
    const int ids[2] = {ST_RAY_CELLS, ST_RAY_STEPS};  // every cell of a ray is loaded here
    int vals[2] = {visited, visited};
    block_stats(d.stats, ids, vals);
}

__global__ __launch_bounds__(256) void k_b_finalize(BatchDev d, int clear_min)
{
    // The concatenated arrays are one big storage array: no map needed.
    const Accum acc{d.cnt, d.wsum, d.ssum, d.stash, d.clr, nullptr, 0};
    const PointBinds pb{};
    int touched = 0, cleared = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d.total_cells;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int r = finalize_cell((int)i, acc, clear_min, d.h, d.v, pb);
        touched += r == 1;
        cleared += r == 2;
    }
    const int ids[2] = {ST_TOUCHED, ST_CLEARED};
    int vals[2] = {touched, cleared};
    block_stats(d.stats, ids, vals);
}

// tile side T: the workgroup covers (256 / T^2) tiles per item step.
__global__ __launch_bounds__(kBatchWG) void k_b_project(BatchDev d, int tile)
{
    __shared__ int s_item;
    int visited = 0, in_view_all = 0, vis_all = 0;
    const int per = tile * tile;
    const int sub = threadIdx.x / per;          // tile within the item group
    const int tx = (threadIdx.x % per) % tile, ty = (threadIdx.x % per) / tile;
    const int group = kBatchWG / per;           // tiles per queue pull
    const int n_groups = (d.n_tiles + group - 1) / group;
    for (int it = next_item(d.qctr, 3, n_groups, &s_item); it >= 0;
         it = next_item(d.qctr, 3, n_groups, &s_item)) {
        const int t = it * group + sub;
        int code[kMaxImages];
#pragma unroll
        for (int k = 0; k < kMaxImages; k++) code[k] = -1;
        int st = 0, map = 0, in_view = 0;
        if (t < d.n_tiles) {
            const BatchItem I = d.tiles[t];
            map = I.map;
            const BatchMap& m = d.maps[map];
            const int ix = I.a + tx, iy = I.b + ty;
            if (m.cam.n > 0 && ix < m.g.W && iy < m.g.H) {
                st = storage_index(m.g, ix, iy);
                visited += project_cell(m.g, m.cam, d.h + m.cell_off, ix, iy, st, code, in_view);
            }
        }
        in_view_all += in_view;
        const bool vis = code[0] >= 0;
        vis_all += vis;
        // A wave covers one tile (tile 8: 64 lanes; tile 16: four rows), so
        // its visible lanes share one map.  Pairs hold global cell indices.
        const int64_t off = d.maps[map].cell_off;
        append_pair(vis, (int)off + st, code[0], d.pairs + off, &d.pair_count[map]);
    }
    const int ids[4] = {ST_IN_VIEW, ST_VISIBLE, ST_OCCL_CELLS, ST_OCCL_STEPS};
    int vals[4] = {in_view_all, vis_all, visited, visited};
    block_stats(d.stats, ids, vals);
}

template <int IMG, int S>
__global__ __launch_bounds__(kBatchWG) void k_b_gather(BatchDev d, int queue,
                                                       const void* __restrict__ images, int cam_c,
                                                       int cam_w, int ch_first, LayerDev L,
                                                       int lpp_log2)
{
    __shared__ int s_item;
    const int lane = threadIdx.x & 63;
    const int LPP = 1 << lpp_log2;
    const int sub = lane >> lpp_log2;
    const int q0 = lane & (LPP - 1);
    const int ppw = 64 >> lpp_log2;
    const int wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const int esz = IMG == MEM_U8 ? 1 : 4;
    for (int it = next_item(d.qctr, queue, d.n_gitems, &s_item); it >= 0;
         it = next_item(d.qctr, queue, d.n_gitems, &s_item)) {
        const BatchItem I = d.gitems[it];
        const BatchMap& m = d.maps[I.map];
        const int N = d.pair_count[I.map];
        const int end = I.a + kGatherItem < N ? I.a + kGatherItem : N;
        const char* img = (const char*)images + m.img_off * esz;
        const int2* pairs = d.pairs + m.cell_off;
        for (int p = I.a + wave * ppw + sub; p < end; p += nw * ppw)
            gather_pair<IMG, S>(pairs[p], img, (int64_t)cam_w * cam_c, cam_c, 1, cam_w, ch_first, L,
                                q0, LPP);
    }
}

}  // namespace

size_t batch_ingest_lds_bytes(int chunk)
{
    return (size_t)2 * chunk * (4 + 4 + 4 + 4 + 8);
}

void launch_batch_step(hipStream_t s, const BatchDev& d, const BatchLaunch& bl, const float* xyz,
                       float c0, float c1, float mr2, float margin, int clear_min,
                       const LayerDev* L, int nL, const void* images, int img_dtype, int cam_c,
                       int cam_w, const mem_binding* ib, int n_ib)
{
    const int pre = (d.n_maps > kQueues ? d.n_maps : kQueues);
    hipLaunchKernelGGL(k_b_prep, dim3((pre + 255) / 256), dim3(256), 0, s, d);
    BatchLayers ls;
    ls.n = nL;
    for (int l = 0; l < nL; l++) ls.L[l] = L[l];
    hipLaunchKernelGGL(k_b_reset, dim3(bl.grid), dim3(kBatchWG), 0, s, d, ls);
    int64_t zb = (d.total_cells + 255) / 256;
    if (zb > 8192) zb = 8192;
    hipLaunchKernelGGL(k_b_zero, dim3((unsigned)zb), dim3(256), 0, s, d);
    int slots_log2 = 0;
    while ((1 << slots_log2) < 2 * bl.chunk) slots_log2++;
    hipLaunchKernelGGL(k_b_ingest, dim3(bl.grid), dim3(kBatchWG), batch_ingest_lds_bytes(bl.chunk), s,
                       d, xyz, c0, c1, mr2, slots_log2);
    if (clear_min > 0)
        hipLaunchKernelGGL(k_b_march, dim3(bl.grid), dim3(kBatchWG), 0, s, d, xyz, mr2, margin);
    hipLaunchKernelGGL(k_b_finalize, dim3((unsigned)zb), dim3(256), 0, s, d, clear_min);
    if (!images) return;
    hipLaunchKernelGGL(k_b_project, dim3(bl.grid), dim3(kBatchWG), 0, s, d, bl.tile);
    for (int b = 0; b < n_ib; b++) {
        const LayerDev& Lb = L[ib[b].layer - MEM_LAYER_USER0];
        int lpp_log2 = 0;
        while ((1 << lpp_log2) < Lb.C && lpp_log2 < 6) lpp_log2++;
        // one gather pass per binding, each with its own queue (4 + b)
#define MEM_BG(IMG, S)                                                                            \
    hipLaunchKernelGGL((k_b_gather<IMG, S>), dim3(bl.grid), dim3(kBatchWG), 0, s, d, 4 + b, images, \
                       cam_c, cam_w, ib[b].ch_first, Lb, lpp_log2)
        if (img_dtype == MEM_U8) {
            if (Lb.storage == MEM_BF16) MEM_BG(MEM_U8, MEM_BF16);
            else if (Lb.storage == MEM_FP8_E4M3) MEM_BG(MEM_U8, MEM_FP8_E4M3);
            else MEM_BG(MEM_U8, MEM_F32);
        } else {
            if (Lb.storage == MEM_BF16) MEM_BG(MEM_F32, MEM_BF16);
            else if (Lb.storage == MEM_FP8_E4M3) MEM_BG(MEM_F32, MEM_FP8_E4M3);
            else MEM_BG(MEM_F32, MEM_F32);
        }
#undef MEM_BG
    }
}

}  // namespace memk
