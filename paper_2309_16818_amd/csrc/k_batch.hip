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
//   k_b_bin       map items: accepted points binned by ingest tile (counting
//                 sort in LDS)
//   k_b_tile_ingest (map, cell block) items: per-cloud sums of the block's
//                 binned points in LDS, written with plain stores (no
//                 zeroing pass, no global atomics)
//   k_b_march     (map, point chunk) items: clearing walks
//   k_b_finalize  every cell (dense): height fusion and clearing
//   k_b_project   (map, tile) items: frustum, pixel, occlusion, pair lists
//   k_b_gather    (map, pair chunk) items: pixel gather and fusion
#include "prof.h"
#include "update.h"

namespace memk {

namespace {

constexpr int kBatchWG = 256;

// Items of a stage with uniform work, dealt to the workgroups in turn:
// workgroup b takes items b, b + grid, ...  (no shared counter: atomics on
// one address serialise).  Every thread of the workgroup calls both;
// next_static starts with a barrier, as next_item does.
__device__ __forceinline__ int first_static(int n)
{
    return (int)blockIdx.x < n ? (int)blockIdx.x : -1;
}
__device__ __forceinline__ int next_static(int it, int n)
{
    __syncthreads();
    const int r = it + (int)gridDim.x;
    return r < n ? r : -1;
}

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

// The per-map prefix of point-chunk items copied into LDS (s_cs, kChunkLds
// ints) when it fits, so that an item's map is found by a search in LDS
// rather than a chain of dependent global loads; else the global table.
// Every thread of the workgroup calls it; it ends with a barrier.
constexpr int kChunkLds = 1088;
__device__ __forceinline__ const int* stage_chunk_start(const BatchDev& d, int* s_cs)
{
    if (d.n_maps + 1 > kChunkLds) return d.chunk_start;
    for (int k = threadIdx.x; k <= d.n_maps; k += blockDim.x) s_cs[k] = d.chunk_start[k];
    __syncthreads();
    return s_cs;
}

// Map of point-chunk item `it` (binary search over the per-map prefix cs)
// and the item's point range.
__device__ __forceinline__ int chunk_item(const BatchDev& d, const int* cs, int it, int64_t& begin, int64_t& end)
{
    int lo = 0, hi = d.n_maps;  // cs[lo] <= it < cs[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cs[mid] <= it) lo = mid;
        else hi = mid;
    }
    const BatchMap& m = d.maps[lo];
    begin = m.pt_begin + (int64_t)(it - cs[lo]) * d.chunk;
    end = begin + d.chunk < m.pt_end ? begin + d.chunk : m.pt_end;
    return lo;
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
    for (int k = i; k < d.n_itiles; k += gridDim.x * blockDim.x) d.tile_cnt[k] = 0;
}

__global__ __launch_bounds__(kBatchWG) void k_b_reset(BatchDev d, BatchLayers ls)
{
    const int n = d.n_items[0];
    for (int r = first_static(n); r >= 0; r = next_static(r, n)) {
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

// Binning of the accepted points by ingest tile (a counting sort over the
// whole batch), in three stages so that every stage runs on uniform items:
//   k_b_bin        (map, chunk) items: each chunk's accepted points counted
//                  per tile in LDS and added to the tile's count with one
//                  atomic per tile the chunk reaches; the points and drops;
//   k_b_bin_scan   map items: the map's tiles' first records (exclusive
//                  prefix of the counts from the map's first point), which
//                  also start the tiles' scatter cursors;
//   k_b_bin_scatter (map, chunk) items: each chunk reserves its points' room
//                  in every tile it reaches with one atomic on the tile's
//                  cursor and writes a 16-byte record per accepted point
//                  (storage cell, z, variance).
// Records of map m fill [pt_begin, pt_begin + accepted) in tile order (the
// order within a tile is the order of the reservations).  A map with more
// tiles than kBinTiles counts and reserves with one global atomic per point.
__device__ __forceinline__ int bin_tile(const BatchMap& m, int itile_h, int ix, int iy)
{
    const int sh = itile_h == 64 ? 6 : 5;
    int sx = ix + m.g.rx;
    sx -= (sx >= m.g.W) ? m.g.W : 0;
    int sy = iy + m.g.ry;
    sy -= (sy >= m.g.H) ? m.g.H : 0;
    return (sy >> sh) * m.itiles_x + (sx >> 6);
}

__device__ __forceinline__ int bin_ntiles(const BatchMap& m, int itile_h)
{
    return m.itiles_x * ((m.g.H + itile_h - 1) / itile_h);
}

__global__ __launch_bounds__(kBatchWG) void k_b_bin(BatchDev d, const float* __restrict__ xyz, float mr2)
{
    __shared__ int s_hist[kBinTiles];
    __shared__ int s_cs[kChunkLds];
    const int* cs = stage_chunk_start(d, s_cs);
    PointCounts pc;
    int points_in = 0;
    const int n = d.n_items[1];
    for (int it = first_static(n); it >= 0; it = next_static(it, n)) {
        int64_t b0, b1;
        const BatchMap& m = d.maps[chunk_item(d, cs, it, b0, b1)];
        const int ntiles = bin_ntiles(m, d.itile_h);
        const bool lds = ntiles <= kBinTiles;
        if (lds)
            for (int k = threadIdx.x; k < ntiles; k += blockDim.x) s_hist[k] = 0;
        __syncthreads();
        // every point of the chunk (at most 2048) loaded before any is binned
        constexpr int U = 8;
        static_assert(U * kBatchWG >= 2048, "a chunk's points fit the workgroup's registers");
        float p3[U][3];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t i = b0 + threadIdx.x + (int64_t)u * blockDim.x;
            const bool in = i < b1;
            p3[u][0] = in ? xyz[3 * i] : 0.0f;
            p3[u][1] = in ? xyz[3 * i + 1] : 0.0f;
            p3[u][2] = in ? xyz[3 * i + 2] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (b0 + threadIdx.x + (int64_t)u * blockDim.x >= b1) continue;
            float px, py, pz, r2;
            int ix, iy;
            const int r = point_cell(m.g, m.T, mr2, p3[u][0], p3[u][1], p3[u][2], px, py, pz, r2, ix, iy);
            points_in++;
            pc.acc += (r == 0);
            pc.nonfinite += (r == -1);
            pc.range += (r == -2);
            pc.outside += (r == -3);
            if (r != 0) continue;
            const int t = bin_tile(m, d.itile_h, ix, iy);
            if (lds)
                atomicAdd(&s_hist[t], 1);
            else
                atomicAdd(&d.tile_cnt[m.itile_base + t], 1);
        }
        __syncthreads();
        if (lds)
            for (int k = threadIdx.x; k < ntiles; k += blockDim.x)
                if (s_hist[k] > 0) atomicAdd(&d.tile_cnt[m.itile_base + k], s_hist[k]);
    }
    const int ids[5] = {ST_ACCEPTED, ST_NONFINITE, ST_RANGE, ST_OUTSIDE, ST_POINTS_IN};
    int vals[5] = {pc.acc, pc.nonfinite, pc.range, pc.outside, points_in};
    block_stats(d.stats, ids, vals);
}

__global__ __launch_bounds__(kBatchWG) void k_b_bin_scan(BatchDev d)
{
    __shared__ int s_wave[kBatchWG / 64];
    __shared__ int s_run;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int it = first_static(d.n_maps); it >= 0; it = next_static(it, d.n_maps)) {
        const BatchMap& m = d.maps[it];
        const int ntiles = bin_ntiles(m, d.itile_h);
        if (t == 0) s_run = 0;
        __syncthreads();
        for (int k0 = 0; k0 < ntiles; k0 += kBatchWG) {
            const int k = k0 + t;
            const int c = k < ntiles ? d.tile_cnt[m.itile_base + k] : 0;
            int incl = c;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int u = __shfl_up(incl, o);
                if (lane >= o) incl += u;
            }
            if (lane == 63) s_wave[w] = incl;
            __syncthreads();
            int pre = s_run + incl - c;
            for (int q = 0; q < w; q++) pre += s_wave[q];
            if (k < ntiles) {
                d.tile_start[m.itile_base + k] = (int)(m.pt_begin + pre);
                d.tile_cur[m.itile_base + k] = (int)(m.pt_begin + pre);
            }
            __syncthreads();
            if (t == kBatchWG - 1) s_run = pre + c;
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(kBatchWG) void k_b_bin_scatter(BatchDev d, const float* __restrict__ xyz, float c0,
                                                            float c1, float mr2)
{
    __shared__ int s_hist[kBinTiles];
    __shared__ int s_cs[kChunkLds];
    const int* cs = stage_chunk_start(d, s_cs);
    const int n = d.n_items[1];
    for (int it = first_static(n); it >= 0; it = next_static(it, n)) {
        int64_t b0, b1;
        const BatchMap& m = d.maps[chunk_item(d, cs, it, b0, b1)];
        const int ntiles = bin_ntiles(m, d.itile_h);
        const bool lds = ntiles <= kBinTiles;
        if (lds)
            for (int k = threadIdx.x; k < ntiles; k += blockDim.x) s_hist[k] = 0;
        __syncthreads();
        // pass 1: each point's rank among the chunk's points in its tile
        constexpr int U = 8;  // points per thread: chunks of at most 2048 points (the tuning's largest)
        static_assert(U * kBatchWG >= 2048, "a chunk's points fit the workgroup's registers");
        int tile[U], rank[U];
        float4 recu[U];
        float p3[U][3];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t i = b0 + threadIdx.x + (int64_t)u * blockDim.x;
            const bool in = i < b1;
            p3[u][0] = in ? xyz[3 * i] : 0.0f;
            p3[u][1] = in ? xyz[3 * i + 1] : 0.0f;
            p3[u][2] = in ? xyz[3 * i + 2] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            tile[u] = -1;
            const int64_t i = b0 + threadIdx.x + (int64_t)u * blockDim.x;
            if (i >= b1) continue;
            float px, py, pz, r2;
            int ix, iy;
            if (point_cell(m.g, m.T, mr2, p3[u][0], p3[u][1], p3[u][2], px, py, pz, r2, ix, iy) != 0)
                continue;
            tile[u] = bin_tile(m, d.itile_h, ix, iy);
            int sx = ix + m.g.rx;
            sx -= (sx >= m.g.W) ? m.g.W : 0;
            int sy = iy + m.g.ry;
            sy -= (sy >= m.g.H) ? m.g.H : 0;
            const float sig = c0 + c1 * r2;
            recu[u] = make_float4(__int_as_float(sx | (sy << 16)), pz, sig * sig, 0.0f);
            rank[u] = lds ? atomicAdd(&s_hist[tile[u]], 1) : 0;
        }
        __syncthreads();
        // the chunk's room in each tile it reaches: one atomic per tile
        if (lds)
            for (int k = threadIdx.x; k < ntiles; k += blockDim.x)
                if (s_hist[k] > 0) s_hist[k] = atomicAdd(&d.tile_cur[m.itile_base + k], s_hist[k]);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (tile[u] < 0) continue;
            const int pos = lds ? s_hist[tile[u]] + rank[u] : atomicAdd(&d.tile_cur[m.itile_base + tile[u]], 1);
            d.rec[pos] = recu[u];
        }
    }
}

// (map, tile) items: the workgroup owns a kIngestTileW x itile_h block of
// its map's storage cells, sums the block's binned points in dense LDS
// arrays (counts, 1/v, z/v and the (z, v) of the first point) and writes
// every cell of the block with plain stores: per-cloud sums, the
// single-point stash and a zero vote count.  No global atomics, and the
// block is written whether or not it received points, so no separate
// zeroing pass is needed.
__global__ __launch_bounds__(kBatchWG) void k_b_tile_ingest(BatchDev d)
{
    extern __shared__ char s_raw[];
    const int TH = d.itile_h, NC = kIngestTileW * TH;
    int* s_cnt = (int*)s_raw;
    float* s_w = (float*)(s_cnt + NC);
    float* s_s = s_w + NC;
    float2* s_first = (float2*)(s_s + NC);
    for (int it = first_static(d.n_itiles); it >= 0; it = next_static(it, d.n_itiles)) {
        const BatchItem I = d.itiles[it];
        const BatchMap& m = d.maps[I.map];
        const int W = m.g.W, x0 = I.a, y0 = I.b;
        for (int k = threadIdx.x; k < NC; k += blockDim.x) {
            s_cnt[k] = 0;
            s_w[k] = 0.0f;
            s_s[k] = 0.0f;
        }
        __syncthreads();
        const int r0 = d.tile_start[it], n = d.tile_cnt[it];
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            const float4 rc = d.rec[r0 + j];
            const int c = __float_as_int(rc.x);
            const int k = ((c >> 16) - y0) * kIngestTileW + (c & 0xffff) - x0;
            const float w = 1.0f / rc.z;
            if (atomicAdd(&s_cnt[k], 1) == 0) s_first[k] = make_float2(rc.y, rc.z);
            atomicAdd(&s_w[k], w);
            atomicAdd(&s_s[k], rc.y * w);
        }
        __syncthreads();
        const int tw = min(kIngestTileW, W - x0), th = min(TH, m.g.H - y0);
        for (int k = threadIdx.x; k < kIngestTileW * th; k += blockDim.x) {
            const int lx = k % kIngestTileW, ly = k / kIngestTileW;
            if (lx >= tw) continue;
            const int64_t st = m.cell_off + (int64_t)(y0 + ly) * W + x0 + lx;
            const int c = s_cnt[k];
            d.cnt[st] = c;
            d.wsum[st] = s_w[k];
            d.ssum[st] = s_s[k];
            d.clr[st] = 0;
            if (c == 1) d.stash[st] = s_first[k];  // a single point sets an empty cell exactly
        }
    }
}

// Every map's heights copied into logical order (index y * W + x within the
// map) for the clearing walks: dense over the arena, each workgroup taking
// ranges of kLogicalRange cells, finding the map of a range's first cell by
// bisection over the maps' first cells and stepping to the next map where a
// thread's cell lies past a boundary.
constexpr int kLogicalRange = 4096;
__global__ __launch_bounds__(256) void k_b_logical(BatchDev d)
{
    __shared__ int s_map;
    for (int64_t c0 = (int64_t)blockIdx.x * kLogicalRange; c0 < d.total_cells;
         c0 += (int64_t)gridDim.x * kLogicalRange) {
        if (threadIdx.x == 0) {
            int lo = 0, hi = d.n_maps;  // maps[lo].cell_off <= c0 < maps[hi].cell_off
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (d.maps[mid].cell_off <= c0) lo = mid;
                else hi = mid;
            }
            s_map = lo;
        }
        __syncthreads();
        int lo = s_map;
        for (int k = 0; k < kLogicalRange; k += 256) {
            const int64_t i = c0 + k + threadIdx.x;
            if (i >= d.total_cells) break;
            while (lo + 1 < d.n_maps && d.maps[lo + 1].cell_off <= i) lo++;
            const BatchMap& m = d.maps[lo];
            int ix, iy;
            logical_index(m.g, (int)(i - m.cell_off), ix, iy);
            d.hl[m.cell_off + (int64_t)iy * m.g.W + ix] = d.h[i];
        }
        __syncthreads();  // s_map is rewritten for the next range
    }
}

__global__ __launch_bounds__(kBatchWG) void k_b_march(BatchDev d, const float* __restrict__ xyz,
                                                      float mr2, float margin)
{
    static_assert(kBatchWG == 256, "one ray per thread of a 256-thread group");
    constexpr int kNB = 10;  // length buckets: none, 1-8, ..., 57-64, longer
    __shared__ int s_item;
    __shared__ int s_off[kNB];
    __shared__ int s_order[256];
    __shared__ int s_steps[256];
    __shared__ float4 s_pt[256];
    __shared__ int2 s_cell[256];
    __shared__ int s_cs[kChunkLds];
    const int* cs = stage_chunk_start(d, s_cs);
    const int t = threadIdx.x;
    int visited = 0, all_steps = 0;
    const int n = d.n_items[1];
    for (int it = next_item(d.qctr, 2, n, &s_item); it >= 0; it = next_item(d.qctr, 2, n, &s_item)) {
        int64_t b0, b1;
        const BatchMap& m = d.maps[chunk_item(d, cs, it, b0, b1)];
        Grid gl = m.g;  // the walks read the logical-order height copy
        gl.rx = 0;
        gl.ry = 0;
        const float sx = m.T.m[3], sy = m.T.m[7], sz = m.T.m[11];
        int ax, ay;
        lattice_cell(m.g, sx, sy, ax, ay);
        for (int64_t base = b0; base < b1; base += 256) {
            const int64_t i = base + t;
            float px = 0.f, py = 0.f, pz = 0.f, r2;
            int ix = 0, iy = 0, steps = 0;
            if (i < b1 &&
                point_cell(m.g, m.T, mr2, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], px, py, pz, r2, ix, iy) == 0)
                steps = max(max(abs(ix - ax), abs(iy - ay)) - 1, 0);
            all_steps += steps;
            s_steps[t] = steps;
            s_pt[t] = make_float4(px, py, pz, 0.f);
            s_cell[t] = make_int2(ix, iy);
            const int src = order_by_length<kNB>(steps, s_off, s_order);
            if (s_steps[src] > 0) {
                const float4 p = s_pt[src];
                const int2 c = s_cell[src];
                Ray ray(gl, ax, ay, c.x, c.y, sx, sy, sz, p.x, p.y, p.z);
                visited += walk_votes<8>(gl, ray, d.hl + m.cell_off, 1, ray.L.steps - 1,
                                         ClearVoteLogical{d.clr + m.cell_off, m.g, margin});
            }
            __syncthreads();  // the next group overwrites the LDS tables
        }
    }
    const int ids[2] = {ST_RAY_CELLS, ST_RAY_STEPS};
    int vals[2] = {visited, all_steps};
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
    int visited = 0, in_view_all = 0, vis_all = 0;
    const int per = tile * tile;
    const int sub = threadIdx.x / per;          // tile within the item group
    const int tx = (threadIdx.x % per) % tile, ty = (threadIdx.x % per) / tile;
    const int group = kBatchWG / per;           // tiles per queue pull
    const int n_groups = (d.n_tiles + group - 1) / group;
    for (int it = first_static(n_groups); it >= 0; it = next_static(it, n_groups)) {
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

template <int IMG, int S, int V>
__global__ __launch_bounds__(kBatchWG) void k_b_gather(BatchDev d, int queue,
                                                       const void* __restrict__ images, int cam_c,
                                                       int cam_w, int ch_first, LayerDev L,
                                                       int lpp_log2, int topk)
{
    const int lane = threadIdx.x & 63;
    const int LPP = 1 << lpp_log2;
    const int sub = lane >> lpp_log2;
    const int q0 = lane & (LPP - 1);
    const int ppw = 64 >> lpp_log2;
    const int wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const int esz = IMG == MEM_U8 ? 1 : 4;
    for (int it = first_static(d.n_gitems); it >= 0; it = next_static(it, d.n_gitems)) {
        const BatchItem I = d.gitems[it];
        const BatchMap& m = d.maps[I.map];
        const int N = d.pair_count[I.map];
        const int end = I.a + kGatherItem < N ? I.a + kGatherItem : N;
        const char* img = (const char*)images + m.img_off * esz;
        const int2* pairs = d.pairs + m.cell_off;
        for (int p = I.a + wave * ppw + sub; p < end; p += nw * ppw) {
            if (topk > 0)  // top-k class input: one lane per pair (lpp_log2 = 0)
                gather_topk<IMG>(pairs[p], img, (int64_t)cam_w * cam_c, cam_c, 1, cam_w, ch_first, L, topk);
            else if constexpr (V > 1)
                gather_pair_vec<IMG, S, V>(pairs[p], img, (int64_t)cam_w * cam_c, cam_c, cam_w, ch_first, L, q0,
                                           LPP);
            else
                gather_pair<IMG, S>(pairs[p], img, (int64_t)cam_w * cam_c, cam_c, 1, cam_w, ch_first, L,
                                    q0, LPP);
        }
    }
}

}  // namespace

// Dynamic LDS of k_b_tile_ingest: per-cell sums of a kIngestTileW x tile_h tile.
static size_t tile_ingest_dyn_lds(int tile_h)
{
    return (size_t)kIngestTileW * tile_h * (sizeof(int) + 2 * sizeof(float) + sizeof(float2));
}

// All LDS of a k_b_tile_ingest workgroup: the kernel's static variables as
// the compiler laid them out plus the dynamic per-cell sums.
size_t batch_tile_ingest_lds_bytes(int tile_h)
{
    static const size_t fixed = [] {
        hipFuncAttributes a{};
        const bool ok = hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_b_tile_ingest)) == hipSuccess;
        (void)hipGetLastError();
        return ok ? (size_t)a.sharedSizeBytes : (size_t)1024;
    }();
    return fixed + tile_ingest_dyn_lds(tile_h);
}

void launch_batch_step(hipStream_t s, const BatchDev& d, const BatchLaunch& bl, const float* xyz,
                       float c0, float c1, float mr2, float margin, int clear_min,
                       const LayerDev* L, int nL, const void* images, int img_dtype, int cam_c,
                       int cam_w, const mem_binding* ib, int n_ib, Profiler* prof)
{
    // every stage bracketed by events while a profiler is given
    auto stage = [&](const char* name, auto&& f) {
        if (prof)
            prof->timed(s, name, f);
        else
            f();
    };
    const int pre = (d.n_maps > kQueues ? d.n_maps : kQueues);
    stage("b_prep", [&] { hipLaunchKernelGGL(k_b_prep, dim3((pre + 255) / 256), dim3(256), 0, s, d); });
    BatchLayers ls;
    ls.n = nL;
    for (int l = 0; l < nL; l++) ls.L[l] = L[l];
    stage("b_reset", [&] { hipLaunchKernelGGL(k_b_reset, dim3(bl.grid), dim3(kBatchWG), 0, s, d, ls); });
    int64_t zb = (d.total_cells + 255) / 256;
    if (zb > 8192) zb = 8192;
    stage("b_bin", [&] { hipLaunchKernelGGL(k_b_bin, dim3(bl.grid), dim3(kBatchWG), 0, s, d, xyz, mr2); });
    stage("b_bin_scan", [&] { hipLaunchKernelGGL(k_b_bin_scan, dim3(bl.grid), dim3(kBatchWG), 0, s, d); });
    stage("b_bin_scatter", [&] {
        hipLaunchKernelGGL(k_b_bin_scatter, dim3(bl.grid), dim3(kBatchWG), 0, s, d, xyz, c0, c1, mr2);
    });
    stage("b_tile_ingest", [&] {
        hipLaunchKernelGGL(k_b_tile_ingest, dim3(bl.grid), dim3(kBatchWG), tile_ingest_dyn_lds(d.itile_h), s, d);
    });
    if (clear_min > 0) {
        int64_t lb = (d.total_cells + kLogicalRange - 1) / kLogicalRange;
        if (lb > 4096) lb = 4096;
        stage("b_logical", [&] { hipLaunchKernelGGL(k_b_logical, dim3((unsigned)lb), dim3(256), 0, s, d); });
        stage("b_march", [&] {
            hipLaunchKernelGGL(k_b_march, dim3(bl.grid), dim3(kBatchWG), 0, s, d, xyz, mr2, margin);
        });
    }
    stage("b_finalize", [&] {
        hipLaunchKernelGGL(k_b_finalize, dim3((unsigned)zb), dim3(256), 0, s, d, clear_min);
    });
    if (!images) return;
    stage("b_project", [&] { hipLaunchKernelGGL(k_b_project, dim3(bl.grid), dim3(kBatchWG), 0, s, d, bl.tile); });
    for (int b = 0; b < n_ib; b++) {
        const LayerDev& Lb = L[ib[b].layer - MEM_LAYER_USER0];
        // every map's image starts at a multiple of cam_c channels, so the
        // first map's alignment holds for all
        const int V = ib[b].topk ? 1
                                 : gather_vec_width(Lb.storage, Lb.C, img_dtype, images, (int64_t)cam_w * cam_c,
                                                    cam_c, 1, ib[b].ch_first, Lb);
        const int lpp_log2 = gather_lanes_log2(Lb.C, V, ib[b].topk != 0);
        // one gather pass per binding, each with its own queue (4 + b)
#define MEM_BG(IMG, S, VV)                                                                            \
    hipLaunchKernelGGL((k_b_gather<IMG, S, VV>), dim3(bl.grid), dim3(kBatchWG), 0, s, d, 4 + b, images, \
                       cam_c, cam_w, ib[b].ch_first, Lb, lpp_log2, ib[b].topk)
#define MEM_BG2(IMG, S, VV) \
    do {                    \
        if (V > 1)          \
            MEM_BG(IMG, S, VV); \
        else                \
            MEM_BG(IMG, S, 1);  \
    } while (0)
        stage("b_gather", [&] {
            if (img_dtype == MEM_U8) {
                if (Lb.storage == MEM_BF16) MEM_BG2(MEM_U8, MEM_BF16, 8);
                else if (Lb.storage == MEM_FP8_E4M3) MEM_BG2(MEM_U8, MEM_FP8_E4M3, 8);
                else MEM_BG2(MEM_U8, MEM_F32, 4);
            } else {
                if (Lb.storage == MEM_BF16) MEM_BG2(MEM_F32, MEM_BF16, 8);
                else if (Lb.storage == MEM_FP8_E4M3) MEM_BG2(MEM_F32, MEM_FP8_E4M3, 8);
                else MEM_BG2(MEM_F32, MEM_F32, 4);
            }
        });
#undef MEM_BG2
#undef MEM_BG
    }
}

}  // namespace memk
