// k_image.hip - image path of the map update (Sec. III-B, Fig. 3), one map.
//
//   k_view         one lane per cell (16x16 cell tiles): frustum test and
//                  pin-hole pixel of every image of one camera pose; cells
//                  inside any view are compacted into a list with one
//                  wave-aggregated append.
//   k_occlude      kOccLanes lanes per listed cell split its Bresenham
//                  occlusion line; runs of cells that the block maxima of the
//                  heights rule out are skipped without loading them, the
//                  others are tested cell by cell; an occluded cell's pixel
//                  codes are overwritten with -1 in place (no atomics).
//   k_gather_fuse  grid-stride over the listed cells; for those visible in
//                  the image a group of lanes (a power of two >= the layer's
//                  channels / V, at most 64) reads the pixel's channels and
//                  read-modify-writes the cell's channel-contiguous layer row
//                  with the layer's rule, V channels per lane (4 FP32, 8 BF16
//                  or FP8 where rows and pixels are aligned for it, else 1);
//                  a top-k class input takes one lane per cell, which adds
//                  each listed probability to its class.
//   k_gather_multi k_gather_fuse of several images (of one or more poses)
//                  into different layers in one launch, each image on its own
//                  range of workgroups.
#include <algorithm>
#include <utility>

#include "update.h"

namespace memk {

namespace {

constexpr int kTile = 16;

// Pass 1 of the two-pass projection: frustum test and pixel of every image
// per cell; cells inside at least one view are appended to vlist
// (st, ix | iy << 16, intermediate cells of the occlusion line, the cell's
// height as bits; sides are at most 16384 cells) and their codes to
// vcode[k * cap + position].
__global__ __launch_bounds__(256) void k_view(Grid g, CameraSet cs, const float* __restrict__ h,
                                              int4* __restrict__ vlist, int* __restrict__ vcode, int cap,
                                              int* __restrict__ vcount, int* __restrict__ vcount_next,
                                              int32_t* __restrict__ dbg,
                                              unsigned long long* __restrict__ stats)
{
    // one pose per grid layer z: its list, codes and counter
    const int pose = blockIdx.z;
    const Camera& cam = cs.c[pose];
    vlist += (int64_t)pose * cap;
    vcode += (int64_t)pose * kMaxImages * cap;
    vcount += pose;
    // the next projection's counter (this one's was cleared by the last)
    if (vcount_next && blockIdx.x == 0 && blockIdx.y == 0 && pose == 0 && threadIdx.x == 0 && threadIdx.y == 0)
        *vcount_next = 0;
    const int ix = blockIdx.x * kTile + threadIdx.x;
    const int iy = blockIdx.y * kTile + threadIdx.y;
    int code[kMaxImages];
#pragma unroll
    for (int k = 0; k < kMaxImages; k++) code[k] = -1;
    int st = 0, in_view = 0, steps = 0;
    if (ix < g.W && iy < g.H) {
        st = storage_index(g, ix, iy);
        in_view = view_cell(g, cam, h, ix, iy, st, code);
        if (in_view) {
            int ax, ay;
            lattice_cell(g, cam.T.m[3], cam.T.m[7], ax, ay);
            steps = max(abs(ix - ax), abs(iy - ay)) - 1;
        }
    }
    // one global atomic per workgroup: lanes rank within the wave, waves
    // within the workgroup (LDS), the workgroup within the list
    __shared__ int s_cnt, s_base;
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    if (tid == 0) s_cnt = 0;
    __syncthreads();
    const bool any = in_view > 0;
    const unsigned long long mask = __ballot(any);
    const int lane = __lane_id();
    int woff = 0;
    if (lane == 0 && mask) woff = atomicAdd(&s_cnt, __popcll(mask));
    woff = __shfl(woff, 0);
    __syncthreads();
    if (tid == 0) s_base = s_cnt ? atomicAdd(vcount, s_cnt) : 0;
    __syncthreads();
    if (any) {
        const int pos = s_base + woff + __popcll(mask & ((1ull << lane) - 1ull));
        vlist[pos] = make_int4(st, ix | (iy << 16), steps > 0 ? steps : 0, __float_as_int(h[st]));
#pragma unroll
        for (int k = 0; k < kMaxImages; k++)
            if (k < cam.n) vcode[(int64_t)k * cap + pos] = code[k];
    }
    if (dbg && ix < g.W && iy < g.H && !any) dbg[iy * g.W + ix] = code[0];
    const int ids[1] = {ST_IN_VIEW};
    int vals[1] = {in_view};
    block_stats(stats, ids, vals);
}

// Pass 2: kOccLanes lanes per in-view cell split its occlusion line into
// equal runs of cells; the cell is visible iff no lane finds an occluder.
// The first lane of the group overwrites the cell's pixel codes with -1
// when one does (8 lanes: of 4, 8, 16 and 32, 8 measured fastest with the
// cell height carried in the list entry).
constexpr int kOccLanes = 8;
static_assert(kOccLanes < 64 && 64 % kOccLanes == 0, "groups of lanes within one wave (mask of kOccLanes bits)");

__global__ __launch_bounds__(256) void k_occlude(Grid g, CameraSet cs, const float* __restrict__ h, TileMax tm,
                                                 const int4* __restrict__ vlist,
                                                 int* __restrict__ vcode, int cap,
                                                 const int* __restrict__ vcount,
                                                 int32_t* __restrict__ dbg,
                                                 unsigned long long* __restrict__ stats)
{
    // one pose per grid row y
    const int pose = blockIdx.y;
    const Camera& cam = cs.c[pose];
    vlist += (int64_t)pose * cap;
    vcode += (int64_t)pose * kMaxImages * cap;
    const int N = vcount[pose];
    const int lane = __lane_id();
    const int sub = lane % kOccLanes;        // lane within the cell's group
    const int grp = lane / kOccLanes;        // group within the wave
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int per_wave = 64 / kOccLanes;
    const float* T = cam.T.m;
    int visited = 0, n_vis = 0, steps = 0;
    for (int64_t base = wave * per_wave; base < N; base += nwaves * per_wave) {
        const int64_t pos = base + grp;
        bool occ = false;
        int4 e = make_int4(0, 0, 0, 0);
        if (pos < N) {
            e = vlist[pos];
            const int total = e.z;  // intermediate cells of the line
            const int run = (total + kOccLanes - 1) / kOccLanes;
            const int first = 1 + sub * run;
            const int cnt = min(run, total - sub * run);
            if (cnt > 0) {
                const int ix = e.y & 0xffff, iy = e.y >> 16;
                const float hj = __int_as_float(e.w);
                const float xc = ((float)(g.ox + ix) + 0.5f) * g.res;
                const float yc = ((float)(g.oy + iy) + 0.5f) * g.res;
                int ax, ay;
                lattice_cell(g, T[3], T[7], ax, ay);
                const Ray ray(g, ax, ay, ix, iy, T[3], T[7], T[11], xc, yc, hj);
                steps += cnt;
                visited += walk_range_skip(
                    g, ray, h, tm, first, cnt, [&](float hm, float z0, float z1) { return hm < fminf(z0, z1); },
                    [&](int, float hk, float zr) {
                        if (hk >= zr) occ = true;  // NaN (no height) never occludes
                        return occ;
                    });
            }
        }
        const unsigned long long om = __ballot(occ);
        const bool occluded = ((om >> (grp * kOccLanes)) & ((1ull << kOccLanes) - 1ull)) != 0;
        const bool lead = sub == 0 && pos < N;
        if (lead) {
            const int c0 = vcode[pos];
#pragma unroll
            for (int k = 0; k < kMaxImages; k++) {
                if (k >= cam.n) break;
                const int64_t q = (int64_t)k * cap + pos;
                const int code = k == 0 ? c0 : vcode[q];
                if (code < 0) continue;
                if (occluded)
                    vcode[q] = -1;
                else
                    n_vis++;
            }
            if (dbg) dbg[(e.y >> 16) * g.W + (e.y & 0xffff)] = (c0 >= 0 && occluded) ? -3 : c0;
        }
    }
    const int ids[3] = {ST_VISIBLE, ST_OCCL_CELLS, ST_OCCL_STEPS};
    int vals[3] = {n_vis, visited, steps};
    block_stats(stats, ids, vals);
}

// The gather of one job on workgroups blk = 0 .. nblk - 1 (grid-stride over
// the listed cells, one entry per lane group at a time; its cell is read
// with its code).
template <int IMG, int S, int V>
__device__ __forceinline__ void gather_blocks(const int4* __restrict__ vlist, const int* __restrict__ vcode,
                                              const int* __restrict__ count, const void* __restrict__ img,
                                              int64_t s0, int64_t s1, int64_t s2, int w, int ch_first,
                                              const LayerDev& L, int lpp_log2, int topk, int64_t blk,
                                              int64_t nblk)
{
    const int N = *count;
    const int lane = threadIdx.x & 63;
    const int LPP = 1 << lpp_log2;
    const int sub = lane >> lpp_log2;
    const int q0 = lane & (LPP - 1);
    const int ppw = 64 >> lpp_log2;
    const int64_t wave = (blk * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = (nblk * blockDim.x) >> 6;
    for (int64_t pbase = wave * ppw; pbase < N; pbase += nwaves * ppw) {
        const int64_t p = pbase + sub;
        const bool in = p < N;
        const int code = in ? vcode[p] : -1;
        const int st = in ? vlist[p].x : 0;
        if (code < 0) continue;
        if (topk > 0)  // one lane per pair (lpp_log2 = 0)
            gather_topk<IMG>(make_int2(st, code), img, s0, s1, s2, w, ch_first, L, topk);
        else if constexpr (V > 1)
            gather_pair_vec<IMG, S, V>(make_int2(st, code), img, s0, s1, w, ch_first, L, q0, LPP);
        else
            gather_pair<IMG, S>(make_int2(st, code), img, s0, s1, s2, w, ch_first, L, q0, LPP);
    }
}

template <int IMG, int S, int V>
__global__ __launch_bounds__(256) void k_gather_fuse(const int4* __restrict__ vlist,
                                                     const int* __restrict__ vcode,
                                                     const int* __restrict__ count,
                                                     const void* __restrict__ img, int64_t s0,
                                                     int64_t s1, int64_t s2, int w, int ch_first,
                                                     LayerDev L, int lpp_log2, int topk)
{
    gather_blocks<IMG, S, V>(vlist, vcode, count, img, s0, s1, s2, w, ch_first, L, lpp_log2, topk, blockIdx.x,
                             gridDim.x);
}

// Variants of a gather job: image type (u8, f32) x storage (FP32, BF16, FP8)
// x channels per lane (the storage's vector width, or one; top-k inputs take
// one).
constexpr int kind_of(int img_dtype, int storage, bool vec)
{
    return (img_dtype == MEM_U8 ? 0 : 6) + (storage == MEM_F32 ? 0 : storage == MEM_BF16 ? 2 : 4) + (vec ? 0 : 1);
}

template <int IMG, int S, int V>
__device__ __forceinline__ void run_job(const GatherJob& J, int64_t blk)
{
    gather_blocks<IMG, S, V>(J.vlist, J.vcode, J.count, J.img, J.s0, J.s1, J.s2, J.w, J.ch_first, J.L, J.lpp_log2,
                             J.topk, blk, J.blocks);
}

// Bit of storage type S in the set of storage types a fused launch holds.
constexpr int storage_bit(int storage)
{
    return storage == MEM_F32 ? 1 : storage == MEM_BF16 ? 2 : 4;
}

// Several jobs in one launch: workgroup b runs the job whose range of
// workgroups holds b.  Jobs write different layers, so the order in which
// their workgroups run does not matter.  SM is the set of the jobs' storage
// types (storage_bit), so that a launch carries the registers of those
// variants only.
template <int SM>
__global__ __launch_bounds__(256) void k_gather_multi(GatherJobs js)
{
    int j = 0;
    for (int k = 1; k < js.n; k++)
        if ((int)blockIdx.x >= js.j[k].block0) j = k;
    const GatherJob& J = js.j[j];
    const int64_t blk = (int64_t)blockIdx.x - J.block0;
#define MEM_JOB(IMG, S, V)                                                                  \
    case kind_of(IMG, S, V > 1):                                                            \
        if constexpr ((SM & storage_bit(S)) != 0) run_job<IMG, S, V>(J, blk);               \
        break;
    switch (J.kind) {
        MEM_JOB(MEM_U8, MEM_F32, 4)
        MEM_JOB(MEM_U8, MEM_F32, 1)
        MEM_JOB(MEM_U8, MEM_BF16, 8)
        MEM_JOB(MEM_U8, MEM_BF16, 1)
        MEM_JOB(MEM_U8, MEM_FP8_E4M3, 8)
        MEM_JOB(MEM_U8, MEM_FP8_E4M3, 1)
        MEM_JOB(MEM_F32, MEM_F32, 4)
        MEM_JOB(MEM_F32, MEM_F32, 1)
        MEM_JOB(MEM_F32, MEM_BF16, 8)
        MEM_JOB(MEM_F32, MEM_BF16, 1)
        MEM_JOB(MEM_F32, MEM_FP8_E4M3, 8)
        MEM_JOB(MEM_F32, MEM_FP8_E4M3, 1)
    default:
        break;
    }
#undef MEM_JOB
}

__global__ void k_zero_int(int* p, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

}  // namespace

void launch_zero_int(hipStream_t s, int* p, int n)
{
    hipLaunchKernelGGL(k_zero_int, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
}

void launch_project(hipStream_t s, const Grid& g, const CameraSet& cs, const float* h, const TileMax& tm, int cap,
                    int* vcount, int* vcount_next, int4* vlist, int* vcode, int32_t* dbg,
                    unsigned long long* stats, LaunchEv ev)
{
    dim3 grid((g.W + kTile - 1) / kTile, (g.H + kTile - 1) / kTile, (unsigned)cs.n);
    int32_t* d = cs.n == 1 ? dbg : nullptr;
    hipExtLaunchKernelGGL(k_view, grid, dim3(kTile, kTile), 0, s, ev.start, nullptr, 0, g, cs, h, vlist, vcode, cap,
                          vcount, vcount_next, d, stats);
    int64_t blocks = ((int64_t)cap * kOccLanes + 255) / 256;
    if (blocks > 1024) blocks = 1024;  // per pose; 256..4096 measured, 1024 fastest
    if (blocks < 1) blocks = 1;
    hipExtLaunchKernelGGL(k_occlude, dim3((unsigned)blocks, (unsigned)cs.n), dim3(256), 0, s, nullptr, ev.stop, 0, g,
                          cs, h, tm, vlist, vcode, cap, vcount, d, stats);
}

GatherJob gather_job(const int4* vlist, const int* vcode, const int* count, int max_pairs, const void* img,
                     int img_dtype, int64_t s0, int64_t s1, int64_t s2, int w, int ch_first, const LayerDev& L,
                     int topk, bool one_channel)
{
    GatherJob J{};
    J.vlist = vlist;
    J.vcode = vcode;
    J.count = count;
    J.img = img;
    J.s0 = s0;
    J.s1 = s1;
    J.s2 = s2;
    J.L = L;
    J.w = w;
    J.ch_first = ch_first;
    J.topk = topk;
    const int V = topk || one_channel ? 1 : gather_vec_width(L.storage, L.C, img_dtype, img, s0, s1, s2, ch_first, L);
    J.kind = kind_of(img_dtype, L.storage, V > 1);
    const int lpp_log2 = gather_lanes_log2(L.C, V, topk != 0);
    J.lpp_log2 = lpp_log2;
    const int ppw = 64 >> lpp_log2;
    const int64_t waves = ((int64_t)max_pairs + ppw - 1) / ppw;
    int64_t blocks = (waves + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    J.blocks = (int)blocks;
    J.block0 = 0;
    return J;
}

void launch_gather_multi(hipStream_t s, GatherJobs& js, LaunchEv ev)
{
    // the jobs with the most lanes per pair (the longest rows) first, and at
    // most 1024 workgroups each (512-4096 and the call order measured slower)
    for (int a = 1; a < js.n; a++)
        for (int b = a; b > 0 && js.j[b].lpp_log2 > js.j[b - 1].lpp_log2; b--) std::swap(js.j[b], js.j[b - 1]);
    int total = 0;
    for (int k = 0; k < js.n; k++) {
        js.j[k].blocks = std::min(js.j[k].blocks, 1024);
        js.j[k].block0 = total;
        total += js.j[k].blocks;
    }
    int sm = 0;
    for (int k = 0; k < js.n; k++) sm |= storage_bit(js.j[k].L.storage);
    const dim3 gr((unsigned)total), bl(256);
    switch (sm) {
    case 1: hipExtLaunchKernelGGL(k_gather_multi<1>, gr, bl, 0, s, ev.start, ev.stop, 0, js); break;
    case 2: hipExtLaunchKernelGGL(k_gather_multi<2>, gr, bl, 0, s, ev.start, ev.stop, 0, js); break;
    case 3: hipExtLaunchKernelGGL(k_gather_multi<3>, gr, bl, 0, s, ev.start, ev.stop, 0, js); break;
    case 4: hipExtLaunchKernelGGL(k_gather_multi<4>, gr, bl, 0, s, ev.start, ev.stop, 0, js); break;
    case 5: hipExtLaunchKernelGGL(k_gather_multi<5>, gr, bl, 0, s, ev.start, ev.stop, 0, js); break;
    case 6: hipExtLaunchKernelGGL(k_gather_multi<6>, gr, bl, 0, s, ev.start, ev.stop, 0, js); break;
    default: hipExtLaunchKernelGGL(k_gather_multi<7>, gr, bl, 0, s, ev.start, ev.stop, 0, js); break;
    }
}

void launch_gather_fuse(hipStream_t s, const int4* vlist, const int* vcode, const int* count, int max_pairs,
                        const void* img, int img_dtype, int64_t s0, int64_t s1, int64_t s2, int w,
                        int ch_first, const LayerDev& L, int topk, bool one_channel, LaunchEv ev)
{
    const GatherJob J =
        gather_job(vlist, vcode, count, max_pairs, img, img_dtype, s0, s1, s2, w, ch_first, L, topk, one_channel);
    const bool vec = J.kind % 2 == 0;
    dim3 gr((unsigned)J.blocks), bl(256);
#define MEM_GF(IMG, S, V) \
    hipExtLaunchKernelGGL((k_gather_fuse<IMG, S, V>), gr, bl, 0, s, ev.start, ev.stop, 0, vlist, vcode, count, img, \
                          s0, s1, s2, w, ch_first, L, J.lpp_log2, topk)
#define MEM_GF2(IMG, S, VV) \
    do {                    \
        if (vec)            \
            MEM_GF(IMG, S, VV); \
        else                \
            MEM_GF(IMG, S, 1);  \
    } while (0)
    if (img_dtype == MEM_U8) {
        if (L.storage == MEM_BF16) MEM_GF2(MEM_U8, MEM_BF16, 8);
        else if (L.storage == MEM_FP8_E4M3) MEM_GF2(MEM_U8, MEM_FP8_E4M3, 8);
        else MEM_GF2(MEM_U8, MEM_F32, 4);
    } else {
        if (L.storage == MEM_BF16) MEM_GF2(MEM_F32, MEM_BF16, 8);
        else if (L.storage == MEM_FP8_E4M3) MEM_GF2(MEM_F32, MEM_FP8_E4M3, 8);
        else MEM_GF2(MEM_F32, MEM_F32, 4);
    }
#undef MEM_GF2
#undef MEM_GF
}

}  // namespace memk
