// k_image.hip - image path of the map update (Sec. III-B, Fig. 3), one map.
//
//   k_project      one lane per cell (16x16 cell tiles, so neighbouring rays
//                  share the cells they walk): frustum test and pin-hole pixel
//                  of every image of one camera pose, one Bresenham occlusion
//                  walk against the map heights, and a wave-aggregated append
//                  of visible (cell, pixel) pairs per image.
//   k_gather_fuse  grid-stride over one image's visible pairs; a group of
//                  lanes (a power of two >= the layer's channels, at most 64)
//                  reads one pixel's channels and read-modify-writes the
//                  cell's channel-contiguous layer row with the layer's rule.
#include "update.h"

namespace memk {

namespace {

constexpr int kTile = 16;

// Image k's visible pairs go to pairs[k * cap ...] and their number to
// count[k].  dbg (optional) receives image 0's code per logical cell.
__global__ __launch_bounds__(256) void k_project(Grid g, Camera cam, const float* __restrict__ h,
                                                 int2* __restrict__ pairs, int cap,
                                                 int* __restrict__ count, int32_t* __restrict__ dbg,
                                                 unsigned long long* __restrict__ stats)
{
    const int ix = blockIdx.x * kTile + threadIdx.x;
    const int iy = blockIdx.y * kTile + threadIdx.y;
    int code[kMaxImages];
#pragma unroll
    for (int k = 0; k < kMaxImages; k++) code[k] = -1;
    int st = 0, visited = 0, in_view = 0, n_vis = 0;
    if (ix < g.W && iy < g.H) {
        st = storage_index(g, ix, iy);
        visited = project_cell(g, cam, h, ix, iy, st, code, in_view);
    }
#pragma unroll
    for (int k = 0; k < kMaxImages; k++) {
        if (k >= cam.n) break;
        n_vis += code[k] >= 0 ? 1 : 0;
        append_pair(code[k] >= 0, st, code[k], pairs + (int64_t)k * cap, &count[k]);
    }
    if (dbg && ix < g.W && iy < g.H) dbg[iy * g.W + ix] = code[0];
    const int ids[3] = {ST_IN_VIEW, ST_VISIBLE, ST_OCCL_CELLS};
    int vals[3] = {in_view, n_vis, visited};
    block_stats(stats, ids, vals);
}

template <int IMG, int S>
__global__ __launch_bounds__(256) void k_gather_fuse(const int2* __restrict__ pairs,
                                                     const int* __restrict__ count,
                                                     const void* __restrict__ img, int64_t s0,
                                                     int64_t s1, int64_t s2, int w, int ch_first,
                                                     LayerDev L, int lpp_log2)
{
    const int N = *count;
    const int lane = threadIdx.x & 63;
    const int LPP = 1 << lpp_log2;
    const int sub = lane >> lpp_log2;
    const int q0 = lane & (LPP - 1);
    const int ppw = 64 >> lpp_log2;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t pbase = wave * ppw; pbase < N; pbase += nwaves * ppw) {
        const int64_t p = pbase + sub;
        if (p < N) gather_pair<IMG, S>(pairs[p], img, s0, s1, s2, w, ch_first, L, q0, LPP);
    }
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

void launch_project(hipStream_t s, const Grid& g, const Camera& cam, const float* h, int2* pairs,
                    int cap, int* count, int32_t* dbg, unsigned long long* stats)
{
    dim3 grid((g.W + kTile - 1) / kTile, (g.H + kTile - 1) / kTile);
    hipLaunchKernelGGL(k_project, grid, dim3(kTile, kTile), 0, s, g, cam, h, pairs, cap, count, dbg,
                       stats);
}

void launch_gather_fuse(hipStream_t s, const int2* pairs, const int* count, int max_pairs,
                        const void* img, int img_dtype, int64_t s0, int64_t s1, int64_t s2, int w,
                        int ch_first, const LayerDev& L)
{
    int lpp_log2 = 0;
    while ((1 << lpp_log2) < L.C && lpp_log2 < 6) lpp_log2++;
    int ppw = 64 >> lpp_log2;
    int64_t waves = ((int64_t)max_pairs + ppw - 1) / ppw;
    int64_t blocks = (waves + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    dim3 gr((unsigned)blocks), bl(256);
#define MEM_GF(IMG, S) \
    hipLaunchKernelGGL((k_gather_fuse<IMG, S>), gr, bl, 0, s, pairs, count, img, s0, s1, s2, w, ch_first, L, lpp_log2)
    if (img_dtype == MEM_U8) {
        if (L.storage == MEM_BF16) MEM_GF(MEM_U8, MEM_BF16);
        else if (L.storage == MEM_FP8_E4M3) MEM_GF(MEM_U8, MEM_FP8_E4M3);
        else MEM_GF(MEM_U8, MEM_F32);
    } else {
        if (L.storage == MEM_BF16) MEM_GF(MEM_F32, MEM_BF16);
        else if (L.storage == MEM_FP8_E4M3) MEM_GF(MEM_F32, MEM_FP8_E4M3);
        else MEM_GF(MEM_F32, MEM_F32);
    }
#undef MEM_GF
}

}  // namespace memk
