// k_image.hip - image path of the map update (Sec. III-B, Fig. 3).
//
//   k_project      one lane per cell (16x16 cell tiles, so neighbouring rays
//                  share the cells they walk): frustum test, pin-hole pixel,
//                  Bresenham occlusion walk against the map heights, and a
//                  wave-aggregated append of visible (cell, pixel) pairs.
//   k_gather_fuse  grid-stride over the visible pairs; a group of lanes
//                  (a power of two >= the layer's channels, at most 64) reads
//                  one pixel's channels and read-modify-writes the cell's
//                  channel-contiguous layer row with the layer's rule.
#include "codec.h"
#include "fuse.h"
#include "geom.h"
#include "mem_internal.h"

namespace memk {

namespace {

constexpr int kTile = 16;

__global__ __launch_bounds__(256) void k_project(Grid g, Camera cam, const float* __restrict__ h,
                                                 int2* __restrict__ pairs, int* __restrict__ count,
                                                 int32_t* __restrict__ dbg,
                                                 unsigned long long* __restrict__ stats)
{
    const int ix = blockIdx.x * kTile + threadIdx.x;
    const int iy = blockIdx.y * kTile + threadIdx.y;
    const float* T = cam.T.m;
    int code = -1, st = 0, visited = 0, in_view = 0;
    if (ix < g.W && iy < g.H) {
        st = storage_index(g, ix, iy);
        float hj = h[st];
        if (!isnan(hj)) {
            float xc = ((float)(g.ox + ix) + 0.5f) * g.res;
            float yc = ((float)(g.oy + iy) + 0.5f) * g.res;
            float dx = xc - T[3], dy = yc - T[7], dz = hj - T[11];
            float P[3];
#pragma unroll
            for (int k = 0; k < 3; k++) {  // R^T d
                float a = T[0 + k] * dx;
                float b = T[4 + k] * dy;
                float c = T[8 + k] * dz;
                float s = a + b;
                P[k] = s + c;
            }
            code = -2;
            if (P[2] > cam.min_depth) {
                float u = cam.fx * P[0];
                u = u / P[2];
                u = u + cam.cx;
                float v = cam.fy * P[1];
                v = v / P[2];
                v = v + cam.cy;
                float uf = floorf(u + 0.5f);
                float vf = floorf(v + 0.5f);
                if (uf >= 0.0f && uf < (float)cam.w && vf >= 0.0f && vf < (float)cam.h) {
                    in_view = 1;
                    int ax, ay;
                    lattice_cell(g, T[3], T[7], ax, ay);
                    LineWalk L(ax, ay, ix, iy);
                    const float s_major = L.xmajor ? T[3] : T[7];
                    const float p_major = L.xmajor ? xc : yc;
                    const int o_major = L.xmajor ? g.ox : g.oy;
                    const float inv_d = 1.0f / (p_major - s_major);
                    const float dzr = hj - T[11];
                    bool occluded = false;
                    for (int s = 1; s < L.steps; s++) {
                        L.step();
                        if (L.x < 0 || L.x >= g.W || L.y < 0 || L.y >= g.H) continue;
                        visited++;
                        float hk = h[storage_index(g, L.x, L.y)];
                        float zr = ray_height(o_major + (L.xmajor ? L.x : L.y), g.res, s_major,
                                              inv_d, T[11], dzr);
                        if (hk >= zr) {  // NaN (no height) never occludes
                            occluded = true;
                            break;
                        }
                    }
                    code = occluded ? -3 : (int)vf * cam.w + (int)uf;
                }
            }
        }
    }
    const bool vis = code >= 0;
    unsigned long long mask = __ballot(vis);
    if (mask) {
        int lane = __lane_id();
        int leader = __ffsll((long long)mask) - 1;
        int base = 0;
        if (lane == leader) base = atomicAdd(count, __popcll(mask));
        base = __shfl(base, leader);
        if (vis) {
            int rank = __popcll(mask & ((1ull << lane) - 1ull));
            pairs[base + rank] = make_int2(st, code);
        }
    }
    if (dbg && ix < g.W && iy < g.H) dbg[iy * g.W + ix] = code;
    wave_stat_add(&stats[ST_IN_VIEW], in_view);
    wave_stat_add(&stats[ST_VISIBLE], vis ? 1 : 0);
    wave_stat_add(&stats[ST_OCCL_CELLS], visited);
}

template <int IMG>
__device__ __forceinline__ float pixel_value(const void* img, int64_t off)
{
    if (IMG == MEM_U8) return (float)((const uint8_t*)img)[off] / 255.0f;
    return ((const float*)img)[off];
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
    const int C = L.C;
    for (int64_t pbase = wave * ppw; pbase < N; pbase += nwaves * ppw) {
        int64_t p = pbase + sub;
        if (p >= N) continue;
        int2 pr = pairs[p];
        const int st = pr.x;
        const int row = pr.y / w, col = pr.y - (pr.y / w) * w;
        const int64_t pix = (int64_t)row * s0 + (int64_t)col * s1 + (int64_t)ch_first * s2;
        GaussCoef gc{0.0f, 1.0f, 0.0f, true};
        if (L.rule == MEM_GAUSS) gc = gauss_coef(L.param, L.var[st], 1);
        for (int q = q0; q < C; q += LPP) {
            float m = pixel_value<IMG>(img, pix + (int64_t)q * s2);
            int64_t idx = (int64_t)st * C + q;
            float old = Store<S>::load(L.val, idx, S == MEM_FP8_E4M3 ? L.scale[q] : 1.0f);
            float nv = fuse_value(L.rule, L.param, old, m, m, gc);
            Store<S>::store(L.val, idx, nv, S == MEM_FP8_E4M3 ? L.scale[q] : 1.0f);
        }
        if (L.rule == MEM_GAUSS && q0 == 0) L.var[st] = gc.var;
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
                    int* count, int32_t* dbg, unsigned long long* stats)
{
    dim3 grid((g.W + kTile - 1) / kTile, (g.H + kTile - 1) / kTile);
    hipLaunchKernelGGL(k_project, grid, dim3(kTile, kTile), 0, s, g, cam, h, pairs, count, dbg, stats);
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
