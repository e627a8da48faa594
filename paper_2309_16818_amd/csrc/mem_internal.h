// mem_internal.h - state and kernel launchers of the MI355X map update.
//
// Storage layout in HBM (one map):
//   h, v        float[H*W]   height and its variance; h is NaN where the
//                            cell holds no height (the validity flag).
//   n, clr      int32[H*W]   per-cloud point count and clearing votes.
//   wsum, ssum  float[H*W]   per-cloud sum 1/v_i and sum z_i/v_i.
//   stash       float2[H*W]  (z, v) of a cell's only point when one
//                            workgroup saw exactly one point there.
//   chsum       float[Cb][H*W] per-cloud channel sums, planar.
//   layer val   T[H*W][C]    channel-contiguous per cell (T = f32, bf16, fp8).
//   layer var   float[H*W]   Gaussian layers: posterior variance.
//   pairs       int2[H*W]    (storage cell, pixel) of visible cells.
//
// Cells are stored toroidally: logical cell (ix, iy) lives at storage
// ((iy + ry) mod H) * W + (ix + rx) mod W, so moving the map with the robot
// rewrites only the cells that enter the grid.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mem.h"

namespace memk {

constexpr int kMaxBind = 8;
constexpr int kStats = 11;  // device counters, order of mem_stats

enum Stat {
    ST_POINTS_IN = 0,
    ST_ACCEPTED,
    ST_NONFINITE,
    ST_RANGE,
    ST_OUTSIDE,
    ST_TOUCHED,
    ST_CLEARED,
    ST_RAY_CELLS,
    ST_IN_VIEW,
    ST_VISIBLE,
    ST_OCCL_CELLS
};

// Grid geometry handed to every kernel.
struct Grid {
    int W, H;
    int ox, oy;  // absolute lattice index of logical cell (0, 0)
    int rx, ry;  // toroidal offsets
    float res, inv_res;
};

struct Pose {
    float m[12];  // row-major [R | t]
};

// One user layer as the kernels see it.
struct LayerDev {
    void* val;
    float* var;
    float* scale;  // FP8: per-channel amax/448 (device)
    int C, rule, storage;
    float param;
};

// Point channel binding resolved against the map's layers.
struct PointBind {
    int layer;     // index into layers
    int ch_first;  // input channel
    int C;
    int sum_off;   // first plane of this binding in chsum
};

struct PointBinds {
    int n;
    int c_in;    // channels per input point
    int Cb;      // total bound channels (planes of chsum)
    int lds_ch;  // 1: channel sums are reduced in LDS before the global atomics
    PointBind b[kMaxBind];
    LayerDev L[kMaxBind];
};

struct Camera {
    Pose T;
    float fx, fy, cx, cy;
    int h, w;
    float min_depth;
};

// ---- launchers (implemented in the .hip files) ----
void launch_zero_accum(hipStream_t s, const Grid& g, int* n, float* wsum, float* ssum, int* clr,
                       float* chsum, int Cb);
// LDS bytes of the ingest kernel for `Cb` channel planes reduced in LDS.
size_t ingest_lds_bytes(int Cb);
void launch_ingest(hipStream_t s, const Grid& g, const float* xyz, int64_t n, const float* ch,
                   const Pose& T, float c0, float c1, float mr2, const PointBinds& pb, int* cnt,
                   float* wsum, float* ssum, float2* stash, float* chsum,
                   unsigned long long* stats);
void launch_clear_march(hipStream_t s, const Grid& g, const float* xyz, int64_t n, const Pose& T,
                        float mr2, float margin, const float* h, int* clr,
                        unsigned long long* stats);
void launch_finalize(hipStream_t s, const Grid& g, const int* cnt, const float* wsum,
                     const float* ssum, const float2* stash, const int* clr, int clear_min,
                     float* h, float* v, const float* chsum, const PointBinds& pb,
                     unsigned long long* stats);
void launch_point_cells(hipStream_t s, const Grid& g, const float* xyz, int64_t n, const Pose& T,
                        float mr2, int32_t* out);

void launch_zero_int(hipStream_t s, int* p, int n);
void launch_project(hipStream_t s, const Grid& g, const Camera& cam, const float* h, int2* pairs,
                    int* count, int32_t* dbg, unsigned long long* stats);
void launch_gather_fuse(hipStream_t s, const int2* pairs, const int* count, int max_pairs,
                        const void* img, int img_dtype, int64_t s0, int64_t s1, int64_t s2, int w,
                        int ch_first, const LayerDev& L);

void launch_reset_rect(hipStream_t s, const Grid& g, int x0, int x1, int y0, int y1, float* h,
                       float* v, int* cnt, int* clr, const LayerDev* L, int nL);
void launch_readout(hipStream_t s, const Grid& g, int layer, int view, const float* h,
                    const float* v, const int* cnt, const int* clr, const LayerDev* L, float* out);
void launch_setlayer(hipStream_t s, const Grid& g, int layer, int view, float* h, float* v,
                     const LayerDev* L, const float* in);

}  // namespace memk
