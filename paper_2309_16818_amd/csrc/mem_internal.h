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
#include <cstring>
#include <string>
#include <vector>

#include <hip/hip_ext.h>

#include "../../include/mem.h"

namespace memk {

constexpr int kMaxBind = 8;
constexpr int kMaxTopk = 64;  // classes listed per top-k class input
constexpr int kStats = 15;  // device counters, order of mem_stats
// Device counters are [kStats][kStatSlots]: a workgroup adds into slot
// (block id mod kStatSlots), so no single address sees more than
// 1/kStatSlots of the atomics.
constexpr int kStatSlots = 64;

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
    ST_OCCL_CELLS,
    ST_RAY_STEPS,
    ST_OCCL_STEPS,
    ST_FLUSHES,
    ST_SEGMENTS
};

// Grid geometry handed to every kernel.
struct Grid {
    int W, H;
    int ox, oy;  // absolute lattice index of logical cell (0, 0)
    int rx, ry;  // toroidal offsets
    float res, inv_res;
};

// Largest height over square blocks of logical cells (-inf where no cell of
// the block holds a height): side 8 in t8 ([th8][tw8]) and side 64 in t64.
struct TileMax {
    const float* t8;
    const float* t64;
    int tw8, th8, tw64, th64;
};

struct Pose {
    float m[12];  // row-major [R | t]
};

// One user layer as the kernels see it.
// A layer's FP8 scales in one device block: C binary32 scales, then, from
// a 16-byte aligned offset, their reciprocals rounded to binary32.
inline size_t scale_block_floats(int C) { return 2 * (size_t)((C + 3) & ~3); }
inline float* scale_block_rcp(float* scale, int C) { return scale ? scale + ((C + 3) & ~3) : nullptr; }
// Scales for which the vector gather divides through the reciprocal
// (div_rcp): over this range the corrected product gives the E4M3 code of
// the correctly rounded quotient.  A layer with a scale outside it leaves
// the reciprocals unused and takes the one-channel gather, which divides.
inline bool scale_rcp_ok(float s) { return s >= 0x1p-60f && s <= 0x1p60f; }
// The block of scales sc; *rcp_ok tells whether every scale is in range.
inline std::vector<float> scale_block_host(const std::vector<float>& sc, bool* rcp_ok)
{
    const int C = (int)sc.size();
    std::vector<float> blk(scale_block_floats(C), 0.0f);
    *rcp_ok = true;
    for (int q = 0; q < C; q++) {
        blk[q] = sc[q];
        blk[((C + 3) & ~3) + q] = (float)(1.0 / (double)sc[q]);  // correctly rounded: 53 >= 2 * 24 + 2
        *rcp_ok = *rcp_ok && scale_rcp_ok(sc[q]);
    }
    return blk;
}

struct LayerDev {
    void* val;
    float* var;
    float* scale;   // FP8: per-channel amax/448 (device)
    float* rscale;  // FP8: 1 / scale rounded to binary32 (device), or null (scale_rcp_ok)
    int C, rule, storage;
    float param;
};

// Point channel binding resolved against the map's layers.
struct PointBind {
    int layer;     // index into layers
    int ch_first;  // input channel
    int C;         // the layer's channels (planes of chsum)
    int sum_off;   // first plane of this binding in chsum
    int topk;      // 0: C dense inputs; k > 0: k class indices, then k probabilities
};

struct PointBinds {
    int n;
    int c_in;    // channels per input point
    int Cb;      // total bound channels (planes of chsum)
    int lds_ch;  // 1: channel sums are reduced in LDS before the global atomics
    PointBind b[kMaxBind];
    LayerDev L[kMaxBind];
};

// Drift compensation of one point cloud: the consistent points' binary64
// sums, their count, and the binary32 offset that was applied (0 if none).
struct DriftDev {
    double sw;   // sum of 1 / (v + v_i)
    double swe;  // sum of e_i / (v + v_i)
    int n;       // consistent points
    float d;     // offset applied to the held heights
};

constexpr int kMaxImages = 4;  // images sharing one camera pose per call

// One camera pose and the intrinsics / sizes of the images taken from it.
struct Camera {
    Pose T;
    int n;
    float fx[kMaxImages], fy[kMaxImages], cx[kMaxImages], cy[kMaxImages];
    int h[kMaxImages], w[kMaxImages];
    float min_depth;
};

// Camera poses projected by one launch: their lists, pixel codes and
// counters lie at pose * cap, pose * kMaxImages * cap and pose.
constexpr int kMaxPoses = 4;
struct CameraSet {
    Camera c[kMaxPoses];
    int n;
};

// Events a profiled launcher hands to hipExtLaunchKernel: `start` is
// recorded when its first kernel starts executing and `stop` when its last
// one ends, so their interval is the kernels' own time (no dispatch gap);
// null when not profiling.
struct LaunchEv {
    hipEvent_t start = nullptr, stop = nullptr;
};

// ---- launchers (implemented in the .hip files) ----
// `march_counts`, if not null, are the clearing march's kSegLists list
// counts, cleared as well.
// `hl`, if not null, receives a copy of the heights `h` in logical order
// (index y * W + x).
void launch_zero_accum(hipStream_t s, const Grid& g, int* n, float* wsum, float* ssum, int* clr,
                       float* chsum, int Cb, int* march_counts, const float* h, float* hl, DriftDev* drift,
                       LaunchEv ev = {});
// LDS bytes of the ingest kernel for `Cb` channel planes reduced in LDS.
size_t ingest_lds_bytes(int Cb);
struct MarchBufs;
// `march`, if not null: also lists the clearing march's segments of this
// cloud's rays (a single pass: n <= march->cap_pts).
void launch_ingest(hipStream_t s, const Grid& g, const float* xyz, int64_t n, const float* ch,
                   const Pose& T, float c0, float c1, float mr2, const PointBinds& pb, int* cnt,
                   float* wsum, float* ssum, float2* stash, float* chsum, const MarchBufs* march,
                   unsigned long long* stats, LaunchEv ev = {});
// The clearing march's buffers: a pass's rays (1 / major extent, height
// difference, cell), the
// kSegSubs sub-lists of their full segments of kSegLen cells (full_sub
// entries each), the 4 x kSegSubs sub-lists of their last, shorter segments
// by length class (part_sub entries each) and the kSegLists x kSegSubs
// counts (cleared by launch_zero_accum).
constexpr int kSegLen = 64;
constexpr int kSegLists = 5;
constexpr int kSegSubs = 64;
constexpr int64_t kMarchPass = 1 << 20;        // points per pass at most
constexpr int64_t kMarchFullCap = 1 << 24;     // full segments per pass at most
struct MarchSizes {
    int64_t full_sub = 0, part_sub = 0;
};
struct MarchBufs {
    float4* rec = nullptr;  // cap_pts: (inv_d, dz, ix | iy << 16, 0) of rays with cells to walk
    int2* full = nullptr;   // kSegSubs * full_sub: (ray, segment)
    int2* part = nullptr;   // 4 * kSegSubs * part_sub
    int* counts = nullptr;  // kSegLists * kSegSubs, list-major
    int64_t cap_pts = 0, full_sub = 0, part_sub = 0;
};
// Clouds binned by one launch (launch_ingest_clouds): each with its own
// sums and ray lists (a single clearing pass: n <= mb.cap_pts), no bound
// channels.
struct IngestCloud {
    const float* xyz;
    int64_t n;
    Pose T;
    int* cnt;  // the cloud's sums (as for launch_ingest)
    float* wsum;
    float* ssum;
    float2* stash;
    MarchBufs mb;
};
constexpr int kMaxClouds = 8;
struct IngestClouds {
    IngestCloud c[kMaxClouds];
    int n;
};
void launch_ingest_clouds(hipStream_t s, const Grid& g, const IngestClouds& cl, float c0, float c1, float mr2,
                          unsigned long long* stats, LaunchEv ev = {});
// Points per pass for a cloud of n points (at most kMarchPass, and few
// enough that the full list holds every segment) and the full segments a
// ray within the map's range can have.
void march_pass(float mr2, float res, int64_t n, int64_t* pts, int64_t* full_per_ray);
// Sub-list capacities for passes of `pts` points.
MarchSizes march_sizes(int64_t pts, int64_t full_per_ray);
// The march reads the heights in logical order (`hl`, written by
// launch_zero_accum) and counts votes into the storage-order layer `clr`.
// `prepared`: the point ingest already listed the first pass's segments
// (launch_ingest with `march`, for a cloud of at most cap_pts points).
void launch_clear_march(hipStream_t s, const Grid& g, const float* xyz, int64_t n, const Pose& T,
                        float mr2, float margin, const float* hl, int* clr, const MarchBufs& mb,
                        bool prepared, unsigned long long* stats, LaunchEv ev = {});
// z-error count and drift compensation of one cloud: the consistent points'
// sums into `drift`, then, with at least min_points of them, the shift of
// every held height h (and its logical-order copy hl, if given) by their
// precision-weighted mean error.  Reads h and v before the height update.
// `part` holds drift_part_bytes() of per-workgroup partial sums.
void launch_drift(hipStream_t s, const Grid& g, const float* xyz, int64_t n, const Pose& T, float c0,
                  float c1, float mr2, float* h, const float* v, float kappa2, int min_points,
                  DriftDev* drift, void* part, float* hl);
size_t drift_part_bytes();
// The cloud's end: fuses the accumulated sums into the heights and bound
// layers.  With clean set it also prepares the next cloud, so that it needs
// no separate clearing pass: the sums of every cell that received points
// return to zero (cnt and clr stay: they become the last cloud's counts),
// the count buffers of the cloud before (zero_cnt, zero_clr: the next
// cloud's accumulators) are zeroed, march_counts too and, if given, the
// drift record; if hl is given (hl equal to h in logical order before the
// call), every changed height is written into it.
void launch_finalize(hipStream_t s, const Grid& g, int* cnt, float* wsum, float* ssum, const float2* stash,
                     int* clr, int clear_min, float* h, float* v, float* chsum, const PointBinds& pb,
                     unsigned long long* stats, bool clean = false, int* zero_cnt = nullptr,
                     int* zero_clr = nullptr, float* hl = nullptr, int* march_counts = nullptr,
                     DriftDev* drift = nullptr, LaunchEv ev = {});
void launch_point_cells(hipStream_t s, const Grid& g, const float* xyz, int64_t n, const Pose& T,
                        float mr2, int32_t* out);

void launch_zero_int(hipStream_t s, int* p, int n);
// Block maxima of h (sizes from tile_max_dims: ceil(W/8) x ceil(H/8) and
// ceil(W/64) x ceil(H/64) floats).
TileMax tile_max_dims(const Grid& g, const float* t8, const float* t64);
void launch_tile_max(hipStream_t s, const Grid& g, const float* h, float* t8, float* t64);
// Two passes: k_view lists the cells inside any image's view in vlist
// (st, ix | iy << 16, intermediate cells of the occlusion line, height
// bits; *vcount entries, at most cap) with their pixel codes in
// vcode[k * cap + position] (-1 outside image k), k_occlude overwrites the
// codes of occluded cells with -1.
// Every pose's counter must be zero on entry; k_view clears *vcount_next (a
// different counter, the next projection's; may be null) so that no
// separate clear is launched.  dbg is written for a single pose only.
void launch_project(hipStream_t s, const Grid& g, const CameraSet& cs, const float* h, const TileMax& tm, int cap,
                    int* vcount, int* vcount_next, int4* vlist, int* vcode, int32_t* dbg,
                    unsigned long long* stats, LaunchEv ev = {});
// Fuses image channels into layer L for the listed cells whose code (image's
// row of vcode) is >= 0.
// topk > 0: the binding's inputs are topk class indices then their
// probabilities (Dirichlet layers), fused by one lane per visible pair.
void launch_gather_fuse(hipStream_t s, const int4* vlist, const int* vcode, const int* count, int max_pairs,
                        const void* img, int img_dtype, int64_t s0, int64_t s1, int64_t s2, int w,
                        int ch_first, const LayerDev& L, int topk = 0, bool one_channel = false,
                        LaunchEv ev = {});
// One image binding's gather (launch_gather_fuse's arguments) as a job of a
// fused launch: gather_job fills in its variant and lane count.
struct GatherJob {
    const int4* vlist;
    const int* vcode;
    const int* count;
    const void* img;
    int64_t s0, s1, s2;
    LayerDev L;
    int w, ch_first, topk;
    int lpp_log2;  // lanes per visible pair: 2^lpp_log2
    int kind;      // image type x storage type x (vector, one channel, top-k)
    int blocks;    // workgroups of the job
    int block0;    // its first workgroup in the fused grid
};
constexpr int kMaxGatherJobs = 8;
struct GatherJobs {
    GatherJob j[kMaxGatherJobs];
    int n;
};
GatherJob gather_job(const int4* vlist, const int* vcode, const int* count, int max_pairs, const void* img,
                     int img_dtype, int64_t s0, int64_t s1, int64_t s2, int w, int ch_first, const LayerDev& L,
                     int topk, bool one_channel);
// Runs jobs.j[0 .. n) as one launch, each on its own workgroups.  The jobs
// must write different layers: their order inside the launch is not defined.
void launch_gather_multi(hipStream_t s, GatherJobs& jobs, LaunchEv ev = {});

// ---- batches of maps ----

// One map of a batch as the kernels see it during a step.
struct BatchMap {
    Grid g;
    int64_t cell_off;       // first cell of the map in the concatenated arrays
    int64_t pt_begin, pt_end;
    int64_t img_off;        // first element of the map's image
    Pose T;                 // sensor pose of this step
    Camera cam;             // this step's camera (cam.n = 0: none)
    int itile_base;         // first ingest tile of the map
    int itiles_x;           // ingest tiles per row of storage cells
    int pad0, pad1;
};

struct BatchRect {          // cells of map `map` entering the grid this step
    int map, x0, x1, y0, y1, pad0, pad1, pad2;
};

struct BatchItem {          // a work item: map plus two item-specific fields
    int map, a, b, pad;
};

// Device pointers of a batch (concatenated over maps).
struct BatchDev {
    float* h;
    float* hl;              // this step's heights in logical order, for the clearing walks
    float* v;
    int* cnt;
    int* clr;
    float* wsum;
    float* ssum;
    float2* stash;
    int2* pairs;            // per map at cell_off
    int* pair_count;        // [n_maps]
    int* qctr;              // work-queue counters, [kQueues]
    int* n_items;           // [0] rects, [1] point chunks (this step)
    const BatchMap* maps;
    const BatchRect* rects;
    const int* chunk_start;  // [n_maps + 1]: first point-chunk item of each map
    const BatchItem* tiles;  // (map, x0, y0): projection tiles
    const BatchItem* gitems; // (map, first pair): gather items
    const BatchItem* itiles; // (map, sx0, sy0): ingest tiles of storage cells
    float4* rec;             // accepted points binned by ingest tile: (sx | sy << 16, z, v, -)
    int* tile_start;         // [n_itiles] first record of each ingest tile
    int* tile_cnt;           // [n_itiles] its records
    int* tile_cur;           // [n_itiles] the binning's scatter cursors
    int n_tiles, n_gitems, n_maps, chunk;
    int n_itiles, itile_h;   // ingest tiles are kIngestTileW x itile_h cells
    int64_t total_cells;
    unsigned long long* stats;
};

constexpr int kQueues = 10;  // 0 reset, 1 ingest tiles, 2 march, 3 project, 4-7 gathers, 8 binning
constexpr int kIngestTileW = 64;  // ingest tile width (storage cells)
constexpr int kGatherItem = 4096;  // visible pairs per gather work item

struct BatchLaunch {        // tuning of one step
    int chunk;              // points per ingest / march item (power of two)
    int grid;               // persistent workgroups per stage
    int tile;               // projection tile side (8 or 16)
};

struct Profiler;
// prof: every stage's launch bracketed by events (NULL: none).
void launch_batch_step(hipStream_t s, const BatchDev& d, const BatchLaunch& bl, const float* xyz,
                       float c0, float c1, float mr2, float margin, int clear_min,
                       const LayerDev* L, int nL, const void* images, int img_dtype, int cam_c,
                       int cam_w, const mem_binding* ib, int n_ib, Profiler* prof);
// All LDS (static and dynamic) a tile-owned ingest workgroup needs for tiles
// of kIngestTileW x tile_h cells.
size_t batch_tile_ingest_lds_bytes(int tile_h);
constexpr int kBinTiles = 4096;  // ingest tiles a binning pass histograms at once

void launch_reset_rect(hipStream_t s, const Grid& g, int x0, int x1, int y0, int y1, float* h,
                       float* v, int* cnt, int* clr, const LayerDev* L, int nL);
void launch_readout(hipStream_t s, const Grid& g, int layer, int view, const float* h,
                    const float* v, const int* cnt, const int* clr, const LayerDev* L, float* out);
void launch_setlayer(hipStream_t s, const Grid& g, int layer, int view, float* h, float* v,
                     const LayerDev* L, const float* in);
// Overlap clearance: held heights within rxy of (sx, sy) horizontally and more
// than rz from sz vertically are removed.
void launch_overlap_clear(hipStream_t s, const Grid& g, float sx, float sy, float sz, float rxy, float rz, float* h);
// PCA layer of a feature layer of at most kPcaMaxC channels: the mean, the
// three leading components and eigenvalues into `res` (device), the
// projections into out ([H][W][3], logical order).  `scratch` holds
// pca_scratch_bytes().
constexpr int kPcaMaxC = 64;
constexpr int kPcaK = 3;
struct PcaOut {
    double mean[kPcaMaxC];
    double comp[kPcaK][kPcaMaxC];
    double lam[kPcaK];
    double n;  // cells with every channel observed
};
size_t pca_scratch_bytes();
// The same for kPcaMaxC + 1 .. kPcaWideC channels (k_pca_wide.hip): the
// covariance in 64 x 64 tiles and the three leading eigenpairs by orthogonal
// iteration with Rayleigh-Ritz.  `scratch` holds pca_wide_scratch_bytes(cells).
constexpr int kPcaWideC = 512;
struct PcaWideOut {
    double mean[kPcaWideC];
    double comp[kPcaK][kPcaWideC];
    double lam[kPcaK];
    double n;   // cells with every channel observed
    int iters;  // iterations the eigensolver took
};
size_t pca_wide_scratch_bytes(int64_t cells);
void launch_pca_wide(hipStream_t s, const Grid& g, const LayerDev& L, void* scratch, PcaWideOut* res, float* out,
                     float* lam_out);
// lam_out: device, kPcaK floats (the eigenvalues), or NULL.
void launch_pca(hipStream_t s, const Grid& g, const LayerDev& L, void* scratch, PcaOut* res, float* out,
                float* lam_out);
// The PCA's partial sums and result in the library's static device array on
// `device` (looked up on the first call for that device).
size_t pca_static_scratch_bytes();
hipError_t pca_static_scratch(int device, void** parts, PcaOut** res);
// Surface normals of the heights h (storage order) into out ([H][W][3], logical order).
void launch_normals(hipStream_t s, const Grid& g, const float* h, float* out);

}  // namespace memk
