// batch_api.hip - host side of the mem_batch_* entry points (include/mem.h).
//
// A batch keeps every map's per-cell state in one arena (concatenated in
// map order), so the persistent kernels index any map's cells with a global
// cell index and the autotuner can snapshot / restore all maps with one copy.
// Per step the host computes each map's move (same binary32 formula as
// mem_move), the rectangles of cells entering each grid and the point-chunk
// work items, writes them to a pinned staging buffer (two, used in turn) and
// launches a HIP graph that copies them to the device and runs the stages.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mem_internal.h"
#include "prof.h"

using namespace memk;

namespace memk {
mem_status api_fail(mem_status code, const char* fmt, ...);
}

namespace {

struct BLayer {
    int C, rule, storage;
    float param;
    void* val = nullptr;
    float* var = nullptr;
    float* scale = nullptr;
    bool rcp = false;  // the scales allow the reciprocal divide
    LayerDev dev(int64_t off = 0) const
    {
        LayerDev d;
        int esz = storage == MEM_BF16 ? 2 : storage == MEM_FP8_E4M3 ? 1 : 4;
        d.val = (char*)val + off * C * esz;
        d.var = var ? var + off : nullptr;
        d.scale = scale;
        d.rscale = rcp ? scale_block_rcp(scale, C) : nullptr;
        d.C = C;
        d.rule = rule;
        d.storage = storage;
        d.param = param;
        return d;
    }
};

struct Staging {
    char* host = nullptr;  // pinned
    hipEvent_t done = nullptr;
    bool used = false;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    const void* key_xyz = nullptr;
    const void* key_img = nullptr;
    BatchLaunch key_bl{0, 0, 0};
};

}  // namespace

struct mem_batch {
    int n = 0;
    std::vector<int> W, H;
    std::vector<int64_t> cell_off;
    int64_t total = 0;
    std::vector<Grid> grid;  // current centre / ring offsets per map
    float res = 0, inv_res = 0, c0 = 0, c1 = 0, mr2 = 0, margin = 0, min_depth = 0;
    int clear_min = 0;
    int64_t max_points = 0;
    int cam_h = 0, cam_w = 0, cam_c = 0, cam_dtype = MEM_F32;
    std::vector<mem_binding> img_bind;
    std::vector<BLayer> layers;
    int n_cu = 256, max_lds = 65536;
    bool broken = false;

    char* arena = nullptr;
    size_t arena_bytes = 0;
    float *h = nullptr, *v = nullptr, *wsum = nullptr, *ssum = nullptr, *hl = nullptr;
    int *cnt = nullptr, *clr = nullptr;
    float2* stash = nullptr;

    int2* pairs = nullptr;
    int* pair_count = nullptr;
    int* qctr = nullptr;
    unsigned long long* stats = nullptr;
    char* tables = nullptr;  // device: n_items | maps | rects | chunks
    size_t tables_bytes = 0;
    size_t off_maps = 0, off_rects = 0, off_chunks = 0;
    BatchItem* tiles = nullptr;
    int n_tiles = 0, tiles_side = 0;
    BatchItem* gitems = nullptr;
    int n_gitems = 0;
    BatchItem* itiles = nullptr;
    int n_itiles = 0, itile_h = 64;
    std::vector<int> itile_base, itiles_x;  // per map
    float4* rec = nullptr;                  // binned points, max_points records
    int* tile_start = nullptr;
    int* tile_cnt = nullptr;
    int* tile_cur = nullptr;

    Staging stg[2];
    int next_stg = 0;
    hipStream_t cap_stream = nullptr;
    BatchLaunch bl{1024, 1024, 16};
    bool use_graph = true;
    double tuned_ms = 0.0;
    Profiler prof;  // while on, steps launch directly with events around every stage
};

namespace {

mem_status bfail(mem_batch* b, hipError_t e, const char* what)
{
    if (b) b->broken = true;
    return api_fail(MEM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define BTRY(b, call)                                      \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return bfail((b), e_, #call); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

mem_status busable(const mem_batch* b)
{
    if (!b) return api_fail(MEM_E_ARG, "batch is NULL");
    if (b->broken) return api_fail(MEM_E_STATE, "batch is unusable after an earlier HIP error");
    return MEM_OK;
}

void free_batch(mem_batch* b)
{
    b->prof.release();
    for (auto& s : b->stg) {
        if (s.exec) (void)hipGraphExecDestroy(s.exec);
        if (s.graph) (void)hipGraphDestroy(s.graph);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.host) (void)hipHostFree(s.host);
    }
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    (void)hipFree(b->arena);
    (void)hipFree(b->pairs);
    (void)hipFree(b->pair_count);
    (void)hipFree(b->qctr);
    (void)hipFree(b->stats);
    (void)hipFree(b->tables);
    (void)hipFree(b->tiles);
    (void)hipFree(b->gitems);
    (void)hipFree(b->itiles);
    (void)hipFree(b->rec);
    (void)hipFree(b->tile_start);
    (void)hipFree(b->tile_cnt);
    (void)hipFree(b->tile_cur);
    for (auto& L : b->layers) (void)hipFree(L.scale);
    delete b;
}

Grid initial_grid(const mem_batch* b, int m)
{
    Grid g;
    g.W = b->W[m];
    g.H = b->H[m];
    g.ox = -(g.W / 2);
    g.oy = -(g.H / 2);
    g.rx = 0;
    g.ry = 0;
    g.res = b->res;
    g.inv_res = b->inv_res;
    return g;
}

// Same checks as the single-map path's pose validation.
mem_status check_pose_b(const mem_batch* b, const Grid& g, const float* T, const char* what, int m)
{
    for (int k = 0; k < 12; k++)
        if (!std::isfinite(T[k])) return api_fail(MEM_E_ARG, "map %d: %s has a non-finite entry", m, what);
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++) {
            double d = 0;
            for (int k = 0; k < 3; k++) d += (double)T[4 * a + k] * T[4 * c + k];
            if (std::fabs(d - (a == c ? 1.0 : 0.0)) > 1e-4)
                return api_fail(MEM_E_ARG, "map %d: %s rotation is not orthonormal", m, what);
        }
    const double lim = 4194304.0;
    if (std::fabs((double)T[3] * b->inv_res) > lim || std::fabs((double)T[7] * b->inv_res) > lim)
        return api_fail(MEM_E_ARG, "map %d: %s translation is too far from the origin", m, what);
    const int cx = g.ox + g.W / 2, cy = g.oy + g.H / 2;
    const double reach = 4.0 * std::max(g.W, g.H) + 2.0;
    if (std::fabs(std::floor((double)(T[3] * b->inv_res)) - cx) > reach ||
        std::fabs(std::floor((double)(T[7] * b->inv_res)) - cy) > reach)
        return api_fail(MEM_E_ARG, "map %d: %s lies more than 4 grid widths from the grid", m, what);
    return MEM_OK;
}

mem_status build_tiles(mem_batch* b, int side)
{
    std::vector<BatchItem> t;
    for (int m = 0; m < b->n; m++)
        for (int y = 0; y < b->H[m]; y += side)
            for (int x = 0; x < b->W[m]; x += side) t.push_back(BatchItem{m, x, y, 0});
    (void)hipFree(b->tiles);
    b->tiles = nullptr;
    BTRY(b, hipMalloc((void**)&b->tiles, sizeof(BatchItem) * t.size()));
    BTRY(b, hipMemcpy(b->tiles, t.data(), sizeof(BatchItem) * t.size(), hipMemcpyHostToDevice));
    b->n_tiles = (int)t.size();
    b->tiles_side = side;
    return MEM_OK;
}

// Ingest tiles: kIngestTileW x itile_h blocks of every map's storage cells,
// as tall as the device's LDS allows (64 or 32 rows).
mem_status build_itiles(mem_batch* b)
{
    b->itile_h = batch_tile_ingest_lds_bytes(64) <= (size_t)b->max_lds ? 64 : 32;
    std::vector<BatchItem> t;
    for (int m = 0; m < b->n; m++) {
        b->itile_base.push_back((int)t.size());
        b->itiles_x.push_back((b->W[m] + kIngestTileW - 1) / kIngestTileW);
        for (int y = 0; y < b->H[m]; y += b->itile_h)
            for (int x = 0; x < b->W[m]; x += kIngestTileW) t.push_back(BatchItem{m, x, y, 0});
    }
    BTRY(b, hipMalloc((void**)&b->itiles, sizeof(BatchItem) * t.size()));
    BTRY(b, hipMemcpy(b->itiles, t.data(), sizeof(BatchItem) * t.size(), hipMemcpyHostToDevice));
    b->n_itiles = (int)t.size();
    BTRY(b, hipMalloc((void**)&b->tile_start, sizeof(int) * t.size()));
    BTRY(b, hipMalloc((void**)&b->tile_cnt, sizeof(int) * t.size()));
    BTRY(b, hipMalloc((void**)&b->tile_cur, sizeof(int) * t.size()));
    BTRY(b, hipMalloc((void**)&b->rec, sizeof(float4) * (size_t)std::max<int64_t>(b->max_points, 1)));
    return MEM_OK;
}

void drop_graphs(mem_batch* b)
{
    for (auto& s : b->stg) {
        if (s.exec) (void)hipGraphExecDestroy(s.exec);
        if (s.graph) (void)hipGraphDestroy(s.graph);
        s.exec = nullptr;
        s.graph = nullptr;
    }
}

BatchDev device_view(const mem_batch* b)
{
    BatchDev d;
    d.h = b->h;
    d.hl = b->hl;
    d.v = b->v;
    d.cnt = b->cnt;
    d.clr = b->clr;
    d.wsum = b->wsum;
    d.ssum = b->ssum;
    d.stash = b->stash;
    d.pairs = b->pairs;
    d.pair_count = b->pair_count;
    d.qctr = b->qctr;
    d.n_items = (int*)b->tables;
    d.maps = (const BatchMap*)(b->tables + b->off_maps);
    d.rects = (const BatchRect*)(b->tables + b->off_rects);
    d.chunk_start = (const int*)(b->tables + b->off_chunks);
    d.chunk = b->bl.chunk;
    d.tiles = b->tiles;
    d.gitems = b->gitems;
    d.itiles = b->itiles;
    d.n_itiles = b->n_itiles;
    d.itile_h = b->itile_h;
    d.rec = b->rec;
    d.tile_start = b->tile_start;
    d.tile_cnt = b->tile_cnt;
    d.tile_cur = b->tile_cur;
    d.n_tiles = b->n_tiles;
    d.n_gitems = b->n_gitems;
    d.n_maps = b->n;
    d.total_cells = b->total;
    d.stats = b->stats;
    return d;
}

// Fills staging buffer s for input `in`; returns the bytes to copy.
mem_status prepare(mem_batch* b, const mem_batch_input* in, Staging& s, size_t* bytes)
{
    const int n = b->n;
    const bool cams = in->images != nullptr;
    // validation (nothing is written to the maps' state on failure)
    if (!in->robot_xy || !in->offsets || !in->T_map_sensor)
        return api_fail(MEM_E_ARG, "robot_xy, offsets and T_map_sensor are required");
    if (in->offsets[0] != 0) return api_fail(MEM_E_ARG, "offsets[0] must be 0");
    for (int m = 0; m < n; m++)
        if (in->offsets[m + 1] < in->offsets[m]) return api_fail(MEM_E_ARG, "offsets must not decrease");
    if (in->offsets[n] > b->max_points) return api_fail(MEM_E_ARG, "more points than max_points");
    if (in->offsets[n] > 0 && !in->xyz) return api_fail(MEM_E_ARG, "xyz is NULL");
    if (cams && (b->cam_h == 0 || !in->K || !in->T_map_cam))
        return api_fail(MEM_E_ARG, "images need a batch with cameras, K and T_map_cam");
    std::vector<Grid> g2 = b->grid;
    std::vector<BatchRect> rects;
    for (int m = 0; m < n; m++) {
        const float x = in->robot_xy[2 * m], y = in->robot_xy[2 * m + 1];
        if (!std::isfinite(x) || !std::isfinite(y)) return api_fail(MEM_E_ARG, "map %d: position must be finite", m);
        if (std::fabs((double)x * b->inv_res) > 4194304.0 || std::fabs((double)y * b->inv_res) > 4194304.0)
            return api_fail(MEM_E_ARG, "map %d: position is too far from the origin", m);
        Grid& g = g2[m];
        const int cx = g.ox + g.W / 2, cy = g.oy + g.H / 2;
        const float gx = floorf(x * b->inv_res), gy = floorf(y * b->inv_res);
        const int ncx = (int)gx, ncy = (int)gy, sx = ncx - cx, sy = ncy - cy;
        if (sx != 0 || sy != 0) {
            g.ox = ncx - g.W / 2;
            g.oy = ncy - g.H / 2;
            if (std::abs(sx) >= g.W || std::abs(sy) >= g.H) {
                g.rx = 0;
                g.ry = 0;
                rects.push_back(BatchRect{m, 0, g.W, 0, g.H, 0, 0, 0});
            } else {
                g.rx = ((g.rx + sx) % g.W + g.W) % g.W;
                g.ry = ((g.ry + sy) % g.H + g.H) % g.H;
                if (sx > 0) rects.push_back(BatchRect{m, g.W - sx, g.W, 0, g.H, 0, 0, 0});
                if (sx < 0) rects.push_back(BatchRect{m, 0, -sx, 0, g.H, 0, 0, 0});
                if (sy > 0) rects.push_back(BatchRect{m, 0, g.W, g.H - sy, g.H, 0, 0, 0});
                if (sy < 0) rects.push_back(BatchRect{m, 0, g.W, 0, -sy, 0, 0, 0});
            }
        }
        if (mem_status st = check_pose_b(b, g, in->T_map_sensor + 12 * m, "T_map_sensor", m)) return st;
        if (cams) {
            if (mem_status st = check_pose_b(b, g, in->T_map_cam + 12 * m, "T_map_cam", m)) return st;
            const float* K = in->K + 4 * m;
            for (int q = 0; q < 4; q++)
                if (!std::isfinite(K[q])) return api_fail(MEM_E_ARG, "map %d: K must be finite", m);
            if (!(K[0] > 0.0f) || !(K[1] > 0.0f)) return api_fail(MEM_E_ARG, "map %d: fx, fy must be positive", m);
        }
    }
    // tables
    int* n_items = (int*)s.host;
    BatchMap* maps = (BatchMap*)(s.host + b->off_maps);
    BatchRect* R = (BatchRect*)(s.host + b->off_rects);
    int* C = (int*)(s.host + b->off_chunks);
    int64_t nc = 0;
    for (int m = 0; m < n; m++) {
        BatchMap& M = maps[m];
        M.g = g2[m];
        M.cell_off = b->cell_off[m];
        M.pt_begin = in->offsets[m];
        M.pt_end = in->offsets[m + 1];
        M.img_off = (int64_t)m * b->cam_h * b->cam_w * b->cam_c;
        memcpy(M.T.m, in->T_map_sensor + 12 * m, sizeof(M.T.m));
        memset(&M.cam, 0, sizeof(M.cam));
        if (cams) {
            memcpy(M.cam.T.m, in->T_map_cam + 12 * m, sizeof(M.cam.T.m));
            M.cam.n = 1;
            M.cam.fx[0] = in->K[4 * m];
            M.cam.fy[0] = in->K[4 * m + 1];
            M.cam.cx[0] = in->K[4 * m + 2];
            M.cam.cy[0] = in->K[4 * m + 3];
            M.cam.h[0] = b->cam_h;
            M.cam.w[0] = b->cam_w;
            M.cam.min_depth = b->min_depth;
        }
        M.itile_base = b->itile_base[m];
        M.itiles_x = b->itiles_x[m];
        M.pad0 = M.pad1 = 0;
        C[m] = (int)nc;
        nc += (M.pt_end - M.pt_begin + b->bl.chunk - 1) / b->bl.chunk;
    }
    C[n] = (int)nc;
    for (size_t r = 0; r < rects.size(); r++) R[r] = rects[r];
    n_items[0] = (int)rects.size();
    n_items[1] = (int)nc;
    *bytes = b->tables_bytes;
    b->grid = g2;  // the maps move with this step
    return MEM_OK;
}

void enqueue_step(mem_batch* b, hipStream_t s, Staging& st, size_t bytes, const mem_batch_input* in, Profiler* prof)
{
    (void)hipMemcpyAsync(b->tables, st.host, bytes, hipMemcpyHostToDevice, s);
    std::vector<LayerDev> L;
    for (auto& l : b->layers) L.push_back(l.dev());
    launch_batch_step(s, device_view(b), b->bl, in->xyz, b->c0, b->c1, b->mr2, b->margin, b->clear_min,
                      L.data(), (int)L.size(), in->images, b->cam_dtype, b->cam_c, b->cam_w,
                      b->img_bind.data(), (int)b->img_bind.size(), prof);
}

mem_status run_step(mem_batch* b, const mem_batch_input* in, hipStream_t s)
{
    Staging& st = b->stg[b->next_stg];
    if (st.used) BTRY(b, hipEventSynchronize(st.done));  // its previous copy has been read
    size_t bytes = 0;
    std::vector<Grid> saved = b->grid;
    if (mem_status r = prepare(b, in, st, &bytes)) {
        b->grid = saved;
        return r;
    }
    if (b->use_graph && !b->prof.on) {
        // The graph copies the whole table region, so its node is independent
        // of this step's item count.
        const size_t full = b->tables_bytes;
        const bool stale = !st.exec || st.key_xyz != (const void*)in->xyz ||
                           st.key_img != in->images || st.key_bl.chunk != b->bl.chunk ||
                           st.key_bl.grid != b->bl.grid || st.key_bl.tile != b->bl.tile;
        if (stale) {
            if (st.exec) (void)hipGraphExecDestroy(st.exec);
            if (st.graph) (void)hipGraphDestroy(st.graph);
            st.exec = nullptr;
            st.graph = nullptr;
            BTRY(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
            enqueue_step(b, b->cap_stream, st, full, in, nullptr);
            BTRY(b, hipStreamEndCapture(b->cap_stream, &st.graph));
            BTRY(b, hipGraphInstantiate(&st.exec, st.graph, nullptr, nullptr, 0));
            st.key_xyz = in->xyz;
            st.key_img = in->images;
            st.key_bl = b->bl;
        }
        BTRY(b, hipGraphLaunch(st.exec, s));
    } else {
        enqueue_step(b, s, st, bytes, in, b->prof.on ? &b->prof : nullptr);
        BTRY(b, hipGetLastError());
    }
    BTRY(b, hipEventRecord(st.done, s));
    st.used = true;
    b->next_stg ^= 1;
    return MEM_OK;
}

}  // namespace

extern "C" {

mem_status mem_batch_create(const mem_batch_params* p, void* stream, mem_batch** out)
{
    if (!p || !out) return api_fail(MEM_E_ARG, "params and out must not be NULL");
    *out = nullptr;
    if (p->n_maps < 1 || p->n_maps > 65536 || !p->width || !p->height)
        return api_fail(MEM_E_ARG, "n_maps must be 1..65536 with width and height arrays");
    int64_t total = 0;
    for (int m = 0; m < p->n_maps; m++) {
        if (p->width[m] < 1 || p->width[m] > 16384 || p->height[m] < 1 || p->height[m] > 16384)
            return api_fail(MEM_E_ARG, "map %d: grid %dx%d outside 1..16384", m, p->width[m], p->height[m]);
        total += (int64_t)p->width[m] * p->height[m];
    }
    if (total >= ((int64_t)1 << 31)) return api_fail(MEM_E_ARG, "a batch holds fewer than 2^31 cells");
    if (!(p->resolution > 0.0f) || !std::isfinite(p->resolution)) return api_fail(MEM_E_ARG, "resolution must be positive");
    if (!std::isfinite(p->noise_c0) || !std::isfinite(p->noise_c1) || p->noise_c0 < 0 || p->noise_c1 < 0 ||
        (p->noise_c0 == 0 && p->noise_c1 == 0))
        return api_fail(MEM_E_ARG, "noise model needs c0, c1 >= 0, not both zero");
    if (!(p->max_range > 0.0f)) return api_fail(MEM_E_ARG, "max_range must be positive");
    if (!std::isfinite(p->clear_margin) || p->clear_min_count < 0) return api_fail(MEM_E_ARG, "bad clearing parameters");
    if (p->max_points < 0 || p->max_points >= ((int64_t)1 << 31)) return api_fail(MEM_E_ARG, "max_points must be 0 .. 2^31-1");
    if (p->n_layers < 0 || p->n_layers > 32 || (p->n_layers > 0 && !p->layers))
        return api_fail(MEM_E_ARG, "n_layers must be 0..32 with a layer array");
    for (int l = 0; l < p->n_layers; l++) {
        const mem_layer_desc& d = p->layers[l];
        if (d.channels < 1 || d.channels > 4096 || d.rule < MEM_LATEST || d.rule > MEM_DIRICHLET ||
            (d.storage != MEM_F32 && d.storage != MEM_BF16 && d.storage != MEM_FP8_E4M3) ||
            (d.rule == MEM_DIRICHLET && d.storage != MEM_F32) ||
            (d.rule == MEM_EXPAVG && !(d.param > 0.0f && d.param <= 1.0f)) ||
            ((d.rule == MEM_GAUSS || d.rule == MEM_DIRICHLET) && !(d.param > 0.0f && std::isfinite(d.param))))
            return api_fail(MEM_E_ARG, "layer %d: invalid descriptor", l);
    }
    const bool cams = p->cam_h > 0;
    if (cams) {
        if (p->cam_w < 1 || p->cam_c < 1 || (int64_t)p->cam_h * p->cam_w > (1ll << 30) ||
            (p->cam_dtype != MEM_F32 && p->cam_dtype != MEM_U8))
            return api_fail(MEM_E_ARG, "bad camera image size or dtype");
        if (p->n_img_bind < 0 || p->n_img_bind > 4 || (p->n_img_bind > 0 && !p->img_bind))
            return api_fail(MEM_E_ARG, "n_img_bind must be 0..4 with a binding array");
        for (int k = 0; k < p->n_img_bind; k++) {
            const mem_binding& bd = p->img_bind[k];
            const int l = bd.layer - MEM_LAYER_USER0;
            if (l < 0 || l >= p->n_layers || bd.ch_first < 0 || bd.topk < 0 || bd.topk > kMaxTopk)
                return api_fail(MEM_E_ARG, "image binding %d does not fit", k);
            // dense: the layer's C channels; top-k: 2k inputs into a
            // Dirichlet layer of at least k classes
            const int want = bd.topk > 0 ? 2 * bd.topk : p->layers[l].channels;
            if (bd.topk > 0 && (p->layers[l].rule != MEM_DIRICHLET || bd.topk > p->layers[l].channels))
                return api_fail(MEM_E_ARG, "image binding %d: top-k needs a Dirichlet layer of >= k classes", k);
            if (bd.ch_count != want || (int64_t)bd.ch_first + bd.ch_count > p->cam_c)
                return api_fail(MEM_E_ARG, "image binding %d does not fit", k);
        }
    }

    hipStream_t s = (hipStream_t)stream;
    mem_batch* b = new mem_batch;
    b->n = p->n_maps;
    b->W.assign(p->width, p->width + p->n_maps);
    b->H.assign(p->height, p->height + p->n_maps);
    b->total = total;
    b->res = p->resolution;
    b->inv_res = (float)(1.0 / (double)p->resolution);
    b->c0 = p->noise_c0;
    b->c1 = p->noise_c1;
    b->mr2 = p->max_range * p->max_range;
    b->margin = p->clear_margin;
    b->clear_min = p->clear_min_count;
    b->min_depth = p->min_depth;
    b->max_points = p->max_points;
    if (cams) {
        b->cam_h = p->cam_h;
        b->cam_w = p->cam_w;
        b->cam_c = p->cam_c;
        b->cam_dtype = p->cam_dtype;
        b->img_bind.assign(p->img_bind, p->img_bind + p->n_img_bind);
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipDeviceGetAttribute(&b->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    (void)hipGetLastError();
    if (b->n_cu < 1) b->n_cu = 1;
    b->bl = BatchLaunch{1024, 4 * b->n_cu, 16};
    int64_t off = 0;
    for (int m = 0; m < b->n; m++) {
        b->cell_off.push_back(off);
        off += (int64_t)b->W[m] * b->H[m];
        b->grid.push_back(initial_grid(b, m));
    }

    // arena: per-cell state of every map
    size_t a = 0;
    auto take = [&](size_t bytes) { size_t o = a; a = align256(a + bytes); return o; };
    const size_t o_h = take(4 * total), o_v = take(4 * total), o_cnt = take(4 * total), o_clr = take(4 * total),
                 o_w = take(4 * total), o_s = take(4 * total), o_st = take(8 * total), o_hl = take(4 * total);
    std::vector<size_t> o_val, o_var;
    for (int l = 0; l < p->n_layers; l++) {
        const mem_layer_desc& d = p->layers[l];
        const int esz = d.storage == MEM_BF16 ? 2 : d.storage == MEM_FP8_E4M3 ? 1 : 4;
        o_val.push_back(take((size_t)total * d.channels * esz));
        o_var.push_back(d.rule == MEM_GAUSS ? take(4 * total) : 0);
    }
    b->arena_bytes = a;
    hipError_t e = hipMalloc((void**)&b->arena, a);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_batch(b);
        return api_fail(MEM_E_NOMEM, "batch state of %zu bytes: %s", a, hipGetErrorString(e));
    }
    b->h = (float*)(b->arena + o_h);
    b->v = (float*)(b->arena + o_v);
    b->cnt = (int*)(b->arena + o_cnt);
    b->clr = (int*)(b->arena + o_clr);
    b->wsum = (float*)(b->arena + o_w);
    b->ssum = (float*)(b->arena + o_s);
    b->stash = (float2*)(b->arena + o_st);
    b->hl = (float*)(b->arena + o_hl);
    for (int l = 0; l < p->n_layers; l++) {
        const mem_layer_desc& d = p->layers[l];
        BLayer L;
        L.C = d.channels;
        L.rule = d.rule;
        L.storage = d.storage;
        L.param = d.param;
        L.val = b->arena + o_val[l];
        L.var = d.rule == MEM_GAUSS ? (float*)(b->arena + o_var[l]) : nullptr;
        b->layers.push_back(L);
    }

    // scratch, tables, staging
    b->off_maps = 256;
    b->off_rects = align256(b->off_maps + sizeof(BatchMap) * b->n);
    b->off_chunks = align256(b->off_rects + sizeof(BatchRect) * 2 * b->n);
    b->tables_bytes = align256(b->off_chunks + sizeof(int) * (b->n + 1));
    std::vector<BatchItem> gi;
    for (int m = 0; m < b->n; m++)
        for (int64_t q = 0; q < (int64_t)b->W[m] * b->H[m]; q += kGatherItem) gi.push_back(BatchItem{m, (int)q, 0, 0});
    b->n_gitems = (int)gi.size();
    bool ok = hipMalloc((void**)&b->pairs, sizeof(int2) * (size_t)total) == hipSuccess &&
              hipMalloc((void**)&b->pair_count, sizeof(int) * b->n) == hipSuccess &&
              hipMalloc((void**)&b->qctr, sizeof(int) * kQueues) == hipSuccess &&
              hipMalloc((void**)&b->stats, sizeof(unsigned long long) * kStats * kStatSlots) == hipSuccess &&
              hipMalloc((void**)&b->tables, b->tables_bytes) == hipSuccess &&
              hipMalloc((void**)&b->gitems, sizeof(BatchItem) * gi.size()) == hipSuccess;
    for (auto& st : b->stg)
        ok = ok && hipHostMalloc((void**)&st.host, b->tables_bytes, hipHostMallocDefault) == hipSuccess &&
             hipEventCreateWithFlags(&st.done, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_batch(b);
        return api_fail(MEM_E_NOMEM, "batch scratch allocation failed");
    }
    for (auto& st : b->stg) memset(st.host, 0, b->tables_bytes);
    for (int l = 0; l < p->n_layers; l++) {
        const mem_layer_desc& d = p->layers[l];
        std::vector<float> sc(d.channels, 1.0f / 448.0f);
        if (d.ch_scale)
            for (int q = 0; q < d.channels; q++) sc[q] = d.ch_scale[q] / 448.0f;
        const std::vector<float> blk = scale_block_host(sc, &b->layers[l].rcp);
        if (hipMalloc((void**)&b->layers[l].scale, sizeof(float) * blk.size()) != hipSuccess ||
            hipMemcpy(b->layers[l].scale, blk.data(), sizeof(float) * blk.size(), hipMemcpyHostToDevice) != hipSuccess) {
            free_batch(b);
            return api_fail(MEM_E_NOMEM, "layer scales");
        }
    }
    if (hipMemcpy(b->gitems, gi.data(), sizeof(BatchItem) * gi.size(), hipMemcpyHostToDevice) != hipSuccess ||
        build_tiles(b, 16) != MEM_OK || build_itiles(b) != MEM_OK) {
        free_batch(b);
        return api_fail(MEM_E_HIP, "batch tables");
    }
    // every map starts empty
    std::vector<LayerDev> L;
    for (auto& l : b->layers) L.push_back(l.dev());
    for (int m = 0; m < b->n; m++) {
        const int64_t o = b->cell_off[m];
        std::vector<LayerDev> Lm;
        for (auto& l : b->layers) Lm.push_back(l.dev(o));
        launch_reset_rect(s, b->grid[m], 0, b->W[m], 0, b->H[m], b->h + o, b->v + o, b->cnt + o, b->clr + o,
                          Lm.data(), (int)Lm.size());
    }
    launch_zero_int(s, (int*)b->stats, 2 * kStats * kStatSlots);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        free_batch(b);
        return api_fail(MEM_E_HIP, "initialising the batch: %s", hipGetErrorString(e));
    }
    *out = b;
    return MEM_OK;
}

mem_status mem_batch_destroy(mem_batch* b, void* stream)
{
    if (!b) return MEM_OK;
    (void)hipStreamSynchronize((hipStream_t)stream);
    (void)hipDeviceSynchronize();
    free_batch(b);
    return MEM_OK;
}

mem_status mem_batch_step(mem_batch* b, const mem_batch_input* in, void* stream)
{
    if (mem_status st = busable(b)) return st;
    if (!in) return api_fail(MEM_E_ARG, "input is NULL");
    return run_step(b, in, (hipStream_t)stream);
}

mem_status mem_batch_set_tuning(mem_batch* b, const mem_batch_tuning* t)
{
    if (mem_status st = busable(b)) return st;
    if (!t) return api_fail(MEM_E_ARG, "tuning is NULL");
    if (t->chunk != 512 && t->chunk != 1024 && t->chunk != 2048)
        return api_fail(MEM_E_ARG, "chunk must be 512, 1024 or 2048");
    if (t->wg_per_cu < 1 || t->wg_per_cu > 16) return api_fail(MEM_E_ARG, "wg_per_cu must be 1..16");
    if (t->tile != 8 && t->tile != 16) return api_fail(MEM_E_ARG, "tile must be 8 or 16");
    (void)hipDeviceSynchronize();
    if (t->tile != b->tiles_side)
        if (mem_status st = build_tiles(b, t->tile)) return st;
    b->bl = BatchLaunch{t->chunk, t->wg_per_cu * b->n_cu, t->tile};
    b->use_graph = t->graph != 0;
    drop_graphs(b);
    return MEM_OK;
}

mem_status mem_batch_get_tuning(const mem_batch* b, mem_batch_tuning* out)
{
    if (!b || !out) return api_fail(MEM_E_ARG, "NULL argument");
    out->chunk = b->bl.chunk;
    out->wg_per_cu = b->bl.grid / b->n_cu;
    out->tile = b->bl.tile;
    out->graph = b->use_graph ? 1 : 0;
    out->step_ms = b->tuned_ms;
    return MEM_OK;
}

mem_status mem_batch_tune(mem_batch* b, const mem_batch_input* in, void* stream)
{
    if (mem_status st = busable(b)) return st;
    if (!in) return api_fail(MEM_E_ARG, "input is NULL");
    hipStream_t s = (hipStream_t)stream;
    // Snapshot every map (state arena and grids) so the trial steps leave no trace.
    char* backup = nullptr;
    if (hipMalloc((void**)&backup, b->arena_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return api_fail(MEM_E_NOMEM, "tuning needs a %zu-byte snapshot", b->arena_bytes);
    }
    BTRY(b, hipStreamSynchronize(s));
    BTRY(b, hipMemcpyAsync(backup, b->arena, b->arena_bytes, hipMemcpyDeviceToDevice, s));
    const std::vector<Grid> grid0 = b->grid;
    const BatchLaunch bl0 = b->bl;
    const bool graph0 = b->use_graph;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    double best = 1e30;
    mem_batch_tuning best_t{bl0.chunk, bl0.grid / b->n_cu, bl0.tile, 1, 0.0};
    mem_status err = MEM_OK;
    const int chunks[3] = {512, 1024, 2048}, wgs[3] = {2, 4, 8}, tiles[2] = {8, 16};
    for (int ci = 0; ci < 3 && !err; ci++)
        for (int wi = 0; wi < 3 && !err; wi++)
            for (int ti = 0; ti < 2 && !err; ti++) {
                mem_batch_tuning t{chunks[ci], wgs[wi], tiles[ti], 1, 0.0};
                if ((err = mem_batch_set_tuning(b, &t))) break;
                // warm-up step builds the graph, then 3 timed steps
                if ((err = run_step(b, in, s))) break;
                (void)hipEventRecord(e0, s);
                for (int k = 0; k < 3 && !err; k++) err = run_step(b, in, s);
                (void)hipEventRecord(e1, s);
                (void)hipEventSynchronize(e1);
                float ms = 0;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (ms / 3 < best) {
                    best = ms / 3;
                    best_t = t;
                }
                (void)hipMemcpyAsync(b->arena, backup, b->arena_bytes, hipMemcpyDeviceToDevice, s);
                b->grid = grid0;
            }
    (void)hipStreamSynchronize(s);
    (void)hipFree(backup);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err) return err;
    best_t.graph = graph0 ? 1 : 0;
    if (mem_status st = mem_batch_set_tuning(b, &best_t)) return st;
    b->tuned_ms = best;
    return MEM_OK;
}

mem_status mem_batch_get_center(const mem_batch* b, int32_t map, int32_t* cx, int32_t* cy)
{
    if (!b || !cx || !cy || map < 0 || map >= b->n) return api_fail(MEM_E_ARG, "bad batch, map or output");
    *cx = b->grid[map].ox + b->grid[map].W / 2;
    *cy = b->grid[map].oy + b->grid[map].H / 2;
    return MEM_OK;
}

mem_status mem_batch_get_layer(const mem_batch* bc, int32_t map, int32_t layer, int32_t view, float* out,
                               void* stream)
{
    mem_batch* b = const_cast<mem_batch*>(bc);
    if (mem_status st = busable(b)) return st;
    if (map < 0 || map >= b->n || !out) return api_fail(MEM_E_ARG, "bad map or output");
    LayerDev d{};
    const int64_t o = b->cell_off[map];
    if (layer >= 0 && layer <= MEM_LAYER_CLEAR) {
        if (view != MEM_VIEW_VALUE) return api_fail(MEM_E_ARG, "built-in layers have only the value view");
    } else {
        const int l = layer - MEM_LAYER_USER0;
        if (l < 0 || l >= (int)b->layers.size()) return api_fail(MEM_E_ARG, "no user layer %d", layer);
        const BLayer& L = b->layers[l];
        const bool ok = view == MEM_VIEW_VALUE || (view == MEM_VIEW_AUX && (L.rule == MEM_GAUSS || L.rule == MEM_DIRICHLET)) ||
                        (view == MEM_VIEW_ARGMAX && L.rule == MEM_DIRICHLET);
        if (!ok) return api_fail(MEM_E_ARG, "layer %d has no view %d", layer, view);
        d = L.dev(o);
    }
    launch_readout((hipStream_t)stream, b->grid[map], layer, view, b->h + o, b->v + o, b->cnt + o, b->clr + o,
                   layer >= MEM_LAYER_USER0 ? &d : nullptr, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bfail(b, e, "mem_batch_get_layer");
    return MEM_OK;
}

mem_status mem_batch_set_layer(mem_batch* b, int32_t map, int32_t layer, int32_t view, const float* in,
                               void* stream)
{
    if (mem_status st = busable(b)) return st;
    if (map < 0 || map >= b->n || !in) return api_fail(MEM_E_ARG, "bad map or input");
    LayerDev d{};
    const int64_t o = b->cell_off[map];
    if (layer == MEM_LAYER_ELEVATION || layer == MEM_LAYER_VARIANCE) {
        if (view != MEM_VIEW_VALUE) return api_fail(MEM_E_ARG, "built-in layers have only the value view");
    } else {
        const int l = layer - MEM_LAYER_USER0;
        if (l < 0 || l >= (int)b->layers.size()) return api_fail(MEM_E_ARG, "layer %d is not settable", layer);
        const BLayer& L = b->layers[l];
        const bool ok = (view == MEM_VIEW_VALUE && L.rule != MEM_DIRICHLET) ||
                        (view == MEM_VIEW_AUX && (L.rule == MEM_GAUSS || L.rule == MEM_DIRICHLET));
        if (!ok) return api_fail(MEM_E_ARG, "view %d of layer %d is not settable", view, layer);
        d = L.dev(o);
    }
    launch_setlayer((hipStream_t)stream, b->grid[map], layer, view, b->h + o, b->v + o,
                    layer >= MEM_LAYER_USER0 ? &d : nullptr, in);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bfail(b, e, "mem_batch_set_layer");
    return MEM_OK;
}

mem_status mem_batch_get_stats(mem_batch* b, mem_stats* out, void* stream)
{
    if (mem_status st = busable(b)) return st;
    if (!out) return api_fail(MEM_E_ARG, "out is NULL");
    std::vector<unsigned long long> buf(kStats * kStatSlots);
    BTRY(b, hipMemcpyAsync(buf.data(), b->stats, sizeof(unsigned long long) * buf.size(), hipMemcpyDeviceToHost,
                           (hipStream_t)stream));
    BTRY(b, hipStreamSynchronize((hipStream_t)stream));
    int64_t* o = (int64_t*)out;
    for (int k = 0; k < kStats; k++) {
        o[k] = 0;
        for (int j = 0; j < kStatSlots; j++) o[k] += (int64_t)buf[k * kStatSlots + j];
    }
    return MEM_OK;
}

mem_status mem_batch_reset_stats(mem_batch* b, void* stream)
{
    if (mem_status st = busable(b)) return st;
    launch_zero_int((hipStream_t)stream, (int*)b->stats, 2 * kStats * kStatSlots);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bfail(b, e, "mem_batch_reset_stats");
    return MEM_OK;
}

mem_status mem_batch_profile_enable(mem_batch* b, int32_t on)
{
    if (mem_status st = busable(b)) return st;
    b->prof.enable(on != 0);
    return MEM_OK;
}

mem_status mem_batch_profile_read(mem_batch* b, mem_kernel_time* out, int32_t max, int32_t* count)
{
    if (mem_status st = busable(b)) return st;
    if (!count || (max > 0 && !out)) return api_fail(MEM_E_ARG, "NULL output");
    *count = b->prof.read(out, max);
    return MEM_OK;
}

}  // extern "C"
