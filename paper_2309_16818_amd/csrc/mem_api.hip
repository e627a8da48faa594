// mem_api.hip - host side of the C ABI declared in include/mem.h.
//
// Every entry point validates its arguments before it enqueues anything,
// then enqueues kernels on the caller's stream and returns without waiting.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "mem_internal.h"
#include "prof.h"

using namespace memk;

namespace {

thread_local std::string g_err;

mem_status fail(mem_status code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

}  // namespace

namespace memk {
// Error reporting shared with the batch entry points (batch_api.hip).
mem_status api_fail(mem_status code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
}  // namespace memk

namespace {

struct Layer {
    int C, rule, storage;
    float param;
    void* val = nullptr;
    float* var = nullptr;
    float* scale = nullptr;
    bool rcp = false;  // the scales allow the reciprocal divide
    LayerDev dev() const
    {
        LayerDev d;
        d.val = val;
        d.var = var;
        d.scale = scale;
        d.rscale = rcp ? scale_block_rcp(scale, C) : nullptr;
        d.C = C;
        d.rule = rule;
        d.storage = storage;
        d.param = param;
        return d;
    }
};


size_t elem_size(int storage)
{
    return storage == MEM_BF16 ? 2 : storage == MEM_FP8_E4M3 ? 1 : 4;
}

}  // namespace

// Sums, counts and ray lists of one more cloud of a mem_input_pointclouds
// call (the map's own serve its first cloud); zero between calls.
struct CloudSet {
    int* cnt = nullptr;
    int* clr = nullptr;
    float* wsum = nullptr;
    float* ssum = nullptr;
    float2* stash = nullptr;
    MarchBufs march;
};

struct mem_map {
    int W = 0, H = 0;
    float res = 0, inv_res = 0;
    float c0 = 0, c1 = 0, max_range = 0, mr2 = 0, clear_margin = 0, min_depth = 0;
    int clear_min = 0;
    int gather_v1 = 0;  // image gathers forced to one channel per lane (tests)
    int cx = 0, cy = 0, rx = 0, ry = 0;
    int device = 0;
    int max_lds = 65536;  // LDS bytes a workgroup may use on this device
    bool broken = false;

    float* h = nullptr;
    float* v = nullptr;
    int* cnt = nullptr;         // per-cloud accumulators: points per cell,
    int* clr = nullptr;         // clearing votes
    int* cnt_last = nullptr;    // the last cloud's (read out as hits and clears; swapped with cnt, clr
    int* clr_last = nullptr;    // at every cloud's end)
    float* wsum = nullptr;
    float* ssum = nullptr;
    float2* stash = nullptr;
    int4* vlist_poses = nullptr; // lists, codes and counters of several poses (first use)
    int* vcode_poses = nullptr;
    int* vcount_poses = nullptr;
    int* vcount = nullptr;      // cells listed in vlist: two counters used by turns (vpar)
    int vpar = 0;               // the counter the next projection uses; its k_view clears the other
    bool tmax_stale = true;     // the heights changed since the block maxima were built
    bool acc_clean = false;     // accumulators and march counts are zero (the last cloud's finalize cleared them)
    bool hl_fresh = false;      // hl holds the heights in logical order
    MarchBufs march;            // clearing march: rays and segment lists (grown on first use)
    std::vector<CloudSet> csets; // further per-cloud sums and lists of mem_input_pointclouds (first use)
    float* hl = nullptr;        // heights in logical order, for the clearing march
    DriftDev* drift = nullptr;  // the last cloud's drift compensation
    char* drift_part = nullptr; // its per-workgroup partial sums
    bool drift_on = false;
    float drift_kappa2 = 0.0f;  // binary32 kappa * kappa
    int drift_min = 0;
    void* pca_scratch = nullptr; // partial sums of the PCA layer (allocated on first use)
    PcaOut* pca_out = nullptr;
    char* pcw_scratch = nullptr;   // the same for more than kPcaMaxC channels (first use)
    PcaWideOut* pcw_out = nullptr;
    bool overlap_on = false;    // overlap clearance after each point cloud
    float overlap_xy = 0.0f, overlap_z = 0.0f;
    int4* vlist = nullptr;      // cells inside a camera's view
    float* tmax = nullptr;      // block maxima of h: side 8, then side 64
    int* vcode = nullptr;       // their pixel per image
    unsigned long long* stats = nullptr;
    float* chsum = nullptr;
    int chsum_planes = 0;
    std::vector<Layer> layers;

    Profiler prof;

    // Block maxima of the heights for the exact skipping of ray walks.
    int64_t tmax_size() const
    {
        const int64_t n8 = (int64_t)((W + 7) / 8) * ((H + 7) / 8);
        return n8 + (int64_t)((W + 63) / 64) * ((H + 63) / 64);
    }
    // Block maxima of the current heights, rebuilt only when a call changed
    // the heights (or the ring offsets) since they were last built.
    TileMax tiles(hipStream_t s)
    {
        const Grid g = grid();
        const int64_t n8 = (int64_t)((W + 7) / 8) * ((H + 7) / 8);
        if (tmax_stale) {
            launch_tile_max(s, g, h, tmax, tmax + n8);
            tmax_stale = false;
        }
        return tile_max_dims(g, tmax, tmax + n8);
    }

    // The projection counter for this call; the call's k_view clears the
    // other one for the next call (calls on a map are stream ordered).
    int* take_vcount()
    {
        int* c = vcount + vpar;
        vpar ^= 1;
        return c;
    }

    Grid grid() const
    {
        Grid g;
        g.W = W;
        g.H = H;
        g.ox = cx - W / 2;
        g.oy = cy - H / 2;
        g.rx = rx;
        g.ry = ry;
        g.res = res;
        g.inv_res = inv_res;
        return g;
    }
    int64_t cells() const { return (int64_t)W * H; }
};

namespace {

mem_status hip_fail(mem_map* m, hipError_t e, const char* what)
{
    if (m) m->broken = true;
    return fail(MEM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(m, call)                                          \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return hip_fail((m), e_, #call);    \
    } while (0)

mem_status check_launch(mem_map* m, const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(m, e, what);
    return MEM_OK;
}

// Runs a launcher, bracketed by events on `s` while profiling is on.
template <class F>
void timed(mem_map* m, hipStream_t s, const char* name, F&& f)
{
    m->prof.timed(s, name, f);
}

// Runs a launcher that takes LaunchEv (events recorded by its kernels' own
// dispatch) while profiling is on.
template <class F>
void timed_ext(mem_map* m, hipStream_t s, const char* name, F&& f)
{
    m->prof.timed_ext(s, name, f);
}

mem_status usable(const mem_map* m)
{
    if (!m) return fail(MEM_E_ARG, "map is NULL");
    if (m->broken) return fail(MEM_E_STATE, "map is unusable after an earlier HIP error");
    return MEM_OK;
}

// Finite pose with an orthonormal rotation and a translation whose lattice
// coordinates stay far inside int32.
mem_status check_pose(const mem_map* m, const float* T, const char* what)
{
    if (!T) return fail(MEM_E_ARG, "%s is NULL", what);
    for (int k = 0; k < 12; k++)
        if (!std::isfinite(T[k])) return fail(MEM_E_ARG, "%s has a non-finite entry", what);
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double d = 0;
            for (int k = 0; k < 3; k++) d += (double)T[4 * a + k] * T[4 * b + k];
            if (std::fabs(d - (a == b ? 1.0 : 0.0)) > 1e-4)
                return fail(MEM_E_ARG, "%s rotation is not orthonormal", what);
        }
    const double lim = 4194304.0;  // 2^22 cells
    if (std::fabs((double)T[3] * m->inv_res) > lim || std::fabs((double)T[7] * m->inv_res) > lim)
        return fail(MEM_E_ARG, "%s translation is too far from the origin", what);
    // Rays start at the sensor: keep it within a few grid widths of the grid
    // so that every ray walk is short.
    const double reach = 4.0 * (m->W > m->H ? m->W : m->H) + 2.0;
    if (std::fabs(std::floor((double)(T[3] * m->inv_res)) - m->cx) > reach ||
        std::fabs(std::floor((double)(T[7] * m->inv_res)) - m->cy) > reach)
        return fail(MEM_E_ARG, "%s lies more than 4 grid widths from the grid", what);
    return MEM_OK;
}

mem_status resolve_layer(const mem_map* m, int layer, const Layer** out)
{
    int l = layer - MEM_LAYER_USER0;
    if (l < 0 || l >= (int)m->layers.size()) return fail(MEM_E_ARG, "no user layer %d", layer);
    *out = &m->layers[l];
    return MEM_OK;
}

template <class T>
mem_status dev_alloc(mem_map* m, T** p, size_t count)
{
    hipError_t e = hipMalloc((void**)p, sizeof(T) * (count ? count : 1));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(MEM_E_NOMEM, "hipMalloc of %zu bytes failed: %s", sizeof(T) * count,
                    hipGetErrorString(e));
    }
    (void)m;
    return MEM_OK;
}

void free_map(mem_map* m)
{
    (void)hipFree(m->h);
    (void)hipFree(m->v);
    (void)hipFree(m->cnt);
    (void)hipFree(m->clr);
    (void)hipFree(m->cnt_last);
    (void)hipFree(m->clr_last);
    (void)hipFree(m->wsum);
    (void)hipFree(m->ssum);
    (void)hipFree(m->stash);
    (void)hipFree(m->vcount);
    (void)hipFree(m->march.rec);
    (void)hipFree(m->march.full);
    (void)hipFree(m->march.part);
    (void)hipFree(m->march.counts);
    for (CloudSet& c : m->csets) {
        (void)hipFree(c.cnt);
        (void)hipFree(c.clr);
        (void)hipFree(c.wsum);
        (void)hipFree(c.ssum);
        (void)hipFree(c.stash);
        (void)hipFree(c.march.rec);
        (void)hipFree(c.march.full);
        (void)hipFree(c.march.part);
        (void)hipFree(c.march.counts);
    }
    (void)hipFree(m->hl);
    (void)hipFree(m->drift);
    (void)hipFree(m->drift_part);
    (void)hipFree(m->vlist_poses);
    (void)hipFree(m->vcode_poses);
    (void)hipFree(m->vcount_poses);
    (void)hipFree(m->pca_scratch);
    (void)hipFree(m->pca_out);
    (void)hipFree(m->pcw_scratch);
    (void)hipFree(m->pcw_out);
    (void)hipFree(m->vlist);
    (void)hipFree(m->vcode);
    (void)hipFree(m->tmax);
    (void)hipFree(m->stats);
    (void)hipFree(m->chsum);
    for (auto& L : m->layers) {
        (void)hipFree(L.val);
        (void)hipFree(L.var);
        (void)hipFree(L.scale);
    }
    m->prof.release();
    delete m;
}

std::vector<LayerDev> layer_devs(const mem_map* m)
{
    std::vector<LayerDev> d;
    for (auto& L : m->layers) d.push_back(L.dev());
    return d;
}

}  // namespace

extern "C" {

const char* mem_last_error(void)
{
    return g_err.c_str();
}

mem_status mem_create(const mem_params* p, void* stream, mem_map** out)
{
    if (!p || !out) return fail(MEM_E_ARG, "params and out must not be NULL");
    *out = nullptr;
    if (p->width < 1 || p->width > 16384 || p->height < 1 || p->height > 16384)
        return fail(MEM_E_ARG, "grid %dx%d outside 1..16384", p->width, p->height);
    if (!(p->resolution > 0.0f) || !std::isfinite(p->resolution))
        return fail(MEM_E_ARG, "resolution must be positive");
    if (!std::isfinite(p->noise_c0) || !std::isfinite(p->noise_c1) || p->noise_c0 < 0 || p->noise_c1 < 0 ||
        (p->noise_c0 == 0 && p->noise_c1 == 0))
        return fail(MEM_E_ARG, "noise model needs c0, c1 >= 0, not both zero");
    if (!(p->max_range > 0.0f)) return fail(MEM_E_ARG, "max_range must be positive");
    if (!std::isfinite(p->clear_margin) || p->clear_min_count < 0)
        return fail(MEM_E_ARG, "bad clearing parameters");
    if (!std::isfinite(p->min_depth)) return fail(MEM_E_ARG, "min_depth must be finite");
    if (p->n_layers < 0 || p->n_layers > 32 || (p->n_layers > 0 && !p->layers))
        return fail(MEM_E_ARG, "n_layers must be 0..32 with a layer array");
    for (int l = 0; l < p->n_layers; l++) {
        const mem_layer_desc& d = p->layers[l];
        if (d.channels < 1 || d.channels > 4096) return fail(MEM_E_ARG, "layer %d: channels", l);
        if (d.rule < MEM_LATEST || d.rule > MEM_DIRICHLET) return fail(MEM_E_ARG, "layer %d: rule", l);
        if (d.storage != MEM_F32 && d.storage != MEM_BF16 && d.storage != MEM_FP8_E4M3)
            return fail(MEM_E_ARG, "layer %d: storage", l);
        if (d.rule == MEM_DIRICHLET && d.storage != MEM_F32)
            return fail(MEM_E_ARG, "layer %d: Dirichlet layers are stored in f32", l);
        if (d.rule == MEM_EXPAVG && !(d.param > 0.0f && d.param <= 1.0f))
            return fail(MEM_E_ARG, "layer %d: exponential averaging weight must be in (0, 1]", l);
        if ((d.rule == MEM_GAUSS || d.rule == MEM_DIRICHLET) && !(d.param > 0.0f && std::isfinite(d.param)))
            return fail(MEM_E_ARG, "layer %d: parameter must be positive", l);
        if (d.ch_scale)
            for (int q = 0; q < d.channels; q++)
                if (!(d.ch_scale[q] > 0.0f) || !std::isfinite(d.ch_scale[q]))
                    return fail(MEM_E_ARG, "layer %d: ch_scale must be positive", l);
    }

    hipStream_t s = (hipStream_t)stream;
    mem_map* m = new mem_map;
    m->W = p->width;
    m->H = p->height;
    m->res = p->resolution;
    m->inv_res = (float)(1.0 / (double)p->resolution);
    m->c0 = p->noise_c0;
    m->c1 = p->noise_c1;
    m->max_range = p->max_range;
    m->mr2 = p->max_range * p->max_range;
    m->clear_margin = p->clear_margin;
    m->clear_min = p->clear_min_count;
    m->min_depth = p->min_depth;
    (void)hipGetDevice(&m->device);
    {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, m->device) == hipSuccess && v > 0)
            m->max_lds = v;
        (void)hipGetLastError();
    }
    const int64_t HW = m->cells();
    mem_status st = MEM_OK;
    if ((st = dev_alloc(m, &m->h, HW)) || (st = dev_alloc(m, &m->v, HW)) ||
        (st = dev_alloc(m, &m->cnt, HW)) || (st = dev_alloc(m, &m->clr, HW)) ||
        (st = dev_alloc(m, &m->cnt_last, HW)) || (st = dev_alloc(m, &m->clr_last, HW)) ||
        (st = dev_alloc(m, &m->wsum, HW)) || (st = dev_alloc(m, &m->ssum, HW)) ||
        (st = dev_alloc(m, &m->stash, HW)) ||
        (st = dev_alloc(m, &m->vlist, HW)) || (st = dev_alloc(m, &m->vcode, HW * kMaxImages)) ||
        (st = dev_alloc(m, &m->vcount, 2)) || (st = dev_alloc(m, &m->tmax, m->tmax_size())) ||
        (st = dev_alloc(m, &m->march.counts, kSegLists * kSegSubs)) || (st = dev_alloc(m, &m->drift, 1)) || (st = dev_alloc(m, &m->drift_part, drift_part_bytes())) ||
        (st = dev_alloc(m, &m->hl, HW)) ||
        (st = dev_alloc(m, &m->stats, kStats * kStatSlots))) {
        free_map(m);
        return st;
    }
    for (int l = 0; l < p->n_layers; l++) {
        const mem_layer_desc& d = p->layers[l];
        Layer L;
        L.C = d.channels;
        L.rule = d.rule;
        L.storage = d.storage;
        L.param = d.param;
        m->layers.push_back(L);
        Layer& M = m->layers.back();
        if ((st = dev_alloc(m, (uint8_t**)&M.val, HW * d.channels * elem_size(d.storage))) ||
            (d.rule == MEM_GAUSS && (st = dev_alloc(m, &M.var, HW))) ||
            (st = dev_alloc(m, &M.scale, scale_block_floats(d.channels)))) {
            free_map(m);
            return st;
        }
        std::vector<float> sc(d.channels, 1.0f / 448.0f);
        if (d.ch_scale)
            for (int q = 0; q < d.channels; q++) sc[q] = d.ch_scale[q] / 448.0f;
        const std::vector<float> blk = scale_block_host(sc, &M.rcp);
        hipError_t e = hipMemcpy(M.scale, blk.data(), sizeof(float) * blk.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            free_map(m);
            return fail(MEM_E_HIP, "hipMemcpy: %s", hipGetErrorString(e));
        }
    }
    Grid g = m->grid();
    auto devs = layer_devs(m);
    launch_reset_rect(s, g, 0, m->W, 0, m->H, m->h, m->v, m->cnt_last, m->clr_last, devs.data(),
                      (int)devs.size());
    launch_zero_accum(s, g, m->cnt, m->wsum, m->ssum, m->clr, nullptr, 0, nullptr, nullptr, nullptr, m->drift);
    launch_zero_int(s, (int*)m->stats, 2 * kStats * kStatSlots);
    launch_zero_int(s, m->vcount, 2);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        free_map(m);
        return fail(MEM_E_HIP, "initialising the map: %s", hipGetErrorString(e));
    }
    *out = m;
    return MEM_OK;
}

mem_status mem_destroy(mem_map* m, void* stream)
{
    if (!m) return MEM_OK;
    (void)hipStreamSynchronize((hipStream_t)stream);
    free_map(m);
    return MEM_OK;
}

mem_status mem_get_center(const mem_map* m, int32_t* cx, int32_t* cy)
{
    if (!m || !cx || !cy) return fail(MEM_E_ARG, "NULL argument");
    *cx = m->cx;
    *cy = m->cy;
    return MEM_OK;
}

mem_status mem_move(mem_map* m, float x, float y, void* stream)
{
    if (mem_status st = usable(m)) return st;
    if (!std::isfinite(x) || !std::isfinite(y)) return fail(MEM_E_ARG, "position must be finite");
    const double lim = 4194304.0;
    if (std::fabs((double)x * m->inv_res) > lim || std::fabs((double)y * m->inv_res) > lim)
        return fail(MEM_E_ARG, "position is too far from the origin");
    hipStream_t s = (hipStream_t)stream;
    float gx = floorf(x * m->inv_res);
    float gy = floorf(y * m->inv_res);
    int ncx = (int)gx, ncy = (int)gy;
    int sx = ncx - m->cx, sy = ncy - m->cy;
    if (sx == 0 && sy == 0) return MEM_OK;
    m->tmax_stale = true;
    m->hl_fresh = false;
    m->cx = ncx;
    m->cy = ncy;
    auto devs = layer_devs(m);
    timed(m, s, "reset_rect", [&] {
        if (std::abs(sx) >= m->W || std::abs(sy) >= m->H) {
            m->rx = 0;
            m->ry = 0;
            launch_reset_rect(s, m->grid(), 0, m->W, 0, m->H, m->h, m->v, m->cnt_last, m->clr_last, devs.data(),
                              (int)devs.size());
            return;
        }
        m->rx = ((m->rx + sx) % m->W + m->W) % m->W;
        m->ry = ((m->ry + sy) % m->H + m->H) % m->H;
        Grid g = m->grid();
        if (sx > 0)
            launch_reset_rect(s, g, m->W - sx, m->W, 0, m->H, m->h, m->v, m->cnt_last, m->clr_last, devs.data(),
                              (int)devs.size());
        else if (sx < 0)
            launch_reset_rect(s, g, 0, -sx, 0, m->H, m->h, m->v, m->cnt_last, m->clr_last, devs.data(),
                              (int)devs.size());
        if (sy > 0)
            launch_reset_rect(s, g, 0, m->W, m->H - sy, m->H, m->h, m->v, m->cnt_last, m->clr_last, devs.data(),
                              (int)devs.size());
        else if (sy < 0)
            launch_reset_rect(s, g, 0, m->W, 0, -sy, m->h, m->v, m->cnt_last, m->clr_last, devs.data(),
                              (int)devs.size());
    });
    return check_launch(m, "mem_move");
}

// A binding's inputs fit `c` channels and match its layer: C dense channels,
// or 2k inputs (k class indices, then their probabilities) for a top-k class
// input into a Dirichlet layer of K >= k classes.
static mem_status check_binding(const mem_binding& bd, const Layer* L, int c, const char* what)
{
    if (bd.topk < 0 || bd.topk > kMaxTopk) return fail(MEM_E_ARG, "%s: topk must be 0..%d", what, kMaxTopk);
    if (bd.topk > 0) {
        if (L->rule != MEM_DIRICHLET) return fail(MEM_E_ARG, "%s: a top-k class input needs a Dirichlet layer", what);
        if (bd.topk > L->C) return fail(MEM_E_ARG, "%s: topk %d exceeds the layer's %d classes", what, bd.topk, L->C);
        if (bd.ch_count != 2 * bd.topk)
            return fail(MEM_E_ARG, "%s: a top-%d class input reads %d channels, not %d", what, bd.topk, 2 * bd.topk,
                        bd.ch_count);
    } else if (bd.ch_count != L->C) {
        return fail(MEM_E_ARG, "%s: %d channels for a layer of %d", what, bd.ch_count, L->C);
    }
    if (bd.ch_first < 0 || (int64_t)bd.ch_first + bd.ch_count > c)
        return fail(MEM_E_ARG, "%s: channels [%d, %lld) do not fit %d inputs", what, bd.ch_first,
                    (long long)bd.ch_first + bd.ch_count, c);
    return MEM_OK;
}

mem_status mem_input_pointcloud(mem_map* m, const float* xyz, int64_t n, const float* ch, int32_t c,
                                const mem_binding* bind, int32_t n_bind, const float T_map_sensor[12],
                                void* stream)
{
    if (mem_status st = usable(m)) return st;
    if (n < 0) return fail(MEM_E_ARG, "n must be >= 0");
    if (n > 0 && !xyz) return fail(MEM_E_ARG, "xyz is NULL");
    if (c < 0 || (c > 0 && n > 0 && !ch)) return fail(MEM_E_ARG, "channels given without data");
    if (n_bind < 0 || n_bind > kMaxBind || (n_bind > 0 && !bind))
        return fail(MEM_E_ARG, "n_bind must be 0..%d with a binding array", kMaxBind);
    if (mem_status st = check_pose(m, T_map_sensor, "T_map_sensor")) return st;
    PointBinds pb{};
    pb.n = n_bind;
    pb.c_in = c;
    for (int b = 0; b < n_bind; b++) {
        const Layer* L = nullptr;
        if (mem_status st = resolve_layer(m, bind[b].layer, &L)) return st;
        char what[32];
        snprintf(what, sizeof what, "binding %d", b);
        if (mem_status st = check_binding(bind[b], L, c, what)) return st;
        pb.b[b].layer = bind[b].layer - MEM_LAYER_USER0;
        pb.b[b].ch_first = bind[b].ch_first;
        pb.b[b].topk = bind[b].topk;
        pb.b[b].C = L->C;
        pb.b[b].sum_off = pb.Cb;
        pb.L[b] = L->dev();
        pb.Cb += L->C;
    }
    pb.lds_ch = (pb.Cb > 0 && ingest_lds_bytes(pb.Cb) <= (size_t)m->max_lds) ? 1 : 0;
    hipStream_t s = (hipStream_t)stream;
    if (pb.Cb > m->chsum_planes) {
        // Stream-ordered growth: wait for earlier users of the old buffer.
        HIP_TRY(m, hipStreamSynchronize(s));
        (void)hipFree(m->chsum);
        m->chsum = nullptr;
        m->chsum_planes = 0;
        m->acc_clean = false;
        if (mem_status st = dev_alloc(m, &m->chsum, (size_t)pb.Cb * m->cells())) return st;
        m->chsum_planes = pb.Cb;
    }
    Grid g = m->grid();
    const bool march = m->clear_min > 0 && n > 0;
    if (march) {
        int64_t pts = 0, fpr = 0;
        march_pass(m->mr2, m->res, n, &pts, &fpr);
        if (pts > m->march.cap_pts) {
            // Stream-ordered growth: wait for earlier users of the old buffers.
            HIP_TRY(m, hipStreamSynchronize(s));
            (void)hipFree(m->march.rec);
            (void)hipFree(m->march.full);
            (void)hipFree(m->march.part);
            m->march.rec = nullptr;
            m->march.full = nullptr;
            m->march.part = nullptr;
            m->march.cap_pts = 0;
            const MarchSizes z = march_sizes(pts, fpr);
            if (mem_status st = dev_alloc(m, &m->march.rec, pts)) return st;
            if (mem_status st = dev_alloc(m, &m->march.full, kSegSubs * z.full_sub)) return st;
            if (mem_status st = dev_alloc(m, &m->march.part, 4 * kSegSubs * z.part_sub)) return st;
            m->march.cap_pts = pts;
            m->march.full_sub = z.full_sub;
            m->march.part_sub = z.part_sub;
        }
    }
    // The clearing pass runs only where the last cloud's finalize left work:
    // dirty accumulators, or heights changed since hl was written.
    if (!m->acc_clean || (march && !m->hl_fresh)) {
        timed_ext(m, s, "zero_accum", [&](LaunchEv ev) {
            launch_zero_accum(s, g, m->cnt, m->wsum, m->ssum, m->clr, m->chsum, pb.Cb, m->march.counts, m->h,
                              march ? m->hl : nullptr, m->drift, ev);
        });
        if (march) m->hl_fresh = true;
    }
    m->acc_clean = false;
    const bool drift_runs = m->drift_on && n > 0;
    Pose T;
    memcpy(T.m, T_map_sensor, sizeof(T.m));
    // a cloud that fits one march pass has its rays listed by the ingest
    const bool fused = march && n <= m->march.cap_pts;
    if (n > 0)
        timed_ext(m, s, "ingest", [&](LaunchEv ev) {
            launch_ingest(s, g, xyz, n, ch, T, m->c0, m->c1, m->mr2, pb, m->cnt, m->wsum, m->ssum, m->stash,
                          m->chsum, fused ? &m->march : nullptr, m->stats, ev);
        });
    if (drift_runs)
        timed(m, s, "drift", [&] {
            launch_drift(s, g, xyz, n, T, m->c0, m->c1, m->mr2, m->h, m->v, m->drift_kappa2, m->drift_min,
                         m->drift, m->drift_part, march ? m->hl : nullptr);
        });
    if (march)
        timed_ext(m, s, "clear_march", [&](LaunchEv ev) {
            launch_clear_march(s, g, xyz, n, T, m->mr2, m->clear_margin, m->hl, m->clr, m->march, fused,
                               m->stats, ev);
        });
    m->tmax_stale = true;
    // finalize leaves the accumulators and counts zero, keeps hl equal to
    // the heights (when the march kept it so), and clears the drift record
    // of a cloud without drift compensation
    timed_ext(m, s, "finalize", [&](LaunchEv ev) {
        launch_finalize(s, g, m->cnt, m->wsum, m->ssum, m->stash, m->clr, m->clear_min, m->h, m->v,
                        m->chsum, pb, m->stats, true, m->cnt_last, m->clr_last, march ? m->hl : nullptr,
                        m->march.counts, drift_runs ? nullptr : m->drift, ev);
    });
    std::swap(m->cnt, m->cnt_last);
    std::swap(m->clr, m->clr_last);
    m->acc_clean = true;
    if (!march && n > 0) m->hl_fresh = false;
    if (m->overlap_on) {
        timed(m, s, "overlap_clear", [&] {
            launch_overlap_clear(s, g, T.m[3], T.m[7], T.m[11], m->overlap_xy, m->overlap_z, m->h);
        });
        m->hl_fresh = false;
    }
    return check_launch(m, "mem_input_pointcloud");
}

// Ray lists with room for passes of `pts` points (grown with a stream
// synchronisation, as the map's own); counts zeroed when (re)allocated.
static mem_status grow_march(mem_map* m, MarchBufs* mb, int64_t pts, int64_t fpr, hipStream_t s)
{
    if (!mb->counts) {
        if (mem_status st = dev_alloc(m, &mb->counts, kSegLists * kSegSubs)) return st;
        launch_zero_int(s, mb->counts, kSegLists * kSegSubs);
    }
    if (pts <= mb->cap_pts) return MEM_OK;
    HIP_TRY(m, hipStreamSynchronize(s));
    (void)hipFree(mb->rec);
    (void)hipFree(mb->full);
    (void)hipFree(mb->part);
    mb->rec = nullptr;
    mb->full = nullptr;
    mb->part = nullptr;
    mb->cap_pts = 0;
    const MarchSizes z = march_sizes(pts, fpr);
    if (mem_status st = dev_alloc(m, &mb->rec, pts)) return st;
    if (mem_status st = dev_alloc(m, &mb->full, kSegSubs * z.full_sub)) return st;
    if (mem_status st = dev_alloc(m, &mb->part, 4 * kSegSubs * z.part_sub)) return st;
    mb->cap_pts = pts;
    mb->full_sub = z.full_sub;
    mb->part_sub = z.part_sub;
    return MEM_OK;
}

static mem_status check_cloud(const mem_map* m, const mem_cloud& c, int k)
{
    if (c.n < 0) return fail(MEM_E_ARG, "cloud %d: n must be >= 0", k);
    if (c.n > 0 && !c.xyz) return fail(MEM_E_ARG, "cloud %d: xyz is NULL", k);
    if (c.c < 0 || (c.c > 0 && c.n > 0 && !c.ch)) return fail(MEM_E_ARG, "cloud %d: channels given without data", k);
    if (c.n_bind < 0 || c.n_bind > kMaxBind || (c.n_bind > 0 && !c.bind))
        return fail(MEM_E_ARG, "cloud %d: n_bind must be 0..%d with a binding array", k, kMaxBind);
    if (mem_status st = check_pose(m, c.T_map_sensor, "T_map_sensor")) return st;
    for (int b = 0; b < c.n_bind; b++) {
        const Layer* L = nullptr;
        if (mem_status st = resolve_layer(m, c.bind[b].layer, &L)) return st;
        char what[48];
        snprintf(what, sizeof what, "cloud %d binding %d", k, b);
        if (mem_status st = check_binding(c.bind[b], L, c.c, what)) return st;
    }
    return MEM_OK;
}

mem_status mem_input_pointclouds(mem_map* m, const mem_cloud* clouds, int32_t n_clouds, void* stream)
{
    if (mem_status st = usable(m)) return st;
    if (n_clouds < 1 || n_clouds > kMaxClouds || !clouds)
        return fail(MEM_E_ARG, "n_clouds must be 1..%d with a cloud array", kMaxClouds);
    for (int k = 0; k < n_clouds; k++)
        if (mem_status st = check_cloud(m, clouds[k], k)) return st;
    // the clouds' ingest in one launch where its conditions hold
    bool one_launch = n_clouds > 1 && m->clear_min > 0 && !m->drift_on && !m->overlap_on;
    int64_t pmax = 0, fpr = 0;
    for (int k = 0; k < n_clouds && one_launch; k++) {
        int64_t pts = 0;
        march_pass(m->mr2, m->res, clouds[k].n, &pts, &fpr);
        one_launch = clouds[k].n_bind == 0 && clouds[k].n > 0 && pts == clouds[k].n;
        pmax = std::max(pmax, pts);
    }
    if (!one_launch) {
        for (int k = 0; k < n_clouds; k++) {
            const mem_cloud& c = clouds[k];
            if (mem_status st = mem_input_pointcloud(m, c.xyz, c.n, c.ch, c.c, c.bind, c.n_bind, c.T_map_sensor,
                                                     stream))
                return st;
        }
        return MEM_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    const int K = n_clouds;
    const int64_t HW = m->cells();
    while ((int)m->csets.size() < K - 1) {
        CloudSet c;
        mem_status st = MEM_OK;
        (void)((st = dev_alloc(m, &c.cnt, HW)) || (st = dev_alloc(m, &c.clr, HW)) ||
               (st = dev_alloc(m, &c.wsum, HW)) || (st = dev_alloc(m, &c.ssum, HW)) ||
               (st = dev_alloc(m, &c.stash, HW)));
        if (st == MEM_OK) {
            launch_zero_int(s, c.cnt, (int)HW);
            launch_zero_int(s, c.clr, (int)HW);
            launch_zero_int(s, (int*)c.wsum, (int)HW);
            launch_zero_int(s, (int*)c.ssum, (int)HW);
            launch_zero_int(s, (int*)c.stash, (int)(2 * HW));
        }
        m->csets.push_back(c);  // freed with the map, also when incomplete
        if (st) return st;
    }
    if (mem_status st = grow_march(m, &m->march, pmax, fpr, s)) return st;
    for (int k = 0; k < K - 1; k++)
        if (mem_status st = grow_march(m, &m->csets[k].march, pmax, fpr, s)) return st;
    Grid g = m->grid();
    if (!m->acc_clean || !m->hl_fresh) {
        timed_ext(m, s, "zero_accum", [&](LaunchEv ev) {
            launch_zero_accum(s, g, m->cnt, m->wsum, m->ssum, m->clr, m->chsum, m->chsum_planes, m->march.counts,
                              m->h, m->hl, m->drift, ev);
        });
        m->hl_fresh = true;
    }
    m->acc_clean = false;
    // cloud k (1-based) counts into cnt[k], clr[k]; cnt[0], clr[0] hold the
    // last call's counts, zeroed by the first cloud's finalize, and each
    // finalize zeroes the counts of the cloud before it
    std::vector<int*> cnt(K + 1), clr(K + 1);
    cnt[0] = m->cnt_last;
    clr[0] = m->clr_last;
    cnt[1] = m->cnt;
    clr[1] = m->clr;
    for (int k = 2; k <= K; k++) {
        cnt[k] = m->csets[k - 2].cnt;
        clr[k] = m->csets[k - 2].clr;
    }
    auto march_of = [&](int k) -> MarchBufs& { return k == 1 ? m->march : m->csets[k - 2].march; };
    IngestClouds cl{};
    cl.n = K;
    for (int k = 1; k <= K; k++) {
        IngestCloud& c = cl.c[k - 1];
        c.xyz = clouds[k - 1].xyz;
        c.n = clouds[k - 1].n;
        memcpy(c.T.m, clouds[k - 1].T_map_sensor, sizeof(c.T.m));
        c.cnt = cnt[k];
        c.wsum = k == 1 ? m->wsum : m->csets[k - 2].wsum;
        c.ssum = k == 1 ? m->ssum : m->csets[k - 2].ssum;
        c.stash = k == 1 ? m->stash : m->csets[k - 2].stash;
        c.mb = march_of(k);
    }
    timed_ext(m, s, "ingest", [&](LaunchEv ev) { launch_ingest_clouds(s, g, cl, m->c0, m->c1, m->mr2, m->stats, ev); });
    const PointBinds pb{};
    for (int k = 1; k <= K; k++) {
        const IngestCloud& c = cl.c[k - 1];
        timed_ext(m, s, "clear_march", [&](LaunchEv ev) {
            launch_clear_march(s, g, c.xyz, c.n, c.T, m->mr2, m->clear_margin, m->hl, clr[k], c.mb, true, m->stats,
                               ev);
        });
        timed_ext(m, s, "finalize", [&](LaunchEv ev) {
            launch_finalize(s, g, cnt[k], c.wsum, c.ssum, c.stash, clr[k], m->clear_min, m->h, m->v, nullptr, pb,
                            m->stats, true, cnt[k - 1], clr[k - 1], m->hl, c.mb.counts, m->drift, ev);
        });
    }
    m->cnt = cnt[0];
    m->clr = clr[0];
    m->cnt_last = cnt[K];
    m->clr_last = clr[K];
    for (int k = 0; k < K - 1; k++) {
        m->csets[k].cnt = cnt[k + 1];
        m->csets[k].clr = clr[k + 1];
    }
    m->tmax_stale = true;
    m->acc_clean = true;
    return check_launch(m, "mem_input_pointclouds");
}

mem_status mem_set_drift_compensation(mem_map* m, int32_t enable, float kappa, int32_t min_points)
{
    if (mem_status st = usable(m)) return st;
    if (enable) {
        if (!(kappa > 0.0f) || !std::isfinite(kappa)) return fail(MEM_E_ARG, "kappa must be positive and finite");
        if (min_points < 1) return fail(MEM_E_ARG, "min_points must be >= 1");
    }
    m->drift_on = enable != 0;
    m->drift_kappa2 = kappa * kappa;
    m->drift_min = min_points;
    return MEM_OK;
}

mem_status mem_pca(const mem_map* mc, int32_t layer, float* out, float eigenvalues[3], void* stream)
{
    mem_map* m = const_cast<mem_map*>(mc);
    if (mem_status st = usable(m)) return st;
    if (!out) return fail(MEM_E_ARG, "out is NULL");
    const Layer* L = nullptr;
    if (mem_status st = resolve_layer(m, layer, &L)) return st;
    if (L->rule == MEM_DIRICHLET) return fail(MEM_E_ARG, "layer %d is a class layer, not a feature layer", layer);
    if (L->C > kPcaWideC) return fail(MEM_E_UNSUPPORTED, "PCA of %d channels (at most %d)", L->C, kPcaWideC);
    hipStream_t s = (hipStream_t)stream;
    if (L->C > kPcaMaxC) {
        if (!m->pcw_scratch || !m->pcw_out) {  // both or neither
            char* p = nullptr;
            PcaWideOut* o = nullptr;
            if (mem_status st = dev_alloc(m, &p, pca_wide_scratch_bytes(m->cells()))) return st;
            if (mem_status st = dev_alloc(m, &o, 1)) {
                (void)hipFree(p);
                return st;
            }
            (void)hipFree(m->pcw_scratch);
            (void)hipFree(m->pcw_out);
            m->pcw_scratch = p;
            m->pcw_out = o;
        }
        timed(m, s, "pca", [&] { launch_pca_wide(s, m->grid(), L->dev(), m->pcw_scratch, m->pcw_out, out, nullptr); });
        if (mem_status st = check_launch(m, "mem_pca")) return st;
        if (eigenvalues) {
            double lam[kPcaK];
            HIP_TRY(m, hipMemcpyAsync(lam, m->pcw_out->lam, sizeof lam, hipMemcpyDeviceToHost, s));
            HIP_TRY(m, hipStreamSynchronize(s));
            for (int k = 0; k < kPcaK; k++) eigenvalues[k] = (float)lam[k];
        }
        return MEM_OK;
    }
    if (!m->pca_scratch || !m->pca_out) {  // both or neither: a failed call leaves neither
        char* p = nullptr;
        PcaOut* o = nullptr;
        if (mem_status st = dev_alloc(m, &p, pca_scratch_bytes())) return st;
        if (mem_status st = dev_alloc(m, &o, 1)) {
            (void)hipFree(p);
            return st;
        }
        (void)hipFree(m->pca_scratch);
        (void)hipFree(m->pca_out);
        m->pca_scratch = p;
        m->pca_out = o;
    }
    timed(m, s, "pca", [&] { launch_pca(s, m->grid(), L->dev(), m->pca_scratch, m->pca_out, out, nullptr); });
    if (mem_status st = check_launch(m, "mem_pca")) return st;
    if (eigenvalues) {
        double lam[kPcaK];
        HIP_TRY(m, hipMemcpyAsync(lam, m->pca_out->lam, sizeof lam, hipMemcpyDeviceToHost, s));
        HIP_TRY(m, hipStreamSynchronize(s));
        for (int k = 0; k < kPcaK; k++) eigenvalues[k] = (float)lam[k];
    }
    return MEM_OK;
}

mem_status mem_pca_noalloc(const mem_map* mc, int32_t layer, float* out, float* eigenvalues, void* stream)
{
    mem_map* m = const_cast<mem_map*>(mc);
    if (mem_status st = usable(m)) return st;
    if (!out) return fail(MEM_E_ARG, "out is NULL");
    const Layer* L = nullptr;
    if (mem_status st = resolve_layer(m, layer, &L)) return st;
    if (L->rule == MEM_DIRICHLET) return fail(MEM_E_ARG, "layer %d is a class layer, not a feature layer", layer);
    if (L->C > kPcaMaxC)
        return fail(MEM_E_UNSUPPORTED, "PCA of %d channels: the static scratch holds at most %d", L->C, kPcaMaxC);
    void* parts = nullptr;
    PcaOut* res = nullptr;
    const hipError_t e = pca_static_scratch(m->device, &parts, &res);
    if (e != hipSuccess)
        return fail(MEM_E_HIP, "address of the PCA's static scratch on device %d: %s", m->device, hipGetErrorString(e));
    hipStream_t s = (hipStream_t)stream;
    launch_pca(s, m->grid(), L->dev(), parts, res, out, eigenvalues);
    return check_launch(m, "mem_pca_noalloc");
}

mem_status mem_set_overlap_clearance(mem_map* m, int32_t enable, float range_xy, float range_z)
{
    if (mem_status st = usable(m)) return st;
    if (enable && (!(range_xy >= 0.0f) || !std::isfinite(range_xy) || !(range_z >= 0.0f) || !std::isfinite(range_z)))
        return fail(MEM_E_ARG, "ranges must be finite and >= 0");
    m->overlap_on = enable != 0;
    m->overlap_xy = range_xy;
    m->overlap_z = range_z;
    return MEM_OK;
}

mem_status mem_get_drift(const mem_map* mc, float* offset, int32_t* consistent, void* stream)
{
    mem_map* m = const_cast<mem_map*>(mc);
    if (mem_status st = usable(m)) return st;
    if (!offset || !consistent) return fail(MEM_E_ARG, "NULL argument");
    DriftDev dd{};
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(m, hipMemcpyAsync(&dd, m->drift, sizeof dd, hipMemcpyDeviceToHost, s));
    HIP_TRY(m, hipStreamSynchronize(s));
    *offset = dd.d;
    *consistent = dd.n;
    return MEM_OK;
}

// Adds image k's intrinsics and size to `cam`.
static mem_status check_intrinsics(int32_t h, int32_t w, const float K[4], int k, Camera* cam)
{
    if (h < 1 || w < 1 || (int64_t)h * w > (1ll << 30)) return fail(MEM_E_ARG, "image size %dx%d", w, h);
    if (!K) return fail(MEM_E_ARG, "K is NULL");
    for (int q = 0; q < 4; q++)
        if (!std::isfinite(K[q])) return fail(MEM_E_ARG, "K must be finite");
    if (!(K[0] > 0.0f) || !(K[1] > 0.0f)) return fail(MEM_E_ARG, "fx and fy must be positive");
    cam->fx[k] = K[0];
    cam->fy[k] = K[1];
    cam->cx[k] = K[2];
    cam->cy[k] = K[3];
    cam->h[k] = h;
    cam->w[k] = w;
    return MEM_OK;
}

static mem_status check_image(const mem_map* m, const mem_image& im, int k, Camera* cam)
{
    if (!im.data) return fail(MEM_E_ARG, "image %d: data is NULL", k);
    if (im.dtype != MEM_F32 && im.dtype != MEM_U8)
        return fail(MEM_E_ARG, "image %d: dtype must be MEM_F32 or MEM_U8", k);
    if (im.c < 1) return fail(MEM_E_ARG, "image %d needs at least one channel", k);
    if (im.strides[0] < 0 || im.strides[1] < 0 || im.strides[2] < 0)
        return fail(MEM_E_ARG, "image %d: strides must be non-negative", k);
    if (im.n_bind < 0 || im.n_bind > kMaxBind || (im.n_bind > 0 && !im.bind))
        return fail(MEM_E_ARG, "image %d: n_bind must be 0..%d with a binding array", k, kMaxBind);
    if (mem_status st = check_intrinsics(im.h, im.w, im.K, k, cam)) return st;
    for (int b = 0; b < im.n_bind; b++) {
        const Layer* L = nullptr;
        if (mem_status st = resolve_layer(m, im.bind[b].layer, &L)) return st;
        char what[48];
        snprintf(what, sizeof what, "image %d binding %d", k, b);
        if (mem_status st = check_binding(im.bind[b], L, im.c, what)) return st;
    }
    return MEM_OK;
}

// Images of n_poses camera poses (counts[p] images of pose p, consecutive
// in `images`).  The poses' projections are independent of each other (no
// image changes a height), so they run as one view launch and one
// occlusion launch; the gathers then follow in call order.
static mem_status input_poses(mem_map* m, const mem_image* images, const int32_t* counts, int n_poses,
                              const float* T_map_cam, void* stream)
{
    if (mem_status st = usable(m)) return st;
    if (n_poses < 1 || n_poses > kMaxPoses || !counts || !T_map_cam)
        return fail(MEM_E_ARG, "n_poses must be 1..%d with counts and poses", kMaxPoses);
    if (!images) return fail(MEM_E_ARG, "images is NULL");
    CameraSet cs{};
    cs.n = n_poses;
    int first = 0;
    for (int p = 0; p < n_poses; p++) {
        if (counts[p] < 1 || counts[p] > kMaxImages)
            return fail(MEM_E_ARG, "pose %d: n_images must be 1..%d", p, kMaxImages);
        Camera& cam = cs.c[p];
        if (mem_status st = check_pose(m, T_map_cam + 12 * p, "T_map_cam")) return st;
        memcpy(cam.T.m, T_map_cam + 12 * p, sizeof(cam.T.m));
        cam.n = counts[p];
        cam.min_depth = m->min_depth;
        for (int k = 0; k < counts[p]; k++)
            if (mem_status st = check_image(m, images[first + k], k, &cam)) return st;
        first += counts[p];
    }
    hipStream_t s = (hipStream_t)stream;
    Grid g = m->grid();
    const int cap = (int)m->cells();
    int4* vlist = m->vlist;
    int* vcode = m->vcode;
    int* vc = nullptr;
    int* vc_next = nullptr;
    if (n_poses == 1) {
        vc = m->take_vcount();
        vc_next = m->vcount + m->vpar;
    } else {
        if (!m->vlist_poses) {  // lists of kMaxPoses poses, allocated on first use
            int4* l = nullptr;
            int* c = nullptr;
            int* n = nullptr;
            if (mem_status st = dev_alloc(m, &l, (size_t)kMaxPoses * cap)) return st;
            if (mem_status st = dev_alloc(m, &c, (size_t)kMaxPoses * kMaxImages * cap)) {
                (void)hipFree(l);
                return st;
            }
            if (mem_status st = dev_alloc(m, &n, kMaxPoses)) {
                (void)hipFree(l);
                (void)hipFree(c);
                return st;
            }
            m->vlist_poses = l;
            m->vcode_poses = c;
            m->vcount_poses = n;
        }
        vlist = m->vlist_poses;
        vcode = m->vcode_poses;
        vc = m->vcount_poses;
        launch_zero_int(s, vc, n_poses);
    }
    TileMax tm;
    timed(m, s, "tile_max", [&] { tm = m->tiles(s); });
    timed_ext(m, s, "project", [&](LaunchEv ev) {
        launch_project(s, g, cs, m->h, tm, cap, vc, vc_next, vlist, vcode, nullptr, m->stats, ev);
    });
    // The gathers in call order, grouped into launches: a binding joins the
    // open group unless the group already writes its layer (bindings of
    // different layers commute, those of one layer keep their order).
    GatherJobs js{};
    int group_layers[kMaxGatherJobs];
    auto flush = [&] {
        if (js.n == 0) return;
        timed_ext(m, s, "gather_fuse", [&](LaunchEv ev) {
            if (js.n == 1) {
                const GatherJob& J = js.j[0];
                launch_gather_fuse(s, J.vlist, J.vcode, J.count, cap, J.img, J.kind >= 6 ? MEM_F32 : MEM_U8, J.s0,
                                   J.s1, J.s2, J.w, J.ch_first, J.L, J.topk, J.kind % 2 != 0, ev);
            } else {
                launch_gather_multi(s, js, ev);
            }
        });
        js.n = 0;
    };
    first = 0;
    for (int p = 0; p < n_poses; p++) {
        for (int k = 0; k < counts[p]; k++) {
            const mem_image& im = images[first + k];
            for (int b = 0; b < im.n_bind; b++) {
                const Layer* L = nullptr;
                resolve_layer(m, im.bind[b].layer, &L);
                bool taken = js.n == kMaxGatherJobs;
                for (int q = 0; q < js.n; q++) taken = taken || group_layers[q] == im.bind[b].layer;
                if (taken) flush();
                group_layers[js.n] = im.bind[b].layer;
                js.j[js.n++] = gather_job(vlist + (int64_t)p * cap, vcode + ((int64_t)p * kMaxImages + k) * cap,
                                          vc + p, cap, im.data, im.dtype, im.strides[0], im.strides[1],
                                          im.strides[2], im.w, im.bind[b].ch_first, L->dev(), im.bind[b].topk,
                                          m->gather_v1 != 0);
            }
        }
        first += counts[p];
    }
    flush();
    return check_launch(m, "mem_input_images");
}

mem_status mem_input_images(mem_map* m, const mem_image* images, int32_t n_images,
                            const float T_map_cam[12], void* stream)
{
    if (!images || n_images < 1 || n_images > kMaxImages)
        return fail(MEM_E_ARG, "n_images must be 1..%d with an image array", kMaxImages);
    return input_poses(m, images, &n_images, 1, T_map_cam, stream);
}

mem_status mem_input_image_poses(mem_map* m, const mem_image* images, const int32_t* n_images,
                                 int32_t n_poses, const float* T_map_cam, void* stream)
{
    return input_poses(m, images, n_images, n_poses, T_map_cam, stream);
}

mem_status mem_input_image(mem_map* m, const void* img, int32_t dtype, int32_t h, int32_t w, int32_t c,
                           const int64_t strides[3], const float K[4], const float T_map_cam[12],
                           const mem_binding* bind, int32_t n_bind, void* stream)
{
    if (!strides) return fail(MEM_E_ARG, "strides is NULL");
    if (!K) return fail(MEM_E_ARG, "K is NULL");
    mem_image im;
    im.data = img;
    im.dtype = dtype;
    im.h = h;
    im.w = w;
    im.c = c;
    memcpy(im.strides, strides, sizeof(im.strides));
    memcpy(im.K, K, sizeof(im.K));
    im.bind = bind;
    im.n_bind = n_bind;
    return mem_input_images(m, &im, 1, T_map_cam, stream);
}

mem_status mem_get_layer(const mem_map* mc, int32_t layer, int32_t view, float* out, void* stream)
{
    mem_map* m = const_cast<mem_map*>(mc);
    if (mem_status st = usable(m)) return st;
    if (!out) return fail(MEM_E_ARG, "out is NULL");
    LayerDev d{};
    if (layer >= 0 && layer <= MEM_LAYER_CLEAR) {
        if (view != MEM_VIEW_VALUE) return fail(MEM_E_ARG, "built-in layers have only the value view");
    } else {
        const Layer* L = nullptr;
        if (mem_status st = resolve_layer(m, layer, &L)) return st;
        bool ok = view == MEM_VIEW_VALUE || (view == MEM_VIEW_AUX && (L->rule == MEM_GAUSS || L->rule == MEM_DIRICHLET)) ||
                  (view == MEM_VIEW_ARGMAX && L->rule == MEM_DIRICHLET);
        if (!ok) return fail(MEM_E_ARG, "layer %d has no view %d", layer, view);
        d = L->dev();
    }
    hipStream_t s = (hipStream_t)stream;
    timed(m, s, "readout", [&] {
        launch_readout(s, m->grid(), layer, view, m->h, m->v, m->cnt_last, m->clr_last,
                       layer >= MEM_LAYER_USER0 ? &d : nullptr, out);
    });
    return check_launch(m, "mem_get_layer");
}

mem_status mem_normals(const mem_map* mc, float* out, void* stream)
{
    mem_map* m = const_cast<mem_map*>(mc);
    if (mem_status st = usable(m)) return st;
    if (!out) return fail(MEM_E_ARG, "out is NULL");
    hipStream_t s = (hipStream_t)stream;
    timed(m, s, "normals", [&] { launch_normals(s, m->grid(), m->h, out); });
    return check_launch(m, "mem_normals");
}

mem_status mem_set_layer(mem_map* m, int32_t layer, int32_t view, const float* in, void* stream)
{
    if (mem_status st = usable(m)) return st;
    if (!in) return fail(MEM_E_ARG, "in is NULL");
    LayerDev d{};
    if (layer == MEM_LAYER_ELEVATION || layer == MEM_LAYER_VARIANCE) {
        if (view != MEM_VIEW_VALUE) return fail(MEM_E_ARG, "built-in layers have only the value view");
    } else if (layer >= 0 && layer < MEM_LAYER_USER0) {
        return fail(MEM_E_ARG, "layer %d is not settable", layer);
    } else {
        const Layer* L = nullptr;
        if (mem_status st = resolve_layer(m, layer, &L)) return st;
        bool ok = (view == MEM_VIEW_VALUE && L->rule != MEM_DIRICHLET) ||
                  (view == MEM_VIEW_AUX && (L->rule == MEM_GAUSS || L->rule == MEM_DIRICHLET));
        if (!ok) return fail(MEM_E_ARG, "view %d of layer %d is not settable", view, layer);
        d = L->dev();
    }
    hipStream_t s = (hipStream_t)stream;
    if (layer == MEM_LAYER_ELEVATION) {
        m->tmax_stale = true;
        m->hl_fresh = false;
    }
    timed(m, s, "setlayer", [&] {
        launch_setlayer(s, m->grid(), layer, view, m->h, m->v, layer >= MEM_LAYER_USER0 ? &d : nullptr, in);
    });
    return check_launch(m, "mem_set_layer");
}

mem_status mem_debug_point_cells(const mem_map* mc, const float* xyz, int64_t n, const float T[12],
                                 int32_t* out, void* stream)
{
    mem_map* m = const_cast<mem_map*>(mc);
    if (mem_status st = usable(m)) return st;
    if (n < 0 || (n > 0 && (!xyz || !out))) return fail(MEM_E_ARG, "bad points / output");
    if (mem_status st = check_pose(m, T, "T_map_sensor")) return st;
    Pose P;
    memcpy(P.m, T, sizeof(P.m));
    launch_point_cells((hipStream_t)stream, m->grid(), xyz, n, P, m->mr2, out);
    return check_launch(m, "mem_debug_point_cells");
}

mem_status mem_debug_gather_width(mem_map* m, int32_t width)
{
    if (mem_status st = usable(m)) return st;
    if (width != 0 && width != 1) return fail(MEM_E_ARG, "width must be 0 (automatic) or 1");
    m->gather_v1 = width;
    return MEM_OK;
}

mem_status mem_debug_cell_pixels(const mem_map* mc, int32_t h, int32_t w, const float K[4],
                                 const float T[12], int32_t* out, void* stream)
{
    mem_map* m = const_cast<mem_map*>(mc);
    if (mem_status st = usable(m)) return st;
    if (!out) return fail(MEM_E_ARG, "out is NULL");
    Camera cam{};
    if (mem_status st = check_pose(m, T, "T_map_cam")) return st;
    if (mem_status st = check_intrinsics(h, w, K, 0, &cam)) return st;
    memcpy(cam.T.m, T, sizeof(cam.T.m));
    cam.n = 1;
    cam.min_depth = m->min_depth;
    CameraSet cs{};
    cs.c[0] = cam;
    cs.n = 1;
    hipStream_t s = (hipStream_t)stream;
    const TileMax tm = m->tiles(s);
    int* vc = m->take_vcount();
    launch_project(s, m->grid(), cs, m->h, tm, (int)m->cells(), vc, m->vcount + m->vpar, m->vlist, m->vcode, out,
                   m->stats);
    return check_launch(m, "mem_debug_cell_pixels");
}

mem_status mem_get_stats(mem_map* m, mem_stats* out, void* stream)
{
    if (mem_status st = usable(m)) return st;
    if (!out) return fail(MEM_E_ARG, "out is NULL");
    unsigned long long buf[kStats * kStatSlots];
    HIP_TRY(m, hipMemcpyAsync(buf, m->stats, sizeof buf, hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIP_TRY(m, hipStreamSynchronize((hipStream_t)stream));
    int64_t* o = (int64_t*)out;
    for (int k = 0; k < kStats; k++) {
        o[k] = 0;
        for (int j = 0; j < kStatSlots; j++) o[k] += (int64_t)buf[k * kStatSlots + j];
    }
    return MEM_OK;
}

mem_status mem_reset_stats(mem_map* m, void* stream)
{
    if (mem_status st = usable(m)) return st;
    launch_zero_int((hipStream_t)stream, (int*)m->stats, 2 * kStats * kStatSlots);
    return check_launch(m, "mem_reset_stats");
}

mem_status mem_profile_enable(mem_map* m, int32_t on)
{
    if (mem_status st = usable(m)) return st;
    m->prof.enable(on != 0);
    return MEM_OK;
}

mem_status mem_profile_read(mem_map* m, mem_kernel_time* out, int32_t max, int32_t* count)
{
    if (mem_status st = usable(m)) return st;
    if (!count || (max > 0 && !out)) return fail(MEM_E_ARG, "NULL output");
    *count = m->prof.read(out, max);
    return MEM_OK;
}

}  // extern "C"

namespace memk {

// The current height and variance layers of a map, for the completion network.
mem_status map_height_view(const mem_map* m, const float** h, const float** v, Grid* g)
{
    if (!m) return api_fail(MEM_E_ARG, "map is NULL");
    if (m->broken) return api_fail(MEM_E_STATE, "map is unusable after an earlier HIP error");
    *h = m->h;
    *v = m->v;
    *g = m->grid();
    return MEM_OK;
}

}  // namespace memk

