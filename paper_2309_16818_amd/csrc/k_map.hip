// k_map.hip - grid maintenance: resetting cells that enter the moving grid,
// the layer read-out / write-in views, and the per-cell surface normals.
#include <cmath>

#include "update.h"

namespace memk {

namespace {

constexpr float kNaN = __builtin_nanf("");

struct LayerSet {
    LayerDev L[32];
    int n;
};

constexpr int kResetCells = 32;  // cells of one row per k_reset_rect workgroup

// Resets the logical rectangle [x0, x1) x [y0, y1): a workgroup per run of
// up to kResetCells cells of one row, its threads over the run's (cell,
// channel) elements of each layer, so that a cell's channel row is written
// by consecutive lanes (the strips a move resets are often 1-3 cells wide).
__global__ __launch_bounds__(256) void k_reset_rect(Grid g, int x0, int x1, int y0, int y1,
                                                    float* __restrict__ h, float* __restrict__ v,
                                                    int* __restrict__ cnt, int* __restrict__ clr,
                                                    LayerSet ls)
{
    const int xa = x0 + blockIdx.x * kResetCells;
    const int n = min(kResetCells, x1 - xa);
    for (int iy = y0 + blockIdx.y; iy < y1; iy += gridDim.y) {
        if ((int)threadIdx.x < n) {
            const int st = storage_index(g, xa + threadIdx.x, iy);
            h[st] = kNaN;
            v[st] = __builtin_inff();
            cnt[st] = 0;
            clr[st] = 0;
        }
        for (int l = 0; l < ls.n; l++) {
            const LayerDev& L = ls.L[l];
            const float init = (L.rule == MEM_DIRICHLET) ? L.param : kNaN;
            for (int e = threadIdx.x; e < n * L.C; e += blockDim.x) {
                const int j = e / L.C, q = e - j * L.C;
                const int st = storage_index(g, xa + j, iy);
                layer_store(L.val, L.storage, L.scale, (int64_t)st * L.C + q, q, init);
            }
            if (L.rule == MEM_GAUSS && (int)threadIdx.x < n) L.var[storage_index(g, xa + threadIdx.x, iy)] = __builtin_inff();
        }
    }
}

// out[(iy*W + ix)*C + q], logical order.  layer < 8: built-in layers.
__global__ __launch_bounds__(256) void k_readout(Grid g, int layer, int view,
                                                 const float* __restrict__ h,
                                                 const float* __restrict__ v,
                                                 const int* __restrict__ cnt,
                                                 const int* __restrict__ clr, LayerDev L,
                                                 float* __restrict__ out)
{
    const int HW = g.W * g.H;
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= HW) return;
    int ix = j % g.W, iy = j / g.W;
    int st = storage_index(g, ix, iy);
    if (layer < 8) {
        float o;
        float hv = h[st];
        switch (layer) {
        case MEM_LAYER_ELEVATION: o = hv; break;
        case MEM_LAYER_VARIANCE: o = isnan(hv) ? kNaN : v[st]; break;
        case MEM_LAYER_VALID: o = isnan(hv) ? 0.0f : 1.0f; break;
        case MEM_LAYER_HITS: o = (float)cnt[st]; break;
        default: o = (float)clr[st]; break;
        }
        out[j] = o;
        return;
    }
    const int C = L.C;
    if (view == MEM_VIEW_AUX && L.rule == MEM_GAUSS) {
        out[j] = L.var[st];
        return;
    }
    if (view == MEM_VIEW_ARGMAX) {  // lowest index on ties
        int best = 0;
        float bv = layer_load(L.val, L.storage, L.scale, (int64_t)st * C, 0);
        for (int q = 1; q < C; q++) {
            float x = layer_load(L.val, L.storage, L.scale, (int64_t)st * C + q, q);
            if (x > bv) {
                bv = x;
                best = q;
            }
        }
        out[j] = (float)best;
        return;
    }
    if (view == MEM_VIEW_VALUE && L.rule == MEM_DIRICHLET) {  // Eq. (11)
        float s = 0.0f;
        for (int q = 0; q < C; q++) s += layer_load(L.val, L.storage, L.scale, (int64_t)st * C + q, q);
        for (int q = 0; q < C; q++)
            out[(int64_t)j * C + q] = layer_load(L.val, L.storage, L.scale, (int64_t)st * C + q, q) / s;
        return;
    }
    for (int q = 0; q < C; q++)
        out[(int64_t)j * C + q] = layer_load(L.val, L.storage, L.scale, (int64_t)st * C + q, q);
}

__global__ __launch_bounds__(256) void k_setlayer(Grid g, int layer, int view,
                                                  float* __restrict__ h, float* __restrict__ v,
                                                  LayerDev L, const float* __restrict__ in)
{
    const int HW = g.W * g.H;
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= HW) return;
    int ix = j % g.W, iy = j / g.W;
    int st = storage_index(g, ix, iy);
    if (layer == MEM_LAYER_ELEVATION) {
        h[st] = in[j];
        return;
    }
    if (layer == MEM_LAYER_VARIANCE) {
        if (!isnan(in[j])) v[st] = in[j];
        return;
    }
    if (view == MEM_VIEW_AUX && L.rule == MEM_GAUSS) {
        L.var[st] = in[j];
        return;
    }
    for (int q = 0; q < L.C; q++)
        layer_store(L.val, L.storage, L.scale, (int64_t)st * L.C + q, q, in[(int64_t)j * L.C + q]);
}


// Surface normal of every logical cell (Table I, normal calculation): the
// height gradient from central differences of the four 4-neighbours, the
// normal (-gx, -gy, 1) / |(-gx, -gy, 1)|.  NaN where the cell lies on the
// border or it or a 4-neighbour holds no height.  Tiles of 64 x 4 cells: a
// wave reads one row run of heights and its two neighbour rows, and writes
// 64 x 3 consecutive floats.
__global__ __launch_bounds__(256) void k_normals(Grid g, const float* __restrict__ h, float* __restrict__ out)
{
    const int ix = blockIdx.x * 64 + threadIdx.x;
    const int iy = blockIdx.y * 4 + threadIdx.y;
    if (ix >= g.W || iy >= g.H) return;
    float nx = kNaN, ny = kNaN, nz = kNaN;
    if (ix >= 1 && ix <= g.W - 2 && iy >= 1 && iy <= g.H - 2) {
        const float hc = h[storage_index(g, ix, iy)];
        const float hw = h[storage_index(g, ix - 1, iy)];
        const float he = h[storage_index(g, ix + 1, iy)];
        const float hs = h[storage_index(g, ix, iy - 1)];
        const float hn = h[storage_index(g, ix, iy + 1)];
        if (!isnan(hc) && !isnan(hw) && !isnan(he) && !isnan(hs) && !isnan(hn)) {
            const float d = 2.0f * g.res;
            const float gx = (he - hw) / d;
            const float gy = (hn - hs) / d;
            const float r = 1.0f / sqrtf(gx * gx + gy * gy + 1.0f);
            nx = -gx * r;
            ny = -gy * r;
            nz = r;
        }
    }
    float* o = out + 3 * (int64_t)(iy * g.W + ix);
    o[0] = nx;
    o[1] = ny;
    o[2] = nz;
}

// Overlap clearance (Table I, after the multi-modal update): logical cells
// [x0, x1) x [y0, y1), a box that holds every cell whose centre can lie
// within the horizontal range; a held height there more than rz above or
// below the sensor is removed.  Binary32 decisions with the cell centre of
// the camera association.
__global__ __launch_bounds__(256) void k_overlap_clear(Grid g, int x0, int x1, int y0, int y1, float sx, float sy,
                                                       float sz, float r2max, float rz, float* __restrict__ h)
{
    const int bw = x1 - x0;
    const int64_t nb = (int64_t)bw * (y1 - y0);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nb; k += stride) {
        const int ix = x0 + (int)(k % bw), iy = y0 + (int)(k / bw);
        const int st = storage_index(g, ix, iy);
        const float hj = h[st];
        if (isnan(hj)) continue;
        const float dx = ((float)(g.ox + ix) + 0.5f) * g.res - sx;
        const float dy = ((float)(g.oy + iy) + 0.5f) * g.res - sy;
        const float d2 = dx * dx + dy * dy;
        if (d2 <= r2max && fabsf(hj - sz) > rz) h[st] = kNaN;
    }
}

}  // namespace

void launch_reset_rect(hipStream_t s, const Grid& g, int x0, int x1, int y0, int y1, float* h,
                       float* v, int* cnt, int* clr, const LayerDev* L, int nL)
{
    if (x1 <= x0 || y1 <= y0) return;
    LayerSet ls;
    ls.n = nL;
    for (int l = 0; l < nL; l++) ls.L[l] = L[l];
    dim3 grid((unsigned)((x1 - x0 + kResetCells - 1) / kResetCells), (unsigned)(y1 - y0 < 2048 ? y1 - y0 : 2048));
    hipLaunchKernelGGL(k_reset_rect, grid, dim3(256), 0, s, g, x0, x1, y0, y1, h, v, cnt, clr, ls);
}

void launch_readout(hipStream_t s, const Grid& g, int layer, int view, const float* h,
                    const float* v, const int* cnt, const int* clr, const LayerDev* L, float* out)
{
    int HW = g.W * g.H;
    LayerDev l{};
    if (L) l = *L;
    hipLaunchKernelGGL(k_readout, dim3((HW + 255) / 256), dim3(256), 0, s, g, layer, view, h, v, cnt,
                       clr, l, out);
}

void launch_setlayer(hipStream_t s, const Grid& g, int layer, int view, float* h, float* v,
                     const LayerDev* L, const float* in)
{
    int HW = g.W * g.H;
    LayerDev l{};
    if (L) l = *L;
    hipLaunchKernelGGL(k_setlayer, dim3((HW + 255) / 256), dim3(256), 0, s, g, layer, view, h, v, l, in);
}

void launch_normals(hipStream_t s, const Grid& g, const float* h, float* out)
{
    dim3 grid((unsigned)((g.W + 63) / 64), (unsigned)((g.H + 3) / 4));
    hipLaunchKernelGGL(k_normals, grid, dim3(64, 4), 0, s, g, h, out);
}

void launch_overlap_clear(hipStream_t s, const Grid& g, float sx, float sy, float sz, float rxy, float rz, float* h)
{
    // a box one cell wider than the disc on every side: binary32 rounding
    // of the centres cannot reach a cell outside it
    const double r = (double)rxy;
    // clamped in double before the conversion (the range may be huge)
    auto cell = [&](double pos, int origin, int add, int n) {
        const double c = std::floor(pos / g.res) - origin + add;
        return (int)(c < 0.0 ? 0.0 : c > n ? (double)n : c);
    };
    const int x0 = cell((double)sx - r, g.ox, -1, g.W), x1 = cell((double)sx + r, g.ox, 2, g.W);
    const int y0 = cell((double)sy - r, g.oy, -1, g.H), y1 = cell((double)sy + r, g.oy, 2, g.H);
    if (x1 <= x0 || y1 <= y0) return;
    int64_t blocks = ((int64_t)(x1 - x0) * (y1 - y0) + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_overlap_clear, dim3((unsigned)blocks), dim3(256), 0, s, g, x0, x1, y0, y1, sx, sy, sz,
                       rxy * rxy, rz, h);
}

}  // namespace memk
