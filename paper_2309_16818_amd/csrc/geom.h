// geom.h - binary32 decision formulas of the map update (device side).
//
// Every function here decides an integer (a cell, a pixel, a vote) and must
// evaluate exactly as specified in include/mem.h: binary32, the written
// operation order, no fused multiply-add (the library is compiled with
// -ffp-contract=off and correctly rounded division).
#pragma once

#include <hip/hip_runtime.h>

#include "mem_internal.h"

namespace memk {

// Storage index of logical cell (ix, iy), both inside the grid.
__device__ __forceinline__ int storage_index(const Grid& g, int ix, int iy)
{
    int sx = ix + g.rx;
    sx -= (sx >= g.W) ? g.W : 0;
    int sy = iy + g.ry;
    sy -= (sy >= g.H) ? g.H : 0;
    return (int)__umul24((unsigned)sy, (unsigned)g.W) + sx;  // sides <= 16384 < 2^24
}

// h[st] for a storage index st >= 0 of a grid under 2^30 cells, addressed
// with a 32-bit byte offset from the base (one address operation instead of
// a 64-bit pointer sum per load).
__device__ __forceinline__ float load_cell(const float* __restrict__ h, int st)
{
    return *(const float*)((const char*)h + (uint32_t)st * 4u);
}

// Logical cell of a storage index.
__device__ __forceinline__ void logical_index(const Grid& g, int st, int& ix, int& iy)
{
    int sy = st / g.W;
    int sx = st - sy * g.W;
    ix = sx - g.rx;
    ix += (ix < 0) ? g.W : 0;
    iy = sy - g.ry;
    iy += (iy < 0) ? g.H : 0;
}

// Sensor-frame point -> map frame and grid cell (Sec. III-B association by
// horizontal coordinates).  Returns 0 (accepted) or -1 non-finite, -2 out of
// range, -3 outside the grid.  r2 receives the sensor-frame range squared.
__device__ __forceinline__ int point_cell(const Grid& g, const Pose& T, float mr2, float x,
                                          float y, float z, float& px, float& py, float& pz,
                                          float& r2, int& ix, int& iy)
{
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) return -1;
    float xx = x * x, yy = y * y, zz = z * z;
    r2 = xx + yy;
    r2 = r2 + zz;
    if (r2 > mr2) return -2;
    const float* m = T.m;
    float a, b, c;
    a = m[0] * x; b = m[1] * y; c = m[2] * z;
    px = ((a + b) + c) + m[3];
    a = m[4] * x; b = m[5] * y; c = m[6] * z;
    py = ((a + b) + c) + m[7];
    a = m[8] * x; b = m[9] * y; c = m[10] * z;
    pz = ((a + b) + c) + m[11];
    if (!(isfinite(px) && isfinite(py) && isfinite(pz))) return -3;
    float gx = floorf(px * g.inv_res);
    float gy = floorf(py * g.inv_res);
    if (!(gx >= (float)g.ox && gx < (float)(g.ox + g.W))) return -3;
    if (!(gy >= (float)g.oy && gy < (float)(g.oy + g.H))) return -3;
    ix = (int)gx - g.ox;
    iy = (int)gy - g.oy;
    return 0;
}

// Logical lattice cell of a position (may lie outside the grid).
__device__ __forceinline__ void lattice_cell(const Grid& g, float x, float y, int& ix, int& iy)
{
    ix = (int)floorf(x * g.inv_res) - g.ox;
    iy = (int)floorf(y * g.inv_res) - g.oy;
}

// Incremental Bresenham walk from (ax, ay) towards (bx, by).  step() moves
// to the next cell: one cell along the major axis, plus one along the minor
// axis when the error term D > 0.  The two moves are kept as increments
// (mx, my) and (nx, ny) so a step has no branch on the line's octant.
struct LineWalk {
    int x, y, mx, my, nx, ny, dmaj2, dmin2, D, steps;
    bool xmajor;
    __device__ __forceinline__ LineWalk(int ax, int ay, int bx, int by)
    {
        const int dx = abs(bx - ax), dy = abs(by - ay);
        const int sx = (bx >= ax) ? 1 : -1;
        const int sy = (by >= ay) ? 1 : -1;
        x = ax;
        y = ay;
        xmajor = dx >= dy;
        const int dmaj = xmajor ? dx : dy, dmin = xmajor ? dy : dx;
        D = 2 * dmin - dmaj;
        dmaj2 = 2 * dmaj;
        dmin2 = 2 * dmin;
        steps = dmaj;
        mx = xmajor ? sx : 0;
        my = xmajor ? 0 : sy;
        nx = xmajor ? 0 : sx;
        ny = xmajor ? sy : 0;
    }
    // Moves from the start cell directly to the cell after i steps.  With
    // dmaj = |major extent| and dmin = |minor extent|, the minor offset after
    // i steps is m = floor((2 i dmin + dmaj - 1) / (2 dmaj)) (the nearest
    // lattice point to the ideal line, ties toward the start) and the error
    // term is D = 2 dmin (i + 1) - dmaj - 2 dmaj m, exactly what i calls of
    // step() produce.
    __device__ __forceinline__ void jump_from_start(int i)
    {
        const int dmaj = dmaj2 >> 1, dmin = dmin2 >> 1;
        if (i <= 0 || dmaj == 0) return;
        int m;
        if (dmaj < 32768) {
            // 2 i dmin + dmaj - 1 < 2^31 since i, dmin <= dmaj: 32-bit division
            m = (int)((2u * (unsigned)i * (unsigned)dmin + (unsigned)dmaj - 1u) / (2u * (unsigned)dmaj));
        } else {
            m = (int)((2 * (int64_t)i * dmin + dmaj - 1) / (2 * (int64_t)dmaj));
        }
        D = (int)(2 * (int64_t)dmin * ((int64_t)i + 1) - dmaj - 2 * (int64_t)dmaj * m);
        x += mx * i + nx * m;
        y += my * i + ny * m;
    }
    __device__ __forceinline__ void step()
    {
        const bool c = D > 0;
        x += mx + (c ? nx : 0);
        y += my + (c ? ny : 0);
        D += dmin2 - (c ? dmaj2 : 0);
    }
    __device__ __forceinline__ int major() const { return xmajor ? x : y; }
};

// Height of the ray s -> p above the cell whose absolute major-axis lattice
// index is k: the ray parameter is taken at that cell's centre.
// inv_d = 1 / (p_major - s_major), dz = p_z - s_z.
__device__ __forceinline__ float ray_height(int k_abs, float res, float s_major, float inv_d,
                                            float s_z, float dz)
{
    float c = (float)k_abs + 0.5f;
    c = c * res;
    float t = (c - s_major) * inv_d;
    return s_z + dz * t;
}

// A ray from s (map frame) to p over the Bresenham cells between the
// sensor's cell and the target cell.
struct Ray {
    LineWalk L;
    int o_major;       // absolute lattice index of logical 0 along the major axis
    float s_major, inv_d, s_z, dz;
    bool all_inside;   // both ends inside the grid, so every cell between is
    __device__ __forceinline__ Ray(const Grid& g, int ax, int ay, int bx, int by, float sx,
                                   float sy, float sz, float px, float py, float pz)
        : L(ax, ay, bx, by)
    {
        o_major = L.xmajor ? g.ox : g.oy;
        s_major = L.xmajor ? sx : sy;
        const float p_major = L.xmajor ? px : py;
        inv_d = 1.0f / (p_major - s_major);
        s_z = sz;
        dz = pz - sz;
        all_inside = ax >= 0 && ax < g.W && ay >= 0 && ay < g.H;
    }
    // The same ray from its reciprocal major extent and height difference
    // as the constructor above computes them.
    __device__ __forceinline__ Ray(const Grid& g, int ax, int ay, int bx, int by, float sx, float sy, float sz,
                                   float inv_d_, float dz_, int /*tag*/)
        : L(ax, ay, bx, by)
    {
        o_major = L.xmajor ? g.ox : g.oy;
        s_major = L.xmajor ? sx : sy;
        inv_d = inv_d_;
        s_z = sz;
        dz = dz_;
        all_inside = ax >= 0 && ax < g.W && ay >= 0 && ay < g.H;
    }
};

// Visits the cells strictly between the ray's end cells, in order, U at a
// time: the U cells' heights are loaded together before any of them is
// tested, so a lane keeps U loads in flight.  visit(st, h, z_ray) returns
// true to stop the walk.  Cells outside the grid are skipped.  Returns the
// number of in-grid cells loaded.  The batch of U is computed without
// branches: past the last cell the walk keeps stepping and loads cell 0
// (always in bounds) in place of the cells it does not visit, and a walk
// that starts inside the grid (so every cell up to the target is inside)
// needs no bounds test at all.  Cells not visited reach `visit` with a NaN
// height, which every visit must ignore (NaN is also an empty cell's
// height).  The walker's position after the call is unspecified.
template <int U, bool Inside, class Visit>
__device__ __forceinline__ int walk_cells_impl(const Grid& g, Ray& r, const float* __restrict__ h,
                                               Visit& visit)
{
    int rem = r.L.steps - 1;
    int loaded = 0;
    while (rem > 0) {
        int st[U];
        float zr[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            r.L.step();
            ok[u] = u < rem;
            if (!Inside) ok[u] = ok[u] && r.L.x >= 0 && r.L.x < g.W && r.L.y >= 0 && r.L.y < g.H;
            const int si = storage_index(g, r.L.x, r.L.y);  // computed always: a select, not a branch
            st[u] = ok[u] ? si : 0;
            zr[u] = ray_height(r.o_major + r.L.major(), g.res, r.s_major, r.inv_d, r.s_z, r.dz);
        }
        float hk[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const float x = load_cell(h, st[u]);
            hk[u] = ok[u] ? x : __builtin_nanf("");
        }
        bool stop = false;
#pragma unroll
        for (int u = 0; u < U; u++) {
            loaded += ok[u] ? 1 : 0;
            if (!stop && visit(st[u], hk[u], zr[u])) stop = true;
        }
        if (stop) break;
        rem -= U;
    }
    return loaded;
}

template <int U, class Visit>
__device__ __forceinline__ int walk_cells(const Grid& g, Ray& r, const float* __restrict__ h,
                                          Visit&& visit)
{
    if (r.all_inside) return walk_cells_impl<U, true>(g, r, h, visit);
    return walk_cells_impl<U, false>(g, r, h, visit);
}

// walk_cells over a grid stored in logical order (`g` with rx = ry = 0, so
// cell (x, y) is at y * W + x) for a ray that starts inside the grid, so
// that every cell up to its target is inside: the linear index advances by
// the major step plus, when Bresenham's error term says so, the minor
// step, and the cell's major lattice coordinate is carried as a float
// (k + 0.5 is exact below 2^22, so each ray height equals ray_height's).
// Rays reaching beyond that range take walk_cells.
// The pipelined walk itself: batch(st, z, h, n) tests a batch of U cells
// (storage indices, ray heights, heights; the first n are cells of the ray,
// the rest past its end) and returns true to stop the walk; `visit` serves
// the rays that take walk_cells instead.
template <int U, class Visit, class Batch>
__device__ __forceinline__ int walk_logical_batches(const Grid& g, Ray& r, const float* __restrict__ h,
                                                    Visit& visit, Batch&& batch)
{
    const LineWalk& L = r.L;
    const int k0 = r.o_major + L.major();
    const int sgn = L.xmajor ? L.mx : L.my;
    const int k1 = k0 + sgn * L.steps;
    if (!r.all_inside || max(abs(k0), abs(k1)) >= (1 << 22)) return walk_cells_impl<U, false>(g, r, h, visit);
    const int inc_maj = L.mx + L.my * g.W, inc_min = L.nx + L.ny * g.W;
    const int last = g.W * g.H - 1;
    const float fs = (float)sgn;
    float c = (float)k0 + 0.5f;
    int lin = L.y * g.W + L.x;
    int D = L.D;
    int rem = L.steps - 1;
    if (rem <= 0) return 0;
    // Software pipelined: the next batch's loads are issued before the
    // current batch is tested, so 2U loads are in flight.  The loop body
    // always fetches (its batch is full) and the last batch is tested after
    // the loop, so every path into a test has the same loads outstanding and
    // each wait is for exactly the value it needs.
    int st[U];
    float zr[U], hk[U];
    auto fetch = [&](int (&s_)[U], float (&z_)[U], float (&h_)[U]) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            const bool diag = D > 0;
            lin += inc_maj + (diag ? inc_min : 0);
            D += L.dmin2 - (diag ? L.dmaj2 : 0);
            c += fs;
            // past the target the walk may leave the grid: clamp, then ignore
            s_[u] = min((unsigned)lin, (unsigned)last);
            float t = c * g.res;
            t = (t - r.s_major) * r.inv_d;
            z_[u] = r.s_z + r.dz * t;
        }
#pragma unroll
        for (int u = 0; u < U; u++) h_[u] = load_cell(h, s_[u]);
    };
    // Two batches alternate between the buffers (no copies, so no register
    // of a load in flight is reused before its value is tested).
    int st2[U];
    float zr2[U], hk2[U];
    int loaded = 0;
    auto test = [&](const int (&s_)[U], const float (&z_)[U], const float (&h_)[U], int n) {
        loaded += min(n, U);
        return batch(s_, z_, h_, n);
    };
    fetch(st, zr, hk);
    while (true) {
        if (rem <= U) {
            test(st, zr, hk, rem);
            break;
        }
        fetch(st2, zr2, hk2);
        if (test(st, zr, hk, U)) break;
        rem -= U;
        if (rem <= U) {
            test(st2, zr2, hk2, rem);
            break;
        }
        fetch(st, zr, hk);
        if (test(st2, zr2, hk2, U)) break;
        rem -= U;
    }
    return loaded;
}

template <int U, class Visit>
__device__ __forceinline__ int walk_logical(const Grid& g, Ray& r, const float* __restrict__ h,
                                            Visit&& visit)
{
    return walk_logical_batches<U>(g, r, h, visit,
                                   [&](const int (&s_)[U], const float (&z_)[U], const float (&h_)[U], int n) {
                                       bool stop = false;
#pragma unroll
                                       for (int u = 0; u < U; u++) {
                                           const float hu = u < n ? h_[u] : __builtin_nanf("");
                                           if (!stop && visit(s_[u], hu, z_[u])) stop = true;
                                       }
                                       return stop;
                                   });
}

// walk_logical over `count` cells from intermediate cell `first`.
template <int U, class Visit>
__device__ __forceinline__ int walk_range_logical(const Grid& g, Ray& r, const float* __restrict__ h,
                                                  int first, int count, Visit&& visit)
{
    r.L.jump_from_start(first - 1);
    r.L.steps = count + 1;
    return walk_logical<U>(g, r, h, visit);
}

// Largest entry of a block-max table (blocks of side 1 << shift) over the
// blocks that the logical cells between (x0, y0) and (x1, y1) (inclusive,
// either order, clamped to the grid) fall in; -inf if none is inside.
__device__ __forceinline__ float box_max(const Grid& g, const float* __restrict__ t, int tw, int shift, int x0,
                                         int y0, int x1, int y1)
{
    const int xa = max(min(x0, x1), 0), xb = min(max(x0, x1), g.W - 1);
    const int ya = max(min(y0, y1), 0), yb = min(max(y0, y1), g.H - 1);
    float m = -__builtin_inff();
    if (xa > xb || ya > yb) return m;
    for (int ty = ya >> shift; ty <= (yb >> shift); ty++)
        for (int tx = xa >> shift; tx <= (xb >> shift); tx++) m = fmaxf(m, t[ty * tw + tx]);
    return m;
}

// box_max for a box at most two blocks wide in each direction (a run of at
// most 1 << shift cells of a line): its four corner blocks' maxima, loaded
// together (the same block twice where the box is one block wide).
__device__ __forceinline__ float box_max2(const Grid& g, const float* __restrict__ t, int tw, int shift, int x0,
                                          int y0, int x1, int y1)
{
    const int xa = max(min(x0, x1), 0), xb = min(max(x0, x1), g.W - 1);
    const int ya = max(min(y0, y1), 0), yb = min(max(y0, y1), g.H - 1);
    if (xa > xb || ya > yb) return -__builtin_inff();
    const int tx0 = xa >> shift, tx1 = xb >> shift, ty0 = ya >> shift, ty1 = yb >> shift;
    const float a = t[ty0 * tw + tx0], b = t[ty0 * tw + tx1];
    const float c = t[ty1 * tw + tx0], d = t[ty1 * tw + tx1];
    return fmaxf(fmaxf(a, b), fmaxf(c, d));
}

// Ray height above the cell the walk stands on.
__device__ __forceinline__ float walk_height(const Grid& g, const Ray& r, const LineWalk& L)
{
    return ray_height(r.o_major + L.major(), g.res, r.s_major, r.inv_d, r.s_z, r.dz);
}

// walk_range with exact skipping.  The ray height is a composition of
// monotone binary32 operations of the cell's major index, so along any run
// of cells its smallest value is the one at an end of the run; a run whose
// cells' largest height `hmax` (from the block maxima) cannot meet the
// visit's condition at the lower of the two end heights is skipped without
// loading a cell: skip(hmax, z_first, z_last) must return true only if no
// cell with height <= hmax and ray height >= min(z_first, z_last) can make
// visit act.  Runs are 64 cells (checked against blocks of 64) and then 8
// cells (blocks of 8; a run spans at most two blocks each way, whose maxima
// are loaded together); the remaining cells are visited as walk_range does.
// `r` must be at the start cell.  Returns the number of cells loaded.
template <class Skip, class Visit>
__device__ __forceinline__ int walk_range_skip(const Grid& g, const Ray& r, const float* __restrict__ h,
                                               const TileMax& tm, int first, int count, Skip&& skip,
                                               Visit&& visit)
{
    constexpr int U = 8;
    const int end = first + count;  // one past the last intermediate cell
    int i = first;
    LineWalk L = r.L;
    L.jump_from_start(i - 1);  // on the cell before `i`
    int loaded = 0;
    while (i < end) {
        if (end - i >= 64) {
            LineWalk A = L;
            A.step();
            LineWalk E = r.L;
            E.jump_from_start(i + 63);
            const float hm = box_max2(g, tm.t64, tm.tw64, 6, A.x, A.y, E.x, E.y);
            if (skip(hm, walk_height(g, r, A), walk_height(g, r, E))) {
                L = E;
                i += 64;
                continue;
            }
        }
        // up to U cells: positions only (a few integer operations per cell);
        // ray heights, storage indices and loads only if the run may matter
        const int n = min(U, end - i);
        int px[U], py[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (u < n) L.step();
            px[u] = L.x;
            py[u] = L.y;
        }
        i += n;
        {
            LineWalk A = L, B = L;  // first and last cell of the run
            A.x = px[0];
            A.y = py[0];
            if (skip(box_max2(g, tm.t8, tm.tw8, 3, px[0], py[0], L.x, L.y), walk_height(g, r, A),
                     walk_height(g, r, B)))
                continue;
        }
        int st[U];
        float zr[U], hk[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            st[u] = -1;
            zr[u] = 0.0f;
            if (u < n && (r.all_inside || (px[u] >= 0 && px[u] < g.W && py[u] >= 0 && py[u] < g.H))) {
                st[u] = storage_index(g, px[u], py[u]);
                zr[u] = ray_height(r.o_major + (L.xmajor ? px[u] : py[u]), g.res, r.s_major, r.inv_d, r.s_z, r.dz);
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++) hk[u] = st[u] >= 0 ? h[st[u]] : __builtin_nanf("");
        bool stop = false;
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (st[u] >= 0) {
                loaded++;
                if (!stop && visit(st[u], hk[u], zr[u])) stop = true;
            }
        }
        if (stop) break;
    }
    return loaded;
}

}  // namespace memk
