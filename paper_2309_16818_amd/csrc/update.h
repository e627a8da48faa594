// update.h - per-item bodies of the map update kernels (device side).
//
// The single-map kernels (k_points.hip, k_image.hip, k_map.hip) and the
// batched persistent kernels (k_batch.hip) run exactly these functions, so a
// map updated inside a batch makes the same decisions and the same
// arithmetic as a map updated on its own.
#pragma once

#include "codec.h"
#include "fuse.h"
#include "geom.h"
#include "mem_internal.h"

namespace memk {

// Per-cloud accumulators of one map (storage-indexed).
struct Accum {
    int* cnt;
    float* wsum;
    float* ssum;
    float2* stash;
    int* clr;
    float* chsum;  // [Cb][HW]
    int HW;
};

// LDS hash table of one ingest workgroup.
struct IngestLds {
    int* key;
    int* cnt;
    float* w;
    float* s;
    float2* first;
    float* ch;  // [Cb][slots] or unused
    int slots_log2;
};

struct PointCounts {
    int acc = 0, nonfinite = 0, range = 0, outside = 0;
    int flushed = 0;  // cells whose sums this thread flushed with global atomics
    int ray_steps = 0;  // cells the clearing rays of this thread's points walk (when listed)
    int ray_segs = 0;   // the segments they are listed in
};

// Aggregates points [begin, end) of a cloud (at most 2^slots_log2 / 2
// points, and at most P per thread) into the LDS table, then flushes one
// global atomic per (cell, field).  A thread loads all its points before
// hashing any, so their loads overlap.  Every thread of the workgroup must
// call it; it starts and ends with a workgroup barrier.
// Class of a listed top-k index v among K classes, or -1 when v is not an
// integer in [0, K) (NaN included).
__device__ __forceinline__ int class_index(float v, int K)
{
    return (v >= 0.0f && v < (float)K && v == floorf(v)) ? (int)v : -1;
}

// The clearing march's segment lists (see k_points.hip): the ray of point
// i (index within the pass) with `steps` cells to walk gets its segments of
// kSegLen cells.  In two steps, so that the reservation's atomics are in
// flight while the caller does other work: march_reserve (every thread of
// the workgroup, with its P points, steps 0 for none) scans the workgroup's
// full segments, counts its partial ones per length class in LDS and lets
// threads 0..kSegLists-1 reserve room in sub-list (block id mod kSegSubs)
// of every list with one atomic each; march_write (every thread) writes
// the entries.  s_march: kMarchLds ints of LDS (s_cnt, s_base, one int per
// wave, at most 16 waves).  march_reserve starts with a barrier,
// march_write ends with one.
constexpr int kMarchLds = 2 * kSegLists + 16;  // ints of LDS the listing takes
template <int P>
struct MarchSlots {
    int fpos;     // first entry of this thread's full segments within the workgroup's
    int ppos[P];  // rank of each partial segment within its list
    int list[P];  // its list (1..4)
    int base;     // threads < kSegLists: the reservation in their list
};

template <int P>
__device__ __forceinline__ MarchSlots<P> march_reserve(const MarchBufs& mb, const int (&steps)[P], int* s_march)
{
    int* s_cnt = s_march;
    int* s_wave = s_march + 2 * kSegLists;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int sub = blockIdx.x % kSegSubs;
    MarchSlots<P> r;
    __syncthreads();
    if (t < kSegLists) s_cnt[t] = 0;
    int nfull = 0;
#pragma unroll
    for (int k = 0; k < P; k++) nfull += steps[k] / kSegLen;
    int incl = nfull;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(incl, o);
        if (lane >= o) incl += u;
    }
    if (lane == 63) s_wave[w] = incl;
    __syncthreads();
    r.fpos = incl - nfull;
    for (int k = 0; k < w; k++) r.fpos += s_wave[k];
#pragma unroll
    for (int k = 0; k < P; k++) {
        const int rem = steps[k] % kSegLen;
        r.list[k] = 1 + (kSegLen - 1 - rem) * 4 / kSegLen;  // for rem > 0: 1 (longest quarter) .. 4
        r.ppos[k] = rem > 0 ? atomicAdd(&s_cnt[r.list[k]], 1) : 0;
    }
    if (t == (int)blockDim.x - 1) s_cnt[0] = r.fpos + nfull;
    __syncthreads();
    r.base = 0;
    if (t < kSegLists && s_cnt[t] > 0) r.base = atomicAdd(&mb.counts[t * kSegSubs + sub], s_cnt[t]);
    return r;
}

template <int P>
__device__ __forceinline__ void march_write(const MarchBufs& mb, const int (&ri)[P], const int (&steps)[P],
                                            const MarchSlots<P>& r, int* s_march)
{
    int* s_base = s_march + kSegLists;
    const int t = threadIdx.x;
    const int sub = blockIdx.x % kSegSubs;
    if (t < kSegLists) s_base[t] = r.base;
    __syncthreads();
    // (the capacities bound every sub-list; the tests only guard them)
    int2* fl = mb.full + (int64_t)sub * mb.full_sub;
    int f = s_base[0] + r.fpos;
#pragma unroll
    for (int k = 0; k < P; k++) {
        const int nf = steps[k] / kSegLen, rem = steps[k] - nf * kSegLen;
        for (int j = 0; j < nf; j++, f++)
            if (f < mb.full_sub) fl[f] = make_int2(ri[k], j);
        const int l = r.list[k];
        if (rem > 0 && (int64_t)s_base[l] + r.ppos[k] < mb.part_sub)
            mb.part[((int64_t)(l - 1) * kSegSubs + sub) * mb.part_sub + s_base[l] + r.ppos[k]] = make_int2(ri[k], nf);
    }
    __syncthreads();
}

// Both steps at once.
template <int P>
__device__ __forceinline__ void march_lists(const MarchBufs& mb, const int (&ri)[P], const int (&steps)[P],
                                            int* s_march)
{
    const MarchSlots<P> r = march_reserve<P>(mb, steps, s_march);
    march_write<P>(mb, ri, steps, r, s_march);
}

template <int P>
__device__ __forceinline__ void ingest_range(const Grid& g, const float* __restrict__ xyz,
                                             int64_t begin, int64_t end,
                                             const float* __restrict__ ch, const Pose& T, float c0,
                                             float c1, float mr2, const PointBinds& pb,
                                             const Accum& acc, const IngestLds& lds,
                                             PointCounts& pc, bool march = false,
                                             const MarchBufs& mb = MarchBufs{}, int* s_march = nullptr)
{
    const int slots = 1 << lds.slots_log2;
    const int nthr = blockDim.x;
    const bool lds_ch = pb.lds_ch != 0;
    __syncthreads();
    for (int i = threadIdx.x; i < slots; i += nthr) {
        lds.key[i] = -1;
        lds.cnt[i] = 0;
        lds.w[i] = 0.0f;
        lds.s[i] = 0.0f;
    }
    if (lds_ch)
        for (int i = threadIdx.x; i < slots * pb.Cb; i += nthr) lds.ch[i] = 0.0f;
    __syncthreads();

    float in[P][3];
    int msteps[P], mri[P];
#pragma unroll
    for (int k = 0; k < P; k++) {
        const int64_t i = begin + threadIdx.x + (int64_t)k * nthr;
        msteps[k] = 0;
        mri[k] = (int)i;
        if (i < end) {
            in[k][0] = xyz[3 * i];
            in[k][1] = xyz[3 * i + 1];
            in[k][2] = xyz[3 * i + 2];
        }
    }
    if (march) {
        // the clearing rays of the accepted points (cell decisions as below)
        int ax, ay;
        lattice_cell(g, T.m[3], T.m[7], ax, ay);
#pragma unroll
        for (int k = 0; k < P; k++) {
            const int64_t i = begin + threadIdx.x + (int64_t)k * nthr;
            float px, py, pz, r2;
            int ix, iy;
            if (i < end && point_cell(g, T, mr2, in[k][0], in[k][1], in[k][2], px, py, pz, r2, ix, iy) == 0) {
                msteps[k] = max(max(abs(ix - ax), abs(iy - ay)) - 1, 0);
                pc.ray_steps += msteps[k];
                pc.ray_segs += (msteps[k] + kSegLen - 1) / kSegLen;
                if (msteps[k] > 0) {
                    const Ray ray(g, ax, ay, ix, iy, T.m[3], T.m[7], T.m[11], px, py, pz);
                    mb.rec[i] = make_float4(ray.inv_d, ray.dz, __int_as_float(ix | (iy << 16)), 0.0f);
                }
            }
        }
    }
    // the reservation's atomics stay in flight during the hashing below
    MarchSlots<P> mslots;
    if (march) mslots = march_reserve<P>(mb, msteps, s_march);
#pragma unroll
    for (int k = 0; k < P; k++) {
        const int64_t i = begin + threadIdx.x + (int64_t)k * nthr;
        if (i >= end) break;
        float px, py, pz, r2;
        int ix, iy;
        int r = point_cell(g, T, mr2, in[k][0], in[k][1], in[k][2], px, py, pz, r2, ix, iy);
        if (r != 0) {
            pc.nonfinite += (r == -1);
            pc.range += (r == -2);
            pc.outside += (r == -3);
            continue;
        }
        pc.acc++;
        const int st = storage_index(g, ix, iy);
        const float sig = c0 + c1 * r2;
        const float var = sig * sig;
        const float w = 1.0f / var;
        // Slot: the cell's index within its aligned block of `slots` cells,
        // xored with a hash of the block in multiples of 16.  Cells that are
        // neighbours in memory stay neighbours in the table (each aligned
        // group of 16 cells in one aligned group of 16 slots), so the lanes
        // of the flush below, which take consecutive slots, add into
        // consecutive cells and the memory side merges their atomics per
        // cache line; distinct blocks spread over the table.
        const unsigned blk = (unsigned)st >> lds.slots_log2;
        int slot = (int)(((unsigned)st ^ ((blk * 2654435761u) << 4)) & (unsigned)(slots - 1));
        for (;;) {
            int old = atomicCAS(&lds.key[slot], -1, st);
            if (old == -1) {
                lds.first[slot] = make_float2(pz, var);
                break;
            }
            if (old == st) break;
            slot = (slot + 1) & (slots - 1);
        }
        atomicAdd(&lds.cnt[slot], 1);
        atomicAdd(&lds.w[slot], w);
        atomicAdd(&lds.s[slot], pz * w);
        for (int b = 0; b < pb.n; b++) {
            const float* src = ch + i * pb.c_in + pb.b[b].ch_first;
            const int k = pb.b[b].topk;
            // dense: channel q into plane q; top-k: the q-th listed
            // probability into its class's plane
            for (int q = 0; q < (k > 0 ? k : pb.b[b].C); q++) {
                const int c = k > 0 ? class_index(src[q], pb.b[b].C) : q;
                if (c < 0) continue;
                const float val = src[k > 0 ? k + q : q];
                const int plane = pb.b[b].sum_off + c;
                if (lds_ch)
                    atomicAdd(&lds.ch[plane * slots + slot], val);
                else
                    unsafeAtomicAdd(&acc.chsum[(int64_t)plane * acc.HW + st], val);
            }
        }
    }
    if (march) march_write<P>(mb, mri, msteps, mslots, s_march);
    __syncthreads();

    // Flush: one global atomic per (cell, field) seen by this workgroup.
    for (int slot = threadIdx.x; slot < slots; slot += nthr) {
        const int st = lds.key[slot];
        if (st < 0) continue;
        pc.flushed++;
        const int c = lds.cnt[slot];
        atomicAdd(&acc.cnt[st], c);
        unsafeAtomicAdd(&acc.wsum[st], lds.w[slot]);
        unsafeAtomicAdd(&acc.ssum[st], lds.s[slot]);
        // A cell whose only point in the whole cloud is this one takes
        // (z, v) verbatim; any other writer implies a count above one.
        if (c == 1) acc.stash[st] = lds.first[slot];
        if (lds_ch)
            for (int q = 0; q < pb.Cb; q++)
                unsafeAtomicAdd(&acc.chsum[(int64_t)q * acc.HW + st], lds.ch[q * slots + slot]);
    }
    __syncthreads();
}

// Clearing vote of a cell reached by a walk over logical-order heights: the
// ray passes below the cell's height by more than the margin (NaN, no
// height, never votes).  The vote is counted in the storage-order layer, so
// the logical index is converted only for the rare cells that vote.
struct ClearVoteLogical {
    int* clr;  // storage order
    Grid g;    // the map's grid with its ring offsets
    float margin;
    __device__ __forceinline__ bool votes(float hk, float zr) const { return hk > zr + margin; }
    __device__ __forceinline__ void add(int lin) const
    {
        const int y = lin / g.W, x = lin - y * g.W;
        atomicAdd(&clr[storage_index(g, x, y)], 1);
    }
    __device__ __forceinline__ bool operator()(int lin, float hk, float zr) const
    {
        if (votes(hk, zr)) add(lin);
        return false;
    }
};

// walk_range_logical for the clearing votes: each batch's U comparisons are
// taken without a branch and the rare votes added afterwards, one atomic per
// voting cell (the same votes as visiting the cells one by one).
template <int U>
__device__ __forceinline__ int walk_votes(const Grid& g, Ray& r, const float* __restrict__ h, int first,
                                          int count, const ClearVoteLogical& vote)
{
    r.L.jump_from_start(first - 1);
    r.L.steps = count + 1;
    ClearVoteLogical v = vote;
    return walk_logical_batches<U>(g, r, h, v,
                                   [&](const int (&s_)[U], const float (&z_)[U], const float (&h_)[U], int n) {
                                       unsigned m = 0;
#pragma unroll
                                       for (int u = 0; u < U; u++)
                                           m |= (unsigned)(u < n && vote.votes(h_[u], z_[u])) << u;
                                       if (m) {
#pragma unroll
                                           for (int u = 0; u < U; u++)
                                               if ((m >> u) & 1u) vote.add(s_[u]);
                                       }
                                       return false;
                                   });
}

// Orders a workgroup's 256 rays by length bucket of 8 cells (bucket 0: no
// cell; the last bucket takes every ray longer than 8 (NB - 2) cells) with
// a counting sort in LDS, so that each wave walks rays of similar length.
// Returns the thread whose ray this thread walks; s_off[b] is left holding
// the first position of bucket b.  Every thread of the workgroup must call
// it; it ends with a barrier.
template <int NB>
__device__ __forceinline__ int order_by_length(int steps, int* s_off, int* s_order)
{
    const int t = threadIdx.x;
    if (t < NB) s_off[t] = 0;
    __syncthreads();
    const int bucket = min((steps + 7) >> 3, NB - 1);
    const int pos = atomicAdd(&s_off[bucket], 1);  // rank within the bucket
    __syncthreads();
    if (t == 0) {
        int acc = 0;
        for (int q = 0; q < NB; q++) {
            const int c = s_off[q];
            s_off[q] = acc;
            acc += c;
        }
    }
    __syncthreads();
    s_order[s_off[bucket] + pos] = t;
    __syncthreads();
    return s_order[t];
}

// Height fusion, clearing and bound point channels of storage cell st from
// the cloud's sums for the cell, read through S: S.n() points, S.w() = sum
// of 1/v, S.s() = sum of z/v, S.first() = (z, v) of its only point when
// n = 1, S.ch(plane) = a bound channel's sum (the sums are read only for a
// cell with points).  votes() gives the cell's clearing votes (read only
// for a cell without points).  Returns 1 if the cell received points, 2 if
// it was cleared, else 0.
template <class Sums, class Votes>
__device__ __forceinline__ int fuse_cell(int st, const Sums& S, int clear_min, float* __restrict__ h,
                                         float* __restrict__ v, const PointBinds& pb, Votes&& votes)
{
    const int N = S.n();
    if (N == 0) {
        if (clear_min > 0 && votes() >= clear_min && !isnan(h[st])) {
            h[st] = __uint_as_float(0x7fc00000u);
            return 2;
        }
        return 0;
    }
    const float hv = h[st];
    float hn, vn;
    if (!isnan(hv)) {  // prior plus the cloud, information form
        const float vv = v[st];
        vn = 1.0f / (1.0f / vv + S.w());
        hn = vn * (hv / vv + S.s());
    } else if (N == 1) {  // a single point sets an empty cell exactly
        const float2 zv = S.first();
        hn = zv.x;
        vn = zv.y;
    } else {
        vn = 1.0f / S.w();
        hn = S.s() * vn;
    }
    h[st] = hn;
    v[st] = vn;
    for (int b = 0; b < pb.n; b++) {
        const LayerDev& L = pb.L[b];
        const int C = pb.b[b].C, off = pb.b[b].sum_off;
        GaussCoef gc{0.0f, 1.0f, 0.0f, true};
        if (L.rule == MEM_GAUSS) gc = gauss_coef(L.param, L.var[st], N);
        for (int q = 0; q < C; q++) {
            const float sum = S.ch(off + q);
            const float a = sum / (float)N;
            const int64_t idx = (int64_t)st * C + q;
            const float old = layer_load(L.val, L.storage, L.scale, idx, q);
            layer_store(L.val, L.storage, L.scale, idx, q, fuse_value(L.rule, L.param, old, a, sum, gc));
        }
        if (L.rule == MEM_GAUSS) L.var[st] = gc.var;
    }
    return 1;
}

// The sums of storage cell st in the per-cloud accumulator arrays.
struct AccumSums {
    const Accum& acc;
    int st;
    __device__ __forceinline__ int n() const { return acc.cnt[st]; }
    __device__ __forceinline__ float w() const { return acc.wsum[st]; }
    __device__ __forceinline__ float s() const { return acc.ssum[st]; }
    __device__ __forceinline__ float2 first() const { return acc.stash[st]; }
    __device__ __forceinline__ float ch(int plane) const { return acc.chsum[(int64_t)plane * acc.HW + st]; }
};

// fuse_cell from the accumulator arrays.
template <class Votes>
__device__ __forceinline__ int finalize_cell_v(int st, const Accum& acc, int clear_min,
                                               float* __restrict__ h, float* __restrict__ v,
                                               const PointBinds& pb, Votes&& votes)
{
    return fuse_cell(st, AccumSums{acc, st}, clear_min, h, v, pb, votes);
}

// finalize_cell_v with the votes in acc.clr at the same storage index.
__device__ __forceinline__ int finalize_cell(int st, const Accum& acc, int clear_min,
                                             float* __restrict__ h, float* __restrict__ v,
                                             const PointBinds& pb)
{
    return finalize_cell_v(st, acc, clear_min, h, v, pb, [&] { return acc.clr[st]; });
}

// Association of logical cell (ix, iy) with every image of one camera pose
// (Sec. III-B, Fig. 3).  code[k] = pixel, or -1 no height, -2 outside image
// k's view, -3 occluded.  Returns the number of in-grid cells the occlusion
// walk loaded; in_view counts the images whose view holds the cell.
// Frustum test and pixel of logical cell (ix, iy) in every image of one
// camera pose, without the occlusion walk.  code[k] = pixel, or -1 no
// height, -2 outside image k's view.  Returns the number of images whose
// view holds the cell.
__device__ __forceinline__ int view_cell(const Grid& g, const Camera& cam,
                                         const float* __restrict__ h, int ix, int iy, int st,
                                         int (&code)[kMaxImages])
{
#pragma unroll
    for (int k = 0; k < kMaxImages; k++) code[k] = -1;
    const float hj = h[st];
    if (isnan(hj)) return 0;
    const float* T = cam.T.m;
    const float xc = ((float)(g.ox + ix) + 0.5f) * g.res;
    const float yc = ((float)(g.oy + iy) + 0.5f) * g.res;
    const float dx = xc - T[3], dy = yc - T[7], dz = hj - T[11];
    float P[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {  // R^T d
        float a = T[0 + k] * dx;
        float b = T[4 + k] * dy;
        float c = T[8 + k] * dz;
        float s = a + b;
        P[k] = s + c;
    }
    int in_view = 0;
#pragma unroll
    for (int k = 0; k < kMaxImages; k++) {
        if (k >= cam.n) break;
        code[k] = -2;
        if (P[2] > cam.min_depth) {
            float u = cam.fx[k] * P[0];
            u = u / P[2];
            u = u + cam.cx[k];
            float v = cam.fy[k] * P[1];
            v = v / P[2];
            v = v + cam.cy[k];
            const float uf = floorf(u + 0.5f);
            const float vf = floorf(v + 0.5f);
            if (uf >= 0.0f && uf < (float)cam.w[k] && vf >= 0.0f && vf < (float)cam.h[k]) {
                code[k] = (int)vf * cam.w[k] + (int)uf;
                in_view++;
            }
        }
    }
    return in_view;
}

__device__ __forceinline__ int project_cell(const Grid& g, const Camera& cam,
                                            const float* __restrict__ h, int ix, int iy, int st,
                                            int (&code)[kMaxImages], int& in_view)
{
#pragma unroll
    for (int k = 0; k < kMaxImages; k++) code[k] = -1;
    in_view = 0;
    const float hj = h[st];
    if (isnan(hj)) return 0;
    const float* T = cam.T.m;
    const float xc = ((float)(g.ox + ix) + 0.5f) * g.res;
    const float yc = ((float)(g.oy + iy) + 0.5f) * g.res;
    const float dx = xc - T[3], dy = yc - T[7], dz = hj - T[11];
    float P[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {  // R^T d
        float a = T[0 + k] * dx;
        float b = T[4 + k] * dy;
        float c = T[8 + k] * dz;
        float s = a + b;
        P[k] = s + c;
    }
    bool any = false;
#pragma unroll
    for (int k = 0; k < kMaxImages; k++) {
        if (k >= cam.n) break;
        code[k] = -2;
        if (P[2] > cam.min_depth) {
            float u = cam.fx[k] * P[0];
            u = u / P[2];
            u = u + cam.cx[k];
            float v = cam.fy[k] * P[1];
            v = v / P[2];
            v = v + cam.cy[k];
            const float uf = floorf(u + 0.5f);
            const float vf = floorf(v + 0.5f);
            if (uf >= 0.0f && uf < (float)cam.w[k] && vf >= 0.0f && vf < (float)cam.h[k]) {
                code[k] = (int)vf * cam.w[k] + (int)uf;
                in_view++;
                any = true;
            }
        }
    }
    if (!any) return 0;
    // One occlusion walk serves every image of this pose.
    int ax, ay;
    lattice_cell(g, T[3], T[7], ax, ay);
    Ray ray(g, ax, ay, ix, iy, T[3], T[7], T[11], xc, yc, hj);
    bool occluded = false;
    const int visited = walk_cells<8>(g, ray, h, [&](int, float hk, float zr) {
        if (hk >= zr) occluded = true;  // NaN (no height) never occludes
        return occluded;
    });
    if (occluded)
#pragma unroll
        for (int k = 0; k < kMaxImages; k++)
            if (code[k] >= 0) code[k] = -3;
    return visited;
}

// Wave-aggregated append of (st, code) for the lanes with code >= 0.  All
// lanes of the wave must call it.
__device__ __forceinline__ void append_pair(bool vis, int st, int code, int2* __restrict__ list,
                                            int* __restrict__ count)
{
    const unsigned long long mask = __ballot(vis);
    if (!mask) return;
    const int lane = __lane_id();
    const int leader = __ffsll((long long)mask) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(count, __popcll(mask));
    base = __shfl(base, leader);
    if (vis) {
        const int rank = __popcll(mask & ((1ull << lane) - 1ull));
        list[base + rank] = make_int2(st, code);
    }
}

template <int IMG>
__device__ __forceinline__ float pixel_value(const void* img, int64_t off)
{
    if (IMG == MEM_U8) return (float)((const uint8_t*)img)[off] / 255.0f;
    return ((const float*)img)[off];
}

// A class index as an input carries it: u8 images the byte itself.
template <int IMG>
__device__ __forceinline__ float pixel_index(const void* img, int64_t off)
{
    if (IMG == MEM_U8) return (float)((const uint8_t*)img)[off];
    return ((const float*)img)[off];
}

// Top-k class input of one visible pair (Eq. (12) with the K-vector that
// holds each listed probability at its class): one lane adds the k
// probabilities to the cell's concentrations in list order, so a class
// listed twice adds twice.  Dirichlet layers are binary32.
template <int IMG>
__device__ __forceinline__ void gather_topk(int2 pr, const void* __restrict__ img, int64_t s0, int64_t s1,
                                            int64_t s2, int w, int ch_first, const LayerDev& L, int k)
{
    const int st = pr.x;
    const int row = pr.y / w, col = pr.y - (pr.y / w) * w;
    const int64_t pix = (int64_t)row * s0 + (int64_t)col * s1 + (int64_t)ch_first * s2;
    float* alpha = (float*)L.val + (int64_t)st * L.C;
    for (int q = 0; q < k; q++) {
        const int c = class_index(pixel_index<IMG>(img, pix + (int64_t)q * s2), L.C);
        if (c >= 0) alpha[c] += pixel_value<IMG>(img, pix + (int64_t)(k + q) * s2);
    }
}

// Fuses channels q0, q0 + LPP, ... of one visible pair's pixel into layer L
// (N = 1).  The LPP lanes of a pair call it together; lane q0 == 0 writes
// the Gaussian variance.
template <int IMG, int S>
__device__ __forceinline__ void gather_pair(int2 pr, const void* __restrict__ img, int64_t s0,
                                            int64_t s1, int64_t s2, int w, int ch_first,
                                            const LayerDev& L, int q0, int LPP)
{
    const int st = pr.x;
    const int row = pr.y / w, col = pr.y - (pr.y / w) * w;
    const int64_t pix = (int64_t)row * s0 + (int64_t)col * s1 + (int64_t)ch_first * s2;
    GaussCoef gc{0.0f, 1.0f, 0.0f, true};
    if (L.rule == MEM_GAUSS) gc = gauss_coef(L.param, L.var[st], 1);
    const int C = L.C;
    for (int q = q0; q < C; q += LPP) {
        const float m = pixel_value<IMG>(img, pix + (int64_t)q * s2);
        const int64_t idx = (int64_t)st * C + q;
        const float sc = S == MEM_FP8_E4M3 ? L.scale[q] : 1.0f;
        const float old = Store<S>::load(L.val, idx, sc);
        Store<S>::store(L.val, idx, fuse_value(L.rule, L.param, old, m, m, gc), sc);
    }
    if (L.rule == MEM_GAUSS && q0 == 0) L.var[st] = gc.var;
}

// NW consecutive 32-bit words at p (aligned to min(4 NW, 16) bytes) in
// loads / stores of up to 16 bytes.
template <int NW>
__device__ __forceinline__ void load_words(const void* __restrict__ p, uint32_t (&w)[NW])
{
    if constexpr (NW % 4 == 0) {
#pragma unroll
        for (int i = 0; i < NW / 4; i++) {
            const uint4 v = ((const uint4*)p)[i];
            w[4 * i] = v.x;
            w[4 * i + 1] = v.y;
            w[4 * i + 2] = v.z;
            w[4 * i + 3] = v.w;
        }
    } else if constexpr (NW == 2) {
        const uint2 v = *(const uint2*)p;
        w[0] = v.x;
        w[1] = v.y;
    } else {
        static_assert(NW == 1, "1, 2 or a multiple of 4 words");
        w[0] = *(const uint32_t*)p;
    }
}

template <int NW>
__device__ __forceinline__ void store_words(void* __restrict__ p, const uint32_t (&w)[NW])
{
    if constexpr (NW % 4 == 0) {
#pragma unroll
        for (int i = 0; i < NW / 4; i++)
            ((uint4*)p)[i] = make_uint4(w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3]);
    } else if constexpr (NW == 2) {
        *(uint2*)p = make_uint2(w[0], w[1]);
    } else {
        static_assert(NW == 1, "1, 2 or a multiple of 4 words");
        *(uint32_t*)p = w[0];
    }
}

// Element k of a little-endian run of B-byte elements held in words.
template <int B, int NW>
__device__ __forceinline__ uint32_t word_elem(const uint32_t (&w)[NW], int k)
{
    if constexpr (B == 4) return w[k];
    constexpr int per = 4 / B;
    return (w[k / per] >> (8 * B * (k % per))) & ((1u << (8 * B)) - 1u);
}

// The FP8 scales of the V channels from q and their binary32 reciprocals;
// 1 for other storage types.
template <int S, int V>
struct ChanScales {
    float sc[V];
    float rc[V];
    __device__ __forceinline__ void load(const LayerDev& L, int q)
    {
#pragma unroll
        for (int k = 0; k < V; k++) {
            sc[k] = 1.0f;
            rc[k] = 1.0f;
        }
        if constexpr (S == MEM_FP8_E4M3) {
            uint32_t ws[V], wr[V];
            load_words(L.scale + q, ws);
            load_words(L.rscale + q, wr);
#pragma unroll
            for (int k = 0; k < V; k++) {
                sc[k] = __uint_as_float(ws[k]);
                rc[k] = __uint_as_float(wr[k]);
            }
        }
    }
};

// gather_pair with V consecutive channels per lane: one pass moves 4V image
// bytes and V storage elements per lane in word loads and stores (16 bytes
// of FP32 or BF16 storage, 8 of FP8), so a BF16 row takes half FP32's
// memory instructions.  The per-element arithmetic is gather_pair's, so
// both give the same bits.  Needs C % V == 0 and the pixel's channels
// contiguous (s2 == 1) at an offset that is a multiple of V.
template <int IMG, int S, int V, int R>
__device__ __forceinline__ void gather_pair_vec_rule(int2 pr, const void* __restrict__ img, int64_t s0,
                                                     int64_t s1, int w, int ch_first, const LayerDev& L,
                                                     int q0, int LPP)
{
    constexpr int B = S == MEM_F32 ? 4 : S == MEM_BF16 ? 2 : 1;
    constexpr int NW = V * B / 4;                  // storage words per lane and pass
    constexpr int NI = IMG == MEM_U8 ? V / 4 : V;  // image words
    static_assert(V * B % 4 == 0 && (IMG != MEM_U8 || V % 4 == 0), "whole words");
    const int st = pr.x;
    const int row = pr.y / w, col = pr.y - (pr.y / w) * w;
    const int64_t pix = (int64_t)row * s0 + (int64_t)col * s1 + ch_first;
    GaussCoef gc{0.0f, 1.0f, 0.0f, true};
    if constexpr (R == MEM_GAUSS) gc = gauss_coef(L.param, L.var[st], 1);
    const int C = L.C;
    for (int q = q0 * V; q < C; q += LPP * V) {
        ChanScales<S, V> cs;  // (keeping a lane's scales across passes measured no faster)
        cs.load(L, q);
        uint32_t wi[NI], wv[NW], out[NW];
        static_assert(S != MEM_FP8_E4M3 || V % 4 == 0, "whole words of FP8 codes");
        load_words(IMG == MEM_U8 ? (const void*)((const uint8_t*)img + pix + q)
                                 : (const void*)((const float*)img + pix + q), wi);
        uint8_t* row_p = (uint8_t*)L.val + ((int64_t)st * C + q) * B;
        load_words(row_p, wv);
        float nv[V];
#pragma unroll
        for (int k = 0; k < V; k++) {
            const uint32_t pe = word_elem<IMG == MEM_U8 ? 1 : 4>(wi, k);
            const float a = IMG == MEM_U8 ? (float)pe / 255.0f : __uint_as_float(pe);
            float old;
            if constexpr (S == MEM_F32) old = __uint_as_float(wv[k]);
            else if constexpr (S == MEM_BF16) old = bf16_to_f32((uint16_t)word_elem<2>(wv, k));
            else old = e4m3_word_to_f32(wv[k / 4], k % 4) * cs.sc[k];
            nv[k] = fuse_rule<R>(L.param, old, a, a, gc);
        }
#pragma unroll
        for (int i = 0; i < NW; i++) {
            if constexpr (S == MEM_F32) out[i] = __float_as_uint(nv[i]);
            else if constexpr (S == MEM_BF16)
                out[i] = (uint32_t)f32_to_bf16(nv[2 * i]) | ((uint32_t)f32_to_bf16(nv[2 * i + 1]) << 16);
            else  // v / sc[k] through the reciprocal, corrected: the correctly rounded quotient
                out[i] = f32x4_to_e4m3(div_rcp(nv[4 * i], cs.sc[4 * i], cs.rc[4 * i]),
                                       div_rcp(nv[4 * i + 1], cs.sc[4 * i + 1], cs.rc[4 * i + 1]),
                                       div_rcp(nv[4 * i + 2], cs.sc[4 * i + 2], cs.rc[4 * i + 2]),
                                       div_rcp(nv[4 * i + 3], cs.sc[4 * i + 3], cs.rc[4 * i + 3]));
        }
        store_words(row_p, out);
    }
    if (R == MEM_GAUSS && q0 == 0) L.var[st] = gc.var;
}

// The rule as a compile-time constant, so that no element pays for the choice.
template <int IMG, int S, int V>
__device__ __forceinline__ void gather_pair_vec(int2 pr, const void* __restrict__ img, int64_t s0,
                                                int64_t s1, int w, int ch_first, const LayerDev& L,
                                                int q0, int LPP)
{
    switch (L.rule) {
    case MEM_LATEST:
        gather_pair_vec_rule<IMG, S, V, MEM_LATEST>(pr, img, s0, s1, w, ch_first, L, q0, LPP);
        break;
    case MEM_EXPAVG:
        gather_pair_vec_rule<IMG, S, V, MEM_EXPAVG>(pr, img, s0, s1, w, ch_first, L, q0, LPP);
        break;
    case MEM_GAUSS:
        gather_pair_vec_rule<IMG, S, V, MEM_GAUSS>(pr, img, s0, s1, w, ch_first, L, q0, LPP);
        break;
    default:
        gather_pair_vec_rule<IMG, S, V, MEM_DIRICHLET>(pr, img, s0, s1, w, ch_first, L, q0, LPP);
        break;
    }
}

// Channels per lane of the vector gather for a layer of storage S (4 FP32,
// 8 BF16, 8 FP8: 16 bytes of storage, 8 for FP8, whose 8 scales and
// reciprocals a lane keeps in registers) where the layer's rows, the
// pixel's channels and every address allow it, else 1.
inline int gather_vec_width(int storage, int C, int img_dtype, const void* img, int64_t s0, int64_t s1,
                            int64_t s2, int ch_first, const LayerDev& L)
{
    const int V = storage == MEM_F32 ? 4 : 8;
    const int ib = img_dtype == MEM_U8 ? 1 : 4;
    const int64_t ia = V * ib < 16 ? V * ib : 16;  // alignment of the image loads
    const bool ok = C % V == 0 && s2 == 1 && s0 % V == 0 && s1 % V == 0 && ch_first % V == 0 &&
                    (uintptr_t)img % ia == 0 && (uintptr_t)L.val % 16 == 0 &&
                    (storage != MEM_FP8_E4M3 || ((uintptr_t)L.scale % 16 == 0 && L.rscale));
    return ok ? V : 1;
}

// log2 of the lanes that share one (cell, image) pair: enough for the
// pair's groups of V channels in one pass (at most 64 lanes), or 32 or 16
// lanes over several passes where that leaves fewer lanes idle (ties keep
// the wider group, with fewer passes).  384 channels in groups of 8 take 16
// lanes over three passes rather than 64 lanes with 16 idle.  Which lane
// takes an element does not change its arithmetic.  Top-k inputs take one
// lane per pair.
inline int gather_lanes_log2(int C, int V, bool topk)
{
    if (topk) return 0;
    const int G = (C + V - 1) / V;
    auto slots = [G](int lg) { return ((G + (1 << lg) - 1) >> lg) << lg; };
    int l = 0;
    while ((1 << l) < G && l < 6) l++;
    int best = l;
    for (int lg = l - 1; lg >= 4; lg--)
        if (slots(lg) < slots(best)) best = lg;
    return best;
}

// An empty cell: no height, never observed layers, Dirichlet alpha_0.
__device__ __forceinline__ void reset_cell(int st, float* __restrict__ h, float* __restrict__ v,
                                           int* __restrict__ cnt, int* __restrict__ clr,
                                           const LayerDev* L, int nL)
{
    h[st] = __builtin_nanf("");
    v[st] = __builtin_inff();
    cnt[st] = 0;
    clr[st] = 0;
    for (int l = 0; l < nL; l++) {
        const float init = (L[l].rule == MEM_DIRICHLET) ? L[l].param : __builtin_nanf("");
        for (int q = 0; q < L[l].C; q++)
            layer_store(L[l].val, L[l].storage, L[l].scale, (int64_t)st * L[l].C + q, q, init);
        if (L[l].rule == MEM_GAUSS) L[l].var[st] = __builtin_inff();
    }
}

}  // namespace memk
