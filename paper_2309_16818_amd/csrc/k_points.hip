// k_points.hip - point-cloud path of the map update.
//
//   k_zero_accum   clears the per-cloud accumulators (dense, HBM-bound).
//   k_ingest       point transform + cell association (Sec. III-B) and
//                  LDS-binned per-cell sums: a workgroup hashes its 1024
//                  points into an LDS table keyed by cell, reduces equal cells
//                  with LDS atomics, then issues one global atomic per
//                  (cell, field) it saw.
//   k_clear_march  the ray cast of Table I's "height update & ray cast":
//                  one ray per accepted point along Bresenham's line, voting
//                  to clear cells whose height lies above the ray.
//   k_finalize     per-cell information-form Gaussian height fusion, clear
//                  application, and fusion of bound point channels with the
//                  layer's rule (Sec. III-C, Eq. (1), (2), (6)-(7), (12)).
#include "codec.h"
#include "fuse.h"
#include "geom.h"
#include "mem_internal.h"

namespace memk {

namespace {

constexpr int kWG = 256;
constexpr int kPPT = 4;
constexpr int kChunk = kWG * kPPT;  // points per ingest workgroup
constexpr int kSlotsLog2 = 11;
constexpr int kSlots = 1 << kSlotsLog2;  // LDS hash slots (2 x points)
constexpr int kMaxLdsCh = 16;            // bound channels reduced in LDS at most
constexpr size_t kStaticLds = sizeof(int) * 2 * kSlots + sizeof(float) * 2 * kSlots + sizeof(float2) * kSlots;

static_assert(kSlots >= 2 * kChunk, "hash table must never fill");

__global__ __launch_bounds__(256) void k_zero_accum(int HW, int* __restrict__ n,
                                                    float* __restrict__ wsum,
                                                    float* __restrict__ ssum,
                                                    int* __restrict__ clr,
                                                    float* __restrict__ chsum, int Cb)
{
    int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < HW; i += stride) {
        n[i] = 0;
        wsum[i] = 0.0f;
        ssum[i] = 0.0f;
        clr[i] = 0;
        for (int q = 0; q < Cb; q++) chsum[(int64_t)q * HW + i] = 0.0f;
    }
}

__global__ __launch_bounds__(kWG) void k_ingest(Grid g, const float* __restrict__ xyz, int64_t n,
                                                const float* __restrict__ ch, Pose T, float c0,
                                                float c1, float mr2, PointBinds pb,
                                                int* __restrict__ cnt, float* __restrict__ wsum,
                                                float* __restrict__ ssum,
                                                float2* __restrict__ stash,
                                                float* __restrict__ chsum,
                                                unsigned long long* __restrict__ stats)
{
    __shared__ int s_key[kSlots];
    __shared__ int s_cnt[kSlots];
    __shared__ float s_w[kSlots];
    __shared__ float s_s[kSlots];
    __shared__ float2 s_first[kSlots];
    extern __shared__ float s_ch[];  // [Cb][kSlots] when Cb <= kMaxLdsCh

    const int HW = g.W * g.H;
    const bool lds_ch = pb.lds_ch != 0;
    for (int i = threadIdx.x; i < kSlots; i += kWG) {
        s_key[i] = -1;
        s_cnt[i] = 0;
        s_w[i] = 0.0f;
        s_s[i] = 0.0f;
    }
    if (lds_ch)
        for (int i = threadIdx.x; i < kSlots * pb.Cb; i += kWG) s_ch[i] = 0.0f;
    __syncthreads();

    const int64_t base = (int64_t)blockIdx.x * kChunk;
    int n_acc = 0, n_nf = 0, n_rg = 0, n_out = 0;
#pragma unroll
    for (int k = 0; k < kPPT; k++) {
        int64_t i = base + k * kWG + threadIdx.x;
        if (i >= n) break;
        float x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        float px, py, pz, r2;
        int ix, iy;
        int r = point_cell(g, T, mr2, x, y, z, px, py, pz, r2, ix, iy);
        if (r != 0) {
            n_nf += (r == -1);
            n_rg += (r == -2);
            n_out += (r == -3);
            continue;
        }
        n_acc++;
        int st = storage_index(g, ix, iy);
        float sig = c0 + c1 * r2;
        float var = sig * sig;
        float w = 1.0f / var;
        int slot = (int)(((unsigned)st * 2654435761u) >> (32 - kSlotsLog2));
        for (;;) {
            int old = atomicCAS(&s_key[slot], -1, st);
            if (old == -1) {
                s_first[slot] = make_float2(pz, var);
                break;
            }
            if (old == st) break;
            slot = (slot + 1) & (kSlots - 1);
        }
        atomicAdd(&s_cnt[slot], 1);
        atomicAdd(&s_w[slot], w);
        atomicAdd(&s_s[slot], pz * w);
        for (int b = 0; b < pb.n; b++) {
            const float* src = ch + i * pb.c_in + pb.b[b].ch_first;
            for (int q = 0; q < pb.b[b].C; q++) {
                int plane = pb.b[b].sum_off + q;
                if (lds_ch)
                    atomicAdd(&s_ch[plane * kSlots + slot], src[q]);
                else
                    unsafeAtomicAdd(&chsum[(int64_t)plane * HW + st], src[q]);
            }
        }
    }
    wave_stat_add(&stats[ST_ACCEPTED], n_acc);
    wave_stat_add(&stats[ST_NONFINITE], n_nf);
    wave_stat_add(&stats[ST_RANGE], n_rg);
    wave_stat_add(&stats[ST_OUTSIDE], n_out);
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&stats[ST_POINTS_IN], (unsigned long long)n);
    __syncthreads();

    // Flush: one global atomic per (cell, field) seen by this workgroup.
    for (int slot = threadIdx.x; slot < kSlots; slot += kWG) {
        int st = s_key[slot];
        if (st < 0) continue;
        int c = s_cnt[slot];
        atomicAdd(&cnt[st], c);
        unsafeAtomicAdd(&wsum[st], s_w[slot]);
        unsafeAtomicAdd(&ssum[st], s_s[slot]);
        // A cell whose only point in the whole cloud is this one takes
        // (z, v) verbatim; any other writer implies a count above one.
        if (c == 1) stash[st] = s_first[slot];
        if (lds_ch)
            for (int q = 0; q < pb.Cb; q++)
                unsafeAtomicAdd(&chsum[(int64_t)q * HW + st], s_ch[q * kSlots + slot]);
    }
}

__global__ __launch_bounds__(256) void k_clear_march(Grid g, const float* __restrict__ xyz,
                                                     int64_t n, Pose T, float mr2, float margin,
                                                     const float* __restrict__ h,
                                                     int* __restrict__ clr,
                                                     unsigned long long* __restrict__ stats)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int visited = 0;
    if (i < n) {
        float px, py, pz, r2;
        int ix, iy;
        int r = point_cell(g, T, mr2, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], px, py, pz, r2,
                           ix, iy);
        if (r == 0) {
            const float sx = T.m[3], sy = T.m[7], sz = T.m[11];
            int ax, ay;
            lattice_cell(g, sx, sy, ax, ay);
            LineWalk L(ax, ay, ix, iy);
            const float s_major = L.xmajor ? sx : sy;
            const float p_major = L.xmajor ? px : py;
            const int o_major = L.xmajor ? g.ox : g.oy;
            const float inv_d = 1.0f / (p_major - s_major);
            const float dz = pz - sz;
            for (int s = 1; s < L.steps; s++) {
                L.step();
                if (L.x < 0 || L.x >= g.W || L.y < 0 || L.y >= g.H) continue;
                visited++;
                int st = storage_index(g, L.x, L.y);
                float hk = h[st];
                float zr = ray_height(o_major + (L.xmajor ? L.x : L.y), g.res, s_major, inv_d, sz, dz);
                float thr = zr + margin;
                if (hk > thr) atomicAdd(&clr[st], 1);
            }
        }
    }
    wave_stat_add(&stats[ST_RAY_CELLS], visited);
}

__global__ __launch_bounds__(256) void k_finalize(Grid g, const int* __restrict__ cnt,
                                                  const float* __restrict__ wsum,
                                                  const float* __restrict__ ssum,
                                                  const float2* __restrict__ stash,
                                                  const int* __restrict__ clr, int clear_min,
                                                  float* __restrict__ h, float* __restrict__ v,
                                                  const float* __restrict__ chsum, PointBinds pb,
                                                  unsigned long long* __restrict__ stats)
{
    const int HW = g.W * g.H;
    int st = blockIdx.x * blockDim.x + threadIdx.x;
    int touched = 0, cleared = 0;
    if (st < HW) {
        int N = cnt[st];
        if (N == 0) {
            if (clear_min > 0 && clr[st] >= clear_min && !isnan(h[st])) {
                h[st] = __uint_as_float(0x7fc00000u);
                cleared = 1;
            }
        } else {
            touched = 1;
            float hv = h[st];
            float hn, vn;
            if (!isnan(hv)) {  // prior plus the cloud, information form
                float vv = v[st];
                vn = 1.0f / (1.0f / vv + wsum[st]);
                hn = vn * (hv / vv + ssum[st]);
            } else if (N == 1) {  // a single point sets an empty cell exactly
                float2 zv = stash[st];
                hn = zv.x;
                vn = zv.y;
            } else {
                vn = 1.0f / wsum[st];
                hn = ssum[st] * vn;
            }
            h[st] = hn;
            v[st] = vn;
            for (int b = 0; b < pb.n; b++) {
                const LayerDev& L = pb.L[b];
                const int C = pb.b[b].C, off = pb.b[b].sum_off;
                GaussCoef gc{0.0f, 1.0f, 0.0f, true};
                if (L.rule == MEM_GAUSS) gc = gauss_coef(L.param, L.var[st], N);
                for (int q = 0; q < C; q++) {
                    float sum = chsum[(int64_t)(off + q) * HW + st];
                    float a = sum / (float)N;
                    int64_t idx = (int64_t)st * C + q;
                    float old = layer_load(L.val, L.storage, L.scale, idx, q);
                    layer_store(L.val, L.storage, L.scale, idx, q,
                                fuse_value(L.rule, L.param, old, a, sum, gc));
                }
                if (L.rule == MEM_GAUSS) L.var[st] = gc.var;
            }
        }
    }
    wave_stat_add(&stats[ST_TOUCHED], touched);
    wave_stat_add(&stats[ST_CLEARED], cleared);
}

__global__ __launch_bounds__(256) void k_point_cells(Grid g, const float* __restrict__ xyz,
                                                     int64_t n, Pose T, float mr2,
                                                     int32_t* __restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float px, py, pz, r2;
    int ix = 0, iy = 0;
    int r = point_cell(g, T, mr2, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], px, py, pz, r2, ix, iy);
    out[i] = (r == 0) ? iy * g.W + ix : r;
}

inline unsigned blocks_for(int64_t n, int per)
{
    return (unsigned)((n + per - 1) / per);
}

}  // namespace

void launch_zero_accum(hipStream_t s, const Grid& g, int* n, float* wsum, float* ssum, int* clr,
                       float* chsum, int Cb)
{
    int HW = g.W * g.H;
    unsigned b = blocks_for(HW, 256);
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(k_zero_accum, dim3(b), dim3(256), 0, s, HW, n, wsum, ssum, clr, chsum, Cb);
}

size_t ingest_lds_bytes(int Cb)
{
    return kStaticLds + (Cb > kMaxLdsCh ? (size_t)1 << 30 : sizeof(float) * kSlots * Cb);
}

void launch_ingest(hipStream_t s, const Grid& g, const float* xyz, int64_t n, const float* ch,
                   const Pose& T, float c0, float c1, float mr2, const PointBinds& pb, int* cnt,
                   float* wsum, float* ssum, float2* stash, float* chsum,
                   unsigned long long* stats)
{
    if (n <= 0) return;
    size_t lds = pb.lds_ch ? sizeof(float) * kSlots * pb.Cb : 0;
    hipLaunchKernelGGL(k_ingest, dim3(blocks_for(n, kChunk)), dim3(kWG), lds, s, g, xyz, n, ch, T,
                       c0, c1, mr2, pb, cnt, wsum, ssum, stash, chsum, stats);
}

void launch_clear_march(hipStream_t s, const Grid& g, const float* xyz, int64_t n, const Pose& T,
                        float mr2, float margin, const float* h, int* clr,
                        unsigned long long* stats)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_clear_march, dim3(blocks_for(n, 256)), dim3(256), 0, s, g, xyz, n, T, mr2,
                       margin, h, clr, stats);
}

void launch_finalize(hipStream_t s, const Grid& g, const int* cnt, const float* wsum,
                     const float* ssum, const float2* stash, const int* clr, int clear_min,
                     float* h, float* v, const float* chsum, const PointBinds& pb,
                     unsigned long long* stats)
{
    int HW = g.W * g.H;
    hipLaunchKernelGGL(k_finalize, dim3(blocks_for(HW, 256)), dim3(256), 0, s, g, cnt, wsum, ssum,
                       stash, clr, clear_min, h, v, chsum, pb, stats);
}

void launch_point_cells(hipStream_t s, const Grid& g, const float* xyz, int64_t n, const Pose& T,
                        float mr2, int32_t* out)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_point_cells, dim3(blocks_for(n, 256)), dim3(256), 0, s, g, xyz, n, T, mr2,
                       out);
}

}  // namespace memk
