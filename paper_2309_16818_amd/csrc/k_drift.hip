// k_drift.hip - z-error count and drift compensation of a point cloud
// (Table I, the two steps before the height update; the paper defers their
// definition, read here from its Gaussian model).
//
//   k_drift_count  grid-stride over the cloud: each accepted point whose
//                  cell holds a height tests its height error against the
//                  combined variance in binary32; consistent points add
//                  1 / (v + v_i) and e / (v + v_i) to binary64 sums, one
//                  partial per workgroup (no atomics).
//   k_drift_apply  every workgroup reduces the partials in one fixed order
//                  (so the offset is the same in every workgroup and run)
//                  and, with enough consistent points, shifts its share of
//                  the held heights and of their logical-order copy.
#include "update.h"

namespace memk {

namespace {

constexpr int kDriftBlocks = 512;  // partials: the most k_drift_count workgroups

struct DriftPart {
    double sw, swe;
    int n, pad;
};

__global__ __launch_bounds__(256) void k_drift_count(Grid g, const float* __restrict__ xyz, int64_t n, Pose T,
                                                     float c0, float c1, float mr2,
                                                     const float* __restrict__ h,
                                                     const float* __restrict__ v, float kappa2,
                                                     DriftPart* __restrict__ part)
{
    double sw = 0.0, swe = 0.0;
    int cnt = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        float px, py, pz, r2;
        int ix, iy;
        if (point_cell(g, T, mr2, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], px, py, pz, r2, ix, iy) != 0)
            continue;
        const int st = storage_index(g, ix, iy);
        const float hj = h[st];
        if (isnan(hj)) continue;
        const float sig = c0 + c1 * r2;  // the point's standard deviation (height update's model)
        const float vi = sig * sig;
        const float e = pz - hj;
        const float tot = v[st] + vi;
        if (!(e * e <= kappa2 * tot)) continue;
        sw += 1.0 / (double)tot;
        swe += (double)e / (double)tot;
        cnt++;
    }
    for (int off = 32; off > 0; off >>= 1) {
        sw += __shfl_down(sw, off);
        swe += __shfl_down(swe, off);
        cnt += __shfl_down(cnt, off);
    }
    __shared__ double s_sw[4], s_swe[4];
    __shared__ int s_n[4];
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_sw[wave] = sw;
        s_swe[wave] = swe;
        s_n[wave] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; w++) {
            sw += s_sw[w];
            swe += s_swe[w];
            cnt += s_n[w];
        }
        part[blockIdx.x] = DriftPart{sw, swe, cnt, 0};
    }
}

__global__ __launch_bounds__(256) void k_drift_apply(Grid g, const DriftPart* __restrict__ part, int nparts,
                                                     DriftDev* __restrict__ drift, int min_points,
                                                     float* __restrict__ h, float* __restrict__ hl)
{
    __shared__ double s_sw[256], s_swe[256];
    __shared__ int s_n[256];
    const int t = threadIdx.x;
    double sw = 0.0, swe = 0.0;
    int cnt = 0;
    for (int i = t; i < nparts; i += 256) {
        sw += part[i].sw;
        swe += part[i].swe;
        cnt += part[i].n;
    }
    s_sw[t] = sw;
    s_swe[t] = swe;
    s_n[t] = cnt;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) {
            s_sw[t] += s_sw[t + off];
            s_swe[t] += s_swe[t + off];
            s_n[t] += s_n[t + off];
        }
        __syncthreads();
    }
    const int N = s_n[0];
    const bool apply = N >= min_points && N > 0;
    const float d = apply ? (float)(s_swe[0] / s_sw[0]) : 0.0f;
    if (blockIdx.x == 0 && t == 0) *drift = DriftDev{s_sw[0], s_swe[0], N, d};
    if (!apply) return;
    const int HW = g.W * g.H;
    const int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + t; i < HW; i += stride) {
        const float x = h[i];
        if (isnan(x)) continue;
        const float y = x + d;
        h[i] = y;
        if (hl) {
            int ix, iy;
            logical_index(g, i, ix, iy);
            hl[iy * g.W + ix] = y;
        }
    }
}

}  // namespace

size_t drift_part_bytes()
{
    return sizeof(DriftPart) * kDriftBlocks;
}

void launch_drift(hipStream_t s, const Grid& g, const float* xyz, int64_t n, const Pose& T, float c0,
                  float c1, float mr2, float* h, const float* v, float kappa2, int min_points,
                  DriftDev* drift, void* part, float* hl)
{
    if (n <= 0) return;
    int64_t bc = (n + 255) / 256;
    if (bc > kDriftBlocks) bc = kDriftBlocks;
    DriftPart* p = static_cast<DriftPart*>(part);
    hipLaunchKernelGGL(k_drift_count, dim3((unsigned)bc), dim3(256), 0, s, g, xyz, n, T, c0, c1, mr2, h, v, kappa2,
                       p);
    int64_t ba = ((int64_t)g.W * g.H + 255) / 256;
    if (ba > 1024) ba = 1024;
    hipLaunchKernelGGL(k_drift_apply, dim3((unsigned)ba), dim3(256), 0, s, g, p, (int)bc, drift, min_points, h, hl);
}

}  // namespace memk
