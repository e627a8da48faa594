// k_pca.hip - PCA layer of a feature layer (the post-processing plugin that
// turns feature layers into a three-channel layer).
//
//   k_pca_sum      one wave per cell, one lane per channel: a ballot keeps
//                  the cells whose channels are all observed; binary64 sums
//                  per channel, one partial row per workgroup.
//   k_pca_total    the partial sums' totals, in one fixed order.
//   k_pca_cov      from the totals' mean, the centred outer products: lane
//                  c holds row c of the workgroup's covariance (the cell's
//                  centred vector is broadcast from LDS); the four waves
//                  are summed in LDS into one partial matrix.
//   k_pca_reduce   fixed-order sum of the partial matrices (16 lanes per
//                  entry, combined in lane order), divided by N.
//   k_pca_eig      one workgroup of 1024 lanes: parallel cyclic Jacobi rotations (disjoint
//                  index pairs of a round-robin schedule) on the matrix and
//                  its eigenvector matrix in LDS, then the three largest
//                  eigenpairs with the sign convention.
//   k_pca_project  one lane per logical cell: the centred vector's three
//                  projections, NaN for cells with an unobserved channel.
#include <mutex>

#include "update.h"

namespace memk {

namespace {

constexpr int kPcaBlocks = 512;  // workgroups of the two passes over the cells
constexpr int kPcaSweeps = 40;   // Jacobi sweeps at most

struct PcaParts {
    double sum[kPcaBlocks][kPcaMaxC + 1];            // channel sums, then the count
    double cov[kPcaBlocks][kPcaMaxC * kPcaMaxC];     // partial centred outer products
    double S[kPcaMaxC * kPcaMaxC];                   // the covariance
    double tot[kPcaMaxC + 1];                        // channel sums, then the count
};

__device__ __forceinline__ float feature(const LayerDev& L, int64_t st, int lane)
{
    return lane < L.C ? layer_load(L.val, L.storage, L.scale, st * L.C + lane, lane) : 0.0f;
}

__global__ __launch_bounds__(256) void k_pca_sum(LayerDev L, int HW, PcaParts* __restrict__ P)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double s = 0.0;
    int n = 0;
    for (int64_t st = (int64_t)blockIdx.x * 4 + w; st < HW; st += (int64_t)gridDim.x * 4) {
        const float v = feature(L, st, lane);
        if (__ballot(!isfinite(v))) continue;  // wave-uniform: the cell has an unobserved channel
        s += (double)v;
        n++;
    }
    __shared__ double sh[4][64];
    __shared__ int shn[4];
    sh[w][lane] = s;
    if (lane == 0) shn[w] = n;
    __syncthreads();
    if (threadIdx.x < 64) {
        P->sum[blockIdx.x][lane] = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
        if (lane == 0) P->sum[blockIdx.x][kPcaMaxC] = (double)(((shn[0] + shn[1]) + shn[2]) + shn[3]);
    }
}

// Totals of the sum partials: 16 entries (channel sums, then the count) per
// workgroup, each summed by 16 lanes over every 16th partial and the 16
// sums added in lane order.
__global__ __launch_bounds__(256) void k_pca_total(PcaParts* __restrict__ P, int nblk)
{
    const int q = threadIdx.x & 15, part = threadIdx.x >> 4;
    const int e = blockIdx.x * 16 + q;
    double s = 0.0;
    if (e <= kPcaMaxC)
        for (int b = part; b < nblk; b += 16) s += P->sum[b][e];
    __shared__ double red[16][17];
    red[part][q] = s;
    __syncthreads();
    if (threadIdx.x < 16 && e <= kPcaMaxC) {
        double t = 0.0;
        for (int k = 0; k < 16; k++) t += red[k][q];
        P->tot[e] = t;
    }
}

// Mean of channel `lane` and the count of cells with every channel observed.
__device__ __forceinline__ double pca_mean(const PcaParts* __restrict__ P, int lane, double& N)
{
    N = P->tot[kPcaMaxC];
    return N > 0.0 ? P->tot[lane] / N : 0.0;
}

__global__ __launch_bounds__(256) void k_pca_cov(LayerDev L, int HW, PcaParts* __restrict__ P)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double N;
    const double mean = pca_mean(P, lane, N);
    __shared__ double sd[4][64];
    double acc[kPcaMaxC];
#pragma unroll
    for (int k = 0; k < kPcaMaxC; k++) acc[k] = 0.0;
    for (int64_t st = (int64_t)blockIdx.x * 4 + w; st < HW; st += (int64_t)gridDim.x * 4) {
        const float v = feature(L, st, lane);
        if (__ballot(!isfinite(v))) continue;
        const double d = lane < L.C ? (double)v - mean : 0.0;
        sd[w][lane] = d;
        __builtin_amdgcn_wave_barrier();  // the wave's row is written before any lane reads it
#pragma unroll
        for (int k = 0; k < kPcaMaxC; k++) acc[k] += d * sd[w][k];
        __builtin_amdgcn_wave_barrier();  // ... and read before the next cell overwrites it
    }
    // the four waves' rows summed in LDS, in wave order
    __shared__ double tile[kPcaMaxC][kPcaMaxC + 1];
    for (int ww = 0; ww < 4; ww++) {
        if (w == ww)
#pragma unroll
            for (int k = 0; k < kPcaMaxC; k++) tile[lane][k] = ww == 0 ? acc[k] : tile[lane][k] + acc[k];
        __syncthreads();
    }
    for (int e = threadIdx.x; e < kPcaMaxC * kPcaMaxC; e += 256)
        P->cov[blockIdx.x][e] = tile[e / kPcaMaxC][e % kPcaMaxC];
}

// 16 entries per workgroup, each summed by 16 lanes over every 16th partial
// and the 16 sums added in lane order: a fixed order at any launch.
__global__ __launch_bounds__(256) void k_pca_reduce(PcaParts* __restrict__ P, int nblk)
{
    const int q = threadIdx.x & 15, part = threadIdx.x >> 4;
    const int e = blockIdx.x * 16 + q;
    double s = 0.0;
    for (int b = part; b < nblk; b += 16) s += P->cov[b][e];
    __shared__ double red[16][17];
    red[part][q] = s;
    __syncthreads();
    if (threadIdx.x < 16) {
        double t = 0.0;
        for (int k = 0; k < 16; k++) t += red[k][q];
        const double N = P->tot[kPcaMaxC];
        P->S[e] = N > 0.0 ? t / N : 0.0;
    }
}

// Jacobi eigensolver of the C x C covariance, one workgroup of 1024 lanes.
// The matrix is held as kPcaMaxC x kPcaMaxC with zero rows and columns past
// C (their rotations are identities), so a sweep is always kPcaMaxC - 1
// rounds of kPcaMaxC / 2 disjoint pairs (a round-robin tournament); the
// pairs' Givens rotations commute and are applied together: rows, then
// columns of S and of V, two elements per lane and phase.
constexpr int kEigLanes = 1024;
static_assert(kPcaMaxC == 64 && (kPcaMaxC / 2) * kPcaMaxC == 2 * kEigLanes, "two (pair, column) elements per lane");

__global__ __launch_bounds__(kEigLanes) void k_pca_eig(const PcaParts* __restrict__ P, int C,
                                                       PcaOut* __restrict__ out, float* __restrict__ lam_out)
{
    constexpr int n = kPcaMaxC, half = kPcaMaxC / 2;
    __shared__ double S[n][n + 1];
    __shared__ double V[n][n + 1];
    __shared__ double cs[half], sn[half];
    __shared__ int pa[half], pb[half];
    __shared__ double red[kEigLanes];
    const int t = threadIdx.x;
    for (int e = t; e < n * n; e += kEigLanes) {
        const int r = e >> 6, c = e & 63;
        S[r][c] = (r < C && c < C) ? P->S[r * kPcaMaxC + c] : 0.0;
        V[r][c] = r == c ? 1.0 : 0.0;
    }
    if (t < kPcaMaxC) {
        double N;
        out->mean[t] = t < C ? pca_mean(P, t, N) : 0.0;
        if (t == 0) out->n = N;
    }
    __syncthreads();
    // squared Frobenius norm (scale of the stopping test) and, per sweep,
    // the squared off-diagonal norm, reduced over the workgroup
    auto block_sum = [&](double x) {
        red[t] = x;
        __syncthreads();
        for (int o = kEigLanes / 2; o > 0; o >>= 1) {
            if (t < o) red[t] += red[t + o];
            __syncthreads();
        }
        const double r = red[0];
        __syncthreads();
        return r;
    };
    double f = 0.0;
    for (int e = t; e < n * n; e += kEigLanes) f += S[e >> 6][e & 63] * S[e >> 6][e & 63];
    const double fro2 = block_sum(f);
    for (int sweep = 0; sweep < kPcaSweeps && C > 1; sweep++) {
        for (int r = 0; r < n - 1; r++) {
            if (t < half) {
                // player 0 stays, the others move one seat each round
                auto player = [&](int i) { return i == 0 ? 0 : (i - 1 + r) % (n - 1) + 1; };
                const int a = player(t), b = player(n - 1 - t);
                const double apq = S[a][b];
                double c = 1.0, s = 0.0;
                if (apq != 0.0) {
                    const double tau = (S[b][b] - S[a][a]) / (2.0 * apq);
                    const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + tt * tt);
                    s = tt * c;
                }
                cs[t] = c;
                sn[t] = s;
                pa[t] = a;
                pb[t] = b;
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 2; u++) {  // rows: S <- G^T S
                const int e = t + u * kEigLanes, p = e >> 6, k = e & 63;
                const double c = cs[p], s = sn[p];
                const double x = S[pa[p]][k], y = S[pb[p]][k];
                S[pa[p]][k] = c * x - s * y;
                S[pb[p]][k] = s * x + c * y;
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 2; u++) {  // columns: S <- S G, V <- V G
                const int e = t + u * kEigLanes, p = e >> 6, k = e & 63;
                const double c = cs[p], s = sn[p];
                const double x = S[k][pa[p]], y = S[k][pb[p]];
                S[k][pa[p]] = c * x - s * y;
                S[k][pb[p]] = s * x + c * y;
                const double v = V[k][pa[p]], z = V[k][pb[p]];
                V[k][pa[p]] = c * v - s * z;
                V[k][pb[p]] = s * v + c * z;
            }
            __syncthreads();
        }
        double off = 0.0;
        for (int e = t; e < n * n; e += kEigLanes)
            if ((e >> 6) != (e & 63)) off += S[e >> 6][e & 63] * S[e >> 6][e & 63];
        // off-diagonal norm at 1e-10 of the matrix's (eigenvector error about
        // that over the relative eigenvalue gap; rounding keeps the norm near
        // n eps, so a bound much tighter would never be met)
        if (block_sum(off) <= 1e-20 * fro2) break;
    }
    if (t == 0) {
        // the three largest eigenvalues, descending (the lower index first
        // among equal ones), each vector signed by its largest entry
        int taken[kPcaK] = {-1, -1, -1};
        for (int k = 0; k < kPcaK; k++) {
            int best = -1;
            for (int i = 0; i < C; i++) {
                bool used = false;
                for (int q = 0; q < k; q++) used = used || taken[q] == i;
                if (!used && (best < 0 || S[i][i] > S[best][best])) best = i;
            }
            taken[k] = best;
            if (best < 0) {
                out->lam[k] = 0.0;
                for (int i = 0; i < kPcaMaxC; i++) out->comp[k][i] = 0.0;
                continue;
            }
            int j = 0;
            for (int i = 1; i < C; i++)
                if (fabs(V[i][best]) > fabs(V[j][best])) j = i;
            const double sg = V[j][best] > 0.0 ? 1.0 : -1.0;
            out->lam[k] = S[best][best];
            for (int i = 0; i < kPcaMaxC; i++) out->comp[k][i] = i < C ? sg * V[i][best] : 0.0;
        }
        if (lam_out)
            for (int k = 0; k < kPcaK; k++) lam_out[k] = (float)out->lam[k];
    }
}

__global__ __launch_bounds__(256) void k_pca_project(Grid g, LayerDev L, const PcaOut* __restrict__ pc,
                                                     float* __restrict__ out)
{
    __shared__ double s_m[kPcaMaxC], s_e[kPcaK][kPcaMaxC];
    for (int i = threadIdx.x; i < kPcaMaxC; i += blockDim.x) {
        s_m[i] = pc->mean[i];
        for (int k = 0; k < kPcaK; k++) s_e[k][i] = pc->comp[k][i];
    }
    __syncthreads();
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.W * g.H) return;
    const int ix = j % g.W, iy = j / g.W;
    const int64_t st = storage_index(g, ix, iy);
    double p[kPcaK] = {0.0, 0.0, 0.0};
    bool ok = true;
    for (int c = 0; c < L.C; c++) {
        const float v = layer_load(L.val, L.storage, L.scale, st * L.C + c, c);
        ok = ok && isfinite(v);
        const double d = (double)v - s_m[c];
#pragma unroll
        for (int k = 0; k < kPcaK; k++) p[k] += d * s_e[k][c];
    }
#pragma unroll
    for (int k = 0; k < kPcaK; k++) out[(int64_t)j * kPcaK + k] = ok ? (float)p[k] : __builtin_nanf("");
}

}  // namespace

size_t pca_scratch_bytes()
{
    return sizeof(PcaParts);
}

// The scratch of mem_pca_noalloc: the partial sums, then the result, of one
// PCA in a device array that every GPU the library runs on holds until the
// process ends (about 17 MB), so that the call allocates nothing.  Its
// address on a device comes from hipGetSymbolAddress, looked up once per
// device with that device current; host code never uses the array's name.
constexpr size_t kPcaPartsBytes = (sizeof(PcaParts) + 255) & ~(size_t)255;
constexpr size_t kPcaStaticBytes = kPcaPartsBytes + sizeof(PcaOut);
static __device__ __align__(256) char scratch[kPcaStaticBytes];

size_t pca_static_scratch_bytes()
{
    return kPcaStaticBytes;
}

hipError_t pca_static_scratch(int device, void** parts, PcaOut** res)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static char* addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = static_cast<char*>(p);
    }
    *parts = addr[device];
    *res = reinterpret_cast<PcaOut*>(addr[device] + kPcaPartsBytes);
    return hipSuccess;
}

void launch_pca(hipStream_t s, const Grid& g, const LayerDev& L, void* scratch, PcaOut* res, float* out,
                float* lam_out)
{
    PcaParts* P = static_cast<PcaParts*>(scratch);
    const int HW = g.W * g.H;
    int nblk = (HW + 3) / 4;
    if (nblk > kPcaBlocks) nblk = kPcaBlocks;
    if (nblk < 1) nblk = 1;
    hipLaunchKernelGGL(k_pca_sum, dim3(nblk), dim3(256), 0, s, L, HW, P);
    hipLaunchKernelGGL(k_pca_total, dim3((kPcaMaxC + 1 + 15) / 16), dim3(256), 0, s, P, nblk);
    hipLaunchKernelGGL(k_pca_cov, dim3(nblk), dim3(256), 0, s, L, HW, P);
    hipLaunchKernelGGL(k_pca_reduce, dim3(kPcaMaxC * kPcaMaxC / 16), dim3(256), 0, s, P, nblk);
    hipLaunchKernelGGL(k_pca_eig, dim3(1), dim3(kEigLanes), 0, s, P, L.C, res, lam_out);
    hipLaunchKernelGGL(k_pca_project, dim3((HW + 255) / 256), dim3(256), 0, s, g, L, res, out);
}

}  // namespace memk
