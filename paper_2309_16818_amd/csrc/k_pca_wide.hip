// k_pca_wide.hip - PCA layer of a feature layer of kPcaMaxC + 1 ..
// kPcaWideC channels (the post-processing plugin that turns feature layers
// into a three-channel layer; the same definition as k_pca.hip).
//
//   k_pcw_sum      one wave per cell, lanes over channels (stride 64): the
//                  cells whose channels are all observed are marked in a
//                  byte mask; binary64 channel sums, one partial row per
//                  workgroup.
//   k_pcw_total    the partial sums' totals, in one fixed order.
//   k_pcw_cov      the covariance in 64 x 64 tiles of its upper triangle:
//                  workgroup (b, q) sums tile q over the b-th share of the
//                  cells, lane c holding the tile's row c (the cell's
//                  centred column slice broadcast from LDS), the four waves
//                  added in LDS.
//   k_pcw_reduce   fixed-order sum of the tile partials, divided by N, into
//                  the full symmetric C x C matrix.
//   k_pcw_eig      one workgroup: orthogonal (subspace) iteration with
//                  Rayleigh-Ritz on a block of kPcwBlock vectors in LDS (lane
//                  i owns row i); the block is re-orthonormalised by shifted
//                  Cholesky QR (three passes) every step; it stops when the
//                  three leading Ritz pairs' residuals fall below 1e-12 of
//                  the largest eigenvalue (or after kPcwIters steps).
//   k_pcw_project  one lane per logical cell: the centred vector's three
//                  projections, NaN for cells with an unobserved channel.
#include "update.h"

namespace memk {

namespace {

constexpr int kPcwSumBlocks = 512;  // workgroups of the pass that sums the cells
constexpr int kPcwCellBlocks = 32;  // cell shares of the covariance pass
constexpr int kPcwT = kPcaWideC / 64;
constexpr int kPcwTiles = kPcwT * (kPcwT + 1) / 2;
constexpr int kPcwBlock = 8;    // vectors of the iterated block (3 wanted + 5 for the convergence rate)
constexpr int kPcwIters = 300;  // iterations at most
constexpr int kPcwLanes = 512;
static_assert(kPcaWideC <= kPcwLanes, "one lane per row of the block");

struct PcwParts {
    double sum[kPcwSumBlocks][kPcaWideC + 1];           // channel sums, then the count
    double cov[kPcwCellBlocks][kPcwTiles][64 * 64];     // tile partials
    double S[kPcaWideC * kPcaWideC];                    // the covariance
    double tot[kPcaWideC + 1];                          // channel sums, then the count
    // then HW bytes: 1 where every channel of the (storage-order) cell is finite
};

__device__ __forceinline__ unsigned char* cell_mask(PcwParts* P) { return reinterpret_cast<unsigned char*>(P + 1); }

// Tile q of the upper triangle (row-major over ti <= tj).
__device__ __forceinline__ void tile_of(int q, int T, int& ti, int& tj)
{
    ti = 0;
    while (q >= T - ti) {
        q -= T - ti;
        ti++;
    }
    tj = ti + q;
}

__global__ __launch_bounds__(256) void k_pcw_sum(LayerDev L, int HW, PcwParts* __restrict__ P)
{
    constexpr int J = kPcaWideC / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    unsigned char* mask = cell_mask(P);
    double s[J];
#pragma unroll
    for (int j = 0; j < J; j++) s[j] = 0.0;
    int n = 0;
    for (int64_t st = (int64_t)blockIdx.x * 4 + w; st < HW; st += (int64_t)gridDim.x * 4) {
        float v[J];
        bool bad = false;
#pragma unroll
        for (int j = 0; j < J; j++) {
            const int c = lane + 64 * j;
            v[j] = c < L.C ? layer_load(L.val, L.storage, L.scale, st * L.C + c, c) : 0.0f;
            bad = bad || !isfinite(v[j]);
        }
        const bool ok = __ballot(bad) == 0;  // wave-uniform
        if (lane == 0) mask[st] = ok ? 1 : 0;
        if (!ok) continue;
#pragma unroll
        for (int j = 0; j < J; j++) s[j] += (double)v[j];
        n++;
    }
    __shared__ double sh[4][kPcaWideC];
    __shared__ int shn[4];
#pragma unroll
    for (int j = 0; j < J; j++) sh[w][lane + 64 * j] = s[j];
    if (lane == 0) shn[w] = n;
    __syncthreads();
    for (int c = threadIdx.x; c < L.C; c += 256)
        P->sum[blockIdx.x][c] = ((sh[0][c] + sh[1][c]) + sh[2][c]) + sh[3][c];
    if (threadIdx.x == 0) P->sum[blockIdx.x][kPcaWideC] = (double)(((shn[0] + shn[1]) + shn[2]) + shn[3]);
}

// 16 entries (channel sums, then the count) per workgroup, each summed by
// 16 lanes over every 16th partial and the 16 sums added in lane order.
__global__ __launch_bounds__(256) void k_pcw_total(PcwParts* __restrict__ P, int nblk, int C)
{
    const int q = threadIdx.x & 15, part = threadIdx.x >> 4;
    const int i = blockIdx.x * 16 + q;
    const int e = i < C ? i : kPcaWideC;  // entry C is the count
    double s = 0.0;
    if (i <= C)
        for (int b = part; b < nblk; b += 16) s += P->sum[b][e];
    __shared__ double red[16][17];
    red[part][q] = s;
    __syncthreads();
    if (threadIdx.x < 16 && i <= C) {
        double t = 0.0;
        for (int k = 0; k < 16; k++) t += red[k][q];
        P->tot[e] = t;
    }
}

__device__ __forceinline__ double pcw_mean(const PcwParts* __restrict__ P, int c, int C)
{
    const double N = P->tot[kPcaWideC];
    return (c < C && N > 0.0) ? P->tot[c] / N : 0.0;
}

__global__ __launch_bounds__(256) void k_pcw_cov(LayerDev L, int HW, int T, PcwParts* __restrict__ P)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int ti, tj;
    tile_of(blockIdx.y, T, ti, tj);
    const int ci = ti * 64 + lane, cj = tj * 64 + lane;
    const double mi = pcw_mean(P, ci, L.C), mj = pcw_mean(P, cj, L.C);
    const unsigned char* mask = cell_mask(P);
    __shared__ double sd[4][64];
    double acc[64];
#pragma unroll
    for (int k = 0; k < 64; k++) acc[k] = 0.0;
    for (int64_t st = (int64_t)blockIdx.x * 4 + w; st < HW; st += (int64_t)gridDim.x * 4) {
        if (!mask[st]) continue;  // wave-uniform
        const float vi = ci < L.C ? layer_load(L.val, L.storage, L.scale, st * L.C + ci, ci) : 0.0f;
        const float vj = cj < L.C ? layer_load(L.val, L.storage, L.scale, st * L.C + cj, cj) : 0.0f;
        const double di = ci < L.C ? (double)vi - mi : 0.0;
        sd[w][lane] = cj < L.C ? (double)vj - mj : 0.0;
        __builtin_amdgcn_wave_barrier();  // the wave's slice is written before any lane reads it
#pragma unroll
        for (int k = 0; k < 64; k++) acc[k] += di * sd[w][k];
        __builtin_amdgcn_wave_barrier();  // ... and read before the next cell overwrites it
    }
    __shared__ double tile[64][65];
    for (int ww = 0; ww < 4; ww++) {
        if (w == ww)
#pragma unroll
            for (int k = 0; k < 64; k++) tile[lane][k] = ww == 0 ? acc[k] : tile[lane][k] + acc[k];
        __syncthreads();
    }
    double* out = P->cov[blockIdx.x][blockIdx.y];
    for (int e = threadIdx.x; e < 64 * 64; e += 256) out[e] = tile[e >> 6][e & 63];
}

// 16 matrix entries per workgroup, each summed by 16 lanes over every 16th
// cell share and the 16 sums added in lane order.
__global__ __launch_bounds__(256) void k_pcw_reduce(PcwParts* __restrict__ P, int nblk, int C, int T)
{
    const int q = threadIdx.x & 15, part = threadIdx.x >> 4;
    const int64_t e = (int64_t)blockIdx.x * 16 + q;
    const bool in = e < (int64_t)C * C;
    int i = in ? (int)(e / C) : 0, j = in ? (int)(e % C) : 0;
    if (i > j) {  // the lower triangle from its mirror in the upper tiles
        const int t = i;
        i = j;
        j = t;
    }
    const int ti = i >> 6, tj = j >> 6;
    const int tq = ti * T - ti * (ti - 1) / 2 + (tj - ti);
    const int r = i & 63, c = j & 63;
    double s = 0.0;
    if (in)
        for (int b = part; b < nblk; b += 16) s += P->cov[b][tq][r * 64 + c];
    __shared__ double red[16][17];
    red[part][q] = s;
    __syncthreads();
    if (threadIdx.x < 16 && in) {
        double t = 0.0;
        for (int k = 0; k < 16; k++) t += red[k][q];
        const double N = P->tot[kPcaWideC];
        P->S[e] = N > 0.0 ? t / N : 0.0;
    }
}

constexpr int kPcwPairs = kPcwBlock * (kPcwBlock + 1) / 2;
constexpr int kPcwChunks = kPcwLanes / kPcwPairs;  // lanes per Gram entry

// The block's rows live in LDS (row i of a block: its kPcwBlock entries);
// the small dense steps run on lane 0 and every lane reads their results.
struct PcwSmall {
    double G[kPcwBlock][kPcwBlock];  // a Gram matrix or the Rayleigh quotient V^T S V
    double R[kPcwBlock][kPcwBlock];  // its Cholesky factor, or the Ritz vectors (columns, ordered)
    double theta[kPcwBlock];         // Ritz values, descending
    double Y[kPcwBlock][kPcwBlock];  // Jacobi's vectors
    int ord[kPcwBlock];              // their order
    int bad;                         // a column to reseed, or -1
    double part[kPcwPairs][kPcwChunks];
};

// sm.G = A^T B over rows 0..C-1 (A, B in LDS), in a fixed order: lane
// (entry, chunk) sums every kPcwChunks-th row from its chunk, then lane
// `entry` adds the chunks in order.  Visible to every lane on return.
__device__ __forceinline__ void gram(const double (*A)[kPcwBlock], const double (*B)[kPcwBlock], int C,
                                     PcwSmall& sm)
{
    const int t = threadIdx.x;
    if (t < kPcwPairs * kPcwChunks) {
        const int e = t / kPcwChunks, ch = t % kPcwChunks;
        int p = 0, q = e;  // entry e of the upper triangle, row-major
        while (q >= kPcwBlock - p) {
            q -= kPcwBlock - p;
            p++;
        }
        q += p;
        double x = 0.0;
        for (int i = ch; i < C; i += kPcwChunks) x += A[i][p] * B[i][q];
        sm.part[e][ch] = x;
    }
    __syncthreads();
    if (t < kPcwPairs) {
        int p = 0, q = t;
        while (q >= kPcwBlock - p) {
            q -= kPcwBlock - p;
            p++;
        }
        q += p;
        double x = 0.0;
        for (int ch = 0; ch < kPcwChunks; ch++) x += sm.part[t][ch];
        sm.G[p][q] = x;
        sm.G[q][p] = x;
    }
    __syncthreads();
}

// Deterministic start / replacement vector entries in [-1, 1).
__device__ __forceinline__ double seed_entry(int row, int col, int round)
{
    unsigned h = (unsigned)row * 2654435761u ^ (unsigned)(col + 1) * 2246822519u ^ (unsigned)(round + 7) * 3266489917u;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    h *= 3266489917u;
    h ^= h >> 16;
    return (double)(h >> 8) * (1.0 / 8388608.0) - 1.0;
}

// Cholesky QR of the block Z (in LDS, in place): G = Z^T Z + shift I =
// R^T R, Z <- Z R^-1.  A column whose pivot vanishes is replaced by seeded
// entries instead (the caller orthonormalises again); returns false then.
__device__ __forceinline__ bool chol_qr(double (*Z)[kPcwBlock], double shift_rel, int C, int round, PcwSmall& sm)
{
    const int t = threadIdx.x;
    gram(Z, Z, C, sm);
    if (t == 0) {
        double tr = 0.0;
        for (int p = 0; p < kPcwBlock; p++) tr += sm.G[p][p];
        const double shift = shift_rel * tr;
        sm.bad = -1;
        for (int p = 0; p < kPcwBlock; p++) {
            double d = sm.G[p][p] + shift;
            for (int k = 0; k < p; k++) d -= sm.R[k][p] * sm.R[k][p];
            if (!(tr > 0.0) || !(d > 1e-30 * tr)) {  // a dependent (or zero) column
                sm.bad = p;
                break;
            }
            sm.R[p][p] = sqrt(d);
            for (int q = p + 1; q < kPcwBlock; q++) {
                double x = sm.G[p][q];
                for (int k = 0; k < p; k++) x -= sm.R[k][p] * sm.R[k][q];
                sm.R[p][q] = x / sm.R[p][p];
            }
        }
    }
    __syncthreads();
    const int bad = sm.bad;
    if (bad >= 0) {
        if (t < C) Z[t][bad] = seed_entry(t, bad, round);
        __syncthreads();
        return false;
    }
    if (t < C) {  // y R = z, forward over the columns
        double y[kPcwBlock];
#pragma unroll
        for (int q = 0; q < kPcwBlock; q++) {
            double x = Z[t][q];
#pragma unroll
            for (int k = 0; k < q; k++) x -= y[k] * sm.R[k][q];
            y[q] = x / sm.R[q][q];
        }
#pragma unroll
        for (int q = 0; q < kPcwBlock; q++) Z[t][q] = y[q];
    }
    __syncthreads();
    return true;
}

// Orthonormal columns of Z: shifted Cholesky QR, then two plain passes
// (shifted CholeskyQR3), reseeding dependent columns.
__device__ __forceinline__ void orthonormalise(double (*Z)[kPcwBlock], int C, PcwSmall& sm)
{
    constexpr double u = 1.1102230246251565e-16;  // 2^-53
    const double shift_rel = 11.0 * ((double)C * kPcwBlock + kPcwBlock * (kPcwBlock + 1)) * u;
    for (int round = 0; round < 8; round++) {
        if (!chol_qr(Z, shift_rel, C, round, sm)) continue;
        if (!chol_qr(Z, 0.0, C, round, sm)) continue;
        if (chol_qr(Z, 0.0, C, round, sm)) return;
    }
}

// Lane 0: eigen-decomposition of the symmetric sm.G by cyclic Jacobi; the
// vectors go to sm.R's columns and the values to sm.theta, both ordered by
// value, descending (the lower index first among equal ones).
__device__ __forceinline__ void small_eigen(PcwSmall& sm)
{
    constexpr int n = kPcwBlock;
    double (&H)[n][n] = sm.G;
    double (&Y)[n][n] = sm.Y;
    for (int p = 0; p < n; p++)
        for (int q = 0; q < n; q++) Y[p][q] = p == q ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 30; sweep++) {
        double off = 0.0, all = 0.0;
        for (int p = 0; p < n; p++)
            for (int q = 0; q < n; q++) {
                all += H[p][q] * H[p][q];
                if (p != q) off += H[p][q] * H[p][q];
            }
        if (off <= 1e-30 * all) break;
        for (int p = 0; p < n - 1; p++)
            for (int q = p + 1; q < n; q++) {
                const double apq = H[p][q];
                if (apq == 0.0) continue;
                const double tau = (H[q][q] - H[p][p]) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < n; k++) {  // rows p, q
                    const double x = H[p][k], y = H[q][k];
                    H[p][k] = c * x - s * y;
                    H[q][k] = s * x + c * y;
                }
                for (int k = 0; k < n; k++) {  // columns p, q
                    const double x = H[k][p], y = H[k][q];
                    H[k][p] = c * x - s * y;
                    H[k][q] = s * x + c * y;
                    const double v = Y[k][p], z = Y[k][q];
                    Y[k][p] = c * v - s * z;
                    Y[k][q] = s * v + c * z;
                }
            }
    }
    int (&ord)[n] = sm.ord;
    for (int b = 0; b < n; b++) ord[b] = b;
    for (int a = 1; a < n; a++)
        for (int b = a; b > 0 && H[ord[b]][ord[b]] > H[ord[b - 1]][ord[b - 1]]; b--) {
            const int tmp = ord[b];
            ord[b] = ord[b - 1];
            ord[b - 1] = tmp;
        }
    for (int b = 0; b < n; b++) {
        sm.theta[b] = H[ord[b]][ord[b]];
        for (int a = 0; a < n; a++) sm.R[a][b] = Y[a][ord[b]];
    }
}

__global__ __launch_bounds__(kPcwLanes) void k_pcw_eig(const PcwParts* __restrict__ P, int C,
                                                       PcaWideOut* __restrict__ out, float* __restrict__ lam_out)
{
    __shared__ double V[kPcaWideC][kPcwBlock];  // the orthonormal block, then its Ritz vectors
    __shared__ double W[kPcaWideC][kPcwBlock];  // S V, then S times the Ritz vectors
    __shared__ PcwSmall sm;
    __shared__ double s_r[kPcwLanes / 64][kPcaK];
    const int t = threadIdx.x;  // lane t owns row t of the blocks (rows >= C are never read)
    if (t < kPcaWideC) out->mean[t] = pcw_mean(P, t, C);
    if (t == 0) out->n = P->tot[kPcaWideC];
    if (t < C)
#pragma unroll
        for (int b = 0; b < kPcwBlock; b++) V[t][b] = seed_entry(t, b, 100);
    __syncthreads();
    orthonormalise(V, C, sm);
    int it = 0;
    for (;; it++) {
        // W = S V (S symmetric: column t of S is read row by row, so the
        // lanes' loads of one row are contiguous)
        if (t < C) {
            double w[kPcwBlock];
#pragma unroll
            for (int b = 0; b < kPcwBlock; b++) w[b] = 0.0;
            for (int k = 0; k < C; k++) {
                const double s = P->S[(int64_t)k * C + t];
#pragma unroll
                for (int b = 0; b < kPcwBlock; b++) w[b] += s * V[k][b];
            }
#pragma unroll
            for (int b = 0; b < kPcwBlock; b++) W[t][b] = w[b];
        }
        __syncthreads();
        // Rayleigh-Ritz: H = V^T S V (sm.G, symmetric by construction),
        // Ritz vectors V Y and S V Y = W Y
        gram(V, W, C, sm);
        if (t == 0) small_eigen(sm);
        __syncthreads();
        double r2[kPcaK] = {0.0, 0.0, 0.0};
        double x[kPcwBlock], sx[kPcwBlock];
#pragma unroll
        for (int b = 0; b < kPcwBlock; b++) {
            double xa = 0.0, sa = 0.0;
            if (t < C)
#pragma unroll
                for (int a = 0; a < kPcwBlock; a++) {
                    xa += V[t][a] * sm.R[a][b];
                    sa += W[t][a] * sm.R[a][b];
                }
            x[b] = xa;
            sx[b] = sa;
        }
#pragma unroll
        for (int k = 0; k < kPcaK; k++) {
            const double r = sx[k] - sm.theta[k] * x[k];
            r2[k] = r * r;  // zero for rows >= C
        }
        __syncthreads();  // every lane has read its rows of V and W
        if (t < C)
#pragma unroll
            for (int b = 0; b < kPcwBlock; b++) {
                V[t][b] = x[b];
                W[t][b] = sx[b];
            }
        // residuals of the three leading pairs, summed in a fixed order
#pragma unroll
        for (int k = 0; k < kPcaK; k++)
            for (int o = 32; o > 0; o >>= 1) r2[k] += __shfl_xor(r2[k], o);
        if ((t & 63) == 0)
#pragma unroll
            for (int k = 0; k < kPcaK; k++) s_r[t >> 6][k] = r2[k];
        __syncthreads();
        double rr[kPcaK] = {0.0, 0.0, 0.0};
        for (int ww = 0; ww < kPcwLanes / 64; ww++)
#pragma unroll
            for (int k = 0; k < kPcaK; k++) rr[k] += s_r[ww][k];
        const double tol = 1e-12 * fmax(fabs(sm.theta[0]), 1e-300);
        const bool done = (rr[0] <= tol * tol && rr[1] <= tol * tol && rr[2] <= tol * tol) || it + 1 >= kPcwIters;
        __syncthreads();
        if (done) break;
        // next block: S applied to the Ritz vectors, orthonormalised
        if (t < C)
#pragma unroll
            for (int b = 0; b < kPcwBlock; b++) V[t][b] = W[t][b];
        __syncthreads();
        orthonormalise(V, C, sm);
    }
    // V holds the Ritz vectors in order; signs: the largest-magnitude entry
    // (the first of equal ones) positive
    __shared__ double s_abs[kPcwLanes];
    __shared__ int s_idx[kPcwLanes];
#pragma unroll
    for (int k = 0; k < kPcaK; k++) {
        const double xk = t < C ? V[t][k] : 0.0;
        s_abs[t] = t < C ? fabs(xk) : -1.0;
        s_idx[t] = t;
        __syncthreads();
        for (int o = kPcwLanes / 2; o > 0; o >>= 1) {
            if (t < o) {
                const double a = s_abs[t], b = s_abs[t + o];
                if (b > a || (b == a && s_idx[t + o] < s_idx[t])) {
                    s_abs[t] = b;
                    s_idx[t] = s_idx[t + o];
                }
            }
            __syncthreads();
        }
        const int jmax = s_idx[0];
        __syncthreads();
        if (t == jmax) s_abs[0] = xk;
        __syncthreads();
        const double sg = s_abs[0] > 0.0 ? 1.0 : -1.0;
        __syncthreads();
        if (t < kPcaWideC) out->comp[k][t] = t < C ? sg * xk : 0.0;
        if (t == 0) {
            out->lam[k] = sm.theta[k];
            if (lam_out) lam_out[k] = (float)sm.theta[k];
        }
    }
    if (t == 0) out->iters = it + 1;
}

__global__ __launch_bounds__(256) void k_pcw_project(Grid g, LayerDev L, const PcaWideOut* __restrict__ pc,
                                                     float* __restrict__ out)
{
    __shared__ double s_m[kPcaWideC], s_e[kPcaK][kPcaWideC];
    for (int i = threadIdx.x; i < kPcaWideC; i += blockDim.x) {
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

size_t pca_wide_scratch_bytes(int64_t cells)
{
    return sizeof(PcwParts) + (size_t)cells;
}

void launch_pca_wide(hipStream_t s, const Grid& g, const LayerDev& L, void* scratch, PcaWideOut* res, float* out,
                     float* lam_out)
{
    PcwParts* P = static_cast<PcwParts*>(scratch);
    const int HW = g.W * g.H;
    int nblk = (HW + 3) / 4;
    if (nblk > kPcwSumBlocks) nblk = kPcwSumBlocks;
    if (nblk < 1) nblk = 1;
    const int T = (L.C + 63) / 64;
    const int tiles = T * (T + 1) / 2;
    int ncb = (HW + 3) / 4;
    if (ncb > kPcwCellBlocks) ncb = kPcwCellBlocks;
    if (ncb < 1) ncb = 1;
    hipLaunchKernelGGL(k_pcw_sum, dim3(nblk), dim3(256), 0, s, L, HW, P);
    hipLaunchKernelGGL(k_pcw_total, dim3((L.C + 1 + 15) / 16), dim3(256), 0, s, P, nblk, L.C);
    hipLaunchKernelGGL(k_pcw_cov, dim3(ncb, tiles), dim3(256), 0, s, L, HW, T, P);
    hipLaunchKernelGGL(k_pcw_reduce, dim3((unsigned)(((int64_t)L.C * L.C + 15) / 16)), dim3(256), 0, s, P, ncb, L.C,
                       T);
    hipLaunchKernelGGL(k_pcw_eig, dim3(1), dim3(kPcwLanes), 0, s, P, L.C, res, lam_out);
    hipLaunchKernelGGL(k_pcw_project, dim3((HW + 255) / 256), dim3(256), 0, s, g, L, res, out);
}

}  // namespace memk
