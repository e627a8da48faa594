// k_unet.hip - kernels of the completion U-Net (forward, backward, Adam).
//
// Every 3x3 convolution, transposed convolution and their gradients is a
// BF16 matrix product on the MFMA units (v_mfma_f32_16x16x32_bf16, FP32
// accumulation):
//   gemm_nt  C[m][n] = sum_k A[m][k] B[n][k]      A, B K-contiguous (im2col
//            rows x weight rows); epilogue: bias, ReLU or ReLU-mask, BF16/FP32
//            store, or the 2x2 scatter of a transposed convolution.
//   gemm_tn  C[m][n] += sum_p A[p][m] B[p][n]     reduction over pixels for
//            weight gradients, split over pixel ranges with FP32 atomics.
// Activations are NHWC BF16; a convolution's input is unfolded (im2col)
// into a K-padded BF16 matrix first.
#include <initializer_list>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "codec.h"
#include "unet_internal.h"

namespace memk {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 32;
constexpr float kLogSigmaRef = -4.60517019f;  // ln(0.01 m), the input's standard-deviation unit
constexpr int LDSK = BK + 8;  // padded row (bf16) against bank conflicts

__device__ __forceinline__ uint16_t bf(float f) { return f32_to_bf16(f); }
__device__ __forceinline__ float fb(uint16_t b) { return bf16_to_f32(b); }

// Loads 8 consecutive bf16 of row r (K-contiguous, row stride ld) starting
// at column k0, zero-filling outside [0, rows) x [0, K).
__device__ __forceinline__ uint4 load8(const uint16_t* __restrict__ p, int64_t ld, int r, int rows, int k0,
                                       int K)
{
    uint4 v = make_uint4(0, 0, 0, 0);
    if (r >= rows) return v;
    const uint16_t* q = p + (int64_t)r * ld + k0;
    if (k0 + 8 <= K && ((((uintptr_t)q) & 15) == 0)) return *(const uint4*)q;
    uint16_t t[8];
#pragma unroll
    for (int j = 0; j < 8; j++) t[j] = (k0 + j < K) ? q[j] : (uint16_t)0;
    v.x = t[0] | ((uint32_t)t[1] << 16);
    v.y = t[2] | ((uint32_t)t[3] << 16);
    v.z = t[4] | ((uint32_t)t[5] << 16);
    v.w = t[6] | ((uint32_t)t[7] << 16);
    return v;
}

// Position of one thread's 8-wide K slice inside the unfolded convolution
// input: tap t and channel c of column k, advanced by whole K steps.
struct ConvCursor {
    int t, c;
    __device__ __forceinline__ void start(int k, int ci)
    {
        t = k / ci;
        c = k - t * ci;
    }
    __device__ __forceinline__ void advance(int dk, int ci)
    {
        c += dk;
        while (c >= ci) {
            c -= ci;
            t++;
        }
    }
};

// 8 values of the unfolded input at pixel (n, r, q), slice (t, c); zero
// outside the image or past tap 8.
__device__ __forceinline__ uint4 load8_conv(const ConvSrc& cs, int64_t n, int r, int q, bool valid, const ConvCursor& cc)
{
    uint4 v = make_uint4(0, 0, 0, 0);
    if (!valid || cc.t >= 9) return v;
    const int ty = cc.t / 3;
    const int rr = r + ty - 1, qq = q + (cc.t - 3 * ty) - 1;
    if (rr < 0 || rr >= cs.S || qq < 0 || qq >= cs.S) return v;
    return *(const uint4*)(cs.x + ((n * cs.S + rr) * cs.S + qq) * cs.xs + cc.c);
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v)
{
    bf16x8 r;
    __builtin_memcpy(&r, &v, 16);
    return r;
}

// C = A B^T on a (WTM WM) x (WTN WN) tile, WM WN = 4: four waves, each a
// WTM x WTN block of (WTM / 16) x (WTN / 16) MFMA 16x16x32 blocks.  Lane l
// of an MFMA block supplies A[l % 16][8 (l / 16) .. + 7] and
// B[l % 16][8 (l / 16) .. + 7] and receives D[4 (l / 16) + j][l % 16].  A
// wave reads its WTN / 16 B fragments of a K slice once and each A fragment
// once, so every fragment read from LDS feeds WTN / 16 (or WTM / 16) MFMAs.
// K advances in slices of 32 through two LDS stages: the next slice's
// global loads are in flight while the MFMAs consume the current one, with
// one barrier per slice.
template <int EPI, bool CONV, int WM, int WTM, int WTN>
__global__ __launch_bounds__(256) void k_gemm_nt(const uint16_t* __restrict__ A, int64_t lda, ConvSrc cs,
                                                 const uint16_t* __restrict__ B, int64_t ldb, int M,
                                                 int N, int K, Epilogue ep)
{
    constexpr int WN = 4 / WM, TM = WTM * WM, TN = WTN * WN, IM = WTM / 16, JN = WTN / 16;
    static_assert(TM % 64 == 0 && WTM % 16 == 0 && WTN % 16 == 0, "tile shape");
    constexpr int CA = TM * 4 / 256, CB = (TN * 4 + 255) / 256;  // 8-wide chunks per thread
    __shared__ uint16_t sA[2][TM * LDSK];
    __shared__ uint16_t sB[2][TN * LDSK];
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave / WN) * WTM, wn = (wave % WN) * WTN;
    f32x4 acc[IM][JN];
#pragma unroll
    for (int i = 0; i < IM; i++)
#pragma unroll
        for (int j = 0; j < JN; j++) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int lk = (tid & 3) * 8;  // K offset of every chunk of this thread
    int64_t pn[CA];
    int pr[CA], pq[CA];
    ConvCursor cc{0, 0};
    if (CONV) {
#pragma unroll
        for (int u = 0; u < CA; u++) {
            const int m = m0 + (tid >> 2) + 64 * u;
            pq[u] = m % cs.S;
            pr[u] = (m / cs.S) % cs.S;
            pn[u] = m / (cs.S * cs.S);
        }
        cc.start(lk, cs.ci);
    }
    uint4 va[CA], vb[CB];
    auto load = [&](int k0) {
#pragma unroll
        for (int u = 0; u < CA; u++) {
            const int r = (tid >> 2) + 64 * u;
            va[u] = CONV ? load8_conv(cs, pn[u], pr[u], pq[u], m0 + r < M, cc) : load8(A, lda, m0 + r, M, k0 + lk, K);
        }
        if (CONV) cc.advance(BK, cs.ci);
#pragma unroll
        for (int u = 0; u < CB; u++) {
            const int r = (tid >> 2) + 64 * u;
            vb[u] = (r < TN) ? load8(B, ldb, n0 + r, N, k0 + lk, K) : make_uint4(0, 0, 0, 0);
        }
    };
    auto stash = [&](int st) {
#pragma unroll
        for (int u = 0; u < CA; u++) *(uint4*)&sA[st][((tid >> 2) + 64 * u) * LDSK + lk] = va[u];
#pragma unroll
        for (int u = 0; u < CB; u++) {
            const int r = (tid >> 2) + 64 * u;
            if (r < TN) *(uint4*)&sB[st][r * LDSK + lk] = vb[u];
        }
    };
    load(0);
    stash(0);
    __syncthreads();
    int cur = 0;
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    for (int k0 = 0; k0 < K; k0 += BK) {
        const bool more = k0 + BK < K;
        if (more) load(k0 + BK);
        bf16x8 b[JN];
#pragma unroll
        for (int j = 0; j < JN; j++) b[j] = as_bf16x8(*(const uint4*)&sB[cur][(wn + 16 * j + fr) * LDSK + fk]);
#pragma unroll
        for (int i = 0; i < IM; i++) {
            const bf16x8 a = as_bf16x8(*(const uint4*)&sA[cur][(wm + 16 * i + fr) * LDSK + fk]);
#pragma unroll
            for (int j = 0; j < JN; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j], acc[i][j], 0, 0, 0);
        }
        if (more) stash(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }
#pragma unroll
    for (int i = 0; i < IM; i++)
#pragma unroll
        for (int j = 0; j < JN; j++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                const int n = n0 + wn + 16 * j + (lane & 15);
                if (m < M && n < N) epilogue<EPI>(ep, m, n, acc[i][j][r]);
            }
}

// C[m][n] += sum_p A[p][m] B[p][n] over the pixel range of this block
// (blockIdx.z of gridDim.z equal slices), on a (32 WM) x (32 WN) tile.
// Pixels advance in slices of 32 through two LDS stages holding the slices
// transposed ([column][pixel]), the next slice's loads in flight during the
// MFMAs.
// LDS slot of element (row, k) of a k_gemm_tn operand tile ([row][k], k =
// pixel): the four 8-pixel groups of a row are permuted by bits 3-4 of the
// row.  The pixel-major tiles are transposed into LDS with 2-byte stores in
// which the lanes of one store write rows 8 apart, and rows 8 apart share a
// bank; the permutation spreads them over four banks, and the MFMA operand
// reads (a whole group of one row) follow the same map.
static_assert(BK == 32, "tn_slot permutes the four 8-pixel groups of a row");
__device__ __forceinline__ int tn_slot(int row, int k)
{
    return row * LDSK + ((((k >> 3) ^ (row >> 3)) & 3) << 3) + (k & 7);
}

template <bool CONV, int WM>
__global__ __launch_bounds__(256) void k_gemm_tn(const uint16_t* __restrict__ A, int64_t lda,
                                                 const uint16_t* __restrict__ B, int64_t ldb, ConvSrc cs, int P,
                                                 int M, int N, float* __restrict__ C, int64_t ldc,
                                                 float* __restrict__ parts)
{
    constexpr int WN = 4 / WM, TM = 32 * WM, TN = 32 * WN;
    constexpr int CA = (TM * 4 + 255) / 256, CB = (TN * 4 + 255) / 256;
    __shared__ uint16_t sA[2][TM * LDSK];  // [m][p]
    __shared__ uint16_t sB[2][TN * LDSK];  // [n][p]
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
    const int slice = (P + gridDim.z - 1) / gridDim.z;
    const int p_begin = blockIdx.z * slice;
    const int p_end = min(P, p_begin + slice);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave / WN) * 32, wn = (wave % WN) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // chunk u of a thread: pixel lp = tid / (T / 8) within the slice, columns
    // lc .. lc + 7; 32 pixels x T columns per operand
    constexpr int APR = TM / 8, BPR = TN / 8;  // chunks per pixel row
    ConvCursor cc[CB];
    int64_t pn[CB];
    int pr[CB], pq[CB];
    if (CONV) {
#pragma unroll
        for (int u = 0; u < CB; u++) {
            const int ch = tid + 256 * u;
            const int lp = ch / BPR, lc = (ch % BPR) * 8;
            cc[u].start(n0 + lc, cs.ci);
            const int p = p_begin + lp;
            pq[u] = p % cs.S;
            pr[u] = (p / cs.S) % cs.S;
            pn[u] = p / (cs.S * cs.S);
        }
    }
    uint4 va[CA], vb[CB];
    auto load = [&](int p0) {
#pragma unroll
        for (int u = 0; u < CA; u++) {
            const int ch = tid + 256 * u;
            const int lp = ch / APR, lc = (ch % APR) * 8;
            va[u] = (ch < 32 * APR) ? load8(A, lda, p0 + lp, p_end, m0 + lc, M) : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < CB; u++) {
            const int ch = tid + 256 * u;
            const int lp = ch / BPR, lc = (ch % BPR) * 8;
            if (ch >= 32 * BPR) {
                vb[u] = make_uint4(0, 0, 0, 0);
            } else if (CONV) {
                vb[u] = load8_conv(cs, pn[u], pr[u], pq[u], p0 + lp < p_end && n0 + lc < N, cc[u]);
                pq[u] += BK;
                while (pq[u] >= cs.S) {
                    pq[u] -= cs.S;
                    if (++pr[u] == cs.S) {
                        pr[u] = 0;
                        pn[u]++;
                    }
                }
            } else {
                vb[u] = load8(B, ldb, p0 + lp, p_end, n0 + lc, N);
            }
        }
    };
    auto stash = [&](int st) {
#pragma unroll
        for (int u = 0; u < CA; u++) {
            const int ch = tid + 256 * u;
            if (ch >= 32 * APR) continue;
            const int lp = ch / APR, lc = (ch % APR) * 8;
            const uint16_t* t = (const uint16_t*)&va[u];
#pragma unroll
            for (int j = 0; j < 8; j++) sA[st][tn_slot(lc + j, lp)] = t[j];
        }
#pragma unroll
        for (int u = 0; u < CB; u++) {
            const int ch = tid + 256 * u;
            if (ch >= 32 * BPR) continue;
            const int lp = ch / BPR, lc = (ch % BPR) * 8;
            const uint16_t* t = (const uint16_t*)&vb[u];
#pragma unroll
            for (int j = 0; j < 8; j++) sB[st][tn_slot(lc + j, lp)] = t[j];
        }
    };
    if (p_begin < p_end) {
        load(p_begin);
        stash(0);
    }
    __syncthreads();
    int cur = 0;
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    for (int p0 = p_begin; p0 < p_end; p0 += BK) {
        const bool more = p0 + BK < p_end;
        if (more) load(p0 + BK);
#pragma unroll
        for (int i = 0; i < 2; i++) {
            const bf16x8 a = as_bf16x8(*(const uint4*)&sA[cur][tn_slot(wm + 16 * i + fr, fk)]);
#pragma unroll
            for (int j = 0; j < 2; j++) {
                const bf16x8 b = as_bf16x8(*(const uint4*)&sB[cur][tn_slot(wn + 16 * j + fr, fk)]);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][j], 0, 0, 0);
            }
        }
        if (more) stash(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                const int n = n0 + wn + 16 * j + (lane & 15);
                if (m >= M || n >= N) continue;
                if (parts)  // this pixel slice's partial product, summed in a fixed order later
                    parts[((int64_t)blockIdx.z * M + m) * N + n] = acc[i][j][r];
                else
                    unsafeAtomicAdd(&C[(int64_t)m * ldc + n], acc[i][j][r]);
            }
}

// dst[m][n] (row stride ldd) += sum over k = 0, 1, ... nparts - 1 of
// parts[k pstride + e], e = m N + n < len: per-workgroup partial sums added
// in one fixed order, so the result does not depend on the order in which
// the workgroups ran.  One lane per element, the parts in sequence.
__global__ void k_reduce_parts(const float* __restrict__ parts, int nparts, int64_t pstride, int64_t len, int N,
                               float* __restrict__ dst, int64_t ldd)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int k = 0; k < nparts; k++) s += parts[(int64_t)k * pstride + e];
        const int64_t m = e / N, n = e - m * N;
        dst[m * ldd + n] += s;
    }
}

// The same sums for few elements and many parts: one workgroup per element,
// lane t summing parts t, t + 256, ... in sequence, then a tree over the
// lanes in a fixed pattern.
__global__ __launch_bounds__(256) void k_reduce_parts_wide(const float* __restrict__ parts, int nparts,
                                                           int64_t pstride, int64_t len, int N,
                                                           float* __restrict__ dst, int64_t ldd)
{
    __shared__ float red[256];
    for (int64_t e = blockIdx.x; e < len; e += gridDim.x) {
        float s = 0.f;
        for (int k = threadIdx.x; k < nparts; k += 256) s += parts[(int64_t)k * pstride + e];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const int64_t m = e / N, n = e - m * N;
            dst[m * ldd + n] += red[0];
        }
        __syncthreads();
    }
}

// Unfolds 3x3 neighbourhoods (zero padding): col[p][t * ci + c] =
// x[n][y + ty - 1][x + tx - 1][c] (channel stride xs, offset xo), K padded
// with zeros to kpad.
__global__ void k_im2col3(const uint16_t* __restrict__ x, int xs, int xo, int B, int S, int ci,
                          uint16_t* __restrict__ col, int kpad)
{
    const int64_t total = (int64_t)B * S * S * kpad;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(e % kpad);
        const int64_t p = e / kpad;
        uint16_t v = 0;
        if (k < 9 * ci) {
            const int t = k / ci, c = k - t * ci;
            const int q = (int)(p % S), r = (int)((p / S) % S);
            const int64_t n = p / ((int64_t)S * S);
            const int rr = r + t / 3 - 1, qq = q + t % 3 - 1;
            if (rr >= 0 && rr < S && qq >= 0 && qq < S) v = x[((n * S + rr) * S + qq) * xs + xo + c];
        }
        col[e] = v;
    }
}

// Gathers the 2x2 children of every coarse pixel: g[p][t * c + o] =
// dy[n][2 r + t / 2][2 q + t % 2][o] (channel stride ys, offset yo).
__global__ void k_gather_children(const uint16_t* __restrict__ dy, int ys, int yo, int B, int S, int c,
                                  uint16_t* __restrict__ g)
{
    const int64_t total = (int64_t)B * S * S * 4 * c;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(e % (4 * c));
        const int64_t p = e / (4 * c);
        const int t = k / c, o = k - t * c;
        const int q = (int)(p % S), r = (int)((p / S) % S);
        const int64_t n = p / ((int64_t)S * S);
        const int S2 = 2 * S;
        g[e] = dy[((n * S2 + 2 * r + t / 2) * S2 + 2 * q + t % 2) * ys + yo + o];
    }
}

// 2x2 max pool (ties: first in row-major order) of x (stride xs), keeping the
// winner's index for the backward pass.
__global__ void k_maxpool(const uint16_t* __restrict__ x, int xs, int B, int S, int c,
                          uint16_t* __restrict__ y, uint8_t* __restrict__ arg)
{
    const int H = S / 2;
    const int64_t total = (int64_t)B * H * H * c;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int o = (int)(e % c);
        const int64_t p = e / c;
        const int q = (int)(p % H), r = (int)((p / H) % H);
        const int64_t n = p / ((int64_t)H * H);
        float bv = 0.f;
        int best = 0;
        for (int t = 0; t < 4; t++) {
            const float v = fb(x[((n * S + 2 * r + t / 2) * S + 2 * q + t % 2) * xs + o]);
            if (t == 0 || v > bv) {
                bv = v;
                best = t;
            }
        }
        y[e] = bf(bv);
        arg[e] = (uint8_t)best;
    }
}

// dx[winner] += dy (both FP32; dx stride dxs).
__global__ void k_maxpool_bwd(const float* __restrict__ dy, const uint8_t* __restrict__ arg, int B, int S,
                              int c, float* __restrict__ dx, int dxs)
{
    const int H = S / 2;
    const int64_t total = (int64_t)B * H * H * c;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int o = (int)(e % c);
        const int64_t p = e / c;
        const int q = (int)(p % H), r = (int)((p / H) % H);
        const int64_t n = p / ((int64_t)H * H);
        const int t = arg[e];
        dx[((n * S + 2 * r + t / 2) * S + 2 * q + t % 2) * dxs + o] += dy[e];
    }
}

// g (BF16 out) = (acc + add) * (y > 0), over n x c elements with strides.
__global__ void k_relu_mask_add(const float* __restrict__ acc, int as, const float* __restrict__ add, int ads,
                                const uint16_t* __restrict__ y, int ysd, int64_t rows, int c,
                                uint16_t* __restrict__ g, int gs)
{
    const int64_t total = rows * c;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int o = (int)(e % c);
        const int64_t p = e / c;
        float v = acc[p * as + o] + (add ? add[p * ads + o] : 0.f);
        if (y && !(fb(y[p * ysd + o]) > 0.f)) v = 0.f;  // no y: no ReLU mask
        g[p * gs + o] = bf(v);
    }
}

// Column sums db[o] += sum_p g[p][o] (BF16 g, row stride gs): a workgroup
// sums a contiguous range of rows for 64 columns at a time (4 row lanes per
// column, coalesced 128-byte rows), then one atomic per (workgroup, column).
__global__ __launch_bounds__(256) void k_colsum(const uint16_t* __restrict__ g, int gs, int64_t rows, int c,
                                                float* __restrict__ db, float* __restrict__ parts)
{
    const int oc = threadIdx.x & 63, rl = threadIdx.x >> 6;
    const int64_t per = (rows + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(rows, r0 + per);
    __shared__ float red[4][64];
    for (int c0 = 0; c0 < c; c0 += 64) {
        const int o = c0 + oc;
        float sum = 0.f;
        if (o < c)
            for (int64_t p = r0 + rl; p < r1; p += 4) sum += fb(g[p * gs + o]);
        red[rl][oc] = sum;
        __syncthreads();
        if (rl == 0 && o < c) {
            const float t = red[0][oc] + red[1][oc] + red[2][oc] + red[3][oc];
            if (parts)
                parts[(int64_t)blockIdx.x * c + o] = t;
            else if (t != 0.f)
                unsafeAtomicAdd(&db[o], t);
        }
        __syncthreads();
    }
}

// k_colsum for rows of 8-channel chunks (c % 8 == 0, 256 divisible by c / 8,
// 16-byte aligned rows): each thread reads one 16-byte chunk of a row per
// step and keeps 8 partial sums; the workgroup then adds the partial sums
// of each channel in LDS, one atomic per channel and workgroup.
__global__ __launch_bounds__(256) void k_colsum8(const uint16_t* __restrict__ g, int gs, int64_t rows, int c,
                                                 float* __restrict__ db, float* __restrict__ parts)
{
    __shared__ float red[256][9];  // padded against bank conflicts in the column sums
    const int t = threadIdx.x, cpr = c >> 3, q = t % cpr, rr = t / cpr, rstep = 256 / cpr;
    const int64_t per = (rows + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(rows, r0 + per);
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int64_t p = r0 + rr; p < r1; p += rstep) {
        const uint4 v = *(const uint4*)(g + p * gs + q * 8);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 4; j++) {
            acc[2 * j] += __uint_as_float(w[j] << 16);
            acc[2 * j + 1] += __uint_as_float(w[j] & 0xffff0000u);
        }
    }
#pragma unroll
    for (int j = 0; j < 8; j++) red[t][j] = acc[j];
    __syncthreads();
    if (t < c) {  // channel t = chunk t / 8, element t % 8
        float sum = 0.f;
        for (int k = 0; k < rstep; k++) sum += red[k * cpr + (t >> 3)][t & 7];
        if (parts)
            parts[(int64_t)blockIdx.x * c + t] = sum;
        else if (sum != 0.f)
            unsafeAtomicAdd(&db[t], sum);
    }
}

// Cells of the target that count in the loss (mask > 0) into *count, which
// must hold 0: a wave sum per wave, one integer atomic per workgroup (exact,
// so the total does not depend on the order).
__global__ __launch_bounds__(256) void k_mask_count(const float* __restrict__ mask, int64_t P, int* __restrict__ count)
{
    int n = 0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x)
        n += mask[p] > 0.f;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o);
    __shared__ int red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int tot = red[0] + red[1] + red[2] + red[3];
        if (tot) atomicAdd(count, tot);
    }
}

// Head (1x1 convolution, 2 outputs, FP32 weights) and the Gaussian NLL over
// mask > 0, averaged over the *count such cells (the loss's normaliser):
// writes out (optional); with a target, the per-pixel output
// gradient gout[p] = (dL/dm, dL/ds), the bias gradient and the loss
// (reduced per workgroup, one atomic each), and the gradient with respect to
// d0's pre-activation (BF16, ReLU-masked by d0).
template <bool V8>
__global__ __launch_bounds__(256) void k_head(const uint16_t* __restrict__ d0, int c, int64_t P,
                                              const float* __restrict__ w, const float* __restrict__ b,
                                              const float* __restrict__ target, const float* __restrict__ mask,
                                              const int* __restrict__ count, float* __restrict__ out,
                                              float* __restrict__ loss,
                                              float2* __restrict__ gout, float* __restrict__ gb,
                                              uint16_t* __restrict__ gd0, float* __restrict__ parts)
{
    float l_acc = 0.f, g0_acc = 0.f, g1_acc = 0.f;
    // 1 / (cells in the loss), rounded once from binary64 (an empty mask
    // counts as one cell: the loss and its gradient are then zero)
    const float inv_count = target ? (float)(1.0 / (double)max(*count, 1)) : 0.f;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        float o0 = b[0], o1 = b[1];
        if (V8) {  // the row in 16-byte chunks, summed in the same channel order
            for (int i0 = 0; i0 < c; i0 += 8) {
                const uint4 v = *(const uint4*)(d0 + p * c + i0);
                const uint32_t vw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int j = 0; j < 8; j++) {
                    const float a = __uint_as_float((j & 1) ? (vw[j >> 1] & 0xffff0000u) : (vw[j >> 1] << 16));
                    o0 += a * w[2 * (i0 + j)];
                    o1 += a * w[2 * (i0 + j) + 1];
                }
            }
        } else {
            for (int i = 0; i < c; i++) {
                const float a = fb(d0[p * c + i]);
                o0 += a * w[2 * i];
                o1 += a * w[2 * i + 1];
            }
        }
        if (out) {
            out[2 * p] = o0;
            out[2 * p + 1] = o1;
        }
        if (!target) continue;
        float g0 = 0.f, g1 = 0.f;
        if (mask[p] > 0.f) {
            const float r = target[p] - o0, e = expf(-o1);
            l_acc += 0.5f * (o1 + r * r * e) * inv_count;
            g0 = -r * e * inv_count;
            g1 = 0.5f * (1.f - r * r * e) * inv_count;
        }
        g0_acc += g0;
        g1_acc += g1;
        gout[p] = make_float2(g0, g1);
        if (V8) {
            for (int i0 = 0; i0 < c; i0 += 8) {
                const uint4 v = *(const uint4*)(d0 + p * c + i0);
                const uint32_t vw[4] = {v.x, v.y, v.z, v.w};
                uint32_t ow[4];
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const float a0 = __uint_as_float(vw[j] << 16), a1 = __uint_as_float(vw[j] & 0xffff0000u);
                    const int i = i0 + 2 * j;
                    const uint16_t r0 = bf((a0 > 0.f) ? g0 * w[2 * i] + g1 * w[2 * i + 1] : 0.f);
                    const uint16_t r1 = bf((a1 > 0.f) ? g0 * w[2 * i + 2] + g1 * w[2 * i + 3] : 0.f);
                    ow[j] = (uint32_t)r0 | ((uint32_t)r1 << 16);
                }
                *(uint4*)(gd0 + p * c + i0) = make_uint4(ow[0], ow[1], ow[2], ow[3]);
            }
        } else {
            for (int i = 0; i < c; i++) {
                const float a = fb(d0[p * c + i]);
                gd0[p * c + i] = bf((a > 0.f) ? g0 * w[2 * i] + g1 * w[2 * i + 1] : 0.f);
            }
        }
    }
    if (!target) return;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        l_acc += __shfl_xor(l_acc, o);
        g0_acc += __shfl_xor(g0_acc, o);
        g1_acc += __shfl_xor(g1_acc, o);
    }
    __shared__ float red[3][4];
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wave] = l_acc;
        red[1][wave] = g0_acc;
        red[2][wave] = g1_acc;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const float v = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
        if (parts)
            parts[(int64_t)blockIdx.x * 3 + threadIdx.x] = v;
        else if (v != 0.f)
            unsafeAtomicAdd(threadIdx.x == 0 ? loss : &gb[threadIdx.x - 1], v);
    }
}

// Head weight gradient gw[i][j] = sum_p d0[p][i] gout[p][j]: a workgroup
// sums a range of pixels for 64 channels (4 pixel lanes per channel), then
// one atomic per (workgroup, weight).
__global__ __launch_bounds__(256) void k_head_wgrad(const uint16_t* __restrict__ d0, int c, int64_t P,
                                                    const float2* __restrict__ gout, float* __restrict__ gw,
                                                    float* __restrict__ parts)
{
    const int oc = threadIdx.x & 63, pl = threadIdx.x >> 6;
    const int64_t per = (P + gridDim.x - 1) / gridDim.x;
    const int64_t p0 = (int64_t)blockIdx.x * per, p1 = min(P, p0 + per);
    __shared__ float red[4][64][2];
    for (int c0 = 0; c0 < c; c0 += 64) {
        const int i = c0 + oc;
        float s0 = 0.f, s1 = 0.f;
        if (i < c)
            for (int64_t p = p0 + pl; p < p1; p += 4) {
                const float a = fb(d0[p * c + i]);
                const float2 g = gout[p];
                s0 += a * g.x;
                s1 += a * g.y;
            }
        red[pl][oc][0] = s0;
        red[pl][oc][1] = s1;
        __syncthreads();
        if (pl == 0 && i < c) {
            const float t0 = red[0][oc][0] + red[1][oc][0] + red[2][oc][0] + red[3][oc][0];
            const float t1 = red[0][oc][1] + red[1][oc][1] + red[2][oc][1] + red[3][oc][1];
            if (parts) {
                parts[(int64_t)blockIdx.x * 2 * c + 2 * i] = t0;
                parts[(int64_t)blockIdx.x * 2 * c + 2 * i + 1] = t1;
            } else {
                if (t0 != 0.f) unsafeAtomicAdd(&gw[2 * i], t0);
                if (t1 != 0.f) unsafeAtomicAdd(&gw[2 * i + 1], t1);
            }
        }
        __syncthreads();
    }
}

// 8-channel forms of k_relu_mask_add and k_add_f32 for rows of 8-channel
// chunks (c / 8 a power of two, 2^sh; every stride a multiple of 8 and the
// rows 16-byte aligned): one thread per chunk, vector loads and stores.
__global__ void k_relu_mask_add8(const float* __restrict__ acc, int as, const float* __restrict__ add, int ads,
                                 const uint16_t* __restrict__ y, int ysd, int64_t rows, int sh,
                                 uint16_t* __restrict__ g, int gs)
{
    const int64_t total = rows << sh;
    const int qm = (1 << sh) - 1;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e >> sh;
        const int o = (int)(e & qm) * 8;
        const float4 a0 = *(const float4*)(acc + p * as + o), a1 = *(const float4*)(acc + p * as + o + 4);
        float v[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
        if (add) {
            const float4 d0 = *(const float4*)(add + p * ads + o), d1 = *(const float4*)(add + p * ads + o + 4);
            const float dv[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
#pragma unroll
            for (int j = 0; j < 8; j++) v[j] += dv[j];
        }
        if (y) {  // no y: no ReLU mask
            const uint4 yv = *(const uint4*)(y + p * ysd + o);
            const uint32_t yw[4] = {yv.x, yv.y, yv.z, yv.w};
#pragma unroll
            for (int j = 0; j < 4; j++) {
                if (!(__uint_as_float(yw[j] << 16) > 0.f)) v[2 * j] = 0.f;
                if (!(__uint_as_float(yw[j] & 0xffff0000u) > 0.f)) v[2 * j + 1] = 0.f;
            }
        }
        uint4 out;
        out.x = (uint32_t)bf(v[0]) | ((uint32_t)bf(v[1]) << 16);
        out.y = (uint32_t)bf(v[2]) | ((uint32_t)bf(v[3]) << 16);
        out.z = (uint32_t)bf(v[4]) | ((uint32_t)bf(v[5]) << 16);
        out.w = (uint32_t)bf(v[6]) | ((uint32_t)bf(v[7]) << 16);
        *(uint4*)(g + p * gs + o) = out;
    }
}

__global__ void k_add_f32_8(float* __restrict__ dst, int ds, const float* __restrict__ src, int ss, int64_t rows,
                            int sh)
{
    const int64_t total = rows << sh;
    const int qm = (1 << sh) - 1;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e >> sh;
        const int o = (int)(e & qm) * 8;
        float4* d = (float4*)(dst + p * ds + o);
        const float4* r = (const float4*)(src + p * ss + o);
        float4 x0 = d[0], x1 = d[1];
        const float4 y0 = r[0], y1 = r[1];
        x0.x += y0.x; x0.y += y0.y; x0.z += y0.z; x0.w += y0.w;
        x1.x += y1.x; x1.y += y1.y; x1.z += y1.z; x1.w += y1.w;
        d[0] = x0;
        d[1] = x1;
    }
}

// k_head_wgrad for rows of 8-channel chunks (c % 8 == 0, 256 divisible by
// c / 8, 16-byte aligned rows): a thread sums 8 channels' products for its
// pixels, then the workgroup adds them per weight in LDS.
__global__ __launch_bounds__(256) void k_head_wgrad8(const uint16_t* __restrict__ d0, int c, int64_t P,
                                                     const float2* __restrict__ gout, float* __restrict__ gw,
                                                     float* __restrict__ parts)
{
    __shared__ float red[256][17];  // 8 channels x 2 outputs, padded
    const int t = threadIdx.x, cpr = c >> 3, q = t % cpr, pl = t / cpr, pstep = 256 / cpr;
    const int64_t per = (P + gridDim.x - 1) / gridDim.x;
    const int64_t p0 = (int64_t)blockIdx.x * per, p1 = min(P, p0 + per);
    float s0[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, s1[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int64_t p = p0 + pl; p < p1; p += pstep) {
        const uint4 v = *(const uint4*)(d0 + p * c + q * 8);
        const uint32_t vw[4] = {v.x, v.y, v.z, v.w};
        const float2 g = gout[p];
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const float a = __uint_as_float((j & 1) ? (vw[j >> 1] & 0xffff0000u) : (vw[j >> 1] << 16));
            s0[j] += a * g.x;
            s1[j] += a * g.y;
        }
    }
#pragma unroll
    for (int j = 0; j < 8; j++) {
        red[t][2 * j] = s0[j];
        red[t][2 * j + 1] = s1[j];
    }
    __syncthreads();
    if (t < 2 * c) {  // weight t: channel t / 2, output t % 2
        const int i = t >> 1, o = t & 1;
        float sum = 0.f;
        for (int k = 0; k < pstep; k++) sum += red[k * cpr + (i >> 3)][2 * (i & 7) + o];
        if (parts)
            parts[(int64_t)blockIdx.x * 2 * c + t] = sum;
        else if (sum != 0.f)
            unsafeAtomicAdd(&gw[t], sum);
    }
}

// dst[p][o] += src[p][o] (FP32, strides ds / ss).
__global__ void k_add_f32(float* __restrict__ dst, int ds, const float* __restrict__ src, int ss, int64_t rows, int c)
{
    const int64_t total = rows * c;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int o = (int)(e % c);
        const int64_t p = e / c;
        dst[p * ds + o] += src[p * ss + o];
    }
}

__global__ void k_cast_bf16(const float* __restrict__ x, int64_t n, uint16_t* __restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = bf(x[i]);
}

// Zeroes every segment of `fl` in one launch: blockIdx.y picks the segment.
__global__ void k_zero_many(FillList fl)
{
    const int sgm = blockIdx.y;
    if (sgm >= fl.n) return;
    float* x = fl.p[sgm];
    const int64_t n = fl.len[sgm];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = 0.0f;
}

__global__ void k_fill(float* __restrict__ x, int64_t n, float v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

// Weight layouts.  Master weights are the flat FP32 array (per layer
// [taps][ci][co] then bias).  Forward operand of a 3x3 conv: wf[co][t ci + c]
// (K padded to kpad); its input-gradient operand (flipped taps):
// wd[c][t' co + o] = W[8 - t'][c][o]; transposed conv forward operand
// wu[t co + o][c] = U[t][c][o]; its input-gradient operand
// wub[c][t co + o] = U[t][c][o].
__device__ __forceinline__ void relayout_job(const float* __restrict__ w, int taps, int ci, int co, int kind, int kpad,
                                             uint16_t* __restrict__ dst, int64_t e0, int64_t stride)
{
    const int64_t total = (int64_t)taps * ci * co;
    for (int64_t e = e0; e < total; e += stride) {
        const int o = (int)(e % co);
        const int c = (int)((e / co) % ci);
        const int t = (int)(e / ((int64_t)co * ci));
        const uint16_t v = bf(w[e]);
        switch (kind) {
        case 0: dst[(int64_t)o * kpad + t * ci + c] = v; break;                    // conv fwd
        case 1: dst[(int64_t)c * kpad + (taps - 1 - t) * co + o] = v; break;       // conv dgrad
        case 2: dst[((int64_t)t * co + o) * ci + c] = v; break;                    // convT fwd
        default: dst[(int64_t)c * (taps * co) + t * co + o] = v; break;            // convT dgrad
        }
    }
}

__global__ void k_relayout_many(WJobs js)
{
    if ((int)blockIdx.y >= js.n) return;
    const WJob& J = js.j[blockIdx.y];
    relayout_job((const float*)J.src, J.taps, J.ci, J.co, J.kind, J.kpad, (uint16_t*)J.dst,
                 (int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

// Back to the flat layout: conv gradient g[co][t ci + c] (ld kpad) or convT
// gradient g[t co + o][c] -> flat[t][c][o].
__global__ void k_grad_to_flat_many(WJobs js)
{
    if ((int)blockIdx.y >= js.n) return;
    const WJob& J = js.j[blockIdx.y];
    const float* g = (const float*)J.src;
    float* flat = (float*)J.dst;
    const int64_t total = (int64_t)J.taps * J.ci * J.co;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int o = (int)(e % J.co);
        const int c = (int)((e / J.co) % J.ci);
        const int t = (int)(e / ((int64_t)J.co * J.ci));
        flat[e] = (J.kind == 0) ? g[(int64_t)o * J.kpad + t * J.ci + c] : g[((int64_t)t * J.co + o) * J.ci + c];
    }
}

__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// Network input from a map: (h - z_ref, ln(sqrt(v) / 0.01), mask), all 0
// where the cell has no height.
__global__ void k_map_input(const float* __restrict__ h, const float* __restrict__ v, Grid g, float z_ref,
                            float* __restrict__ x)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.W * g.H) return;
    const int ix = j % g.W, iy = j / g.W;
    int sx = ix + g.rx;
    sx -= (sx >= g.W) ? g.W : 0;
    int sy = iy + g.ry;
    sy -= (sy >= g.H) ? g.H : 0;
    const int st = sy * g.W + sx;
    const float hv = h[st];
    const bool ok = !isnan(hv);
    x[3 * j] = ok ? hv - z_ref : 0.f;
    x[3 * j + 1] = ok ? 0.5f * logf(v[st]) - kLogSigmaRef : 0.f;
    x[3 * j + 2] = ok ? 1.f : 0.f;
}

// Gate: a cell with a classical height keeps it (read from the map's own
// layers when h is given, so it is returned unchanged; else rebuilt from the
// window input); a cell without one takes the network's height where its
// predicted standard deviation is below sigma_max, else NaN.
__global__ void k_gate(const float* __restrict__ x, const float* __restrict__ out, int64_t P, float z_ref,
                       float sigma_max, const float* __restrict__ h, const float* __restrict__ v, Grid g,
                       float* __restrict__ out_h, float* __restrict__ out_sigma)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        const bool observed = x[3 * p + 2] > 0.f;
        if (observed && h) {
            const int ix = (int)(p % g.W), iy = (int)(p / g.W);
            int sx = ix + g.rx;
            sx -= (sx >= g.W) ? g.W : 0;
            int sy = iy + g.ry;
            sy -= (sy >= g.H) ? g.H : 0;
            const int st = sy * g.W + sx;
            out_h[p] = h[st];
            out_sigma[p] = sqrtf(v[st]);
        } else if (observed) {
            out_h[p] = x[3 * p] + z_ref;
            out_sigma[p] = expf(x[3 * p + 1] + kLogSigmaRef);
        } else {
            const float sig = expf(0.5f * out[2 * p + 1]);
            const bool take = sig < sigma_max;
            out_h[p] = take ? out[2 * p] + z_ref : __builtin_nanf("");
            out_sigma[p] = take ? sig : __builtin_nanf("");
        }
    }
}

inline unsigned grid_for(int64_t n)
{
    int64_t b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

}  // namespace

// Tile of a product: 128 x 32 for 32 or fewer output columns (no MFMA block
// on padding), else 64 x 64; both with waves of 32 x 32.  Larger tiles
// (256 x 32 and 128 x 128, waves of 64 x 32 and 64 x 64, so that each LDS
// fragment feeds more MFMAs) measured slower on every layer of the network
// (the products wait on their operand loads, not on LDS): they are kept for
// force_shape >= 0 (0: 64 x 64, 1: 128 x 32, 2: 256 x 32, 3: 128 x 128),
// which the tests use to check that every shape gives the same products.
void unet_gemm_nt(hipStream_t s, int epi, const uint16_t* A, int64_t lda, const ConvSrc* conv, const uint16_t* B,
                  int64_t ldb, int M, int N, int K, const Epilogue& ep, int n_cu, int force_shape)
{
    (void)n_cu;
    const ConvSrc cs = conv ? *conv : ConvSrc{nullptr, 0, 1, 1};
    const int shape = force_shape >= 0 ? (force_shape & 3) : (N <= 32 ? 1 : 0);
    const int TM = shape == 0 ? 64 : shape == 2 ? 256 : 128;
    const int TN = shape == 0 ? 64 : shape == 3 ? 128 : 32;
    dim3 grid((M + TM - 1) / TM, (N + TN - 1) / TN);
#define MEM_GNT(E, CV, W, WTM, WTN) \
    hipLaunchKernelGGL((k_gemm_nt<E, CV, W, WTM, WTN>), grid, dim3(256), 0, s, A, lda, cs, B, ldb, M, N, K, ep)
#define MEM_GNT_S(E, CV)                                            \
    switch (shape) {                                                \
    case 1: MEM_GNT(E, CV, 4, 32, 32); break;                       \
    case 2: MEM_GNT(E, CV, 4, 64, 32); break;                       \
    case 3: MEM_GNT(E, CV, 2, 64, 64); break;                       \
    default: MEM_GNT(E, CV, 2, 32, 32); break;                      \
    }
#define MEM_GNT_E(CV)                                      \
    switch (epi) {                                         \
    case EPI_STORE: MEM_GNT_S(EPI_STORE, CV) break;        \
    case EPI_CONVT: MEM_GNT_S(EPI_CONVT, CV) break;        \
    default: MEM_GNT_S(EPI_F32, CV) break;                 \
    }
    if (conv) {
        MEM_GNT_E(true)
    } else {
        MEM_GNT_E(false)
    }
#undef MEM_GNT_E
#undef MEM_GNT_S
#undef MEM_GNT
}

// Narrow outputs (32 rows or fewer) take 32x128 tiles; the pixels are split
// over enough workgroups to give each CU four.
static int tn_split(int P, int M, int N, int n_cu, int* TM, int* TN)
{
    const bool narrow = M <= 32;
    *TM = narrow ? 32 : 64;
    *TN = narrow ? 128 : 64;
    const int tiles = ((M + *TM - 1) / *TM) * ((N + *TN - 1) / *TN);
    int split = (4 * n_cu + tiles - 1) / tiles;
    const int max_split = (P + 255) / 256;
    if (split > max_split) split = max_split;
    if (split < 1) split = 1;
    return split;
}

size_t unet_tn_parts(int P, int M, int N, int n_cu)
{
    int TM, TN;
    return (size_t)tn_split(P, M, N, n_cu, &TM, &TN) * M * N;
}

// dst (rows of N, stride ldd) += the fixed-order sum of nparts partial
// arrays of len elements (the k-th at parts + k pstride).
static void reduce_parts(hipStream_t s, const float* parts, int nparts, int64_t pstride, int64_t len, int N,
                         float* dst, int64_t ldd)
{
    if (len <= 65536 && nparts > 64) {
        const unsigned g = (unsigned)std::min<int64_t>(len, 4096);
        hipLaunchKernelGGL(k_reduce_parts_wide, dim3(g), dim3(256), 0, s, parts, nparts, pstride, len, N, dst, ldd);
    } else {
        hipLaunchKernelGGL(k_reduce_parts, dim3(grid_for(len)), dim3(256), 0, s, parts, nparts, pstride, len, N, dst,
                           ldd);
    }
}

void unet_gemm_tn(hipStream_t s, const uint16_t* A, int64_t lda, const uint16_t* B, int64_t ldb, const ConvSrc* conv,
                  int P, int M, int N, float* C, int64_t ldc, int n_cu, float* parts)
{
    int TM, TN;
    const int split = tn_split(P, M, N, n_cu, &TM, &TN);
    const bool narrow = M <= 32;
    dim3 grid((M + TM - 1) / TM, (N + TN - 1) / TN, split);
    const ConvSrc cs = conv ? *conv : ConvSrc{nullptr, 0, 1, 1};
    if (conv) {
        if (narrow)
            hipLaunchKernelGGL((k_gemm_tn<true, 1>), grid, dim3(256), 0, s, A, lda, B, ldb, cs, P, M, N, C, ldc, parts);
        else
            hipLaunchKernelGGL((k_gemm_tn<true, 2>), grid, dim3(256), 0, s, A, lda, B, ldb, cs, P, M, N, C, ldc, parts);
    } else {
        if (narrow)
            hipLaunchKernelGGL((k_gemm_tn<false, 1>), grid, dim3(256), 0, s, A, lda, B, ldb, cs, P, M, N, C, ldc, parts);
        else
            hipLaunchKernelGGL((k_gemm_tn<false, 2>), grid, dim3(256), 0, s, A, lda, B, ldb, cs, P, M, N, C, ldc, parts);
    }
    if (parts) reduce_parts(s, parts, split, (int64_t)M * N, (int64_t)M * N, N, C, ldc);
}

void unet_im2col3(hipStream_t s, const uint16_t* x, int xs, int xo, int B, int S, int ci, uint16_t* col, int kpad)
{
    hipLaunchKernelGGL(k_im2col3, dim3(grid_for((int64_t)B * S * S * kpad)), dim3(256), 0, s, x, xs, xo, B, S, ci,
                       col, kpad);
}

void unet_gather_children(hipStream_t s, const uint16_t* dy, int ys, int yo, int B, int S, int c, uint16_t* g)
{
    hipLaunchKernelGGL(k_gather_children, dim3(grid_for((int64_t)B * S * S * 4 * c)), dim3(256), 0, s, dy, ys, yo,
                       B, S, c, g);
}

void unet_maxpool(hipStream_t s, const uint16_t* x, int xs, int B, int S, int c, uint16_t* y, uint8_t* arg)
{
    hipLaunchKernelGGL(k_maxpool, dim3(grid_for((int64_t)B * (S / 2) * (S / 2) * c)), dim3(256), 0, s, x, xs, B, S,
                       c, y, arg);
}

void unet_maxpool_bwd(hipStream_t s, const float* dy, const uint8_t* arg, int B, int S, int c, float* dx,
                      int dxs)
{
    hipLaunchKernelGGL(k_maxpool_bwd, dim3(grid_for((int64_t)B * (S / 2) * (S / 2) * c)), dim3(256), 0, s, dy,
                       arg, B, S, c, dx, dxs);
}

// log2(c / 8) when rows of c channels can be processed in 8-channel chunks
// with the given strides and base pointers, else -1.
static int chunk_shift(int c, std::initializer_list<int> strides, std::initializer_list<const void*> ptrs)
{
    if (c % 8 != 0) return -1;
    const int q = c / 8;
    if (q & (q - 1)) return -1;
    for (int st : strides)
        if (st % 8 != 0) return -1;
    for (const void* p : ptrs)
        if (((uintptr_t)p & 15) != 0) return -1;
    int sh = 0;
    while ((1 << sh) < q) sh++;
    return sh;
}

void unet_relu_mask_add(hipStream_t s, const float* acc, int as, const float* add, int ads, const uint16_t* y,
                        int ys, int64_t rows, int c, uint16_t* g, int gs)
{
    const int sh = chunk_shift(c, {as, add ? ads : 8, y ? ys : 8, gs}, {acc, add, y, g});
    if (sh >= 0) {
        hipLaunchKernelGGL(k_relu_mask_add8, dim3(grid_for(rows << sh)), dim3(256), 0, s, acc, as, add, ads, y, ys,
                           rows, sh, g, gs);
        return;
    }
    hipLaunchKernelGGL(k_relu_mask_add, dim3(grid_for(rows * c)), dim3(256), 0, s, acc, as, add, ads, y, ys, rows,
                       c, g, gs);
}

static int64_t colsum_blocks(int64_t rows)
{
    int64_t blocks = (rows + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    return blocks < 1 ? 1 : blocks;
}

size_t unet_colsum_parts(int64_t rows, int c)
{
    return (size_t)colsum_blocks(rows) * c;
}

void unet_colsum(hipStream_t s, const uint16_t* g, int gs, int64_t rows, int c, float* db, float* parts)
{
    const int64_t blocks = colsum_blocks(rows);
    const int cpr = c / 8;
    if (c % 8 == 0 && gs % 8 == 0 && cpr <= 256 && 256 % cpr == 0 && ((uintptr_t)g & 15) == 0)
        hipLaunchKernelGGL(k_colsum8, dim3((unsigned)blocks), dim3(256), 0, s, g, gs, rows, c, db, parts);
    else
        hipLaunchKernelGGL(k_colsum, dim3((unsigned)blocks), dim3(256), 0, s, g, gs, rows, c, db, parts);
    if (parts) reduce_parts(s, parts, (int)blocks, c, c, c, db, c);
}

static int64_t head_blocks(int64_t P)
{
    int64_t blocks = (P + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    return blocks < 1 ? 1 : blocks;
}

static int64_t head_wgrad_blocks(int64_t P)
{
    int64_t wb = (P + 1023) / 1024;
    if (wb > 512) wb = 512;
    return wb < 1 ? 1 : wb;
}

size_t unet_head_parts(int64_t P, int c)
{
    return (size_t)std::max(head_blocks(P) * 3, head_wgrad_blocks(P) * 2 * c);
}

void unet_head_loss(hipStream_t s, const uint16_t* d0, int c, int64_t P, const float* w, const float* b,
                    const float* target, const float* mask, const int* count, float* out, float* loss, float* gw,
                    float* gb, uint16_t* gd0, float2* gout, float* parts)
{
    const int64_t blocks = head_blocks(P);
    const int cpr = c / 8;
    const bool v8 = c % 8 == 0 && ((uintptr_t)d0 & 15) == 0 && (!gd0 || ((uintptr_t)gd0 & 15) == 0);
    float* hp = target ? parts : nullptr;
    if (v8)
        hipLaunchKernelGGL(k_head<true>, dim3((unsigned)blocks), dim3(256), 0, s, d0, c, P, w, b, target, mask, count,
                           out, loss, gout, gb, gd0, hp);
    else
        hipLaunchKernelGGL(k_head<false>, dim3((unsigned)blocks), dim3(256), 0, s, d0, c, P, w, b, target, mask,
                           count, out, loss, gout, gb, gd0, hp);
    if (!target) return;
    if (hp) {  // the loss, then the two bias gradients
        reduce_parts(s, hp, (int)blocks, 3, 1, 1, loss, 1);
        reduce_parts(s, hp + 1, (int)blocks, 3, 2, 2, gb, 2);
    }
    const int64_t wb = head_wgrad_blocks(P);
    if (v8 && 2 * c <= 256 && 256 % cpr == 0)
        hipLaunchKernelGGL(k_head_wgrad8, dim3((unsigned)wb), dim3(256), 0, s, d0, c, P, gout, gw, parts);
    else
        hipLaunchKernelGGL(k_head_wgrad, dim3((unsigned)wb), dim3(256), 0, s, d0, c, P, gout, gw, parts);
    if (parts) reduce_parts(s, parts, (int)wb, 2 * c, 2 * c, 2 * c, gw, 2 * c);
}

void unet_add_f32(hipStream_t s, float* dst, int ds, const float* src, int ss, int64_t rows, int c)
{
    const int sh = chunk_shift(c, {ds, ss}, {dst, src});
    if (sh >= 0) {
        hipLaunchKernelGGL(k_add_f32_8, dim3(grid_for(rows << sh)), dim3(256), 0, s, dst, ds, src, ss, rows, sh);
        return;
    }
    hipLaunchKernelGGL(k_add_f32, dim3(grid_for(rows * c)), dim3(256), 0, s, dst, ds, src, ss, rows, c);
}

void unet_cast_bf16(hipStream_t s, const float* x, int64_t n, uint16_t* y)
{
    hipLaunchKernelGGL(k_cast_bf16, dim3(grid_for(n)), dim3(256), 0, s, x, n, y);
}

void unet_mask_count(hipStream_t s, const float* mask, int64_t P, int* count)
{
    int64_t blocks = (P + 1023) / 1024;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_mask_count, dim3((unsigned)(blocks < 1 ? 1 : blocks)), dim3(256), 0, s, mask, P, count);
}

void unet_fill(hipStream_t s, float* x, int64_t n, float v)
{
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, s, x, n, v);
}

void unet_zero_many(hipStream_t s, const FillList& fl)
{
    if (fl.n <= 0) return;
    int64_t big = 1;
    for (int i = 0; i < fl.n; i++) big = fl.len[i] > big ? fl.len[i] : big;
    int64_t bx = (big + 255) / 256;
    if (bx > 1024) bx = 1024;
    hipLaunchKernelGGL(k_zero_many, dim3((unsigned)bx, (unsigned)fl.n), dim3(256), 0, s, fl);
}

static unsigned jobs_grid_x(const WJobs& js)
{
    int64_t big = 1;
    for (int i = 0; i < js.n; i++) big = std::max(big, (int64_t)js.j[i].taps * js.j[i].ci * js.j[i].co);
    return grid_for(big);
}

void unet_relayout_many(hipStream_t s, const WJobs& js)
{
    if (js.n > 0)
        hipLaunchKernelGGL(k_relayout_many, dim3(jobs_grid_x(js), (unsigned)js.n), dim3(256), 0, s, js);
}

void unet_grad_to_flat_many(hipStream_t s, const WJobs& js)
{
    if (js.n > 0)
        hipLaunchKernelGGL(k_grad_to_flat_many, dim3(jobs_grid_x(js), (unsigned)js.n), dim3(256), 0, s, js);
}

void unet_adam(hipStream_t s, float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
               float eps, float c1, float c2)
{
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, s, w, g, m, v, n, lr, b1, b2, eps, c1, c2);
}

void unet_map_input(hipStream_t s, const float* h, const float* v, const Grid& g, float z_ref, float* x)
{
    hipLaunchKernelGGL(k_map_input, dim3((g.W * g.H + 255) / 256), dim3(256), 0, s, h, v, g, z_ref, x);
}

void unet_gate(hipStream_t s, const float* x, const float* out, int64_t P, float z_ref, float sigma_max,
               const float* h, const float* v, const Grid& g, float* out_h, float* out_sigma)
{
    hipLaunchKernelGGL(k_gate, dim3(grid_for(P)), dim3(256), 0, s, x, out, P, z_ref, sigma_max, h, v, g, out_h,
                       out_sigma);
}

}  // namespace memk
