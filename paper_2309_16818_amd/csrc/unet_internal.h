// unet_internal.h - launchers and GEMM epilogues of the completion U-Net.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "codec.h"
#include "mem_internal.h"

namespace memk {

enum { EPI_STORE = 0, EPI_CONVT = 1, EPI_F32 = 2 };

// What a gemm_nt tile does with C[m][n].
//   EPI_STORE: out[m * ldo + off + n] = bf16(relu?(C + bias[n]))
//   EPI_CONVT: m is a coarse pixel of a B x S x S grid and n = t * co + o;
//              out[child(m, t) * ldo + off + o] = bf16(C + bias[o])
//   EPI_F32:   outf[m * ldf + n] = C
struct Epilogue {
    const float* bias;
    int relu;
    uint16_t* out;
    int64_t ldo;
    int off;
    float* outf;
    int64_t ldf;
    int S, co;
};

template <int EPI>
__device__ __forceinline__ void epilogue(const Epilogue& ep, int m, int n, float v)
{
    if (EPI == EPI_F32) {
        ep.outf[(int64_t)m * ep.ldf + n] = v;
    } else if (EPI == EPI_STORE) {
        if (ep.bias) v += ep.bias[n];
        if (ep.relu && v < 0.f) v = 0.f;
        ep.out[(int64_t)m * ep.ldo + ep.off + n] = f32_to_bf16(v);
    } else {
        const int t = n / ep.co, o = n - t * ep.co;
        v += ep.bias[o];
        const int q = m % ep.S, r = (m / ep.S) % ep.S, b = m / (ep.S * ep.S);
        const int S2 = 2 * ep.S;
        const int64_t px = ((int64_t)b * S2 + 2 * r + t / 2) * S2 + 2 * q + t % 2;
        ep.out[px * ep.ldo + ep.off + o] = f32_to_bf16(v);
    }
}

// The unfolded (im2col) matrix of a 3x3 zero-padded convolution input,
// read in place: row = pixel of a B x S x S NHWC grid, column k = tap * ci +
// channel, tap = 3 (dy + 1) + (dx + 1); channels at stride xs.  Usable when
// ci and xs are multiples of 8 (a K slice of 8 stays inside one tap and is
// one aligned 16-byte load).
struct ConvSrc {
    const uint16_t* x;
    int xs, ci, S;
};

// A (M x K, row stride lda) is dense, or the unfolded input `conv` (then A
// and lda are ignored and K = 9 ci).
void unet_gemm_nt(hipStream_t s, int epi, const uint16_t* A, int64_t lda, const ConvSrc* conv, const uint16_t* B,
                  int64_t ldb, int M, int N, int K, const Epilogue& ep, int n_cu,
                  int force_shape = -1);
// B (P x N, row stride ldb) is dense, or the unfolded input `conv` (N = 9 ci).
// parts (device, unet_tn_parts floats, or NULL for FP32 atomics): each
// pixel slice's partial product, summed into C in a fixed order afterwards,
// so the gradient does not depend on the order in which workgroups ran.
void unet_gemm_tn(hipStream_t s, const uint16_t* A, int64_t lda, const uint16_t* B, int64_t ldb, const ConvSrc* conv,
                  int P, int M, int N, float* C, int64_t ldc, int n_cu, float* parts);
size_t unet_tn_parts(int P, int M, int N, int n_cu);
// Up to kFillMax float buffers cleared by one launch.
constexpr int kFillMax = 32;
struct FillList {
    float* p[kFillMax];
    int64_t len[kFillMax];
    int n = 0;
    void add(float* q, int64_t l)
    {
        p[n] = q;
        len[n] = l;
        n++;
    }
};
void unet_zero_many(hipStream_t s, const FillList& fl);

// Per-layer weight layout conversions run as one launch (blockIdx.y = job):
// relayout jobs read a layer's FP32 master weights `src` (flat [taps][ci][co])
// and write a BF16 operand `dst`: kind 0 conv forward [co][t ci + c], kind 1
// conv input gradient [c][(taps - 1 - t) co + o] (both rows padded to kpad),
// kind 2 transposed-conv forward [t co + o][c], kind 3 its input gradient
// [c][t co + o]; gradient jobs read a layer's FP32 weight gradient (kind 0:
// [co][t ci + c], row kpad; kind 2: [t co + o][c]) and write it flat.
constexpr int kWJobsMax = 40;
struct WJob {
    const void* src;
    void* dst;
    int taps, ci, co, kind, kpad;
};
struct WJobs {
    WJob j[kWJobsMax];
    int n = 0;
    void add(const void* src, void* dst, int taps, int ci, int co, int kind, int kpad)
    {
        j[n] = WJob{src, dst, taps, ci, co, kind, kpad};
        n++;
    }
};
void unet_relayout_many(hipStream_t s, const WJobs& js);
void unet_grad_to_flat_many(hipStream_t s, const WJobs& js);
void unet_im2col3(hipStream_t s, const uint16_t* x, int xs, int xo, int B, int S, int ci, uint16_t* col,
                  int kpad);
void unet_gather_children(hipStream_t s, const uint16_t* dy, int ys, int yo, int B, int S, int c, uint16_t* g);
void unet_maxpool(hipStream_t s, const uint16_t* x, int xs, int B, int S, int c, uint16_t* y, uint8_t* arg);
void unet_maxpool_bwd(hipStream_t s, const float* dy, const uint8_t* arg, int B, int S, int c, float* dx,
                      int dxs);
void unet_add_f32(hipStream_t s, float* dst, int ds, const float* src, int ss, int64_t rows, int c);
void unet_relu_mask_add(hipStream_t s, const float* acc, int as, const float* add, int ads, const uint16_t* y,
                        int ys, int64_t rows, int c, uint16_t* g, int gs);
// parts: as for unet_gemm_tn (unet_colsum_parts floats, or NULL).
void unet_colsum(hipStream_t s, const uint16_t* g, int gs, int64_t rows, int c, float* db, float* parts);
size_t unet_colsum_parts(int64_t rows, int c);
// Adds the number of mask entries > 0 among P to *count (device int).
void unet_mask_count(hipStream_t s, const float* mask, int64_t P, int* count);
// Head output (out may be NULL) and, with a target, loss and head / d0
// gradients, the loss averaged over the *count masked cells (device int);
// gout (P float2) is scratch.
void unet_head_loss(hipStream_t s, const uint16_t* d0, int c, int64_t P, const float* w, const float* b,
                    const float* target, const float* mask, const int* count, float* out, float* loss, float* gw,
                    float* gb, uint16_t* gd0, float2* gout, float* parts);
size_t unet_head_parts(int64_t P, int c);
void unet_cast_bf16(hipStream_t s, const float* x, int64_t n, uint16_t* y);
void unet_fill(hipStream_t s, float* x, int64_t n, float v);
void unet_adam(hipStream_t s, float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
               float eps, float c1, float c2);
void unet_map_input(hipStream_t s, const float* h, const float* v, const Grid& g, float z_ref, float* x);
void unet_gate(hipStream_t s, const float* x, const float* out, int64_t P, float z_ref, float sigma_max,
               const float* h, const float* v, const Grid& g, float* out_h, float* out_sigma);

}  // namespace memk
