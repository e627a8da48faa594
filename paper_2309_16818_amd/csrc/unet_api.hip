// unet_api.hip - the completion U-Net: buffers, forward, backward, Adam, and
// mem_complete (include/mem.h).
//
// Network (4 levels, width c_l = base 2^l at resolution S / 2^l):
//   enc l:  a_l = relu(conv3(in_l)), e_l = relu(conv3(a_l)), in_{l+1} = pool(e_l)
//   dec l:  u_l = convT2(below) + b, m_l = relu(conv3([u_l, e_l])),
//           d_l = relu(conv3(m_l)), below = d_l (starting from e_3)
//   head:   out = conv1(d_0) -> (height, log variance)
// Levels 0..2 keep [u_l | e_l] in one buffer cat_l, so the encoder writes its
// skip output where the decoder reads it.  Parameters live as one flat FP32
// array (per layer [taps][Cin][Cout] then bias); every step re-lays them out
// as BF16 operands of the MFMA products.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "prof.h"
#include "unet_internal.h"

using namespace memk;

namespace memk {
mem_status api_fail(mem_status code, const char* fmt, ...);
}

namespace {

constexpr int NLAY = 18;
static_assert(NLAY + 6 <= kFillMax, "the gradient clear takes every layer buffer, g, de[0..3] and the loss");
static_assert(2 * NLAY <= kWJobsMax, "two relayout jobs per layer");

struct ULayer {
    int taps, ci, co;
    int64_t off;   // weights in the flat array; the bias follows
    int kind;      // 0 conv3, 2 convT2, 4 head
    int kf, kd;    // forward / input-gradient K (padded for conv3)
    uint16_t* wf = nullptr;
    uint16_t* wd = nullptr;
    float* gbuf = nullptr;  // weight gradient in the forward operand layout
};

int round32(int k) { return (k + 31) / 32 * 32; }

}  // namespace

struct mem_unet {
    int base = 0, S = 0, maxB = 0, n_cu = 256;
    int gemm_shape = -1;  // forced tile shape of the nt products (-1: automatic)
    float* parts = nullptr;  // per-workgroup partial sums of the gradient reductions
    int64_t n_params = 0;
    bool broken = false;
    ULayer L[NLAY];
    float *w = nullptr, *g = nullptr, *am = nullptr, *av = nullptr;  // flat params, grad, Adam moments
    int64_t step = 0;
    // activations (BF16, NHWC)
    uint16_t* x = nullptr;
    uint16_t *a[4] = {}, *cat[3] = {}, *e3 = nullptr, *p[3] = {}, *m[3] = {}, *d[3] = {};
    uint8_t* arg[3] = {};
    float* out = nullptr;
    // backward scratch
    uint16_t *col = nullptr, *g1 = nullptr, *g2 = nullptr, *gch = nullptr;
    float *tmpf = nullptr, *de[4] = {}, *loss = nullptr;
    float* xin = nullptr;  // mem_complete input
    memk::Profiler prof;
};

namespace {

mem_status ufail(mem_unet* u, hipError_t e, const char* what)
{
    if (u) u->broken = true;
    return api_fail(MEM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

int64_t P_at(const mem_unet* u, int B, int l) { return (int64_t)B * (u->S >> l) * (u->S >> l); }

uint16_t* e_ptr(mem_unet* u, int l) { return l < 3 ? u->cat[l] + (u->base << l) : u->e3; }
int e_stride(const mem_unet* u, int l) { return l < 3 ? 2 * (u->base << l) : (u->base << l); }

void build_layout(mem_unet* u)
{
    const int b = u->base;
    const int c[4] = {b, 2 * b, 4 * b, 8 * b};
    int k = 0, prev = 3;
    for (int l = 0; l < 4; l++) {
        u->L[k++] = ULayer{9, prev, c[l], 0, 0, 0, 0};
        u->L[k++] = ULayer{9, c[l], c[l], 0, 0, 0, 0};
        prev = c[l];
    }
    for (int l = 2; l >= 0; l--) {
        u->L[k++] = ULayer{4, c[l + 1], c[l], 0, 2, 0, 0};
        u->L[k++] = ULayer{9, 2 * c[l], c[l], 0, 0, 0, 0};
        u->L[k++] = ULayer{9, c[l], c[l], 0, 0, 0, 0};
    }
    u->L[k++] = ULayer{1, b, 2, 0, 4, 0, 0};
    int64_t off = 0;
    for (int i = 0; i < NLAY; i++) {
        ULayer& Y = u->L[i];
        Y.off = off;
        off += (int64_t)Y.taps * Y.ci * Y.co + Y.co;
        if (Y.kind == 0) {
            Y.kf = round32(9 * Y.ci);
            Y.kd = round32(9 * Y.co);
        } else if (Y.kind == 2) {
            Y.kf = Y.ci;
            Y.kd = 4 * Y.co;
        }
    }
    u->n_params = off;
}

float* bias(const mem_unet* u, float* flat, int i)
{
    const ULayer& Y = u->L[i];
    return flat + Y.off + (int64_t)Y.taps * Y.ci * Y.co;
}

template <class T>
bool ualloc(T** p, size_t n)
{
    return hipMalloc((void**)p, sizeof(T) * (n ? n : 1)) == hipSuccess;
}

void free_unet(mem_unet* u)
{
    u->prof.release();
    for (auto& Y : u->L) {
        (void)hipFree(Y.wf);
        (void)hipFree(Y.wd);
        (void)hipFree(Y.gbuf);
    }
    void* bufs[] = {u->w, u->g, u->am, u->av, u->x, u->e3, u->out, u->col, u->g1, u->g2, u->gch, u->tmpf,
                    u->loss, u->xin, u->parts};
    for (void* b : bufs) (void)hipFree(b);
    for (int l = 0; l < 4; l++) {
        (void)hipFree(u->a[l]);
        (void)hipFree(u->de[l]);
    }
    for (int l = 0; l < 3; l++) {
        (void)hipFree(u->cat[l]);
        (void)hipFree(u->p[l]);
        (void)hipFree(u->m[l]);
        (void)hipFree(u->d[l]);
        (void)hipFree(u->arg[l]);
    }
    delete u;
}

// BF16 operands from the FP32 master weights, every layer in one launch.
// The K padding of the convolution operands is never written here: it was
// zeroed once when the network was created.
void relayout_all(mem_unet* u, hipStream_t s)
{
    WJobs js;
    for (int i = 0; i < NLAY; i++) {
        ULayer& Y = u->L[i];
        if (Y.kind == 4) continue;
        const float* W = u->w + Y.off;
        if (Y.kind == 0) {
            js.add(W, Y.wf, Y.taps, Y.ci, Y.co, 0, Y.kf);
            js.add(W, Y.wd, Y.taps, Y.ci, Y.co, 1, Y.kd);
        } else {
            js.add(W, Y.wf, Y.taps, Y.ci, Y.co, 2, 0);
            js.add(W, Y.wd, Y.taps, Y.ci, Y.co, 3, 0);
        }
    }
    u->prof.timed(s, "relayout", [&] { unet_relayout_many(s, js); });
}

// A convolution input whose channels and stride are multiples of 8 is read
// by the matrix products in place; others (the 3-channel network input,
// narrow test networks) are unfolded into `col` first.
bool implicit(int ci, int xs) { return ci % 8 == 0 && xs % 8 == 0; }

// y = relu(conv3(x) + b) into out (stride ldo, channel offset off).
void conv_fwd(mem_unet* u, hipStream_t s, int i, const uint16_t* x, int xs, int B, int l, uint16_t* out,
              int64_t ldo, int off)
{
    const ULayer& Y = u->L[i];
    const int S = u->S >> l;
    Epilogue ep{bias(u, u->w, i), 1, out, ldo, off, nullptr, 0, 0, 0};
    const int P = (int)P_at(u, B, l);
    if (implicit(Y.ci, xs)) {  // the GEMM reads the unfolded input in place
        const ConvSrc cs{x, xs, Y.ci, S};
        u->prof.timed(s, "gemm_fwd", [&] {
            unet_gemm_nt(s, EPI_STORE, nullptr, 0, &cs, Y.wf, Y.kf, P, Y.co, 9 * Y.ci, ep, u->n_cu, u->gemm_shape);
        });
        return;
    }
    u->prof.timed(s, "im2col", [&] { unet_im2col3(s, x, xs, 0, B, S, Y.ci, u->col, Y.kf); });
    u->prof.timed(s, "gemm_fwd", [&] {
        unet_gemm_nt(s, EPI_STORE, u->col, Y.kf, nullptr, Y.wf, Y.kf, P, Y.co, Y.kf, ep, u->n_cu, u->gemm_shape);
    });
}

void forward(mem_unet* u, hipStream_t s, int B)
{
    const int b = u->base;
    const uint16_t* in = u->x;
    int ci_stride = 3;
    for (int l = 0; l < 4; l++) {
        const int c = b << l;
        conv_fwd(u, s, 2 * l, in, ci_stride, B, l, u->a[l], c, 0);
        conv_fwd(u, s, 2 * l + 1, u->a[l], c, B, l, e_ptr(u, l), e_stride(u, l), 0);
        if (l < 3) {
            u->prof.timed(s, "pool", [&] {
                unet_maxpool(s, e_ptr(u, l), e_stride(u, l), B, u->S >> l, c, u->p[l], u->arg[l]);
            });
            in = u->p[l];
            ci_stride = c;
        }
    }
    const uint16_t* below = u->e3;
    for (int l = 2; l >= 0; l--) {
        const int c = b << l, k = 8 + 3 * (2 - l);
        const ULayer& U = u->L[k];
        Epilogue ep{bias(u, u->w, k), 0, u->cat[l], 2 * c, 0, nullptr, 0, u->S >> (l + 1), c};
        u->prof.timed(s, "gemm_up", [&] {
            unet_gemm_nt(s, EPI_CONVT, below, U.ci, nullptr, U.wf, U.ci, (int)P_at(u, B, l + 1), 4 * c, U.ci, ep, u->n_cu, u->gemm_shape);
        });
        conv_fwd(u, s, k + 1, u->cat[l], 2 * c, B, l, u->m[l], c, 0);
        conv_fwd(u, s, k + 2, u->m[l], c, B, l, u->d[l], c, 0);
        below = u->d[l];
    }
}

// Backward of conv layer i whose input x (stride xs) at level l produced an
// output with pre-activation gradient gy (BF16 [P][co]).  Accumulates the
// weight and bias gradients; if dx is given writes the input gradient (FP32,
// [P][ci]).
void conv_bwd(mem_unet* u, hipStream_t s, int i, const uint16_t* x, int xs, int B, int l, const uint16_t* gy,
              float* dx)
{
    const ULayer& Y = u->L[i];
    const int S = u->S >> l;
    const int P = (int)P_at(u, B, l);
    if (implicit(Y.ci, xs)) {
        const ConvSrc cs{x, xs, Y.ci, S};
        u->prof.timed(s, "gemm_wgrad", [&] {
            unet_gemm_tn(s, gy, Y.co, nullptr, 0, &cs, P, Y.co, 9 * Y.ci, Y.gbuf, Y.kf, u->n_cu, u->parts);
        });
    } else {
        u->prof.timed(s, "im2col", [&] { unet_im2col3(s, x, xs, 0, B, S, Y.ci, u->col, Y.kf); });
        u->prof.timed(s, "gemm_wgrad", [&] {
            unet_gemm_tn(s, gy, Y.co, u->col, Y.kf, nullptr, P, Y.co, Y.kf, Y.gbuf, Y.kf, u->n_cu, u->parts);
        });
    }
    u->prof.timed(s, "colsum", [&] { unet_colsum(s, gy, Y.co, P, Y.co, bias(u, u->g, i), u->parts); });
    if (!dx) return;
    Epilogue ep{nullptr, 0, nullptr, 0, 0, dx, Y.ci, 0, 0};
    if (implicit(Y.co, Y.co)) {
        const ConvSrc cs{gy, Y.co, Y.co, S};
        u->prof.timed(s, "gemm_dgrad", [&] {
            unet_gemm_nt(s, EPI_F32, nullptr, 0, &cs, Y.wd, Y.kd, P, Y.ci, 9 * Y.co, ep, u->n_cu, u->gemm_shape);
        });
        return;
    }
    u->prof.timed(s, "im2col", [&] { unet_im2col3(s, gy, Y.co, 0, B, S, Y.co, u->col, Y.kd); });
    u->prof.timed(s, "gemm_dgrad", [&] {
        unet_gemm_nt(s, EPI_F32, u->col, Y.kd, nullptr, Y.wd, Y.kd, P, Y.ci, Y.kd, ep, u->n_cu, u->gemm_shape);
    });
}

// Loss gradient of every parameter into u->g (flat), loss into u->loss.
void backward(mem_unet* u, hipStream_t s, int B, const float* target, const float* mask)
{
    const int b = u->base;
    FillList fl;  // every accumulated gradient starts at zero: one launch
    for (int i = 0; i < NLAY; i++) {
        const ULayer& Y = u->L[i];
        if (Y.kind == 0) fl.add(Y.gbuf, (int64_t)Y.co * Y.kf);
        if (Y.kind == 2) fl.add(Y.gbuf, (int64_t)4 * Y.co * Y.ci);
    }
    fl.add(u->g, u->n_params);
    for (int l = 0; l < 4; l++) fl.add(u->de[l], P_at(u, B, l) * (b << l));
    fl.add(u->loss, 2);  // the loss and the count of masked cells (int 0)
    u->prof.timed(s, "fill", [&] { unet_zero_many(s, fl); });
    const int H = NLAY - 1;
    const int64_t P0 = P_at(u, B, 0);
    int* count = (int*)(u->loss + 1);
    u->prof.timed(s, "head", [&] {
        unet_mask_count(s, mask, P0, count);
        unet_head_loss(s, u->d[0], b, P0, u->w + u->L[H].off, bias(u, u->w, H), target, mask, count, u->out,
                       u->loss, u->g + u->L[H].off, bias(u, u->g, H), u->g1, (float2*)u->tmpf, u->parts);
    });
    uint16_t* gd = u->g1;  // gradient of d_l's pre-activation
    uint16_t* gt = u->g2;
    for (int l = 0; l <= 2; l++) {
        const int c = b << l, k = 8 + 3 * (2 - l);
        const int64_t P = P_at(u, B, l);
        // d_l = relu(conv3(m_l))
        conv_bwd(u, s, k + 2, u->m[l], c, B, l, gd, u->tmpf);
        u->prof.timed(s, "eltwise", [&] { unet_relu_mask_add(s, u->tmpf, c, nullptr, 0, u->m[l], c, P, c, gt, c); });
        std::swap(gd, gt);  // gd: gradient of m_l's pre-activation
        // m_l = relu(conv3([u_l, e_l]))
        conv_bwd(u, s, k + 1, u->cat[l], 2 * c, B, l, gd, u->tmpf);
        u->prof.timed(s, "eltwise", [&] { unet_add_f32(s, u->de[l], c, u->tmpf + c, 2 * c, P, c); });  // skip -> e_l
        u->prof.timed(s, "eltwise", [&] {
            unet_relu_mask_add(s, u->tmpf, 2 * c, nullptr, 0, nullptr, 0, P, c, gt, c);  // -> u_l (no ReLU)
        });
        // u_l = convT2(below) + b
        const ULayer& U = u->L[k];
        const int64_t Pb = P_at(u, B, l + 1);
        u->prof.timed(s, "eltwise", [&] { unet_gather_children(s, gt, c, 0, B, u->S >> (l + 1), c, u->gch); });
        const uint16_t* below = (l == 2) ? u->e3 : u->d[l + 1];
        u->prof.timed(s, "gemm_wgrad", [&] {
            unet_gemm_tn(s, u->gch, 4 * c, below, U.ci, nullptr, (int)Pb, 4 * c, U.ci, U.gbuf, U.ci, u->n_cu, u->parts);
        });
        u->prof.timed(s, "colsum", [&] { unet_colsum(s, gt, c, P, c, bias(u, u->g, k), u->parts); });
        Epilogue ep{nullptr, 0, nullptr, 0, 0, u->tmpf, U.ci, 0, 0};
        u->prof.timed(s, "gemm_dgrad", [&] {
            unet_gemm_nt(s, EPI_F32, u->gch, 4 * c, nullptr, U.wd, 4 * c, (int)Pb, U.ci, 4 * c, ep, u->n_cu, u->gemm_shape);
        });
        if (l < 2) {
            u->prof.timed(s, "eltwise", [&] {
                unet_relu_mask_add(s, u->tmpf, U.ci, nullptr, 0, u->d[l + 1], U.ci, Pb, U.ci, gd, U.ci);
            });
        } else {
            u->prof.timed(s, "eltwise", [&] { unet_add_f32(s, u->de[3], U.ci, u->tmpf, U.ci, Pb, U.ci); });
        }
    }
    for (int l = 3; l >= 0; l--) {
        const int c = b << l;
        const int64_t P = P_at(u, B, l);
        u->prof.timed(s, "eltwise", [&] {
            unet_relu_mask_add(s, u->de[l], c, nullptr, 0, e_ptr(u, l), e_stride(u, l), P, c, gd, c);
        });
        conv_bwd(u, s, 2 * l + 1, u->a[l], c, B, l, gd, u->tmpf);
        u->prof.timed(s, "eltwise", [&] { unet_relu_mask_add(s, u->tmpf, c, nullptr, 0, u->a[l], c, P, c, gt, c); });
        const uint16_t* in = (l == 0) ? u->x : u->p[l - 1];
        const int ci = (l == 0) ? 3 : c / 2;
        conv_bwd(u, s, 2 * l, in, ci, B, l, gt, l > 0 ? u->tmpf : nullptr);
        if (l > 0) u->prof.timed(s, "pool", [&] {
            unet_maxpool_bwd(s, u->tmpf, u->arg[l - 1], B, u->S >> (l - 1), ci, u->de[l - 1], ci);
        });
    }
    WJobs js;
    for (int i = 0; i < NLAY; i++) {
        const ULayer& Y = u->L[i];
        if (Y.kind == 4) continue;
        js.add(Y.gbuf, u->g + Y.off, Y.taps, Y.ci, Y.co, Y.kind, Y.kf);
    }
    u->prof.timed(s, "eltwise", [&] { unet_grad_to_flat_many(s, js); });
}

mem_status check_batch(const mem_unet* u, int B)
{
    if (!u) return api_fail(MEM_E_ARG, "network is NULL");
    if (u->broken) return api_fail(MEM_E_STATE, "network is unusable after an earlier HIP error");
    if (B < 1 || B > u->maxB) return api_fail(MEM_E_ARG, "batch must be 1..%d", u->maxB);
    return MEM_OK;
}

mem_status finish(mem_unet* u, const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ufail(u, e, what);
    return MEM_OK;
}

// Counter-based normal numbers for the initial weights (splitmix64 then
// Box-Muller), so a seed gives the same network on every machine.
uint64_t splitmix(uint64_t& s)
{
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

}  // namespace

extern "C" {

int64_t mem_unet_num_params(int32_t base)
{
    if (base < 1 || base > 256) return -1;
    mem_unet u;
    u.base = base;
    build_layout(&u);
    return u.n_params;
}

mem_status mem_unet_create(int32_t base, int32_t max_batch, int32_t size, uint64_t seed, float sigma0,
                           void* stream, mem_unet** out)
{
    if (!out) return api_fail(MEM_E_ARG, "out is NULL");
    *out = nullptr;
    if (!(sigma0 > 0.f) || !std::isfinite(sigma0)) return api_fail(MEM_E_ARG, "sigma0 must be positive");
    if (base < 1 || base > 256 || max_batch < 1 || size < 8 || size % 8 != 0 || size > 4096)
        return api_fail(MEM_E_ARG, "base 1..256, max_batch >= 1, size a multiple of 8 in 8..4096");
    if ((int64_t)max_batch * size * size * 2 * base >= (int64_t)1 << 31)
        return api_fail(MEM_E_ARG, "max_batch x size^2 x 2 base must stay below 2^31");
    mem_unet* u = new mem_unet;
    u->base = base;
    u->S = size;
    u->maxB = max_batch;
    build_layout(u);
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&u->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipGetLastError();
    const int B = max_batch;
    bool ok = ualloc(&u->w, u->n_params) && ualloc(&u->g, u->n_params) && ualloc(&u->am, u->n_params) &&
              ualloc(&u->av, u->n_params) && ualloc(&u->loss, 2);
    size_t col = 0;
    for (int i = 0; i < NLAY && ok; i++) {
        ULayer& Y = u->L[i];
        if (Y.kind == 0) {
            ok = ualloc(&Y.wf, (size_t)Y.co * Y.kf) && ualloc(&Y.wd, (size_t)Y.ci * Y.kd) &&
                 ualloc(&Y.gbuf, (size_t)Y.co * Y.kf);
        } else if (Y.kind == 2) {
            ok = ualloc(&Y.wf, (size_t)4 * Y.co * Y.ci) && ualloc(&Y.wd, (size_t)4 * Y.co * Y.ci) &&
                 ualloc(&Y.gbuf, (size_t)4 * Y.co * Y.ci);
        }
    }
    // im2col scratch: the largest (pixels x K) of any conv at its level
    for (int i = 0; i < NLAY; i++) {
        const ULayer& Y = u->L[i];
        if (Y.kind != 0) continue;
        const int l = (i < 8) ? i / 2 : 2 - (i - 8) / 3;
        const size_t kf = implicit(Y.ci, Y.ci) ? 0 : Y.kf, kd = implicit(Y.co, Y.co) ? 0 : Y.kd;
        col = std::max(col, (size_t)P_at(u, B, l) * std::max(kf, kd));
    }
    const int64_t P0 = P_at(u, B, 0);
    // partial sums of the weight and bias gradients and the loss: the largest
    // of any reduction of a batch of at most B windows (fewer windows split
    // into fewer or equal parts)
    size_t parts = unet_head_parts(P0, base);
    for (int i = 0; i < NLAY; i++) {
        const ULayer& Y = u->L[i];
        if (Y.kind == 0) {
            const int l = (i < 8) ? i / 2 : 2 - (i - 8) / 3;
            const int P = (int)P_at(u, B, l);
            parts = std::max({parts, unet_tn_parts(P, Y.co, 9 * Y.ci, u->n_cu), unet_tn_parts(P, Y.co, Y.kf, u->n_cu),
                              unet_colsum_parts(P, Y.co)});
        } else if (Y.kind == 2) {
            const int l = 2 - (i - 8) / 3;  // output level of the transposed convolution
            parts = std::max({parts, unet_tn_parts((int)P_at(u, B, l + 1), 4 * Y.co, Y.ci, u->n_cu),
                              unet_colsum_parts(P_at(u, B, l), Y.co)});
        }
    }
    ok = ok && ualloc(&u->parts, parts);
    ok = ok && ualloc(&u->x, P0 * 3) && ualloc(&u->out, P0 * 2) && ualloc(&u->col, col) &&
         ualloc(&u->g1, P0 * 2 * base) && ualloc(&u->g2, P0 * 2 * base) && ualloc(&u->gch, P0 * base) &&
         ualloc(&u->tmpf, P0 * 2 * base) && ualloc(&u->e3, P_at(u, B, 3) * 8 * base) && ualloc(&u->xin, P0 * 3);
    for (int l = 0; l < 4 && ok; l++)
        ok = ualloc(&u->a[l], P_at(u, B, l) * (base << l)) && ualloc(&u->de[l], P_at(u, B, l) * (base << l));
    for (int l = 0; l < 3 && ok; l++)
        ok = ualloc(&u->cat[l], P_at(u, B, l) * 2 * (base << l)) && ualloc(&u->p[l], P_at(u, B, l + 1) * (base << l)) &&
             ualloc(&u->m[l], P_at(u, B, l) * (base << l)) && ualloc(&u->d[l], P_at(u, B, l) * (base << l)) &&
             ualloc(&u->arg[l], P_at(u, B, l + 1) * (base << l));
    if (!ok) {
        (void)hipGetLastError();
        free_unet(u);
        return api_fail(MEM_E_NOMEM, "network buffers");
    }
    // He-normal convolution weights (std sqrt(2 / fan_in)), zero biases, a
    // zero head predicting (0, 2 ln sigma0), zero moments
    std::vector<float> w(u->n_params, 0.f);
    uint64_t st = seed;
    for (int i = 0; i < NLAY - 1; i++) {
        const ULayer& Y = u->L[i];
        const int64_t nw = (int64_t)Y.taps * Y.ci * Y.co;
        const double sd = std::sqrt(2.0 / ((double)Y.taps * Y.ci));
        for (int64_t k = 0; k < nw; k++) {
            const double u1 = ((splitmix(st) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
            const double u2 = ((splitmix(st) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
            w[Y.off + k] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
        }
    }
    w[u->n_params - 1] = 2.f * std::log(sigma0);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpy(u->w, w.data(), sizeof(float) * u->n_params, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        u->prof.timed(s, "fill", [&] { unet_fill(s, u->am, u->n_params, 0.f); });
        u->prof.timed(s, "fill", [&] { unet_fill(s, u->av, u->n_params, 0.f); });
        for (int i = 0; i < NLAY; i++) {  // the operands' K padding stays zero from here on
            const ULayer& Y = u->L[i];
            if (Y.kind != 0) continue;
            (void)hipMemsetAsync(Y.wf, 0, sizeof(uint16_t) * (size_t)Y.co * Y.kf, s);
            (void)hipMemsetAsync(Y.wd, 0, sizeof(uint16_t) * (size_t)Y.ci * Y.kd, s);
        }
        relayout_all(u, s);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        free_unet(u);
        return api_fail(MEM_E_HIP, "network init: %s", hipGetErrorString(e));
    }
    *out = u;
    return MEM_OK;
}

mem_status mem_unet_destroy(mem_unet* u, void* stream)
{
    if (!u) return MEM_OK;
    (void)hipStreamSynchronize((hipStream_t)stream);
    free_unet(u);
    return MEM_OK;
}

mem_status mem_unet_set_params(mem_unet* u, const float* params, void* stream)
{
    if (!u || !params) return api_fail(MEM_E_ARG, "NULL argument");
    if (u->broken) return api_fail(MEM_E_STATE, "network is unusable after an earlier HIP error");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(u->w, params, sizeof(float) * u->n_params, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return ufail(u, e, "mem_unet_set_params");
    u->prof.timed(s, "fill", [&] { unet_fill(s, u->am, u->n_params, 0.f); });
    u->prof.timed(s, "fill", [&] { unet_fill(s, u->av, u->n_params, 0.f); });
    u->step = 0;
    relayout_all(u, s);
    return finish(u, "mem_unet_set_params");
}

mem_status mem_unet_get_params(const mem_unet* uc, float* params, void* stream)
{
    mem_unet* u = const_cast<mem_unet*>(uc);
    if (!u || !params) return api_fail(MEM_E_ARG, "NULL argument");
    hipError_t e = hipMemcpyAsync(params, u->w, sizeof(float) * u->n_params, hipMemcpyDeviceToDevice,
                                  (hipStream_t)stream);
    if (e != hipSuccess) return ufail(u, e, "mem_unet_get_params");
    return MEM_OK;
}

mem_status mem_unet_forward(mem_unet* u, const float* x, int32_t batch, float* out, void* stream)
{
    if (mem_status st = check_batch(u, batch)) return st;
    if (!x || !out) return api_fail(MEM_E_ARG, "x and out must not be NULL");
    hipStream_t s = (hipStream_t)stream;
    const int64_t P0 = P_at(u, batch, 0);
    u->prof.timed(s, "eltwise", [&] { unet_cast_bf16(s, x, P0 * 3, u->x); });
    forward(u, s, batch);
    // the head alone (no loss)
    const int H = NLAY - 1;
    u->prof.timed(s, "head", [&] {
        unet_head_loss(s, u->d[0], u->base, P0, u->w + u->L[H].off, bias(u, u->w, H), nullptr, nullptr, nullptr, out,
                       nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    });
    return finish(u, "mem_unet_forward");
}

mem_status mem_unet_loss_grad(mem_unet* u, const float* x, const float* target, const float* mask, int32_t batch,
                              float* grad, float* loss, void* stream)
{
    if (mem_status st = check_batch(u, batch)) return st;
    if (!x || !target || !mask) return api_fail(MEM_E_ARG, "x, target and mask must not be NULL");
    hipStream_t s = (hipStream_t)stream;
    u->prof.timed(s, "eltwise", [&] { unet_cast_bf16(s, x, P_at(u, batch, 0) * 3, u->x); });
    forward(u, s, batch);
    backward(u, s, batch, target, mask);
    if (grad) (void)hipMemcpyAsync(grad, u->g, sizeof(float) * u->n_params, hipMemcpyDeviceToDevice, s);
    if (loss) (void)hipMemcpyAsync(loss, u->loss, sizeof(float), hipMemcpyDeviceToDevice, s);
    return finish(u, "mem_unet_loss_grad");
}

mem_status mem_unet_train_step(mem_unet* u, const float* x, const float* target, const float* mask,
                               int32_t batch, float lr, float* loss, void* stream)
{
    if (!(lr > 0.f) || !std::isfinite(lr)) return api_fail(MEM_E_ARG, "lr must be positive");
    if (mem_status st = mem_unet_loss_grad(u, x, target, mask, batch, nullptr, loss, stream)) return st;
    hipStream_t s = (hipStream_t)stream;
    u->step++;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)u->step), c2 = 1.f - std::pow(b2, (float)u->step);
    u->prof.timed(s, "adam", [&] { unet_adam(s, u->w, u->g, u->am, u->av, u->n_params, lr, b1, b2, 1e-8f, c1, c2); });
    relayout_all(u, s);
    return finish(u, "mem_unet_train_step");
}

mem_status mem_unet_debug_tiles(mem_unet* u, int32_t shape)
{
    if (!u) return api_fail(MEM_E_ARG, "network is NULL");
    if (shape < -1 || shape > 3) return api_fail(MEM_E_ARG, "shape must be -1 (automatic) or 0..3");
    u->gemm_shape = shape;
    return MEM_OK;
}

mem_status mem_unet_profile_enable(mem_unet* u, int32_t on)
{
    if (!u) return api_fail(MEM_E_ARG, "network is NULL");
    u->prof.enable(on != 0);
    return MEM_OK;
}

mem_status mem_unet_profile_read(mem_unet* u, mem_kernel_time* out, int32_t max, int32_t* count)
{
    if (!u) return api_fail(MEM_E_ARG, "network is NULL");
    if (!count || (max > 0 && !out)) return api_fail(MEM_E_ARG, "NULL output");
    *count = u->prof.read(out, max);
    return MEM_OK;
}

mem_status mem_unet_save(const mem_unet* uc, const char* path, void* stream)
{
    mem_unet* u = const_cast<mem_unet*>(uc);
    if (!u || !path) return api_fail(MEM_E_ARG, "NULL argument");
    std::vector<float> w(u->n_params);
    hipError_t e = hipMemcpyAsync(w.data(), u->w, sizeof(float) * u->n_params, hipMemcpyDeviceToHost,
                                  (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return ufail(u, e, "mem_unet_save");
    FILE* f = fopen(path, "wb");
    if (!f) return api_fail(MEM_E_ARG, "cannot open %s for writing", path);
    const int32_t base = u->base;
    const int64_t n = u->n_params;
    bool ok = fwrite("MEMUNET1", 1, 8, f) == 8 && fwrite(&base, 4, 1, f) == 1 && fwrite(&n, 8, 1, f) == 1 &&
              fwrite(w.data(), 4, (size_t)n, f) == (size_t)n;
    ok = (fclose(f) == 0) && ok;
    if (!ok) return api_fail(MEM_E_ARG, "writing %s failed", path);
    return MEM_OK;
}

mem_status mem_unet_load(mem_unet* u, const char* path, void* stream)
{
    if (!u || !path) return api_fail(MEM_E_ARG, "NULL argument");
    if (u->broken) return api_fail(MEM_E_STATE, "network is unusable after an earlier HIP error");
    FILE* f = fopen(path, "rb");
    if (!f) return api_fail(MEM_E_ARG, "cannot open %s", path);
    char magic[8] = {};
    int32_t base = 0;
    int64_t n = 0;
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "MEMUNET1", 8) == 0 && fread(&base, 4, 1, f) == 1 &&
              fread(&n, 8, 1, f) == 1 && base == u->base && n == u->n_params;
    std::vector<float> w(ok ? (size_t)n : 0);
    ok = ok && fread(w.data(), 4, (size_t)n, f) == (size_t)n;
    fclose(f);
    if (!ok) return api_fail(MEM_E_ARG, "%s is not a parameter file of this network (base %d)", path, u->base);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(u->g, w.data(), sizeof(float) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return ufail(u, e, "mem_unet_load");
    return mem_unet_set_params(u, u->g, stream);
}

}  // extern "C"

extern "C" mem_status mem_unet_input(const float* h, const float* v, int32_t width, int32_t height, float z_ref,
                                     float* x, void* stream)
{
    if (!h || !v || !x) return api_fail(MEM_E_ARG, "NULL argument");
    if (width < 1 || height < 1 || (int64_t)width * height > ((int64_t)1 << 28))
        return api_fail(MEM_E_ARG, "bad size %d x %d", width, height);
    if (!std::isfinite(z_ref)) return api_fail(MEM_E_ARG, "z_ref must be finite");
    Grid g{};
    g.W = width;
    g.H = height;
    unet_map_input((hipStream_t)stream, h, v, g, z_ref, x);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return api_fail(MEM_E_HIP, "mem_unet_input: %s", hipGetErrorString(e));
    return MEM_OK;
}

extern "C" mem_status mem_unet_complete(mem_unet* u, const float* x, int32_t batch, float z_ref, float sigma_max,
                                        float* out_h, float* out_sigma, void* stream)
{
    if (mem_status st = check_batch(u, batch)) return st;
    if (!x || !out_h || !out_sigma) return api_fail(MEM_E_ARG, "NULL argument");
    if (!std::isfinite(z_ref) || !(sigma_max > 0.f)) return api_fail(MEM_E_ARG, "bad z_ref or sigma_max");
    if (mem_status st = mem_unet_forward(u, x, batch, u->out, stream)) return st;
    unet_gate((hipStream_t)stream, x, u->out, P_at(u, batch, 0), z_ref, sigma_max, nullptr, nullptr, Grid{}, out_h,
              out_sigma);
    return finish(u, "mem_unet_complete");
}

// mem_complete needs the map's internals (mem_api.hip).
namespace memk {
mem_status map_height_view(const mem_map* m, const float** h, const float** v, Grid* g);
}

extern "C" mem_status mem_complete(const mem_map* map, mem_unet* u, float z_ref, float sigma_max, float* out_h,
                                   float* out_sigma, void* stream)
{
    if (mem_status st = check_batch(u, 1)) return st;
    if (!out_h || !out_sigma) return api_fail(MEM_E_ARG, "outputs must not be NULL");
    if (!std::isfinite(z_ref) || !(sigma_max > 0.f)) return api_fail(MEM_E_ARG, "bad z_ref or sigma_max");
    const float *h = nullptr, *v = nullptr;
    Grid g;
    if (mem_status st = map_height_view(map, &h, &v, &g)) return st;
    if (g.W != u->S || g.H != u->S) return api_fail(MEM_E_ARG, "the network was built for %dx%d maps", u->S, u->S);
    unet_map_input((hipStream_t)stream, h, v, g, z_ref, u->xin);
    if (mem_status st = mem_unet_forward(u, u->xin, 1, u->out, stream)) return st;
    unet_gate((hipStream_t)stream, u->xin, u->out, (int64_t)g.W * g.H, z_ref, sigma_max, h, v, g, out_h, out_sigma);
    return finish(u, "mem_complete");
}
