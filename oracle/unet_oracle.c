/*
 * unet_oracle.c - plain binary64 reference of the learned completion network.
 *
 * TEST INFRASTRUCTURE ONLY (see mem_oracle.c).  The paper lets plugins run a
 * neural network that takes map layers and produces a new layer (Sec. III-D,
 * Fig. 5); the completion network here is a 4-level U-Net over the height
 * layer:
 *
 *   input  [B][S][S][3]   (height - reference, log variance, observed mask)
 *   enc l  (l = 0..3, width c_l = base 2^l):
 *            e_l = relu(conv3(relu(conv3(in_l))))  in_0 = input,
 *            in_{l+1} = maxpool2(e_l)
 *   dec l  (l = 2..0): u_l = convT2(d_{l+1}) (d_3 = e_3),
 *            d_l = relu(conv3(relu(conv3([u_l, e_l]))))
 *   head   out = conv1(d_0): 2 channels (height, log variance)
 *   loss   mean over target-valid cells of 1/2 (s + (t - h)^2 exp(-s))
 *          (Gaussian negative log-likelihood, s = predicted log variance)
 *
 * conv3 is a 3x3 convolution with zero padding and bias, convT2 a 2x2
 * stride-2 transposed convolution with bias, maxpool2 a 2x2 max (ties: the
 * first of row-major order).  Activations are NHWC.  Parameters are one flat
 * array; each layer stores its weights [taps][Cin][Cout] then its bias
 * [Cout], in the order enc0a enc0b enc1a enc1b enc2a enc2b enc3a enc3b
 * up2 dec2a dec2b up1 dec1a dec1b up0 dec0a dec0b head.
 *
 * Two number formats:
 *   binary64  every value and sum in binary64;
 *   bf16      the network's storage format: the convolution and transposed
 *             convolution weights, the input, every stored activation
 *             (each convolution output after its ReLU, each transposed
 *             convolution output) and every gradient with respect to a
 *             convolution or transposed convolution output (after the ReLU
 *             mask) are rounded to BF16 (round to binary32, then to the
 *             nearest BF16, ties to even); biases and the head are binary32
 *             values; sums stay binary64.  ReLU masks and max-pool winners
 *             are then decided on the stored BF16 values.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NL 18

typedef struct {
    int taps, cin, cout;
    int64_t off;  /* first weight in the flat array; bias follows */
} layer_t;

static void layout(int base, int in_ch, int out_ch, layer_t L[NL])
{
    int c[4] = {base, 2 * base, 4 * base, 8 * base};
    int k = 0;
    int prev = in_ch;
    for (int l = 0; l < 4; l++) {
        L[k++] = (layer_t){9, prev, c[l], 0};
        L[k++] = (layer_t){9, c[l], c[l], 0};
        prev = c[l];
    }
    for (int l = 2; l >= 0; l--) {
        L[k++] = (layer_t){4, c[l + 1], c[l], 0};  /* up */
        L[k++] = (layer_t){9, 2 * c[l], c[l], 0};
        L[k++] = (layer_t){9, c[l], c[l], 0};
    }
    L[k++] = (layer_t){1, base, out_ch, 0};
    int64_t off = 0;
    for (int i = 0; i < NL; i++) {
        L[i].off = off;
        off += (int64_t)L[i].taps * L[i].cin * L[i].cout + L[i].cout;
    }
}

int64_t orc_unet_num_params(int base, int in_ch, int out_ch)
{
    layer_t L[NL];
    layout(base, in_ch, out_ch, L);
    return L[NL - 1].off + (int64_t)L[NL - 1].taps * L[NL - 1].cin * L[NL - 1].cout + L[NL - 1].cout;
}

/* Offsets of each layer's weights (18 entries) for the tests. */
void orc_unet_layer_offsets(int base, int in_ch, int out_ch, int64_t* off)
{
    layer_t L[NL];
    layout(base, in_ch, out_ch, L);
    for (int i = 0; i < NL; i++) off[i] = L[i].off;
}

/* Nearest BF16 (ties to even) of v rounded to binary32 first. */
double orc_round_bf16(double v)
{
    float f = (float)v;
    if (f != f) return v;
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return f;
}

static void round_all(double* a, int64_t n)
{
    for (int64_t i = 0; i < n; i++) a[i] = orc_round_bf16(a[i]);
}

/* channels [0, c) of each of n rows of stride rs */
static void round_rows(double* a, int64_t n, int rs, int c)
{
    for (int64_t j = 0; j < n; j++)
        for (int i = 0; i < c; i++) a[j * rs + i] = orc_round_bf16(a[j * rs + i]);
}

/* ---------------- building blocks ---------------- */

/* y = conv3x3(x) + b, x [B][S][S][ci] with channel stride xs. */
static void conv3(const double* x, int xs, int B, int S, int ci, const double* w, const double* b,
                  int co, double* y)
{
    for (int n = 0; n < B; n++)
        for (int r = 0; r < S; r++)
            for (int q = 0; q < S; q++)
                for (int o = 0; o < co; o++) {
                    double s = b[o];
                    for (int ky = 0; ky < 3; ky++)
                        for (int kx = 0; kx < 3; kx++) {
                            int rr = r + ky - 1, qq = q + kx - 1;
                            if (rr < 0 || rr >= S || qq < 0 || qq >= S) continue;
                            const double* xp = x + (((int64_t)n * S + rr) * S + qq) * xs;
                            const double* wp = w + (int64_t)(ky * 3 + kx) * ci * co + o;
                            for (int i = 0; i < ci; i++) s += xp[i] * wp[(int64_t)i * co];
                        }
                    y[(((int64_t)n * S + r) * S + q) * co + o] = s;
                }
}

/* Backward of conv3: dx (+)= ..., dw += ..., db += ... from dy. */
static void conv3_bwd(const double* x, int xs, int B, int S, int ci, const double* w, int co,
                      const double* dy, double* dx, int dxs, double* dw, double* db)
{
    for (int n = 0; n < B; n++)
        for (int r = 0; r < S; r++)
            for (int q = 0; q < S; q++)
                for (int o = 0; o < co; o++) {
                    double g = dy[(((int64_t)n * S + r) * S + q) * co + o];
                    if (g == 0.0) continue;
                    db[o] += g;
                    for (int ky = 0; ky < 3; ky++)
                        for (int kx = 0; kx < 3; kx++) {
                            int rr = r + ky - 1, qq = q + kx - 1;
                            if (rr < 0 || rr >= S || qq < 0 || qq >= S) continue;
                            const double* xp = x + (((int64_t)n * S + rr) * S + qq) * xs;
                            double* dxp = dx ? dx + (((int64_t)n * S + rr) * S + qq) * dxs : NULL;
                            int64_t wb = (int64_t)(ky * 3 + kx) * ci * co + o;
                            for (int i = 0; i < ci; i++) {
                                dw[wb + (int64_t)i * co] += g * xp[i];
                                if (dxp) dxp[i] += g * w[wb + (int64_t)i * co];
                            }
                        }
                }
}

/* y[n][2r+dy][2q+dx] = b + sum_i x[n][r][q][i] u[dy*2+dx][i][o] */
static void convT2(const double* x, int B, int S, int ci, const double* u, const double* b, int co,
                   double* y, int ys)
{
    int S2 = 2 * S;
    for (int n = 0; n < B; n++)
        for (int r = 0; r < S; r++)
            for (int q = 0; q < S; q++)
                for (int t = 0; t < 4; t++)
                    for (int o = 0; o < co; o++) {
                        double s = b[o];
                        const double* xp = x + (((int64_t)n * S + r) * S + q) * ci;
                        for (int i = 0; i < ci; i++) s += xp[i] * u[((int64_t)t * ci + i) * co + o];
                        int rr = 2 * r + t / 2, qq = 2 * q + t % 2;
                        y[(((int64_t)n * S2 + rr) * S2 + qq) * ys + o] = s;
                    }
}

static void convT2_bwd(const double* x, int B, int S, int ci, const double* u, int co, const double* dy,
                       int dys, double* dx, double* du, double* db)
{
    int S2 = 2 * S;
    for (int n = 0; n < B; n++)
        for (int r = 0; r < S; r++)
            for (int q = 0; q < S; q++)
                for (int t = 0; t < 4; t++)
                    for (int o = 0; o < co; o++) {
                        int rr = 2 * r + t / 2, qq = 2 * q + t % 2;
                        double g = dy[(((int64_t)n * S2 + rr) * S2 + qq) * dys + o];
                        db[o] += g;
                        const double* xp = x + (((int64_t)n * S + r) * S + q) * ci;
                        double* dxp = dx + (((int64_t)n * S + r) * S + q) * ci;
                        for (int i = 0; i < ci; i++) {
                            du[((int64_t)t * ci + i) * co + o] += g * xp[i];
                            dxp[i] += g * u[((int64_t)t * ci + i) * co + o];
                        }
                    }
}

static void maxpool2(const double* x, int xs, int B, int S, int c, double* y, int* arg)
{
    int H = S / 2;
    for (int n = 0; n < B; n++)
        for (int r = 0; r < H; r++)
            for (int q = 0; q < H; q++)
                for (int o = 0; o < c; o++) {
                    int best = 0;
                    double bv = 0;
                    for (int t = 0; t < 4; t++) {
                        double v = x[(((int64_t)n * S + 2 * r + t / 2) * S + 2 * q + t % 2) * xs + o];
                        if (t == 0 || v > bv) {
                            bv = v;
                            best = t;
                        }
                    }
                    int64_t j = (((int64_t)n * H + r) * H + q) * c + o;
                    y[j] = bv;
                    arg[j] = best;
                }
}

static void maxpool2_bwd(const double* dy, const int* arg, int B, int S, int c, double* dx, int dxs)
{
    int H = S / 2;
    for (int n = 0; n < B; n++)
        for (int r = 0; r < H; r++)
            for (int q = 0; q < H; q++)
                for (int o = 0; o < c; o++) {
                    int64_t j = (((int64_t)n * H + r) * H + q) * c + o;
                    int t = arg[j];
                    dx[(((int64_t)n * S + 2 * r + t / 2) * S + 2 * q + t % 2) * dxs + o] += dy[j];
                }
}

static void relu(double* a, int64_t n)
{
    for (int64_t i = 0; i < n; i++)
        if (a[i] < 0) a[i] = 0;
}

/* dy := dy * (y > 0) */
static void relu_bwd(const double* y, double* dy, int64_t n)
{
    for (int64_t i = 0; i < n; i++)
        if (!(y[i] > 0)) dy[i] = 0;
}

/* ---------------- network ---------------- */

typedef struct {
    int B, S, base, in_ch, out_ch, bf16;
    layer_t L[NL];
    double *a[4], *e[4];      /* enc: first conv output, block output (e_l) */
    double *p[3];             /* pooled inputs of levels 1..3 */
    int* arg[3];
    double *cat[3], *m[3], *d[3];  /* dec: [u, e] concat, first conv, block output */
    double* out;
} net_t;

static int64_t sz(const net_t* N, int l, int c) { return (int64_t)N->B * (N->S >> l) * (N->S >> l) * c; }

static void net_alloc(net_t* N, int B, int S, int base, int in_ch, int out_ch, int bf16)
{
    N->bf16 = bf16;
    N->B = B;
    N->S = S;
    N->base = base;
    N->in_ch = in_ch;
    N->out_ch = out_ch;
    layout(base, in_ch, out_ch, N->L);
    for (int l = 0; l < 4; l++) {
        int c = base << l;
        N->a[l] = calloc(sz(N, l, c), sizeof(double));
        N->e[l] = calloc(sz(N, l, c), sizeof(double));
    }
    for (int l = 0; l < 3; l++) {
        int c = base << l;
        N->p[l] = calloc(sz(N, l + 1, c), sizeof(double));
        N->arg[l] = calloc(sz(N, l + 1, c), sizeof(int));
        N->cat[l] = calloc(sz(N, l, 2 * c), sizeof(double));
        N->m[l] = calloc(sz(N, l, c), sizeof(double));
        N->d[l] = calloc(sz(N, l, c), sizeof(double));
    }
    N->out = calloc(sz(N, 0, out_ch), sizeof(double));
}

static void net_free(net_t* N)
{
    for (int l = 0; l < 4; l++) {
        free(N->a[l]);
        free(N->e[l]);
    }
    for (int l = 0; l < 3; l++) {
        free(N->p[l]);
        free(N->arg[l]);
        free(N->cat[l]);
        free(N->m[l]);
        free(N->d[l]);
    }
    free(N->out);
}

#define W(P, i) ((P) + N->L[i].off)
#define BIAS(P, i) ((P) + N->L[i].off + (int64_t)N->L[i].taps * N->L[i].cin * N->L[i].cout)

static void forward(net_t* N, const double* P, const double* x)
{
    int B = N->B, S = N->S;
    const double* in = x;
    int ci = N->in_ch;
    for (int l = 0; l < 4; l++) {
        int c = N->base << l, Sl = S >> l;
        conv3(in, ci, B, Sl, ci, W(P, 2 * l), BIAS(P, 2 * l), c, N->a[l]);
        relu(N->a[l], sz(N, l, c));
        if (N->bf16) round_all(N->a[l], sz(N, l, c));
        conv3(N->a[l], c, B, Sl, c, W(P, 2 * l + 1), BIAS(P, 2 * l + 1), c, N->e[l]);
        relu(N->e[l], sz(N, l, c));
        if (N->bf16) round_all(N->e[l], sz(N, l, c));
        if (l < 3) {
            maxpool2(N->e[l], c, B, Sl, c, N->p[l], N->arg[l]);
            in = N->p[l];
            ci = c;
        }
    }
    const double* below = N->e[3];
    for (int l = 2; l >= 0; l--) {
        int c = N->base << l, Sl = S >> l, k = 8 + 3 * (2 - l);
        /* concat: channels [0, c) = up-sampled, [c, 2c) = skip */
        convT2(below, B, Sl / 2, 2 * c, W(P, k), BIAS(P, k), c, N->cat[l], 2 * c);
        if (N->bf16) round_rows(N->cat[l], (int64_t)B * Sl * Sl, 2 * c, c);
        for (int64_t j = 0; j < (int64_t)B * Sl * Sl; j++)
            memcpy(N->cat[l] + j * 2 * c + c, N->e[l] + j * c, sizeof(double) * c);
        conv3(N->cat[l], 2 * c, B, Sl, 2 * c, W(P, k + 1), BIAS(P, k + 1), c, N->m[l]);
        relu(N->m[l], sz(N, l, c));
        if (N->bf16) round_all(N->m[l], sz(N, l, c));
        conv3(N->m[l], c, B, Sl, c, W(P, k + 2), BIAS(P, k + 2), c, N->d[l]);
        relu(N->d[l], sz(N, l, c));
        if (N->bf16) round_all(N->d[l], sz(N, l, c));
        below = N->d[l];
    }
    /* head: 1x1 */
    const layer_t* H = &N->L[NL - 1];
    for (int64_t j = 0; j < (int64_t)B * S * S; j++)
        for (int o = 0; o < H->cout; o++) {
            double s = BIAS(P, NL - 1)[o];
            for (int i = 0; i < H->cin; i++) s += N->d[0][j * H->cin + i] * W(P, NL - 1)[(int64_t)i * H->cout + o];
            N->out[j * H->cout + o] = s;
        }
}

static void backward(net_t* N, const double* P, const double* x, const double* dout, double* G)
{
    int B = N->B, S = N->S;
    memset(G, 0, sizeof(double) * orc_unet_num_params(N->base, N->in_ch, N->out_ch));
    const layer_t* H = &N->L[NL - 1];
    double* dd = calloc(sz(N, 0, N->base), sizeof(double));
    for (int64_t j = 0; j < (int64_t)B * S * S; j++)
        for (int o = 0; o < H->cout; o++) {
            double g = dout[j * H->cout + o];
            BIAS(G, NL - 1)[o] += g;
            for (int i = 0; i < H->cin; i++) {
                W(G, NL - 1)[(int64_t)i * H->cout + o] += g * N->d[0][j * H->cin + i];
                dd[j * H->cin + i] += g * W(P, NL - 1)[(int64_t)i * H->cout + o];
            }
        }
    double* de[4];
    for (int l = 0; l < 4; l++) de[l] = calloc(sz(N, l, N->base << l), sizeof(double));
    /* decoder, l = 0..2 (reverse of the forward order) */
    for (int l = 0; l <= 2; l++) {
        int c = N->base << l, Sl = S >> l, k = 8 + 3 * (2 - l);
        relu_bwd(N->d[l], dd, sz(N, l, c));
        if (N->bf16) round_all(dd, sz(N, l, c));
        double* dm = calloc(sz(N, l, c), sizeof(double));
        conv3_bwd(N->m[l], c, B, Sl, c, W(P, k + 2), c, dd, dm, c, W(G, k + 2), BIAS(G, k + 2));
        relu_bwd(N->m[l], dm, sz(N, l, c));
        if (N->bf16) round_all(dm, sz(N, l, c));
        double* dcat = calloc(sz(N, l, 2 * c), sizeof(double));
        conv3_bwd(N->cat[l], 2 * c, B, Sl, 2 * c, W(P, k + 1), c, dm, dcat, 2 * c, W(G, k + 1), BIAS(G, k + 1));
        for (int64_t j = 0; j < (int64_t)B * Sl * Sl; j++)
            for (int i = 0; i < c; i++) de[l][j * c + i] += dcat[j * 2 * c + c + i];
        if (N->bf16) round_rows(dcat, (int64_t)B * Sl * Sl, 2 * c, c);
        const double* below = (l == 2) ? N->e[3] : N->d[l + 1];
        double* dbelow = calloc(sz(N, l + 1, 2 * c), sizeof(double));
        convT2_bwd(below, B, Sl / 2, 2 * c, W(P, k), c, dcat, 2 * c, dbelow, W(G, k), BIAS(G, k));
        free(dm);
        free(dcat);
        free(dd);
        if (l == 2) {
            for (int64_t j = 0; j < sz(N, 3, 2 * c); j++) de[3][j] += dbelow[j];
            free(dbelow);
            dd = NULL;
        } else {
            dd = dbelow;
        }
    }
    /* encoder, l = 3..0 */
    for (int l = 3; l >= 0; l--) {
        int c = N->base << l, Sl = S >> l;
        int ci = (l == 0) ? N->in_ch : (c / 2);
        const double* in = (l == 0) ? x : N->p[l - 1];
        relu_bwd(N->e[l], de[l], sz(N, l, c));
        if (N->bf16) round_all(de[l], sz(N, l, c));
        double* da = calloc(sz(N, l, c), sizeof(double));
        conv3_bwd(N->a[l], c, B, Sl, c, W(P, 2 * l + 1), c, de[l], da, c, W(G, 2 * l + 1), BIAS(G, 2 * l + 1));
        relu_bwd(N->a[l], da, sz(N, l, c));
        if (N->bf16) round_all(da, sz(N, l, c));
        double* din = (l == 0) ? NULL : calloc(sz(N, l, ci), sizeof(double));
        conv3_bwd(in, ci, B, Sl, ci, W(P, 2 * l), c, da, din, ci, W(G, 2 * l), BIAS(G, 2 * l));
        if (l > 0) maxpool2_bwd(din, N->arg[l - 1], B, S >> (l - 1), ci, de[l - 1], ci);
        free(da);
        free(din);
    }
    for (int l = 0; l < 4; l++) free(de[l]);
}

/* The parameters and input as the chosen number format stores them:
 * returns the arrays to use (copies in bf16 format, to be freed with
 * release()). */
static const double* fmt_params(const net_t* N, const double* params, int fmt)
{
    if (!fmt) return params;
    int64_t n = orc_unet_num_params(N->base, N->in_ch, N->out_ch);
    double* q = malloc(sizeof(double) * n);
    for (int64_t j = 0; j < n; j++) q[j] = (float)params[j];
    for (int i = 0; i < NL - 1; i++)
        round_all(q + N->L[i].off, (int64_t)N->L[i].taps * N->L[i].cin * N->L[i].cout);
    return q;
}

static const double* fmt_input(const net_t* N, const double* x, int fmt)
{
    if (!fmt) return x;
    int64_t n = sz(N, 0, N->in_ch);
    double* q = malloc(sizeof(double) * n);
    memcpy(q, x, sizeof(double) * n);
    round_all(q, n);
    return q;
}

static void release(const double* copy, const double* orig)
{
    if (copy != orig) free((void*)copy);
}

/* Forward pass: out [B][S][S][out_ch]; fmt 0 = binary64, 1 = bf16. */
void orc_unet_forward(int base, int in_ch, int out_ch, const double* params, const double* x, int B, int S,
                      double* out, int fmt)
{
    net_t N;
    net_alloc(&N, B, S, base, in_ch, out_ch, fmt);
    const double* P = fmt_params(&N, params, fmt);
    const double* X = fmt_input(&N, x, fmt);
    forward(&N, P, X);
    memcpy(out, N.out, sizeof(double) * sz(&N, 0, out_ch));
    release(P, params);
    release(X, x);
    net_free(&N);
}

/* Gaussian negative log-likelihood over cells with mask > 0 (mean) and its
 * gradient with respect to every parameter.  Returns the loss. */
double orc_unet_loss_grad(int base, int in_ch, const double* params, const double* x, const double* target,
                          const double* mask, int B, int S, double* grad, int fmt)
{
    if (B < 1 || S < 1) return 0.0;
    net_t N;
    net_alloc(&N, B, S, base, in_ch, 2, fmt);
    const double* Pm = fmt_params(&N, params, fmt);
    const double* X = fmt_input(&N, x, fmt);
    forward(&N, Pm, X);
    int64_t P = (int64_t)B * S * S;
    double cnt = 0;
    for (int64_t j = 0; j < P; j++) cnt += mask[j] > 0;
    double denom = cnt > 0 ? cnt : 1.0;
    double loss = 0;
    double* dout = calloc((size_t)(2 * P), sizeof(double));
    for (int64_t j = 0; j < P; j++) {
        if (!(mask[j] > 0)) continue;
        double h = N.out[2 * j], s = N.out[2 * j + 1], r = target[j] - h, e = exp(-s);
        loss += 0.5 * (s + r * r * e);
        dout[2 * j] = -r * e / denom;
        dout[2 * j + 1] = 0.5 * (1.0 - r * r * e) / denom;
    }
    if (grad) backward(&N, Pm, X, dout, grad);
    free(dout);
    release(Pm, params);
    release(X, x);
    net_free(&N);
    return loss / denom;
}
