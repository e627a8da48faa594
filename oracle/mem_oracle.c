/*
 * mem_oracle.c - plain CPU reference of the multi-modal elevation map update.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline leg of the benchmark, never by the product path.  Written from
 * the paper (Erni et al., "MEM: Multi-Modal Elevation Mapping for Robotics and
 * Learning", 2023) without blocking, fusion or reordering, so that every
 * step can be read against the text:
 *   - Sec. III-B  data association: points by horizontal coordinates, cells
 *                 projected into images with a Bresenham occlusion test;
 *   - Sec. III-C  fusion rules: Latest (Eq. (1)), exponential averaging
 *                 (Eq. (2)), Gaussian Bayesian inference (Eq. (3)-(7)),
 *                 Dirichlet Bayesian inference (Eq. (8)-(12));
 *   - Table I     the "height update & ray cast" stage.  The paper defers the
 *                 height update and the ray cast to its predecessor work, so
 *                 this file takes the reading that the height layer is a
 *                 per-cell Gaussian with known per-point variance updated by
 *                 the same conjugate rule as Eq. (6)-(7) (information form),
 *                 and that a ray clears cells the ray passes below.
 *
 * Build: gcc -O2 -ffp-contract=off (no fast-math).  binary32 decisions rely
 * on C's float arithmetic being IEEE binary32 with no excess precision
 * (SSE on x86-64) and on no multiply-add contraction.
 */
#include "mem_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int C;        /* channels (classes K, dimension d)                     */
    int rule;     /* ORC_LATEST .. ORC_DIRICHLET                           */
    double param; /* w | sigma_f^2 | alpha_0                               */
    double* val;  /* [H*W*C]: theta, mu, or alpha                          */
    double* var;  /* [H*W]: GAUSS posterior variance, +inf = no observation */
} orc_layer;

struct orc_map {
    int W, H;
    float res, inv_res;
    double c0, c1;
    float max_range, clear_margin, min_depth;
    int clear_min_count;
    int cx, cy; /* centre cell of the robot-centric grid */
    double* h;
    double* v;
    unsigned char* valid;
    int32_t* hits;
    int32_t* clear;
    int nL;
    orc_layer* L;
    /* drift compensation (off unless set): consistency bound kappa, the
     * consistent points it needs, and what the last cloud found */
    int drift_on, drift_min_points;
    float drift_kappa;
    double drift_offset;
    int drift_count;
    /* overlap clearance (off unless set): horizontal and vertical ranges */
    int overlap_on;
    float overlap_xy, overlap_z;
};

/* ------------------------------------------------------------------ */
/* Cell initial values                                                  */
/* ------------------------------------------------------------------ */

/* An empty cell: no height, never observed layers, Dirichlet prior
 * alpha_0 (Eq. (10) prior, taken as symmetric). */
static void reset_cell(orc_map* m, long j)
{
    m->valid[j] = 0;
    m->h[j] = NAN;
    m->v[j] = INFINITY;
    m->hits[j] = 0;
    m->clear[j] = 0;
    for (int l = 0; l < m->nL; l++) {
        orc_layer* L = &m->L[l];
        for (int q = 0; q < L->C; q++)
            L->val[j * L->C + q] = (L->rule == ORC_DIRICHLET) ? L->param : NAN;
        if (L->rule == ORC_GAUSS) L->var[j] = INFINITY;
    }
}

orc_map* orc_create(int W, int H, float res, float noise_c0, float noise_c1,
                    float max_range, float clear_margin, int clear_min_count,
                    float min_depth, int n_layers, const int* layer_channels,
                    const int* layer_rule, const float* layer_param)
{
    orc_map* m = (orc_map*)calloc(1, sizeof(orc_map));
    long HW = (long)W * H;
    m->W = W;
    m->H = H;
    m->res = res;
    m->inv_res = (float)(1.0 / (double)res);
    m->c0 = noise_c0;
    m->c1 = noise_c1;
    m->max_range = max_range;
    m->clear_margin = clear_margin;
    m->clear_min_count = clear_min_count;
    m->min_depth = min_depth;
    m->cx = 0;
    m->cy = 0;
    m->h = (double*)malloc(sizeof(double) * HW);
    m->v = (double*)malloc(sizeof(double) * HW);
    m->valid = (unsigned char*)malloc(HW);
    m->hits = (int32_t*)malloc(sizeof(int32_t) * HW);
    m->clear = (int32_t*)malloc(sizeof(int32_t) * HW);
    m->nL = n_layers;
    m->L = (orc_layer*)calloc(n_layers > 0 ? n_layers : 1, sizeof(orc_layer));
    for (int l = 0; l < n_layers; l++) {
        m->L[l].C = layer_channels[l];
        m->L[l].rule = layer_rule[l];
        m->L[l].param = layer_param[l];
        m->L[l].val = (double*)malloc(sizeof(double) * HW * layer_channels[l]);
        m->L[l].var = (layer_rule[l] == ORC_GAUSS) ? (double*)malloc(sizeof(double) * HW) : NULL;
    }
    for (long j = 0; j < HW; j++) reset_cell(m, j);
    return m;
}

void orc_destroy(orc_map* m)
{
    if (!m) return;
    for (int l = 0; l < m->nL; l++) {
        free(m->L[l].val);
        free(m->L[l].var);
    }
    free(m->L);
    free(m->h);
    free(m->v);
    free(m->valid);
    free(m->hits);
    free(m->clear);
    free(m);
}

void orc_get_center(const orc_map* m, int* cx, int* cy)
{
    *cx = m->cx;
    *cy = m->cy;
}

void orc_set_center(orc_map* m, int cx, int cy)
{
    m->cx = cx;
    m->cy = cy;
}

/* ------------------------------------------------------------------ */
/* Robot-centric grid: moving the map with the robot                    */
/* ------------------------------------------------------------------ */

/* The map is robot-centric (abstract; Sec. II-B, last paragraph).  Reading: the grid keeps
 * its orientation and translates by whole cells so that the robot's cell is
 * the centre cell; the content of every cell that stays inside the grid
 * moves with it, cells entering the grid start empty. */
void orc_move(orc_map* m, float x, float y)
{
    float gx = floorf(x * m->inv_res);
    float gy = floorf(y * m->inv_res);
    int ncx = (int)gx, ncy = (int)gy;
    int sx = ncx - m->cx, sy = ncy - m->cy;
    if (sx == 0 && sy == 0) return;
    int W = m->W, H = m->H;
    long HW = (long)W * H;

    /* Copy of the old state, then every new cell (ix, iy) takes old cell
     * (ix + sx, iy + sy) if that existed. */
    orc_map old = *m;
    old.h = (double*)malloc(sizeof(double) * HW);
    old.v = (double*)malloc(sizeof(double) * HW);
    old.valid = (unsigned char*)malloc(HW);
    old.hits = (int32_t*)malloc(sizeof(int32_t) * HW);
    old.clear = (int32_t*)malloc(sizeof(int32_t) * HW);
    memcpy(old.h, m->h, sizeof(double) * HW);
    memcpy(old.v, m->v, sizeof(double) * HW);
    memcpy(old.valid, m->valid, HW);
    memcpy(old.hits, m->hits, sizeof(int32_t) * HW);
    memcpy(old.clear, m->clear, sizeof(int32_t) * HW);
    old.L = (orc_layer*)calloc(m->nL > 0 ? m->nL : 1, sizeof(orc_layer));
    for (int l = 0; l < m->nL; l++) {
        old.L[l] = m->L[l];
        old.L[l].val = (double*)malloc(sizeof(double) * HW * m->L[l].C);
        memcpy(old.L[l].val, m->L[l].val, sizeof(double) * HW * m->L[l].C);
        if (m->L[l].var) {
            old.L[l].var = (double*)malloc(sizeof(double) * HW);
            memcpy(old.L[l].var, m->L[l].var, sizeof(double) * HW);
        }
    }

    for (int iy = 0; iy < H; iy++) {
        for (int ix = 0; ix < W; ix++) {
            long j = (long)iy * W + ix;
            int ox = ix + sx, oy = iy + sy;
            if (ox < 0 || ox >= W || oy < 0 || oy >= H) {
                reset_cell(m, j);
                continue;
            }
            long k = (long)oy * W + ox;
            m->h[j] = old.h[k];
            m->v[j] = old.v[k];
            m->valid[j] = old.valid[k];
            m->hits[j] = old.hits[k];
            m->clear[j] = old.clear[k];
            for (int l = 0; l < m->nL; l++) {
                int C = m->L[l].C;
                for (int q = 0; q < C; q++) m->L[l].val[j * C + q] = old.L[l].val[k * C + q];
                if (m->L[l].var) m->L[l].var[j] = old.L[l].var[k];
            }
        }
    }
    m->cx = ncx;
    m->cy = ncy;

    free(old.h);
    free(old.v);
    free(old.valid);
    free(old.hits);
    free(old.clear);
    for (int l = 0; l < m->nL; l++) {
        free(old.L[l].val);
        free(old.L[l].var);
    }
    free(old.L);
}

/* ------------------------------------------------------------------ */
/* Decisions in binary32                                                */
/* ------------------------------------------------------------------ */

/* Lattice origin: the absolute index of logical cell (0, 0). */
static int origin_x(const orc_map* m) { return m->cx - m->W / 2; }
static int origin_y(const orc_map* m) { return m->cy - m->H / 2; }

/* Point -> map frame and cell (Sec. III-B: points are associated to cells
 * by their horizontal coordinates).  Returns 0 and the cell, or a negative
 * drop reason.  p receives the map-frame point (binary32). */
static int point_cell(const orc_map* m, const float T[12], float x, float y,
                      float z, float p[3], int* ix, int* iy)
{
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) return -1;
    float xx = x * x;
    float yy = y * y;
    float zz = z * z;
    float r2 = xx + yy;
    r2 = r2 + zz;
    float mr2 = m->max_range * m->max_range;
    if (r2 > mr2) return -2;
    for (int k = 0; k < 3; k++) {
        float a = T[4 * k + 0] * x;
        float b = T[4 * k + 1] * y;
        float c = T[4 * k + 2] * z;
        float s = a + b;
        s = s + c;
        p[k] = s + T[4 * k + 3];
    }
    if (!isfinite(p[0]) || !isfinite(p[1]) || !isfinite(p[2])) return -3;
    float gx = floorf(p[0] * m->inv_res);
    float gy = floorf(p[1] * m->inv_res);
    int ox = origin_x(m), oy = origin_y(m);
    if (!(gx >= (float)ox && gx < (float)(ox + m->W))) return -3;
    if (!(gy >= (float)oy && gy < (float)(oy + m->H))) return -3;
    *ix = (int)gx - ox;
    *iy = (int)gy - oy;
    return 0;
}

/* Bresenham's line algorithm (cited in Sec. III-B for the cells between the
 * camera and a cell).  Integer form with the error term D; the minor
 * coordinate steps only when D > 0, so an exact tie stays on the start's
 * side. */
int orc_bresenham(int ax, int ay, int bx, int by, int32_t* xs, int32_t* ys, int cap)
{
    int dx = abs(bx - ax), dy = abs(by - ay);
    int sx = (bx >= ax) ? 1 : -1, sy = (by >= ay) ? 1 : -1;
    int n = 0;
    int x = ax, y = ay;
    if (dx >= dy) {
        int D = 2 * dy - dx;
        for (int i = 0; i <= dx; i++) {
            if (n < cap) {
                xs[n] = x;
                ys[n] = y;
            }
            n++;
            if (D > 0) {
                y += sy;
                D -= 2 * dx;
            }
            D += 2 * dy;
            x += sx;
        }
    } else {
        int D = 2 * dx - dy;
        for (int i = 0; i <= dy; i++) {
            if (n < cap) {
                xs[n] = x;
                ys[n] = y;
            }
            n++;
            if (D > 0) {
                x += sx;
                D -= 2 * dy;
            }
            D += 2 * dx;
            y += sy;
        }
    }
    return n;
}

/* Height of the ray from s = (sx, sy, sz) to p = (px, py, pz) above logical
 * cell (kx, ky): the ray parameter is taken at the cell centre along the
 * line's major axis. */
static float ray_height(const orc_map* m, int xmajor, int kx, int ky,
                        float sx, float sy, float sz, float px, float py, float pz)
{
    float c, s, p;
    if (xmajor) {
        c = (float)(origin_x(m) + kx) + 0.5f;
        s = sx;
        p = px;
    } else {
        c = (float)(origin_y(m) + ky) + 0.5f;
        s = sy;
        p = py;
    }
    c = c * m->res;
    float inv_d = 1.0f / (p - s);
    float t = (c - s) * inv_d;
    float dz = pz - sz;
    return sz + dz * t;
}

/* Logical cell of a position (may lie outside the grid). */
static void lattice_cell(const orc_map* m, float x, float y, int* ix, int* iy)
{
    float gx = floorf(x * m->inv_res);
    float gy = floorf(y * m->inv_res);
    *ix = (int)gx - origin_x(m);
    *iy = (int)gy - origin_y(m);
}

static int in_grid(const orc_map* m, int ix, int iy)
{
    return ix >= 0 && ix < m->W && iy >= 0 && iy < m->H;
}

/* Camera association of cell (ix, iy) (Sec. III-B, Fig. 3): frustum test,
 * pin-hole pixel, then the occlusion test along the Bresenham cells between
 * the camera and the cell.  Returns row*w + col, or -1/-2/-3. */
static int cell_pixel(const orc_map* m, int ix, int iy, int h, int w,
                      const float K[4], const float T[12])
{
    long j = (long)iy * m->W + ix;
    if (!m->valid[j]) return -1;
    float hj = (float)m->h[j];
    float xc = ((float)(origin_x(m) + ix) + 0.5f) * m->res;
    float yc = ((float)(origin_y(m) + iy) + 0.5f) * m->res;
    float d[3] = {xc - T[3], yc - T[7], hj - T[11]};
    float P[3];
    for (int k = 0; k < 3; k++) { /* R^T d: column k of R */
        float a = T[0 + k] * d[0];
        float b = T[4 + k] * d[1];
        float c = T[8 + k] * d[2];
        float s = a + b;
        P[k] = s + c;
    }
    if (!(P[2] > m->min_depth)) return -2;
    float u = K[0] * P[0];
    u = u / P[2];
    u = u + K[2];
    float v = K[1] * P[1];
    v = v / P[2];
    v = v + K[3];
    float uf = floorf(u + 0.5f);
    float vf = floorf(v + 0.5f);
    if (!(uf >= 0.0f && uf < (float)w && vf >= 0.0f && vf < (float)h)) return -2;

    /* Every intermediate cell must be below the ray from the focal point to
     * the cell (strict "smaller than", Sec. III-B). */
    int ax, ay;
    lattice_cell(m, T[3], T[7], &ax, &ay);
    int cap = abs(ix - ax) + abs(iy - ay) + 2;
    int32_t* xs = (int32_t*)malloc(sizeof(int32_t) * cap);
    int32_t* ys = (int32_t*)malloc(sizeof(int32_t) * cap);
    int n = orc_bresenham(ax, ay, ix, iy, xs, ys, cap);
    int xmajor = abs(ix - ax) >= abs(iy - ay);
    int occluded = 0;
    for (int s = 1; s < n - 1 && !occluded; s++) {
        if (!in_grid(m, xs[s], ys[s])) continue;
        long k = (long)ys[s] * m->W + xs[s];
        if (!m->valid[k]) continue;
        float zr = ray_height(m, xmajor, xs[s], ys[s], T[3], T[7], T[11], xc, yc, hj);
        if (!((float)m->h[k] < zr)) occluded = 1;
    }
    free(xs);
    free(ys);
    if (occluded) return -3;
    return (int)vf * w + (int)uf;
}

/* ------------------------------------------------------------------ */
/* Fusion rules (Sec. III-C), binary64                                  */
/* ------------------------------------------------------------------ */

/* Fuses N observations of cell j into layer L: `mean` is their per-channel
 * average (Eq. (1)) and `sum` their per-channel sum. */
static void fuse_cell(orc_layer* L, long j, int N, const double* mean, const double* sum)
{
    double* th = &L->val[j * L->C];
    switch (L->rule) {
    case ORC_LATEST: /* keep only this update's average, Eq. (1) */
        for (int q = 0; q < L->C; q++) th[q] = mean[q];
        break;
    case ORC_EXPAVG: /* Eq. (2); a cell without a past value takes a */
        for (int q = 0; q < L->C; q++) {
            double w = L->param;
            if (isnan(th[q]))
                th[q] = mean[q];
            else
                th[q] = w * mean[q] + (1.0 - w) * th[q];
        }
        break;
    case ORC_GAUSS: { /* Eq. (6)-(7): conjugate Gaussian with known variance */
        double sf2 = L->param;
        double s02 = L->var[j];
        if (isinf(s02)) { /* flat prior: posterior is the ML mean */
            for (int q = 0; q < L->C; q++) th[q] = mean[q];
            L->var[j] = sf2 / N;
        } else {
            double den = N * s02 + sf2;
            for (int q = 0; q < L->C; q++)
                th[q] = (sf2 / den) * th[q] + (N * s02 / den) * mean[q];
            L->var[j] = sf2 * s02 / den;
        }
        break;
    }
    case ORC_DIRICHLET: /* Eq. (12): alpha_t = alpha_{t-1} + sum of m_i */
        for (int q = 0; q < L->C; q++) th[q] += sum[q];
        break;
    }
}

/* A class measurement given as its top k classes (Sec. III-C, the top-k
 * class input): values v[0..k) are class indices and v[k..2k) their
 * probabilities; the measurement is the K-vector that holds each listed
 * probability at its class and zero elsewhere (a repeated class adds).  A
 * listed index that is not an integer in [0, K) contributes nothing. */
static int class_index(double v, int K)
{
    if (!(v >= 0.0) || v >= (double)K || v != floor(v)) return -1; /* NaN fails the first test */
    return (int)v;
}

static void expand_topk(const double* v, int k, int K, double* m)
{
    for (int q = 0; q < K; q++) m[q] = 0.0;
    for (int q = 0; q < k; q++) {
        int c = class_index(v[q], K);
        if (c >= 0) m[c] += v[k + q];
    }
}

/* ------------------------------------------------------------------ */
/* Point clouds                                                         */
/* ------------------------------------------------------------------ */

void orc_point_cells(const orc_map* m, const float* xyz, int64_t n, const float T[12],
                     int32_t* out_cells)
{
    for (int64_t i = 0; i < n; i++) {
        float p[3];
        int ix = 0, iy = 0;
        int r = point_cell(m, T, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], p, &ix, &iy);
        out_cells[i] = (r == 0) ? iy * m->W + ix : r;
    }
}

void orc_input_pointcloud(orc_map* m, const float* xyz, int64_t n, const float* ch,
                          int c, const int* bind, int n_bind, const float T[12],
                          int32_t* out_cells)
{
    int W = m->W, H = m->H;
    long HW = (long)W * H;
    memset(m->hits, 0, sizeof(int32_t) * HW);
    memset(m->clear, 0, sizeof(int32_t) * HW);

    double* Wsum = (double*)calloc(HW, sizeof(double)); /* sum 1/v_i   */
    double* Ssum = (double*)calloc(HW, sizeof(double)); /* sum z_i/v_i */
    double* z1 = (double*)calloc(HW, sizeof(double));   /* the point of a cell with N_j = 1 */
    double* v1 = (double*)calloc(HW, sizeof(double));
    int32_t* cell = (int32_t*)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    float* pm = (float*)malloc(sizeof(float) * 3 * (n > 0 ? n : 1));
    double** chs = (double**)calloc(n_bind > 0 ? n_bind : 1, sizeof(double*));
    int maxc = 1; /* widest binding: its inputs and its layer's channels */
    for (int b = 0; b < n_bind; b++) {
        chs[b] = (double*)calloc(HW * m->L[bind[4 * b] - ORC_LAYER_USER0].C, sizeof(double));
        if (bind[4 * b + 2] > maxc) maxc = bind[4 * b + 2];
        if (m->L[bind[4 * b] - ORC_LAYER_USER0].C > maxc) maxc = m->L[bind[4 * b] - ORC_LAYER_USER0].C;
    }
    double* vin = (double*)malloc(sizeof(double) * maxc); /* one point's bound inputs */
    double* mi = (double*)malloc(sizeof(double) * maxc);  /* its measurement m_i */

    /* Association and per-cell sums. */
    for (int64_t i = 0; i < n; i++) {
        float x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        int ix = 0, iy = 0;
        int r = point_cell(m, T, x, y, z, &pm[3 * i], &ix, &iy);
        if (r != 0) {
            cell[i] = r;
            continue;
        }
        long j = (long)iy * W + ix;
        cell[i] = (int32_t)j;
        /* value side in binary64 */
        double r2 = (double)x * x + (double)y * y + (double)z * z;
        double sigma = m->c0 + m->c1 * r2;
        double var = sigma * sigma;
        double zm = (double)T[8] * x + (double)T[9] * y + (double)T[10] * z + (double)T[11];
        m->hits[j] += 1;
        Wsum[j] += 1.0 / var;
        Ssum[j] += zm / var;
        z1[j] = zm;
        v1[j] = var;
        for (int b = 0; b < n_bind; b++) {
            int f = bind[4 * b + 1], cnt = bind[4 * b + 2], k = bind[4 * b + 3];
            int K = m->L[bind[4 * b] - ORC_LAYER_USER0].C;
            for (int q = 0; q < cnt; q++) vin[q] = (double)ch[i * c + f + q];
            if (k > 0) /* the K-vector of a top-k measurement */
                expand_topk(vin, k, K, mi);
            else
                for (int q = 0; q < K; q++) mi[q] = vin[q];
            for (int q = 0; q < K; q++) chs[b][j * K + q] += mi[q];
        }
    }

    /* z-error count and drift compensation (Table I, rows 1-2; the paper
     * defers their definition).  A point whose cell holds a height is
     * consistent with the map when its height error e = z - h satisfies
     * e^2 <= kappa^2 (v + v_i), both variances those of Eq. (6)-(7)'s
     * Gaussian model, decided in binary32 like every association.  The
     * common offset of the consistent errors, their precision-weighted
     * mean (the maximum-likelihood offset of Gaussian errors), summed in
     * binary64 and rounded to binary32, shifts every held height before the
     * height update and the ray cast when at least drift_min_points points
     * are consistent; the shifted heights are binary32 sums. */
    m->drift_offset = 0.0;
    m->drift_count = 0;
    if (m->drift_on) {
        const float kappa2 = m->drift_kappa * m->drift_kappa;
        double sw = 0.0, swe = 0.0;
        int cnt = 0;
        for (int64_t i = 0; i < n; i++) {
            if (cell[i] < 0 || !m->valid[cell[i]]) continue;
            const long j = cell[i];
            float x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
            float r2 = x * x + y * y; /* the binary32 range of point_cell */
            r2 = r2 + z * z;
            const float sig = (float)m->c0 + (float)m->c1 * r2;
            const float vi = sig * sig;
            const float e = pm[3 * i + 2] - (float)m->h[j];
            const float tot = (float)m->v[j] + vi;
            if (!(e * e <= kappa2 * tot)) continue;
            sw += 1.0 / (double)tot;
            swe += (double)e / (double)tot;
            cnt++;
        }
        m->drift_count = cnt;
        if (cnt >= m->drift_min_points && cnt > 0) {
            const float d = (float)(swe / sw);
            m->drift_offset = d;
            for (long j = 0; j < HW; j++)
                if (m->valid[j]) m->h[j] = (double)((float)m->h[j] + d);
        }
    }

    /* Ray cast against the heights held before this call (after the drift
     * shift when one applies). */
    if (m->clear_min_count > 0) {
        int ax, ay;
        lattice_cell(m, T[3], T[7], &ax, &ay);
        for (int64_t i = 0; i < n; i++) {
            if (cell[i] < 0) continue;
            int bx = cell[i] % W, by = cell[i] / W;
            int cap = abs(bx - ax) + abs(by - ay) + 2;
            int32_t* xs = (int32_t*)malloc(sizeof(int32_t) * cap);
            int32_t* ys = (int32_t*)malloc(sizeof(int32_t) * cap);
            int cnt = orc_bresenham(ax, ay, bx, by, xs, ys, cap);
            int xmajor = abs(bx - ax) >= abs(by - ay);
            for (int s = 1; s < cnt - 1; s++) {
                if (!in_grid(m, xs[s], ys[s])) continue;
                long k = (long)ys[s] * W + xs[s];
                if (!m->valid[k]) continue;
                float zr = ray_height(m, xmajor, xs[s], ys[s], T[3], T[7], T[11],
                                      pm[3 * i], pm[3 * i + 1], pm[3 * i + 2]);
                float thr = zr + m->clear_margin;
                if ((float)m->h[k] > thr) m->clear[k] += 1;
            }
            free(xs);
            free(ys);
        }
    }

    /* Height update: Gaussian posterior with the per-point variances, the
     * information form of the conjugate update of Eq. (6)-(7). */
    for (long j = 0; j < HW; j++) {
        if (m->hits[j] > 0) {
            if (m->valid[j]) {
                double vn = 1.0 / (1.0 / m->v[j] + Wsum[j]);
                double hn = vn * (m->h[j] / m->v[j] + Ssum[j]);
                m->h[j] = hn;
                m->v[j] = vn;
            } else if (m->hits[j] == 1) {
                m->h[j] = z1[j];
                m->v[j] = v1[j];
            } else {
                m->v[j] = 1.0 / Wsum[j];
                m->h[j] = Ssum[j] / Wsum[j];
            }
            m->valid[j] = 1;
        } else if (m->clear_min_count > 0 && m->valid[j] && m->clear[j] >= m->clear_min_count) {
            m->valid[j] = 0;
        }
    }

    /* Extra point fields into their layers (Sec. III-C). */
    for (int b = 0; b < n_bind; b++) {
        orc_layer* L = &m->L[bind[4 * b] - ORC_LAYER_USER0];
        int cnt = L->C;
        double* mean = (double*)malloc(sizeof(double) * cnt);
        for (long j = 0; j < HW; j++) {
            int N = m->hits[j];
            if (N == 0) continue;
            for (int q = 0; q < cnt; q++) mean[q] = chs[b][j * cnt + q] / N;
            fuse_cell(L, j, N, mean, &chs[b][j * cnt]);
        }
        free(mean);
    }

    /* Overlap clearance (Table I, after the height update and the
     * multi-modal update; the paper gives no definition).  A held height
     * within the horizontal range overlap_xy of the sensor that lies more
     * than overlap_z above or below the
     * sensor's height belongs to another level overlapping the robot's
     * surroundings (a floor above, an overhang) and is removed.  Decisions
     * in binary32: the cell centre as in the camera association, squared
     * horizontal distance against overlap_xy^2, |h - z_sensor| against
     * overlap_z. */
    if (m->overlap_on) {
        const float r2max = m->overlap_xy * m->overlap_xy;
        for (int iy = 0; iy < H; iy++)
            for (int ix = 0; ix < W; ix++) {
                const long j = (long)iy * W + ix;
                if (!m->valid[j]) continue;
                const float dx = ((float)(origin_x(m) + ix) + 0.5f) * m->res - T[3];
                const float dy = ((float)(origin_y(m) + iy) + 0.5f) * m->res - T[7];
                const float d2 = dx * dx + dy * dy;
                if (!(d2 <= r2max)) continue;
                if (fabsf((float)m->h[j] - T[11]) > m->overlap_z) m->valid[j] = 0;
            }
    }

    if (out_cells)
        for (int64_t i = 0; i < n; i++) out_cells[i] = cell[i];

    for (int b = 0; b < n_bind; b++) free(chs[b]);
    free(chs);
    free(vin);
    free(mi);
    free(Wsum);
    free(Ssum);
    free(z1);
    free(v1);
    free(cell);
    free(pm);
}

/* ------------------------------------------------------------------ */
/* Images                                                               */
/* ------------------------------------------------------------------ */

void orc_cell_pixels(const orc_map* m, int h, int w, const float K[4], const float T[12],
                     int32_t* out_pix)
{
    for (int iy = 0; iy < m->H; iy++)
        for (int ix = 0; ix < m->W; ix++)
            out_pix[(long)iy * m->W + ix] = cell_pixel(m, ix, iy, h, w, K, T);
}

static double pixel_value(const void* img, int dtype, int64_t off)
{
    if (dtype == ORC_IMG_U8) return ((const unsigned char*)img)[off] / 255.0;
    return (double)((const float*)img)[off];
}

/* A class index read from an image: u8 images carry it as the byte itself. */
static double pixel_index(const void* img, int dtype, int64_t off)
{
    if (dtype == ORC_IMG_U8) return (double)((const unsigned char*)img)[off];
    return (double)((const float*)img)[off];
}

void orc_input_image(orc_map* m, const void* img, int dtype, int h, int w, int c,
                     const int64_t strides[3], const float K[4], const float T[12],
                     const int* bind, int n_bind, int32_t* out_pix)
{
    (void)c;
    long HW = (long)m->W * m->H;
    int32_t* pix = (int32_t*)malloc(sizeof(int32_t) * HW);
    /* Association first, against the heights as they are (images carry no
     * height, Sec. III-B), then fusion of every visible cell with N_j = 1. */
    orc_cell_pixels(m, h, w, K, T, pix);
    for (int b = 0; b < n_bind; b++) {
        orc_layer* L = &m->L[bind[4 * b] - ORC_LAYER_USER0];
        int f = bind[4 * b + 1], cnt = bind[4 * b + 2], k = bind[4 * b + 3];
        double* a = (double*)malloc(sizeof(double) * (cnt > L->C ? cnt : L->C));
        double* v = (double*)malloc(sizeof(double) * (cnt > 0 ? cnt : 1));
        for (long j = 0; j < HW; j++) {
            if (pix[j] < 0) continue;
            int row = pix[j] / w, col = pix[j] % w;
            int64_t base = row * strides[0] + col * strides[1];
            if (k > 0) { /* k indices, then k probabilities */
                for (int q = 0; q < cnt; q++)
                    v[q] = (q < k ? pixel_index : pixel_value)(img, dtype, base + (int64_t)(f + q) * strides[2]);
                expand_topk(v, k, L->C, a);
            } else {
                for (int q = 0; q < cnt; q++) a[q] = pixel_value(img, dtype, base + (int64_t)(f + q) * strides[2]);
            }
            fuse_cell(L, j, 1, a, a);
        }
        free(a);
        free(v);
    }
    if (out_pix) memcpy(out_pix, pix, sizeof(int32_t) * HW);
    free(pix);
}

/* ------------------------------------------------------------------ */
/* Layer views                                                          */
/* ------------------------------------------------------------------ */

int orc_layer_channels(const orc_map* m, int layer)
{
    if (layer >= 0 && layer <= ORC_LAYER_CLEAR) return 1;
    int l = layer - ORC_LAYER_USER0;
    if (l < 0 || l >= m->nL) return -1;
    return m->L[l].C;
}

int orc_get_layer(const orc_map* m, int layer, int view, double* out)
{
    long HW = (long)m->W * m->H;
    if (layer >= 0 && layer <= ORC_LAYER_CLEAR) {
        if (view != ORC_VIEW_VALUE) return -1;
        for (long j = 0; j < HW; j++) {
            switch (layer) {
            case ORC_LAYER_ELEVATION: out[j] = m->valid[j] ? m->h[j] : NAN; break;
            case ORC_LAYER_VARIANCE: out[j] = m->valid[j] ? m->v[j] : NAN; break;
            case ORC_LAYER_VALID: out[j] = m->valid[j] ? 1.0 : 0.0; break;
            case ORC_LAYER_HITS: out[j] = m->hits[j]; break;
            default: out[j] = m->clear[j]; break;
            }
        }
        return 0;
    }
    int l = layer - ORC_LAYER_USER0;
    if (l < 0 || l >= m->nL) return -1;
    const orc_layer* L = &m->L[l];
    int C = L->C;
    if (view == ORC_VIEW_VALUE) {
        for (long j = 0; j < HW; j++) {
            if (L->rule == ORC_DIRICHLET) { /* Eq. (11): theta = alpha / sum alpha */
                double s = 0.0;
                for (int q = 0; q < C; q++) s += L->val[j * C + q];
                for (int q = 0; q < C; q++) out[j * C + q] = L->val[j * C + q] / s;
            } else {
                for (int q = 0; q < C; q++) out[j * C + q] = L->val[j * C + q];
            }
        }
        return 0;
    }
    if (view == ORC_VIEW_AUX) {
        if (L->rule == ORC_GAUSS) {
            for (long j = 0; j < HW; j++) out[j] = L->var[j];
            return 0;
        }
        if (L->rule == ORC_DIRICHLET) {
            for (long j = 0; j < HW * C; j++) out[j] = L->val[j];
            return 0;
        }
        return -1;
    }
    if (view == ORC_VIEW_ARGMAX && L->rule == ORC_DIRICHLET) {
        for (long j = 0; j < HW; j++) {
            int best = 0;
            for (int q = 1; q < C; q++)
                if (L->val[j * C + q] > L->val[j * C + best]) best = q;
            out[j] = best;
        }
        return 0;
    }
    return -1;
}

int orc_set_layer(orc_map* m, int layer, int view, const double* in)
{
    long HW = (long)m->W * m->H;
    if (view != ORC_VIEW_VALUE && view != ORC_VIEW_AUX) return -1;
    if (layer == ORC_LAYER_ELEVATION && view == ORC_VIEW_VALUE) {
        for (long j = 0; j < HW; j++) {
            m->valid[j] = !isnan(in[j]);
            m->h[j] = in[j];
        }
        return 0;
    }
    if (layer == ORC_LAYER_VARIANCE && view == ORC_VIEW_VALUE) {
        for (long j = 0; j < HW; j++)
            if (!isnan(in[j])) m->v[j] = in[j];
        return 0;
    }
    if ((layer == ORC_LAYER_HITS || layer == ORC_LAYER_CLEAR) && view == ORC_VIEW_VALUE) {
        int32_t* dst = (layer == ORC_LAYER_HITS) ? m->hits : m->clear;
        for (long j = 0; j < HW; j++) dst[j] = (int32_t)in[j];
        return 0;
    }
    int l = layer - ORC_LAYER_USER0;
    if (l < 0 || l >= m->nL) return -1;
    orc_layer* L = &m->L[l];
    int C = L->C;
    if (view == ORC_VIEW_VALUE && L->rule != ORC_DIRICHLET) {
        for (long j = 0; j < HW * C; j++) L->val[j] = in[j];
        return 0;
    }
    if (view == ORC_VIEW_AUX && L->rule == ORC_GAUSS) {
        for (long j = 0; j < HW; j++) L->var[j] = in[j];
        return 0;
    }
    if (view == ORC_VIEW_AUX && L->rule == ORC_DIRICHLET) {
        for (long j = 0; j < HW * C; j++) L->val[j] = in[j];
        return 0;
    }
    return -1;
}

/* ------------------------------------------------------------------ */
/* Surface normals (Table I "normal calculation"; reading R21)          */
/* ------------------------------------------------------------------ */

/* Unit normal of every cell from the height layer: with the four
 * edge-adjacent neighbours all holding a height, the slopes are central
 * differences g_x = (h(x+1, y) - h(x-1, y)) / (2 res), likewise g_y, and the
 * normal is (-g_x, -g_y, 1) / sqrt(g_x^2 + g_y^2 + 1); a cell without a
 * height, on the grid's border, or with a neighbour without one gets NaN.
 * out: [H][W][3], logical cell order. */
void orc_normals(const orc_map* m, double* out)
{
    const int W = m->W, H = m->H;
    const double res = (double)m->res;
    for (int iy = 0; iy < H; iy++)
        for (int ix = 0; ix < W; ix++) {
            double* o = out + 3 * ((long)iy * W + ix);
            o[0] = o[1] = o[2] = NAN;
            if (ix < 1 || ix > W - 2 || iy < 1 || iy > H - 2) continue;
            const long j = (long)iy * W + ix;
            if (!m->valid[j] || !m->valid[j - 1] || !m->valid[j + 1] || !m->valid[j - W] || !m->valid[j + W])
                continue;
            const double gx = (m->h[j + 1] - m->h[j - 1]) / (2.0 * res);
            const double gy = (m->h[j + W] - m->h[j - W]) / (2.0 * res);
            const double n = sqrt(gx * gx + gy * gy + 1.0);
            o[0] = -gx / n;
            o[1] = -gy / n;
            o[2] = 1.0 / n;
        }
}

void orc_set_drift(orc_map* m, int on, float kappa, int min_points)
{
    m->drift_on = on;
    m->drift_kappa = kappa;
    m->drift_min_points = min_points;
}

void orc_drift_last(const orc_map* m, double* offset, int* count)
{
    *offset = m->drift_offset;
    *count = m->drift_count;
}

void orc_set_overlap(orc_map* m, int on, float range_xy, float range_z)
{
    m->overlap_on = on;
    m->overlap_xy = range_xy;
    m->overlap_z = range_z;
}
