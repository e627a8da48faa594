/*
 * mem_oracle.h - plain CPU reference of the multi-modal elevation map update.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header or constant with the GPU library: every rule below is written out
 * again here from the paper (Erni et al., "MEM: Multi-Modal Elevation Mapping
 * for Robotics and Learning", 2023).
 *
 * Values (heights, variances, layer contents, sums) are IEEE binary64.
 * Decisions (cell of a point, Bresenham cells, ray heights compared with
 * cell heights, camera frustum and pixel) are evaluated in binary32 with the
 * operation order spelled out in mem_oracle.c, because the decision formula
 * itself is part of the specification the GPU path has to meet bit-exactly.
 */
#ifndef MEM_ORACLE_H
#define MEM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Rule numbering (Sec. III-C): 0 Latest, 1 Exponential averaging,
 * 2 Gaussian Bayesian inference, 3 Dirichlet Bayesian inference. */
#define ORC_LATEST 0
#define ORC_EXPAVG 1
#define ORC_GAUSS 2
#define ORC_DIRICHLET 3

/* Image element types. */
#define ORC_IMG_F32 0
#define ORC_IMG_U8 3

/* Layer ids and views (same meaning as the library's read-out). */
#define ORC_LAYER_ELEVATION 0
#define ORC_LAYER_VARIANCE 1
#define ORC_LAYER_VALID 2
#define ORC_LAYER_HITS 3
#define ORC_LAYER_CLEAR 4
#define ORC_LAYER_USER0 8
#define ORC_VIEW_VALUE 0
#define ORC_VIEW_AUX 1
#define ORC_VIEW_ARGMAX 2

typedef struct orc_map orc_map;

/* layer_rule/layer_channels/layer_param: n_layers entries each. */
orc_map* orc_create(int W, int H, float res, float noise_c0, float noise_c1,
                    float max_range, float clear_margin, int clear_min_count,
                    float min_depth, int n_layers, const int* layer_channels,
                    const int* layer_rule, const float* layer_param);
void orc_destroy(orc_map* m);

void orc_move(orc_map* m, float x, float y);
void orc_get_center(const orc_map* m, int* cx, int* cy);
/* Relabels the grid without moving content (used to load a saved state). */
void orc_set_center(orc_map* m, int cx, int cy);

/* bind: n_bind quadruples (layer, ch_first, ch_count, topk).  topk = 0: the
 * ch_count inputs are the layer's channels.  topk = k > 0 (DIRICHLET layers):
 * the ch_count = 2k inputs are k class indices then their probabilities,
 * fused as the K-vector with each probability at its class (a class that is
 * not an integer in [0, K) is ignored; u8 images carry indices as bytes).  out_cells (n int32 or
 * NULL): logical cell iy*W+ix of each point, or -1/-2/-3 (non-finite, out
 * of range, outside the grid). */
void orc_input_pointcloud(orc_map* m, const float* xyz, int64_t n,
                          const float* ch, int c, const int* bind, int n_bind,
                          const float T[12], int32_t* out_cells);

/* Drift compensation of point clouds (off by default): a point whose cell
 * holds a height is consistent when (z - h)^2 <= kappa^2 (v + v_i) in
 * binary32; with at least min_points consistent points every held height
 * is shifted by their precision-weighted mean error before the height
 * update and the ray cast.  orc_drift_last: the last cloud's offset (0 when
 * none applied) and its number of consistent points. */
void orc_set_drift(orc_map* m, int on, float kappa, int min_points);
void orc_drift_last(const orc_map* m, double* offset, int* count);

/* Overlap clearance after each point cloud's height update (off by
 * default): held heights within range_xy of the sensor horizontally and
 * more than range_z above or below it are removed (binary32 decisions). */
void orc_set_overlap(orc_map* m, int on, float range_xy, float range_z);

/* out_pix (H*W int32 or NULL): pixel row*w+col of each logical cell, or
 * -1 no height, -2 outside the view, -3 occluded. */
void orc_input_image(orc_map* m, const void* img, int dtype, int h, int w,
                     int c, const int64_t strides[3], const float K[4],
                     const float T[12], const int* bind, int n_bind,
                     int32_t* out_pix);

/* Pixel association without fusing anything (same out_pix codes). */
void orc_cell_pixels(const orc_map* m, int h, int w, const float K[4],
                     const float T[12], int32_t* out_pix);

/* Cell association of points without fusing anything. */
void orc_point_cells(const orc_map* m, const float* xyz, int64_t n,
                     const float T[12], int32_t* out_cells);

/* Layer views, row-major [H][W][C] binary64. */
int orc_get_layer(const orc_map* m, int layer, int view, double* out);
/* Unit surface normals from the heights, [H][W][3]; NaN where a height of
 * the cell's 4-neighbourhood is missing or the cell is on the border. */
void orc_normals(const orc_map* m, double* out);
int orc_set_layer(orc_map* m, int layer, int view, const double* in);
int orc_layer_channels(const orc_map* m, int layer);

/* Cells of Bresenham's line from (ax, ay) to (bx, by), endpoints included,
 * in walking order.  Returns the count; writes at most `cap` cells. */
int orc_bresenham(int ax, int ay, int bx, int by, int32_t* xs, int32_t* ys,
                  int cap);

#ifdef __cplusplus
}
#endif
#endif
