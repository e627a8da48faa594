/*
 * mem.h - C ABI of the MI355X multi-modal elevation map update.
 *
 * The library implements the per-frame map update of "MEM: Multi-Modal
 * Elevation Mapping for Robotics and Learning" (Erni et al., 2023):
 *   - a robot-centric 2.5D grid (abstract; Sec. II-B) that follows the robot,
 *   - point clouds associated to cells by their horizontal coordinates and
 *     fused into the height/variance layers (Sec. III-B), with the
 *     "height update & ray cast" stage of Table I clearing cells that a
 *     sensor ray passes below,
 *   - the extra point fields and the channels of camera images fused into
 *     task-agnostic layers with one of four rules (Sec. III-C, Eq. (1)-(12)),
 *   - images associated by projecting every cell into the camera with a
 *     Bresenham occlusion test against the map heights (Sec. III-B, Fig. 3).
 *
 * Conventions shared by every entry point
 *   - Every call is asynchronous on the HIP stream passed as `stream`
 *     (a hipStream_t; NULL is the null stream).  Apart from mem_create,
 *     mem_destroy, mem_get_stats and mem_profile_read the library never
 *     synchronises the host with the device.
 *   - Array arguments named "device" are caller-owned device memory (for
 *     example the data_ptr() of a torch tensor).  They are read or written
 *     only by work enqueued on `stream`; the caller keeps them alive until
 *     that work has completed.  The library keeps no pointer after a call
 *     returns.  Arguments named "host" are read during the call only.
 *   - Poses are row-major 3x4 float matrices [R | t] (12 floats, host) that
 *     map a point from the sensor (or camera) frame into the map frame:
 *     p_map = R p_sensor + t.  R must be orthonormal to 1e-4.
 *   - The map frame is the world frame, z up.  The grid is axis-aligned and
 *     only translates (robot-centric map).  Cell (ix, iy) of a W x H grid with
 *     centre cell (cx, cy) covers x in [(cx - W/2 + ix) res, (cx - W/2 + ix + 1) res),
 *     likewise in y; W/2 is integer division.  Layer read-outs are
 *     row-major [H][W][C] with row iy and column ix.
 *   - Errors: every argument is validated on the host before anything is
 *     enqueued, so a call that returns an error leaves the map untouched.
 *     A HIP launch or runtime error returns MEM_E_HIP and is sticky: every
 *     later call on the same map returns MEM_E_STATE.  mem_last_error()
 *     returns a message for the calling thread's last failure.
 *   - A map handle is not thread-safe; distinct handles are independent.
 *
 * Decisions (which cell a point falls in, which cells a ray crosses, the
 * visibility and pixel of a cell) are evaluated in binary32 with a fixed
 * operation order and no fused multiply-add; the exact formulas are written
 * next to each entry point.  Values (heights, variances, layer contents) are
 * binary32 with binary32 accumulation unless a layer's storage says otherwise.
 */
#ifndef MEM_H
#define MEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mem_map mem_map; /* opaque, library-owned */
typedef int32_t mem_status;

enum {
    MEM_OK = 0,
    MEM_E_ARG = -1,         /* invalid argument; nothing was enqueued          */
    MEM_E_NOMEM = -2,       /* device allocation failed                         */
    MEM_E_HIP = -3,         /* a HIP call failed; the map is now unusable       */
    MEM_E_STATE = -4,       /* the map saw an earlier MEM_E_HIP                 */
    MEM_E_UNSUPPORTED = -5  /* a valid request this build does not implement   */
};

/* Fusion rules, Sec. III-C.  `param` of the layer descriptor means:
 *   MEM_LATEST     (Sec. III-C.2, Eq. (1)): unused.
 *   MEM_EXPAVG     (Sec. III-C.3, Eq. (2)): the weight w in (0, 1].
 *   MEM_GAUSS      (Sec. III-C.4, Eq. (6)-(7)): the measurement variance
 *                  sigma_f^2 > 0, one value for every dimension.
 *   MEM_DIRICHLET  (Sec. III-C.5, Eq. (11)-(12)): the initial concentration
 *                  alpha_0 > 0 of every class. */
enum { MEM_LATEST = 0, MEM_EXPAVG = 1, MEM_GAUSS = 2, MEM_DIRICHLET = 3 };

/* Element types.  Layer storage may be MEM_F32, MEM_BF16 or MEM_FP8_E4M3
 * (LATEST, EXPAVG and GAUSS layers); images may be MEM_F32 or MEM_U8
 * (u8 values are divided by 255). */
enum { MEM_F32 = 0, MEM_BF16 = 1, MEM_FP8_E4M3 = 2, MEM_U8 = 3 };

/* Layer ids.  User layers are numbered MEM_LAYER_USER0 + k in the order of
 * mem_params.layers. */
enum {
    MEM_LAYER_ELEVATION = 0, /* h; NaN where the cell holds no height        */
    MEM_LAYER_VARIANCE = 1,  /* v of the height estimate; NaN where invalid   */
    MEM_LAYER_VALID = 2,     /* 1 where the cell holds a height, else 0      */
    MEM_LAYER_HITS = 3,      /* points fused into the cell by the last cloud  */
    MEM_LAYER_CLEAR = 4,     /* clearing votes cast by the last cloud's rays  */
    MEM_LAYER_USER0 = 8
};

/* Views of a layer for mem_get_layer / mem_set_layer. */
enum {
    MEM_VIEW_VALUE = 0,  /* theta (LATEST, EXPAVG; NaN = never observed), mu
                            (GAUSS; NaN = never observed), alpha / sum(alpha)
                            (DIRICHLET, Eq. (11)), or the built-in layer    */
    MEM_VIEW_AUX = 1,    /* sigma^2 (GAUSS, one per cell; +inf = never
                            observed) or alpha (DIRICHLET)                   */
    MEM_VIEW_ARGMAX = 2  /* DIRICHLET: index of the largest alpha, the lowest
                            index on ties (read-only)                        */
};

typedef struct mem_layer_desc {
    int32_t channels;       /* C >= 1 (classes K for DIRICHLET, dimension d for GAUSS) */
    int32_t rule;           /* MEM_LATEST .. MEM_DIRICHLET                      */
    int32_t storage;        /* MEM_F32, MEM_BF16 or MEM_FP8_E4M3                */
    float param;            /* see the rule enum                                */
    const float* ch_scale;  /* host, C floats or NULL: FP8 per-channel amax
                               (code = value / (amax / 448)); NULL means 1.0   */
} mem_layer_desc;

typedef struct mem_params {
    int32_t width, height;   /* W, H cells, 1 .. 16384 each                      */
    float resolution;        /* cell side in metres, > 0                          */
    float noise_c0, noise_c1;/* point noise: sigma = c0 + c1 r^2, v = sigma^2,
                                r the range in the sensor frame                   */
    float max_range;         /* points with r^2 > max_range^2 are dropped         */
    float clear_margin;      /* delta of the clearing test, metres                */
    int32_t clear_min_count; /* votes a cell needs to be cleared; 0 disables rays */
    float min_depth;         /* a cell is in a camera's view only if Z > this     */
    int32_t n_layers;        /* user layers, 0 .. 32                              */
    const mem_layer_desc* layers; /* host, n_layers entries                       */
} mem_params;

/* Binds input channels [ch_first, ch_first + ch_count) of a point cloud or an
 * image to a user layer (Sec. III-C: the user chooses the target layer of
 * every input source).
 *   topk = 0: the ch_count inputs are the layer's channels (ch_count = C).
 *   topk = k in 1..min(K, 64), DIRICHLET layers of K classes only (the top-k
 *     class input of Sec. III-C): the ch_count = 2k inputs are k class
 *     indices followed by their k probabilities.  The measurement fused by
 *     Eq. (12) is the K-vector holding each listed probability at its class
 *     and zero elsewhere (a class listed twice adds both).  A listed index
 *     that is not an integer in [0, K) (or is NaN) contributes nothing.
 *     u8 images carry the index as the byte itself, the probability as
 *     byte / 255.  Batches take top-k image bindings the same way. */
typedef struct mem_binding {
    int32_t layer;    /* MEM_LAYER_USER0 + k */
    int32_t ch_first;
    int32_t ch_count;
    int32_t topk;     /* 0: dense channels; k > 0: top-k class pairs */
} mem_binding;

/* Counters accumulated by the device since the last mem_reset_stats. */
typedef struct mem_stats {
    int64_t points_in;          /* points passed to mem_input_pointcloud        */
    int64_t points_accepted;    /* fused into a cell                             */
    int64_t dropped_nonfinite;  /* a coordinate was NaN or infinite              */
    int64_t dropped_range;      /* r^2 > max_range^2                             */
    int64_t dropped_outside;    /* fell outside the grid                         */
    int64_t cells_touched;      /* (cell, cloud) pairs with at least one point   */
    int64_t cells_cleared;      /* cells invalidated by clearing votes           */
    int64_t ray_cells;          /* cell heights loaded by clearing rays          */
    int64_t cells_in_view;      /* (cell, image) pairs inside the camera frustum */
    int64_t pairs_visible;      /* (cell, image) pairs fused (not occluded)      */
    int64_t occl_cells;         /* cell heights loaded by occlusion rays         */
    int64_t ray_steps;          /* cells between the ends of every clearing ray
                                   (ray_cells is smaller where runs of cells are
                                   ruled out by their block maxima)              */
    int64_t occl_steps;         /* likewise for the occlusion rays               */
    int64_t cell_flushes;       /* (cell, workgroup) sums the point ingest added
                                   into a cloud's per-cell accumulators with
                                   global atomics: 3 each (count, sum of
                                   weights, weighted heights) plus one per
                                   bound channel plane held in LDS; 0 for
                                   batches, whose ingest writes its sums with
                                   plain stores                                 */
    int64_t ray_segments;       /* pieces of at most 64 cells the clearing rays
                                   are cut into, one per lane of the walk (0 for
                                   batches)                                     */
} mem_stats;

/* Creates a map centred on cell (0, 0) with every cell empty: no height,
 * LATEST/EXPAVG/GAUSS layers never observed, DIRICHLET alpha = alpha_0.
 * Allocates the map state on the current HIP device.  `layers` and
 * `ch_scale` are copied.  Synchronises `stream` before returning. */
mem_status mem_create(const mem_params* params, void* stream, mem_map** out);

/* Frees the map after synchronising `stream`.  NULL is a no-op. */
mem_status mem_destroy(mem_map* map, void* stream);

/* Re-centres the robot-centric grid on the robot at (x, y) (abstract: the map
 * follows the robot).  The new centre cell is (floor(x * inv_res),
 * floor(y * inv_res)) in binary32 with inv_res = (float)(1.0 / (double)res);
 * content moves by whole cells and cells that enter the grid are reset to
 * empty.  The device does O(cells entering the grid) work. */
mem_status mem_move(mem_map* map, float x, float y, void* stream);

/* Fuses one point cloud (Sec. III-B, first paragraph; Sec. III-C; Table I
 * rows "point trsf." and "height update & ray cast").
 *   xyz    device, n x 3 float, row-major, sensor frame.
 *   n      number of points, >= 0 (0 is a no-op apart from clearing the
 *          hits/clear layers).
 *   ch     device, n x c float, row-major, or NULL if c == 0.
 *   bind   host, n_bind bindings of point channels to user layers.
 *   T_map_sensor  host, 12 floats.
 * Per point, in binary32 (R = rotation, t = translation of T_map_sensor):
 *   dropped if x, y or z is not finite;
 *   r2 = (x*x + y*y) + z*z, dropped if r2 > max_range * max_range;
 *   p = ((R[k][0]*x + R[k][1]*y) + R[k][2]*z) + t[k];
 *   gx = floor(p.x * inv_res), dropped unless cx - W/2 <= gx < cx - W/2 + W
 *   (same for y); variance v = (c0 + c1 r2)^2.
 * Per cell j with N_j accepted points, information-form Gaussian fusion:
 *   valid prior:  v' = 1 / (1/v + sum 1/v_i),  h' = v' (h/v + sum z_i/v_i);
 *   empty prior:  N_j == 1 -> (h', v') = (z_i, v_i) exactly,
 *                 else     -> v' = 1 / sum 1/v_i, h' = v' sum z_i/v_i.
 * Clearing (if clear_min_count > 0): the ray of every accepted point runs
 * from the sensor's cell to the point's cell along Bresenham's line; each
 * cell strictly between them that held a height before this call receives a
 * vote when h_k > z_ray + clear_margin, z_ray = s_z + (p_z - s_z) t_k and
 * t_k = (centre_k - s) * (1 / (p - s)) along the line's major axis.  A cell
 * with no point in this call and at least clear_min_count votes loses its
 * height.
 * Bound channels: per cell the mean a = (1/N_j) sum m_i (Eq. (1)) is fused by
 * LATEST, EXPAVG (Eq. (2); the first observation sets theta = a) and GAUSS
 * (Eq. (6)-(7) with N = N_j); DIRICHLET adds sum m_i to alpha (Eq. (12)).
 * GAUSS and DIRICHLET layers fed by point clouds must use MEM_F32 storage. */
mem_status mem_input_pointcloud(mem_map* map, const float* xyz, int64_t n,
                                const float* ch, int32_t c,
                                const mem_binding* bind, int32_t n_bind,
                                const float T_map_sensor[12], void* stream);

/* One point cloud of a mem_input_pointclouds call (same meaning as the
 * arguments of mem_input_pointcloud). */
typedef struct mem_cloud {
    const float* xyz;        /* device, n x 3 */
    int64_t n;
    const float* ch;         /* device, n x c, or NULL if c == 0 */
    int32_t c;
    const mem_binding* bind; /* host */
    int32_t n_bind;
    float T_map_sensor[12];
} mem_cloud;

/* Fuses up to 8 point clouds (e.g. the sensors of one robot at one instant,
 * Sec. III-B) with the result of calling mem_input_pointcloud for each in
 * order: every cloud's rays test the heights left by the clouds before it.
 * The association and sums of a cloud do not depend on the heights, so
 * where no cloud binds channels, every cloud's points fit one clearing pass
 * (the clouds of a 100 m range hold up to 262144 points, more for shorter
 * ranges) and neither drift compensation nor overlap clearance is on, the
 * points of all clouds are binned in one launch into per-cloud sums and ray
 * lists, and the clouds' clearing walks and height updates then follow in
 * order; otherwise the clouds run one call each.  The first such call of k
 * clouds allocates k - 1 further sets of sums and ray lists, kept until
 * destroy: each 24 bytes per cell and, per point of the largest cloud,
 * 48 bytes plus 8 bytes per 64-cell segment of a ray at max_range.
 * Height updates add float sums in an order that is not fixed, so results
 * equal the one-call-each results up to rounding (the decisions and counts
 * exactly where no sum is at a threshold).  Every cloud is checked before
 * any work: an invalid call leaves the map untouched. */
mem_status mem_input_pointclouds(mem_map* map, const mem_cloud* clouds, int32_t n_clouds,
                                 void* stream);

/* Fuses one multi-modal image (Sec. III-B, second paragraph; Fig. 3).
 *   img      device, element (row, col, k) at img[row*strides[0] +
 *            col*strides[1] + k*strides[2]] (strides in elements, >= 0).
 *   dtype    MEM_F32 or MEM_U8.
 *   h, w, c  image size and channel count.
 *   K        host, {fx, fy, cx, cy} of a pinhole camera whose pixel centres
 *            sit at integer coordinates.
 *   T_map_cam host, 12 floats; camera axes x right, y down, z forward.
 * For every cell holding a height, in binary32 with (R, t) = T_map_cam:
 *   centre xc = ((float)(cx - W/2 + ix) + 0.5f) * res (same for yc),
 *   d = (xc - t.x, yc - t.y, h - t.z),
 *   X = (R[0][0] d.x + R[1][0] d.y) + R[2][0] d.z, likewise Y, Z (R^T d),
 *   in view iff Z > min_depth and 0 <= floor(u + 0.5) < w, 0 <= floor(v + 0.5) < h,
 *   u = (fx * X) / Z + cx, v = (fy * Y) / Z + cy;
 *   visible iff every cell strictly between the camera's cell and the cell
 *   on Bresenham's line that holds a height is below the ray:
 *   h_k < t.z + (h - t.z) t_k (strict, as in Sec. III-B).
 * A visible cell fuses the pixel's bound channels with its layer's rule and
 * N_j = 1. */
mem_status mem_input_image(mem_map* map, const void* img, int32_t dtype,
                           int32_t h, int32_t w, int32_t c,
                           const int64_t strides[3], const float K[4],
                           const float T_map_cam[12],
                           const mem_binding* bind, int32_t n_bind,
                           void* stream);

/* One image of a mem_input_images call (same meaning as the arguments of
 * mem_input_image). */
typedef struct mem_image {
    const void* data;       /* device */
    int32_t dtype, h, w, c;
    int64_t strides[3];
    float K[4];             /* fx, fy, cx, cy of this image's resolution */
    const mem_binding* bind;/* host */
    int32_t n_bind;
} mem_image;

/* Fuses up to 4 images taken from one camera pose (Sec. III-B), e.g. an RGB
 * image and the feature and class maps computed from it at other
 * resolutions.  The result equals calling mem_input_image for each image in
 * order: fusing an image does not change heights, so the occlusion walk of a
 * cell is shared by all images and evaluated once; each image applies its
 * own frustum test and pixel. */
mem_status mem_input_images(mem_map* map, const mem_image* images, int32_t n_images,
                            const float T_map_cam[12], void* stream);

/* Images of up to 4 camera poses (e.g. the cameras around a robot taken at
 * one instant): n_images[p] images of pose p (1..4), consecutive in
 * `images`, and T_map_cam the n_poses x 12 host array of their poses.  The
 * result equals calling mem_input_images for each pose in order: fusing
 * images does not change heights, so every pose's frustum test, pixel and
 * occlusion walk are evaluated together, and the channels are then fused
 * pose by pose, image by image.  The first call with more than one pose
 * allocates the lists of 4 poses: 128 bytes per cell (an in-view entry of
 * 16 bytes and 4 pixel codes of 4 bytes per pose), kept until destroy.
 * Errors as mem_input_images, checked for every pose before any work. */
mem_status mem_input_image_poses(mem_map* map, const mem_image* images, const int32_t* n_images,
                                 int32_t n_poses, const float* T_map_cam, void* stream);

/* Writes a layer view to `out` (device, H x W x C float, C = 1 for the
 * built-in layers and for MEM_VIEW_ARGMAX).  See the view enum. */
mem_status mem_get_layer(const mem_map* map, int32_t layer, int32_t view,
                         float* out, void* stream);

/* Overwrites a layer view from `in` (device, same layout as mem_get_layer).
 * Settable: ELEVATION/VALUE (NaN = no height), VARIANCE/VALUE, user
 * LATEST/EXPAVG/GAUSS VALUE, GAUSS AUX and DIRICHLET AUX.  Used to restore a
 * saved map and by tests. */
mem_status mem_set_layer(mem_map* map, int32_t layer, int32_t view,
                         const float* in, void* stream);

/* Surface normal of every cell (Table I, "normal calculation"; the paper
 * lists the operation without a formula).  The normal of the height field
 * z = h(x, y) at a cell is (-gx, -gy, 1) / sqrt(gx^2 + gy^2 + 1), with the
 * gradient from central differences of the 4-neighbours' heights:
 *   gx = (h(ix+1, iy) - h(ix-1, iy)) / (2 r),
 *   gy = (h(ix, iy+1) - h(ix, iy-1)) / (2 r),
 * r the map resolution, x along ix and y along iy in the map frame.
 * out: device, H x W x 3 float (nx, ny, nz), logical row-major cell order as
 * mem_get_layer returns it; caller-owned, fully overwritten.  All three
 * components are NaN on the grid's border cells and where the cell or one of
 * its 4-neighbours holds no height.  Computed in binary32.
 * Errors: MEM_E_ARG if out is NULL; MEM_E_STATE / MEM_E_HIP as for every
 * call. */
mem_status mem_normals(const mem_map* map, float* out, void* stream);

/* z-error count and drift compensation of later point clouds (Table I,
 * "point trsf. & z err. cnt" and "drift compensation"; the paper gives no
 * formula).  When enabled, mem_input_pointcloud first tests every accepted
 * point whose cell holds a height h with variance v: its height error
 * e = z - h (z the point's map-frame height) is consistent with the map iff
 *   e * e <= (kappa * kappa) * (v + v_i)   in binary32,
 * v_i = (c0 + c1 r^2)^2 the point's variance.  With at least min_points
 * consistent points, every held height is shifted by
 *   d = binary32( sum e_i / (v + v_i)  /  sum 1 / (v + v_i) )   (sums in binary64),
 * h <- h + d in binary32 (variances unchanged), before the cloud's height
 * update and clearing rays.  Host state only; takes effect from the next
 * call.  Errors: MEM_E_ARG if enabled with kappa not positive and finite or
 * min_points < 1. */
mem_status mem_set_drift_compensation(mem_map* map, int32_t enable, float kappa,
                                      int32_t min_points);

/* PCA layer of a feature layer (the post-processing plugin that turns
 * feature layers into a PCA layer; the paper gives no formula).  Over the
 * cells whose C channels are all observed (finite): the mean m and the
 * population covariance S = (1/N) sum (f - m)(f - m)^T, both accumulated in
 * binary64; e_1..e_3 the eigenvectors of S's three largest eigenvalues in
 * descending order, each signed so that its largest-magnitude entry (the
 * first of equal ones) is positive.  Up to 64 channels the eigenpairs come
 * from Jacobi rotations of the whole matrix in binary64; from 65 to 512
 * channels from orthogonal iteration with Rayleigh-Ritz on a block of eight
 * vectors (binary64), stopped when the three leading pairs' residuals fall
 * below 1e-12 of the largest eigenvalue or after 300 steps: it converges at
 * the rate of the ninth to the third eigenvalue, so nearly equal leading
 * eigenvalues leave the components inexact (they are ill defined there).
 * out: device, H x W x 3 float, logical row-major order as mem_get_layer:
 * ((f - m).e_1, (f - m).e_2, (f - m).e_3) per cell, NaN where a channel is
 * unobserved; caller-owned, fully overwritten.  eigenvalues: host, 3 floats
 * or NULL (then the call does not wait for the stream); 0 for components
 * beyond C or when no cell is observed.  Eigenvectors are defined only up
 * to the span of equal eigenvalues.  The first call allocates scratch for
 * the map: about 17 MB, or 42 MB plus one byte per cell above 64 channels.
 * layer: a LATEST, EXPAVG or GAUSS user layer.
 * Errors: MEM_E_ARG (NULL out, no such layer, a DIRICHLET layer),
 * MEM_E_UNSUPPORTED (more than 512 channels), MEM_E_NOMEM. */
mem_status mem_pca(const mem_map* map, int32_t layer, float* out, float eigenvalues[3],
                   void* stream);

/* mem_pca for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result bit for bit, with the partial sums in a
 * static device array of the library (about 17 MB, held by every GPU the
 * library runs on until the process ends) instead of the map's scratch.
 * Calls no hipMalloc, hipFree or allocating library routine and never waits
 * for the stream.  out: as mem_pca.  eigenvalues: device, 3 floats, written
 * on the stream, or NULL.  Every call on one GPU shares that array: calls
 * that overlap on one GPU (different streams, or different host threads)
 * race and must be serialised by the caller; nothing in the array needs to
 * start cleared (every partial is written before it is read).  The first
 * call on a device looks up the array's address there.  Limit: at most 64
 * channels.  Errors: MEM_E_ARG (NULL out, no such layer, a DIRICHLET
 * layer), MEM_E_UNSUPPORTED (more than 64 channels), MEM_E_HIP (the array's
 * address could not be found, or a launch failed). */
mem_status mem_pca_noalloc(const mem_map* map, int32_t layer, float* out, float* eigenvalues,
                           void* stream);

/* Overlap clearance after every later point cloud (Table I, "overlap
 * clearance", after the multi-modal update; the paper defines it nowhere).
 * When enabled, mem_input_pointcloud ends by removing every held height
 * whose cell centre c (binary32, ((o + i) + 0.5) * res per axis) lies within
 * range_xy of the sensor horizontally and whose height lies more than
 * range_z above or below the sensor:
 *   (c.x - t.x)^2 + (c.y - t.y)^2 <= range_xy^2  and  |h - t.z| > range_z
 * in binary32, t the sensor position of T_map_sensor (an empty cloud
 * included).  Variances and layers are kept, as for the clearing rays.
 * Host state only.  Errors: MEM_E_ARG if enabled with a range that is not
 * finite and >= 0. */
mem_status mem_set_overlap_clearance(mem_map* map, int32_t enable, float range_xy,
                                     float range_z);

/* The last point cloud's applied offset d (0 when none was applied, or the
 * feature is off) and its number of consistent points (0 when off).
 * Host pointers; waits for `stream`. */
mem_status mem_get_drift(const mem_map* map, float* offset, int32_t* consistent,
                         void* stream);

/* Current centre cell of the grid (host values; no device work). */
mem_status mem_get_center(const mem_map* map, int32_t* cx, int32_t* cy);

/* Debug exports, same decisions as the update.
 * mem_debug_point_cells: out (device, n int32) = iy*W + ix of each point's
 *   cell, or -1 non-finite, -2 out of range, -3 outside the grid.
 * mem_debug_cell_pixels: out (device, H*W int32, logical cell order) =
 *   row*w + col of each cell's pixel, -1 no height, -2 outside the view,
 *   -3 occluded. */
mem_status mem_debug_point_cells(const mem_map* map, const float* xyz, int64_t n,
                                 const float T_map_sensor[12], int32_t* out,
                                 void* stream);
mem_status mem_debug_cell_pixels(const mem_map* map, int32_t h, int32_t w,
                                 const float K[4], const float T_map_cam[12],
                                 int32_t* out, void* stream);
/* Tests: channels per lane of this map's image gathers.  1 forces one
 * channel per lane; 0 (the default) lets each gather take 16 bytes of layer
 * storage per lane (4 FP32, 8 BF16 or 16 FP8 E4M3 channels) where the
 * layer's channels, the image's strides and the addresses allow it.  Every
 * element goes through the same arithmetic either way, so both give the
 * same layer bits.  Errors: MEM_E_ARG (other values). */
mem_status mem_debug_gather_width(mem_map* map, int32_t width);

/* Statistics (synchronises `stream`). */
mem_status mem_get_stats(mem_map* map, mem_stats* out, void* stream);
mem_status mem_reset_stats(mem_map* map, void* stream);

/* Per-kernel timing with HIP events recorded on `stream` around every launch
 * while enabled.  mem_profile_read synchronises and returns, per kernel
 * name, the number of launches and the summed milliseconds. */
typedef struct mem_kernel_time {
    char name[32];
    int64_t launches;
    double total_ms;
} mem_kernel_time;
mem_status mem_profile_enable(mem_map* map, int32_t on);
mem_status mem_profile_read(mem_map* map, mem_kernel_time* out, int32_t max,
                            int32_t* count);

/* ---------------------------------------------------------------------- */
/* Batches of independent maps                                             */
/* ---------------------------------------------------------------------- */

/* Many independent robot-centric maps (for example one per simulated robot
 * in a learning task, Sec. I) of different sizes, updated together.  One
 * step of a batch applies, to every map m, exactly the single-map update
 *   mem_move(robot_xy[m]); mem_input_pointcloud(map m's points, no channels);
 *   mem_input_image(map m's image)          (if the batch has cameras)
 * with the same decisions and arithmetic as mem_*; maps share no state.
 * The step is one launch of a captured HIP graph whose stages are persistent
 * work-stealing kernels over (map, chunk) and (map, tile) items of every
 * map at once; chunk, tile and grid sizes come from mem_batch_tune. */
typedef struct mem_batch mem_batch;

typedef struct mem_batch_params {
    int32_t n_maps;           /* 1 .. 65536                                      */
    const int32_t* width;     /* host, n_maps grid widths (1 .. 16384)           */
    const int32_t* height;    /* host, n_maps grid heights                       */
    float resolution, noise_c0, noise_c1, max_range, clear_margin;
    int32_t clear_min_count;
    float min_depth;
    int32_t n_layers;         /* the same user layers in every map               */
    const mem_layer_desc* layers;
    int64_t max_points;       /* most points a step may pass over all maps       */
    int32_t cam_h, cam_w, cam_c; /* every map's image size, or 0 0 0: no cameras */
    int32_t cam_dtype;        /* MEM_F32 or MEM_U8                               */
    int32_t n_img_bind;       /* image channel bindings shared by all maps       */
    const mem_binding* img_bind;
} mem_batch_params;

typedef struct mem_batch_input {
    const float* robot_xy;    /* host, n_maps x 2                                */
    const float* xyz;         /* device, all maps' points, n x 3 (sensor frames) */
    const int64_t* offsets;   /* host, n_maps + 1: map m owns points
                                 [offsets[m], offsets[m + 1]), offsets[0] = 0     */
    const float* T_map_sensor;/* host, n_maps x 12                               */
    const void* images;       /* device, n_maps x cam_h x cam_w x cam_c (HWC), or NULL */
    const float* K;           /* host, n_maps x 4                                */
    const float* T_map_cam;   /* host, n_maps x 12                               */
} mem_batch_input;

/* Sizes the autotuner chooses (read back with mem_batch_get_tuning). */
typedef struct mem_batch_tuning {
    int32_t chunk;            /* points per clearing work item                   */
    int32_t wg_per_cu;        /* persistent workgroups per compute unit          */
    int32_t tile;             /* side of the square cell tiles of projection     */
    int32_t graph;            /* 1: the step runs as a captured HIP graph        */
    double step_ms;           /* measured time of the chosen configuration       */
} mem_batch_tuning;

mem_status mem_batch_create(const mem_batch_params* params, void* stream, mem_batch** out);
mem_status mem_batch_destroy(mem_batch* batch, void* stream);

/* One update of every map.  Host arrays are read during the call; device
 * arrays must stay valid until the step completes on `stream`. */
mem_status mem_batch_step(mem_batch* batch, const mem_batch_input* in, void* stream);

/* Times candidate (chunk, wg_per_cu, tile) settings on `in` (each runs a few
 * steps; the maps are restored afterwards) and keeps the fastest.  The
 * choice never changes integer results. */
mem_status mem_batch_tune(mem_batch* batch, const mem_batch_input* in, void* stream);
mem_status mem_batch_set_tuning(mem_batch* batch, const mem_batch_tuning* t);
mem_status mem_batch_get_tuning(const mem_batch* batch, mem_batch_tuning* out);

/* Per-map views, same meaning and layout as mem_get_layer / mem_set_layer /
 * mem_get_center for map `map`. */
mem_status mem_batch_get_layer(const mem_batch* batch, int32_t map, int32_t layer, int32_t view,
                               float* out, void* stream);
mem_status mem_batch_set_layer(mem_batch* batch, int32_t map, int32_t layer, int32_t view,
                               const float* in, void* stream);
mem_status mem_batch_get_center(const mem_batch* batch, int32_t map, int32_t* cx, int32_t* cy);
mem_status mem_batch_get_stats(mem_batch* batch, mem_stats* out, void* stream);
mem_status mem_batch_reset_stats(mem_batch* batch, void* stream);

/* Per-stage event timing of a batch's steps, as mem_profile_enable /
 * mem_profile_read for a map.  While enabled, mem_batch_step launches its
 * stages directly on `stream` (not as the captured graph) with two events
 * around each; names: b_prep, b_reset, b_bin, b_tile_ingest, b_logical,
 * b_march, b_finalize, b_project, b_gather.  mem_batch_profile_read waits
 * for the recorded events, returns per name the launches and summed
 * milliseconds, and clears the totals. */
mem_status mem_batch_profile_enable(mem_batch* batch, int32_t on);
mem_status mem_batch_profile_read(mem_batch* batch, mem_kernel_time* out, int32_t max, int32_t* count);

/* ---------------------------------------------------------------------- */
/* Learned completion of the height layers                                 */
/* ---------------------------------------------------------------------- */

/* A network that takes map layers and produces a new one (the plugin slot
 * of Sec. III-D): a 4-level U-Net that predicts, for every cell of a
 * size x size window, a height and a log variance from three input channels
 *   x[b][i][j][0] = h - z_ref               (0 where the cell has no height)
 *   x[b][i][j][1] = ln(sqrt(v) / 0.01 m)    (0 where the cell has no height)
 *   x[b][i][j][2] = 1 if the cell has a height, else 0
 * (NHWC FP32, b < batch, row i = logical grid row).  Level l (l = 0..3) works
 * at size / 2^l with base * 2^l channels: two 3x3 convolutions with ReLU,
 * then 2x2 max pooling; the way up is a 2x2 stride-2 transposed convolution,
 * concatenation [up, skip] and two 3x3 convolutions with ReLU; a 1x1 head
 * gives out[b][i][j][0] = predicted h - z_ref, [1] = predicted log sigma^2.
 *
 * Parameters are one flat FP32 array, layer by layer in the order
 *   enc0a enc0b enc1a enc1b enc2a enc2b enc3a enc3b
 *   up2 dec2a dec2b  up1 dec1a dec1b  up0 dec0a dec0b  head
 * each as weights [taps][c_in][c_out] (taps 9 row-major for 3x3, 4 for the
 * transposed 2x2 with tap = 2 dy + dx, 1 for the head) followed by the bias
 * [c_out]; dec*a takes c_in = [up channels, skip channels].  Products run on
 * BF16 operands (activations and a BF16 copy of the weights) with FP32
 * accumulation; the master weights and Adam moments are FP32.
 *
 * Training loss over the N cells with mask > 0, for out = (m, s):
 *   L = (1 / N) sum 0.5 (s + (t - m)^2 exp(-s))
 * the Gaussian negative log-likelihood of the target height t averaged over
 * the cells the target observed (N is counted on the device, 1 / N rounded
 * once from binary64; N = 0 gives L = 0 and a zero gradient). */
typedef struct mem_unet mem_unet;

/* Number of parameters for a base width (1 .. 256), or -1. */
int64_t mem_unet_num_params(int32_t base);

/* Allocates a network for batches of up to max_batch windows of size x size
 * (size a multiple of 8, 8 .. 4096).  Convolution weights are He-normal
 * (standard deviation sqrt(2 / fan_in)) drawn from `seed` (deterministic),
 * their biases zero; the head starts at zero weights with bias
 * (0, 2 ln sigma0), so the untrained network predicts h = z_ref with
 * standard deviation sigma0 > 0 (metres, the height scale of the terrain).
 * MEM_E_ARG on bad sizes, MEM_E_NOMEM. */
mem_status mem_unet_create(int32_t base, int32_t max_batch, int32_t size, uint64_t seed, float sigma0,
                           void* stream, mem_unet** out);
mem_status mem_unet_destroy(mem_unet* net, void* stream);

/* Copies the flat parameters in (device, mem_unet_num_params floats; resets
 * the Adam state) or out. */
mem_status mem_unet_set_params(mem_unet* net, const float* params, void* stream);
mem_status mem_unet_get_params(const mem_unet* net, float* params, void* stream);

/* Per-kernel event timing of the network's launches, as mem_profile_enable /
 * mem_profile_read for a map.  Names: gemm_fwd (3x3 convolutions),
 * gemm_up (transposed convolutions), gemm_dgrad (input gradients),
 * gemm_wgrad (weight gradients), im2col, head, pool, eltwise, colsum, fill,
 * relayout, adam. */
mem_status mem_unet_profile_enable(mem_unet* net, int32_t on);
/* Tests: every product C = A B^T of the network (forward convolutions,
 * transposed convolutions, input gradients) takes workgroup tile `shape`:
 * 0 = 64 x 64, 1 = 128 x 32, 2 = 256 x 32, 3 = 128 x 128 (rows x columns);
 * -1 (the default) chooses by the product's shape.  Every shape sums each
 * output over K in the same order, so the products are equal bit for bit.
 * Errors: MEM_E_ARG. */
mem_status mem_unet_debug_tiles(mem_unet* net, int32_t shape);
mem_status mem_unet_profile_read(mem_unet* net, mem_kernel_time* out, int32_t max, int32_t* count);

/* Writes / reads the parameters as a file: the 8 bytes "MEMUNET1", int32
 * base, int64 count, then count little-endian FP32 values.  Synchronises
 * `stream`.  MEM_E_ARG if the file does not match the network. */
mem_status mem_unet_save(const mem_unet* net, const char* path, void* stream);
mem_status mem_unet_load(mem_unet* net, const char* path, void* stream);

/* out (device, batch x size x size x 2) = network(x) for batch windows x
 * (device, batch x size x size x 3). */
mem_status mem_unet_forward(mem_unet* net, const float* x, int32_t batch, float* out, void* stream);

/* Loss and its gradient with respect to every parameter (flat layout) for
 * targets t and masks (device, batch x size x size each); grad and loss are
 * device pointers and may be NULL.  Nothing is read back to the host. */
mem_status mem_unet_loss_grad(mem_unet* net, const float* x, const float* target, const float* mask,
                              int32_t batch, float* grad, float* loss, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the
 * gradient of mem_unet_loss_grad at learning rate lr; loss (device) may be
 * NULL. */
mem_status mem_unet_train_step(mem_unet* net, const float* x, const float* target, const float* mask,
                               int32_t batch, float lr, float* loss, void* stream);

/* The network input x (device, height x width x 3, NHWC) of one window
 * from its height and variance layers h, v (device, height x width, logical
 * row-major order as mem_get_layer / mem_batch_get_layer return them; NaN
 * height = no height), channels as described above. */
mem_status mem_unet_input(const float* h, const float* v, int32_t width, int32_t height, float z_ref, float* x,
                          void* stream);

/* Gated completion of batch prepared windows x (device, batch x size x
 * size x 3): out_h / out_sigma (device, batch x size x size) follow the rule
 * of mem_complete below, with an observed cell's values rebuilt from its
 * input (x0 + z_ref, 0.01 exp(x1); the height exact for z_ref = 0) and a
 * predicted height reported as (network output + z_ref). */
mem_status mem_unet_complete(mem_unet* net, const float* x, int32_t batch, float z_ref, float sigma_max,
                             float* out_h, float* out_sigma, void* stream);

/* Completion of a map's height layer: runs the network on the whole map
 * (width = height = the network's size, input built from the map's
 * elevation and variance around z_ref) and writes, for every cell in
 * logical row-major order (device, W x H each),
 *   observed cell:                 out_h = h,        out_sigma = sqrt(v)
 *   unobserved, predicted sigma < sigma_max:
 *                                  out_h = network,  out_sigma = predicted
 *   otherwise:                     NaN, NaN.
 * The classical layers are not modified. */
mem_status mem_complete(const mem_map* map, mem_unet* net, float z_ref, float sigma_max, float* out_h,
                        float* out_sigma, void* stream);

/* Message of the calling thread's last failure ("" if none). */
const char* mem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MEM_H */
