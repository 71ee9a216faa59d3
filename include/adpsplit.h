/*
 * adpsplit.h - C-ABI of the MI355X (gfx950) differentiable Gaussian rasterizer
 * and the AdpSplit error-driven adaptive split (arxiv 2605.06876).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named in the structs and arguments below are DEVICE pointers
 *    (HIP global memory) owned by the caller unless stated otherwise; camera
 *    structs and parameter structs are passed by host pointer and copied.
 *  - Calls are asynchronous on the given stream (a hipStream_t passed as
 *    void*, NULL = the null stream) unless stated otherwise.
 *  - Gaussians are stored struct-of-arrays, FP32, contiguous, n rows:
 *      means [3][n], log_scales [3][n] (s = exp), quats [4][n] (w,x,y,z, not
 *      necessarily unit; normalised inside), opacity_logits [n]
 *      (o = 1/(1+exp(-x))), sh [(d+1)^2][3][n] (real spherical harmonics,
 *      degree d <= 3; the colour is max(0, sum_k Y_k(dir) sh_k + 1/2)).
 *    (Sec. 3 defines mean, rotation, scale, opacity and SH colour.)
 *  - Camera: world->camera rotation R (row-major) and translation t with
 *    x_cam = R x_world + t; camera axes x right, y down, z forward, so the
 *    rows of R are the camera's right, down and forward directions (App. A
 *    uses them for unprojection).  Intrinsics fx, fy, cx, cy in pixels; the
 *    centre of pixel (x, y) is (x + 1/2, y + 1/2).
 *  - Images are planar FP32 [3][H][W]; per-pixel maps are [H][W].
 *  - Errors: every call returns an as_status.  AS_ERR_ARG comes from host-side
 *    checks made before anything is enqueued; AS_ERR_HIP wraps a failing HIP
 *    runtime call (text via as_last_error()).  Device-side capacity overflows
 *    are reported through counters the caller reads after synchronising, as
 *    described per call.  No C++ exception crosses this boundary.
 *  - One as_ctx per stream and thread; contexts are not thread-safe.
 */
#ifndef ADPSPLIT_H
#define ADPSPLIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AS_OK = 0,
    AS_ERR_ARG = 1,       /* invalid argument (null pointer, bad size, bad degree) */
    AS_ERR_CAPACITY = 2,  /* a host-visible capacity is too small */
    AS_ERR_HIP = 3,       /* HIP runtime error */
    AS_ERR_STATE = 4      /* call out of order (e.g. backward without a render) */
} as_status;

typedef struct as_ctx as_ctx;
typedef struct as_frame as_frame;

typedef struct {
    float R[9];          /* world -> camera rotation, row-major */
    float t[3];          /* world -> camera translation */
    float fx, fy, cx, cy;
    int32_t width, height;
    float bg[3];         /* background colour added with the final transmittance */
} as_camera;

typedef struct {
    const float *means, *log_scales, *quats, *opacity_logits, *sh;
    int64_t n;
    int32_t sh_degree;
    const int64_t *n_dev;   /* NULL, or device [1]: the rows in use (<= n; n is then the row stride and the
                               capacity).  Taken by the densification calls (as_clone_prune,
                               as_adaptive_split, as_gather_rows) so that a step's row count never
                               travels to the host; every other call refuses it (AS_ERR_ARG) */
} as_gaussians;

typedef struct {
    float *means, *log_scales, *quats, *opacity_logits, *sh;
    int64_t n;           /* row stride of every array (gradients: n; split output: capacity);
                            0 <= n < 2^30, else the calls return AS_ERR_ARG */
    int32_t sh_degree;
} as_gaussians_mut;

/* Split methods: the full AdpSplit and the steps of its ablation (Table 2:
 * an adaptive number of randomly placed children, then child
 * initialisation from the regions without merging) plus the fixed-cardinality
 * random split it replaces (Eq. (vanilla_split_sample); N = 2 is 3DGS,
 * N = 5 the five-child split of Sec. 1). */
enum {
    AS_VARIANT_ADPSPLIT = 0,     /* region children, merged, capped at n_max; parent copy at o/(N+1) */
    AS_VARIANT_FIXED_N = 1,      /* every candidate: fixed_n random children, parent removed */
    AS_VARIANT_ADAPTIVE_N = 2,   /* N = min(proposals, n_max) random children, parent removed */
    AS_VARIANT_CHILD_INIT = 3    /* one child per proposal (no merging), capped at n_max; parent copy */
};

/* Alternative readings of passages the paper leaves open (bit flags; 0 = the
 * readings the oracle and this library take by default). */
enum {
    AS_SPLIT_ERODE_SIDE = 1,     /* erosion element: square of side r_erode + 1 (offsets -r/2 .. r - r/2), not 2 r_erode + 1 */
    AS_SPLIT_CROSS_VIEW = 2,     /* merge only proposals of different views */
    AS_SPLIT_EXTENT_MAX = 4,     /* rank for the n_max cap by the largest scale, not s1 s2 s3 */
    AS_SPLIT_SHARE_OPACITY = 8   /* children and parent copy all get opacity o/(N+1) */
};

/* AdpSplit hyper-parameters (Sec. 5 "Implementation": tau_l1 0.1, r_erode 2,
 * m_min 5, L 3, N_max 19, gamma_d 2.0, gamma_c 0.15); eps is the t*
 * stabiliser of Eq. (tstar), eta the shrink factor of Eq. (vanilla_split_scale).
 * noise_n is the number of standard-normal triples per candidate in the
 * `noise` input of as_adaptive_split (0 means 2); it must cover the largest
 * random split the variant makes (2; fixed_n; n_max). */
typedef struct {
    double tau_l1;
    int32_t r_erode, m_min, L, n_max;
    double gamma_d, gamma_c, eps, eta;
    int32_t variant;     /* AS_VARIANT_* */
    uint32_t flags;      /* AS_SPLIT_* */
    int32_t fixed_n;     /* children per candidate of AS_VARIANT_FIXED_N */
    int32_t noise_n;
} as_split_params;

/* One retained error region (Sec. 4.1 statistics).  Integer moments are over
 * integer pixel indices; the centroid is in the continuous pixel frame; cov is
 * the pixel covariance plus 1/12 per axis (the unit pixel's own variance); e1
 * has a canonical sign (e1x > 0, or e1x == 0 and e1y > 0). */
typedef struct {
    int32_t cand, view, label, area;   /* dominant candidate id, view id, min linear pixel index, pixels */
    int32_t band, pad0;
    int64_t sx, sy, sxx, sxy, syy;
    double cx, cy;
    double cov[3];                     /* xx, xy, yy */
    double e1[2];
    double sigma1, sigma2;
    float rgb[3];                      /* target colour of the pixel holding the centroid */
    float pad1;
} as_region;                           /* 152 bytes */

typedef struct {
    as_region *records;   /* device, capacity rows */
    int64_t capacity;
    int64_t *count;       /* device counter; the caller zeroes it before the first view.
                             After synchronising, count > capacity means records were dropped. */
} as_region_buf;

/* Device views into a frame's state for one of its views, for inspection by
 * tests and tools.  Per-entry arrays are those of the view's own Gaussians
 * (index = Gaussian id); keys, vals and the range values are global over the
 * views of the last render (the pairs of every view sort together). */
typedef struct {
    int32_t width, height, tile_w, tile_h, tiles_x, tiles_y;
    int64_t n_cap, key_cap;
    int32_t tile_base;        /* global id of the view's first tile */
    uint32_t ent_base;        /* global entry id of the view's Gaussian 0 */
    uint32_t *n_keys;         /* [2] (tile, entry) pairs of the last render, all views: [0] the
                                 number it needed, [1] the number written to keys / vals
                                 (fewer when [0] > key_cap) */
    uint32_t *keys;           /* [key_cap] sorted global bin ids (tile ids when bin_size = 16) */
    uint32_t *vals;           /* [key_cap] entry id of each sorted pair (entry = ent_base of its view + Gaussian id) */
    uint32_t *ranges;         /* [tiles][2] start, end into keys/vals of the view's tiles */
    uint32_t *depth_key;      /* [n] float bits of view-space depth */
    int16_t *box;             /* [n][4] inclusive pixel box x0, y0, x1, y1 (valid if ntiles > 0) */
    uint32_t *ntiles;         /* [n] bins touched (0 = culled) */
    float *rec;               /* [n][12] blend record: mean hi (2), mean lo (2), conic (3), opacity, rgb (3), pad */
    float *t_final;           /* [H][W] final transmittance */
    uint32_t *last;           /* [H][W] index into vals of the last contributor (valid if n_contrib > 0) */
    uint32_t *n_contrib;      /* [H][W] number of contributors */
    int32_t *dom;             /* [H][W] dominant Gaussian id, -1 if none */
    double *err;              /* [H][W] L1 error (written when the render gets a target) */
    uint64_t *err_minmax;     /* [2] bit patterns of the error map's min and max */
    float *grad2d;            /* per-entry 2D gradients of the last backward (a later render of the
                                 frame clears them), entry-major: the nine of
                                 entry e (mean x, y; conic a, b, c; opacity; colour r, g, b) at
                                 grad2d[e * grad2d_stride + k], grad2d_stride = 9 */
    int64_t grad2d_stride;
    int32_t bin_size;         /* pixels per side of the squares the pairs were binned by (16 or 32):
                                 keys hold global bin ids, ntiles counts bins, and each 16 x 16
                                 tile's range is that of the bin holding it */
    int32_t bin_base;         /* global id of the view's first bin */
    int32_t bins_x, bins_y;
} as_frame_view;

/* ---- context and state ------------------------------------------------------ */

/* Create a context bound to HIP device `device`.  Frames keep the device
 * they were created on, so a context and its frames may be destroyed in any
 * order (a frame destroyed after its context reads nothing from it); every
 * other call on a frame needs its context alive.  Creation also loads the
 * library's GPU code on the device (one empty launch per code object, then a
 * device synchronisation), so the first call of each kind allocates nothing
 * either. */
as_status as_ctx_create(int device, as_ctx **out);
void as_ctx_destroy(as_ctx *ctx);
/* Text of the last error raised on this thread (static storage). */
const char *as_last_error(void);
const char *as_version(void);

/* Context scratch for the error statistics, the split and the loop's
 * densification calls.  Those calls never allocate: each checks its sizes
 * against the context's reservation and returns AS_ERR_CAPACITY (naming the
 * field to raise) when they exceed it. */
typedef struct {
    int64_t max_pixels;      /* largest W x H given to as_accumulate_error_stats */
    int64_t max_gaussians;   /* largest Gaussian set given to as_adaptive_split, as_densify_select,
                                as_split_row_map and as_clone_prune */
    int64_t max_candidates;  /* largest candidate capacity given to as_adaptive_split */
    int64_t max_regions;     /* largest region-buffer capacity given to as_adaptive_split */
    int32_t max_views;       /* most views given to as_adaptive_split */
} as_reserve;
/* Grow the context's scratch to cover `r` (each field the maximum of the
 * current and the requested value).  A set-up call: it may allocate, so
 * AS_ERR_STATE inside a graph capture. */
as_status as_ctx_reserve(as_ctx *ctx, const as_reserve *r);
/* The context's current reservation. */
as_status as_ctx_get_reserve(const as_ctx *ctx, as_reserve *r);
/* Device bytes of the scratch a context reserved for `r` holds. */
as_status as_ctx_reserve_bytes(const as_reserve *r, size_t *bytes);

/* Frame flags. */
enum {
    AS_FRAME_FORWARD_ONLY = 1   /* no checkpoint buffer (12 KiB per tile): for frames that are only
                                   rendered (serving, error statistics); a reverse pass on such a
                                   frame walks every tile's list in one piece (same results up to
                                   float rounding) */
};

/* Allocate the per-view state of the rasterizer: n_cap Gaussians, a width x
 * height image, and key_cap (tile, Gaussian) pairs (<= 2^32 - 1).  The frame
 * owns its device memory, all of it allocated here (as_frame_bytes gives the
 * total); as_frame_destroy frees it.  The calls that render into a frame and
 * run its reverse pass never allocate and never synchronise.  A render whose
 * pairs exceed key_cap writes the pairs of the entries (in depth order) that
 * fit whole and renders from those; the frame's *n_keys still reports the full
 * demand, so a caller that reads it after synchronising and finds it above
 * key_cap reserves more with as_frame_reserve_keys and renders again.
 *   flags : 0 or AS_FRAME_FORWARD_ONLY.  AS_ERR_STATE inside a graph capture. */
as_status as_frame_create(as_ctx *ctx, int64_t n_cap, int32_t width, int32_t height, int64_t key_cap,
                          uint32_t flags, as_frame **out);
/* A frame for batched renders of up to max_views (<= 16) views of any sizes:
 * entry_cap bounds the sum over the views of their Gaussian counts,
 * pixel_cap the sum of W x H, tile_cap the sum of 16 x 16 tiles (a W x H view
 * has ceil(W/16) ceil(H/16)); key_cap and flags as above. */
as_status as_frame_create_batch(as_ctx *ctx, int32_t max_views, int64_t entry_cap, int64_t pixel_cap,
                                int64_t tile_cap, int64_t key_cap, uint32_t flags, as_frame **out);
/* Grow a frame's pair capacity to key_cap (no-op if it already holds that
 * many).  A set-up call: it waits for the device, frees and reallocates the
 * pair buffers and forgets the last render (render again before a reverse
 * pass).  AS_ERR_STATE inside a graph capture. */
as_status as_frame_reserve_keys(as_frame *f, int64_t key_cap);
/* Device bytes a frame with these capacities and flags holds (the sum of its
 * allocations as requested from hipMalloc), without creating it.  Capacities
 * as as_frame_create_batch; a frame of as_frame_create has max_views 1,
 * pixel_cap W H and tile_cap ceil(W/16) ceil(H/16). */
as_status as_frame_bytes(int32_t max_views, int64_t entry_cap, int64_t pixel_cap, int64_t tile_cap, int64_t key_cap,
                         uint32_t flags, size_t *bytes);
/* Workspace of a render of n Gaussians in each of n_cams (1..16) cameras
 * (host array): the bytes of the frame sized for exactly those views
 * (entries n x n_cams, their pixels and tiles) with key_cap pairs, i.e.
 * as_frame_bytes of that frame. */
as_status as_workspace_size(const as_ctx *ctx, int64_t n, const as_camera *cams, int32_t n_cams, int64_t key_cap,
                            uint32_t flags, size_t *bytes);
void as_frame_destroy(as_frame *f);
/* Copy the pair count of the last render (all views) to dst ([1], device
 * memory) on `stream`, after the work already queued there; lets a caller
 * that never synchronises the render check it against key_cap later. */
as_status as_frame_pair_count(const as_frame *f, uint32_t *dst, void *stream);
/* View 0 (as_frame_get_view) or view v of the last render. */
as_status as_frame_get_view(const as_frame *f, as_frame_view *out);
as_status as_frame_get_view_of(const as_frame *f, int32_t view, as_frame_view *out);

/* ---- the four calls of the path --------------------------------------------- */

/* Forward render of one view (Eq. (rendering), Sec. 3) plus the dominant
 * Gaussian map D_v (Eq. (dominant-map), Sec. 4.1) and, when `gt` is not NULL,
 * the per-pixel L1 error against gt and its min and max over the view (the
 * inputs of Eq. (l1map)), fused into the same per-tile traversal.
 *   g      : Gaussians (n <= frame n_cap, sh_degree 0..3)
 *   cam    : host pointer; width/height must equal the frame's
 *   gt     : NULL or [3][H][W] target
 *   image  : out [3][H][W]
 * State needed by the backward pass and the error statistics stays in the
 * frame until the next render into it. */
as_status as_render(as_ctx *ctx, const as_gaussians *g, const as_camera *cam, as_frame *frame, const float *gt,
                    float *image, void *stream);

/* Reverse pass of the last as_render into `frame` (the differentiable
 * rasterizer of Sec. 3): recomputes the blend per tile backwards from the
 * stored final transmittance and last-contributor index.  Renders into a
 * frame write per-pixel checkpoints (T, colour behind) at the forward's
 * batch boundaries (up to 3 per tile, in the frame's checkpoint buffer), and
 * this pass splits long tile lists at them into independent segments; a
 * forward-only frame has no checkpoints and this pass walks each tile in one
 * piece (same results up to float rounding).  Allocates nothing.
 *   dL_dimage : [3][H][W]
 *   grads     : out, overwritten; same layout and degree as g, stride g->n
 *   g2d_norm  : NULL or [n]; += |dL/d(mean2d)| (pixel units) for each Gaussian
 *               visible in this view (the ADC statistic of Sec. 3)
 *   vis_count : NULL or [n]; += 1 for each visible Gaussian */
as_status as_render_backward(as_ctx *ctx, const as_gaussians *g, const as_camera *cam, as_frame *frame,
                             const float *dL_dimage, as_gaussians_mut *grads, float *g2d_norm, int32_t *vis_count,
                             void *stream);

/* Batched forward render: n_views (1..max_views) cameras of any sizes, view v
 * rendering the Gaussian set scenes[v] (views may share a set; every set has
 * the same sh_degree), in one pass of each stage: one projection launch over
 * all (view, Gaussian) entries, one depth sort, one key sort over the global
 * tile ids, and one blend launch over every tile of every view.  Each view's
 * outputs are those as_render would give for it alone (the pairs of
 * different views never share a tile).
 *   scenes : host array [n_views]
 *   cams   : host array [n_views]
 *   gt     : NULL, or host array [n_views] of [3][H_v][W_v] targets
 *   images : host array [n_views] of out [3][H_v][W_v]
 * AS_ERR_CAPACITY when the views exceed the frame's entry, pixel or tile
 * capacity; a frame created by as_frame_create takes one view of its size. */
as_status as_render_batch(as_ctx *ctx, const as_gaussians *scenes, const as_camera *cams, int32_t n_views,
                          as_frame *frame, const float *const *gt, float *const *images, void *stream);

/* Reverse pass of the last as_render_batch, whose views all rendered the
 * Gaussian set g: per-view 2D gradients from one blend launch, then the
 * parameter gradients summed over the views in view order.
 *   dL_dimages : host array [n_views] of [3][H_v][W_v]
 *   grads, g2d_norm, vis_count : as as_render_backward (visibility counted per view) */
as_status as_render_backward_batch(as_ctx *ctx, const as_gaussians *g, as_frame *frame, const float *const *dL_dimages,
                                   as_gaussians_mut *grads, float *g2d_norm, int32_t *vis_count, void *stream);

/* Per-pixel L1 error e = sum_c |image_c - gt_c| in FP64 and its min and max
 * over the view (the inputs of Eq. (l1map)), for images not produced by
 * as_render with a target.  err: out [H][W]; err_minmax: out [2]. */
as_status as_error_map(as_ctx *ctx, int32_t width, int32_t height, const float *image, const float *gt, double *err,
                       uint64_t *err_minmax, void *stream);

/* Error region partitioning of one sampled view (Sec. 4.1): normalised error
 * E (Eq. (l1map)), metric map M = [E > tau_l1], attribution count
 * attr_count[D(u)] += 1 for high-error pixels dominated by a candidate
 * (counted before erosion), erosion with a (2 r_erode + 1)^2 square (pixels
 * outside the image count as set), L uniform bands over (tau_l1, 1], regions
 * as 8-connected components with equal (D, B) (Eq. (error-region)), area
 * filter (Eq. (min_region_area)) and region statistics.  Regions are appended
 * to `regions` in ascending label order.
 *   err, err_minmax : from as_render (frame view) or as_error_map
 *   dom             : [H][W] dominant map (-1 = none)
 *   gt              : [3][H][W] target (colour at the centroid)
 *   is_candidate    : [n] 0/1 split-candidate mask
 *   attr_count      : [n] accumulated
 * Uses the context's reserved scratch and allocates nothing: AS_ERR_CAPACITY
 * when width x height exceeds the reservation's max_pixels. */
as_status as_accumulate_error_stats(as_ctx *ctx, int32_t width, int32_t height, const double *err,
                                    const uint64_t *err_minmax, const int32_t *dom, const float *gt, int32_t view_id,
                                    int64_t n, const uint8_t *is_candidate, const as_split_params *params,
                                    as_region_buf *regions, int32_t *attr_count, void *stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): as_accumulate_error_stats
 * with the same arguments, kernels and results, but its scratch in one static
 * device array of the library (54 MiB plus 32 KiB, sized for views of up to
 * AS_NOALLOC_MAX_PIXELS pixels) instead of the context's reservation, which it
 * does not need.  Each device the library runs on holds its own copy of that
 * array until the process ends; its address is taken when a context is
 * created on the device.  All calls on one device share the array, so calls
 * that overlap on a device race and must not be issued (one stream, or
 * ordered streams).  AS_ERR_CAPACITY when width x height exceeds
 * AS_NOALLOC_MAX_PIXELS; other errors as as_accumulate_error_stats. */
#define AS_NOALLOC_MAX_PIXELS (1 << 20)
as_status as_accumulate_error_stats_noalloc(as_ctx *ctx, int32_t width, int32_t height, const double *err,
                                            const uint64_t *err_minmax, const int32_t *dom, const float *gt,
                                            int32_t view_id, int64_t n, const uint8_t *is_candidate,
                                            const as_split_params *params, as_region_buf *regions,
                                            int32_t *attr_count, void *stream);

/* The adaptive split of every candidate (Sec. 4.2, 4.3, App. A and Sec. 5
 * "Implementation"): one child proposal per region (centre on the centroid ray
 * at t* of Eq. (tstar); shape from the unprojected, clipped PCA axes; colour
 * from the target), transitive merging under Eq. (merge_conditions) with the
 * merged parameters of Eq. (merge_cov), a cap of N_max children by covariance
 * extent, and the mode: VANILLA (0, no attributed pixel: the fixed N = 2 split
 * of Eq. (vanilla_split_sample)), RESET (1, attributed pixels but no
 * surviving region: no rows, parent kept), ADAPTIVE (2: N_i children plus a
 * parent copy with opacity o / (N_i + 1)); other variants (params->variant)
 * use mode RANDOM (3: count random children of Eq. (vanilla_split_sample)
 * with N = count, parent removed).
 *   cand       : [n_cand] candidate ids, strictly ascending
 *   regions    : the regions of all sampled views (any order)
 *   views      : host array [n_views]; a region's view id indexes it
 *   attr_count : [n]
 *   noise      : [n_cand][noise_n][3] standard normals for the random children
 *   out        : rows = capacity >= n + n_cand * per, per = fixed_n for AS_VARIANT_FIXED_N, else
 *                max(2, n_max + 1) (AS_ERR_CAPACITY below it)
 *   mode, count: out [n_cand]; offset: out [n_cand] exclusive scan of count
 *   n_out      : out [1] device; the new set is the non-removed Gaussians in
 *                order, then one block per candidate in ascending id order
 *                (children by descending extent, then the parent copy).
 *   n_cand_dev : NULL, or device [1]: the candidates in use (<= n_cand, which is
 *                then the capacity of cand, mode, count and offset; entries past
 *                it get mode 0 and count 0).  With g->n_dev as well, nothing of the
 *                call depends on a count the host has not set, so it can follow
 *                as_densify_select and as_clone_prune inside one graph capture.
 * Returns AS_ERR_CAPACITY when out->n is below the bound above, or when the
 * region capacity, n_cand, n_views or g->n exceed the context's reservation
 * (max_regions, max_candidates, max_views, max_gaussians); allocates nothing. */
as_status as_adaptive_split(as_ctx *ctx, const as_gaussians *g, const int32_t *cand, int64_t n_cand,
                            const as_region_buf *regions, const as_camera *views, int32_t n_views,
                            const int32_t *attr_count, const as_split_params *params, const float *noise,
                            as_gaussians_mut *out, uint8_t *mode, int32_t *count, int64_t *offset, int64_t *n_out,
                            const int64_t *n_cand_dev, void *stream);

/* ---- the optimisation loop around the path -------------------------------------- */
/* The split runs inside 3DGS's training loop (Sec. 3: adaptive density
 * control clones small and splits large Gaussians with a high view-averaged
 * screen-space gradient and prunes transparent ones; Sec. 5 "Implementation":
 * AdpSplit replaces the split and keeps the rest).  These entry points are the
 * loop's per-iteration steps (loss, Adam) and its densification bookkeeping
 * (selection, row maps, clone + prune, optimiser-state carry-over).  None of
 * them allocates; as_densify_select, as_split_row_map and as_clone_prune use
 * the context's scratch reserved for max_gaussians rows (AS_ERR_CAPACITY
 * beyond it). */

/* Adam hyper-parameters with the per-group learning rates of 3DGS. */
typedef struct {
    float lr_means, lr_log_scales, lr_quats, lr_opacity, lr_sh_dc, lr_sh_rest;
    float beta1, beta2, eps;
} as_adam_params;

/* One bias-corrected Adam step on every parameter (Kingma and Ba, Alg. 1):
 *   m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
 *   p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 * params, m, v: updated in place; grads: read.  All four sets have the same row
 * count (params->n) and SH degree; SH coefficient 0 takes lr_sh_dc, the others
 * lr_sh_rest.  step = t >= 1.  AS_ERR_ARG on mismatched sets or t < 1. */
as_status as_adam_step(as_ctx *ctx, as_gaussians_mut *params, const as_gaussians *grads, as_gaussians_mut *m,
                       as_gaussians_mut *v, const as_adam_params *hp, int32_t step, void *stream);

/* L1 photometric loss of an image against its target: sums[0] = sum |d|,
 * sums[1] = sum d^2 over the 3 H W values (d = image - gt, FP64 sums; the
 * mean L1 is sums[0] / (3 H W), the PSNR of [0, 1] images is
 * -10 log10(sums[1] / (3 H W))), and, when dL_dimage is not NULL, the
 * gradient of the mean L1: sign(d) / (3 H W) (sign(0) = 0).
 *   image, gt, dL_dimage: [3][H][W]; sums: device [2], overwritten. */
as_status as_l1_loss(as_ctx *ctx, int32_t width, int32_t height, const float *image, const float *gt, float *dL_dimage,
                     double *sums, void *stream);

/* Densification selection of 3DGS's adaptive density control: with the
 * view-averaged gradient a_i = g2d_accum[i] / max(vis_count[i], 1) (FP64) and
 * the largest scale s_i = exp(max_k log_scales[k][i]) (FP64), Gaussian i is
 * selected when a_i >= grad_threshold; a selected Gaussian is cloned when
 * s_i <= size_threshold and is a split candidate otherwise.
 *   clone_mask, is_candidate: out [n] 0/1; cand: out [n], the candidate ids
 *   ascending; n_cand: out device [1]. */
as_status as_densify_select(as_ctx *ctx, const as_gaussians *g, const float *g2d_accum, const int32_t *vis_count,
                            double grad_threshold, double size_threshold, uint8_t *clone_mask, uint8_t *is_candidate,
                            int32_t *cand, int64_t *n_cand, void *stream);

/* Row map of an as_adaptive_split output: row_src[r] = state_in[i] (or i
 * when state_in is NULL) for the input row i that output row r copies (the
 * non-removed Gaussians, in order), and -1 for the rows the split created
 * (children and parent copies).  A candidate's parent is removed unless its
 * mode is RESET (1).  state_in composes maps across successive steps.
 *   cand, mode: [n_cand] as passed to / returned by as_adaptive_split
 *   state_in: NULL or [n]
 *   row_src: out [capacity]; rows past the survivors are -1.
 *   n_dev, n_cand_dev: NULL, or device [1] counts of the input rows and of the
 *   candidates in use (n and n_cand are then capacities), as for
 *   as_adaptive_split. */
as_status as_split_row_map(as_ctx *ctx, int64_t n, const int32_t *cand, int64_t n_cand, const uint8_t *mode,
                           const int32_t *state_in, int32_t *row_src, int64_t capacity, const int64_t *n_dev,
                           const int64_t *n_cand_dev, void *stream);

/* Clone and prune (3DGS adaptive density control): Gaussian i is kept when
 * sigmoid(opacity_logit) >= min_opacity and, if max_scale > 0,
 * exp(max_k log_scales[k][i]) <= max_scale (decisions in FP64).  Output: the
 * kept rows in order, then a copy of every kept row with clone_mask set, in
 * order.  state_src[r] = state_in[i] (or i when state_in is NULL) for the kept
 * copy of row i and -1 for a clone (a clone starts with fresh optimiser state).
 *   g: n rows (or *g->n_dev of a capacity of n); clone_mask, state_in: NULL or [n]
 *   out: capacity rows (row stride out->n; n + clones always suffices)
 *   state_src: out [capacity]; n_out: out device [1].
 * AS_ERR_CAPACITY when out->n < 2 g->n with a clone mask, or < g->n without. */
as_status as_clone_prune(as_ctx *ctx, const as_gaussians *g, const uint8_t *clone_mask, const int32_t *state_in,
                         double min_opacity, double max_scale, as_gaussians_mut *out, int32_t *state_src,
                         int64_t *n_out, void *stream);

/* dst row r = src row map[r] for map[r] >= 0, zeros for map[r] = -1 (carries
 * optimiser state across a densification).  src: rows with stride src->n;
 * dst: n_rows rows with stride dst->n >= n_rows; the same SH degree.
 * n_rows_dev: NULL, or device [1]: the rows to write (<= n_rows, a capacity). */
as_status as_gather_rows(as_ctx *ctx, const as_gaussians *src, const int32_t *map, int64_t n_rows,
                         as_gaussians_mut *dst, const int64_t *n_rows_dev, void *stream);

/* Opacity reset of 3DGS's density control: opacity <- min(opacity,
 * max_opacity), in logit space, and the Adam moments of the opacities (m_op,
 * v_op: NULL or [n]) cleared. */
as_status as_reset_opacity(as_ctx *ctx, as_gaussians_mut *g, double max_opacity, float *m_op, float *v_op,
                           void *stream);

/* ---- launch tuning ---------------------------------------------------------------- */

/* Launch choices that change speed but never results (the autotuner in the
 * Python package measures them on the caller's workload). */
typedef struct {
    int32_t lds_batch;       /* Gaussian records staged per LDS batch by the blend kernels: 256, 512 or 1024 */
    int32_t longest_first;   /* nonzero: tiles are dispatched in descending order of list length */
    int32_t persistent;      /* nonzero: the blend kernels run as one resident grid pulling tiles from a queue */
    int32_t radix_bits;      /* digit width of the (tile, entry) pair sort, 4..8 (the 32-bit
                                depth keys always take 8: four passes) */
    int32_t block_cull;      /* nonzero: the blend kernels skip a Gaussian for a 4x4 pixel block of a
                                tile unless its alpha >= 1/255 ellipse (with a margin above the
                                FP32 evaluation error) meets the block; zero: the pixel box alone
                                decides.  The contributor sets, and so every output, are the same */
    int32_t single_pass_sort; /* bit 0: the depth sort, bit 1: the pair sort takes one launch per digit
                                (decoupled look-back across blocks) instead of three (reduce, scan,
                                scatter); the same order either way */
    int32_t bin_tile;         /* pixels per side of the squares (tile, Gaussian) pairs are binned by:
                                16 (one blend tile) or 32 (2 x 2 blend tiles of 16 x 16 share one
                                list, so fewer pairs are emitted and sorted; each tile skips the
                                records its box masks exclude).  The blend tiles stay 16 x 16 and
                                every output is the same */
} as_tuning;

/* Set / read the context's tuning (defaults: lds_batch 256, longest_first 1,
 * persistent 0, radix_bits 8, block_cull 1, single_pass_sort 0, bin_tile 16).
 * AS_ERR_ARG for an lds_batch other than 256, 512 or 1024, a radix_bits outside
 * 4..8, a single_pass_sort outside 0..3 or a bin_tile other than 16 or 32. */
as_status as_set_tuning(as_ctx *ctx, const as_tuning *t);
as_status as_get_tuning(const as_ctx *ctx, as_tuning *t);

/* ---- per-stage timing ------------------------------------------------------------ */

/* Stages timed when timing is on (indices into as_timing_read's arrays). */
enum {
    AS_STAGE_PROJECT = 0,      /* projection, colour, depth key, box */
    AS_STAGE_SCAN = 1,         /* exclusive scan of tiles per Gaussian */
    AS_STAGE_EMIT = 2,         /* (tile | depth) key emission */
    AS_STAGE_SORT = 3,         /* LSD radix sort of the keys */
    AS_STAGE_RANGES = 4,       /* per-tile ranges */
    AS_STAGE_BLEND_FWD = 5,    /* forward blend + dominant map + fused L1 error */
    AS_STAGE_BLEND_BWD = 6,    /* reverse blend */
    AS_STAGE_PROJECT_BWD = 7,  /* reverse projection */
    AS_STAGE_ERROR_MAP = 8,    /* as_error_map */
    AS_STAGE_ERROR_STATS = 9,  /* as_accumulate_error_stats */
    AS_STAGE_SPLIT = 10,       /* as_adaptive_split */
    AS_NUM_STAGES = 11
};

/* When `on` is nonzero, every stage above records a pair of hipEvents on the
 * stream of the call that runs it, so its duration is measured on the stream
 * its kernels use.  Costs one event pair per stage; off by default. */
as_status as_timing_enable(as_ctx *ctx, int32_t on);

/* Wait for the recorded events, add each stage's elapsed milliseconds to
 * ms[AS_NUM_STAGES] and its number of runs to runs[AS_NUM_STAGES] (host
 * arrays, zeroed by this call first), and forget the records. */
as_status as_timing_read(as_ctx *ctx, double *ms, int64_t *runs);

/* ---- graph capture ------------------------------------------------------------- */

/* Record every call made on `stream` between as_graph_begin and as_graph_end
 * into a HIP graph, replayed by as_graph_launch with the same arguments
 * (the device buffers the calls named must stay allocated, and their
 * contents at replay time are the inputs).  The calls of the path and of
 * the loop never synchronise or allocate, so any of them can be captured once
 * the frames exist and the context's reservation covers the sizes; the
 * set-up calls (frame creation, as_frame_reserve_keys, as_ctx_reserve)
 * return AS_ERR_STATE inside a capture.  Per-stage timing is suspended while
 * capturing. */
typedef struct as_graph as_graph;
as_status as_graph_begin(as_ctx *ctx, void *stream);
as_status as_graph_end(as_ctx *ctx, void *stream, as_graph **out);
as_status as_graph_launch(as_graph *graph, void *stream);
void as_graph_destroy(as_graph *graph);

/* ---- test hooks --------------------------------------------------------------- */

/* Stable LSD radix sort of n (key, value) pairs on the low key_bits bits, in
 * place (the sorter the binning uses, with the context's radix_bits).  A
 * test hook: it grows its own scratch on demand (it allocates).
 * keys [n], vals [n]; bits at and above key_bits are ignored. */
as_status as_debug_sort_pairs(as_ctx *ctx, uint64_t *keys, uint32_t *vals, int64_t n, int32_t key_bits, void *stream);

/* The binning's 32-bit sorter: stable sort of n (key, value) pairs on key bits
 * [lo_bit, hi_bit) with digits of radix_bits (4..8) bits, in place, by one
 * launch per digit (single_pass nonzero) or three.  gather_src / gather_dst
 * (both NULL, or device arrays: gather_src indexed by values, gather_dst [n]):
 * the last digit pass also writes gather_dst[r] = gather_src[value at r].  A
 * test hook: it grows its own scratch on demand (it allocates).  Returns
 * AS_ERR_HIP if a single-pass wait hit its limit. */
as_status as_debug_sort_u32(as_ctx *ctx, uint32_t *keys, uint32_t *vals, int64_t n, int32_t lo_bit, int32_t hi_bit,
                            int32_t radix_bits, int32_t single_pass, const uint32_t *gather_src, uint32_t *gather_dst,
                            void *stream);

/* Element-wise FP64 sqrt(a), a / b, exp(b) and log(a) on the device, used to
 * check that the decision arithmetic rounds like the host's.  out[4][n]. */
as_status as_debug_fp64_ops(as_ctx *ctx, const double *a, const double *b, int64_t n, double *out, void *stream);

/* Test hook: with force_64bit nonzero, the projection and the single-view
 * projection backward of this context address the SH coefficient rows by
 * 64-bit row addresses, the form they take when 48 rows of n floats exceed
 * 32-bit byte offsets (n of 22M and more), instead of one buffer resource with
 * 32-bit row offsets.  The results do not depend on it; it lets the wide form
 * be tested at small n.  Zero restores the default.  AS_ERR_ARG on a null
 * context. */
as_status as_debug_row_addressing(as_ctx *ctx, int32_t force_64bit);

/* The forward and reverse blends' unclamped alpha o G of Eq. (rendering),
 * evaluated in FP32 from the staged record of the last render exactly as the
 * blend kernels evaluate it, for n (pixel, Gaussian) pairs of view 0 of the
 * frame: pix [n][2] (x, y) int32, gauss [n] Gaussian ids (visible in the
 * view: tiles touched > 0), out [n] float.  Used to measure the FP32 rounding
 * of the alpha decisions against an FP64 reference.  AS_ERR_STATE without a
 * render; no bounds checks beyond the arguments' shapes. */
as_status as_debug_blend_alpha(const as_frame *f, int32_t view, int64_t n, const int32_t *pix, const uint32_t *gauss,
                               float *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* ADPSPLIT_H */
