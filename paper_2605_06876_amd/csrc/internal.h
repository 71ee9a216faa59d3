// Internal declarations shared by the HIP translation units of libadpsplit.
// Not part of the C-ABI (include/adpsplit.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adpsplit.h"

#define AS_TILE_W 16
#define AS_TILE_H 16
#define AS_BLOCK 256        // threads per tile block: one 16x16 tile, four wave64
#define AS_CK_MAX 3         // forward checkpoints per tile (the reverse pass splits a tile into up to 4 segments)
#define AS_NEAR 0.2
#define AS_LOWPASS 0.3
#define AS_MAX_VIEWS 16   // views of one batched render

// Blend record of one projected Gaussian, 48 bytes (three float4):
//   [0] mean_x hi, mean_y hi, mean_x lo, mean_y lo  (mean = hi + lo, continuous pixel frame)
//   [1] conic xx, conic xy, conic yy, opacity
//   [2] r, g, b, 0
struct __align__(16) BlendRec {
    float4 m, c, rgb;
};

// Camera in device-friendly form, passed by value to kernels.
struct DevCam {
    float R[9], t[3], fx, fy, cx, cy;
    int32_t W, H;
    float bg[3];
};

static inline DevCam to_devcam(const as_camera &c) {
    DevCam d;
    for (int k = 0; k < 9; k++) d.R[k] = c.R[k];
    for (int k = 0; k < 3; k++) d.t[k] = c.t[k];
    d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
    d.W = c.width; d.H = c.height;
    for (int k = 0; k < 3; k++) d.bg[k] = c.bg[k];
    return d;
}

struct GaussPtrs {
    const float *means, *log_scales, *quats, *opac, *sh;
    int64_t n;               // row stride (and capacity when n_dev is set)
    int32_t deg;
    const int64_t *n_dev;    // NULL, or device [1]: the rows in use (<= n)
};

struct GradPtrs {
    float *means, *log_scales, *quats, *opac, *sh;
    int64_t stride;
};

// A growable device buffer.  devbuf_ensure allocates devbuf_size(bytes),
// and only the set-up calls (as_ctx_create, as_ctx_reserve) call it.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};
static inline size_t devbuf_size(size_t bytes) { return ((bytes < 256 ? 256 : bytes) + 255) & ~(size_t)255; }
hipError_t devbuf_ensure(DevBuf &b, size_t bytes);
void devbuf_free(DevBuf &b);
// True when b holds at least `bytes` (the calls check their scratch with it).
static inline bool devbuf_has(const DevBuf &b, size_t bytes) { return b.p && b.bytes >= bytes; }

// The views of one render, passed by value to the kernels.  View v owns
//   entries  [ent_base[v], ent_base[v+1])  (its Gaussians, projected),
//   tiles    [tile_base[v], tile_base[v+1]) (global tile ids, row-major within the view),
//   pixels   [pix_base[v], pix_base[v+1])   (of the packed per-pixel maps).
struct ViewTable {
    int32_t n_views;
    int32_t tile_base[AS_MAX_VIEWS + 1];
    int32_t tiles_x[AS_MAX_VIEWS];
    // Pairs are binned by square bins of 2^bin_shift pixels (16 or 32): a bin
    // of 32 holds the 2 x 2 blend tiles of 16 x 16 pixels it covers, which
    // share its pair list.
    int32_t bin_shift;
    int32_t bin_base[AS_MAX_VIEWS + 1];
    int32_t bins_x[AS_MAX_VIEWS];
    uint32_t ent_base[AS_MAX_VIEWS + 1];
    int64_t pix_base[AS_MAX_VIEWS + 1];
    DevCam cam[AS_MAX_VIEWS];
};

// Per-view image pointers ([3][H][W] each).
struct ViewImages {
    float *p[AS_MAX_VIEWS];
};
struct ViewImagesC {
    const float *p[AS_MAX_VIEWS];
};
// Per-view Gaussian sets of a render (views may share one).
struct SceneTable {
    GaussPtrs g[AS_MAX_VIEWS];
};

struct as_frame {
    as_ctx *ctx;
    int device;   // the context's device, kept so that destroying the frame never reads the context
    int32_t max_views;
    int32_t fixed_w, fixed_h;   // single-view frames: the one size they render (0: any)
    uint32_t flags;             // AS_FRAME_*
    int64_t ent_cap, pix_cap, tile_cap, key_cap;
    // per entry (a Gaussian in one view)
    BlendRec *rec;
    uint32_t *depth_key;
    int16_t *box;          // [entries][4]
    uint32_t *ntiles;
    uint32_t *offsets;     // key offsets, in depth order
    float *grad2d;         // [ent_cap][9] entry-major: the 2D gradients of entry e at 9 e .. 9 e + 8
    int g2d_zero = 0;      // grad2d is all zeros over the last render's entries (its forward cleared it)
    int g2d_zero_capture = 0;   // the graph capture that render was recorded in (0: run eagerly)
    // depth-first binning: entries sorted by depth, then keys by tile
    uint32_t *dkeys[2];
    uint32_t *dvals[2];
    uint32_t *nt_sorted;   // tiles touched, in depth order
    uint32_t *n_ent;       // [1] device copy of the entry count
    DevBuf dsort_hist;
    // pairs: tile id (key) and entry id (value)
    uint32_t *keys[2];
    uint32_t *vals[2];
    int sorted_sel;
    uint32_t *ranges;      // [tiles][2]
    uint32_t *tile_order;  // [2 tiles + 64] dispatch order of the forward blend (longest list first; with bins
                           // of 32, slots grouped by XCD with empty slots past the image edge)
    uint32_t *tile_work;   // [tiles] contributors summed over the tile's pixels, from the forward blend
    uint32_t *tile_order_bwd;  // [tiles] dispatch order of the reverse blend (most contributors first)
    uint32_t *tile_hi;     // [tiles] one past the tile's last contributor (0: none), from the forward blend
    float *ckpt;           // [tile_cap][AS_CK_MAX][256][4] per pixel (T, colour behind) at the forward's batch
                           // boundaries; NULL in forward-only frames
    uint16_t *bmask;       // [key_cap][4] per sorted pair and blend tile of its bin (mask_slot): the 4x4 pixel
                           // blocks of the tile it may contribute to, from the forward blend for the reverse
                           // blend; NULL in forward-only frames
    int bm_written;        // the last render wrote bmask for every pair the reverse pass walks
    uint32_t *bwd_items;   // [tile_cap * (AS_CK_MAX + 1)][2] (tile, segment) work items of the reverse blend
    uint32_t *n_items;     // [1] device count of bwd_items
    int ck_written;        // the last render wrote checkpoints
    int ck_seg;            // their spacing in list entries (the forward's batch depth)
    int use_order;         // tile_order is valid for the last render
    uint32_t *n_keys;      // [2] device: pairs the render needs, pairs it wrote (fewer when over key_cap)
    uint32_t *queue;       // [2] tile counters of the persistent blend kernels
    // per pixel, packed over the views
    float *t_final;
    uint32_t *last;
    uint32_t *n_contrib;
    int32_t *dom;
    double *err;
    uint64_t *err_minmax;  // [max_views][2]
    uint64_t *tile_err;    // [tile_cap][2] per-tile error min / max (IEEE bits), reduced into err_minmax
    // scratch for scans and the sorter
    DevBuf scan_tmp, sort_hist;
    // state of the last render
    int has_render;
    ViewTable vt;
    SceneTable scenes;
    int32_t has_gt;
    int32_t persistent_last;
};

struct StageRec {
    int stage;
    hipEvent_t beg, end;
};

struct as_ctx {
    int device;
    DevBuf es[16];    // error-statistics scratch (errstats.hip names the slots)
    DevBuf sp[24];    // adaptive-split scratch (split.hip names the slots)
    DevBuf dbg[6];    // test hooks
    DevBuf tr[8];     // optimisation-loop scratch (train.hip kernels; slots named in api.hip)
    as_reserve res{};             // what es, sp and tr hold (as_ctx_reserve)
    int lds_batch = 256;          // launch tuning (as_set_tuning)
    int longest_first = 1;
    int persistent = 0;
    int radix_bits = 8;
    int block_cull = 1;
    int single_pass_sort = 0;   // bit 0 depth sort, bit 1 pair sort
    int bin_tile = 16;          // pixels per side of the binning squares (16 or 32)
    int row_addr64 = 0;         // test hook: SH rows by 64-bit addresses even where buffer offsets fit
    int n_cu = 0;                 // compute units of the device
    int timing = 0;
    StageRec *recs = nullptr;     // recorded stage event pairs
    int n_recs = 0, cap_recs = 0;
    hipEvent_t *pool = nullptr;   // idle events
    int n_pool = 0, cap_pool = 0;
};

// Records a hipEvent pair around one stage on stream s when timing is on.
struct StageTimer {
    as_ctx *ctx;
    int stage;
    hipStream_t s;
    hipEvent_t beg = nullptr;
    StageTimer(as_ctx *c, int st, hipStream_t str);
    ~StageTimer();
};

// ---- launchers (each defined in the .hip file that holds the kernel) -------------

// projection (project.hip): every view's Gaussians into its entry range
// Projection of every entry; also writes the depth sort's input pairs
// (depth key, entry id) and the device entry count.
void launch_project(const SceneTable &sc, const ViewTable &vt, int64_t max_n, int deg, BlendRec *rec,
                    uint32_t *depth_key, int16_t *box, uint32_t *ntiles, uint32_t *sort_keys, uint32_t *sort_vals,
                    uint32_t *n_ent, hipStream_t s, bool force_addr64 = false);
// projection backward (project_bwd.hip): one Gaussian set seen in every view
// of vt; gradients summed over the views in view order
void launch_project_bwd(const GaussPtrs &g, const ViewTable &vt, const uint32_t *ntiles, const float *grad2d,
                        GradPtrs out, float *g2d_norm, int32_t *vis_count, hipStream_t s, bool force_addr64 = false);

// scans (binning.hip): exclusive scans with the total written to *total
size_t scan_tmp_bytes(int64_t n);
void scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total, void *tmp, hipStream_t s);
void scan_u8_to_i64(const uint8_t *in, int64_t *out, int64_t n, int64_t *total, void *tmp, hipStream_t s);
void scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, int64_t *total, void *tmp, hipStream_t s);

// LSD radix sort (radix.hip).  Sorts (keys[0], vals[0]) stably on bits
// [lo_bit, hi_bit) with digits of radix_bits (4..8) bits, ping-ponging with
// (keys[1], vals[1]); returns which buffer holds the result.  The element
// count is read from the device (*n_dev, clamped to cap); n_hint sizes the
// grid.  hist is a workspace of sort_hist_bytes(cap) bytes for the same cap.
size_t sort_hist_bytes(int64_t cap);
// gather_src/gather_dst (optional): the last pass also writes
// gather_dst[r] = gather_src[sorted value r].
// single_pass: one launch per digit with decoupled look-back (used when
// sort_single_pass_ok(cap)); otherwise three launches per digit.  Both give
// the same order.  The single-pass sort raises a flag in the workspace at
// byte sort_wait_flag_offset() if a look-back wait hit its limit.
int radix_sort_u32(uint32_t *keys[2], uint32_t *vals[2], const uint32_t *n_dev, int64_t cap, int64_t n_hint, int lo_bit,
                   int hi_bit, int radix_bits, void *hist, hipStream_t s, const uint32_t *gather_src = nullptr,
                   uint32_t *gather_dst = nullptr, bool single_pass = false);
bool sort_single_pass_ok(int64_t cap);
uint32_t sort_wait_flag_offset();
int radix_sort_u64(uint64_t *keys[2], uint32_t *vals[2], const uint32_t *n_dev, int64_t cap, int64_t n_hint, int lo_bit,
                   int hi_bit, int radix_bits, void *hist, hipStream_t s);
// Depth-first binning: keys emitted in the depth order a stable depth sort
// produced; the emission also empties the tile ranges ([0, 0) for every tile)
// ahead of launch_ranges.  *n_emit gets the number of pairs written: all of
// them when they fit in key_cap, else the offset of the first entry dropped.
void launch_emit_sorted(int64_t n, const uint32_t *order, const ViewTable &vt, const int16_t *box,
                        const uint32_t *nt_sorted, const uint32_t *offsets, int64_t key_cap, uint32_t *keys,
                        uint32_t *vals, uint32_t *n_emit, uint32_t *ranges, int64_t n_tiles, hipStream_t s);
// [start, end) of each tile with keys (ranges emptied by launch_emit_sorted).
void launch_ranges(const uint32_t *keys, const uint32_t *n_dev, int64_t cap, int64_t n_bins, const ViewTable &vt,
                   uint32_t *ranges, hipStream_t s);
void launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s);
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
void launch_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s);
void launch_fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s);
void launch_copy_u32(const uint32_t *src, uint32_t *dst, int64_t n, hipStream_t s);

// blend (blend.hip)
struct BlendLaunch {
    int batch;         // LDS depth: 256, 512 or 1024 records
    int persistent;    // 1: one resident grid pulling tiles from f->queue
    int n_cu;
    int ellipse;       // 1: per-block culling by the alpha >= 1/255 ellipse, not only the box
};
// The forward blend's LDS depth for a launch (256, 512 or 1024 records).
int blend_fwd_batch(const BlendLaunch &bl);
void launch_tile_order(const uint32_t *ranges, const ViewTable &vt, uint32_t *order, hipStream_t s);
// After the forward blend: per-view error ranges, the reverse pass's dispatch
// order (when order_on) and its work items, from the render's checkpoint state.
void launch_after_fwd(const as_frame *f, const ViewTable &vt, const ViewImagesC &gt, int order_on, hipStream_t s);
// Forward blend; with zero_g2d it also clears zero_floats floats there (rounded
// up to a multiple of four: the buffer needs that slack) and returns whether
// it ran (no tiles: nothing launched, nothing cleared).
bool launch_blend_fwd(const as_frame *f, const uint32_t *vals, const uint32_t *tile_order, const BlendLaunch &bl,
                      const ViewTable &vt, const ViewImagesC &gt, const ViewImages &image, hipStream_t s,
                      float *zero_g2d = nullptr, int64_t zero_floats = 0);
void launch_debug_alpha(const as_frame *f, int64_t n, const int32_t *pix, const uint32_t *ent, float *out,
                        hipStream_t s);
void launch_blend_bwd(const as_frame *f, const uint32_t *vals, const uint32_t *tile_order, const BlendLaunch &bl,
                      const ViewTable &vt, const ViewImagesC &dL_dimage, float *grad2d, hipStream_t s);

// optimisation loop (train.hip)
int train_set_rows(int deg);
void launch_adam(const as_gaussians_mut &p, const as_gaussians &g, const as_gaussians_mut &m, const as_gaussians_mut &v,
                 const as_adam_params &hp, int32_t step, hipStream_t s);
size_t l1_partials_bytes();
void launch_l1(int W, int H, const float *img, const float *gt, float *dL, double *sums, double *partials,
               hipStream_t s);
void launch_select(const as_gaussians &g, const float *accum, const int32_t *vis, double thr, double size_thr,
                   uint8_t *clone, uint8_t *cand_flag, hipStream_t s);
void launch_compact_ids(int64_t n, const uint8_t *flag, const int64_t *scan, int32_t *out, hipStream_t s);
void launch_keep_init(int64_t n, const int64_t *n_dev, uint8_t *keep, hipStream_t s);
void launch_mark_kept(const int32_t *cand, int64_t n_cand, const int64_t *n_cand_dev, const uint8_t *mode, int64_t n,
                      uint8_t *keep, hipStream_t s);
void launch_row_map(int64_t n, const uint8_t *keep, const int64_t *pos, const int32_t *state_in, int64_t capacity,
                    int32_t *row_src, hipStream_t s);
void launch_prune_flags(const as_gaussians &g, const uint8_t *clone_mask, double min_op, double max_scale,
                        uint8_t *keep, uint8_t *dup, hipStream_t s);
void launch_clone_prune_write(const as_gaussians &g, const as_gaussians_mut &out, const uint8_t *keep,
                              const uint8_t *dup, const int64_t *kpos, const int64_t *dpos, const int64_t *n_keep,
                              const int64_t *n_dup, const int32_t *state_in, int32_t *state_src, int64_t *n_out,
                              hipStream_t s);
void launch_gather_rows(const as_gaussians &src, const int32_t *map, int64_t n_rows, const int64_t *n_rows_dev,
                        const as_gaussians_mut &dst, hipStream_t s);
void launch_reset_opacity(const as_gaussians_mut &g, float cap, float *m, float *v, hipStream_t s);

// error statistics (errstats.hip)
void launch_error_map(int W, int H, const float *image, const float *gt, double *err, uint64_t *minmax,
                      hipStream_t s);
// Scratch of the error statistics for views of up to max_pixels pixels.
size_t errstats_reserve_bytes(int64_t max_pixels);
hipError_t errstats_reserve(as_ctx *ctx, int64_t max_pixels);
as_status run_error_stats(as_ctx *ctx, int W, int H, const double *err, const uint64_t *minmax, const int32_t *dom,
                          const float *gt, int view, int64_t n, const uint8_t *is_cand, const as_split_params &p,
                          as_region_buf &rb, int32_t *attr, hipStream_t s);
// The no-allocation variant: scratch from a static device array whose address
// on each device errstats_noalloc_init records (called by as_ctx_create with
// the device current).
hipError_t errstats_noalloc_init(int device);
size_t errstats_noalloc_bytes();
as_status run_error_stats_noalloc(as_ctx *ctx, int W, int H, const double *err, const uint64_t *minmax,
                                  const int32_t *dom, const float *gt, int view, const uint8_t *is_cand,
                                  const as_split_params &p, as_region_buf &rb, int32_t *attr, hipStream_t s);

// adaptive split (split.hip)
// Random children per candidate the variant may draw noise for.
static inline int split_noise_need(const as_split_params &p) {
    int need = 2;
    if (p.variant == AS_VARIANT_FIXED_N && p.fixed_n > need) need = p.fixed_n;
    if (p.variant == AS_VARIANT_ADAPTIVE_N && p.n_max > need) need = p.n_max;
    return need;
}

// Rows the split appends per candidate at most: fixed_n for the fixed-N
// split (the parent is removed), else N_max children plus the parent copy
// of the adaptive mode (at least 2: the vanilla fallback).
inline int64_t split_rows_per_candidate(const as_split_params &p) {
    if (p.variant == AS_VARIANT_FIXED_N) return p.fixed_n;
    return p.n_max + 1 > 2 ? p.n_max + 1 : 2;
}
// Scratch of the split for the region, candidate, view and Gaussian maxima of r.
size_t split_reserve_bytes(const as_reserve &r);
hipError_t split_reserve(as_ctx *ctx, const as_reserve &r);
as_status run_adaptive_split(as_ctx *ctx, const GaussPtrs &g, const int32_t *cand, int64_t n_cand,
                             const int64_t *n_cand_dev,
                             const as_region_buf &rb, const as_camera *views, int n_views, const int32_t *attr,
                             const as_split_params &p, const float *noise, GradPtrs out, int64_t out_cap,
                             uint8_t *mode, int32_t *count, int64_t *offset, int64_t *n_out, hipStream_t s);

// Code-object warm-up.  Each source file's kernels are a code object of their
// own, which the runtime loads, allocating device memory for it, at the first
// launch from that file.  The context launches one empty kernel per file at
// creation, so that no call of the path triggers such a load.
#define AS_WARM_KERNEL(name)                                                        \
    __global__ void k_warm_##name() {}                                              \
    void warm_##name(hipStream_t s) { hipLaunchKernelGGL(k_warm_##name, dim3(1), dim3(1), 0, s); }
void warm_api(hipStream_t s);
void warm_binning(hipStream_t s);
void warm_blend(hipStream_t s);
void warm_errstats(hipStream_t s);
void warm_project(hipStream_t s);
void warm_project_bwd(hipStream_t s);
void warm_radix(hipStream_t s);
void warm_split(hipStream_t s);
void warm_train(hipStream_t s);

// debug (binning.hip)
void launch_fp64_ops(const double *a, const double *b, int64_t n, double *out, hipStream_t s);

// error reporting (api.cpp)
void as_set_error(const char *fmt, ...);

// ---- device helpers -----------------------------------------------------------------

#ifdef __HIPCC__
// Rows of a Gaussian set in use, and the entries of a capacity-sized list in
// use: the device count when one is given (at most the capacity), else the
// host size.
__device__ __forceinline__ int64_t count_in_use(int64_t cap, const int64_t *dev) {
    if (!dev) return cap;
    const int64_t c = *dev;
    return c < 0 ? 0 : (c < cap ? c : cap);
}
__device__ __forceinline__ int64_t rows_in_use(const GaussPtrs &g) { return count_in_use(g.n, g.n_dev); }
__device__ __forceinline__ float wave_sum(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_min_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
// View holding a global tile id / an entry id (linear scans over at most
// AS_MAX_VIEWS bases; the tables are kernel arguments).
__device__ __forceinline__ int view_of_tile(const ViewTable &vt, int tile) {
    int v = 0;
    for (int k = 1; k < vt.n_views; k++) v += tile >= vt.tile_base[k] ? 1 : 0;
    return v;
}
__device__ __forceinline__ int view_of_bin(const ViewTable &vt, int bin) {
    int v = 0;
    for (int k = 1; k < vt.n_views; k++) v += bin >= vt.bin_base[k] ? 1 : 0;
    return v;
}
// Index of a blend tile's block mask for sorted pair i: bins of 32 keep the
// masks of their four tiles side by side.
__device__ __forceinline__ size_t mask_slot(const ViewTable &vt, uint32_t i, int tx, int ty) {
    const int q = vt.bin_shift - 4;
    return ((size_t)i << (2 * q)) + (size_t)(((ty & q) << q) | (tx & q));
}
__device__ __forceinline__ int view_of_entry(const ViewTable &vt, uint32_t e) {
    int v = 0;
    for (int k = 1; k < vt.n_views; k++) v += e >= vt.ent_base[k] ? 1 : 0;
    return v;
}
// Element of row `row` of a struct-of-arrays tensor with row stride `n`, for
// the lane whose byte offset in a row is `boff` (Gaussian i: 4 i; sets hold fewer than 2^30 rows).
// The row base is wave-uniform and the lane part one 32-bit offset shared by
// every row, so each access is a load or store with a scalar base and the
// same vector offset, rather than a 64-bit address per row held in vector
// registers (the 48 SH rows alone would take 96 register pairs).
__device__ __forceinline__ const float &at_row(const float *a, int64_t row, int64_t n, uint32_t boff) {
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(a + row * n) + boff);
}
__device__ __forceinline__ float &at_row(float *a, int64_t row, int64_t n, uint32_t boff) {
    return *reinterpret_cast<float *>(reinterpret_cast<char *>(a + row * n) + boff);
}

// Fourth word of a gfx9 buffer resource for raw 32-bit accesses: data format
// 32 (bits 15..18 = 4), no swizzle, no index stride.
#define AS_BUFFER_RSRC_WORD3 0x00020000

__device__ __forceinline__ uint64_t lanemask_lt() {
    const unsigned lane = __lane_id();
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}
#endif
