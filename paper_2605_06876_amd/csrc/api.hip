// Host side of the C-ABI declared in include/adpsplit.h: argument checks,
// frame lifetime and the launch order of each call.  No kernels live here.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <new>

#include "internal.h"

namespace {
thread_local char g_err[1024] = "";
thread_local int g_capturing = 0;   // inside as_graph_begin / as_graph_end on this thread
thread_local int g_capture_id = 0;  // the open capture's number (0: none open)
thread_local int g_captures = 0;    // captures begun on this thread

bool bad(hipError_t e, const char *what) {
    if (e == hipSuccess) return false;
    as_set_error("%s: %s", what, hipGetErrorString(e));
    return true;
}

as_status launch_status(const char *what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        as_set_error("%s: kernel launch failed: %s", what, hipGetErrorString(e));
        return AS_ERR_HIP;
    }
    return AS_OK;
}

int tile_bits(int64_t tiles) {
    int b = 0;
    while ((int64_t(1) << b) < tiles) b++;
    return b;
}

bool check_gauss(const as_gaussians *g, const char *what) {
    if (!g) { as_set_error("%s: null Gaussians", what); return false; }
    // rows are addressed with 32-bit byte offsets (4 n < 2^32)
    if (g->n < 0 || g->n >= (1ll << 30)) { as_set_error("%s: n = %lld not in [0, 2^30)", what, (long long)g->n); return false; }
    if (g->sh_degree < 0 || g->sh_degree > 3) { as_set_error("%s: sh_degree %d not in 0..3", what, g->sh_degree); return false; }
    if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh)) {
        as_set_error("%s: null parameter pointer", what);
        return false;
    }
    return true;
}

bool check_mut(const as_gaussians_mut *g, int64_t rows, int32_t deg, const char *what) {
    if (!g) { as_set_error("%s: null output", what); return false; }
    if (g->n < rows) { as_set_error("%s: output stride %lld < %lld rows", what, (long long)g->n, (long long)rows); return false; }
    if (g->sh_degree != deg) { as_set_error("%s: output sh_degree %d != %d", what, g->sh_degree, deg); return false; }
    if (rows > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh)) {
        as_set_error("%s: null output pointer", what);
        return false;
    }
    return true;
}

GaussPtrs gptrs(const as_gaussians *g) {
    GaussPtrs p;
    p.means = g->means; p.log_scales = g->log_scales; p.quats = g->quats; p.opac = g->opacity_logits; p.sh = g->sh;
    p.n = g->n; p.deg = g->sh_degree; p.n_dev = g->n_dev;
    return p;
}

// Calls whose launches follow the host row count refuse a device count.
bool host_count_only(const as_gaussians *g, const char *what) {
    if (g && g->n_dev) {
        as_set_error("%s: takes no device row count (n_dev); only the densification calls do", what);
        return false;
    }
    return true;
}

GradPtrs mptrs(const as_gaussians_mut *g) {
    GradPtrs p;
    p.means = g->means; p.log_scales = g->log_scales; p.quats = g->quats; p.opac = g->opacity_logits; p.sh = g->sh;
    p.stride = g->n;
    return p;
}

bool check_params(const as_split_params *p, const char *what) {
    if (!p) { as_set_error("%s: null params", what); return false; }
    if (!(p->tau_l1 >= 0.0 && p->tau_l1 < 1.0) || p->r_erode < 0 || p->r_erode > 64 || p->m_min < 1 || p->L < 1 ||
        p->L > 255 || p->n_max < 0 || p->n_max > 4096 || !(p->gamma_d >= 0.0) || !(p->gamma_c >= 0.0) ||
        !(p->eps >= 0.0) || !(p->eta > 0.0)) {
        as_set_error("%s: parameter out of range", what);
        return false;
    }
    if (p->variant < AS_VARIANT_ADPSPLIT || p->variant > AS_VARIANT_CHILD_INIT ||
        (p->flags & ~(uint32_t)(AS_SPLIT_ERODE_SIDE | AS_SPLIT_CROSS_VIEW | AS_SPLIT_EXTENT_MAX | AS_SPLIT_SHARE_OPACITY)) ||
        (p->variant == AS_VARIANT_FIXED_N && (p->fixed_n < 1 || p->fixed_n > 4096)) || p->noise_n < 0) {
        as_set_error("%s: variant %d / flags 0x%x / fixed_n %d / noise_n %d invalid", what, p->variant, p->flags,
                     p->fixed_n, p->noise_n);
        return false;
    }
    return true;
}

template <typename T>
hipError_t dmalloc(T **p, size_t count) {
    return hipMalloc((void **)p, count * sizeof(T) + 256);
}

// scratch slots of ctx->tr (the optimisation loop's calls)
enum { TR_PART, TR_FLAG, TR_SCAN, TR_TMP, TR_DUP, TR_DSCAN, TR_TOT, TR_TMP2 };

// Bytes of the loop's Gaussian-sized slots for up to n rows (TR_PART and
// TR_TOT are fixed and allocated with the context).
void tr_need(int64_t n, size_t need[8]) {
    const size_t m = (size_t)(n > 0 ? n : 1);
    for (int k = 0; k < 8; k++) need[k] = 0;
    need[TR_FLAG] = m;
    need[TR_DUP] = m;
    need[TR_SCAN] = m * 8;
    need[TR_DSCAN] = m * 8;
    need[TR_TMP] = scan_tmp_bytes((int64_t)m);
    need[TR_TMP2] = scan_tmp_bytes((int64_t)m);
}

size_t round256(size_t b) { return ((b < 256 ? 256 : b) + 255) & ~(size_t)255; }

// Every device buffer of a frame with the capacities and flags in f, in one
// table: visit(slot, bytes) is called once per buffer.  frame_alloc,
// as_frame_destroy and the size queries walk the same table, so the bytes a
// query reports are the bytes a frame holds.  `keys_only` visits just the
// buffers that scale with the pair capacity (as_frame_reserve_keys).
template <typename V>
void frame_buffers(as_frame *f, bool keys_only, V &&visit) {
    const int64_t ent = f->ent_cap, pix = f->pix_cap, tile = f->tile_cap, key = f->key_cap;
    auto arr = [&](auto **p, int64_t count) { visit((void **)p, round256((size_t)count * sizeof(**p) + 256)); };
    auto dbuf = [&](DevBuf &b, size_t bytes) {
        b.bytes = round256(bytes);
        visit(&b.p, b.bytes);
    };
    for (int k = 0; k < 2; k++) {
        arr(&f->keys[k], key);
        arr(&f->vals[k], key);
    }
    dbuf(f->sort_hist, sort_hist_bytes(key));
    // block masks: one per sorted pair and blend tile of its bin (four for bins of 32)
    if (!(f->flags & AS_FRAME_FORWARD_ONLY)) arr(&f->bmask, key * 4);
    if (keys_only) return;
    arr(&f->rec, ent); arr(&f->depth_key, ent); arr(&f->box, ent * 4); arr(&f->ntiles, ent); arr(&f->offsets, ent);
    arr(&f->grad2d, ent * 9);
    arr(&f->dkeys[0], ent); arr(&f->dkeys[1], ent); arr(&f->dvals[0], ent); arr(&f->dvals[1], ent);
    arr(&f->nt_sorted, ent); arr(&f->n_ent, 4); arr(&f->n_keys, 4);
    dbuf(f->dsort_hist, sort_hist_bytes(ent));
    dbuf(f->scan_tmp, scan_tmp_bytes(ent));
    // forward dispatch slots: the tiles, or 32 per 8 bins of 32 (at most 2 tile + 64)
    arr(&f->ranges, tile * 2); arr(&f->tile_order, 2 * tile + 64); arr(&f->queue, 2); arr(&f->tile_work, tile);
    arr(&f->tile_order_bwd, tile); arr(&f->tile_hi, tile); arr(&f->n_items, 1);
    arr(&f->bwd_items, tile * (AS_CK_MAX + 1) * 2);
    arr(&f->tile_err, tile * 2);
    if (!(f->flags & AS_FRAME_FORWARD_ONLY)) arr(&f->ckpt, tile * AS_CK_MAX * 256 * 4);
    arr(&f->t_final, pix); arr(&f->last, pix); arr(&f->n_contrib, pix); arr(&f->dom, pix); arr(&f->err, pix);
    arr(&f->err_minmax, 2 * (int64_t)f->max_views);
}

void frame_free_buffers(as_frame *f, bool keys_only) {
    frame_buffers(f, keys_only, [](void **p, size_t) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    });
}

hipError_t frame_alloc_buffers(as_frame *f, bool keys_only) {
    hipError_t e = hipSuccess;
    frame_buffers(f, keys_only, [&](void **p, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, bytes);
    });
    return e;
}
}  // namespace

void as_set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

hipError_t devbuf_ensure(DevBuf &b, size_t bytes) {
    if (b.p && b.bytes >= bytes) return hipSuccess;
    if (g_capturing) return hipErrorStreamCaptureUnsupported;   // no allocation inside a capture
    if (b.p) {
        (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t nb = bytes < 256 ? 256 : bytes;
    nb = (nb + 255) & ~(size_t)255;
    const hipError_t e = hipMalloc(&b.p, nb);
    if (e == hipSuccess) b.bytes = nb;
    return e;
}

void devbuf_free(DevBuf &b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

static hipEvent_t pool_get(as_ctx *c) {
    if (c->n_pool > 0) return c->pool[--c->n_pool];
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

static void pool_put(as_ctx *c, hipEvent_t e) {
    if (!e) return;
    if (c->n_pool == c->cap_pool) {
        const int nc = c->cap_pool ? 2 * c->cap_pool : 64;
        hipEvent_t *p = (hipEvent_t *)realloc(c->pool, sizeof(hipEvent_t) * nc);
        if (!p) { (void)hipEventDestroy(e); return; }
        c->pool = p;
        c->cap_pool = nc;
    }
    c->pool[c->n_pool++] = e;
}

StageTimer::StageTimer(as_ctx *c, int st, hipStream_t str) : ctx(c), stage(st), s(str) {
    if (!ctx || !ctx->timing || g_capturing) return;
    beg = pool_get(ctx);
    if (beg) (void)hipEventRecord(beg, s);
}

StageTimer::~StageTimer() {
    if (!beg) return;
    hipEvent_t end = pool_get(ctx);
    if (!end) { pool_put(ctx, beg); return; }
    (void)hipEventRecord(end, s);
    if (ctx->n_recs == ctx->cap_recs) {
        const int nc = ctx->cap_recs ? 2 * ctx->cap_recs : 256;
        StageRec *p = (StageRec *)realloc(ctx->recs, sizeof(StageRec) * nc);
        if (!p) { pool_put(ctx, beg); pool_put(ctx, end); return; }
        ctx->recs = p;
        ctx->cap_recs = nc;
    }
    ctx->recs[ctx->n_recs++] = StageRec{stage, beg, end};
}

extern "C" {

const char *as_last_error(void) { return g_err; }
const char *as_version(void) { return "adpsplit 0.1.0 (gfx950)"; }

as_status as_ctx_create(int device, as_ctx **out) {
    if (!out) { as_set_error("as_ctx_create: null out"); return AS_ERR_ARG; }
    *out = nullptr;
    if (bad(hipSetDevice(device), "hipSetDevice")) return AS_ERR_HIP;
    hipDeviceProp_t prop;
    if (bad(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties")) return AS_ERR_HIP;
    if (prop.warpSize != 64) {
        as_set_error("device %d has wavefront size %d; the kernels are written for wave64", device, prop.warpSize);
        return AS_ERR_ARG;
    }
    as_ctx *c = new (std::nothrow) as_ctx();
    if (!c) { as_set_error("as_ctx_create: out of host memory"); return AS_ERR_HIP; }
    c->device = device;
    c->n_cu = prop.multiProcessorCount;
    // fixed-size scratch of the loss partials and the loop's totals
    if (bad(devbuf_ensure(c->tr[TR_PART], l1_partials_bytes()), "as_ctx_create: scratch") ||
        bad(devbuf_ensure(c->tr[TR_TOT], 16), "as_ctx_create: scratch")) {
        as_ctx_destroy(c);
        return AS_ERR_HIP;
    }
    // the static scratch of as_accumulate_error_stats_noalloc: its address on this device
    if (bad(errstats_noalloc_init(device), "as_ctx_create: static scratch address")) {
        as_ctx_destroy(c);
        return AS_ERR_HIP;
    }
    // load every source file's code object now (see AS_WARM_KERNEL)
    warm_api(nullptr);
    warm_binning(nullptr);
    warm_blend(nullptr);
    warm_errstats(nullptr);
    warm_project(nullptr);
    warm_project_bwd(nullptr);
    warm_radix(nullptr);
    warm_split(nullptr);
    warm_train(nullptr);
    if (bad(hipGetLastError(), "as_ctx_create: code-object warm-up") ||
        bad(hipDeviceSynchronize(), "as_ctx_create: code-object warm-up")) {
        as_ctx_destroy(c);
        return AS_ERR_HIP;
    }
    *out = c;
    return AS_OK;
}

void as_ctx_destroy(as_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    for (auto &b : ctx->es) devbuf_free(b);
    for (auto &b : ctx->sp) devbuf_free(b);
    for (auto &b : ctx->dbg) devbuf_free(b);
    for (auto &b : ctx->tr) devbuf_free(b);
    for (int k = 0; k < ctx->n_recs; k++) {
        (void)hipEventDestroy(ctx->recs[k].beg);
        (void)hipEventDestroy(ctx->recs[k].end);
    }
    for (int k = 0; k < ctx->n_pool; k++) (void)hipEventDestroy(ctx->pool[k]);
    free(ctx->recs);
    free(ctx->pool);
    delete ctx;
}

static as_reserve reserve_max(const as_reserve &a, const as_reserve &b) {
    as_reserve r;
    r.max_pixels = a.max_pixels > b.max_pixels ? a.max_pixels : b.max_pixels;
    r.max_gaussians = a.max_gaussians > b.max_gaussians ? a.max_gaussians : b.max_gaussians;
    r.max_candidates = a.max_candidates > b.max_candidates ? a.max_candidates : b.max_candidates;
    r.max_regions = a.max_regions > b.max_regions ? a.max_regions : b.max_regions;
    r.max_views = a.max_views > b.max_views ? a.max_views : b.max_views;
    return r;
}

static bool reserve_ok(const as_reserve *r, const char *what) {
    if (!r || r->max_pixels < 0 || r->max_pixels > 0x7FFFFFFFll || r->max_gaussians < 0 ||
        r->max_gaussians > 0xFFFFFFFFll || r->max_candidates < 0 || r->max_candidates > 0xFFFFFFFFll ||
        r->max_regions < 0 || r->max_regions > 0xFFFFFFFFll || r->max_views < 0 || r->max_views > 65536) {
        as_set_error("%s: reservation out of range", what);
        return false;
    }
    return true;
}

static size_t loop_reserve_bytes(int64_t n) {
    if (n <= 0) return 0;
    size_t need[8], total = 0;
    tr_need(n, need);
    for (int k = 0; k < 8; k++)
        if (need[k]) total += devbuf_size(need[k]);
    return total;
}

as_status as_ctx_reserve(as_ctx *ctx, const as_reserve *r) {
    if (!ctx) { as_set_error("as_ctx_reserve: null context"); return AS_ERR_ARG; }
    if (!reserve_ok(r, "as_ctx_reserve")) return AS_ERR_ARG;
    if (g_capturing) { as_set_error("as_ctx_reserve: allocates, so not inside a graph capture"); return AS_ERR_STATE; }
    if (bad(hipSetDevice(ctx->device), "hipSetDevice")) return AS_ERR_HIP;
    const as_reserve nr = reserve_max(ctx->res, *r);
    hipError_t e = errstats_reserve(ctx, nr.max_pixels);
    if (e == hipSuccess) e = split_reserve(ctx, nr);
    if (e == hipSuccess && nr.max_gaussians > 0) {
        size_t need[8];
        tr_need(nr.max_gaussians, need);
        for (int k = 0; k < 8 && e == hipSuccess; k++)
            if (need[k]) e = devbuf_ensure(ctx->tr[k], need[k]);
    }
    if (e != hipSuccess) {
        as_set_error("as_ctx_reserve: allocation failed: %s", hipGetErrorString(e));
        (void)hipGetLastError();
        return AS_ERR_HIP;
    }
    ctx->res = nr;
    return AS_OK;
}

as_status as_ctx_get_reserve(const as_ctx *ctx, as_reserve *r) {
    if (!ctx || !r) { as_set_error("as_ctx_get_reserve: null argument"); return AS_ERR_ARG; }
    *r = ctx->res;
    return AS_OK;
}

as_status as_ctx_reserve_bytes(const as_reserve *r, size_t *bytes) {
    if (!bytes) { as_set_error("as_ctx_reserve_bytes: null argument"); return AS_ERR_ARG; }
    if (!reserve_ok(r, "as_ctx_reserve_bytes")) return AS_ERR_ARG;
    *bytes = errstats_reserve_bytes(r->max_pixels) + split_reserve_bytes(*r) + loop_reserve_bytes(r->max_gaussians);
    return AS_OK;
}

void as_frame_destroy(as_frame *f) {
    if (!f) return;
    (void)hipSetDevice(f->device);
    frame_free_buffers(f, false);
    delete f;
}

static bool frame_caps_ok(int32_t max_views, int64_t ent_cap, int64_t pix_cap, int64_t tile_cap, int64_t key_cap,
                          uint32_t flags, const char *what) {
    if (max_views < 1 || max_views > AS_MAX_VIEWS || ent_cap < 1 || ent_cap > 0xFFFFFFFFll || pix_cap < 1 ||
        pix_cap > 0x7FFFFFFFll || tile_cap < 1 || tile_cap > 0x7FFFFFFFll || key_cap < 1 || key_cap > 0xFFFFFFFFll ||
        (flags & ~(uint32_t)AS_FRAME_FORWARD_ONLY)) {
        as_set_error("%s: size out of range (views %d, entries %lld, pixels %lld, tiles %lld, keys %lld, flags 0x%x)",
                     what, max_views, (long long)ent_cap, (long long)pix_cap, (long long)tile_cap, (long long)key_cap,
                     flags);
        return false;
    }
    return true;
}

static void frame_set_caps(as_frame *f, int32_t max_views, int64_t ent_cap, int64_t pix_cap, int64_t tile_cap,
                           int64_t key_cap, uint32_t flags) {
    f->max_views = max_views;
    f->ent_cap = ent_cap;
    f->pix_cap = pix_cap;
    f->tile_cap = tile_cap;
    f->key_cap = key_cap;
    f->flags = flags;
}

static size_t frame_bytes(int32_t max_views, int64_t ent_cap, int64_t pix_cap, int64_t tile_cap, int64_t key_cap,
                          uint32_t flags) {
    as_frame f;
    frame_set_caps(&f, max_views, ent_cap, pix_cap, tile_cap, key_cap, flags);
    size_t total = 0;
    frame_buffers(&f, false, [&](void **, size_t bytes) { total += bytes; });
    return total;
}

static as_status frame_alloc(as_ctx *ctx, int32_t max_views, int64_t ent_cap, int64_t pix_cap, int64_t tile_cap,
                             int64_t key_cap, uint32_t flags, int32_t fixed_w, int32_t fixed_h, as_frame **out) {
    if (bad(hipSetDevice(ctx->device), "hipSetDevice")) return AS_ERR_HIP;
    if (g_capturing) { as_set_error("as_frame_create: allocates, so not inside a graph capture"); return AS_ERR_STATE; }
    as_frame *f = new (std::nothrow) as_frame();
    if (!f) { as_set_error("as_frame_create: out of host memory"); return AS_ERR_HIP; }
    f->ctx = ctx;
    f->device = ctx->device;
    f->fixed_w = fixed_w;
    f->fixed_h = fixed_h;
    frame_set_caps(f, max_views, ent_cap, pix_cap, tile_cap, key_cap, flags);
    const hipError_t e = frame_alloc_buffers(f, false);
    if (e != hipSuccess) {
        as_set_error("as_frame_create: allocation failed: %s", hipGetErrorString(e));
        (void)hipGetLastError();
        as_frame_destroy(f);
        return AS_ERR_HIP;
    }
    *out = f;
    return AS_OK;
}

as_status as_frame_create(as_ctx *ctx, int64_t n_cap, int32_t width, int32_t height, int64_t key_cap,
                          uint32_t flags, as_frame **out) {
    if (!ctx || !out) { as_set_error("as_frame_create: null argument"); return AS_ERR_ARG; }
    *out = nullptr;
    if (width < 1 || height < 1 || width > 32767 || height > 32767) {
        as_set_error("as_frame_create: size %dx%d out of range", width, height);
        return AS_ERR_ARG;
    }
    const int64_t tiles = (int64_t)((width + AS_TILE_W - 1) / AS_TILE_W) * ((height + AS_TILE_H - 1) / AS_TILE_H);
    if (!frame_caps_ok(1, n_cap, (int64_t)width * height, tiles, key_cap, flags, "as_frame_create")) return AS_ERR_ARG;
    return frame_alloc(ctx, 1, n_cap, (int64_t)width * height, tiles, key_cap, flags, width, height, out);
}

as_status as_frame_create_batch(as_ctx *ctx, int32_t max_views, int64_t entry_cap, int64_t pixel_cap,
                                int64_t tile_cap, int64_t key_cap, uint32_t flags, as_frame **out) {
    if (!ctx || !out) { as_set_error("as_frame_create_batch: null argument"); return AS_ERR_ARG; }
    *out = nullptr;
    if (!frame_caps_ok(max_views, entry_cap, pixel_cap, tile_cap, key_cap, flags, "as_frame_create_batch"))
        return AS_ERR_ARG;
    return frame_alloc(ctx, max_views, entry_cap, pixel_cap, tile_cap, key_cap, flags, 0, 0, out);
}

as_status as_frame_reserve_keys(as_frame *f, int64_t key_cap) {
    if (!f) { as_set_error("as_frame_reserve_keys: null frame"); return AS_ERR_ARG; }
    if (key_cap < 1 || key_cap > 0xFFFFFFFFll) {
        as_set_error("as_frame_reserve_keys: key_cap %lld out of range", (long long)key_cap);
        return AS_ERR_ARG;
    }
    if (key_cap <= f->key_cap) return AS_OK;
    if (g_capturing) { as_set_error("as_frame_reserve_keys: allocates, so not inside a graph capture"); return AS_ERR_STATE; }
    if (bad(hipSetDevice(f->device), "hipSetDevice")) return AS_ERR_HIP;
    // the pair buffers hold no state between renders: the next render rewrites them
    if (bad(hipDeviceSynchronize(), "as_frame_reserve_keys: synchronise")) return AS_ERR_HIP;
    frame_free_buffers(f, true);
    f->key_cap = key_cap;
    f->has_render = 0;
    const hipError_t e = frame_alloc_buffers(f, true);
    if (e != hipSuccess) {
        as_set_error("as_frame_reserve_keys: allocation failed: %s", hipGetErrorString(e));
        (void)hipGetLastError();
        frame_free_buffers(f, true);
        f->key_cap = 0;
        return AS_ERR_HIP;
    }
    return AS_OK;
}

as_status as_frame_bytes(int32_t max_views, int64_t entry_cap, int64_t pixel_cap, int64_t tile_cap, int64_t key_cap,
                         uint32_t flags, size_t *bytes) {
    if (!bytes) { as_set_error("as_frame_bytes: null argument"); return AS_ERR_ARG; }
    if (!frame_caps_ok(max_views, entry_cap, pixel_cap, tile_cap, key_cap, flags, "as_frame_bytes")) return AS_ERR_ARG;
    *bytes = frame_bytes(max_views, entry_cap, pixel_cap, tile_cap, key_cap, flags);
    return AS_OK;
}

as_status as_workspace_size(const as_ctx *ctx, int64_t n, const as_camera *cams, int32_t n_cams, int64_t key_cap,
                            uint32_t flags, size_t *bytes) {
    if (!ctx || !cams || !bytes || n < 1 || n_cams < 1 || n_cams > AS_MAX_VIEWS) {
        as_set_error("as_workspace_size: bad argument");
        return AS_ERR_ARG;
    }
    int64_t pix = 0, tiles = 0;
    for (int v = 0; v < n_cams; v++) {
        const int64_t W = cams[v].width, H = cams[v].height;
        if (W < 1 || H < 1 || W > 32767 || H > 32767) { as_set_error("as_workspace_size: view %d size", v); return AS_ERR_ARG; }
        pix += W * H;
        tiles += ((W + AS_TILE_W - 1) / AS_TILE_W) * ((H + AS_TILE_H - 1) / AS_TILE_H);
    }
    return as_frame_bytes(n_cams, n * n_cams, pix, tiles, key_cap, flags, bytes);
}

as_status as_frame_get_view_of(const as_frame *f, int32_t view, as_frame_view *v) {
    if (!f || !v) { as_set_error("as_frame_get_view: null argument"); return AS_ERR_ARG; }
    const ViewTable &vt = f->vt;
    if (!(view == 0 && !f->has_render) && (view < 0 || view >= vt.n_views)) {
        as_set_error("as_frame_get_view: view %d not in the last render", view);
        return AS_ERR_ARG;
    }
    const bool have = f->has_render && view < vt.n_views;
    const int W = have ? vt.cam[view].W : f->fixed_w, H = have ? vt.cam[view].H : f->fixed_h;
    const int64_t pb = have ? vt.pix_base[view] : 0;
    const uint32_t eb = have ? vt.ent_base[view] : 0;
    const int32_t tb = have ? vt.tile_base[view] : 0;
    v->width = W; v->height = H; v->tile_w = AS_TILE_W; v->tile_h = AS_TILE_H;
    v->tiles_x = (W + AS_TILE_W - 1) / AS_TILE_W;
    v->tiles_y = (H + AS_TILE_H - 1) / AS_TILE_H;
    v->n_cap = have ? (int64_t)(vt.ent_base[view + 1] - eb) : f->ent_cap;
    v->key_cap = f->key_cap;
    v->tile_base = tb;
    v->ent_base = eb;
    v->n_keys = f->n_keys;
    v->keys = f->keys[f->sorted_sel];
    v->vals = f->vals[f->sorted_sel];
    v->ranges = f->ranges + 2 * (int64_t)tb;
    v->depth_key = f->depth_key + eb;
    v->box = f->box + 4 * (int64_t)eb;
    v->ntiles = f->ntiles + eb;
    v->rec = reinterpret_cast<float *>(f->rec + eb);
    v->t_final = f->t_final + pb; v->last = f->last + pb; v->n_contrib = f->n_contrib + pb; v->dom = f->dom + pb;
    v->err = f->err + pb;
    v->err_minmax = f->err_minmax + 2 * (have ? view : 0);
    v->grad2d = f->grad2d + 9 * eb;
    v->grad2d_stride = 9;
    v->bin_size = have ? 1 << vt.bin_shift : AS_TILE_W;
    v->bin_base = have ? vt.bin_base[view] : 0;
    v->bins_x = (W + v->bin_size - 1) / v->bin_size;
    v->bins_y = (H + v->bin_size - 1) / v->bin_size;
    return AS_OK;
}

as_status as_frame_get_view(const as_frame *f, as_frame_view *v) { return as_frame_get_view_of(f, 0, v); }

as_status as_frame_pair_count(const as_frame *f, uint32_t *dst, void *stream) {
    if (!f || !dst) { as_set_error("as_frame_pair_count: null argument"); return AS_ERR_ARG; }
    launch_copy_u32(f->n_keys, dst, 1, (hipStream_t)stream);
    return launch_status("as_frame_pair_count");
}

static bool capturing(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return false;
    return cs == hipStreamCaptureStatusActive;
}

as_status as_render_batch(as_ctx *ctx, const as_gaussians *scenes, const as_camera *cams, int32_t n_views,
                          as_frame *f, const float *const *gt, float *const *images, void *stream) {
    if (!ctx || !scenes || !cams || !f || !images) { as_set_error("as_render: null argument"); return AS_ERR_ARG; }
    if (n_views < 1 || n_views > f->max_views) {
        as_set_error("as_render: %d views for a frame of at most %d", n_views, f->max_views);
        return AS_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    ViewTable vt;
    memset(&vt, 0, sizeof(vt));
    SceneTable sc;
    memset(&sc, 0, sizeof(sc));
    ViewImages im;
    ViewImagesC gi;
    memset(&im, 0, sizeof(im));
    memset(&gi, 0, sizeof(gi));
    vt.n_views = n_views;
    vt.bin_shift = ctx->bin_tile == 32 ? 5 : 4;
    int64_t ents = 0, pix = 0, tiles = 0, bins = 0, max_n = 0;
    const int deg = scenes[0].sh_degree;
    for (int v = 0; v < n_views; v++) {
        const as_gaussians *g = &scenes[v];
        const as_camera *c = &cams[v];
        if (!check_gauss(g, "as_render") || !host_count_only(g, "as_render")) return AS_ERR_ARG;
        if (g->sh_degree != deg) { as_set_error("as_render: views mix SH degrees %d and %d", deg, g->sh_degree); return AS_ERR_ARG; }
        if (!images[v] || (gt && !gt[v])) { as_set_error("as_render: null image or target of view %d", v); return AS_ERR_ARG; }
        if (c->width < 1 || c->height < 1 || c->width > 32767 || c->height > 32767) {
            as_set_error("as_render: view %d size %dx%d out of range", v, c->width, c->height);
            return AS_ERR_ARG;
        }
        if (f->fixed_w && (c->width != f->fixed_w || c->height != f->fixed_h)) {
            as_set_error("as_render: camera %dx%d does not match the frame %dx%d", c->width, c->height, f->fixed_w,
                         f->fixed_h);
            return AS_ERR_ARG;
        }
        if (!(c->fx > 0.f) || !(c->fy > 0.f)) { as_set_error("as_render: focal lengths must be positive"); return AS_ERR_ARG; }
        const int tx = (c->width + AS_TILE_W - 1) / AS_TILE_W, ty = (c->height + AS_TILE_H - 1) / AS_TILE_H;
        vt.tile_base[v] = (int32_t)tiles;
        vt.tiles_x[v] = tx;
        const int bt = 1 << vt.bin_shift;
        const int bx = (c->width + bt - 1) / bt, by = (c->height + bt - 1) / bt;
        vt.bin_base[v] = (int32_t)bins;
        vt.bins_x[v] = bx;
        bins += (int64_t)bx * by;
        vt.ent_base[v] = (uint32_t)ents;
        vt.pix_base[v] = pix;
        vt.cam[v] = to_devcam(*c);
        sc.g[v] = gptrs(g);
        im.p[v] = images[v];
        gi.p[v] = gt ? gt[v] : nullptr;
        ents += g->n;
        pix += (int64_t)c->width * c->height;
        tiles += (int64_t)tx * ty;
        if (g->n > max_n) max_n = g->n;
        if (ents > f->ent_cap || pix > f->pix_cap || tiles > f->tile_cap) {
            as_set_error("as_render: the views need %lld entries, %lld pixels, %lld tiles; the frame holds %lld, %lld, "
                         "%lld", (long long)ents, (long long)pix, (long long)tiles, (long long)f->ent_cap,
                         (long long)f->pix_cap, (long long)f->tile_cap);
            return AS_ERR_CAPACITY;
        }
    }
    vt.tile_base[n_views] = (int32_t)tiles;
    vt.bin_base[n_views] = (int32_t)bins;
    vt.ent_base[n_views] = (uint32_t)ents;
    vt.pix_base[n_views] = pix;
    const int64_t n = ents;
    f->has_render = 0;
    {
        StageTimer t(ctx, AS_STAGE_PROJECT, s);
        launch_project(sc, vt, max_n, deg, f->rec, f->depth_key, f->box, f->ntiles, f->dkeys[0], f->dvals[0], f->n_ent,
                       s, ctx->row_addr64 != 0);
    }
    // Depth-first binning: a stable sort of the entries by depth, keys
    // emitted in that order, then a stable sort on the tile ids alone, gives
    // every tile the order of a stable sort of (tile | depth) keys emitted by id.
    const uint32_t *order;
    {
        StageTimer t(ctx, AS_STAGE_SORT, s);
        // 32-bit keys: 8-bit digits give the fewest passes (four); the last
        // pass also gathers each entry's tile count into depth order
        const int dsel = radix_sort_u32(f->dkeys, f->dvals, f->n_ent, f->ent_cap, n, 0, 32, 8,
                                        f->dsort_hist.p, s, f->ntiles, f->nt_sorted, ctx->single_pass_sort & 1);
        order = f->dvals[dsel];
    }
    {
        StageTimer t(ctx, AS_STAGE_SCAN, s);
        scan_u32(f->nt_sorted, f->offsets, n, f->n_keys, f->scan_tmp.p, s);
    }
    // the pair count stays on the device: the emission writes the pairs that
    // fit (*n_keys keeps the demand for the caller's capacity check) and the
    // pair sort's grid is sized by the capacity
    const int64_t n_hint = f->key_cap;
    {
        StageTimer t(ctx, AS_STAGE_EMIT, s);
        launch_emit_sorted(n, order, vt, f->box, f->nt_sorted, f->offsets, f->key_cap, f->keys[0], f->vals[0],
                           f->n_keys + 1, f->ranges, tiles, s);
    }
    int sel;
    {
        StageTimer t(ctx, AS_STAGE_SORT, s);
        // only the pairs written (a render over the capacity writes a prefix)
        sel = radix_sort_u32(f->keys, f->vals, f->n_keys + 1, f->key_cap, n_hint, 0, tile_bits(bins),
                             ctx->radix_bits, f->sort_hist.p, s, nullptr, nullptr, (ctx->single_pass_sort & 2) != 0);
    }
    f->sorted_sel = sel;
    {
        StageTimer t(ctx, AS_STAGE_RANGES, s);
        launch_ranges(f->keys[sel], f->n_keys + 1, f->key_cap, bins, vt, f->ranges, s);
        f->use_order = ctx->longest_first;
        if (f->use_order) launch_tile_order(f->ranges, vt, f->tile_order, s);
    }
    const BlendLaunch bl{ctx->lds_batch, ctx->persistent, ctx->n_cu, ctx->block_cull};
    {
        StageTimer t(ctx, AS_STAGE_BLEND_FWD, s);
        f->ck_written = f->ckpt != nullptr;
        f->bm_written = f->bmask != nullptr;
        f->ck_seg = blend_fwd_batch(bl);
        // frames that can take a reverse pass have the forward clear the 2D
        // gradient rows it will add into
        const bool zg = !(f->flags & AS_FRAME_FORWARD_ONLY);
        f->g2d_zero = launch_blend_fwd(f, f->vals[sel], f->use_order ? f->tile_order : nullptr, bl, vt, gi, im, s,
                                       zg ? f->grad2d : nullptr, 9 * n) && zg;
        f->g2d_zero_capture = g_capture_id;
        // the reverse pass's cost per tile follows its contributors, which only
        // the forward pass knows: order the reverse dispatch by them
        launch_after_fwd(f, vt, gi, f->use_order, s);
    }
    const as_status st = launch_status("as_render");
    if (st != AS_OK) return st;
    f->has_render = 1;
    f->vt = vt;
    f->scenes = sc;
    f->has_gt = gt != nullptr;
    f->persistent_last = ctx->persistent;
    return AS_OK;
}

as_status as_render(as_ctx *ctx, const as_gaussians *g, const as_camera *cam, as_frame *f, const float *gt,
                    float *image, void *stream) {
    if (!ctx || !g || !cam || !f || !image) { as_set_error("as_render: null argument"); return AS_ERR_ARG; }
    if (!f->fixed_w) { as_set_error("as_render: a batch frame takes as_render_batch"); return AS_ERR_ARG; }
    const float *gts[1] = {gt};
    float *ims[1] = {image};
    return as_render_batch(ctx, g, cam, 1, f, gt ? gts : nullptr, ims, stream);
}

static bool same_set(const GaussPtrs &a, const as_gaussians *g) {
    return a.means == g->means && a.log_scales == g->log_scales && a.quats == g->quats &&
           a.opac == g->opacity_logits && a.sh == g->sh && a.n == g->n && a.deg == g->sh_degree;
}

as_status as_render_backward_batch(as_ctx *ctx, const as_gaussians *g, as_frame *f, const float *const *dL_dimages,
                                   as_gaussians_mut *grads, float *g2d_norm, int32_t *vis_count, void *stream) {
    if (!ctx || !f || !dL_dimages) { as_set_error("as_render_backward: null argument"); return AS_ERR_ARG; }
    if (!check_gauss(g, "as_render_backward") || !host_count_only(g, "as_render_backward")) return AS_ERR_ARG;
    if (!f->has_render) { as_set_error("as_render_backward: the frame holds no render"); return AS_ERR_STATE; }
    const ViewTable &vt = f->vt;
    for (int v = 0; v < vt.n_views; v++) {
        if (!same_set(f->scenes.g[v], g)) {
            as_set_error("as_render_backward: view %d of the last render used another Gaussian set", v);
            return AS_ERR_STATE;
        }
        if (!dL_dimages[v]) { as_set_error("as_render_backward: null gradient image of view %d", v); return AS_ERR_ARG; }
    }
    if (!check_mut(grads, g->n, g->sh_degree, "as_render_backward")) return AS_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    ViewImagesC dl;
    memset(&dl, 0, sizeof(dl));
    for (int v = 0; v < vt.n_views; v++) dl.p[v] = dL_dimages[v];
    const int64_t ents = vt.ent_base[vt.n_views];
    const BlendLaunch bl{ctx->lds_batch, ctx->persistent, ctx->n_cu, ctx->block_cull};
    // Frames hold their checkpoint buffer from creation (unless created
    // forward-only): renders write checkpoints at the forward's batch
    // boundaries and this pass splits long tile lists at them.
    {
        StageTimer t(ctx, AS_STAGE_BLEND_BWD, s);
        // The render's forward cleared the rows, unless this is a second
        // reverse pass of one render, or the render was not recorded in the
        // graph being captured now (or was, and this pass runs eagerly): then
        // the pass clears them itself.
        if (!f->g2d_zero || f->g2d_zero_capture != g_capture_id)
            launch_fill_u32(reinterpret_cast<uint32_t *>(f->grad2d), 0u, 9 * ents, s);
        f->g2d_zero = 0;
        launch_blend_bwd(f, f->vals[f->sorted_sel], f->use_order ? f->tile_order_bwd : nullptr, bl, vt, dl,
                         f->grad2d, s);
    }
    {
        StageTimer t(ctx, AS_STAGE_PROJECT_BWD, s);
        launch_project_bwd(gptrs(g), vt, f->ntiles, f->grad2d, mptrs(grads), g2d_norm, vis_count, s,
                           ctx->row_addr64 != 0);
    }
    return launch_status("as_render_backward");
}

as_status as_render_backward(as_ctx *ctx, const as_gaussians *g, const as_camera *cam, as_frame *f,
                             const float *dL_dimage, as_gaussians_mut *grads, float *g2d_norm, int32_t *vis_count,
                             void *stream) {
    if (!ctx || !cam || !f || !dL_dimage) { as_set_error("as_render_backward: null argument"); return AS_ERR_ARG; }
    if (f->has_render && f->vt.n_views == 1 &&
        (cam->width != f->vt.cam[0].W || cam->height != f->vt.cam[0].H)) {
        as_set_error("as_render_backward: camera/frame size mismatch");
        return AS_ERR_ARG;
    }
    if (f->has_render && f->vt.n_views != 1) {
        as_set_error("as_render_backward: the last render had %d views; use as_render_backward_batch", f->vt.n_views);
        return AS_ERR_STATE;
    }
    const float *dl[1] = {dL_dimage};
    return as_render_backward_batch(ctx, g, f, dl, grads, g2d_norm, vis_count, stream);
}

as_status as_error_map(as_ctx *ctx, int32_t width, int32_t height, const float *image, const float *gt, double *err,
                       uint64_t *err_minmax, void *stream) {
    if (!ctx || !image || !gt || !err || !err_minmax || width < 1 || height < 1) {
        as_set_error("as_error_map: bad argument");
        return AS_ERR_ARG;
    }
    {
        StageTimer t(ctx, AS_STAGE_ERROR_MAP, (hipStream_t)stream);
        launch_error_map(width, height, image, gt, err, err_minmax, (hipStream_t)stream);
    }
    return launch_status("as_error_map");
}

// ---- optimisation loop ----------------------------------------------------------

// The loop's calls over n Gaussians use the reserved slots of ctx->tr.
static bool loop_reserved(const as_ctx *ctx, int64_t n, const char *what) {
    if (n == 0 || n <= ctx->res.max_gaussians) return true;
    as_set_error("%s: %lld Gaussians need max_gaussians >= %lld in as_ctx_reserve (reserved %lld)", what, (long long)n,
                 (long long)n, (long long)ctx->res.max_gaussians);
    return false;
}

static bool same_shape(const as_gaussians_mut *a, int64_t n, int32_t deg, const char *what, const char *name) {
    if (!a) { as_set_error("%s: null %s", what, name); return false; }
    if (a->n != n || a->sh_degree != deg) {
        as_set_error("%s: %s has %lld rows, degree %d (expected %lld, %d)", what, name, (long long)a->n, a->sh_degree,
                     (long long)n, deg);
        return false;
    }
    if (n > 0 && (!a->means || !a->log_scales || !a->quats || !a->opacity_logits || !a->sh)) {
        as_set_error("%s: null pointer in %s", what, name);
        return false;
    }
    return true;
}

as_status as_adam_step(as_ctx *ctx, as_gaussians_mut *params, const as_gaussians *grads, as_gaussians_mut *m,
                       as_gaussians_mut *v, const as_adam_params *hp, int32_t step, void *stream) {
    const char *what = "as_adam_step";
    if (!ctx || !params || !hp) { as_set_error("%s: null argument", what); return AS_ERR_ARG; }
    if (step < 1) { as_set_error("%s: step %d < 1", what, step); return AS_ERR_ARG; }
    if (params->sh_degree < 0 || params->sh_degree > 3) { as_set_error("%s: sh_degree %d", what, params->sh_degree); return AS_ERR_ARG; }
    if (!same_shape(params, params->n, params->sh_degree, what, "params") || !check_gauss(grads, what) ||
        !same_shape(m, params->n, params->sh_degree, what, "m") || !same_shape(v, params->n, params->sh_degree, what, "v"))
        return AS_ERR_ARG;
    if (grads->n != params->n || grads->sh_degree != params->sh_degree) {
        as_set_error("%s: grads has %lld rows, degree %d", what, (long long)grads->n, grads->sh_degree);
        return AS_ERR_ARG;
    }
    launch_adam(*params, *grads, *m, *v, *hp, step, (hipStream_t)stream);
    return launch_status(what);
}

as_status as_l1_loss(as_ctx *ctx, int32_t width, int32_t height, const float *image, const float *gt, float *dL_dimage,
                     double *sums, void *stream) {
    const char *what = "as_l1_loss";
    if (!ctx || !image || !gt || !sums || width < 1 || height < 1) { as_set_error("%s: bad argument", what); return AS_ERR_ARG; }
    launch_l1(width, height, image, gt, dL_dimage, sums, (double *)ctx->tr[TR_PART].p, (hipStream_t)stream);
    return launch_status(what);
}

as_status as_densify_select(as_ctx *ctx, const as_gaussians *g, const float *g2d_accum, const int32_t *vis_count,
                            double grad_threshold, double size_threshold, uint8_t *clone_mask, uint8_t *is_candidate,
                            int32_t *cand, int64_t *n_cand, void *stream) {
    const char *what = "as_densify_select";
    if (!ctx) { as_set_error("%s: null context", what); return AS_ERR_ARG; }
    if (!check_gauss(g, what) || !host_count_only(g, what)) return AS_ERR_ARG;
    if (!n_cand || (g->n > 0 && (!g2d_accum || !vis_count || !clone_mask || !is_candidate || !cand))) {
        as_set_error("%s: null argument", what);
        return AS_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = g->n;
    if (!loop_reserved(ctx, n, what)) return AS_ERR_CAPACITY;
    if (n == 0) {
        launch_fill_i64(n_cand, 0, 1, s);
        return launch_status(what);
    }
    launch_select(*g, g2d_accum, vis_count, grad_threshold, size_threshold, clone_mask, is_candidate, s);
    int64_t *scan = (int64_t *)ctx->tr[TR_SCAN].p;
    scan_u8_to_i64(is_candidate, scan, n, n_cand, ctx->tr[TR_TMP].p, s);
    launch_compact_ids(n, is_candidate, scan, cand, s);
    return launch_status(what);
}

as_status as_split_row_map(as_ctx *ctx, int64_t n, const int32_t *cand, int64_t n_cand, const uint8_t *mode,
                           const int32_t *state_in, int32_t *row_src, int64_t capacity, const int64_t *n_dev,
                           const int64_t *n_cand_dev, void *stream) {
    const char *what = "as_split_row_map";
    if (!ctx || n < 0 || n_cand < 0 || capacity < n || (n_cand > 0 && (!cand || !mode)) || (capacity > 0 && !row_src)) {
        as_set_error("%s: bad argument (n %lld, candidates %lld, capacity %lld)", what, (long long)n, (long long)n_cand,
                     (long long)capacity);
        return AS_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t m = n > 0 ? n : 1;
    if (!loop_reserved(ctx, n, what)) return AS_ERR_CAPACITY;
    if (capacity > 0) launch_fill_u32(reinterpret_cast<uint32_t *>(row_src), 0xFFFFFFFFu, capacity, s);
    if (n == 0) return launch_status(what);
    uint8_t *keep = (uint8_t *)ctx->tr[TR_FLAG].p;
    int64_t *pos = (int64_t *)ctx->tr[TR_SCAN].p;
    launch_keep_init(n, n_dev, keep, s);
    launch_mark_kept(cand, n_cand, n_cand_dev, mode, n, keep, s);
    scan_u8_to_i64(keep, pos, n, (int64_t *)ctx->tr[TR_TOT].p, ctx->tr[TR_TMP].p, s);
    launch_row_map(n, keep, pos, state_in, capacity, row_src, s);
    return launch_status(what);
}

as_status as_clone_prune(as_ctx *ctx, const as_gaussians *g, const uint8_t *clone_mask, const int32_t *state_in,
                         double min_opacity, double max_scale, as_gaussians_mut *out, int32_t *state_src,
                         int64_t *n_out, void *stream) {
    const char *what = "as_clone_prune";
    if (!ctx) { as_set_error("%s: null context", what); return AS_ERR_ARG; }
    if (!check_gauss(g, what)) return AS_ERR_ARG;
    if (!out || !state_src || !n_out) { as_set_error("%s: null output", what); return AS_ERR_ARG; }
    const int64_t need = clone_mask ? 2 * g->n : g->n;   // every row may be cloned
    if (out->n < need) {
        as_set_error("%s: output capacity %lld < %lld rows", what, (long long)out->n, (long long)need);
        return AS_ERR_CAPACITY;
    }
    if (!check_mut(out, need, g->sh_degree, what)) return AS_ERR_ARG;
    if (g->n > 0 && (out->means == g->means || out->sh == g->sh)) { as_set_error("%s: output aliases the input", what); return AS_ERR_ARG; }
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = g->n, m = n > 0 ? n : 1;
    if (!loop_reserved(ctx, n, what)) return AS_ERR_CAPACITY;
    int64_t *tot = (int64_t *)ctx->tr[TR_TOT].p;
    if (n == 0) {
        launch_fill_i64(n_out, 0, 1, s);
        return launch_status(what);
    }
    uint8_t *keep = (uint8_t *)ctx->tr[TR_FLAG].p, *dup = (uint8_t *)ctx->tr[TR_DUP].p;
    int64_t *kpos = (int64_t *)ctx->tr[TR_SCAN].p, *dpos = (int64_t *)ctx->tr[TR_DSCAN].p;
    launch_prune_flags(*g, clone_mask, min_opacity, max_scale, keep, dup, s);
    scan_u8_to_i64(keep, kpos, n, tot, ctx->tr[TR_TMP].p, s);
    scan_u8_to_i64(dup, dpos, n, tot + 1, ctx->tr[TR_TMP2].p, s);
    launch_clone_prune_write(*g, *out, keep, dup, kpos, dpos, tot, tot + 1, state_in, state_src, n_out, s);
    return launch_status(what);
}

as_status as_gather_rows(as_ctx *ctx, const as_gaussians *src, const int32_t *map, int64_t n_rows,
                         as_gaussians_mut *dst, const int64_t *n_rows_dev, void *stream) {
    const char *what = "as_gather_rows";
    if (!ctx || n_rows < 0 || !check_gauss(src, what) || (n_rows > 0 && !map)) { as_set_error("%s: bad argument", what); return AS_ERR_ARG; }
    if (!check_mut(dst, n_rows, src->sh_degree, what)) return AS_ERR_ARG;
    launch_gather_rows(*src, map, n_rows, n_rows_dev, *dst, (hipStream_t)stream);
    return launch_status(what);
}

as_status as_reset_opacity(as_ctx *ctx, as_gaussians_mut *g, double max_opacity, float *m_op, float *v_op,
                           void *stream) {
    const char *what = "as_reset_opacity";
    if (!ctx || !g || g->n < 0 || (g->n > 0 && !g->opacity_logits) || !(max_opacity > 0.0 && max_opacity < 1.0)) {
        as_set_error("%s: bad argument", what);
        return AS_ERR_ARG;
    }
    launch_reset_opacity(*g, (float)log(max_opacity / (1.0 - max_opacity)), m_op, v_op, (hipStream_t)stream);
    return launch_status(what);
}

as_status as_accumulate_error_stats(as_ctx *ctx, int32_t width, int32_t height, const double *err,
                                    const uint64_t *err_minmax, const int32_t *dom, const float *gt, int32_t view_id,
                                    int64_t n, const uint8_t *is_candidate, const as_split_params *params,
                                    as_region_buf *regions, int32_t *attr_count, void *stream) {
    if (!ctx || !err || !err_minmax || !dom || !gt || !is_candidate || !regions || !regions->records ||
        !regions->count || !attr_count || width < 1 || height < 1 || n < 1 || view_id < 0) {
        as_set_error("as_accumulate_error_stats: bad argument");
        return AS_ERR_ARG;
    }
    if ((int64_t)width * height > 0x7FFFFFFFll) { as_set_error("as_accumulate_error_stats: image too large"); return AS_ERR_ARG; }
    if (!check_params(params, "as_accumulate_error_stats")) return AS_ERR_ARG;
    as_status st;
    {
        StageTimer t(ctx, AS_STAGE_ERROR_STATS, (hipStream_t)stream);
        st = run_error_stats(ctx, width, height, err, err_minmax, dom, gt, view_id, n, is_candidate, *params, *regions,
                             attr_count, (hipStream_t)stream);
    }
    if (st != AS_OK) return st;
    return launch_status("as_accumulate_error_stats");
}

as_status as_accumulate_error_stats_noalloc(as_ctx *ctx, int32_t width, int32_t height, const double *err,
                                            const uint64_t *err_minmax, const int32_t *dom, const float *gt,
                                            int32_t view_id, int64_t n, const uint8_t *is_candidate,
                                            const as_split_params *params, as_region_buf *regions,
                                            int32_t *attr_count, void *stream) {
    if (!ctx || !err || !err_minmax || !dom || !gt || !is_candidate || !regions || !regions->records ||
        !regions->count || !attr_count || width < 1 || height < 1 || n < 1 || view_id < 0) {
        as_set_error("as_accumulate_error_stats_noalloc: bad argument");
        return AS_ERR_ARG;
    }
    if (!check_params(params, "as_accumulate_error_stats_noalloc")) return AS_ERR_ARG;
    as_status st;
    {
        StageTimer t(ctx, AS_STAGE_ERROR_STATS, (hipStream_t)stream);
        st = run_error_stats_noalloc(ctx, width, height, err, err_minmax, dom, gt, view_id, is_candidate, *params,
                                     *regions, attr_count, (hipStream_t)stream);
    }
    if (st != AS_OK) return st;
    return launch_status("as_accumulate_error_stats_noalloc");
}

as_status as_adaptive_split(as_ctx *ctx, const as_gaussians *g, const int32_t *cand, int64_t n_cand,
                            const as_region_buf *regions, const as_camera *views, int32_t n_views,
                            const int32_t *attr_count, const as_split_params *params, const float *noise,
                            as_gaussians_mut *out, uint8_t *mode, int32_t *count, int64_t *offset, int64_t *n_out,
                            const int64_t *n_cand_dev, void *stream) {
    if (!ctx || !regions || !regions->records || !regions->count || !attr_count || !n_out || n_cand < 0 ||
        n_views < 0 || (n_views > 0 && !views)) {
        as_set_error("as_adaptive_split: bad argument");
        return AS_ERR_ARG;
    }
    if (n_cand > 0 && (!cand || !noise || !mode || !count || !offset)) {
        as_set_error("as_adaptive_split: null per-candidate pointer");
        return AS_ERR_ARG;
    }
    if (!check_gauss(g, "as_adaptive_split") || !check_params(params, "as_adaptive_split")) return AS_ERR_ARG;
    if ((params->noise_n ? params->noise_n : 2) < split_noise_need(*params)) {
        as_set_error("as_adaptive_split: noise_n %d below the %d random children this variant may draw",
                     params->noise_n, split_noise_need(*params));
        return AS_ERR_ARG;
    }
    const int64_t per = split_rows_per_candidate(*params);
    const int64_t bound = g->n + n_cand * per;
    if (!check_mut(out, 0, g->sh_degree, "as_adaptive_split")) return AS_ERR_ARG;
    if (out->n < bound) {
        as_set_error("as_adaptive_split: output capacity %lld below the bound %lld", (long long)out->n, (long long)bound);
        return AS_ERR_CAPACITY;
    }
    for (int v = 0; v < n_views; v++)
        if (!(views[v].fx > 0.f) || !(views[v].fy > 0.f) || views[v].width < 1 || views[v].height < 1) {
            as_set_error("as_adaptive_split: view %d is invalid", v);
            return AS_ERR_ARG;
        }
    as_status st;
    {
        StageTimer t(ctx, AS_STAGE_SPLIT, (hipStream_t)stream);
        st = run_adaptive_split(ctx, gptrs(g), cand, n_cand, n_cand_dev, *regions, views, n_views, attr_count, *params,
                                noise,
                                mptrs(out), out->n, mode, count, offset, n_out, (hipStream_t)stream);
    }
    if (st != AS_OK) return st;
    return launch_status("as_adaptive_split");
}

as_status as_set_tuning(as_ctx *ctx, const as_tuning *t) {
    if (!ctx || !t) { as_set_error("as_set_tuning: null argument"); return AS_ERR_ARG; }
    if (t->lds_batch != 256 && t->lds_batch != 512 && t->lds_batch != 1024) {
        as_set_error("as_set_tuning: lds_batch %d not in {256, 512, 1024}", t->lds_batch);
        return AS_ERR_ARG;
    }
    if (t->radix_bits < 4 || t->radix_bits > 8) {
        as_set_error("as_set_tuning: radix_bits %d not in 4..8", t->radix_bits);
        return AS_ERR_ARG;
    }
    if (t->single_pass_sort < 0 || t->single_pass_sort > 3) {
        as_set_error("as_set_tuning: single_pass_sort %d not in 0..3", t->single_pass_sort);
        return AS_ERR_ARG;
    }
    if (t->bin_tile != 16 && t->bin_tile != 32) {
        as_set_error("as_set_tuning: bin_tile %d not 16 or 32", t->bin_tile);
        return AS_ERR_ARG;
    }
    ctx->lds_batch = t->lds_batch;
    ctx->longest_first = t->longest_first != 0;
    ctx->persistent = t->persistent != 0;
    ctx->radix_bits = t->radix_bits;
    ctx->block_cull = t->block_cull != 0;
    ctx->single_pass_sort = t->single_pass_sort;
    ctx->bin_tile = t->bin_tile;
    return AS_OK;
}

as_status as_get_tuning(const as_ctx *ctx, as_tuning *t) {
    if (!ctx || !t) { as_set_error("as_get_tuning: null argument"); return AS_ERR_ARG; }
    t->lds_batch = ctx->lds_batch;
    t->longest_first = ctx->longest_first;
    t->persistent = ctx->persistent;
    t->radix_bits = ctx->radix_bits;
    t->block_cull = ctx->block_cull;
    t->single_pass_sort = ctx->single_pass_sort;
    t->bin_tile = ctx->bin_tile;
    return AS_OK;
}

as_status as_timing_enable(as_ctx *ctx, int32_t on) {
    if (!ctx) { as_set_error("as_timing_enable: null context"); return AS_ERR_ARG; }
    ctx->timing = on != 0;
    return AS_OK;
}

as_status as_timing_read(as_ctx *ctx, double *ms, int64_t *runs) {
    if (!ctx || !ms || !runs) { as_set_error("as_timing_read: null argument"); return AS_ERR_ARG; }
    for (int k = 0; k < AS_NUM_STAGES; k++) { ms[k] = 0.0; runs[k] = 0; }
    as_status st = AS_OK;
    for (int k = 0; k < ctx->n_recs; k++) {
        StageRec &r = ctx->recs[k];
        float e = 0.f;
        if (st == AS_OK && (bad(hipEventSynchronize(r.end), "as_timing_read") ||
                            bad(hipEventElapsedTime(&e, r.beg, r.end), "as_timing_read")))
            st = AS_ERR_HIP;
        if (st == AS_OK && r.stage >= 0 && r.stage < AS_NUM_STAGES) {
            ms[r.stage] += e;
            runs[r.stage] += 1;
        }
        pool_put(ctx, r.beg);
        pool_put(ctx, r.end);
    }
    ctx->n_recs = 0;
    return st;
}

struct as_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

as_status as_graph_begin(as_ctx *ctx, void *stream) {
    if (!ctx || !stream) { as_set_error("as_graph_begin: needs a context and a non-null stream"); return AS_ERR_ARG; }
    if (g_capturing) { as_set_error("as_graph_begin: a capture is already open on this thread"); return AS_ERR_STATE; }
    if (bad(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal), "as_graph_begin"))
        return AS_ERR_HIP;
    g_capturing = 1;
    g_capture_id = ++g_captures;
    return AS_OK;
}

as_status as_graph_end(as_ctx *ctx, void *stream, as_graph **out) {
    if (!ctx || !stream || !out) { as_set_error("as_graph_end: null argument"); return AS_ERR_ARG; }
    *out = nullptr;
    if (!g_capturing) { as_set_error("as_graph_end: no capture open on this thread"); return AS_ERR_STATE; }
    g_capturing = 0;
    g_capture_id = 0;
    hipGraph_t g = nullptr;
    if (bad(hipStreamEndCapture((hipStream_t)stream, &g), "as_graph_end")) return AS_ERR_HIP;
    as_graph *gr = new (std::nothrow) as_graph();
    if (!gr) {
        (void)hipGraphDestroy(g);
        as_set_error("as_graph_end: out of host memory");
        return AS_ERR_HIP;
    }
    gr->graph = g;
    if (bad(hipGraphInstantiate(&gr->exec, g, nullptr, nullptr, 0), "as_graph_end: instantiate")) {
        (void)hipGraphDestroy(g);
        delete gr;
        return AS_ERR_HIP;
    }
    *out = gr;
    return AS_OK;
}

as_status as_graph_launch(as_graph *graph, void *stream) {
    if (!graph) { as_set_error("as_graph_launch: null graph"); return AS_ERR_ARG; }
    if (bad(hipGraphLaunch(graph->exec, (hipStream_t)stream), "as_graph_launch")) return AS_ERR_HIP;
    return AS_OK;
}

void as_graph_destroy(as_graph *graph) {
    if (!graph) return;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
}

as_status as_debug_sort_pairs(as_ctx *ctx, uint64_t *keys, uint32_t *vals, int64_t n, int32_t key_bits, void *stream) {
    if (!ctx || (n > 0 && (!keys || !vals)) || n < 0 || n > 0xFFFFFFFFll || key_bits < 0 || key_bits > 64) {
        as_set_error("as_debug_sort_pairs: bad argument");
        return AS_ERR_ARG;
    }
    if (n == 0) return AS_OK;
    hipStream_t s = (hipStream_t)stream;
    if (bad(devbuf_ensure(ctx->dbg[0], n * 8), "sort scratch") || bad(devbuf_ensure(ctx->dbg[1], n * 4), "sort scratch") ||
        bad(devbuf_ensure(ctx->dbg[2], sort_hist_bytes(n)), "sort scratch") || bad(devbuf_ensure(ctx->dbg[3], 64), "sort scratch"))
        return AS_ERR_HIP;
    uint64_t *kk[2] = {keys, (uint64_t *)ctx->dbg[0].p};
    uint32_t *vv[2] = {vals, (uint32_t *)ctx->dbg[1].p};
    uint32_t *n_dev = (uint32_t *)ctx->dbg[3].p;
    launch_fill_u32(n_dev, (uint32_t)n, 1, s);
    const int sel = radix_sort_u64(kk, vv, n_dev, n, n, 0, key_bits, ctx->radix_bits, ctx->dbg[2].p, s);
    if (sel == 1) {
        if (bad(hipMemcpyAsync(keys, kk[1], n * 8, hipMemcpyDeviceToDevice, s), "sort copy-back") ||
            bad(hipMemcpyAsync(vals, vv[1], n * 4, hipMemcpyDeviceToDevice, s), "sort copy-back"))
            return AS_ERR_HIP;
    }
    return launch_status("as_debug_sort_pairs");
}

as_status as_debug_sort_u32(as_ctx *ctx, uint32_t *keys, uint32_t *vals, int64_t n, int32_t lo_bit, int32_t hi_bit,
                            int32_t radix_bits, int32_t single_pass, const uint32_t *gather_src, uint32_t *gather_dst,
                            void *stream) {
    if (!ctx || n < 0 || n > 0x3FFFFFFEll || (n > 0 && (!keys || !vals)) || lo_bit < 0 || hi_bit > 32 ||
        lo_bit > hi_bit || radix_bits < 4 || radix_bits > 8 || (!gather_src) != (!gather_dst)) {
        as_set_error("as_debug_sort_u32: bad argument");
        return AS_ERR_ARG;
    }
    if (n == 0 || hi_bit == lo_bit) return AS_OK;
    hipStream_t s = (hipStream_t)stream;
    if (bad(devbuf_ensure(ctx->dbg[4], n * 4), "sort scratch") || bad(devbuf_ensure(ctx->dbg[5], n * 4), "sort scratch") ||
        bad(devbuf_ensure(ctx->dbg[2], sort_hist_bytes(n)), "sort scratch") || bad(devbuf_ensure(ctx->dbg[3], 64), "sort scratch"))
        return AS_ERR_HIP;
    uint32_t *kk[2] = {keys, (uint32_t *)ctx->dbg[4].p};
    uint32_t *vv[2] = {vals, (uint32_t *)ctx->dbg[5].p};
    uint32_t *n_dev = (uint32_t *)ctx->dbg[3].p;
    launch_fill_u32(n_dev, (uint32_t)n, 1, s);
    uint32_t *flag = (uint32_t *)((char *)ctx->dbg[2].p + sort_wait_flag_offset());
    launch_fill_u32(flag, 0u, 1, s);
    const int sel = radix_sort_u32(kk, vv, n_dev, n, n, lo_bit, hi_bit, radix_bits, ctx->dbg[2].p, s, gather_src,
                                   gather_dst, single_pass != 0);
    if (sel == 1) {
        if (bad(hipMemcpyAsync(keys, kk[1], n * 4, hipMemcpyDeviceToDevice, s), "sort copy-back") ||
            bad(hipMemcpyAsync(vals, vv[1], n * 4, hipMemcpyDeviceToDevice, s), "sort copy-back"))
            return AS_ERR_HIP;
    }
    if (single_pass) {
        uint32_t hflag = 0;
        if (bad(hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s), "sort flag") ||
            bad(hipStreamSynchronize(s), "sort flag"))
            return AS_ERR_HIP;
        if (hflag) {
            as_set_error("as_debug_sort_u32: a look-back wait hit its limit");
            return AS_ERR_HIP;
        }
    }
    return launch_status("as_debug_sort_u32");
}

as_status as_debug_fp64_ops(as_ctx *ctx, const double *a, const double *b, int64_t n, double *out, void *stream) {
    if (!ctx || n < 0 || (n > 0 && (!a || !b || !out))) { as_set_error("as_debug_fp64_ops: bad argument"); return AS_ERR_ARG; }
    launch_fp64_ops(a, b, n, out, (hipStream_t)stream);
    return launch_status("as_debug_fp64_ops");
}

as_status as_debug_row_addressing(as_ctx *ctx, int32_t force_64bit) {
    if (!ctx) { as_set_error("as_debug_row_addressing: null context"); return AS_ERR_ARG; }
    ctx->row_addr64 = force_64bit != 0;
    return AS_OK;
}

as_status as_debug_blend_alpha(const as_frame *f, int32_t view, int64_t n, const int32_t *pix,
                               const uint32_t *gauss, float *out, void *stream) {
    if (!f || n < 0 || (n > 0 && (!pix || !gauss || !out))) {
        as_set_error("as_debug_blend_alpha: bad argument");
        return AS_ERR_ARG;
    }
    if (!f->has_render || view < 0 || view >= f->vt.n_views) {
        as_set_error("as_debug_blend_alpha: view %d not in the last render", view);
        return AS_ERR_STATE;
    }
    if (f->vt.ent_base[view] != 0) {
        as_set_error("as_debug_blend_alpha: only the first view's entries are addressed by Gaussian id");
        return AS_ERR_ARG;
    }
    launch_debug_alpha(f, n, pix, gauss, out, (hipStream_t)stream);
    return launch_status("as_debug_blend_alpha");
}

}  // extern "C"

AS_WARM_KERNEL(api)
