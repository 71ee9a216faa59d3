// Per-tile front-to-back alpha blending (Eq. (rendering), Sec. 3) with the
// dominant Gaussian map (Eq. (dominant-map), Sec. 4.1) and the per-pixel L1
// error of Eq. (l1map) fused into the same traversal, and the matching reverse
// pass.
//
// Work decomposition (gfx950, wave64): one 16x16 tile per 256-thread block;
// the tile is cut into sixteen 4x4 pixel blocks and each 16-lane row of a
// wave owns one of them.  Gaussian records are staged through LDS in batches
// of BATCH records (the tunable "LDS depth"; each thread fetches BATCH/256
// records one batch ahead, so the gather latency overlaps the previous batch's
// blending).  A staged record carries the Gaussian's pixel box as two 16-bit
// masks over the tile's columns and rows.  After staging, every row compacts
// the indices of the records whose box meets its 4x4 block (ballots), so a
// wave advances four rows through four different Gaussians per instruction,
// and a pixel outside a box never composites it: the contributor set is
// exactly {box holds the pixel, alpha >= 1/255}.  A block stops fetching once
// all 256 pixels have saturated.
//
// One launch covers every tile of every view of a batch (global tile ids;
// each view's size, camera, pixel and entry ranges come from the view table).
// Tiles are visited in a given order (longest list first) and either one
// block per tile, or by a persistent grid sized to the resident capacity of
// the device whose blocks pull tile after tile from a global atomic queue.
//
// Alpha is evaluated as exp2(q) with q = a' dx^2 + b' dx dy + c' dy^2 + log2(o)
// (conic pre-scaled by -log2(e)/2, opacity folded into the exponent); the
// forward and the reverse pass share the staged values and the helper below,
// so they take identical alpha decisions.
#include <type_traits>

#include "internal.h"

namespace {

constexpr float ALPHA_MIN = 1.0f / 255.0f;
constexpr float ALPHA_MAX = 0.99f;
constexpr float T_STOP = 1e-4f;
constexpr float LOG2E = 1.4426950408889634f;
constexpr float LN2 = 0.6931471805599453f;

// A staged record: 48 bytes, read by the hit loops as three 16-byte LDS loads
// issued together.
struct StagedRec {
    float4 mc;  // mean x, mean y (tile-relative), a', b'
    float4 cc;  // c', log2(o), r, g
    float4 ex;  // b, box masks (bits), entry id (bits), 0
};

// q = a' dx^2 + b' dx dy + c' dy^2 + log2(o) as (a' dx + b' dy) dx + (c' dy dy
// + log2(o)): two multiplies and three fused multiply-adds.
__device__ __forceinline__ float blend_exponent(float dx, float dy, const float4 &mc, const float4 &cc) {
#pragma clang fp contract(off)
    return __fmaf_rn(__fmaf_rn(mc.z, dx, mc.w * dy), dx, __fmaf_rn(cc.x * dy, dy, cc.y));
}

__device__ __forceinline__ uint32_t span_mask(int lo, int hi) {   // bits lo..hi of 16, clamped
    lo = lo < 0 ? 0 : lo;
    hi = hi > 15 ? 15 : hi;
    if (hi < lo) return 0u;
    return ((2u << hi) - 1u) & ~((1u << lo) - 1u);
}

// Index type of the per-row hit lists: one byte covers a batch of 256.
template <int BATCH>
using HitT = typename std::conditional<(BATCH <= 256), uint8_t, uint16_t>::type;

// Registers of one record fetched ahead of its batch.
struct Fetched {
    BlendRec r;
    short4 b;
    uint32_t id;
    bool live;   // the record may touch the tile: only then are its box and blend record staged
};

__device__ __forceinline__ bool box_meets_tile(short4 b, int ox, int oy) {
    return b.x < ox + AS_TILE_W && b.z >= ox && b.y < oy + AS_TILE_H && b.w >= oy;
}

// Forward: the pixel box decides whether the 48-byte blend record is loaded
// (a list of a bin of 32 also holds the records of the bin's other tiles).
__device__ __forceinline__ void fetch(const uint32_t *__restrict__ vals, const BlendRec *__restrict__ rec,
                                      const short4 *__restrict__ box, uint32_t idx, int ox, int oy, Fetched &f) {
    f.id = vals[idx];
    f.b = box[f.id];
    f.live = box_meets_tile(f.b, ox, oy);
    if (f.live) f.r = rec[f.id];
}

// Reverse: the forward's block mask for this tile decides when it is stored
// (zero: no block can hold a contributor), else the pixel box.  `force`
// loads the record whatever they say: the first slot of every batch is
// always staged, because the lanes of a row past its own hits evaluate slot
// 0 and multiply its values by zero, which must stay finite.
__device__ __forceinline__ void fetch_masked(const uint32_t *__restrict__ vals, const BlendRec *__restrict__ rec,
                                             const short4 *__restrict__ box, const uint16_t *__restrict__ bm_in,
                                             uint32_t idx, size_t slot, int ox, int oy, bool force, Fetched &f,
                                             uint16_t &m) {
    f.id = vals[idx];
    if (bm_in) {
        m = bm_in[slot];
        f.live = m != 0;
        if (f.live || force) {
            f.b = box[f.id];
            f.r = rec[f.id];
        }
    } else {
        f.b = box[f.id];
        f.live = box_meets_tile(f.b, ox, oy);
        if (f.live || force) f.r = rec[f.id];
    }
}

__device__ __forceinline__ StagedRec make_staged(const Fetched &f, int ox, int oy) {
#pragma clang fp contract(off)
    const float mx = (f.r.m.x - (float)ox) + f.r.m.z;
    const float my = (f.r.m.y - (float)oy) + f.r.m.w;
    const float k = -0.5f * LOG2E;
    const uint32_t mask = span_mask(f.b.x - ox, f.b.z - ox) | (span_mask(f.b.y - oy, f.b.w - oy) << 16);
    StagedRec sr;
    sr.mc = make_float4(mx, my, k * f.r.c.x, -LOG2E * f.r.c.y);
    sr.cc = make_float4(k * f.r.c.z, __log2f(f.r.c.w), f.r.rgb.x, f.r.rgb.y);
    sr.ex = make_float4(f.r.rgb.z, __uint_as_float(mask), __uint_as_float(f.id), 1.0f / f.r.c.w);
    return sr;
}

__device__ __forceinline__ void stage(const Fetched &f, int ox, int oy, StagedRec *s_rec, int t) {
    s_rec[t] = make_staged(f, ox, oy);
}

// Which of the tile's sixteen 4x4 pixel blocks a staged record may
// contribute to: bit 4 by + bx for the block at tile columns 4 bx .. 4 bx + 3
// and rows 4 by .. 4 by + 3.  Always a subset of the blocks its pixel box
// meets; with `ellipse` also of the blocks the ellipse alpha >= 1/255 meets.
//
// A pixel contributes only if exp2(q) >= 1/255, i.e. (with P = -a', R = -b'/2,
// S = -c', L = log2 o and d = pixel - mean) the quadratic form
// P dx^2 + 2 R dx dy + S dy^2 <= L + log2(255).  The kernels evaluate q in
// FP32, with an error below 5 ulp of the sum of the terms' magnitudes; inside
// the ellipse that sum is at most 4 t / (1 - rho^2) (rho^2 = R^2 / (P S), t
// <= 8), so the threshold is raised by 2e-5 (1 + 1 / (1 - rho^2)), above that
// bound, and the extents below (FP32, hardware reciprocal and square root,
// each within a few ulp) are padded for their own rounding.  Every
// pixel the kernels can take as a contributor therefore lies in a block whose
// bit is set; a block skipped holds no contributor, so the outputs are those
// of the box test alone.
//
// Per band of four pixel rows the ellipse's x-extent is taken in closed form:
// for fixed dy the ellipse spans xc(dy) -+ hw(dy) with xc = -(R/P) dy and
// hw = sqrt((t - (det/P) dy^2) / P), det = P S - R^2; the left edge
// xc - hw is convex in dy with its minimum -hx at the ellipse's leftmost point
// (dy = R hx / S), so over a band its minimum is -hx when that point lies in
// the band and the value at the band's nearer end otherwise; the right edge
// mirrors it.
__device__ __forceinline__ uint32_t block_mask(const StagedRec &sr, bool ellipse) {
    const uint32_t m = __float_as_uint(sr.ex.y);
    // blocks the pixel box meets: nonzero nibbles of the column and row masks
    auto nib = [](uint32_t x) {
        const uint32_t t = (x | (x >> 1) | (x >> 2) | (x >> 3)) & 0x1111u;
        return (t | (t >> 3) | (t >> 6) | (t >> 9)) & 0xFu;
    };
    const uint32_t cb = nib(m & 0xFFFFu), rb = nib(m >> 16);
    const uint32_t rspread = (rb & 1u) | ((rb & 2u) << 3) | ((rb & 4u) << 6) | ((rb & 8u) << 9);
    const uint32_t box16 = rspread * cb;   // cb copied into the nibble of every row block
    if (!ellipse || box16 == 0u) return box16;
    const float P = -sr.mc.z, R = -0.5f * sr.mc.w, S = -sr.cc.x, L = sr.cc.y;
    if (!(P > 0.f) || !(S > 0.f)) return box16;
    // 1 - rho^2 from FP32 products: its absolute error is below 4u, so it is
    // lowered by 5e-7 (8.4u); det = P S (1 - rho^2) then errs low, which only
    // widens the extents below
    const float PS = P * S;
    const float omr = (1.0f - (R * R) * __builtin_amdgcn_rcpf(PS)) - 5e-7f;
    if (!(omr > 1e-6f)) return box16;       // (near-)degenerate ellipse: the box's blocks
    const float t = L + 7.99435343685886f + 2e-5f * (1.0f + __builtin_amdgcn_rcpf(omr));
    if (!(t > 0.f)) return t <= 0.f ? 0u : box16;
    const float det = PS * omr, idet = __builtin_amdgcn_rcpf(det), iP = __builtin_amdgcn_rcpf(P);
    const float hx = __builtin_amdgcn_sqrtf(t * S * idet), hy = __builtin_amdgcn_sqrtf(t * P * idet);
    if (!(hx < 1e6f) || !(hy < 1e6f)) return box16;
    const float kc = -R * iP, u = t * iP, e = det * iP * iP;
    const float dyL = R * hx * __builtin_amdgcn_rcpf(S);   // leftmost point's dy; the rightmost is at -dyL
    const float hyp = hy * (1.0f + 1e-5f) + 1e-3f;
    const float padx = 1e-3f + 4e-5f * hx;
    const float slack = 1e-5f * u;          // keeps rounding in u - e y^2 from narrowing the band
    auto edge = [&](float y, float sgn) {
        return kc * y + sgn * __builtin_amdgcn_sqrtf(fmaxf(0.f, u - e * y * y + slack));
    };
    uint32_t ell = 0u;
#pragma unroll
    for (int b = 0; b < 4; b++) {
        const float y0 = fmaxf((float)(4 * b) + 0.5f - sr.mc.y, -hyp);
        const float y1 = fminf((float)(4 * b) + 3.5f - sr.mc.y, hyp);
        const float xmin = (dyL >= y0 && dyL <= y1 ? -hx : edge(dyL < y0 ? y0 : y1, -1.0f)) - padx;
        const float xmax = (-dyL >= y0 && -dyL <= y1 ? hx : edge(-dyL < y0 ? y0 : y1, 1.0f)) + padx;
        // columns 4k .. 4k + 3 have pixel centres 4k + 0.5 .. 4k + 3.5
        const float kmin = fminf(fmaxf(ceilf((xmin + sr.mc.x - 3.5f) * 0.25f), 0.f), 4.f);
        const float kmax = fminf(fmaxf(floorf((xmax + sr.mc.x - 0.5f) * 0.25f), -1.f), 3.f);
        const int k0 = (int)kmin, k1 = (int)kmax;
        const uint32_t bits = (y0 <= y1 && k0 <= k1) ? ((2u << k1) - (1u << k0)) : 0u;
        ell |= bits << (4 * b);
    }
    return ell & box16;
}

// Pixel geometry of a lane: 16-lane row `row` of wave w owns 4x4 block
// sb = 4 w + row of the tile (blocks in row-major order).
struct LaneGeom {
    int lx, ly, row;
    uint32_t pbits;    // this pixel's column and row bits in a record's box masks
    uint32_t bx, by;   // the block's column / row bits in a record's box masks
};

__device__ __forceinline__ LaneGeom lane_geom(int tid) {
    LaneGeom g;
    const int w = tid >> 6, lane = tid & 63;
    g.row = lane >> 4;
    const int sb = w * 4 + g.row, c = lane & 15;
    const int sbx = sb & 3, sby = sb >> 2;
    g.lx = sbx * 4 + (c & 3);
    g.ly = sby * 4 + (c >> 2);
    g.bx = 0xFu << (sbx * 4);
    g.by = (0xFu << (sby * 4)) << 16;
    g.pbits = (1u << g.lx) | (1u << (16 + g.ly));
    return g;
}

// For each row of this wave, the indices j < cnt (ascending) of the staged
// records whose block mask (block_mask) meets the row's pixel block, into
// hits[row][..]; returns this lane's row count.  Row r takes the blocks of
// sel0 << r (sel0: the bits of row 0's block or blocks).  `ok(j)` adds a
// condition that is the same for the whole wave.
template <int BATCH, typename Ok>
__device__ __forceinline__ int compact_rows(const uint16_t *s_bm, int cnt, HitT<BATCH> (*hits)[BATCH + 4],
                                            uint32_t sel0, int row, Ok ok) {
    const int lane = threadIdx.x & 63;
    const uint64_t lt = lanemask_lt();
    int n[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < BATCH / 64; k++) {
        const int j = k * 64 + lane;
        const uint32_t bm = j < cnt ? (uint32_t)s_bm[j] : 0u;
        const bool any = (bm & (sel0 * 0xFu)) && ok(j);
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const bool hit = any && (bm & (sel0 << r));
            const uint64_t bal = __ballot(hit);
            if (hit) hits[r][n[r] + __popcll(bal & lt)] = (HitT<BATCH>)j;
            n[r] += __popcll(bal);
        }
    }
    return row == 0 ? n[0] : row == 1 ? n[1] : row == 2 ? n[2] : n[3];
}

// Row sums of nine values over the 16 lanes of each DPP row, scattered over
// the row's four banks (bank b = lanes 4b .. 4b + 3 of the row).  On return
// every lane of bank b holds in g[0] the row total of value {0, 2, 1, 3}[b],
// in g[4] that of value 4 + {0, 2, 1, 3}[b], and every lane holds in g[8] the
// total of value 8; the other entries are spent.  The first two levels halve
// the row (lanes l and l + 8, then l and l + 4): a DPP add whose bank mask
// leaves half the banks unwritten carries one value there and another value in
// the other half, so two values cost one add per level.  The two levels inside
// a bank are plain quad-permutation butterflies on the three remaining
// registers: 20 DPP adds instead of 36 for nine separate row sums.
//
// Written as one block so the DPP hazard is handled here: a DPP source must
// be written by a VALU instruction at least two instructions earlier, which
// the opening s_nop covers for the inputs and the instruction order covers
// inside (every register is read two or more instructions after its last
// write).  Every lane of the wave must be active.
__device__ __forceinline__ void row_sums9(float (&g)[9]) {
    asm volatile(
        "s_nop 1\n\t"
        // lanes l <-> l + 8: banks 0,1 keep value 2i, banks 2,3 take value 2i+1
        "v_add_f32_dpp %0, %0, %0 row_ror:8 row_mask:0xf bank_mask:0x3\n\t"
        "v_add_f32_dpp %0, %1, %1 row_ror:8 row_mask:0xf bank_mask:0xc\n\t"
        "v_add_f32_dpp %2, %2, %2 row_ror:8 row_mask:0xf bank_mask:0x3\n\t"
        "v_add_f32_dpp %2, %3, %3 row_ror:8 row_mask:0xf bank_mask:0xc\n\t"
        "v_add_f32_dpp %4, %4, %4 row_ror:8 row_mask:0xf bank_mask:0x3\n\t"
        "v_add_f32_dpp %4, %5, %5 row_ror:8 row_mask:0xf bank_mask:0xc\n\t"
        "v_add_f32_dpp %6, %6, %6 row_ror:8 row_mask:0xf bank_mask:0x3\n\t"
        "v_add_f32_dpp %6, %7, %7 row_ror:8 row_mask:0xf bank_mask:0xc\n\t"
        "v_add_f32_dpp %8, %8, %8 row_ror:8 row_mask:0xf bank_mask:0xf\n\t"
        // lanes l <-> l + 4 (row_ror:n reads lane l - n of the row): banks 0,2
        // keep the first register, banks 1,3 take the second
        "v_add_f32_dpp %0, %0, %0 row_ror:12 row_mask:0xf bank_mask:0x5\n\t"
        "v_add_f32_dpp %0, %2, %2 row_ror:4 row_mask:0xf bank_mask:0xa\n\t"
        "v_add_f32_dpp %4, %4, %4 row_ror:12 row_mask:0xf bank_mask:0x5\n\t"
        "v_add_f32_dpp %4, %6, %6 row_ror:4 row_mask:0xf bank_mask:0xa\n\t"
        "v_add_f32_dpp %8, %8, %8 row_ror:4 row_mask:0xf bank_mask:0xf\n\t"
        // the four lanes of a bank
        "v_add_f32_dpp %0, %0, %0 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %4, %4, %4 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %8, %8, %8 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %0, %0, %0 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %4, %4, %4 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %8, %8, %8 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf"
        : "+v"(g[0]), "+v"(g[1]), "+v"(g[2]), "+v"(g[3]), "+v"(g[4]), "+v"(g[5]), "+v"(g[6]), "+v"(g[7]),
          "+v"(g[8]));
}

template <int BATCH>
struct BlendShared {
    StagedRec rec[BATCH];
    uint16_t bm[BATCH];                              // block masks (block_mask)
    HitT<BATCH> hits[AS_BLOCK / 64][4][BATCH + 4];  // +4: the loops read one index ahead
};

// Next tile of this block: a queue slot (persistent grid) or the block index;
// returns false when the block is done.
template <bool PERSIST>
__device__ __forceinline__ bool next_tile(uint32_t *queue, int n_tiles, int iter, uint32_t &idx, uint32_t *s_next) {
    if (!PERSIST) {
        idx = blockIdx.x;
        return iter == 0 && idx < (uint32_t)n_tiles;
    }
    if (threadIdx.x == 0) *s_next = atomicAdd(queue, 1u);
    __syncthreads();
    idx = *s_next;
    __syncthreads();   // all have read the slot before thread 0 takes the next one
    return idx < (uint32_t)n_tiles;
}

// Forward dispatch slots (k_tile_order): a tile id, or ORDER_NONE for a slot
// without a tile (slots grouped by bin of 32 past the image edge).
constexpr uint32_t ORDER_NONE = 0xFFFFFFFFu;

__host__ __device__ inline int order_slots(const ViewTable &vt) {
    if (vt.bin_shift == 4) return vt.tile_base[vt.n_views];
    return 32 * ((vt.bin_base[vt.n_views] + 7) / 8);
}

template <int BATCH, bool PERSIST>
__global__ void __launch_bounds__(AS_BLOCK) k_blend_fwd(const uint32_t *__restrict__ ranges,
                                                        const uint32_t *__restrict__ tile_order,
                                                        const uint32_t *__restrict__ vals,
                                                        const BlendRec *__restrict__ rec,
                                                        const short4 *__restrict__ box, const ViewTable vt,
                                                        const ViewImagesC gts, const ViewImages images,
                                                        float *__restrict__ t_final, uint32_t *__restrict__ last_out,
                                                        uint32_t *__restrict__ ncontrib_out,
                                                        int32_t *__restrict__ dom_out, double *__restrict__ err,
                                                        unsigned long long *__restrict__ tile_err,
                                                        uint32_t *__restrict__ tile_work,
                                                        uint32_t *__restrict__ tile_hi, float4 *__restrict__ ckpt,
                                                        uint16_t *__restrict__ bm_out, int ellipse,
                                                        uint32_t *queue, int n_tiles, uint4 *__restrict__ zero4,
                                                        int64_t zero_n4) {
    constexpr int R = BATCH / AS_BLOCK;
    // Side job: clear the 2D gradient rows the reverse pass adds into, spread
    // over every block of the grid, so the reverse pass needs no fill launch.
    for (int64_t i = (int64_t)blockIdx.x * AS_BLOCK + threadIdx.x; i < zero_n4; i += (int64_t)gridDim.x * AS_BLOCK)
        zero4[i] = make_uint4(0u, 0u, 0u, 0u);
    __shared__ BlendShared<BATCH> sh;
    __shared__ uint32_t s_next;
    __shared__ unsigned long long s_emin[AS_BLOCK / 64], s_emax[AS_BLOCK / 64];
    __shared__ uint32_t s_nc[AS_BLOCK / 64], s_hi[AS_BLOCK / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const LaneGeom lg = lane_geom(tid);
    const HitT<BATCH> *hits = sh.hits[w][lg.row];
    const float px = (float)lg.lx + 0.5f, py = (float)lg.ly + 0.5f;
    uint32_t idx;
    for (int iter = 0; next_tile<PERSIST>(queue, n_tiles, iter, idx, &s_next); iter++) {
        const uint32_t slot = tile_order ? tile_order[idx] : idx;
        if (slot == ORDER_NONE) continue;   // a dispatch slot past the image edge (block-uniform)
        const int tile = (int)slot;
        const int v = view_of_tile(vt, tile);
        const int lt = tile - vt.tile_base[v], tiles_x = vt.tiles_x[v];
        const int W = vt.cam[v].W, H = vt.cam[v].H;
        const int tx = lt % tiles_x, ty = lt / tiles_x;
        const int ox = tx * AS_TILE_W, oy = ty * AS_TILE_H;
        const int x = ox + lg.lx, y = oy + lg.ly;
        const bool inside = x < W && y < H;
        const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];

        float T = 1.0f, C0 = 0.f, C1 = 0.f, C2 = 0.f, wbest = 0.f;
        int32_t dom = -1;
        uint32_t last = 0, nc = 0;
        int done = inside ? 0 : 1;
        // checkpoint slots of this pixel: (T, colour composited so far) at
        // the top of batches 1 .. AS_CK_MAX; the epilogue turns the colour
        // into the colour behind the boundary
        float4 *ck = ckpt ? ckpt + (size_t)tile * AS_CK_MAX * 256 + lg.ly * 16 + lg.lx : nullptr;
        int nck = 0;

        Fetched nf[R];
#pragma unroll
        for (int k = 0; k < R; k++)
            if (start + k * AS_BLOCK + tid < end) fetch(vals, rec, box, start + k * AS_BLOCK + tid, ox, oy, nf[k]);
        for (uint32_t b0 = start; b0 < end; b0 += BATCH) {
            if (__syncthreads_count(done) == AS_BLOCK) break;   // also: the previous batch is consumed
            if (ck && b0 > start && nck < AS_CK_MAX) {
                if (inside) ck[nck * 256] = make_float4(T, C0, C1, C2);
                nck++;
            }
#pragma unroll
            for (int k = 0; k < R; k++) {
                const int t = k * AS_BLOCK + tid;
                if (b0 + t < end) {
                    uint32_t bm = 0u;   // a record whose box misses the tile is not staged
                    if (nf[k].live) {
                        const StagedRec sr = make_staged(nf[k], ox, oy);
                        bm = block_mask(sr, ellipse != 0);
                        sh.rec[t] = sr;
                    }
                    sh.bm[t] = (uint16_t)bm;
                    if (bm_out) bm_out[mask_slot(vt, b0 + t, tx, ty)] = (uint16_t)bm;   // the reverse pass reuses it
                }
                if (b0 + BATCH + t < end) fetch(vals, rec, box, b0 + BATCH + t, ox, oy, nf[k]);
            }
            __syncthreads();
            if (__ballot(!done) == 0) continue;                 // the whole wave has saturated
            const int cnt = (int)min((uint32_t)BATCH, end - b0);
            // wave w's rows are the 4x4 blocks 4 w .. 4 w + 3
            const int nh = compact_rows<BATCH>(sh.bm, cnt, sh.hits[w], 1u << (4 * w), lg.row,
                                               [](int) { return true; });
            if (done) continue;
            // Two hits per step: both records' loads and alpha evaluations are
            // independent and overlap; only the compositing is sequential.
            // The next step's indices are loaded one step ahead.
            int ja = hits[0], jb = hits[1];
            int h = 0;
            for (; h < nh; h += 2) {
                const bool two = h + 1 < nh;
                const int j0 = ja, j1 = two ? jb : ja;
                ja = hits[h + 2];
                jb = hits[h + 3];
                const float4 a0 = sh.rec[j0].mc, a1 = sh.rec[j0].cc, a2 = sh.rec[j0].ex;
                const float4 b0q = sh.rec[j1].mc, b1q = sh.rec[j1].cc, b2q = sh.rec[j1].ex;
                const uint32_t ma = __float_as_uint(a2.y), mb = __float_as_uint(b2q.y);
                const float dxa = a0.x - px, dya = a0.y - py, dxb = b0q.x - px, dyb = b0q.y - py;
                const float rawa = __builtin_amdgcn_exp2f(blend_exponent(dxa, dya, a0, a1));
                const float rawb = __builtin_amdgcn_exp2f(blend_exponent(dxb, dyb, b0q, b1q));
                const float alpha_a = fminf(ALPHA_MAX, rawa), alpha_b = fminf(ALPHA_MAX, rawb);
                const bool oka = (ma & lg.pbits) == lg.pbits && alpha_a >= ALPHA_MIN;   // box holds the pixel
                const bool okb = two && (mb & lg.pbits) == lg.pbits && alpha_b >= ALPHA_MIN;
                // Both records are decided with selects and the loop leaves
                // once after them, so the second record's loads are not held
                // back behind a branch.  A record that would take T below the
                // stop threshold is not added, and nothing after it is; a
                // non-contributor adds exactly zero and changes nothing.
                const float tA = T * (1.0f - alpha_a);
                const bool stopA = oka && tA < T_STOP;
                const bool useA = oka && !stopA;
                float wgt = useA ? alpha_a * T : 0.0f;
                C0 += wgt * a1.z;
                C1 += wgt * a1.w;
                C2 += wgt * a2.x;
                if (wgt > wbest) {
                    wbest = wgt;
                    dom = (int32_t)__float_as_uint(a2.z);
                }
                T = useA ? tA : T;
                last = useA ? b0 + (uint32_t)j0 : last;
                nc += useA ? 1u : 0u;
                const float tB = T * (1.0f - alpha_b);
                const bool stopB = !stopA && okb && tB < T_STOP;
                const bool useB = !stopA && okb && !stopB;
                wgt = useB ? alpha_b * T : 0.0f;
                C0 += wgt * b1q.z;
                C1 += wgt * b1q.w;
                C2 += wgt * b2q.x;
                if (wgt > wbest) {
                    wbest = wgt;
                    dom = (int32_t)__float_as_uint(b2q.z);
                }
                T = useB ? tB : T;
                last = useB ? b0 + (uint32_t)j1 : last;
                nc += useB ? 1u : 0u;
                if (stopA || stopB) {
                    done = 1;
                    break;
                }
            }
        }

        const float *gt = gts.p[v];
        double e = 0.0;
        if (inside) {
            const int64_t P = (int64_t)W * H;
            const int64_t pl = (int64_t)y * W + x, pix = vt.pix_base[v] + pl;
            float *image = images.p[v];
            const float r0 = C0 + T * vt.cam[v].bg[0];
            const float r1 = C1 + T * vt.cam[v].bg[1];
            const float r2 = C2 + T * vt.cam[v].bg[2];
            image[pl] = r0;
            image[P + pl] = r1;
            image[2 * P + pl] = r2;
            t_final[pix] = T;
            last_out[pix] = last;
            ncontrib_out[pix] = nc;
            for (int k = 0; k < nck; k++) {
                const float4 c = ck[k * 256];
                ck[k * 256] = make_float4(c.x, C0 - c.y, C1 - c.z, C2 - c.w);
            }
            dom_out[pix] = dom < 0 ? -1 : dom - (int32_t)vt.ent_base[v];
            if (gt) {
                const double d0 = fabs((double)r0 - (double)gt[pl]);
                const double d1 = fabs((double)r1 - (double)gt[P + pl]);
                const double d2 = fabs((double)r2 - (double)gt[2 * P + pl]);
                e = (d0 + d1) + d2;
                err[pix] = e;
            }
        }
        // Per tile: the contributors summed over its pixels (the reverse
        // pass's dispatch order) and, with a target, the error range, which a
        // second kernel reduces per view: device-wide atomics on one word per
        // view serialise at the memory side and stall every block's gathers.
        // e >= 0, so the IEEE bit patterns order like the values.
        uint32_t ncs = inside ? nc : 0u;
        uint32_t hi = inside && nc ? last + 1 : 0u;
        for (int o = 32; o > 0; o >>= 1) {
            ncs += (uint32_t)__shfl_xor((int)ncs, o, 64);
            hi = max(hi, (uint32_t)__shfl_xor((int)hi, o, 64));
        }
        double emin = 0.0, emax = 0.0;
        if (gt) {
            emin = wave_min_d(inside ? e : __longlong_as_double(0x7ff0000000000000ll));
            emax = wave_max_d(inside ? e : 0.0);
        }
        if (lane == 0) {
            s_nc[w] = ncs;
            s_hi[w] = hi;
            s_emin[w] = (unsigned long long)__double_as_longlong(emin);
            s_emax[w] = (unsigned long long)__double_as_longlong(emax);
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t nsum = s_nc[0], hmax = s_hi[0];
            unsigned long long a = s_emin[0], b = s_emax[0];
#pragma unroll
            for (int k = 1; k < AS_BLOCK / 64; k++) {
                nsum += s_nc[k];
                hmax = max(hmax, s_hi[k]);
                a = s_emin[k] < a ? s_emin[k] : a;
                b = s_emax[k] > b ? s_emax[k] : b;
            }
            tile_work[tile] = nsum;
            tile_hi[tile] = hmax;
            if (gt) {
                tile_err[2 * tile] = a;
                tile_err[2 * tile + 1] = b;
            }
        }
    }
}

// Reverse pass.  For contributor k of a pixel with alpha a_k and transmittance
// T_k in front of it, dC/dc_k = a_k T_k and
//   dL/da_k = T_k (c_k . dL) - B_k / (1 - a_k),
// where B_k = sum over the contributors j behind k of (c_j . dL) a_j T_j plus
// (bg . dL) T_final; walking the list backwards from the last contributor
// restores T_k = T_{k+1}/(1-a_k) and B_k incrementally.  Gradients reach
// (o, conic, mean) only where alpha = o G is below the 0.99 clamp.
//
// Work decomposition: one 16x16 tile per block of two wave64, two pixels per
// lane.  Row `row` of wave w owns the 4x8 pixel block at tile columns
// 4 row .. 4 row + 3 and tile rows 8 w .. 8 w + 7; lane c of the row holds
// pixel A = (4 row + c % 4, 8 w + c / 4) and pixel B four rows below it.  A
// step of a row visits one Gaussian for its 32 pixels, so each staged record
// read, index, reduction and LDS update serves two pixels.  Per step the row
// sums over its pixels, with DPP, the colour gradients and the moments
// dp, dp dx, dp dy, dp dx^2, dp dx dy, dp dy^2 of dp = dL/dp (p the
// Gaussian's exponent, dx, dy the offsets mean - pixel; A and B share dx),
// reduced and scattered over the row's four lane banks so that one lane per
// bank adds two or three of the nine sums into the batch slot of that
// Gaussian in LDS; after the batch one pass turns the moments into mean,
// conic and opacity gradients and issues the global atomics: one set per
// (Gaussian, tile).
constexpr int BWD_BLOCK = 128;

template <int BATCH>
struct BwdShared {
    StagedRec rec[BATCH];
    uint16_t bm[BATCH];
    HitT<BATCH> hits[BWD_BLOCK / 64][4][BATCH + 4];   // +4: the loop reads one index ahead
    float gacc[9][BATCH + 1];   // +1: the four banks' adds of one step fall in four LDS banks
    uint8_t gflag[BATCH];
};

// Next work item of a reverse-pass block: a queue slot (persistent grid) or
// a grid-strided index; false when the block is done.
template <bool PERSIST>
__device__ __forceinline__ bool next_item(uint32_t *queue, uint32_t n, int iter, uint32_t &idx, uint32_t *s_next) {
    if (!PERSIST) {
        idx = blockIdx.x + (uint32_t)iter * gridDim.x;
        return idx < n;
    }
    if (threadIdx.x == 0) *s_next = atomicAdd(queue, 1u);
    __syncthreads();
    idx = *s_next;
    __syncthreads();
    return idx < n;
}

// A work item is one segment of a tile's list: with checkpoints, segment k
// covers entries [start + k S, start + (k + 1) S) and the last segment runs to
// one past the tile's last contributor; a walk starts from the state at the
// segment's end (the forward's checkpoint, or T_final for the last segment).
template <int BATCH, bool PERSIST>
__global__ void __launch_bounds__(BWD_BLOCK) k_blend_bwd(const uint32_t *__restrict__ ranges,
                                                         const uint32_t *__restrict__ items,
                                                         const uint32_t *__restrict__ n_items,
                                                         const uint32_t *__restrict__ tile_hi,
                                                         const float4 *__restrict__ ckpt, uint32_t seg_len,
                                                         const uint32_t *__restrict__ vals,
                                                         const BlendRec *__restrict__ rec,
                                                         const short4 *__restrict__ box, const ViewTable vt,
                                                         const float *__restrict__ t_final,
                                                         const uint32_t *__restrict__ last_in,
                                                         const uint32_t *__restrict__ ncontrib_in,
                                                         const ViewImagesC dLs, float *__restrict__ grad2d,
                                                         const uint16_t *__restrict__ bm_in, uint32_t *queue) {
    constexpr int R = BATCH / BWD_BLOCK;
    __shared__ BwdShared<BATCH> sh;
    __shared__ uint32_t s_next;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int row = lane >> 4, c = lane & 15;
    const int lx = row * 4 + (c & 3), ly = w * 8 + (c >> 2);
    const uint32_t pbA = (1u << lx) | (1u << (16 + ly)), pbB = (1u << lx) | (1u << (20 + ly));
    // row r of wave w covers the 4x4 blocks (r, 2 w) and (r, 2 w + 1)
    const uint32_t sel0 = (1u << (8 * w)) | (1u << (8 * w + 4));
    const HitT<BATCH> *hits = sh.hits[w][row];
    const float px = (float)lx + 0.5f, pyA = (float)ly + 0.5f, pyB = (float)(ly + 4) + 0.5f;
    for (int i = tid; i < BATCH; i += BWD_BLOCK) {
        sh.gflag[i] = 0;
#pragma unroll
        for (int k = 0; k < 9; k++) sh.gacc[k][i] = 0.f;
    }
    const uint32_t n_it = *n_items;
    uint32_t idx;
    for (int iter = 0; next_item<PERSIST>(queue, n_it, iter, idx, &s_next); iter++) {
        const int tile = (int)items[2 * idx];
        const uint32_t seg = items[2 * idx + 1];
        const int v = view_of_tile(vt, tile);
        const int lt = tile - vt.tile_base[v], tiles_x = vt.tiles_x[v];
        const int W = vt.cam[v].W, H = vt.cam[v].H;
        const int tx = lt % tiles_x, ty = lt / tiles_x;
        const int ox = tx * AS_TILE_W, oy = ty * AS_TILE_H;
        const int x = ox + lx, yA = oy + ly, yB = yA + 4;
        const uint32_t start = ranges[2 * tile], hi = tile_hi[tile];
        uint32_t s0 = start, s1 = hi;
        bool last_seg = true;
        if (ckpt) {
            const uint32_t nseg = min((hi - start + seg_len - 1) / seg_len, (uint32_t)AS_CK_MAX + 1u);
            s0 = start + seg * seg_len;
            last_seg = seg + 1 == nseg;
            s1 = last_seg ? hi : s0 + seg_len;
        }

        const int64_t P = (int64_t)W * H;
        const int64_t plA = (int64_t)yA * W + x, plB = plA + 4 * (int64_t)W;
        const float bg0 = vt.cam[v].bg[0], bg1 = vt.cam[v].bg[1], bg2 = vt.cam[v].bg[2];
        // per pixel: one past the last contributor (0: none), dL and the
        // state at the segment's end: T and
        //   Bb = bg.dL T_final + sum over the contributors behind of
        //        (c_j . dL) alpha_j T_j
        // (the colour behind, in absolute terms)
        float TA = 1.0f, TB = 1.0f, BbA = 0.f, BbB = 0.f;
        float dA0 = 0.f, dA1 = 0.f, dA2 = 0.f, dB0 = 0.f, dB1 = 0.f, dB2 = 0.f;
        uint32_t lA = 0, lB = 0;
        const float *dL_dimage = dLs.p[v];
        const float4 *ck = last_seg ? nullptr : ckpt + ((size_t)tile * AS_CK_MAX + seg) * 256;
        if (x < W && yA < H) {
            const int64_t pix = vt.pix_base[v] + plA;
            const float Tf = t_final[pix];
            lA = ncontrib_in[pix] > 0 ? last_in[pix] + 1 : 0u;
            dA0 = dL_dimage[plA];
            dA1 = dL_dimage[P + plA];
            dA2 = dL_dimage[2 * P + plA];
            BbA = Tf * (bg0 * dA0 + bg1 * dA1 + bg2 * dA2);
            TA = Tf;
            if (ck) {
                const float4 q = ck[ly * 16 + lx];
                TA = q.x;
                BbA += q.y * dA0 + q.z * dA1 + q.w * dA2;
            }
        }
        if (x < W && yB < H) {
            const int64_t pix = vt.pix_base[v] + plB;
            const float Tf = t_final[pix];
            lB = ncontrib_in[pix] > 0 ? last_in[pix] + 1 : 0u;
            dB0 = dL_dimage[plB];
            dB1 = dL_dimage[P + plB];
            dB2 = dL_dimage[2 * P + plB];
            BbB = Tf * (bg0 * dB0 + bg1 * dB1 + bg2 * dB2);
            TB = Tf;
            if (ck) {
                const float4 q = ck[(ly + 4) * 16 + lx];
                TB = q.x;
                BbB += q.y * dB0 + q.z * dB1 + q.w * dB2;
            }
        }
        uint32_t wlast = max(lA, lB);   // one past the wave's last contributor (wave-uniform)
        for (int o = 32; o > 0; o >>= 1) wlast = max(wlast, (uint32_t)__shfl_xor((int)wlast, o, 64));

        // batches [b0, b1) walk the segment backwards from its end
        // block masks come from the forward (bm_in); frames without that
        // buffer take the box's blocks (any mask that keeps every block
        // holding a contributor gives the same outputs)
        Fetched nf[R];
        uint16_t nbm[R];
        {
            const uint32_t b0 = s1 - s0 > (uint32_t)BATCH ? s1 - BATCH : s0;
#pragma unroll
            for (int k = 0; k < R; k++)
                if (b0 + k * BWD_BLOCK + tid < s1) {
                    const uint32_t i = b0 + k * BWD_BLOCK + tid;
                    fetch_masked(vals, rec, box, bm_in, i, mask_slot(vt, i, tx, ty), ox, oy, k == 0 && tid == 0, nf[k],
                                 nbm[k]);
                }
        }
        for (uint32_t b1 = s1; b1 > s0;) {
            const uint32_t b0 = b1 - s0 > (uint32_t)BATCH ? b1 - BATCH : s0;
            const uint32_t n1 = b0, n0 = n1 - s0 > (uint32_t)BATCH ? n1 - BATCH : s0;
#pragma unroll
            for (int k = 0; k < R; k++) {
                const int t = k * BWD_BLOCK + tid;
                if (b0 + t < b1) {
                    uint16_t bm = 0;   // records that cannot touch the tile are not staged (slot 0 always is)
                    if (nf[k].live || t == 0) {
                        const StagedRec sr = make_staged(nf[k], ox, oy);
                        sh.rec[t] = sr;
                        if (nf[k].live) bm = bm_in ? nbm[k] : (uint16_t)block_mask(sr, false);
                    }
                    sh.bm[t] = bm;
                }
                if (n0 + t < n1)
                    fetch_masked(vals, rec, box, bm_in, n0 + t, mask_slot(vt, n0 + t, tx, ty), ox, oy, t == 0, nf[k],
                                 nbm[k]);
            }
            __syncthreads();
            const int nh = compact_rows<BATCH>(sh.bm, (int)(b1 - b0), sh.hits[w], sel0, row,
                                               [&](int j) { return b0 + (uint32_t)j < wlast; });
            // the wave walks max over its rows of the row counts; rows past their
            // own count idle
            int nmax = nh;
            for (int o = 16; o < 64; o <<= 1) nmax = max(nmax, __shfl_xor(nmax, o, 64));
            nmax = __builtin_amdgcn_readfirstlane(nmax);   // wave-uniform: scalar loop control
            // The step's geometry (mean, conic, log2 o, box mask) is read from
            // LDS one step ahead, so its exponent does not wait on the read;
            // the record index two steps ahead.
            int jcur = nmax > 0 && nmax - 1 < nh ? hits[nmax - 1] : 0;
            float4 pq0 = sh.rec[jcur].mc;
            float4 pq1 = sh.rec[jcur].cc;
            float2 pq2 = make_float2(sh.rec[jcur].ex.x, sh.rec[jcur].ex.y);
            int jn = hits[nmax > 1 ? nmax - 2 : 0];
            for (int h = nmax - 1; h >= 0; h--) {
                const bool valid = h < nh;
                const int j = jcur;
                const float4 q0 = pq0, q1 = pq1;
                const float2 q2xy = pq2;
                const uint32_t m = __float_as_uint(q2xy.y);
                // the next step's record
                jcur = h > 0 && h - 1 < nh ? jn : 0;
                jn = hits[h > 1 ? h - 2 : 0];
                pq0 = sh.rec[jcur].mc;
                pq1 = sh.rec[jcur].cc;
                pq2 = make_float2(sh.rec[jcur].ex.x, sh.rec[jcur].ex.y);
                const uint32_t gidx = b0 + (uint32_t)j;
                const float dx = q0.x - px, dyA = q0.y - pyA, dyB = q0.y - pyB;
                const float arA = __builtin_amdgcn_exp2f(blend_exponent(dx, dyA, q0, q1));
                const float arB = __builtin_amdgcn_exp2f(blend_exponent(dx, dyB, q0, q1));
                const float alA = fminf(ALPHA_MAX, arA), alB = fminf(ALPHA_MAX, arB);
                const bool cA = valid && gidx < lA && (m & pbA) == pbA && alA >= ALPHA_MIN;
                const bool cB = valid && gidx < lB && (m & pbB) == pbB && alB >= ALPHA_MIN;
                const uint64_t cb = __ballot(cA || cB);
                if (!cb) continue;
                // Every lane evaluates the step for both pixels; a
                // non-contributor's weight and dp are zero, so its sums and
                // state stay unchanged.
                const float cdlA = q1.z * dA0 + q1.w * dA1 + q2xy.x * dA2;
                const float cdlB = q1.z * dB0 + q1.w * dB1 + q2xy.x * dB2;
                const float romA = __builtin_amdgcn_rcpf(1.0f - alA), romB = __builtin_amdgcn_rcpf(1.0f - alB);
                const float TkA = TA * romA, TkB = TB * romB;
                TA = cA ? TkA : TA;
                TB = cB ? TkB : TB;
                const float wA = cA ? alA * TkA : 0.0f, wB = cB ? alB * TkB : 0.0f;
                // dL/dalpha_k = T_k (c_k . dL) - Bb / (1 - alpha_k)
                const float dLdaA = TkA * cdlA - BbA * romA, dLdaB = TkB * cdlB - BbB * romB;
                BbA += wA * cdlA;
                BbB += wB * cdlB;
                // alpha = o exp(p): dalpha/dp = alpha below the clamp
                const float dpA = (cA && arA < ALPHA_MAX) ? dLdaA * arA : 0.0f;
                const float dpB = (cB && arB < ALPHA_MAX) ? dLdaB * arB : 0.0f;
                const float dpyA = dpA * dyA, dpyB = dpB * dyB;
                const float s0 = dpA + dpB, sy = dpyA + dpyB, sx = s0 * dx;
                float g[9] = {s0,
                              sx,
                              sy,
                              sx * dx,
                              sy * dx,
                              dpyA * dyA + dpyB * dyB,
                              wA * dA0 + wB * dB0,
                              wA * dA1 + wB * dB1,
                              wA * dA2 + wB * dB2};
                row_sums9(g);
                // the first lane of each bank adds its two sums (bank 0 also
                // the ninth) into the batch slot of the row's Gaussian
                if ((c & 3) == 0 && ((cb >> (row * 16)) & 0xFFFFull)) {
                    const int bank = c >> 2, k0 = ((bank & 1) << 1) | (bank >> 1);
                    atomicAdd(&sh.gacc[k0][j], g[0]);
                    atomicAdd(&sh.gacc[4 + k0][j], g[4]);
                    if (bank == 0) {
                        atomicAdd(&sh.gacc[8][j], g[8]);
                        sh.gflag[j] = 1;
                    }
                }
            }
            __syncthreads();
            // One set of global atomics per entry of the batch that received
            // gradients.  With p = -(a dx^2 + c dy^2)/2 - b dx dy (unscaled
            // conic a, b, c): dp/dmean = -(a dx + b dy, c dy + b dx),
            // dp/d(a, b, c) = -(dx^2/2, dx dy, dy^2/2) and dalpha/do = alpha/o.
            // First a thread per entry turns its sums into the nine
            // gradients, in place; then lanes take (entry, value) pairs, so
            // the nine atomics of an entry go to the nine consecutive words of
            // its entry-major row from neighbouring lanes of one instruction.
            // A lane clears the word it read and skips an exact zero (adding
            // it changes nothing), which also passes over the entries that
            // received nothing.
            for (int i = tid; i < (int)(b1 - b0); i += BWD_BLOCK) {
                if (sh.gflag[i]) {
                    sh.gflag[i] = 0;
                    const float4 q0 = sh.rec[i].mc;
                    const float q1x = sh.rec[i].cc.x, inv_o = sh.rec[i].ex.w;
                    const float a = -2.0f * LN2 * q0.z, b = -LN2 * q0.w, cc = -2.0f * LN2 * q1x;
                    float g[6];
#pragma unroll
                    for (int k = 0; k < 6; k++) g[k] = sh.gacc[k][i];
                    sh.gacc[0][i] = -(a * g[1] + b * g[2]);
                    sh.gacc[1][i] = -(cc * g[2] + b * g[1]);
                    sh.gacc[2][i] = -0.5f * g[3];
                    sh.gacc[3][i] = -g[4];
                    sh.gacc[4][i] = -0.5f * g[5];
                    sh.gacc[5][i] = g[0] * inv_o;   // colour gradients (k = 6, 7, 8) as summed
                }
            }
            __syncthreads();
            for (int f = tid; f < 9 * (int)(b1 - b0); f += BWD_BLOCK) {
                const int i = f / 9, k = f - 9 * i;
                const float gv = sh.gacc[k][i];
                if (gv != 0.0f) {
                    sh.gacc[k][i] = 0.f;
                    const int64_t id = (int64_t)__float_as_uint(sh.rec[i].ex.z);
                    atomicAdd(&grad2d[id * 9 + k], gv);
                }
            }
            __syncthreads();
            b1 = b0;
        }
    }
}

// Tiles ordered by descending list length (33 length classes with power-of-two
// boundaries), so the longest lists are dispatched first.  The order within a
// class is irrelevant: every tile's outputs are independent of the others.
//
// With bins of 32 the four tiles of a bin read the same list: bins are
// ordered instead, and the tiles of the bin at rank q take the dispatch slots
// 32 (q / 8) + q % 8 + 8 i (i = 0..3), which the hardware hands to one XCD
// (workgroups go to the eight XCDs round robin), so the bin's records are
// fetched from HBM once into that XCD's L2.  Slots of tiles past the image
// edge hold ORDER_NONE and their blocks do nothing.
__global__ void __launch_bounds__(1024) k_tile_order(const uint32_t *__restrict__ ranges, const ViewTable vt,
                                                     uint32_t *__restrict__ order) {
    __shared__ uint32_t s_cnt[33], s_off[33];
    const int tid = threadIdx.x;
    const bool bins = vt.bin_shift != 4;
    const int n = bins ? vt.bin_base[vt.n_views] : vt.tile_base[vt.n_views];
    // the first tile of unit u (a tile, or the top-left tile of a bin) and
    // the tile of quadrant i of bin u (-1 past the image edge)
    auto quad = [&](int u, int i) -> int {
        if (!bins) return i == 0 ? u : -1;
        const int v = view_of_bin(vt, u);
        const int lb = u - vt.bin_base[v], bx = lb % vt.bins_x[v], by = lb / vt.bins_x[v];
        const int tx_n = vt.tiles_x[v], ty_n = (vt.tile_base[v + 1] - vt.tile_base[v]) / tx_n;
        const int tx = 2 * bx + (i & 1), ty = 2 * by + (i >> 1);
        return tx < tx_n && ty < ty_n ? vt.tile_base[v] + ty * tx_n + tx : -1;
    };
    auto cls_of = [&](int u) {
        const int t = quad(u, 0);
        const uint32_t len = ranges[2 * t + 1] - ranges[2 * t];
        return len ? 32 - __clz(len) : 0;   // 0..32, larger = longer
    };
    constexpr int TO_LDS_UNITS = 16384;   // classes of up to this many units are kept for the scatter pass
    __shared__ uint8_t s_cls[TO_LDS_UNITS];
    const bool keep = n <= TO_LDS_UNITS;
    if (tid < 33) s_cnt[tid] = 0;
    if (bins)
        for (int i = tid; i < order_slots(vt); i += blockDim.x) order[i] = ORDER_NONE;
    __syncthreads();
    for (int u = tid; u < n; u += blockDim.x) {
        const int c = cls_of(u);
        if (keep) s_cls[u] = (uint8_t)c;
        atomicAdd(&s_cnt[32 - c], 1u);
    }
    __syncthreads();
    if (tid < 64) {   // exclusive prefix over the 33 classes, one wave
        const uint32_t v = tid < 33 ? s_cnt[tid] : 0u;
        uint32_t inc = v;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = (uint32_t)__shfl_up((int)inc, o, 64);
            if (tid >= o) inc += t;
        }
        if (tid < 33) s_off[tid] = inc - v;
    }
    __syncthreads();
    for (int u = tid; u < n; u += blockDim.x) {
        const uint32_t q = atomicAdd(&s_off[32 - (keep ? (int)s_cls[u] : cls_of(u))], 1u);
        if (!bins) {
            order[q] = (uint32_t)u;
            continue;
        }
        for (int i = 0; i < 4; i++) {
            const int t = quad(u, i);
            if (t >= 0) order[32 * (q >> 3) + (q & 7) + 8 * i] = (uint32_t)t;
        }
    }
}

// Tiles ordered by descending work (contributors summed over the tile's
// pixels), in 129 classes: four per octave, so tiles of similar cost share a
// class and the heaviest are dispatched first.
__device__ __forceinline__ int work_class(uint32_t wk) {
    if (wk == 0) return 0;
    const int lg = 31 - __clz(wk);
    const int frac = lg >= 2 ? (int)((wk >> (lg - 2)) & 3u) : (int)((wk << (2 - lg)) & 3u);
    return 1 + 4 * lg + frac;   // 1..128
}

// Exclusive prefix over the 129 work classes (s_cnt -> s_off), by the
// block's first wave, three classes per lane.
__device__ __forceinline__ void class_prefix129(const uint32_t *s_cnt, uint32_t *s_off, int tid) {
    if (tid >= 64) return;
    uint32_t v[3], sum = 0;
    for (int k = 0; k < 3; k++) {
        const int c = 3 * tid + k;
        v[k] = c < 129 ? s_cnt[c] : 0u;
        sum += v[k];
    }
    uint32_t inc = sum;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)inc, o, 64);
        if (tid >= o) inc += t;
    }
    uint32_t run = inc - sum;
    for (int k = 0; k < 3; k++) {
        const int c = 3 * tid + k;
        if (c < 129) s_off[c] = run;
        run += v[k];
    }
}

// After the forward blend, in one block: the error range of each view with a
// target (minimum and maximum over its tiles' ranges; device-wide atomics on
// one word per view would serialise at the memory side), the reverse pass's
// dispatch order (tiles by descending contributor count, 129 classes: four
// per octave, heaviest first) and its work items: the tiles in that order,
// each expanded into its segments (one without checkpoints), by a block-wide
// exclusive scan of the segment counts.
__global__ void __launch_bounds__(1024) k_after_fwd(const ViewTable vt, const ViewImagesC gts,
                                                    const unsigned long long *__restrict__ tile_err,
                                                    unsigned long long *__restrict__ minmax,
                                                    const uint32_t *__restrict__ work, int order_on,
                                                    uint32_t *__restrict__ order, const uint32_t *__restrict__ ranges,
                                                    const uint32_t *__restrict__ tile_hi, uint32_t seg_len, int ck,
                                                    uint32_t *__restrict__ items, uint32_t *__restrict__ n_items) {
    // up to AF_LDS_TILES tiles, the ordered tiles and their segment counts
    // are also kept in LDS, so the item expansion gathers nothing from memory
    constexpr int AF_LDS_TILES = 16384;
    __shared__ uint16_t s_tile[AF_LDS_TILES];
    __shared__ uint8_t s_nseg[AF_LDS_TILES];
    __shared__ uint32_t s_cnt[129], s_off[129];
    __shared__ unsigned long long s_mn[16], s_mx[16];
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_carry;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int tiles = vt.tile_base[vt.n_views];
    const bool in_lds = order_on && tiles <= AF_LDS_TILES;
    // segments of a tile: one per checkpointed batch boundary it crosses, plus one
    auto nseg_from = [&](uint32_t start, uint32_t hi) -> uint32_t {
        if (hi <= start) return 0u;
        return ck ? min((hi - start + seg_len - 1) / seg_len, (uint32_t)AS_CK_MAX + 1u) : 1u;
    };
    auto nseg_of = [&](uint32_t tile) -> uint32_t { return nseg_from(ranges[2 * tile], tile_hi[tile]); };
    // Up to AF_K tiles per thread (8192 tiles) every per-tile input (error
    // range, work, range and end of list) is loaded once, all loads issued
    // before the first use, and the passes below work from registers; the
    // loops over memory that larger counts take wait for one load round trip
    // per iteration in each pass.
    constexpr int AF_K = 8;
    constexpr unsigned long long ERR_HI = 0x7ff0000000000000ull;
    if (tiles <= AF_K * 1024) {
        unsigned long long ea[AF_K], eb[AF_K];
        uint32_t wk[AF_K], r0[AF_K], rh[AF_K];
#pragma unroll
        for (int k = 0; k < AF_K; k++) {
            const int t = tid + 1024 * k;
            const bool in = t < tiles;
            ea[k] = in ? tile_err[2 * t] : ERR_HI;
            eb[k] = in ? tile_err[2 * t + 1] : 0ull;
            wk[k] = in && order_on ? work[t] : 0u;
            r0[k] = in && in_lds ? ranges[2 * t] : 0u;
            rh[k] = in && in_lds ? tile_hi[t] : 0u;
        }
        for (int v = 0; v < vt.n_views; v++) {
            if (!gts.p[v]) continue;
            unsigned long long mn = ERR_HI, mx = 0ull;
#pragma unroll
            for (int k = 0; k < AF_K; k++) {
                const int t = tid + 1024 * k;
                if (t >= vt.tile_base[v] && t < vt.tile_base[v + 1]) {
                    mn = ea[k] < mn ? ea[k] : mn;
                    mx = eb[k] > mx ? eb[k] : mx;
                }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const unsigned long long a = __shfl_xor(mn, o, 64), b = __shfl_xor(mx, o, 64);
                mn = a < mn ? a : mn;
                mx = b > mx ? b : mx;
            }
            if (lane == 0) {
                s_mn[w] = mn;
                s_mx[w] = mx;
            }
            __syncthreads();
            if (tid == 0) {
                for (int k = 1; k < 16; k++) {
                    mn = s_mn[k] < mn ? s_mn[k] : mn;
                    mx = s_mx[k] > mx ? s_mx[k] : mx;
                }
                minmax[2 * v] = mn;
                minmax[2 * v + 1] = mx;
            }
            __syncthreads();
        }
        if (order_on) {
            if (tid < 129) s_cnt[tid] = 0;
            __syncthreads();
#pragma unroll
            for (int k = 0; k < AF_K; k++)
                if (tid + 1024 * k < tiles) atomicAdd(&s_cnt[128 - work_class(wk[k])], 1u);
            __syncthreads();
            class_prefix129(s_cnt, s_off, tid);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < AF_K; k++) {
                const int t = tid + 1024 * k;
                if (t < tiles) {
                    const uint32_t slot = atomicAdd(&s_off[128 - work_class(wk[k])], 1u);
                    order[slot] = (uint32_t)t;
                    if (in_lds) {
                        s_tile[slot] = (uint16_t)t;
                        s_nseg[slot] = (uint8_t)nseg_from(r0[k], rh[k]);
                    }
                }
            }
        }
    } else {
        for (int v = 0; v < vt.n_views; v++) {
            if (!gts.p[v]) continue;
            unsigned long long mn = 0x7ff0000000000000ull, mx = 0ull;
            for (int t = vt.tile_base[v] + tid; t < vt.tile_base[v + 1]; t += 1024) {
                const unsigned long long a = tile_err[2 * t], b = tile_err[2 * t + 1];
                mn = a < mn ? a : mn;
                mx = b > mx ? b : mx;
            }
            for (int o = 32; o > 0; o >>= 1) {
                const unsigned long long a = __shfl_xor(mn, o, 64), b = __shfl_xor(mx, o, 64);
                mn = a < mn ? a : mn;
                mx = b > mx ? b : mx;
            }
            if (lane == 0) {
                s_mn[w] = mn;
                s_mx[w] = mx;
            }
            __syncthreads();
            if (tid == 0) {
                for (int k = 1; k < 16; k++) {
                    mn = s_mn[k] < mn ? s_mn[k] : mn;
                    mx = s_mx[k] > mx ? s_mx[k] : mx;
                }
                minmax[2 * v] = mn;
                minmax[2 * v + 1] = mx;
            }
            __syncthreads();
        }
        if (order_on) {
            if (tid < 129) s_cnt[tid] = 0;
            __syncthreads();
            for (int t = tid; t < tiles; t += 1024) atomicAdd(&s_cnt[128 - work_class(work[t])], 1u);
            __syncthreads();
            class_prefix129(s_cnt, s_off, tid);
            __syncthreads();
            for (int t = tid; t < tiles; t += 1024) {
                const uint32_t ns = in_lds ? nseg_of((uint32_t)t) : 0u;
                const uint32_t slot = atomicAdd(&s_off[128 - work_class(work[t])], 1u);
                order[slot] = (uint32_t)t;
                if (in_lds) {
                    s_tile[slot] = (uint16_t)t;
                    s_nseg[slot] = (uint8_t)ns;
                }
            }
        }
    }
    if (tid == 0) s_carry = 0;
    __syncthreads();   // also: the order written above is visible to the whole block
    // four consecutive dispatch slots per thread, 4096 per block-wide scan
    for (int base = 0; base < tiles; base += 4096) {
        uint32_t tl[4], ns[4], sum = 0;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int i = base + 4 * tid + k;
            tl[k] = 0u;
            ns[k] = 0u;
            if (i < tiles) {
                if (in_lds) {
                    tl[k] = s_tile[i];
                    ns[k] = s_nseg[i];
                } else {
                    tl[k] = order_on ? order[i] : (uint32_t)i;
                    ns[k] = nseg_of(tl[k]);
                }
            }
            sum += ns[k];
        }
        uint32_t incl = sum;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = (uint32_t)__shfl_up((int)incl, o, 64);
            if (lane >= o) incl += t;
        }
        if (lane == 63) s_w[w] = incl;
        __syncthreads();
        uint32_t before = s_carry;
        for (int k = 0; k < w; k++) before += s_w[k];
        uint32_t off = before + incl - sum;
        uint2 *it = reinterpret_cast<uint2 *>(items);   // (tile, segment) pairs
#pragma unroll
        for (int k = 0; k < 4; k++)
            for (uint32_t j = 0; j < ns[k]; j++) it[off++] = make_uint2(tl[k], j);
        __syncthreads();
        if (tid == 1023) s_carry = before + incl;
        __syncthreads();
    }
    if (tid == 0) *n_items = s_carry;
}

// Test hook: the blend's unclamped alpha o G = exp2(q) of entry ent[i] at
// pixel pix[i] (view coordinates), staged for the pixel's tile exactly as the
// blend kernels stage it.
__global__ void k_debug_alpha(const BlendRec *__restrict__ rec, const short4 *__restrict__ box, int64_t n,
                              const int32_t *__restrict__ pix, const uint32_t *__restrict__ ent,
                              float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int x = pix[2 * i], y = pix[2 * i + 1];
    const int ox = (x / AS_TILE_W) * AS_TILE_W, oy = (y / AS_TILE_H) * AS_TILE_H;
    Fetched f;
    f.id = ent[i];
    f.r = rec[f.id];
    f.b = box[f.id];
    const StagedRec sr = make_staged(f, ox, oy);
    const float px = (float)(x - ox) + 0.5f, py = (float)(y - oy) + 0.5f;
    out[i] = __builtin_amdgcn_exp2f(blend_exponent(sr.mc.x - px, sr.mc.y - py, sr.mc, sr.cc));
}

}  // namespace

void launch_debug_alpha(const as_frame *f, int64_t n, const int32_t *pix, const uint32_t *ent, float *out,
                        hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_debug_alpha, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, f->rec,
                       reinterpret_cast<const short4 *>(f->box), n, pix, ent, out);
}

void launch_tile_order(const uint32_t *ranges, const ViewTable &vt, uint32_t *order, hipStream_t s) {
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(1024), 0, s, ranges, vt, order);
}

void launch_after_fwd(const as_frame *f, const ViewTable &vt, const ViewImagesC &gt, int order_on, hipStream_t s) {
    const int tiles = vt.tile_base[vt.n_views];
    if (tiles == 0) return;
    hipLaunchKernelGGL(k_after_fwd, dim3(1), dim3(1024), 0, s, vt, gt,
                       reinterpret_cast<const unsigned long long *>(f->tile_err),
                       reinterpret_cast<unsigned long long *>(f->err_minmax), f->tile_work, order_on, f->tile_order_bwd,
                       f->ranges, f->tile_hi, (uint32_t)f->ck_seg, f->ck_written ? 1 : 0, f->bwd_items, f->n_items);
}

namespace {
// Resident blocks of a kernel on the whole device (persistent grid size).
template <typename Kern>
int resident_blocks(Kern k, int n_cu, int block = AS_BLOCK) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, block, 0) != hipSuccess || per_cu < 1) per_cu = 1;
    return per_cu * (n_cu > 0 ? n_cu : 1);
}
}  // namespace

int blend_fwd_batch(const BlendLaunch &bl) { return bl.batch >= 1024 ? 1024 : bl.batch >= 512 ? 512 : 256; }

bool launch_blend_fwd(const as_frame *f, const uint32_t *vals, const uint32_t *tile_order, const BlendLaunch &bl,
                      const ViewTable &vt, const ViewImagesC &gt, const ViewImages &image, hipStream_t s,
                      float *zero_g2d, int64_t zero_floats) {
    if (vt.tile_base[vt.n_views] == 0) return false;
    // whole 16-byte groups covering the floats (the buffer has slack past its count)
    uint4 *z4 = reinterpret_cast<uint4 *>(zero_g2d);
    const int64_t zn4 = zero_g2d ? (zero_floats + 3) / 4 : 0;
    // dispatch slots: the tiles, or with an order over bins of 32 its slots
    const int tiles = tile_order ? order_slots(vt) : vt.tile_base[vt.n_views];
    const short4 *b4 = reinterpret_cast<const short4 *>(f->box);
    unsigned long long *te = reinterpret_cast<unsigned long long *>(f->tile_err);
    if (bl.persistent) launch_fill_u32(f->queue, 0u, 1, s);
#define AS_FWD(B, PER)                                                                                             \
    do {                                                                                                           \
        static int grid_p = 0;                                                                                     \
        int grid = tiles;                                                                                          \
        if (PER) {                                                                                                 \
            if (!grid_p) grid_p = resident_blocks(k_blend_fwd<B, PER>, bl.n_cu);                                   \
            grid = grid_p < tiles ? grid_p : tiles;                                                                \
        }                                                                                                          \
        hipLaunchKernelGGL((k_blend_fwd<B, PER>), dim3(grid), dim3(AS_BLOCK), 0, s, f->ranges, tile_order, vals,  \
                           f->rec, b4, vt, gt, image, f->t_final, f->last, f->n_contrib, f->dom, f->err, te,      \
                           f->tile_work, f->tile_hi, reinterpret_cast<float4 *>(f->ckpt), f->bmask,               \
                           bl.ellipse, f->queue, tiles, z4, zn4);                                                  \
    } while (0)
    if (bl.persistent) {
        if (bl.batch >= 1024) AS_FWD(1024, true);
        else if (bl.batch >= 512) AS_FWD(512, true);
        else AS_FWD(256, true);
    } else {
        if (bl.batch >= 1024) AS_FWD(1024, false);
        else if (bl.batch >= 512) AS_FWD(512, false);
        else AS_FWD(256, false);
    }
#undef AS_FWD
    return true;
}

void launch_blend_bwd(const as_frame *f, const uint32_t *vals, const uint32_t *tile_order, const BlendLaunch &bl,
                      const ViewTable &vt, const ViewImagesC &dL_dimage, float *grad2d, hipStream_t s) {
    const int tiles = vt.tile_base[vt.n_views];
    if (tiles == 0) return;
    const short4 *b4 = reinterpret_cast<const short4 *>(f->box);
    const bool ck = f->ck_written && f->ckpt;
    const uint32_t seg_len = (uint32_t)f->ck_seg;
    if (bl.persistent) launch_fill_u32(f->queue + 1, 0u, 1, s);
    const float4 *ckp = ck ? reinterpret_cast<const float4 *>(f->ckpt) : nullptr;
    // one block per item for the usual count (most tiles are one segment);
    // blocks stride over the items beyond the grid
    const int grid_items = ck ? 2 * tiles : tiles;
#define AS_BWD(B, PER)                                                                                             \
    do {                                                                                                           \
        static int grid_p = 0;                                                                                     \
        int grid = grid_items;                                                                                     \
        if (PER) {                                                                                                 \
            if (!grid_p) grid_p = resident_blocks(k_blend_bwd<B, PER>, bl.n_cu, BWD_BLOCK);                        \
            grid = grid_p < grid_items ? grid_p : grid_items;                                                      \
        }                                                                                                          \
        hipLaunchKernelGGL((k_blend_bwd<B, PER>), dim3(grid), dim3(BWD_BLOCK), 0, s, f->ranges, f->bwd_items,     \
                           f->n_items, f->tile_hi, ckp, seg_len, vals, f->rec, b4, vt, f->t_final, f->last,        \
                           f->n_contrib, dL_dimage, grad2d, f->bm_written ? f->bmask : nullptr, f->queue + 1);    \
    } while (0)
    // the reverse pass stages half the forward's depth: two waves per tile
    if (bl.persistent) {
        if (bl.batch >= 512) AS_BWD(256, true);
        else AS_BWD(128, true);
    } else {
        if (bl.batch >= 512) AS_BWD(256, false);
        else AS_BWD(128, false);
    }
#undef AS_BWD
}

AS_WARM_KERNEL(blend)
