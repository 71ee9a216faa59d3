// Tile binning: exclusive scans, tile key emission and per-tile ranges (the
// radix sort between them is in radix.hip).
//
// The rasterizer composites each pixel over the Gaussians in ascending
// (depth, id) order (Sec. 3, front-to-back blending).  The host sorts the
// entries stably by the float bits of their depth (ids ascending on ties),
// emits each entry's tile ids in that order, and sorts the (tile, entry) pairs
// stably on the tile id alone: every tile's list then comes out in exactly
// the order a stable sort of tile << 32 | depth keys emitted by id gives.
#include "internal.h"

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int lane = __lane_id();
    for (int o = 1; o < 64; o <<= 1) {
        T t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan of one value per thread across a 256-thread block; returns
// the thread's exclusive prefix, *total gets the block sum.
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T *s_wave, T *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T inc = wave_incl_scan(v);
    if (lane == 63) s_wave[w] = inc;
    __syncthreads();
    T wpre = 0, tot = 0;
    for (int k = 0; k < SCAN_THREADS / 64; k++) {
        T x = s_wave[k];
        if (k < w) wpre += x;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return wpre + inc - v;
}

template <typename Tin, typename Tout>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_reduce(const Tin *__restrict__ in, int64_t n,
                                                              Tout *__restrict__ partials) {
    __shared__ Tout s_wave[4];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    Tout sum = 0;
    for (int k = 0; k < SCAN_ITEMS; k++) {
        const int64_t idx = base + k;
        if (idx < n) sum += (Tout)in[idx];
    }
    Tout tot;
    block_excl_scan<Tout>(sum, s_wave, &tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

template <typename Tout>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_partials(Tout *__restrict__ partials, int64_t nb,
                                                                Tout *__restrict__ total) {
    __shared__ Tout s_wave[4];
    Tout carry = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += SCAN_TILE) {
        const int64_t base = c0 + (int64_t)threadIdx.x * SCAN_ITEMS;
        Tout v[SCAN_ITEMS];
        Tout sum = 0;
        for (int k = 0; k < SCAN_ITEMS; k++) {
            v[k] = (base + k < nb) ? partials[base + k] : (Tout)0;
            sum += v[k];
        }
        Tout tot;
        Tout pre = block_excl_scan<Tout>(sum, s_wave, &tot);
        Tout run = carry + pre;
        for (int k = 0; k < SCAN_ITEMS; k++) {
            if (base + k < nb) partials[base + k] = run;
            run += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

template <typename Tin, typename Tout>
// `in` and `out` may alias (in-place scan): each thread reads all its items
// before the block scan's barriers and writes only those items afterwards.
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_down(const Tin *in, int64_t n, const Tout *__restrict__ partials,
                                                            Tout *out) {
    __shared__ Tout s_wave[4];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    Tout v[SCAN_ITEMS];
    Tout sum = 0;
    for (int k = 0; k < SCAN_ITEMS; k++) {
        const int64_t idx = base + k;
        v[k] = idx < n ? (Tout)in[idx] : (Tout)0;
        sum += v[k];
    }
    Tout tot;
    Tout run = block_excl_scan<Tout>(sum, s_wave, &tot) + partials[blockIdx.x];
    for (int k = 0; k < SCAN_ITEMS; k++) {
        const int64_t idx = base + k;
        if (idx < n) out[idx] = run;
        run += v[k];
    }
}

// Up to SCAN_DIRECT_BLOCKS blocks, the downsweep takes each block's offset
// by summing the block sums before it itself (at most a few loads per
// thread), so the scan is two launches instead of three; the last block also
// writes the total.
constexpr int64_t SCAN_DIRECT_BLOCKS = 1024;

template <typename Tin, typename Tout>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_down_direct(const Tin *in, int64_t n,
                                                                   const Tout *__restrict__ partials, Tout *out,
                                                                   Tout *__restrict__ total) {
    __shared__ Tout s_wave[4];
    Tout pre = 0;
    for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += SCAN_THREADS) pre += partials[b];
    Tout ptot;
    block_excl_scan<Tout>(pre, s_wave, &ptot);   // ptot: the sum of the block sums before this block
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    Tout v[SCAN_ITEMS];
    Tout sum = 0;
    for (int k = 0; k < SCAN_ITEMS; k++) {
        const int64_t idx = base + k;
        v[k] = idx < n ? (Tout)in[idx] : (Tout)0;
        sum += v[k];
    }
    Tout tot;
    Tout run = block_excl_scan<Tout>(sum, s_wave, &tot) + ptot;
    for (int k = 0; k < SCAN_ITEMS; k++) {
        const int64_t idx = base + k;
        if (idx < n) out[idx] = run;
        run += v[k];
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = ptot + tot;
}

template <typename Tin, typename Tout>
void scan_impl(const Tin *in, Tout *out, int64_t n, Tout *total, void *tmp, hipStream_t s) {
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    Tout *partials = reinterpret_cast<Tout *>(tmp);
    if (n > 0 && nb <= SCAN_DIRECT_BLOCKS) {
        hipLaunchKernelGGL((k_scan_reduce<Tin, Tout>), dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, in, n, partials);
        hipLaunchKernelGGL((k_scan_down_direct<Tin, Tout>), dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, in, n,
                           partials, out, total);
        return;
    }
    if (n > 0) hipLaunchKernelGGL((k_scan_reduce<Tin, Tout>), dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, in, n, partials);
    hipLaunchKernelGGL((k_scan_partials<Tout>), dim3(1), dim3(SCAN_THREADS), 0, s, partials, nb, total);
    if (n > 0) hipLaunchKernelGGL((k_scan_down<Tin, Tout>), dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, in, n, partials, out);
}

// ---- key emission -------------------------------------------------------------------

// Bin keys in depth order: rank r holds entry order[r] and owns key positions
// [offsets[r], offsets[r] + ntiles) (the scan of its bin counts in that
// order), its bins row-major over its bin rectangle, as global bin ids.
// Consecutive ranks own consecutive positions, so a wave writes one contiguous
// run of keys: each lane takes positions lane, lane + 64, ... of the run and
// finds its owner among the wave's 64 ranks by binary search over their
// offsets, which keeps the stores coalesced whatever the per-entry tile
// counts are.
__global__ void __launch_bounds__(256) k_emit_sorted(int64_t n, const uint32_t *__restrict__ order, const ViewTable vt,
                                                     const short4 *__restrict__ box,
                                                     const uint32_t *__restrict__ nt_sorted,
                                                     const uint32_t *__restrict__ offsets, int64_t key_cap,
                                                     uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                                     uint32_t *__restrict__ n_emit, uint32_t *__restrict__ ranges,
                                                     int64_t range_words) {
    __shared__ uint32_t s_off[4][64], s_id[4][64], s_nt[4][64];
    __shared__ int32_t s_t0[4][64], s_bw[4][64], s_tx[4][64];
    // the tile ranges start empty: tiles without keys keep [0, 0)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < range_words;
         i += (int64_t)gridDim.x * blockDim.x)
        ranges[i] = 0u;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t r0 = (int64_t)blockIdx.x * blockDim.x + w * 64;
    if (r0 >= n) return;   // wave-uniform
    const int64_t r = r0 + lane;
    uint32_t nt = 0, off = 0xFFFFFFFFu, e = 0;
    uint64_t end = 0;
    if (r < n) {
        e = order[r];
        nt = nt_sorted[r];   // the tiles-touched counts in depth order (read in sequence, not gathered)
        off = offsets[r];
        end = (uint64_t)off + nt;
        // the pairs actually written: all of them when they fit, else those
        // before the one entry whose run crosses the capacity (it and every
        // later entry are dropped whole, so [0, *n_emit) holds no gap)
        if (nt && (uint64_t)off <= (uint64_t)key_cap && (uint64_t)key_cap < end) *n_emit = off;
        if (r == n - 1 && end <= (uint64_t)key_cap) *n_emit = (uint32_t)end;
        if (nt) {
            const int v = view_of_entry(vt, e);
            const short4 b = box[e];
            const int bs = vt.bin_shift;
            const int tx0 = b.x >> bs, ty0 = b.y >> bs;
            s_t0[w][lane] = vt.bin_base[v] + ty0 * vt.bins_x[v] + tx0;
            s_bw[w][lane] = (b.z >> bs) - tx0 + 1;
            s_tx[w][lane] = vt.bins_x[v];
        }
    }
    s_off[w][lane] = off;   // non-decreasing over the valid ranks; the sentinel sorts last
    s_id[w][lane] = e;
    s_nt[w][lane] = nt;
    for (int o = 32; o > 0; o >>= 1) end = max(end, (uint64_t)__shfl_xor((unsigned long long)end, o, 64));
    const uint64_t beg = (uint32_t)__shfl((int)off, 0, 64);   // lane 0 is a valid rank
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint64_t lim = end < (uint64_t)key_cap ? end : (uint64_t)key_cap;
    for (uint64_t pos = beg + lane; pos < lim; pos += 64) {
        // the last rank whose first position is <= pos owns pos (ranks with no
        // tiles share their successor's offset and are passed over)
        int lo = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1)   // probes stay within 1..63
            if ((uint64_t)s_off[w][lo + step] <= pos) lo += step;
        const uint64_t o = s_off[w][lo];
        if (o + s_nt[w][lo] > (uint64_t)key_cap) continue;   // an entry that does not fit is dropped whole
        const uint32_t q = (uint32_t)(pos - o), bw = (uint32_t)s_bw[w][lo];
        const uint32_t qy = q / bw, qx = q - qy * bw;
        keys[pos] = (uint32_t)s_t0[w][lo] + qy * (uint32_t)s_tx[w][lo] + qx;
        vals[pos] = s_id[w][lo];
    }
}

// [start, end) of every bin in the sorted bin keys, written as the range of
// each blend tile of the bin (tiles without keys keep the [0, 0) the caller
// filled).
__device__ __forceinline__ void set_bin_range(const ViewTable &vt, uint32_t bin, int end, uint32_t val,
                                              uint32_t *__restrict__ ranges) {
    if (vt.bin_shift == 4) {   // bins are the tiles
        ranges[2 * bin + end] = val;
        return;
    }
    const int v = view_of_bin(vt, (int)bin);
    const int lb = (int)bin - vt.bin_base[v], bx = lb % vt.bins_x[v], by = lb / vt.bins_x[v];
    const int tx_n = vt.tiles_x[v], ty_n = (vt.tile_base[v + 1] - vt.tile_base[v]) / tx_n;
    const int f = 1 << (vt.bin_shift - 4);
    for (int dy = 0; dy < f; dy++)
        for (int dx = 0; dx < f; dx++) {
            const int tx = bx * f + dx, ty = by * f + dy;
            if (tx < tx_n && ty < ty_n) ranges[2 * (vt.tile_base[v] + ty * tx_n + tx) + end] = val;
        }
}

__global__ void k_ranges(const uint32_t *__restrict__ keys, const uint32_t *n_dev, int64_t cap, int64_t n_bins,
                         const ViewTable vt, uint32_t *__restrict__ ranges) {
    int64_t n = *n_dev;
    if (n > cap) n = cap;
    // four consecutive keys per thread from one 16-byte load (the buffers are
    // 256-byte aligned with slack past their capacity), plus one neighbour on
    // each side; a sentinel stands for "no key" at the ends
    constexpr uint32_t NONE = 0xFFFFFFFFu;
    const int64_t chunks = (n + 3) / 4;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < chunks; c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i0 = 4 * c;
        const uint4 q = *reinterpret_cast<const uint4 *>(keys + i0);
        const uint32_t k[4] = {q.x, q.y, q.z, q.w};
        uint32_t prev = i0 > 0 ? keys[i0 - 1] : NONE;
        const uint32_t after = i0 + 4 < n ? keys[i0 + 4] : NONE;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int64_t i = i0 + j;
            if (i >= n) break;
            const uint32_t t = k[j];
            const uint32_t nx = j < 3 ? (i + 1 < n ? k[j + 1] : NONE) : after;
            if (t < (uint64_t)n_bins) {
                if (prev != t) set_bin_range(vt, t, 0, (uint32_t)i, ranges);
                if (nx != t) set_bin_range(vt, t, 1, (uint32_t)(i + 1), ranges);
            }
            prev = t;
        }
    }
}

template <typename T>
__global__ void k_fill(T *p, T v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fp64_ops(const double *a, const double *b, int64_t n, double *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = sqrt(a[i]);
    out[n + i] = a[i] / b[i];
    out[2 * n + i] = exp(b[i]);
    out[3 * n + i] = log(a[i]);
}

__global__ void k_copy_u32(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

template <typename T>
void fill_impl(T *p, T v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((k_fill<T>), dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
}

}  // namespace

size_t scan_tmp_bytes(int64_t n) { return (size_t)((n + SCAN_TILE - 1) / SCAN_TILE + 1) * 8 + 256; }

void scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total, void *tmp, hipStream_t s) {
    scan_impl<uint32_t, uint32_t>(in, out, n, total, tmp, s);
}
void scan_u8_to_i64(const uint8_t *in, int64_t *out, int64_t n, int64_t *total, void *tmp, hipStream_t s) {
    scan_impl<uint8_t, int64_t>(in, out, n, total, tmp, s);
}
void scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, int64_t *total, void *tmp, hipStream_t s) {
    scan_impl<int32_t, int64_t>(in, out, n, total, tmp, s);
}

void launch_emit_sorted(int64_t n, const uint32_t *order, const ViewTable &vt, const int16_t *box,
                        const uint32_t *nt_sorted, const uint32_t *offsets, int64_t key_cap, uint32_t *keys,
                        uint32_t *vals, uint32_t *n_emit, uint32_t *ranges, int64_t n_tiles, hipStream_t s) {
    if (n == 0) {
        fill_impl<uint32_t>(ranges, 0u, 2 * n_tiles, s);
        fill_impl<uint32_t>(n_emit, 0u, 1, s);
        return;
    }
    hipLaunchKernelGGL(k_emit_sorted, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, order, vt,
                       reinterpret_cast<const short4 *>(box), nt_sorted, offsets, key_cap, keys, vals, n_emit, ranges,
                       2 * n_tiles);
}

void launch_ranges(const uint32_t *keys, const uint32_t *n_dev, int64_t cap, int64_t n_bins, const ViewTable &vt,
                   uint32_t *ranges, hipStream_t s) {
    // the key emission has zeroed the ranges
    hipLaunchKernelGGL(k_ranges, dim3(2048), dim3(256), 0, s, keys, n_dev, cap, n_bins, vt, ranges);
}

void launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s) { fill_impl<uint8_t>(p, v, n, s); }
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) { fill_impl<uint32_t>(p, v, n, s); }
void launch_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s) { fill_impl<uint64_t>(p, v, n, s); }
void launch_fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s) { fill_impl<int64_t>(p, v, n, s); }
void launch_copy_u32(const uint32_t *src, uint32_t *dst, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_copy_u32, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n);
}

void launch_fp64_ops(const double *a, const double *b, int64_t n, double *out, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_fp64_ops, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n, out);
}

AS_WARM_KERNEL(binning)
