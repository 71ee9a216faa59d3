// Tile binning: exclusive scans, (tile | depth) key emission, a stable LSD radix
// sort on 8-bit digits staged through LDS, and per-tile ranges.
//
// The rasterizer composites each pixel over the Gaussians in ascending
// (depth, id) order (Sec. 3, front-to-back blending); sorting the keys
// tile << 32 | float_bits(depth) stably, after emitting them in ascending id
// order, gives every tile its list in exactly that order.
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

template <typename Tin, typename Tout>
void scan_impl(const Tin *in, Tout *out, int64_t n, Tout *total, void *tmp, hipStream_t s) {
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    Tout *partials = reinterpret_cast<Tout *>(tmp);
    if (n > 0) hipLaunchKernelGGL((k_scan_reduce<Tin, Tout>), dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, in, n, partials);
    hipLaunchKernelGGL((k_scan_partials<Tout>), dim3(1), dim3(SCAN_THREADS), 0, s, partials, nb, total);
    if (n > 0) hipLaunchKernelGGL((k_scan_down<Tin, Tout>), dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, in, n, partials, out);
}

// ---- key emission -------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_emit(int64_t n, const uint32_t *__restrict__ depth_key,
                                              const short4 *__restrict__ box, const uint32_t *__restrict__ ntiles,
                                              const uint32_t *__restrict__ offsets, int tiles_x, int64_t key_cap,
                                              uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t nt = ntiles[i];
    if (nt == 0) return;
    const uint64_t off = offsets[i];
    if (off + nt > (uint64_t)key_cap) return;   // over capacity: the count tells the caller
    const short4 b = box[i];
    const uint64_t dk = depth_key[i];
    const int tx0 = b.x / AS_TILE_W, tx1 = b.z / AS_TILE_W, ty0 = b.y / AS_TILE_H, ty1 = b.w / AS_TILE_H;
    uint64_t k = off;
    for (int ty = ty0; ty <= ty1; ty++)
        for (int tx = tx0; tx <= tx1; tx++) {
            keys[k] = ((uint64_t)(ty * tiles_x + tx) << 32) | dk;
            vals[k] = (uint32_t)i;
            k++;
        }
}

// Keys of one Gaussian, emitted in depth order: rank r holds Gaussian order[r]
// and writes its keys at offsets[r] (the scan of ntiles in that order).
__global__ void __launch_bounds__(256) k_emit_sorted(int64_t n, const uint32_t *__restrict__ order,
                                                     const uint32_t *__restrict__ depth_key,
                                                     const short4 *__restrict__ box,
                                                     const uint32_t *__restrict__ ntiles,
                                                     const uint32_t *__restrict__ offsets, int tiles_x, int64_t key_cap,
                                                     uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint32_t i = order[r];
    const uint32_t nt = ntiles[i];
    if (nt == 0) return;
    const uint64_t off = offsets[r];
    if (off + nt > (uint64_t)key_cap) return;   // over capacity: the count tells the caller
    const short4 b = box[i];
    const uint64_t dk = depth_key[i];
    const int tx0 = b.x / AS_TILE_W, tx1 = b.z / AS_TILE_W, ty0 = b.y / AS_TILE_H, ty1 = b.w / AS_TILE_H;
    uint64_t k = off;
    for (int ty = ty0; ty <= ty1; ty++)
        for (int tx = tx0; tx <= tx1; tx++) {
            keys[k] = ((uint64_t)(ty * tiles_x + tx) << 32) | dk;
            vals[k] = i;
            k++;
        }
}

// (depth key, id) pairs of every Gaussian for the depth sort.
__global__ void k_depth_pairs(int64_t n, const uint32_t *__restrict__ depth_key, uint64_t *__restrict__ keys,
                              uint32_t *__restrict__ vals, uint32_t *__restrict__ n32) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *n32 = (uint32_t)n;
    if (i >= n) return;
    keys[i] = depth_key[i];
    vals[i] = (uint32_t)i;
}

__global__ void k_gather_u32(int64_t n, const uint32_t *__restrict__ src, const uint32_t *__restrict__ idx,
                             uint32_t *__restrict__ dst) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) dst[r] = src[idx[r]];
}

// ---- LSD radix sort --------------------------------------------------------------------

constexpr int RS_THREADS = 256;
constexpr int RS_TILE = 1024;   // keys per block iteration: 4 waves x 4 rounds x 64 lanes

__device__ __forceinline__ void rs_chunk(int64_t n, int G, int b, int64_t *beg, int64_t *end) {
    int64_t chunk = (n + G - 1) / G;
    chunk = (chunk + RS_TILE - 1) / RS_TILE * RS_TILE;
    *beg = (int64_t)b * chunk;
    *end = *beg + chunk < n ? *beg + chunk : n;
}

__global__ void __launch_bounds__(RS_THREADS) k_radix_hist(const uint64_t *__restrict__ kin, const uint32_t *n_dev,
                                                           int64_t cap, int shift, uint32_t *__restrict__ hist) {
    __shared__ uint32_t s_h[4][256];
    const int tid = threadIdx.x, w = tid >> 6;
    for (int k = 0; k < 4; k++) s_h[k][tid] = 0;
    __syncthreads();
    int64_t n = *n_dev;
    if (n > cap) n = cap;
    int64_t beg, end;
    rs_chunk(n, gridDim.x, blockIdx.x, &beg, &end);
    for (int64_t idx = beg + tid; idx < end; idx += RS_THREADS) {
        const uint32_t d = (uint32_t)(kin[idx] >> shift) & 255u;
        atomicAdd(&s_h[w][d], 1u);
    }
    __syncthreads();
    hist[(int64_t)tid * gridDim.x + blockIdx.x] = s_h[0][tid] + s_h[1][tid] + s_h[2][tid] + s_h[3][tid];
}

__global__ void __launch_bounds__(RS_THREADS) k_radix_scatter(const uint64_t *__restrict__ kin,
                                                              const uint32_t *__restrict__ vin,
                                                              uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                              const uint32_t *n_dev, int64_t cap, int shift,
                                                              const uint32_t *__restrict__ hist) {
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_cnt[4][256];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    int64_t n = *n_dev;
    if (n > cap) n = cap;
    int64_t beg, end;
    rs_chunk(n, gridDim.x, blockIdx.x, &beg, &end);
    s_base[tid] = hist[(int64_t)tid * gridDim.x + blockIdx.x];
    const uint64_t lt = lanemask_lt();
    for (int64_t t0 = beg; t0 < end; t0 += RS_TILE) {
        for (int k = 0; k < 4; k++) s_cnt[k][tid] = 0;
        __syncthreads();
        uint64_t key[4];
        uint32_t val[4], dig[4], loc[4];
        bool ok[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int64_t idx = t0 + w * 256 + j * 64 + lane;
            ok[j] = idx < end;
            key[j] = ok[j] ? kin[idx] : 0ull;
            val[j] = ok[j] ? vin[idx] : 0u;
            const uint32_t d = (uint32_t)(key[j] >> shift) & 255u;
            dig[j] = d;
            uint64_t peers = __ballot(ok[j]);
#pragma unroll
            for (int bit = 0; bit < 8; bit++) {
                const bool set = (d >> bit) & 1u;
                const uint64_t m = __ballot(set);
                peers &= set ? m : ~m;
            }
            const uint32_t rank = (uint32_t)__popcll(peers & lt);
            const uint32_t before = s_cnt[w][d];
            __builtin_amdgcn_wave_barrier();
            if (ok[j] && rank == 0) s_cnt[w][d] = before + (uint32_t)__popcll(peers);
            __builtin_amdgcn_wave_barrier();
            loc[j] = before + rank;
        }
        __syncthreads();
        {
            const uint32_t c0 = s_cnt[0][tid], c1 = s_cnt[1][tid], c2 = s_cnt[2][tid], c3 = s_cnt[3][tid];
            const uint32_t base = s_base[tid];
            s_cnt[0][tid] = base;
            s_cnt[1][tid] = base + c0;
            s_cnt[2][tid] = base + c0 + c1;
            s_cnt[3][tid] = base + c0 + c1 + c2;
            s_base[tid] = base + c0 + c1 + c2 + c3;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 4; j++) {
            if (ok[j]) {
                const uint32_t pos = s_cnt[w][dig[j]] + loc[j];
                kout[pos] = key[j];
                vout[pos] = val[j];
            }
        }
        __syncthreads();
    }
}

__global__ void k_ranges(const uint64_t *__restrict__ keys, const uint32_t *n_dev, int64_t cap, int64_t n_tiles,
                         uint32_t *__restrict__ ranges) {
    int64_t n = *n_dev;
    if (n > cap) n = cap;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t t = keys[i] >> 32;
        if (t >= (uint64_t)n_tiles) continue;
        if (i == 0 || (keys[i - 1] >> 32) != t) ranges[2 * t] = (uint32_t)i;
        if (i == n - 1 || (keys[i + 1] >> 32) != t) ranges[2 * t + 1] = (uint32_t)(i + 1);
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

void launch_emit_keys(int64_t n, const uint32_t *depth_key, const int16_t *box, const uint32_t *ntiles,
                      const uint32_t *offsets, int tiles_x, int64_t key_cap, uint64_t *keys, uint32_t *vals,
                      hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_emit, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, depth_key,
                       reinterpret_cast<const short4 *>(box), ntiles, offsets, tiles_x, key_cap, keys, vals);
}

static int rs_grid(int64_t n_hint) {
    int64_t g = (n_hint + 8 * RS_TILE - 1) / (8 * RS_TILE);
    if (g < 1) g = 1;
    if (g > 2048) g = 2048;
    return (int)g;
}

size_t sort_hist_bytes(int64_t n_hint) {
    const int64_t G = rs_grid(n_hint);
    return (size_t)(256 * G) * 4 + scan_tmp_bytes(256 * G) + 64;
}

int radix_sort_pairs(uint64_t *keys[2], uint32_t *vals[2], const uint32_t *n_dev, int64_t cap, int64_t n_hint,
                     int key_bits, void *hist, hipStream_t s) {
    return radix_sort_pairs_range(keys, vals, n_dev, cap, n_hint, 0, key_bits, hist, s);
}

int radix_sort_pairs_range(uint64_t *keys[2], uint32_t *vals[2], const uint32_t *n_dev, int64_t cap, int64_t n_hint,
                           int lo_bit, int hi_bit, void *hist, hipStream_t s) {
    const int G = rs_grid(n_hint);
    uint32_t *h = reinterpret_cast<uint32_t *>(hist);
    void *tmp = reinterpret_cast<char *>(hist) + (size_t)(256 * G) * 4;
    int sel = 0;
    for (int shift = lo_bit; shift < hi_bit; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3(G), dim3(RS_THREADS), 0, s, keys[sel], n_dev, cap, shift, h);
        scan_impl<uint32_t, uint32_t>(h, h, (int64_t)256 * G, (uint32_t *)nullptr, tmp, s);
        hipLaunchKernelGGL(k_radix_scatter, dim3(G), dim3(RS_THREADS), 0, s, keys[sel], vals[sel], keys[sel ^ 1],
                           vals[sel ^ 1], n_dev, cap, shift, h);
        sel ^= 1;
    }
    return sel;
}

void launch_depth_pairs(int64_t n, const uint32_t *depth_key, uint64_t *keys, uint32_t *vals, uint32_t *n32,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_depth_pairs, dim3((unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1)), dim3(256), 0, s, n,
                       depth_key, keys, vals, n32);
}

void launch_gather_u32(int64_t n, const uint32_t *src, const uint32_t *idx, uint32_t *dst, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_gather_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, src, idx, dst);
}

void launch_emit_sorted(int64_t n, const uint32_t *order, const uint32_t *depth_key, const int16_t *box,
                        const uint32_t *ntiles, const uint32_t *offsets, int tiles_x, int64_t key_cap, uint64_t *keys,
                        uint32_t *vals, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_emit_sorted, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, order, depth_key,
                       reinterpret_cast<const short4 *>(box), ntiles, offsets, tiles_x, key_cap, keys, vals);
}

void launch_ranges(const uint64_t *keys, const uint32_t *n_dev, int64_t cap, int64_t n_tiles, uint32_t *ranges,
                   hipStream_t s) {
    fill_impl<uint32_t>(ranges, 0u, 2 * n_tiles, s);
    hipLaunchKernelGGL(k_ranges, dim3(2048), dim3(256), 0, s, keys, n_dev, cap, n_tiles, ranges);
}

void launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s) { fill_impl<uint8_t>(p, v, n, s); }
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) { fill_impl<uint32_t>(p, v, n, s); }
void launch_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s) { fill_impl<uint64_t>(p, v, n, s); }
void launch_fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s) { fill_impl<int64_t>(p, v, n, s); }

void launch_fp64_ops(const double *a, const double *b, int64_t n, double *out, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_fp64_ops, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n, out);
}
