// Stable LSD radix sort of (key, u32 value) pairs for gfx950, reduce-then-scan
// organisation: no block ever waits on another.
//
// Keys are taken in tiles of 4096 (256 threads x 16 rounds), or of 2048
// (256 x 8) when the element count hint gives fewer than 512 of the larger
// tiles: one block per CU leaves each CU's loads waiting on each other, two
// overlap.  Each digit pass is three launches:
//   up     per-tile digit counts, from an LDS histogram kept in 8 copies (a
//          lane adds into copy lane % 8, so lanes with equal digits mostly hit
//          different words), stored digit-major: counts[d][tile];
//   scan   one block per digit turns its column into the exclusive prefix
//          over tiles and writes the column's total;
//   down   each tile scans the digit totals for the start of every digit's
//          output range, ranks its keys among equal digits (per wave: RB ballots
//          give the lanes with the same digit; per-wave counters in LDS carry
//          offsets across the wave's rounds, which keeps the sort stable),
//          reorders the tile by digit in LDS and writes each digit's run to its
//          offset, consecutive threads to consecutive addresses.
// All of a tile's loads are issued before the ranking starts: the wave
// barriers of the ranking would otherwise hold every round's loads back
// behind the previous round.
//
// Counts are sized by the capacity the buffers were allocated for and read
// only for the tiles the device-side element count uses, so nothing has to be
// cleared first.  Grids are sized from the host's element count hint (at most
// 4096 blocks); blocks loop over tiles until the device-side count is covered.
//
// Workspace (sort_hist_bytes(cap)): digit totals [256] u32, then counts
// [256][tiles(cap)] u32, sized for the 2048-key tiles and used with the row
// stride of the tile size a sort takes.
//
// 32-bit keys can instead take one launch per digit (single_pass): a first
// kernel counts the digits of every pass over all keys at once; then each
// pass is one kernel whose blocks take tiles in the order of a ticket counter
// and find where each digit of their tile goes by decoupled look-back: a
// tile publishes its digit counts (flag AGG) as soon as it has ranked its
// keys, then walks back over its predecessors' words, adding counts until it
// meets an inclusive prefix (flag INC), and publishes its own inclusive
// prefix.  Flag and count share one 32-bit word, written and read with
// relaxed device-scope atomics, so no fence orders them.  A block waits only
// on tiles whose tickets are lower than its own; those were taken by running
// blocks that publish their counts before they wait on anything, so every
// wait ends.  Waits are bounded all the same (a word polled more than
// OS_SPIN_MAX times raises a flag in the workspace and the block goes on with
// a wrong prefix instead of hanging).  Per sort: one small kernel clears the
// digit counts and tickets, the counting kernel clears the first pass's
// words, and each pass clears the next pass's (two word arrays alternate).
// The counts must stay below 2^30 (two flag bits).
#include "internal.h"

namespace {

constexpr int RS_THREADS = 256;
// Keys per thread and tile: 16 (4096-key tiles), or 8 (2048-key tiles) where
// the larger tiles would give the device fewer than two blocks per CU.
constexpr int RS_ROUNDS_BIG = 16, RS_ROUNDS_SMALL = 8;
constexpr int RS_TILE_MIN = RS_THREADS * RS_ROUNDS_SMALL;
constexpr int64_t RS_SMALL_BELOW = 512;             // 4096-key tiles under which the small tiles are used
constexpr int RS_COPIES = 8;                        // LDS histogram copies of the up pass
constexpr int64_t RS_MAX_BLOCKS = 4096;
constexpr size_t RS_HEAD = 256 * 4;                 // digit totals, bytes

__device__ __forceinline__ int64_t clamp_n(const uint32_t *n_dev, int64_t cap) {
    const int64_t n = *n_dev;
    return n > cap ? cap : n;
}

__device__ __forceinline__ int64_t tiles_of(int64_t n, int64_t tstride, int tile) {
    const int64_t t = (n + tile - 1) / tile;
    return t < tstride ? t : tstride;
}

// Exclusive scan of v over the block's threads (256); returns the prefix.
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t *s_wave) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) s_wave[w] = inc;
    __syncthreads();
    uint32_t pre = 0;
    for (int k = 0; k < w; k++) pre += s_wave[k];
    __syncthreads();
    return pre + inc - v;
}

template <typename K, int RB, int RS_ROUNDS>
__global__ void __launch_bounds__(RS_THREADS) k_rs_up(const K *__restrict__ keys, const uint32_t *n_dev, int64_t cap,
                                                      int shift, uint32_t mask, uint32_t *__restrict__ counts,
                                                      int64_t tstride) {
    constexpr int NB = 1 << RB, HS = NB + 1;   // copy stride: equal digits of different copies sit in different banks
    constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;
    __shared__ uint32_t s_h[RS_COPIES * HS];
    const int tid = threadIdx.x;
    const int64_t n = clamp_n(n_dev, cap);
    const int64_t T = tiles_of(n, tstride, RS_TILE);
    const int cp = (tid & (RS_COPIES - 1)) * HS;
    for (int64_t t = blockIdx.x; t < T; t += gridDim.x) {
        for (int i = tid; i < RS_COPIES * HS; i += RS_THREADS) s_h[i] = 0;
        const int64_t base = t * RS_TILE;
        const int cnt = n - base < RS_TILE ? (int)(n - base) : RS_TILE;
        K k[RS_ROUNDS];
#pragma unroll
        for (int j = 0; j < RS_ROUNDS; j++) {
            const int idx = j * RS_THREADS + tid;
            k[j] = idx < cnt ? keys[base + idx] : (K)0;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < RS_ROUNDS; j++)
            if (j * RS_THREADS + tid < cnt) atomicAdd(&s_h[cp + ((uint32_t)(k[j] >> shift) & mask)], 1u);
        __syncthreads();
        for (int d = tid; d < NB; d += RS_THREADS) {
            uint32_t c = 0;
#pragma unroll
            for (int q = 0; q < RS_COPIES; q++) c += s_h[q * HS + d];
            counts[(int64_t)d * tstride + t] = c;
        }
        __syncthreads();   // the histogram is cleared for the next tile
    }
}

// One block per digit: the column's exclusive prefix over tiles, in place,
// and the column's total.
__global__ void __launch_bounds__(RS_THREADS) k_rs_scan(uint32_t *__restrict__ counts, int64_t tstride,
                                                        const uint32_t *n_dev, int64_t cap, int tile,
                                                        uint32_t *__restrict__ total) {
    constexpr int PER = 8;   // consecutive tiles per thread
    __shared__ uint32_t s_wave[4];
    __shared__ uint32_t s_tot;
    const int tid = threadIdx.x, d = blockIdx.x;
    const int64_t T = tiles_of(clamp_n(n_dev, cap), tstride, tile);
    uint32_t carry = 0;
    uint32_t *col = counts + (int64_t)d * tstride;
    for (int64_t t0 = 0; t0 < T; t0 += RS_THREADS * PER) {
        uint32_t v[PER], sum = 0;
#pragma unroll
        for (int i = 0; i < PER; i++) {
            const int64_t t = t0 + (int64_t)tid * PER + i;
            v[i] = t < T ? col[t] : 0u;
            sum += v[i];
        }
        const uint32_t pre = block_scan_excl(sum, s_wave);
        uint32_t run = carry + pre;
#pragma unroll
        for (int i = 0; i < PER; i++) {
            const int64_t t = t0 + (int64_t)tid * PER + i;
            if (t < T) col[t] = run;
            run += v[i];
        }
        if (tid == RS_THREADS - 1) s_tot = pre + sum;
        __syncthreads();
        carry += s_tot;
        __syncthreads();
    }
    if (tid == 0) total[d] = carry;
}

template <typename K, int RB, int RS_ROUNDS>
__global__ void __launch_bounds__(RS_THREADS, sizeof(K) == 4 ? 3 : 2)
    k_rs_down(const K *__restrict__ kin, const uint32_t *__restrict__ vin, K *__restrict__ kout,
              uint32_t *__restrict__ vout, const uint32_t *n_dev, int64_t cap, int shift, uint32_t mask,
              const uint32_t *__restrict__ offs, const uint32_t *__restrict__ total, int64_t tstride,
              const uint32_t *__restrict__ gsrc, uint32_t *__restrict__ gdst) {
    constexpr int NB = 1 << RB;
    constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;
    __shared__ uint32_t s_wcnt[4][NB];   // per-wave digit counts, then each wave's offset inside the tile's digit run
    __shared__ uint32_t s_boff[NB];      // tile-local start of each digit's run
    __shared__ uint32_t s_gdst[NB];      // output offset of the tile's run of each digit
    __shared__ uint32_t s_wave[4];
    __shared__ K s_key[RS_TILE];
    __shared__ uint32_t s_val[RS_TILE];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t n = clamp_n(n_dev, cap);
    const int64_t T = tiles_of(n, tstride, RS_TILE);
    const uint64_t lt = lanemask_lt();
    for (int64_t tile = blockIdx.x; tile < T; tile += gridDim.x) {
        // the tile's offset in each digit's column and the digit totals are
        // loaded first, so the scan below waits for them alone
        const uint32_t go = tid < NB ? offs[(int64_t)tid * tstride + tile] : 0u;
        const uint32_t tt = tid < NB ? total[tid] : 0u;
        for (int i = tid; i < 4 * NB; i += RS_THREADS) (&s_wcnt[0][0])[i] = 0;
        const int64_t base = tile * RS_TILE;
        const int cnt = n - base < RS_TILE ? (int)(n - base) : RS_TILE;
        // wave w takes keys [w*1024, (w+1)*1024) of the tile, 64 per round
        K key[RS_ROUNDS];
        uint32_t val[RS_ROUNDS], loc[RS_ROUNDS];
#pragma unroll
        for (int j = 0; j < RS_ROUNDS; j++) {
            const int idx = w * (RS_TILE / 4) + j * 64 + lane;
            const bool ok = idx < cnt;
            key[j] = ok ? kin[base + idx] : (K)0;
            val[j] = ok ? vin[base + idx] : 0u;
        }
        const uint32_t gstart = block_scan_excl(tt, s_wave);   // start of each digit's output range
#pragma unroll
        for (int j = 0; j < RS_ROUNDS; j++) {
            const bool ok = w * (RS_TILE / 4) + j * 64 + lane < cnt;
            const uint32_t d = (uint32_t)(key[j] >> shift) & mask;
            uint64_t peers = __ballot(ok);
#pragma unroll
            for (int bit = 0; bit < RB; bit++) {
                const bool set = (d >> bit) & 1u;
                const uint64_t m = __ballot(set);
                peers &= set ? m : ~m;
            }
            const uint32_t rank = (uint32_t)__popcll(peers & lt);
            const uint32_t before = s_wcnt[w][d];
            __builtin_amdgcn_wave_barrier();
            if (ok && rank == 0) s_wcnt[w][d] = before + (uint32_t)__popcll(peers);
            __builtin_amdgcn_wave_barrier();
            loc[j] = before + rank;
        }
        __syncthreads();
        // per digit: tile total, wave offsets, tile-local run starts
        uint32_t tot = 0;
        if (tid < NB) {
            const uint32_t c0 = s_wcnt[0][tid], c1 = s_wcnt[1][tid], c2 = s_wcnt[2][tid], c3 = s_wcnt[3][tid];
            tot = c0 + c1 + c2 + c3;
            s_wcnt[0][tid] = 0;
            s_wcnt[1][tid] = c0;
            s_wcnt[2][tid] = c0 + c1;
            s_wcnt[3][tid] = c0 + c1 + c2;
        }
        const uint32_t boff = block_scan_excl(tot, s_wave);
        if (tid < NB) {
            s_boff[tid] = boff;
            s_gdst[tid] = gstart + go;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < RS_ROUNDS; j++) {
            if (w * (RS_TILE / 4) + j * 64 + lane < cnt) {
                const uint32_t d = (uint32_t)(key[j] >> shift) & mask;
                const uint32_t lp = s_boff[d] + s_wcnt[w][d] + loc[j];
                s_key[lp] = key[j];
                s_val[lp] = val[j];
            }
        }
        __syncthreads();
        for (int i = tid; i < cnt; i += RS_THREADS) {
            const K k = s_key[i];
            const uint32_t d = (uint32_t)(k >> shift) & mask;
            const uint32_t g = s_gdst[d] + (uint32_t)(i - (int)s_boff[d]);
            kout[g] = k;
            vout[g] = s_val[i];
            if (gsrc) gdst[g] = gsrc[s_val[i]];   // optional gather through the sorted values
        }
        __syncthreads();   // the LDS of this tile is free for the next
    }
}

// ---- one launch per digit (32-bit keys) ----------------------------------------------

constexpr int OS_MAX_PASSES = 8;                    // 32 bits in digits of at least 4 bits
constexpr uint32_t OS_AGG = 1u << 30, OS_INC = 2u << 30, OS_VAL = OS_AGG - 1u;
constexpr int OS_SPIN_MAX = 1 << 22;
constexpr int OS_WINDOW = 16;                       // predecessors read per look-back step
// head: digit counts [passes][256], tickets [passes], the wait-limit flag
constexpr size_t OS_HEAD = ((size_t)OS_MAX_PASSES * 256 + OS_MAX_PASSES + 1) * 4 + 220;
constexpr int OS_TICKET = OS_MAX_PASSES * 256, OS_ERR = OS_TICKET + OS_MAX_PASSES;

__global__ void __launch_bounds__(256) k_os_init(uint32_t *__restrict__ head, int passes) {
    for (int i = threadIdx.x; i < passes * 256; i += 256) head[i] = 0u;
    if (threadIdx.x < passes) head[OS_TICKET + threadIdx.x] = 0u;
}

// Digit counts of every pass over all keys (LDS histograms in RS_COPIES
// copies, then one device atomic per nonzero (pass, digit) per block), and
// the first pass's look-back words cleared for the tiles in use.
template <int RB>
__global__ void __launch_bounds__(256) k_os_hist(const uint32_t *__restrict__ keys, const uint32_t *n_dev, int64_t cap,
                                                 int lo, int hi, uint32_t *__restrict__ head,
                                                 uint32_t *__restrict__ st0, int tile) {
    constexpr int NB = 1 << RB, HS = NB + 1;
    extern __shared__ uint32_t s_h[];   // [RS_COPIES][passes][HS]
    const int tid = threadIdx.x;
    const int P = (hi - lo + RB - 1) / RB;
    const int64_t n = clamp_n(n_dev, cap);
    for (int i = tid; i < RS_COPIES * P * HS; i += 256) s_h[i] = 0u;
    __syncthreads();
    uint32_t *h = s_h + (tid & (RS_COPIES - 1)) * P * HS;
    auto add = [&](uint32_t k) {
        for (int p = 0; p < P; p++) {
            const int sh = lo + p * RB;
            const int wd = hi - sh < RB ? hi - sh : RB;
            atomicAdd(&h[p * HS + ((k >> sh) & ((1u << wd) - 1u))], 1u);
        }
    };
    const int64_t gt = (int64_t)blockIdx.x * 256 + tid, gs = (int64_t)gridDim.x * 256;
    const int64_t n4 = n >> 2;
    const uint4 *k4 = reinterpret_cast<const uint4 *>(keys);
    for (int64_t i = gt; i < n4; i += gs) {
        const uint4 v = k4[i];
        add(v.x);
        add(v.y);
        add(v.z);
        add(v.w);
    }
    for (int64_t i = (n4 << 2) + gt; i < n; i += gs) add(keys[i]);
    const int64_t T = (n + tile - 1) / tile;
    for (int64_t i = gt; i < T * NB; i += gs) st0[i] = 0u;
    __syncthreads();
    for (int i = tid; i < P * NB; i += 256) {
        const int p = i / NB, d = i - p * NB;
        uint32_t c = 0;
#pragma unroll
        for (int q = 0; q < RS_COPIES; q++) c += s_h[(q * P + p) * HS + d];
        if (c) atomicAdd(&head[p * 256 + d], c);
    }
}

// One digit pass.  st: this pass's look-back words [tiles][NB]; st_next: the
// next pass's, cleared here for the tiles in use.
template <int RB, int ROUNDS>
__global__ void __launch_bounds__(RS_THREADS, ROUNDS >= 32 ? 1 : 2)
    k_os_pass(const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
              uint32_t *__restrict__ vout, const uint32_t *n_dev, int64_t cap, int shift, uint32_t mask,
              uint32_t *__restrict__ head, int pass, uint32_t *st, uint32_t *__restrict__ st_next,
              const uint32_t *__restrict__ gsrc, uint32_t *__restrict__ gdst) {
    constexpr int NB = 1 << RB;
    constexpr int TILE = RS_THREADS * ROUNDS;
    __shared__ uint32_t s_wcnt[4][NB];
    __shared__ uint32_t s_boff[NB];
    __shared__ uint32_t s_gdst[NB];
    __shared__ uint32_t s_wave[4];
    __shared__ uint32_t s_key[TILE];
    __shared__ uint32_t s_val[TILE];
    __shared__ uint32_t s_tile;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t n = clamp_n(n_dev, cap);
    const int64_t T = (n + TILE - 1) / TILE;
    const uint64_t lt = lanemask_lt();
    // the start of each digit's output range, the same for every tile
    const uint32_t gstart = block_scan_excl(tid < NB ? head[pass * 256 + tid] : 0u, s_wave);
    for (;;) {
        if (tid == 0) s_tile = atomicAdd(&head[OS_TICKET + pass], 1u);
        for (int i = tid; i < 4 * NB; i += RS_THREADS) (&s_wcnt[0][0])[i] = 0u;
        __syncthreads();
        const int64_t tile = s_tile;
        if (tile >= T) break;   // every thread reads the same ticket
        const int64_t base = tile * TILE;
        const int cnt = n - base < TILE ? (int)(n - base) : TILE;
        uint32_t key[ROUNDS], val[ROUNDS], loc[ROUNDS];
#pragma unroll
        for (int j = 0; j < ROUNDS; j++) {
            const int idx = w * (TILE / 4) + j * 64 + lane;
            const bool ok = idx < cnt;
            key[j] = ok ? kin[base + idx] : 0u;
            val[j] = ok ? vin[base + idx] : 0u;
        }
#pragma unroll
        for (int j = 0; j < ROUNDS; j++) {
            const bool ok = w * (TILE / 4) + j * 64 + lane < cnt;
            const uint32_t d = (key[j] >> shift) & mask;
            uint64_t peers = __ballot(ok);
#pragma unroll
            for (int bit = 0; bit < RB; bit++) {
                const bool set = (d >> bit) & 1u;
                const uint64_t m = __ballot(set);
                peers &= set ? m : ~m;
            }
            const uint32_t rank = (uint32_t)__popcll(peers & lt);
            const uint32_t before = s_wcnt[w][d];
            __builtin_amdgcn_wave_barrier();
            if (ok && rank == 0) s_wcnt[w][d] = before + (uint32_t)__popcll(peers);
            __builtin_amdgcn_wave_barrier();
            loc[j] = before + rank;
        }
        __syncthreads();
        uint32_t tot = 0;
        if (tid < NB) {
            const uint32_t c0 = s_wcnt[0][tid], c1 = s_wcnt[1][tid], c2 = s_wcnt[2][tid], c3 = s_wcnt[3][tid];
            tot = c0 + c1 + c2 + c3;
            s_wcnt[0][tid] = 0;
            s_wcnt[1][tid] = c0;
            s_wcnt[2][tid] = c0 + c1;
            s_wcnt[3][tid] = c0 + c1 + c2;
            __hip_atomic_store(&st[tile * NB + tid], (tile == 0 ? OS_INC : OS_AGG) | tot, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        const uint32_t boff = block_scan_excl(tot, s_wave);
        if (tid < NB) s_boff[tid] = boff;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < ROUNDS; j++) {
            if (w * (TILE / 4) + j * 64 + lane < cnt) {
                const uint32_t d = (key[j] >> shift) & mask;
                const uint32_t lp = s_boff[d] + s_wcnt[w][d] + loc[j];
                s_key[lp] = key[j];
                s_val[lp] = val[j];
            }
        }
        if (tid < NB) {
            // look-back: OS_WINDOW predecessors per step, newest first; add
            // counts up to the first inclusive prefix, re-read from the first
            // word not yet published
            uint32_t excl = 0;
            int64_t k = tile - 1;
            int spins = 0;
            bool done = tile == 0;
            while (!done) {
                uint32_t v[OS_WINDOW];
#pragma unroll
                for (int i = 0; i < OS_WINDOW; i++)
                    v[i] = k - i >= 0 ? __hip_atomic_load(&st[(k - i) * NB + tid], __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT)
                                      : OS_INC;
                int used = 0;
#pragma unroll
                for (int i = 0; i < OS_WINDOW; i++) {
                    if (done || used < i) break;
                    const uint32_t f = v[i] & ~OS_VAL;
                    if (f == 0u) break;
                    excl += v[i] & OS_VAL;
                    used = i + 1;
                    done = f == OS_INC;
                }
                k -= used;
                if (!done && used == 0) {
                    if (++spins > OS_SPIN_MAX) {
                        atomicOr(&head[OS_ERR], 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            if (tile > 0)
                __hip_atomic_store(&st[tile * NB + tid], OS_INC | (excl + tot), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            s_gdst[tid] = gstart + excl;
            if (st_next) st_next[tile * NB + tid] = 0u;
        }
        __syncthreads();
        for (int i = tid; i < cnt; i += RS_THREADS) {
            const uint32_t k = s_key[i];
            const uint32_t d = (k >> shift) & mask;
            const uint32_t g = s_gdst[d] + (uint32_t)(i - (int)s_boff[d]);
            kout[g] = k;
            vout[g] = s_val[i];
            if (gsrc) gdst[g] = gsrc[s_val[i]];
        }
        __syncthreads();   // LDS and s_tile are free for the next tile
    }
}

int64_t rs_tiles(int64_t n, int tile) { return (n + tile - 1) / tile > 0 ? (n + tile - 1) / tile : 1; }

constexpr int OS_TILE_MIN = RS_THREADS * 16;        // the look-back words are sized for 4096-key tiles
constexpr int64_t OS_BIG_TILES_BELOW = 1 << 21;     // fewer keys: 8192-key tiles (shorter look-back chains)
constexpr int64_t OS_MAX_BLOCKS = 1024;

size_t os_words_bytes(int64_t cap) { return (size_t)rs_tiles(cap, OS_TILE_MIN) * 256 * 4; }

template <int RB, int R>
void os_pass_r(uint32_t *ki, uint32_t *vi, uint32_t *ko, uint32_t *vo, const uint32_t *n_dev, int64_t cap, int64_t nh,
               int shift, uint32_t mask, uint32_t *head, int pass, uint32_t *st, uint32_t *st_next,
               const uint32_t *gsrc, uint32_t *gdst, hipStream_t s) {
    int64_t grid = rs_tiles(nh, RS_THREADS * R);
    if (grid > OS_MAX_BLOCKS) grid = OS_MAX_BLOCKS;
    hipLaunchKernelGGL((k_os_pass<RB, R>), dim3((unsigned)grid), dim3(RS_THREADS), 0, s, ki, vi, ko, vo, n_dev, cap,
                       shift, mask, head, pass, st, st_next, gsrc, gdst);
}

template <int RB>
int os_sort(uint32_t *keys[2], uint32_t *vals[2], const uint32_t *n_dev, int64_t cap, int64_t nh, int lo_bit,
            int hi_bit, void *ws, const uint32_t *gsrc, uint32_t *gdst, hipStream_t s) {
    uint32_t *head = reinterpret_cast<uint32_t *>(ws);
    uint32_t *words[2] = {reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(ws) + OS_HEAD),
                          reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(ws) + OS_HEAD + os_words_bytes(cap))};
    const int P = (hi_bit - lo_bit + RB - 1) / RB;
    const bool big = nh < OS_BIG_TILES_BELOW;
    const int tile = RS_THREADS * (big ? 32 : 16);
    hipLaunchKernelGGL(k_os_init, dim3(1), dim3(256), 0, s, head, P);
    int64_t hg = (nh + 8191) / 8192;
    hg = hg < 1 ? 1 : (hg > 512 ? 512 : hg);
    const size_t lds = (size_t)RS_COPIES * P * ((1 << RB) + 1) * 4;
    hipLaunchKernelGGL((k_os_hist<RB>), dim3((unsigned)hg), dim3(256), lds, s, keys[0], n_dev, cap, lo_bit, hi_bit,
                       head, words[0], tile);
    int sel = 0;
    for (int p = 0; p < P; p++) {
        const int sh = lo_bit + p * RB;
        const int wdt = hi_bit - sh < RB ? hi_bit - sh : RB;
        const uint32_t mask = (1u << wdt) - 1u;
        const bool last = p == P - 1;
        uint32_t *st = words[p & 1], *stn = last ? nullptr : words[(p + 1) & 1];
        if (big)
            os_pass_r<RB, 32>(keys[sel], vals[sel], keys[sel ^ 1], vals[sel ^ 1], n_dev, cap, nh, sh, mask, head, p, st,
                              stn, last ? gsrc : nullptr, last ? gdst : nullptr, s);
        else
            os_pass_r<RB, 16>(keys[sel], vals[sel], keys[sel ^ 1], vals[sel ^ 1], n_dev, cap, nh, sh, mask, head, p, st,
                              stn, last ? gsrc : nullptr, last ? gdst : nullptr, s);
        sel ^= 1;
    }
    return sel;
}

template <typename K, int RB, int R>
void rs_pass_r(K *ki, uint32_t *vi, K *ko, uint32_t *vo, const uint32_t *n_dev, int64_t cap, int64_t grid, int shift,
               uint32_t mask, uint32_t *total, uint32_t *counts, int64_t tstride, const uint32_t *gsrc, uint32_t *gdst,
               hipStream_t s) {
    hipLaunchKernelGGL((k_rs_up<K, RB, R>), dim3((unsigned)grid), dim3(RS_THREADS), 0, s, ki, n_dev, cap, shift, mask,
                       counts, tstride);
    hipLaunchKernelGGL(k_rs_scan, dim3(1u << RB), dim3(RS_THREADS), 0, s, counts, tstride, n_dev, cap,
                       RS_THREADS * R, total);
    hipLaunchKernelGGL((k_rs_down<K, RB, R>), dim3((unsigned)grid), dim3(RS_THREADS), 0, s, ki, vi, ko, vo, n_dev,
                       cap, shift, mask, counts, total, tstride, gsrc, gdst);
}

template <typename K, int RB>
void rs_pass(bool small, K *ki, uint32_t *vi, K *ko, uint32_t *vo, const uint32_t *n_dev, int64_t cap, int64_t grid,
             int shift, uint32_t mask, uint32_t *total, uint32_t *counts, int64_t tstride, const uint32_t *gsrc,
             uint32_t *gdst, hipStream_t s) {
    if (small)
        rs_pass_r<K, RB, RS_ROUNDS_SMALL>(ki, vi, ko, vo, n_dev, cap, grid, shift, mask, total, counts, tstride, gsrc,
                                          gdst, s);
    else
        rs_pass_r<K, RB, RS_ROUNDS_BIG>(ki, vi, ko, vo, n_dev, cap, grid, shift, mask, total, counts, tstride, gsrc,
                                        gdst, s);
}

template <typename K>
int rs_sort(K *keys[2], uint32_t *vals[2], const uint32_t *n_dev, int64_t cap, int64_t n_hint, int lo_bit, int hi_bit,
            int rb, void *ws, const uint32_t *gsrc, uint32_t *gdst, hipStream_t s) {
    if (rb < 4) rb = 4;
    if (rb > 8) rb = 8;
    const int kbits = (int)sizeof(K) * 8;
    if (hi_bit > kbits) hi_bit = kbits;
    const int64_t nh = n_hint < cap ? n_hint : cap;
    const bool small = rs_tiles(nh, RS_THREADS * RS_ROUNDS_BIG) < RS_SMALL_BELOW;
    const int tile = RS_THREADS * (small ? RS_ROUNDS_SMALL : RS_ROUNDS_BIG);
    const int64_t tstride = rs_tiles(cap, tile);   // within the workspace: sized for the smallest tile
    int64_t grid = rs_tiles(nh, tile);
    if (grid > RS_MAX_BLOCKS) grid = RS_MAX_BLOCKS;
    uint32_t *total = reinterpret_cast<uint32_t *>(ws);
    uint32_t *counts = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(ws) + RS_HEAD);
    int sel = 0;
    for (int sh = lo_bit; sh < hi_bit; sh += rb) {
        const int wdt = hi_bit - sh < rb ? hi_bit - sh : rb;   // the last digit holds only the bits that are left
        const uint32_t mask = (1u << wdt) - 1u;
        K *ki = keys[sel], *ko = keys[sel ^ 1];
        uint32_t *vi = vals[sel], *vo = vals[sel ^ 1];
        const bool last = sh + rb >= hi_bit;
        const uint32_t *gs = last ? gsrc : nullptr;
        uint32_t *gd = last ? gdst : nullptr;
        switch (rb) {
        case 4: rs_pass<K, 4>(small, ki, vi, ko, vo, n_dev, cap, grid, sh, mask, total, counts, tstride, gs, gd, s); break;
        case 5: rs_pass<K, 5>(small, ki, vi, ko, vo, n_dev, cap, grid, sh, mask, total, counts, tstride, gs, gd, s); break;
        case 6: rs_pass<K, 6>(small, ki, vi, ko, vo, n_dev, cap, grid, sh, mask, total, counts, tstride, gs, gd, s); break;
        case 7: rs_pass<K, 7>(small, ki, vi, ko, vo, n_dev, cap, grid, sh, mask, total, counts, tstride, gs, gd, s); break;
        default: rs_pass<K, 8>(small, ki, vi, ko, vo, n_dev, cap, grid, sh, mask, total, counts, tstride, gs, gd, s); break;
        }
        sel ^= 1;
    }
    return sel;
}

}  // namespace

size_t sort_hist_bytes(int64_t cap) {
    const size_t rts = RS_HEAD + (size_t)rs_tiles(cap, RS_TILE_MIN) * 256 * 4 + 256;
    const size_t os = OS_HEAD + 2 * os_words_bytes(cap);
    return rts > os ? rts : os;
}

bool sort_single_pass_ok(int64_t cap) { return cap < (int64_t)OS_VAL; }

int radix_sort_u32(uint32_t *keys[2], uint32_t *vals[2], const uint32_t *n_dev, int64_t cap, int64_t n_hint, int lo_bit,
                   int hi_bit, int radix_bits, void *hist, hipStream_t s, const uint32_t *gather_src,
                   uint32_t *gather_dst, bool single_pass) {
    if (single_pass && sort_single_pass_ok(cap) && hi_bit > lo_bit) {
        int rb = radix_bits < 4 ? 4 : (radix_bits > 8 ? 8 : radix_bits);
        if (hi_bit > 32) hi_bit = 32;
        if ((hi_bit - lo_bit + rb - 1) / rb > OS_MAX_PASSES) rb = 8;
        const int64_t nh = n_hint < cap ? n_hint : cap;
        switch (rb) {
        case 4: return os_sort<4>(keys, vals, n_dev, cap, nh, lo_bit, hi_bit, hist, gather_src, gather_dst, s);
        case 5: return os_sort<5>(keys, vals, n_dev, cap, nh, lo_bit, hi_bit, hist, gather_src, gather_dst, s);
        case 6: return os_sort<6>(keys, vals, n_dev, cap, nh, lo_bit, hi_bit, hist, gather_src, gather_dst, s);
        case 7: return os_sort<7>(keys, vals, n_dev, cap, nh, lo_bit, hi_bit, hist, gather_src, gather_dst, s);
        default: return os_sort<8>(keys, vals, n_dev, cap, nh, lo_bit, hi_bit, hist, gather_src, gather_dst, s);
        }
    }
    return rs_sort<uint32_t>(keys, vals, n_dev, cap, n_hint, lo_bit, hi_bit, radix_bits, hist, gather_src, gather_dst,
                             s);
}

uint32_t sort_wait_flag_offset() { return OS_ERR * 4; }

int radix_sort_u64(uint64_t *keys[2], uint32_t *vals[2], const uint32_t *n_dev, int64_t cap, int64_t n_hint, int lo_bit,
                   int hi_bit, int radix_bits, void *hist, hipStream_t s) {
    return rs_sort<uint64_t>(keys, vals, n_dev, cap, n_hint, lo_bit, hi_bit, radix_bits, hist, nullptr, nullptr, s);
}

AS_WARM_KERNEL(radix)
