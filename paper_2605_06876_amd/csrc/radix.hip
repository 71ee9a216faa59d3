// Stable LSD radix sort of (key, u32 value) pairs with one scatter launch per
// digit ("onesweep" organisation) for gfx950.
//
// 1. One read of the keys builds the global digit histogram of every pass.
// 2. Each pass is a single kernel.  Blocks claim tiles of 4096 consecutive
//    keys in order from an atomic counter.  A block ranks its keys among equal
//    digits (per wave: RB ballots give the lanes with the same digit; per-wave
//    digit counters in LDS carry offsets across the wave's 16 rounds), then
//    publishes its per-digit counts and looks back over the earlier tiles'
//    published counts (decoupled look-back) for the number of keys of each
//    digit that precede the tile.  Keys are reordered by digit in LDS and
//    written out so that consecutive threads write consecutive addresses of a
//    digit's run.
//
// Forward progress of the look-back: a block waits only on tiles claimed
// before its own, whose blocks are already resident and publish their counts
// without waiting on anything; so every wait ends.
//
// Workspace (sort_hist_bytes): digit histograms [16][256] u32, tile counters
// [16] u32, tile status [passes][tiles][2^RB] u64 (2 flag bits: aggregate /
// inclusive prefix; 62 count bits).  Every sort first clears the histograms,
// counters and the status rows its device-side element count will use.  The
// grids are sized for the buffers' capacity, but launch at most 4096 blocks,
// which take tiles until the device-side count is exhausted.
#include "internal.h"

namespace {

constexpr int OS_THREADS = 256;
constexpr int OS_ROUNDS = 16;                       // rounds of 64 keys per wave
constexpr int OS_TILE = OS_THREADS * OS_ROUNDS;     // 4096 keys per tile
constexpr int OS_MAXP = 16;                         // passes (64 bits at 4 bits per digit)
constexpr unsigned long long OS_AGG = 1ull << 62;
constexpr unsigned long long OS_INC = 2ull << 62;
constexpr unsigned long long OS_VAL = (1ull << 62) - 1;
constexpr size_t OS_HEAD = (OS_MAXP * 256 + OS_MAXP) * 4;   // histograms + counters, bytes

struct Passes {
    int n;
    int shift[OS_MAXP];
    uint32_t mask[OS_MAXP];
};

template <typename K>
__device__ __forceinline__ int64_t clamp_n(const uint32_t *n_dev, int64_t cap) {
    const int64_t n = *n_dev;
    return n > cap ? cap : n;
}

// Global digit histograms of all passes: per-wave LDS histograms, then one
// global atomic per nonzero bucket and block.
template <typename K, int RB>
__global__ void __launch_bounds__(OS_THREADS) k_os_hist(const K *__restrict__ keys, const uint32_t *n_dev, int64_t cap,
                                                        const Passes ps, uint32_t *__restrict__ ghist) {
    constexpr int NB = 1 << RB;
    constexpr int NH = (64 + RB - 1) / RB * NB;   // passes x buckets of a 64-bit key, the most there can be
    __shared__ uint32_t s_h[4][NH];
    const int tid = threadIdx.x, w = tid >> 6;
    for (int i = tid; i < 4 * NH; i += OS_THREADS) (&s_h[0][0])[i] = 0;
    __syncthreads();
    const int64_t n = clamp_n<K>(n_dev, cap);
    for (int64_t i = (int64_t)blockIdx.x * OS_THREADS + tid; i < n; i += (int64_t)gridDim.x * OS_THREADS) {
        const K k = keys[i];
        for (int p = 0; p < ps.n; p++) atomicAdd(&s_h[w][p * NB + (uint32_t)((k >> ps.shift[p]) & ps.mask[p])], 1u);
    }
    __syncthreads();
    for (int i = tid; i < ps.n * NB; i += OS_THREADS) {
        const uint32_t c = s_h[0][i] + s_h[1][i] + s_h[2][i] + s_h[3][i];
        if (c) atomicAdd(&ghist[(i / NB) * 256 + (i % NB)], c);
    }
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

template <typename K, int RB>
__global__ void __launch_bounds__(OS_THREADS, 3) k_os_scatter(const K *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                           K *__restrict__ kout, uint32_t *__restrict__ vout,
                                                           const uint32_t *n_dev, int64_t cap, int shift, uint32_t mask,
                                                           const uint32_t *__restrict__ ghist,
                                                           unsigned long long *status, uint32_t *counter) {
    constexpr int NB = 1 << RB;
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wcnt[4][NB];   // per-wave digit counts, then each wave's offset inside the block's digit run
    __shared__ uint32_t s_boff[NB];      // block-local start of each digit's run
    __shared__ uint32_t s_gdst[NB];      // global start of this block's run of each digit
    __shared__ uint32_t s_wave[4];
    __shared__ K s_key[OS_TILE];
    __shared__ uint32_t s_val[OS_TILE];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t n = clamp_n<K>(n_dev, cap);
    // the grid is sized for the largest count the buffers hold; blocks take
    // tiles until the device-side count is exhausted
    for (;;) {
    if (tid == 0) s_tile = atomicAdd(counter, 1u);
    for (int i = tid; i < 4 * NB; i += OS_THREADS) (&s_wcnt[0][0])[i] = 0;
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t base = (int64_t)tile * OS_TILE;
    if (base >= n) break;   // block-uniform; every later tile is empty too
    const int cnt = n - base < OS_TILE ? (int)(n - base) : OS_TILE;

    // rank: wave w takes keys [w*1024, (w+1)*1024) of the tile, 64 per round
    const uint64_t lt = lanemask_lt();
    K key[OS_ROUNDS];
    uint32_t val[OS_ROUNDS], loc[OS_ROUNDS];
#pragma unroll
    for (int j = 0; j < OS_ROUNDS; j++) {
        const int idx = w * (OS_TILE / 4) + j * 64 + lane;
        const bool ok = idx < cnt;
        key[j] = ok ? kin[base + idx] : (K)0;
        val[j] = ok ? vin[base + idx] : 0u;
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

    // per digit: block total, wave offsets, block-local run starts
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
    const uint32_t gh = tid < NB ? ghist[tid] : 0u;
    const uint32_t gbase = block_scan_excl(gh, s_wave);   // global start of each digit
    if (tid < NB) {
        s_boff[tid] = boff;
        unsigned long long *st = status + (size_t)tile * NB + tid;
        uint64_t excl = 0;
        if (tile == 0) {
            __hip_atomic_store(st, OS_INC | (unsigned long long)tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(st, OS_AGG | (unsigned long long)tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // look back over the earlier tiles of this digit; the spin bound
            // only guards against a broken invariant (the wait is short)
            uint32_t spins = 0;
            for (int64_t t = (int64_t)tile - 1; t >= 0;) {
                const unsigned long long v =
                    __hip_atomic_load(status + (size_t)t * NB + tid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((v & ~OS_VAL) == 0) {   // not published yet: that tile's block is resident, wait
                    if (++spins > (1u << 22)) break;
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                excl += v & OS_VAL;
                if ((v & ~OS_VAL) == OS_INC) break;
                t--;
            }
            __hip_atomic_store(st, OS_INC | (unsigned long long)(excl + tot), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        s_gdst[tid] = gbase + (uint32_t)excl;
    }
    __syncthreads();

    // reorder by digit in LDS
#pragma unroll
    for (int j = 0; j < OS_ROUNDS; j++) {
        const int idx = w * (OS_TILE / 4) + j * 64 + lane;
        if (idx < cnt) {
            const uint32_t d = (uint32_t)(key[j] >> shift) & mask;
            const uint32_t lp = s_boff[d] + s_wcnt[w][d] + loc[j];
            s_key[lp] = key[j];
            s_val[lp] = val[j];
        }
    }
    __syncthreads();
    // write out: consecutive threads, consecutive addresses within a digit's run
    for (int i = tid; i < cnt; i += OS_THREADS) {
        const K k = s_key[i];
        const uint32_t d = (uint32_t)(k >> shift) & mask;
        const uint32_t g = s_gdst[d] + (uint32_t)(i - (int)s_boff[d]);
        kout[g] = k;
        vout[g] = s_val[i];
    }
    __syncthreads();   // the LDS of this tile is free for the next
    }
}

// Clear the histograms, tile counters and the status rows the device-side
// count will use (not the whole table sized for the capacity).
__global__ void k_os_clear(uint32_t *__restrict__ head, unsigned long long *__restrict__ status, int64_t per_pass,
                           int passes, int nb, const uint32_t *n_dev, int64_t cap) {
    const int64_t n = clamp_n<uint32_t>(n_dev, cap);
    const int64_t rows = ((n + OS_TILE - 1) / OS_TILE) * nb;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < (int64_t)(OS_HEAD / 4); i += stride) head[i] = 0u;
    for (int64_t i = tid; i < rows * passes; i += stride) status[(i / rows) * per_pass + i % rows] = 0ull;
}

int64_t os_tiles(int64_t n_hint) { return (n_hint + OS_TILE - 1) / OS_TILE > 0 ? (n_hint + OS_TILE - 1) / OS_TILE : 1; }

constexpr int64_t OS_MAX_BLOCKS = 4096;   // blocks of a scatter launch; each takes tiles until none are left

template <typename K, int RB>
void os_scatter(K *ki, uint32_t *vi, K *ko, uint32_t *vo, const uint32_t *n_dev, int64_t cap, int64_t tiles, int shift,
                uint32_t mask, const uint32_t *gh, unsigned long long *st, uint32_t *ctr, hipStream_t s) {
    const int64_t g = tiles < OS_MAX_BLOCKS ? tiles : OS_MAX_BLOCKS;
    hipLaunchKernelGGL((k_os_scatter<K, RB>), dim3((unsigned)g), dim3(OS_THREADS), 0, s, ki, vi, ko, vo, n_dev, cap,
                       shift, mask, gh, st, ctr);
}

template <typename K, int RB>
void os_hist(const K *keys, const uint32_t *n_dev, int64_t cap, int64_t tiles, const Passes &ps, uint32_t *gh,
             hipStream_t s) {
    const int64_t g = tiles < 1024 ? tiles : 1024;
    hipLaunchKernelGGL((k_os_hist<K, RB>), dim3((unsigned)g), dim3(OS_THREADS), 0, s, keys, n_dev, cap, ps, gh);
}

template <typename K>
int onesweep(K *keys[2], uint32_t *vals[2], const uint32_t *n_dev, int64_t cap, int64_t n_hint, int lo_bit, int hi_bit,
             int rb, void *ws, hipStream_t s) {
    if (rb < 4) rb = 4;
    if (rb > 8) rb = 8;
    const int kbits = (int)sizeof(K) * 8;
    if (hi_bit > kbits) hi_bit = kbits;
    Passes ps;
    ps.n = 0;
    int width[OS_MAXP];
    for (int sh = lo_bit; sh < hi_bit && ps.n < OS_MAXP; sh += rb) {
        const int wdt = hi_bit - sh < rb ? hi_bit - sh : rb;   // the last digit holds only the bits that are left
        ps.shift[ps.n] = sh;
        ps.mask[ps.n] = (1u << wdt) - 1u;
        width[ps.n] = wdt;
        ps.n++;
    }
    if (ps.n == 0) return 0;
    const int64_t tiles = os_tiles(n_hint);
    uint32_t *gh = reinterpret_cast<uint32_t *>(ws);
    uint32_t *ctr = gh + OS_MAXP * 256;
    unsigned long long *st = reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(ws) + OS_HEAD);
    const int64_t per_pass = tiles << rb;
    {
        int64_t cb = (tiles * ps.n << rb) / 256 + 1;
        if (cb > 2048) cb = 2048;
        hipLaunchKernelGGL(k_os_clear, dim3((unsigned)cb), dim3(256), 0, s, gh, st, per_pass, ps.n, 1 << rb, n_dev, cap);
    }
    switch (rb) {
    case 4: os_hist<K, 4>(keys[0], n_dev, cap, tiles, ps, gh, s); break;
    case 5: os_hist<K, 5>(keys[0], n_dev, cap, tiles, ps, gh, s); break;
    case 6: os_hist<K, 6>(keys[0], n_dev, cap, tiles, ps, gh, s); break;
    case 7: os_hist<K, 7>(keys[0], n_dev, cap, tiles, ps, gh, s); break;
    default: os_hist<K, 8>(keys[0], n_dev, cap, tiles, ps, gh, s); break;
    }
    int sel = 0;
    for (int p = 0; p < ps.n; p++) {
        K *ki = keys[sel], *ko = keys[sel ^ 1];
        uint32_t *vi = vals[sel], *vo = vals[sel ^ 1];
        unsigned long long *stp = st + p * per_pass;
        const uint32_t *ghp = gh + p * 256;
        // the status rows of pass p are 2^rb wide whatever the digit width
        switch (rb) {
        case 4: os_scatter<K, 4>(ki, vi, ko, vo, n_dev, cap, tiles, ps.shift[p], ps.mask[p], ghp, stp, ctr + p, s); break;
        case 5: os_scatter<K, 5>(ki, vi, ko, vo, n_dev, cap, tiles, ps.shift[p], ps.mask[p], ghp, stp, ctr + p, s); break;
        case 6: os_scatter<K, 6>(ki, vi, ko, vo, n_dev, cap, tiles, ps.shift[p], ps.mask[p], ghp, stp, ctr + p, s); break;
        case 7: os_scatter<K, 7>(ki, vi, ko, vo, n_dev, cap, tiles, ps.shift[p], ps.mask[p], ghp, stp, ctr + p, s); break;
        default: os_scatter<K, 8>(ki, vi, ko, vo, n_dev, cap, tiles, ps.shift[p], ps.mask[p], ghp, stp, ctr + p, s); break;
        }
        (void)width;
        sel ^= 1;
    }
    return sel;
}

}  // namespace

size_t sort_hist_bytes(int64_t n_hint) {
    // the largest status table over digit widths 4..8 and keys up to 64 bits:
    // ceil(64 / rb) * 2^rb rows is largest at rb = 8 (8 * 256)
    return OS_HEAD + (size_t)os_tiles(n_hint) * 8 * 256 * 8 + 256;
}

int radix_sort_u32(uint32_t *keys[2], uint32_t *vals[2], const uint32_t *n_dev, int64_t cap, int64_t n_hint, int lo_bit,
                   int hi_bit, int radix_bits, void *hist, hipStream_t s) {
    return onesweep<uint32_t>(keys, vals, n_dev, cap, n_hint, lo_bit, hi_bit, radix_bits, hist, s);
}

int radix_sort_u64(uint64_t *keys[2], uint32_t *vals[2], const uint32_t *n_dev, int64_t cap, int64_t n_hint, int lo_bit,
                   int hi_bit, int radix_bits, void *hist, hipStream_t s) {
    return onesweep<uint64_t>(keys, vals, n_dev, cap, n_hint, lo_bit, hi_bit, radix_bits, hist, s);
}
