// Tile binning and ordering (gfx950): the pair-offset scan, a stable LSD
// radix sort of (u32 key, u32 value) pairs, (convex, tile) pair emission and
// per-tile list ranges.
//
// The front-to-back order within a tile (paper Sec. 3.2: convexes sorted by
// increasing distance) comes from a two-stage LSD sort of the (tile | depth)
// key: the depth digits are sorted once over the N convexes, the convexes are
// expanded into (tile, convex) pairs in that order, and a stable sort of the
// pairs on the tile digits alone completes the lexicographic order.  This moves
// the depth passes from the M pairs (about 13 per convex at 1080p) to the N
// convexes.
#include <algorithm>
#include <utility>

#include "common.hpp"

namespace cs {

// ----------------------------------------------------------------- scan ----

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 5); }

// Exclusive scan of the block's SCAN_ITEMS values per thread held in LDS
// (padded layout); returns the block total.
__device__ uint32_t block_scan_lds(uint32_t *s, uint32_t *s_wave)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t v[SCAN_ITEMS], sum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = s[lds_pad(tid * SCAN_ITEMS + k)];
        sum += v[k];
    }
    // inclusive wave scan of the per-thread sums
    uint32_t incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    uint32_t wbase = 0, total = 0;
    for (int w = 0; w < SCAN_BLOCK / 64; ++w) {
        const uint32_t c = s_wave[w];
        if (w < wave) wbase += c;
        total += c;
    }
    uint32_t run = wbase + incl - sum;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        s[lds_pad(tid * SCAN_ITEMS + k)] = run;
        run += v[k];
    }
    __syncthreads();
    return total;
}

// Pair counts in depth order and their exclusive scan (the pair offsets), in
// one pass: each workgroup claims the next tile of SCAN_TILE ranks, gathers
// the binning records bins[sorted_ids[r]] (copied out in depth order for the
// pair emission) and their pair counts, scans the counts in LDS, publishes the tile's sum and
// finds its prefix by a decoupled look-back in which one wave reads 64
// predecessors' 64-bit status words at a time.  The last tile stores the total.
constexpr uint64_t SS_AGG = 1ull << 62, SS_INC = 2ull << 62, SS_VAL = SS_AGG - 1ull;
constexpr uint32_t SS_SPIN_LIMIT = 1u << 22;

__device__ __forceinline__ uint64_t ss_load(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void ss_store(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// host_word (nullable): a word of coherent pinned host memory that also
// receives the pair count, as tag << 32 | count: the host waits for its tag
// there, with no copy or event in the stream.
__global__ __launch_bounds__(SCAN_BLOCK) void gather_scan_kernel(
    uint32_t n, const uint32_t *__restrict__ sorted_ids, const uint4 *__restrict__ bins,
    uint4 *__restrict__ bins_sorted, uint32_t *__restrict__ counts_sorted, uint32_t *__restrict__ offsets,
    uint32_t *__restrict__ counters, uint64_t *__restrict__ status, unsigned long long *__restrict__ host_word,
    uint32_t tag, uint32_t capacity, ZeroSpans zero)
{
    zero_share(zero); // the tile ranges, when this scan also prepares the pair pass
    __shared__ uint32_t s[SCAN_TILE + SCAN_TILE / 32];
    __shared__ uint32_t s_wave[SCAN_BLOCK / 64];
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_excl;
    const int tid = threadIdx.x, lane = tid & 63;
    if (tid == 0) s_tile = atomicAdd(&counters[CNT_SCAN_TILE], 1u);
    __syncthreads();
    const uint32_t t = s_tile;
    const size_t base = (size_t)t * SCAN_TILE;
    if (base >= n) return;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const size_t i = base + (size_t)k * SCAN_BLOCK + tid;
        uint32_t c = 0;
        if (i < n) {
            const uint4 b = bins[sorted_ids[i]]; // the one random read per instance
            c = bin_count(b);
            bins_sorted[i] = b;
            counts_sorted[i] = c;
        }
        s[lds_pad(k * SCAN_BLOCK + tid)] = c;
    }
    __syncthreads();
    const uint32_t tile_total = block_scan_lds(s, s_wave);
    if (tid < 64) {
        if (tid == 0) ss_store(&status[t], (t == 0 ? SS_INC : SS_AGG) | (uint64_t)tile_total);
        uint64_t excl = 0;
        if (t > 0) {
            int64_t j = (int64_t)t - 1; // the window's newest tile
            uint32_t spins = 0;
            for (;;) {
                const int64_t idx = j - lane;
                const uint64_t sv = idx >= 0 ? ss_load(&status[idx]) : SS_INC; // before tile 0: inclusive 0
                const uint64_t flag = sv & ~SS_VAL;
                const uint64_t notready = __ballot(flag == 0ull), inc = __ballot(flag == SS_INC);
                const int fi = inc ? __builtin_ctzll(inc) : 64; // nearest inclusive prefix in the window
                const uint64_t need = (fi >= 63) ? ~0ull : ((2ull << fi) - 1ull);
                if (notready & need) {
                    if (++spins > SS_SPIN_LIMIT) {
                        if (lane == 0) atomicOr(&counters[CNT_SORT_ERR], 2u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                uint64_t v = (lane <= fi) ? (sv & SS_VAL) : 0ull;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
                excl += v;
                if (fi < 64) break;
                j -= 64;
            }
            if (tid == 0) ss_store(&status[t], SS_INC | (excl + tile_total));
        }
        if (tid == 0) {
            s_excl = excl;
            if (base + SCAN_TILE >= n) {
                const uint32_t m = (uint32_t)(excl + tile_total);
                counters[CNT_PAIRS] = m;
                if (capacity) { // the pair pass's count, clamped to the buffers, and the overflow flag
                    counters[CNT_PAIRS_EFF] = m < capacity ? m : capacity;
                    counters[CNT_OVERFLOW] = m > capacity ? 1u : 0u;
                }
                if (host_word)
                    __hip_atomic_store(host_word, ((unsigned long long)tag << 32) | (uint32_t)(excl + tile_total),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
    }
    __syncthreads();
    const uint32_t ex = (uint32_t)s_excl;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const size_t i = base + (size_t)k * SCAN_BLOCK + tid;
        if (i < n) offsets[i] = s[lds_pad(k * SCAN_BLOCK + tid)] + ex;
    }
}

// 32-bit words of the scan's look-back status (u64 per tile of SCAN_TILE ranks).
size_t scan_status_words(uint32_t n) { return 2 * (((size_t)n + SCAN_TILE - 1) / SCAN_TILE + 1); }

// bins_sorted[r] = bins[sorted_ids[r]], counts_sorted[r] its pair count,
// offsets = their exclusive scan, counters[CNT_PAIRS] = the total.  counters
// must hold CNT_WORDS words, zeroed, followed by scan_status_words(n) zeroed words.
void launch_gather_scan(hipStream_t st, uint32_t n, const uint32_t *sorted_ids, const uint4 *bins,
                        uint4 *bins_sorted, uint32_t *counts_sorted, uint32_t *offsets, uint32_t *counters,
                        unsigned long long *host_word, uint32_t tag, uint32_t capacity, uint32_t *ranges,
                        uint32_t range_words)
{
    if (n == 0) return;
    const uint32_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    const ZeroSpans z{{capacity ? ranges : nullptr, nullptr}, {capacity ? range_words : 0u, 0u}};
    hipLaunchKernelGGL(gather_scan_kernel, dim3(tiles), dim3(SCAN_BLOCK), 0, st, n, sorted_ids, bins, bins_sorted,
                       counts_sorted, offsets, counters, reinterpret_cast<uint64_t *>(counters + CNT_STATUS),
                       host_word, tag, capacity, z);
}

// ----------------------------------------------------------- radix sort ----
//
// Stable LSD radix sort of (u32 key, u32 value) pairs with one kernel per
// digit (single-pass scatter with decoupled look-back, after Merrill and
// Garland's single-pass prefix scan as used by the "Onesweep" radix sort):
//  1. one kernel reads the keys once and builds the global digit histograms of
//     every pass;
//  2. per pass, each workgroup claims the next tile of elements from an
//     atomic counter (tiles are claimed in order by running workgroups), ranks
//     its elements per digit (wave ballots), publishes its per-digit counts,
//     then walks back over its predecessors' published counts until it meets an
//     inclusive prefix, publishes its own inclusive prefix, and writes its
//     elements digit-sorted to their global positions.
// A predecessor publishes its counts before it waits on anything, so every
// wait ends; it is still bounded (OS_SPIN_LIMIT), and a wait that runs out
// sets the caller's error word instead of spinning on.

constexpr int OS_BLOCK = 512;
constexpr int OS_WAVES = OS_BLOCK / 64;
constexpr int OS_ITEMS_MIN = 8;                       // keys per thread of the smaller tiles
constexpr int OS_TILE_MIN = OS_BLOCK * OS_ITEMS_MIN;  // 4096 keys
constexpr int OS_RADIX = 256; // digits of up to 8 bits
constexpr int OS_MAX_PASSES = 8;
constexpr uint32_t OS_AGG = 1u << 30, OS_INC = 2u << 30, OS_VAL = OS_AGG - 1u;
constexpr uint32_t OS_SPIN_LIMIT = 1u << 22;
constexpr int OS_WINDOW = 8; // predecessors read per look-back round trip
// temporary layout (words): histograms [P][256] | tile counters [64] | status [P][tiles][256]
constexpr size_t OS_CTR = (size_t)OS_MAX_PASSES * OS_RADIX, OS_STATUS = OS_CTR + 64;

__host__ __device__ constexpr int os_passes(int end_bit, int digit_bits) { return (end_bit + digit_bits - 1) / digit_bits; }
// The end_bit bits are split over the passes as evenly as possible (13 bits in
// two passes: 7 + 6); pass p covers bits [os_shift, os_shift + os_width).
__host__ __device__ constexpr int os_width(int end_bit, int passes, int p)
{
    return end_bit / passes + (p < end_bit % passes ? 1 : 0);
}
__host__ __device__ constexpr int os_shift(int end_bit, int passes, int p)
{
    return p * (end_bit / passes) + (p < end_bit % passes ? p : end_bit % passes);
}

__device__ __forceinline__ uint32_t os_load(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void os_store(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Lanes of the wave holding the same BITS-bit digit (ballot per bit).
template <int BITS> __device__ __forceinline__ uint64_t digit_peers(uint32_t dg, bool valid)
{
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const uint64_t bal = __ballot((dg >> b) & 1u);
        peers &= ((dg >> b) & 1u) ? bal : ~bal;
    }
    return peers;
}

// Exclusive scan of one value per thread over the workgroup (OS_BLOCK threads).
__device__ __forceinline__ uint32_t os_block_excl(uint32_t x, uint32_t *s_wsum)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) s_wsum[wave] = incl;
    __syncthreads();
    uint32_t wb = 0;
    for (int w = 0; w < wave; ++w) wb += s_wsum[w];
    __syncthreads();
    return wb + incl - x;
}

// Global histograms of every pass: hist[p * 256 + digit].  A workgroup takes
// tiles of OS_BLOCK x ITEMS keys (grid-stride), loads a tile's keys at
// once and counts them into per-wave LDS histograms (fewer same-address
// collisions), then adds its nonzero bins to the global histogram.
template <int BITS, int ITEMS>
__global__ __launch_bounds__(OS_BLOCK) void os_hist_kernel(const uint32_t *__restrict__ keys,
                                                           const uint32_t *__restrict__ n_dev, uint32_t n_host,
                                                           int end_bit, int P, uint32_t *__restrict__ hist)
{
    constexpr int TILE = OS_BLOCK * ITEMS;
    constexpr int R = 1 << BITS; // bins per pass (BITS: the widest pass)
    constexpr int HW = 1024;     // bins per wave: P * R <= 1024 for keys of up to 32 bits
    __shared__ uint32_t h[OS_WAVES][HW];
    const uint32_t n = n_dev ? *n_dev : n_host;
    const int wave = threadIdx.x >> 6;
    for (int d = threadIdx.x; d < OS_WAVES * HW; d += OS_BLOCK) (&h[0][0])[d] = 0;
    __syncthreads();
    const uint32_t ntiles = (n + TILE - 1) / TILE;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        // each thread counts a contiguous run of ITEMS keys (16-byte loads), so
        // the lanes of a wave hold keys ITEMS apart: runs of equal digits (pairs
        // of one convex in neighbouring tiles) fall to one thread instead of
        // colliding on one LDS counter across the wave
        const size_t base = (size_t)t * TILE + (size_t)threadIdx.x * ITEMS;
        uint32_t k[ITEMS];
        int cnt;
        if (base + ITEMS <= n) {
            const uint4 *src = reinterpret_cast<const uint4 *>(keys + base);
#pragma unroll
            for (int q = 0; q < ITEMS / 4; ++q) {
                const uint4 w = src[q];
                k[4 * q] = w.x; k[4 * q + 1] = w.y; k[4 * q + 2] = w.z; k[4 * q + 3] = w.w;
            }
            cnt = ITEMS;
        } else {
            cnt = base < n ? (int)(n - base) : 0;
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) k[i] = i < cnt ? keys[base + i] : 0u;
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
            if (i < cnt)
                for (int p = 0; p < P; ++p)
                    atomicAdd(&h[wave][p * R + ((k[i] >> os_shift(end_bit, P, p)) & ((1u << os_width(end_bit, P, p)) - 1u))],
                              1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < P * R; d += OS_BLOCK) {
        uint32_t c = 0;
#pragma unroll
        for (int w = 0; w < OS_WAVES; ++w) c += h[w][d];
        if (c) atomicAdd(&hist[(d / R) * OS_RADIX + d % R], c);
    }
}

template <int BITS, int ITEMS>
__global__ __launch_bounds__(OS_BLOCK) void os_scatter_kernel(
    const uint32_t *__restrict__ keys_in, const uint32_t *__restrict__ vals_in, uint32_t *__restrict__ keys_out,
    uint32_t *__restrict__ vals_out, const uint32_t *__restrict__ n_dev, uint32_t n_host, int shift,
    const uint32_t *__restrict__ hist, uint32_t *__restrict__ tile_counter, uint32_t *__restrict__ status,
    uint32_t *__restrict__ err)
{
    constexpr int TILE = OS_BLOCK * ITEMS;
    constexpr int R = 1 << BITS;
    __shared__ uint32_t s_keys[TILE];
    __shared__ uint32_t s_vals[TILE];
    __shared__ uint32_t s_wcnt[OS_WAVES][R];
    __shared__ uint32_t s_dstart[R];
    __shared__ uint32_t s_gofs[R];
    __shared__ uint32_t s_wsum[OS_WAVES];
    __shared__ uint32_t s_tile;

    const uint32_t n = n_dev ? *n_dev : n_host;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (tid == 0) s_tile = atomicAdd(tile_counter, 1u);
    for (int d = tid; d < OS_WAVES * R; d += OS_BLOCK) (&s_wcnt[0][0])[d] = 0;
    __syncthreads();
    const uint32_t t = s_tile;
    const size_t tbase = (size_t)t * TILE;
    if (tbase >= n) return; // past the data (capacity-sized grids): nobody waits on this tile

    // rank: element order within the tile is (wave, item, lane)
    uint32_t k[ITEMS], v[ITEMS], off[ITEMS];
    const size_t wbase = tbase + (size_t)wave * 64 * ITEMS;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const size_t idx = wbase + i * 64 + lane;
        const bool valid = idx < n;
        k[i] = valid ? keys_in[idx] : 0u;
        v[i] = valid ? vals_in[idx] : 0u;
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const size_t idx = wbase + i * 64 + lane;
        const bool valid = idx < n;
        const uint32_t dg = (k[i] >> shift) & (R - 1);
        const uint64_t peers = digit_peers<BITS>(dg, valid);
        const uint32_t rank = __popcll(peers & lt_mask);
        const uint32_t before = valid ? s_wcnt[wave][dg] : 0u;
        off[i] = before + rank;
        if (valid && rank == 0) s_wcnt[wave][dg] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // per digit: exclusive over waves and the tile's count, published at once
    uint32_t total = 0;
    if (tid < R) {
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < OS_WAVES; ++w) {
            const uint32_t c = s_wcnt[w][tid];
            s_wcnt[w][tid] = run;
            run += c;
        }
        total = run;
        os_store(&status[(size_t)t * R + tid], (t == 0 ? OS_INC : OS_AGG) | total);
    }
    const uint32_t dstart = os_block_excl(tid < R ? total : 0u, s_wsum);
    const uint32_t dbase = os_block_excl(tid < R ? hist[tid] : 0u, s_wsum);
    if (tid < R) {
        s_dstart[tid] = dstart;
        uint32_t excl = 0;
        if (t > 0) {
            // look back to the nearest inclusive prefix, OS_WINDOW predecessors
            // per round trip (entries before tile 0 read as inclusive zero)
            int64_t j = (int64_t)t - 1; // newest predecessor not yet consumed
            uint32_t spins = 0;
            for (;;) {
                uint32_t sv[OS_WINDOW];
#pragma unroll
                for (int w = 0; w < OS_WINDOW; ++w)
                    sv[w] = (j - w >= 0) ? os_load(&status[(size_t)(j - w) * R + tid]) : OS_INC;
                int used = 0;
                bool found = false, pending = false;
#pragma unroll
                for (int w = 0; w < OS_WINDOW; ++w) {
                    if (found || pending) continue;
                    const uint32_t f = sv[w] & ~OS_VAL;
                    if (f == 0u) { pending = true; continue; } // not published yet: re-read from here
                    excl += sv[w] & OS_VAL;
                    ++used;
                    found = (f == OS_INC);
                }
                if (found) break;
                j -= used;
                if (pending) {
                    if (++spins > OS_SPIN_LIMIT) { atomicOr(err, 1u); break; }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            os_store(&status[(size_t)t * R + tid], OS_INC | (excl + total));
        }
        s_gofs[tid] = dbase + excl;
    }
    __syncthreads();
    // digit-sorted tile in LDS, then each digit's run to its global position
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const size_t idx = wbase + i * 64 + lane;
        if (idx < n) {
            const uint32_t dg = (k[i] >> shift) & (R - 1);
            const uint32_t lp = s_dstart[dg] + s_wcnt[wave][dg] + off[i];
            s_keys[lp] = k[i];
            s_vals[lp] = v[i];
        }
    }
    __syncthreads();
    const uint32_t nvalid = (uint32_t)min((size_t)TILE, (size_t)n - tbase);
    for (uint32_t j = tid; j < nvalid; j += OS_BLOCK) {
        const uint32_t kk = s_keys[j];
        const uint32_t dg = (kk >> shift) & (R - 1);
        const uint32_t pos = s_gofs[dg] + (j - s_dstart[dg]);
        keys_out[pos] = kk;
        vals_out[pos] = s_vals[j];
    }
}

__global__ void fill_u32_kernel(uint32_t *__restrict__ p, size_t n, uint32_t v);

size_t sort_temp_words(uint32_t n_capacity, int end_bit, int digit_bits)
{
    digit_bits = std::min(8, std::max(4, digit_bits));
    const size_t tiles = ((size_t)n_capacity + OS_TILE_MIN - 1) / OS_TILE_MIN; // the smaller tiles: more of them
    return OS_STATUS + (size_t)os_passes(end_bit, digit_bits) * std::max<size_t>(tiles, 1) * OS_RADIX;
}

template <int B, int I>
static void os_launch_hist(hipStream_t st, const uint32_t *keys, uint32_t n_host, const uint32_t *n_dev, int blocks,
                           int end_bit, int P, uint32_t *hist)
{
    hipLaunchKernelGGL((os_hist_kernel<B, I>), dim3(blocks), dim3(OS_BLOCK), 0, st, keys, n_dev, n_host, end_bit, P, hist);
}

template <int B, int I>
static void os_launch_scatter(hipStream_t st, const uint32_t *keys, const uint32_t *vals, uint32_t *keys_out,
                              uint32_t *vals_out, uint32_t n_host, const uint32_t *n_dev, int tiles, int shift,
                              const uint32_t *hist, uint32_t *ctr, uint32_t *status, uint32_t *err)
{
    hipLaunchKernelGGL((os_scatter_kernel<B, I>), dim3(tiles), dim3(OS_BLOCK), 0, st, keys, vals, keys_out, vals_out, n_dev,
                       n_host, shift, hist, ctr, status, err);
}

#define OS_DISPATCH(BITS, CALL)                                                                                    \
    switch (BITS) {                                                                                                \
    case 1: { constexpr int BB = 1; CALL; } break;                                                                 \
    case 2: { constexpr int BB = 2; CALL; } break;                                                                 \
    case 3: { constexpr int BB = 3; CALL; } break;                                                                 \
    case 4: { constexpr int BB = 4; CALL; } break;                                                                 \
    case 5: { constexpr int BB = 5; CALL; } break;                                                                 \
    case 6: { constexpr int BB = 6; CALL; } break;                                                                 \
    case 7: { constexpr int BB = 7; CALL; } break;                                                                 \
    default: { constexpr int BB = 8; CALL; } break;                                                                \
    }

// Sorts bits [0, end_bit) of the keys in ceil(end_bit / digit_bits) passes
// (digit_bits in 4..8; the bits are split evenly over the passes).  On
// return *keys/*vals point at the sorted arrays (one of the two buffer pairs).
// n_dev may be NULL (n_host used); with n_dev the element count is read on the
// device (graph capture needs no host read-back) and n_capacity bounds it.
// temp: sort_temp_words(n_capacity, end_bit, digit_bits) words.  *err (device)
// gets bit 0 set if a look-back wait ran out of its bound.  The key arrays must
// be 16-byte aligned (the histogram pass reads them in 16-byte loads).
// Words of temp that radix_sort uses (and clears first, unless told that they
// are clear) for these arguments.
size_t radix_sort_words(uint32_t n_host, bool n_on_device, uint32_t n_capacity, int end_bit, int digit_bits)
{
    digit_bits = std::min(8, std::max(4, digit_bits));
    const uint32_t n_grid = n_on_device ? n_capacity : n_host;
    if (n_grid == 0 || end_bit <= 0) return 0;
    const int P = os_passes(end_bit, digit_bits);
    const int tile = n_grid <= (1u << 22) ? OS_TILE_MIN : 2 * OS_TILE_MIN;
    const size_t tiles = ((size_t)n_grid + tile - 1) / tile;
    return OS_STATUS + (size_t)P * tiles * OS_RADIX;
}

void radix_sort(hipStream_t st, uint32_t **keys, uint32_t **vals, uint32_t **keys_alt, uint32_t **vals_alt,
                uint32_t n_host, const uint32_t *n_dev, uint32_t n_capacity, int end_bit, uint32_t *temp,
                int digit_bits, uint32_t *err, bool temp_clear)
{
    digit_bits = std::min(8, std::max(4, digit_bits));
    const uint32_t n_grid = n_dev ? n_capacity : n_host;
    if (n_grid == 0 || end_bit <= 0) return;
    const int P = os_passes(end_bit, digit_bits);
    // up to 4M elements: tiles of OS_TILE_MIN (more workgroups in flight);
    // beyond: twice as large (half the look-back chain)
    const bool small = n_grid <= (1u << 22);
    const int tile = small ? OS_TILE_MIN : 2 * OS_TILE_MIN;
    const int tiles = (int)((n_grid + tile - 1) / tile);
    const size_t words = radix_sort_words(n_host, n_dev != nullptr, n_capacity, end_bit, digit_bits);
    if (!temp_clear) {
        const size_t fb = std::min<size_t>((words + 255) / 256, 4096);
        hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)fb), dim3(256), 0, st, temp, words, 0u);
    }
    const int hb = std::max(1, std::min(tiles, 256)); // one workgroup per CU: fewer same-address global adds
    const int widest = os_width(end_bit, P, 0);
    if (small) {
        OS_DISPATCH(widest, (os_launch_hist<BB, OS_ITEMS_MIN>(st, *keys, n_host, n_dev, hb, end_bit, P, temp)));
    } else {
        OS_DISPATCH(widest, (os_launch_hist<BB, 2 * OS_ITEMS_MIN>(st, *keys, n_host, n_dev, hb, end_bit, P, temp)));
    }
    for (int p = 0; p < P; ++p) {
        const int shift = os_shift(end_bit, P, p);
        const int b = os_width(end_bit, P, p);
        uint32_t *status = temp + OS_STATUS + (size_t)p * tiles * OS_RADIX;
        if (small) {
            OS_DISPATCH(b, (os_launch_scatter<BB, OS_ITEMS_MIN>(st, *keys, *vals, *keys_alt, *vals_alt, n_host, n_dev,
                                                                tiles, shift, temp + (size_t)p * OS_RADIX,
                                                                temp + OS_CTR + p, status, err)));
        } else {
            OS_DISPATCH(b, (os_launch_scatter<BB, 2 * OS_ITEMS_MIN>(st, *keys, *vals, *keys_alt, *vals_alt, n_host,
                                                                    n_dev, tiles, shift, temp + (size_t)p * OS_RADIX,
                                                                    temp + OS_CTR + p, status, err)));
        }
        std::swap(*keys, *keys_alt);
        std::swap(*vals, *vals_alt);
    }
}

// ------------------------------------------------------------- binning ----

// Pairs of 256 consecutive instances in depth order, written cooperatively:
// their pair ranges are contiguous ([offsets[r], offsets[r] + counts[r]) in
// rank order), so the workgroup strides over the whole run with one pair per
// thread (coalesced stores) and finds each pair's instance by a binary search
// over the offsets staged in LDS.  Within an instance the pairs run row-major
// over its tile rectangle (over the kept tiles of a rectangle of at most 64
// tiles), read from the binning records in depth order.  Instance id = view * n_convex + convex; the view's
// tiles start at its tile_off.
constexpr int EMIT_BLOCK = 256;
constexpr int EMIT_ITEMS = 8;
constexpr int EMIT_CHUNK = EMIT_BLOCK * EMIT_ITEMS; // pairs whose owners are found per round

// Position of the q-th set bit of m (q < popcount(m)).
__device__ __forceinline__ uint32_t nth_set_bit(uint64_t m, uint32_t q)
{
    uint32_t pos = 0;
    uint32_t w = (uint32_t)m;
    const uint32_t c32 = __popc(w);
    if (q >= c32) { q -= c32; w = (uint32_t)(m >> 32); pos = 32; }
#pragma unroll
    for (int half = 16; half >= 1; half >>= 1) {
        const uint32_t c = __popc(w & ((1u << half) - 1u));
        if (q >= c) { q -= c; w >>= half; pos += half; }
    }
    return pos;
}

__global__ __launch_bounds__(EMIT_BLOCK) void emit_pairs_kernel(
    uint32_t n, uint32_t n_convex, const uint32_t *__restrict__ sorted_ids, const uint32_t *__restrict__ offsets,
    const uint32_t *__restrict__ counts_sorted, const uint4 *__restrict__ bins_sorted,
    const FrameHeader *__restrict__ frame, uint32_t capacity, uint32_t *__restrict__ pair_tiles,
    uint32_t *__restrict__ pair_ids, ZeroSpans zero)
{
    zero_share(zero); // the tile sort's temporaries
    __shared__ uint32_t s_off[EMIT_BLOCK];
    __shared__ uint32_t s_id[EMIT_BLOCK];
    __shared__ uint32_t s_x0w[EMIT_BLOCK];  // tx0 | rect width << 16
    __shared__ uint32_t s_base[EMIT_BLOCK]; // global tile of the rectangle's first row start: toff + ty0 * tiles_x
    __shared__ uint32_t s_tx[EMIT_BLOCK];   // the view's tiles_x
    __shared__ uint64_t s_mask[EMIT_BLOCK]; // kept tiles (binning record encoding)
    __shared__ uint32_t s_small[EMIT_BLOCK];
    __shared__ uint32_t s_th[EMIT_BLOCK];    // rect height
    __shared__ uint32_t s_bend[EMIT_BLOCK][BIG_BANDS]; // large rectangles: pairs up to the end of each band
    __shared__ float s_rw[EMIT_BLOCK];       // 1 / rect width
    __shared__ uint32_t s_own[EMIT_CHUNK];  // owner (block-local convex) of each pair of the chunk
    __shared__ uint32_t s_wmax[EMIT_BLOCK / 64];
    __shared__ uint32_t s_end;
    const uint32_t r0 = blockIdx.x * EMIT_BLOCK;
    const int cnt = (int)min((uint32_t)EMIT_BLOCK, n - r0);
    const int tid = threadIdx.x;
    const ViewDesc *views = reinterpret_cast<const ViewDesc *>(frame + 1);
    if (tid < cnt) {
        const uint32_t r = r0 + tid;
        const uint32_t id = sorted_ids[r];
        const uint32_t off = offsets[r];
        s_off[tid] = off;
        s_id[tid] = id;
        uint32_t x0w = 0, base = 0, tx = 1, small = 0, th = 0;
        uint64_t mask = 0;
        if (counts_sorted[r] > 0) {
            const uint4 b = bins_sorted[r];
            const uint32_t tx0 = b.x & 0xFFFFu, ty0 = b.x >> 16, tx1 = b.y & 0xFFFFu, ty1 = b.y >> 16;
            const ViewDesc &vd = views[id / n_convex];
            tx = (uint32_t)vd.tiles_x;
            x0w = tx0 | ((tx1 - tx0 + 1) << 16);
            base = (uint32_t)vd.tile_off + ty0 * tx;
            th = ty1 - ty0 + 1;
            small = (tx1 - tx0 + 1) * th <= 64u;
            mask = (uint64_t)b.z | ((uint64_t)b.w << 32);
        }
        s_x0w[tid] = x0w;
        s_base[tid] = base;
        s_tx[tid] = tx;
        s_mask[tid] = mask;
        s_small[tid] = small;
        s_th[tid] = th;
        if (!small && th > 0) {
            uint32_t acc = 0;
#pragma unroll
            for (int r = 0; r < BIG_BANDS; ++r) {
                int row0, nrow, col0, ncol;
                big_band(mask, (int)(x0w >> 16), (int)th, r, &row0, &nrow, &col0, &ncol);
                acc += (uint32_t)(nrow * ncol);
                s_bend[tid][r] = acc;
            }
        }
        s_rw[tid] = 1.0f / (float)max(x0w >> 16, 1u);
        if (tid == cnt - 1) s_end = off + counts_sorted[r];
    }
    __syncthreads();
    const uint32_t p0 = s_off[0], p1 = min(s_end, capacity);
    const int lane = tid & 63, wave = tid >> 6;
    // The pairs' owners, EMIT_CHUNK pairs at a time: each convex marks the first
    // pair of its run (entries with no pairs share the next one's offset: the
    // larger index, the owner, wins), the chunk's first pair gets its owner by
    // one binary search, and a running maximum carries the marks along the runs.
    for (uint32_t c0 = p0; c0 < p1; c0 += EMIT_CHUNK) {
        const uint32_t cn = min((uint32_t)EMIT_CHUNK, p1 - c0);
        for (int j = tid; j < EMIT_CHUNK; j += EMIT_BLOCK) s_own[j] = 0u;
        __syncthreads();
        if (tid == 0) { // last entry with s_off <= c0
            int lo = 0, hi = cnt - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_off[mid] <= c0) lo = mid;
                else hi = mid - 1;
            }
            atomicMax(&s_own[0], (uint32_t)lo);
        }
        if (tid < cnt) {
            const uint32_t o = s_off[tid];
            if (o >= c0 && o < c0 + cn) atomicMax(&s_own[o - c0], (uint32_t)tid);
        }
        __syncthreads();
        // inclusive running maximum over the chunk: EMIT_ITEMS consecutive entries per thread
        uint32_t v[EMIT_ITEMS], m = 0u;
#pragma unroll
        for (int k = 0; k < EMIT_ITEMS; ++k) {
            m = max(m, s_own[tid * EMIT_ITEMS + k]);
            v[k] = m;
        }
        uint32_t incl = m;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o, 64);
            if (lane >= o) incl = max(incl, y);
        }
        if (lane == 63) s_wmax[wave] = incl;
        __syncthreads();
        uint32_t before = __shfl_up(incl, 1, 64);
        if (lane == 0) before = 0u;
        for (int w = 0; w < wave; ++w) before = max(before, s_wmax[w]);
#pragma unroll
        for (int k = 0; k < EMIT_ITEMS; ++k) s_own[tid * EMIT_ITEMS + k] = max(before, v[k]);
        __syncthreads();
        for (uint32_t j = tid; j < cn; j += EMIT_BLOCK) {
            const uint32_t p = c0 + j;
            const int lo = (int)s_own[j];
            uint32_t q = p - s_off[lo];
            const uint32_t x0w = s_x0w[lo], w = x0w >> 16;
            uint32_t row, col;
            if (s_small[lo]) {
                q = nth_set_bit(s_mask[lo], q); // the q-th kept tile of the rectangle
                // q / w through the reciprocal (q < 2^24), corrected by one step
                row = (uint32_t)((float)q * s_rw[lo]);
                if (row * w > q) --row;
                else if ((row + 1) * w <= q) ++row;
                col = q - row * w;
            } else { // the q-th tile of the kept bands, band by band, row-major in each
                int r = 0;
                uint32_t before = 0;
#pragma unroll
                for (int k = 0; k < BIG_BANDS - 1; ++k) {
                    const uint32_t e = s_bend[lo][k];
                    if (q >= e) { r = k + 1; before = e; }
                }
                int row0, nrow, col0, ncol;
                big_band(s_mask[lo], (int)w, (int)s_th[lo], r, &row0, &nrow, &col0, &ncol);
                const uint32_t qb = q - before, nc = (uint32_t)max(ncol, 1);
                uint32_t rr = (uint32_t)((float)qb / (float)nc); // qb < 2^24, corrected by one step
                if (rr * nc > qb) --rr;
                else if ((rr + 1) * nc <= qb) ++rr;
                row = (uint32_t)row0 + rr;
                col = (uint32_t)col0 + (qb - rr * nc);
            }
            pair_tiles[p] = s_base[lo] + row * s_tx[lo] + (x0w & 0xFFFFu) + col;
            pair_ids[p] = s_id[lo];
        }
        __syncthreads();
    }
}

// Sort keys that put long tile lists first: key = 0xFFFF - min(length, 0xFFFF).
__global__ void tile_length_keys_kernel(uint32_t ntiles, const uint2 *__restrict__ ranges,
                                        uint32_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    const uint2 r = ranges[t];
    const uint32_t len = r.y - r.x;
    keys[t] = 0xFFFFu - (len < 0xFFFFu ? len : 0xFFFFu);
    vals[t] = t;
}

// Zero up to four ranges of words in one launch.
struct FillRanges {
    uint32_t *p[4];
    size_t n[4];
};
__global__ void zero_ranges_kernel(FillRanges r)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < r.n[k]; i += stride) r.p[k][i] = 0u;
}

// The pair count that fits the buffers and the overflow flag, and the tile
// ranges cleared, in one launch.
__global__ void prepare_tail_kernel(uint32_t *__restrict__ counters, uint32_t capacity, uint32_t *__restrict__ ranges,
                                    size_t nwords)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t m = counters[CNT_PAIRS];
        counters[CNT_PAIRS_EFF] = m < capacity ? m : capacity;
        counters[CNT_OVERFLOW] = m > capacity ? 1u : 0u;
    }
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nwords; i += (size_t)gridDim.x * blockDim.x)
        ranges[i] = 0u;
}

__global__ void fill_u32_kernel(uint32_t *__restrict__ p, size_t n, uint32_t v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// [start, end) of every tile's run in the sorted tile ids.  Each thread takes
// RANGE_ITEMS consecutive ids in 16-byte loads (the sorted ids are 16-byte
// aligned) plus the id before them, and marks the run boundaries among them.
constexpr int RANGE_ITEMS = 8;

// ntiles bounds the tile ids written (every id of a pair is below it; the
// bound keeps a wrong count from writing past the ranges).
__global__ __launch_bounds__(256) void tile_ranges_kernel(const uint32_t *__restrict__ tiles,
                                                          const uint32_t *__restrict__ n_dev, uint32_t n_host,
                                                          uint2 *__restrict__ ranges, uint32_t ntiles)
{
    const uint32_t n = n_dev ? *n_dev : n_host;
    const size_t i0 = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) * RANGE_ITEMS;
    if (i0 >= n) return;
    uint32_t t[RANGE_ITEMS];
    if (i0 + RANGE_ITEMS <= n) {
        const uint4 *src = reinterpret_cast<const uint4 *>(tiles + i0);
#pragma unroll
        for (int q = 0; q < RANGE_ITEMS / 4; ++q) {
            const uint4 w = src[q];
            t[4 * q] = w.x; t[4 * q + 1] = w.y; t[4 * q + 2] = w.z; t[4 * q + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < RANGE_ITEMS; ++k) t[k] = i0 + k < n ? tiles[i0 + k] : 0u;
    }
    uint32_t prev = i0 > 0 ? tiles[i0 - 1] : 0xFFFFFFFFu;
#pragma unroll
    for (int k = 0; k < RANGE_ITEMS; ++k) {
        const size_t i = i0 + k;
        if (i >= n) break;
        if (t[k] != prev) { // a run starts at i and the previous one ends there
            if (t[k] < ntiles) ranges[t[k]].x = (uint32_t)i;
            if (i > 0 && prev < ntiles) ranges[prev].y = (uint32_t)i;
        }
        prev = t[k];
    }
    if (i0 + RANGE_ITEMS >= n && prev < ntiles) ranges[prev].y = n; // the last run
}

void launch_fill_u32(hipStream_t st, uint32_t *p, size_t n, uint32_t v)
{
    if (n == 0) return;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
}

void launch_emit_pairs(hipStream_t st, uint32_t n, uint32_t n_convex, const uint32_t *sorted_ids,
                       const uint32_t *offsets, const uint32_t *counts_sorted, const uint4 *bins_sorted,
                       const FrameHeader *views, uint32_t capacity, uint32_t *pair_tiles, uint32_t *pair_ids,
                       uint32_t *zero, uint32_t zero_words)
{
    if (n == 0) return;
    const ZeroSpans z{{zero, nullptr}, {zero ? zero_words : 0u, 0u}};
    hipLaunchKernelGGL(emit_pairs_kernel, dim3((n + EMIT_BLOCK - 1) / EMIT_BLOCK), dim3(EMIT_BLOCK), 0, st, n,
                       n_convex, sorted_ids, offsets, counts_sorted, bins_sorted, views, capacity, pair_tiles,
                       pair_ids, z);
}

void launch_prepare_tail(hipStream_t st, uint32_t *counters, uint32_t capacity, uint32_t *ranges, size_t nwords)
{
    const size_t blocks = std::max<size_t>(1, std::min<size_t>((nwords + 255) / 256, 1024));
    hipLaunchKernelGGL(prepare_tail_kernel, dim3((unsigned)blocks), dim3(256), 0, st, counters, capacity, ranges,
                       nwords);
}

void launch_zero_ranges(hipStream_t st, uint32_t *p0, size_t n0, uint32_t *p1, size_t n1, uint32_t *p2, size_t n2)
{
    FillRanges r = {{p0, p1, p2, p0}, {n0, n1, n2, 0}};
    const size_t most = std::max(std::max(n0, n1), n2);
    if (most == 0) return;
    const size_t blocks = std::min<size_t>((most + 255) / 256, 4096);
    hipLaunchKernelGGL(zero_ranges_kernel, dim3((unsigned)blocks), dim3(256), 0, st, r);
}

void launch_tile_length_keys(hipStream_t st, uint32_t ntiles, const uint2 *ranges, uint32_t *keys, uint32_t *vals)
{
    if (ntiles == 0) return;
    hipLaunchKernelGGL(tile_length_keys_kernel, dim3((ntiles + 255) / 256), dim3(256), 0, st, ntiles, ranges, keys,
                       vals);
}

void launch_tile_ranges(hipStream_t st, const uint32_t *tiles, uint32_t n_host, const uint32_t *n_dev,
                        uint32_t n_capacity, uint2 *ranges, uint32_t ntiles)
{
    if (n_capacity == 0) return;
    const size_t threads = ((size_t)n_capacity + RANGE_ITEMS - 1) / RANGE_ITEMS;
    hipLaunchKernelGGL(tile_ranges_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, tiles, n_dev,
                       n_host, ranges, ntiles);
}

} // namespace cs
