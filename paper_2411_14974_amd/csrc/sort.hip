// Tile binning and ordering (gfx950): device-wide exclusive scan, a stable
// LSD radix sort of (u32 key, u32 value) pairs, (convex, tile) pair emission
// and per-tile list ranges.
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

__global__ __launch_bounds__(SCAN_BLOCK) void scan_reduce_kernel(const uint32_t *__restrict__ in, uint32_t n,
                                                                  uint32_t *__restrict__ block_sums)
{
    __shared__ uint32_t s_wave[SCAN_BLOCK / 64];
    const size_t base = (size_t)blockIdx.x * SCAN_TILE;
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const size_t i = base + (size_t)k * SCAN_BLOCK + threadIdx.x;
        if (i < n) sum += in[i];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
    if ((threadIdx.x & 63) == 0) s_wave[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < SCAN_BLOCK / 64; ++w) t += s_wave[w];
        block_sums[blockIdx.x] = t;
    }
}

// One block scans the block sums in place (exclusive) and stores the total.
__global__ __launch_bounds__(SCAN_BLOCK) void scan_top_kernel(uint32_t *__restrict__ sums, uint32_t nb,
                                                               uint32_t *__restrict__ total)
{
    __shared__ uint32_t s[SCAN_TILE + SCAN_TILE / 32];
    __shared__ uint32_t s_wave[SCAN_BLOCK / 64];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nb; base += SCAN_TILE) {
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            const uint32_t i = base + k * SCAN_BLOCK + threadIdx.x;
            s[lds_pad(k * SCAN_BLOCK + threadIdx.x)] = i < nb ? sums[i] : 0u;
        }
        __syncthreads();
        const uint32_t t = block_scan_lds(s, s_wave);
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            const uint32_t i = base + k * SCAN_BLOCK + threadIdx.x;
            if (i < nb) sums[i] = s[lds_pad(k * SCAN_BLOCK + threadIdx.x)] + carry;
        }
        carry += t;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(SCAN_BLOCK) void scan_down_kernel(const uint32_t *__restrict__ in, uint32_t n,
                                                                const uint32_t *__restrict__ block_offsets,
                                                                uint32_t *__restrict__ out)
{
    __shared__ uint32_t s[SCAN_TILE + SCAN_TILE / 32];
    __shared__ uint32_t s_wave[SCAN_BLOCK / 64];
    const size_t base = (size_t)blockIdx.x * SCAN_TILE;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const size_t i = base + (size_t)k * SCAN_BLOCK + threadIdx.x;
        s[lds_pad(k * SCAN_BLOCK + threadIdx.x)] = i < n ? in[i] : 0u;
    }
    __syncthreads();
    block_scan_lds(s, s_wave);
    const uint32_t off = block_offsets[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const size_t i = base + (size_t)k * SCAN_BLOCK + threadIdx.x;
        if (i < n) out[i] = s[lds_pad(k * SCAN_BLOCK + threadIdx.x)] + off;
    }
}

size_t scan_temp_words(uint32_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

// out[i] = sum_{j<i} in[j]; *total (device) = sum of all.  tmp: scan_temp_words(n) words.
void scan_exclusive(hipStream_t st, const uint32_t *in, uint32_t *out, uint32_t n, uint32_t *total, uint32_t *tmp)
{
    const uint32_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 0) {
        hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(SCAN_BLOCK), 0, st, tmp, 0u, total);
        return;
    }
    hipLaunchKernelGGL(scan_reduce_kernel, dim3(nb), dim3(SCAN_BLOCK), 0, st, in, n, tmp);
    hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(SCAN_BLOCK), 0, st, tmp, nb, total);
    hipLaunchKernelGGL(scan_down_kernel, dim3(nb), dim3(SCAN_BLOCK), 0, st, in, n, tmp, out);
}

// ----------------------------------------------------------- radix sort ----

constexpr int RS_MAX_BITS = 8;
constexpr int RS_MAX_RADIX = 1 << RS_MAX_BITS;
constexpr int RS_BLOCK = 256;
constexpr int RS_WAVES = RS_BLOCK / 64;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_BLOCK * RS_ITEMS;

// Tiles [t0, t1) of block b under an even split of ceil(n / RS_TILE) tiles.
__device__ __forceinline__ void rs_block_tiles(uint32_t n, int nblocks, uint32_t &t0, uint32_t &t1)
{
    const uint32_t ntiles = (n + RS_TILE - 1) / RS_TILE;
    const uint32_t per = (ntiles + nblocks - 1) / nblocks;
    t0 = min(ntiles, blockIdx.x * per);
    t1 = min(ntiles, t0 + per);
}

template <int RS_BITS>
__global__ __launch_bounds__(RS_BLOCK) void radix_hist_kernel(const uint32_t *__restrict__ keys,
                                                               const uint32_t *__restrict__ n_dev, uint32_t n_host,
                                                               int shift, int nblocks, uint32_t *__restrict__ hist)
{
    constexpr int RS_RADIX = 1 << RS_BITS;
    __shared__ uint32_t h[RS_WAVES][RS_RADIX];
    const uint32_t n = n_dev ? *n_dev : n_host;
    const int wave = threadIdx.x >> 6;
    for (int d = threadIdx.x; d < RS_WAVES * RS_RADIX; d += RS_BLOCK) (&h[0][0])[d] = 0;
    __syncthreads();
    uint32_t t0, t1;
    rs_block_tiles(n, nblocks, t0, t1);
    for (uint32_t t = t0; t < t1; ++t) {
#pragma unroll
        for (int i = 0; i < RS_ITEMS; ++i) {
            const size_t idx = (size_t)t * RS_TILE + i * RS_BLOCK + threadIdx.x;
            if (idx < n) atomicAdd(&h[wave][(keys[idx] >> shift) & (RS_RADIX - 1)], 1u);
        }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < RS_RADIX; d += RS_BLOCK) {
        uint32_t c = 0;
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w) c += h[w][d];
        hist[(size_t)d * nblocks + blockIdx.x] = c;
    }
}

// Stable scatter of one digit of RS_BITS (<= 8) bits.  Within a tile the element order is
// (wave, item, lane); each wave ranks its elements with ballots over the digit
// bits, the block places the tile digit-sorted in LDS and writes each digit's
// run contiguously to its global position.
template <int RS_BITS>
__global__ __launch_bounds__(RS_BLOCK) void radix_scatter_kernel(
    const uint32_t *__restrict__ keys_in, const uint32_t *__restrict__ vals_in, uint32_t *__restrict__ keys_out,
    uint32_t *__restrict__ vals_out, const uint32_t *__restrict__ n_dev, uint32_t n_host, int shift, int nblocks,
    const uint32_t *__restrict__ hist_scanned)
{
    constexpr int RS_RADIX = 1 << RS_BITS;
    __shared__ uint32_t s_keys[RS_TILE];
    __shared__ uint32_t s_vals[RS_TILE];
    __shared__ uint32_t s_wcnt[RS_WAVES][RS_RADIX];
    __shared__ uint32_t s_dstart[RS_RADIX];
    __shared__ uint32_t s_total[RS_RADIX];
    __shared__ uint32_t s_gofs[RS_RADIX];
    __shared__ uint32_t s_wsum[RS_WAVES];

    const uint32_t n = n_dev ? *n_dev : n_host;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t t0, t1;
    rs_block_tiles(n, nblocks, t0, t1);
    for (int d = tid; d < RS_RADIX; d += RS_BLOCK) s_gofs[d] = hist_scanned[(size_t)d * nblocks + blockIdx.x];

    for (uint32_t t = t0; t < t1; ++t) {
        for (int d = tid; d < RS_WAVES * RS_RADIX; d += RS_BLOCK) (&s_wcnt[0][0])[d] = 0;
        __syncthreads();
        uint32_t k[RS_ITEMS], v[RS_ITEMS], off[RS_ITEMS];
        const size_t wbase = (size_t)t * RS_TILE + (size_t)wave * 64 * RS_ITEMS;
#pragma unroll
        for (int i = 0; i < RS_ITEMS; ++i) {
            const size_t idx = wbase + i * 64 + lane;
            const bool valid = idx < n;
            k[i] = valid ? keys_in[idx] : 0u;
            v[i] = valid ? vals_in[idx] : 0u;
            const uint32_t dg = (k[i] >> shift) & (RS_RADIX - 1);
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < RS_BITS; ++b) {
                const uint64_t bal = __ballot((dg >> b) & 1u);
                peers &= ((dg >> b) & 1u) ? bal : ~bal;
            }
            const uint32_t rank = __popcll(peers & lt_mask);
            const uint32_t cnt = __popcll(peers);
            const uint32_t before = valid ? s_wcnt[wave][dg] : 0u;
            off[i] = before + rank;
            if (valid && rank == 0) s_wcnt[wave][dg] = before + cnt;
        }
        __syncthreads();
        // per digit: exclusive over waves, and the tile total
        for (int d = tid; d < RS_RADIX; d += RS_BLOCK) {
            uint32_t run = 0;
#pragma unroll
            for (int w = 0; w < RS_WAVES; ++w) {
                const uint32_t c = s_wcnt[w][d];
                s_wcnt[w][d] = run;
                run += c;
            }
            s_total[d] = run;
        }
        __syncthreads();
        // exclusive scan of the digit totals (one digit per thread)
        {
            const uint32_t x = tid < RS_RADIX ? s_total[tid] : 0u;
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
            if (tid < RS_RADIX) s_dstart[tid] = wb + incl - x;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < RS_ITEMS; ++i) {
            const size_t idx = wbase + i * 64 + lane;
            if (idx < n) {
                const uint32_t dg = (k[i] >> shift) & (RS_RADIX - 1);
                const uint32_t lp = s_dstart[dg] + s_wcnt[wave][dg] + off[i];
                s_keys[lp] = k[i];
                s_vals[lp] = v[i];
            }
        }
        __syncthreads();
        const size_t tbase = (size_t)t * RS_TILE;
        const uint32_t nvalid = (uint32_t)min((size_t)RS_TILE, (size_t)n - tbase);
        for (uint32_t j = tid; j < nvalid; j += RS_BLOCK) {
            const uint32_t kk = s_keys[j];
            const uint32_t dg = (kk >> shift) & (RS_RADIX - 1);
            const uint32_t pos = s_gofs[dg] + (j - s_dstart[dg]);
            keys_out[pos] = kk;
            vals_out[pos] = s_vals[j];
        }
        __syncthreads();
        for (int d = tid; d < RS_RADIX; d += RS_BLOCK) s_gofs[d] += s_total[d];
        __syncthreads();
    }
}

int radix_blocks(uint32_t n_capacity)
{
    const uint32_t tiles = (n_capacity + RS_TILE - 1) / RS_TILE;
    return (int)std::max<uint32_t>(1u, std::min<uint32_t>(tiles, 1024u));
}

size_t radix_hist_words(int nblocks) { return (size_t)nblocks * RS_MAX_RADIX; }

template <int B>
static void radix_pass(hipStream_t st, const uint32_t *keys, const uint32_t *vals, uint32_t *keys_out,
                       uint32_t *vals_out, uint32_t n_host, const uint32_t *n_dev, int nblocks, int shift,
                       uint32_t *hist, uint32_t *scan_tmp)
{
    hipLaunchKernelGGL(radix_hist_kernel<B>, dim3(nblocks), dim3(RS_BLOCK), 0, st, keys, n_dev, n_host, shift,
                       nblocks, hist);
    scan_exclusive(st, hist, hist, (uint32_t)(nblocks * (1 << B)), nullptr, scan_tmp);
    hipLaunchKernelGGL(radix_scatter_kernel<B>, dim3(nblocks), dim3(RS_BLOCK), 0, st, keys, vals, keys_out,
                       vals_out, n_dev, n_host, shift, nblocks, hist);
}

// Sorts bits [0, end_bit) of the keys in passes of `digit_bits` (4..8; the
// last pass takes what remains).  On return *keys/*vals point at the sorted
// arrays (one of the two buffer pairs).  n_dev may be NULL (n_host used); with
// n_dev the element count is read on the device (graph capture needs no
// host read-back) and nblocks must cover the capacity.
void radix_sort(hipStream_t st, uint32_t **keys, uint32_t **vals, uint32_t **keys_alt, uint32_t **vals_alt,
                uint32_t n_host, const uint32_t *n_dev, int nblocks, int end_bit, uint32_t *hist, uint32_t *scan_tmp,
                int digit_bits)
{
    digit_bits = std::min(8, std::max(4, digit_bits));
    for (int shift = 0; shift < end_bit; shift += digit_bits) {
        const int b = std::min(digit_bits, end_bit - shift);
        switch (b) {
        case 1: case 2: case 3: case 4: radix_pass<4>(st, *keys, *vals, *keys_alt, *vals_alt, n_host, n_dev, nblocks, shift, hist, scan_tmp); break;
        case 5: radix_pass<5>(st, *keys, *vals, *keys_alt, *vals_alt, n_host, n_dev, nblocks, shift, hist, scan_tmp); break;
        case 6: radix_pass<6>(st, *keys, *vals, *keys_alt, *vals_alt, n_host, n_dev, nblocks, shift, hist, scan_tmp); break;
        case 7: radix_pass<7>(st, *keys, *vals, *keys_alt, *vals_alt, n_host, n_dev, nblocks, shift, hist, scan_tmp); break;
        default: radix_pass<8>(st, *keys, *vals, *keys_alt, *vals_alt, n_host, n_dev, nblocks, shift, hist, scan_tmp); break;
        }
        std::swap(*keys, *keys_alt);
        std::swap(*vals, *vals_alt);
    }
}

// ------------------------------------------------------------- binning ----

__global__ void gather_counts_kernel(uint32_t n, const uint32_t *__restrict__ sorted_ids,
                                     const uint32_t *__restrict__ counts, uint32_t *__restrict__ out)
{
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) out[r] = counts[sorted_ids[r]];
}

// One thread per (view, convex) instance in depth order: write its (global
// tile, instance) pairs, row-major over its tile rectangle.  Instance id =
// view * n_convex + convex; the view's tiles start at its tile_off.
__global__ void emit_pairs_kernel(uint32_t n, uint32_t n_convex, const uint32_t *__restrict__ sorted_ids,
                                  const uint32_t *__restrict__ offsets, const uint2 *__restrict__ rects,
                                  const FrameHeader *__restrict__ frame, uint32_t capacity,
                                  uint32_t *__restrict__ pair_tiles, uint32_t *__restrict__ pair_ids)
{
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint32_t id = sorted_ids[r];
    const uint2 rc = rects[id];
    const int tx0 = rc.x & 0xFFFF, ty0 = rc.x >> 16, tx1 = rc.y & 0xFFFF, ty1 = rc.y >> 16;
    if (tx0 > tx1 || ty0 > ty1) return;
    const ViewDesc &vd = reinterpret_cast<const ViewDesc *>(frame + 1)[id / n_convex];
    const int tiles_x = vd.tiles_x, toff = vd.tile_off;
    uint32_t off = offsets[r];
    for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx, ++off)
            if (off < capacity) {
                pair_tiles[off] = (uint32_t)(toff + ty * tiles_x + tx);
                pair_ids[off] = id;
            }
}

// Pair count that fits the buffers, and the overflow flag (for fixed-capacity frames).
__global__ void clamp_pairs_kernel(uint32_t *__restrict__ counters, uint32_t capacity)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const uint32_t m = counters[CNT_PAIRS];
        counters[CNT_PAIRS_EFF] = m < capacity ? m : capacity;
        counters[CNT_OVERFLOW] = m > capacity ? 1u : 0u;
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

__global__ void fill_u32_kernel(uint32_t *__restrict__ p, size_t n, uint32_t v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void tile_ranges_kernel(const uint32_t *__restrict__ tiles, const uint32_t *__restrict__ n_dev,
                                   uint32_t n_host, uint2 *__restrict__ ranges)
{
    const uint32_t n = n_dev ? *n_dev : n_host;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t t = tiles[i];
    if (i == 0 || tiles[i - 1] != t) ranges[t].x = i;
    if (i == n - 1 || tiles[i + 1] != t) ranges[t].y = i + 1;
}

void launch_fill_u32(hipStream_t st, uint32_t *p, size_t n, uint32_t v)
{
    if (n == 0) return;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
}

void launch_gather_counts(hipStream_t st, uint32_t n, const uint32_t *sorted_ids, const uint32_t *counts,
                          uint32_t *out)
{
    if (n == 0) return;
    hipLaunchKernelGGL(gather_counts_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, sorted_ids, counts, out);
}

void launch_emit_pairs(hipStream_t st, uint32_t n, uint32_t n_convex, const uint32_t *sorted_ids,
                       const uint32_t *offsets, const uint2 *rects, const FrameHeader *views, uint32_t capacity,
                       uint32_t *pair_tiles, uint32_t *pair_ids)
{
    if (n == 0) return;
    hipLaunchKernelGGL(emit_pairs_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, n_convex, sorted_ids, offsets,
                       rects, views, capacity, pair_tiles, pair_ids);
}

void launch_clamp_pairs(hipStream_t st, uint32_t *counters, uint32_t capacity)
{
    hipLaunchKernelGGL(clamp_pairs_kernel, dim3(1), dim3(64), 0, st, counters, capacity);
}

void launch_tile_length_keys(hipStream_t st, uint32_t ntiles, const uint2 *ranges, uint32_t *keys, uint32_t *vals)
{
    if (ntiles == 0) return;
    hipLaunchKernelGGL(tile_length_keys_kernel, dim3((ntiles + 255) / 256), dim3(256), 0, st, ntiles, ranges, keys,
                       vals);
}

void launch_tile_ranges(hipStream_t st, const uint32_t *tiles, uint32_t n_host, const uint32_t *n_dev,
                        uint32_t n_capacity, uint2 *ranges)
{
    if (n_capacity == 0) return;
    hipLaunchKernelGGL(tile_ranges_kernel, dim3((n_capacity + 255) / 256), dim3(256), 0, st, tiles, n_dev, n_host,
                       ranges);
}

} // namespace cs
