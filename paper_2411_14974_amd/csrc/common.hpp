// Shared definitions of the convex rasterizer's HIP kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace cs {

constexpr int MAXK = 8;
constexpr int WAVE = 64;
constexpr double LOG2E = 1.4426950408889634;
constexpr double LN2 = 0.6931471805599453;
constexpr uint32_t KEY_CULLED = 0xFFFFFFFFu;

// Convex status codes (also reported by the debug dump).
enum : int32_t { ST_VISIBLE = 0, ST_NEAR = 1, ST_HULL = 2, ST_FAINT = 3 };

// Per-convex record read by the compositing kernels: a 64-byte header then
// one 24-byte line (a, b, c as double) per hull edge.  A line evaluates
//   x2 = a*dx + b*dy + c = log2(e) * delta' * L_j(q),   dx = qx - ox, dy = qy - oy,
// so the LogSumExp runs in base 2 on the hardware exp2/log2.
struct RecHeader {
    float ox, oy;     // integer pixel origin of the line coefficients
    float sigma_p;    // sigma' = d * sigma
    float thr2;       // a pair is skipped when max_j x2_j > thr2 (alpha < eps certain)
    float opacity;
    float rgb[3];
    int32_t T;        // number of hull lines
    int32_t id;       // convex index
    uint32_t box_u;   // pixel columns u0 | u1 << 16 (inclusive) where alpha can reach eps
    uint32_t box_v;   // pixel rows    v0 | v1 << 16
};
// the K lines (three doubles each) follow the header; slots past the hull's
// T lines hold the null line (0, 0, NULL_LINE_C): its value is so negative
// that it never sets the maximum, its exponential is 0 and its gradient
// terms vanish, so consumers need no per-slot test against T
constexpr int REC_HEADER = 48;
constexpr double NULL_LINE_C = -1e30;
static_assert(sizeof(RecHeader) == REC_HEADER, "record header is 48 bytes");

__host__ __device__ constexpr int rec_stride(int K) { return (REC_HEADER + 24 * K + 15) & ~15; }
// accumulator slots per convex for the backward pass:
//   a[K] b[K] c[K]  (base-2 line coefficients), sigma', opacity, rgb[3], and
//   sum_j dL/dx2_j * x2_j  (= delta' dL/ddelta', accumulated per pair because
//   the same quantity rebuilt from the line slots cancels badly)
constexpr int acc_values(int K) { return 3 * K + 6; }
__host__ __device__ constexpr int acc_stride(int K) { return (acc_values(K) + 3) & ~3; }

// Camera as the kernels take it (by value).
struct CamArgs {
    int32_t W, H;
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    float znear;
    double campos[3]; // -R^T t
};

struct RenderArgs {
    float eps_alpha, t_min;
    float bg[3];
    int32_t tile;
};

// One view of a (possibly batched) render, as the kernels read it from device
// memory.  Tiles of all views share one global index space: view v owns
// [tile_off, tile_off + tiles_x * tiles_y); its per-pixel state starts at pix_off.
struct ViewDesc {
    CamArgs cam;
    int32_t tiles_x, tiles_y, tile_off, pad;
    int64_t pix_off;
    float *out_rgb;        // [H][W][3]
    const float *dl_drgb;  // [H][W][3], backward only
};

// Header of the device view table; the ViewDesc array follows it.  Kernels
// read the view count and the tile total from here, so a captured graph can be
// replayed with other cameras and resolutions.
struct FrameHeader {
    uint32_t nviews, total_tiles;
    int64_t total_pix;
    uint32_t pad[12];
};
static_assert(sizeof(FrameHeader) == 64, "frame header is 64 bytes");

constexpr int MAX_VIEWS = 256;
constexpr int NUM_QUEUES = 8; // one work queue per XCD
// Per-workgroup slots of the forward's work counters (tested, full pairs): each
// workgroup of the persistent grid stores its sums in a slot of its own and
// readers add the slots (same-address atomics from every wavefront serialise)
constexpr int EVAL_SLOTS = 16384;
// fields of a slot: pairs tested (pixel in the record's box), pairs past the
// max-line test (full), the sum of the hull size T over the full pairs, and
// wavefront-level record evaluations (some lane full); the backward's slots
// follow the forward's EVAL_SLOTS
enum : int { EV_TESTED = 0, EV_FULL = 1, EV_SUM_T = 2, EV_WAVES = 3, EVAL_FIELDS = 4 };

// Device counters of one frame (u32 words).
// Per-instance binning record (16 bytes): the tile rectangle, tx0 | ty0 << 16
// and tx1 | ty1 << 16 (empty when tx0 > tx1), and 64 bits of kept tiles:
//  - a rectangle of at most 64 tiles: the mask of kept tiles (bit
//    (ty - ty0) * width + (tx - tx0));
//  - a larger one: its rows are grouped into at most BIG_BANDS bands of
//    ceil(th / BIG_BANDS) tile rows and its columns into at most 2^BIG_BITS
//    blocks of ceil(tw / 2^BIG_BITS) tiles; field r (2 BIG_BITS bits) holds
//    band r's kept blocks as the interval bx0 | bx1 << BIG_BITS (empty when
//    bx0 > bx1), and the band keeps every tile of those blocks.
__host__ __device__ inline uint4 make_bin(int tx0, int ty0, int tx1, int ty1, uint64_t mask)
{
    return make_uint4((uint32_t)tx0 | ((uint32_t)ty0 << 16), (uint32_t)tx1 | ((uint32_t)ty1 << 16), (uint32_t)mask,
                      (uint32_t)(mask >> 32));
}
#ifndef CS_BIG_BANDS
#define CS_BIG_BANDS 4
#endif
constexpr int BIG_BANDS = CS_BIG_BANDS;
constexpr int BIG_BITS = 32 / BIG_BANDS;
constexpr uint64_t BIG_FIELD = (1ull << (2 * BIG_BITS)) - 1ull;
constexpr uint64_t big_empty()
{
    uint64_t m = 0;
    for (int r = 0; r < BIG_BANDS; ++r) m |= ((1ull << BIG_BITS) - 1ull) << (2 * BIG_BITS * r);
    return m;
}
constexpr uint64_t BIG_EMPTY = big_empty(); // every band of a large rectangle empty
__host__ __device__ inline int big_bw(int tw) { return (tw + (1 << BIG_BITS) - 1) >> BIG_BITS; }
__host__ __device__ inline int big_bh(int th) { return (th + BIG_BANDS - 1) / BIG_BANDS; }
__host__ __device__ inline uint64_t big_field(int bx0, int bx1, int r)
{
    return ((uint64_t)bx0 | ((uint64_t)bx1 << BIG_BITS)) << (2 * BIG_BITS * r);
}
// Band r of a large rectangle: its first tile row (rectangle-relative) *row0,
// its tile rows *nrow, first kept tile column *col0 and kept columns *ncol
// (both 0 when the band is empty).
__host__ __device__ inline void big_band(uint64_t mask, int tw, int th, int r, int *row0, int *nrow, int *col0,
                                         int *ncol)
{
    const int bw = big_bw(tw), bh = big_bh(th);
    const uint32_t f = (uint32_t)(mask >> (2 * BIG_BITS * r)) & (uint32_t)BIG_FIELD;
    const int bx0 = (int)(f & ((1u << BIG_BITS) - 1u)), bx1 = (int)(f >> BIG_BITS);
    *row0 = r * bh;
    *nrow = th - r * bh < bh ? th - r * bh : bh;
    const int cend = (bx1 + 1) * bw < tw ? (bx1 + 1) * bw : tw;
    *col0 = bx0 * bw;
    *ncol = (bx0 <= bx1 && *nrow > 0) ? cend - bx0 * bw : 0;
    if (*ncol == 0) *nrow = 0;
}
__device__ inline uint32_t bin_count(uint4 b)
{
    const int tx0 = (int)(b.x & 0xFFFFu), ty0 = (int)(b.x >> 16), tx1 = (int)(b.y & 0xFFFFu), ty1 = (int)(b.y >> 16);
    if (tx0 > tx1 || ty0 > ty1) return 0u;
    const int tw = tx1 - tx0 + 1, th = ty1 - ty0 + 1;
    const uint64_t mask = (uint64_t)b.z | ((uint64_t)b.w << 32);
    if (tw * th <= 64) return (uint32_t)(__popc(b.z) + __popc(b.w));
    uint32_t c = 0;
#pragma unroll
    for (int r = 0; r < BIG_BANDS; ++r) {
        int row0, nrow, col0, ncol;
        big_band(mask, tw, th, r, &row0, &nrow, &col0, &ncol);
        c += (uint32_t)(nrow * ncol);
    }
    return c;
}

// Up to two word ranges that a kernel clears on the side (each block its
// share), in place of clearing launches of their own: the ranges' next users
// run after the kernel in the stream.
struct ZeroSpans {
    uint32_t *p[2];
    uint32_t n[2];
};
__device__ inline void zero_share(const ZeroSpans &z)
{
    const uint32_t nb = gridDim.x * gridDim.y, b = blockIdx.y * gridDim.x + blockIdx.x;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (!z.p[k]) continue;
        const uint32_t per = (z.n[k] + nb - 1) / nb;
        const uint32_t lo = min(b * per, z.n[k]), hi = min(lo + per, z.n[k]);
        for (uint32_t i = lo + threadIdx.x; i < hi; i += blockDim.x) z.p[k][i] = 0u;
    }
}

// Layout of a frame's counter buffer (32-bit words):
//   [0, CNT_WORDS)            counters read back by the host:
//     CNT_SORT_ERR: a radix-sort look-back wait ran out of its bound (never expected)
//     CNT_SCAN_TILE: tile claims of the pair-offset scan
//   [CNT_QUEUE, CNT_QUEUE_B)  the forward compositing's work queues' claim
//                             counters, one per QUEUE_STRIDE words: device-scope
//                             atomics on one memory block serialise, so each
//                             queue's counter sits in a block of its own
//   [CNT_QUEUE_B, CNT_STATUS) the backward compositing's (cleared with the rest
//                             when the forward starts)
//   [CNT_STATUS, ...)         the pair-offset scan's look-back status (u64 per tile)
enum : int { CNT_PAIRS = 0, CNT_PAIRS_EFF = 1, CNT_OVERFLOW = 2, CNT_SORT_ERR = 3, CNT_SCAN_TILE = 20, CNT_WORDS = 32 };
constexpr int QUEUE_STRIDE = 1024; // 4 KiB
constexpr int CNT_QUEUE = CNT_WORDS;
constexpr int QUEUE_WORDS = NUM_QUEUES * QUEUE_STRIDE;
constexpr int CNT_QUEUE_B = CNT_QUEUE + QUEUE_WORDS;
constexpr int CNT_STATUS = CNT_QUEUE_B + QUEUE_WORDS;

// Host-visible debug record (mirrors cs_debug_convex of the public header).
struct DebugConvex {
    int32_t status, T;
    int32_t hull[MAXK];
    uint32_t depth_key;
    int32_t clampmask;
    double A[MAXK], B[MAXK], C[MAXK];
    double d, delta_p, sigma_p;
    float rgb[3];
    int32_t tile_rect[4];
};

} // namespace cs
