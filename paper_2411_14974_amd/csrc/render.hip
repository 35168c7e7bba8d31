// Per-tile compositing, forward and backward (gfx950).
//
// One workgroup per tile (8x8, 16x16 or 32x32 pixels), one pixel per thread,
// in a persistent grid that pulls tiles of all views from per-XCD work queues.
// The tile's depth-ordered convex list is streamed through LDS in batches of
// records; every thread walks the batch front to back and evaluates, for its pixel,
//   x2_j = log2(e) delta' L_j(q)           (FP64: hull lines, Supp. B scaling)
//   phi  = LogSumExp of the x_j            (Sec. 3.1 Eq. smoothness, base 2)
//   I    = Sigmoid(-sigma' phi)            (Sec. 3.1 Eq. sharpness)
//   alpha = o I,  C += T alpha c,  T *= 1 - alpha   (Sec. 3.2 compositing eq.)
// skipping pairs with alpha < eps_alpha and stopping after the convex that
// brings T below t_min.  Only x2_j is FP64: at the configured sharpness the
// indicator moves by sigma' delta' / 4 per pixel of line offset, so the line
// must be exact to ~1e-9 px; everything after it runs in FP32 on the hardware
// exp2 / log2 / reciprocal.
//
// The backward kernel walks the same lists back to front from each pixel's
// last contributor, recomputing alpha with the same function (bit-identical
// decisions), recovering T_n = T_{n+1} / (1 - alpha_n); the per-pair gradients
// are reduced over the wavefront (lane swaps + DPP), summed over the
// workgroup's waves in LDS, and leave as one float atomic add per
// (convex, value) and workgroup.
#include <algorithm>
#include <cstddef>
#include <mutex>
#include <unordered_map>
#include <utility>

#include "common.hpp"

namespace cs {

namespace {

// A pixel's (u, y) lies in a record's box (box_u, box_v), outside of which alpha < eps.
__device__ __forceinline__ bool in_box(uint32_t box_u, uint32_t box_v, int u, int y)
{
    return u >= (int)(box_u & 0xFFFFu) && u <= (int)(box_u >> 16) && y >= (int)(box_v & 0xFFFFu) &&
           y <= (int)(box_v >> 16);
}

template <int K> struct PairEval {
    float I, omI, alpha, oma, phi2, inv_sum;
    float e[K];  // 2^(x2_j - max)
    float x2[K]; // x2_j rounded to float
};

// Runs the statements with the compile-time constant NLL equal to the wave-
// uniform hull size TV (3..K; records in tile lists always have T >= 3).
#define CS_NL_CASE(n, K, ...) \
    case n:                   \
        if constexpr (n <= K) { \
            constexpr int NLL = n; \
            __VA_ARGS__;      \
        }                     \
        break;
#define CS_DISPATCH_NL(K, TV, ...)                                                                               \
    switch (TV) {                                                                                                \
        CS_NL_CASE(3, K, __VA_ARGS__) CS_NL_CASE(4, K, __VA_ARGS__) CS_NL_CASE(5, K, __VA_ARGS__)                \
        CS_NL_CASE(6, K, __VA_ARGS__) CS_NL_CASE(7, K, __VA_ARGS__) CS_NL_CASE(8, K, __VA_ARGS__) default: break; \
    }

// The FP32 part of a pair evaluation from the line values x (m: their
// maximum, full: the pair passed the max-line test): softmax weights,
// LogSumExp, indicator and alpha.  Returns whether the pair contributes.
template <int K, int NL>
__device__ __forceinline__ bool finish_pair(const RecHeader &h, const double *x, double m, bool full, float eps,
                                            PairEval<K> &pe)
{
    const float mf = (float)m;
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < NL; ++j) {
        const float xf = (float)x[j];
        const float e = __builtin_amdgcn_exp2f(xf - mf);
        pe.e[j] = e;
        pe.x2[j] = xf;
        s += e;
    }
    pe.inv_sum = __builtin_amdgcn_rcpf(s);
    const float phi2 = mf + __builtin_amdgcn_logf(s);
    const float z = h.sigma_p * phi2; // I = 1 / (1 + 2^z)
    const float ez = __builtin_amdgcn_exp2f(-fabsf(z));
    const float r = __builtin_amdgcn_rcpf(1.0f + ez);
    pe.I = z > 0.0f ? ez * r : r;
    pe.omI = z > 0.0f ? r : ez * r;
    pe.alpha = h.opacity * pe.I;
    pe.oma = (1.0f - h.opacity) + h.opacity * pe.omI;
    pe.phi2 = phi2;
    return full && !(pe.alpha < eps);
}

// The one evaluation of a (pixel, convex) pair shared by both passes, called
// by every lane of the wavefront (live: the pixel still takes convexes).
// Returns whether the pair contributes: the pixel lies in the record's pixel
// box (tested), the largest line value passes the skip threshold (full), and
// alpha >= eps_alpha.  When some lane passes the threshold, every field of pe
// is computed, and finite, for every lane, so that callers can use them
// without branches; otherwise the wavefront leaves early.
//
// The record (header and all K line slots) is read from LDS in one burst of
// 16-byte reads with a single wait (a branch per line would serialise the LDS
// round trips; slots past T hold null lines).  The lines are evaluated in FP64; the exponents are taken
// as differences of the FP32-rounded values (phi already starts from the
// rounded maximum, and where the sigmoid is sensitive |x2| is small).
// NL: the record's hull size T (its line count), a compile-time constant of
// the caller's dispatch on the wave-uniform T, so that only the hull's lines
// are read and evaluated.
template <int K, int NL>
__device__ __forceinline__ bool eval_pair(const uint8_t *rec, bool live, int u, int y, float pxf, float pyf,
                                          float eps, PairEval<K> &pe, bool &tested, bool &full)
{
    static_assert(NL >= 3 && NL <= K, "hull size out of range");
    // the pixel box first: its test then waits for it alone, with the line
    // reads still in flight
    const uint2 box = *reinterpret_cast<const uint2 *>(rec + offsetof(RecHeader, box_u));
    const RecHeader h = *reinterpret_cast<const RecHeader *>(rec);
    double L[3 * NL + 1]; // one spare slot: odd 3 NL reads one double past the last line (still in the record)
    const double2 *l2 = reinterpret_cast<const double2 *>(rec + REC_HEADER);
#pragma unroll
    for (int q = 0; q < (3 * NL + 1) / 2; ++q) {
        const double2 w = l2[q];
        L[2 * q] = w.x;
        L[2 * q + 1] = w.y;
    }
    tested = live & in_box(box.x, box.y, u, y); // no short circuit: no branch around the box test
    const double dx = (double)(pxf - h.ox), dy = (double)(pyf - h.oy);
    double x[NL];
    double m = -INFINITY;
#pragma unroll
    for (int j = 0; j < NL; ++j) {
        x[j] = fma(L[3 * j], dx, fma(L[3 * j + 1], dy, L[3 * j + 2]));
        m = fmax(m, x[j]);
    }
    // LogSumExp >= its largest term: past thr2 alpha < eps for certain
    full = tested && (m <= (double)h.thr2);
    if (!__any(full)) return false;
    return finish_pair<K, NL>(h, x, m, full, eps, pe);
}

// First half of a whole-wavefront sum of NP values (NP a multiple of 4), by
// transposition: a 32-lane swap (v_permlane32_swap) pairs value j with value
// j + NP/2 so that one add leaves the two half-wave sums of j in the lower
// half and of j + NP/2 in the upper half; a 16-lane swap (v_permlane16_swap)
// does the same between rows.  On return lane l of row r holds in v[j],
// j < NP/4, a partial sum of value j + r NP/4 (the row reduction finishes it).
template <int NP> __device__ __forceinline__ void wave_to_rows(float *v)
{
    static_assert(NP % 4 == 0, "pad the values to a multiple of 4");
    constexpr int H = NP / 2, Q = NP / 4;
#pragma unroll
    for (int j = 0; j < H; ++j) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[j]), __float_as_uint(v[j + H]), false, false);
        v[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[j]), __float_as_uint(v[j + Q]), false, false);
        v[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
}

// Row totals of Q values over the 16 lanes of each row, transposed like the
// swaps above: four DPP stages pair every lane with a partner (row mirror,
// half-row mirror, quad swap of 2, of 1), and at each stage the registers are
// taken in pairs: both values of a pair are added to the partner's, and the
// lanes on one side of the stage keep the first sum, the others the second
// (an unpaired last register is summed in place).  The register count halves
// per stage, so Q values cost about 1.5 (Q + Q/2 + Q/4 + Q/8) instructions
// where plain row sums take 4 Q; at the end lane i of a row holds the row
// total of value rr_value(Q, i).
__host__ __device__ constexpr bool rr_keeps_first(int stage, int i)
{
    return stage == 0 ? (i < 8) : stage == 1 ? ((i & 7) < 4) : stage == 2 ? ((i & 2) == 0) : ((i & 1) == 0);
}
__host__ __device__ constexpr int rr_value(int Q, int lane)
{
    int reg[16] = {};
    int m = Q;
    for (int k = 0; k < Q; ++k) reg[k] = k;
    for (int s = 0; s < 4; ++s) {
        const bool first = rr_keeps_first(s, lane);
        int nm = 0;
        for (int p = 0; p + 1 < m; p += 2) reg[nm++] = first ? reg[p] : reg[p + 1];
        if (m & 1) reg[nm++] = reg[m - 1];
        m = nm;
    }
    return reg[0];
}
// 4 bits per lane: the value whose total the lane holds
__host__ __device__ constexpr uint64_t rr_map(int Q)
{
    uint64_t t = 0;
    for (int i = 0; i < 16; ++i) t |= (uint64_t)rr_value(Q, i) << (4 * i);
    return t;
}
// the lanes that hold a value no lower lane of the row holds
__host__ __device__ constexpr uint32_t rr_first_lanes(int Q)
{
    uint32_t f = 0;
    for (int i = 0; i < 16; ++i) {
        bool first = true;
        for (int j = 0; j < i; ++j) first = first && rr_value(Q, j) != rr_value(Q, i);
        if (first) f |= 1u << i;
    }
    return f;
}
// every value's total reaches exactly one first lane
__host__ __device__ constexpr bool rr_covers(int Q)
{
    const uint32_t f = rr_first_lanes(Q);
    int holders[16] = {};
    for (int i = 0; i < 16; ++i)
        if ((f >> i) & 1u) ++holders[rr_value(Q, i)];
    bool ok = true;
    for (int q = 0; q < 16; ++q) ok = ok && holders[q] == (q < Q ? 1 : 0);
    return ok;
}
static_assert(rr_covers(4) && rr_covers(5) && rr_covers(6) && rr_covers(7) && rr_covers(8),
              "row reduction lane map");
template <int S, int M> __device__ __forceinline__ void rr_stage(float *v, int li)
{
    constexpr int CTRL = S == 0 ? 0x140 : S == 1 ? 0x141 : S == 2 ? 0x4E : 0xB1; // DPP partner of the stage
    const bool first = rr_keeps_first(S, li);
#pragma unroll
    for (int p = 0; p + 1 < M; p += 2) {
        // the sums first, then the choice: a choice between the two array
        // elements would become a per-lane index into the array
        const float a = v[p], b = v[p + 1];
        const float sa = a + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(a), CTRL, 0xF, 0xF, true));
        const float sb = b + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(b), CTRL, 0xF, 0xF, true));
        v[p / 2] = first ? sa : sb;
    }
    if constexpr ((M & 1) != 0) {
        const float a = v[M - 1];
        v[M / 2] = a + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(a), CTRL, 0xF, 0xF, true));
    }
}
template <int Q> __device__ __forceinline__ float row_reduce(float *v)
{
    static_assert(Q >= 1 && Q <= 16, "at most 16 values per row");
    const int li = threadIdx.x & 15;
    constexpr int M1 = (Q + 1) / 2, M2 = (M1 + 1) / 2, M3 = (M2 + 1) / 2;
    rr_stage<0, Q>(v, li);
    rr_stage<1, M1>(v, li);
    rr_stage<2, M2>(v, li);
    rr_stage<3, M3>(v, li);
    return v[0];
}

// Pixel of a thread within its tile: each wavefront covers an 8x8 square
// (a compact patch: more of its lanes fall inside the same convex than in a
// 16x4 strip), wavefronts tile the TILE x TILE tile row-major.
template <int TILE> __device__ __forceinline__ void tile_pixel(int &dx, int &dy)
{
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    dx = (w % (TILE / 8)) * 8 + (l & 7);
    dy = (w / (TILE / 8)) * 8 + (l >> 3);
}


// Can a record reach alpha >= eps_alpha at a pixel centre of the RW x RH
// rectangle [su, su + RW - 1] x [sv, sv + RH - 1] (a wavefront's pixels)?  Its pixel box must meet the square, and no
// hull line may keep x2 above the skip threshold over all pixel centres of
// the square's part of the box (then the pair evaluation skips every one of
// them).  A line's minimum over a rectangle is at a corner; the margin covers
// the rounding of this test and of the pair evaluation.
template <int K, int RW = 8, int RH = 8> __device__ __forceinline__ bool square_meets(const uint8_t *rec, int su, int sv)
{
    const RecHeader h = *reinterpret_cast<const RecHeader *>(rec);
    double L[3 * K + 1];
    const double2 *l2 = reinterpret_cast<const double2 *>(rec + REC_HEADER);
#pragma unroll
    for (int q = 0; q < (3 * K + 1) / 2; ++q) {
        const double2 w = l2[q];
        L[2 * q] = w.x;
        L[2 * q + 1] = w.y;
    }
    const int u0 = max(su, (int)(h.box_u & 0xFFFFu)), u1 = min(su + RW - 1, (int)(h.box_u >> 16));
    const int v0 = max(sv, (int)(h.box_v & 0xFFFFu)), v1 = min(sv + RH - 1, (int)(h.box_v >> 16));
    if (u0 > u1 || v0 > v1) return false;
    const double a0 = (double)u0 + 0.5 - (double)h.ox, a1 = (double)u1 + 0.5 - (double)h.ox;
    const double c0 = (double)v0 + 0.5 - (double)h.oy, c1 = (double)v1 + 0.5 - (double)h.oy;
    const double lim = (double)h.thr2 + 1e-3;
    bool ok = true;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const double mn = L[3 * j + 2] + fmin(L[3 * j] * a0, L[3 * j] * a1) + fmin(L[3 * j + 1] * c0, L[3 * j + 1] * c1);
        ok = ok && !(mn > lim); // null lines never reject
    }
    return ok;
}

// Software pipeline of the LDS record batches.  While a batch is composited
// from LDS, the records of the next batch are in flight into registers and
// the list ids of the batch after that into a register, so a record load never
// waits on its id load; one LDS record buffer and two LDS id buffers suffice.
template <int K, int NT, int BATCH> constexpr int pipe_regs() { return (BATCH * (rec_stride(K) / 16) + NT - 1) / NT; }

// native 16-byte vector (HIP's uint4 is a struct with a union, which keeps a
// register array of it in scratch)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t pipe_load_id(const uint32_t *__restrict__ ids, int base, int cnt)
{
    return (int)threadIdx.x < cnt ? ids[base + threadIdx.x] : 0u;
}

template <int K, int NT, int NL>
__device__ __forceinline__ void pipe_load_records(u32x4 (&pre)[NL], const uint32_t *s_ids,
                                                  const uint8_t *__restrict__ records, int cnt)
{
    constexpr int CH = rec_stride(K) / 16;
    const int last = cnt * CH - 1; // chunks past the batch reload its last chunk (never stored)
#pragma clang loop unroll(full)
    for (int r = 0; r < NL; ++r) {
        const int c = min((int)threadIdx.x + r * NT, last);
        const int e = c / CH, part = c - e * CH;
        pre[r] = reinterpret_cast<const u32x4 *>(records + (size_t)s_ids[e] * rec_stride(K))[part];
    }
}

template <int K, int NT>
__device__ __forceinline__ void load_records_direct(uint4 *lds, const uint32_t *s_ids, const uint8_t *__restrict__ records,
                                                    int cnt)
{
    constexpr int CH = rec_stride(K) / 16;
    for (int c = threadIdx.x; c < cnt * CH; c += NT) {
        const int e = c / CH, part = c - e * CH;
        reinterpret_cast<u32x4 *>(lds)[c] = reinterpret_cast<const u32x4 *>(records + (size_t)s_ids[e] * rec_stride(K))[part];
    }
}

template <int K, int NT, int NL>
__device__ __forceinline__ void pipe_store_records(const u32x4 (&pre)[NL], uint4 *lds, int cnt)
{
    constexpr int CH = rec_stride(K) / 16;
#pragma clang loop unroll(full)
    for (int r = 0; r < NL; ++r) {
        const int c = (int)threadIdx.x + r * NT;
        if (c < cnt * CH) reinterpret_cast<u32x4 *>(lds)[c] = pre[r];
    }
}

// Work distribution of the persistent compositing grid.  Items (tiles of all
// views, in the order given by `order`, or natural order) are split into one
// contiguous band per XCD; a workgroup takes items from the queue of its own XCD
// (workgroups are dealt to the 8 XCDs round-robin), so neighbouring tiles, which
// share convex records, meet in one L2, and steals from the other queues when
// its own runs dry.  Every workgroup exits once all queues are empty.
// CHUNK items are claimed per atomic (the workgroup keeps the rest of its
// run in cnext..cend).
template <uint32_t CHUNK>
__device__ __forceinline__ uint32_t next_item(uint32_t *queues, uint32_t total, int &q, int &tried,
                                              uint32_t &cnext, uint32_t &cend, uint32_t *s_item)
{
    if (threadIdx.x == 0) {
        uint32_t item = 0xFFFFFFFFu;
        if (cnext < cend) {
            item = cnext++;
        } else {
            const uint32_t per = (total + NUM_QUEUES - 1) / NUM_QUEUES;
            while (tried < NUM_QUEUES) {
                const uint32_t lo = q * per, hi = min(total, lo + per);
                if (lo < hi) {
                    const uint32_t k = atomicAdd(&queues[QUEUE_STRIDE * q], CHUNK);
                    if (lo + k < hi) {
                        item = lo + k;
                        cnext = item + 1;
                        cend = min(hi, item + CHUNK);
                        break;
                    }
                }
                q = (q + 1) % NUM_QUEUES;
                ++tried;
            }
        }
        *s_item = item;
    }
    __syncthreads();
    const uint32_t item = *s_item;
    __syncthreads();
    return item;
}

__device__ __forceinline__ int find_view(const ViewDesc *__restrict__ views, int nviews, int gt)
{
    int lo = 0, hi = nviews - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_off <= gt) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The workgroup's work counters (per-lane tested / full / hull-size sums and
// the wavefront's evaluation count, which every lane of a wavefront holds),
// stored in the workgroup's own slot of EVAL_FIELDS words.
__device__ __forceinline__ void store_work_counts(unsigned long long *evalcount, unsigned long long *s_ev,
                                                  uint32_t nevals, uint32_t nfull, uint32_t nsumT, uint32_t nwave)
{
    unsigned long long c = nevals, f = nfull, t = nsumT;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        c += __shfl_xor(c, o, 64);
        f += __shfl_xor(f, o, 64);
        t += __shfl_xor(t, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&s_ev[EV_TESTED], c);
        atomicAdd(&s_ev[EV_FULL], f);
        atomicAdd(&s_ev[EV_SUM_T], t);
        atomicAdd(&s_ev[EV_WAVES], (unsigned long long)nwave);
    }
    __syncthreads();
    if (threadIdx.x < EVAL_FIELDS) evalcount[EVAL_FIELDS * blockIdx.x + threadIdx.x] = s_ev[threadIdx.x];
}

} // namespace

// Tiles the forward claims per queue atomic: its per-tile cost is even enough
// that runs of 2 balance; the backward's varies more and claims one at a time.
constexpr uint32_t FWD_CHUNK = 2;

// 5 wavefronts per SIMD (at most 96 VGPRs): the compiler keeps a few values
// of the batch loop (one record prefetch register among them) in scratch,
// outside the record loop, and the extra wavefront hides more of the LDS and
// transcendental latency (0.183 -> 0.169 ms at 1M convexes, 1080p, against 4
// wavefronts and 106 VGPRs without spills).
template <int K, int TILE, int BATCH>
__global__ __launch_bounds__(TILE *TILE) __attribute__((amdgpu_waves_per_eu(5))) void render_fwd_kernel(
    const FrameHeader *__restrict__ frame, const uint32_t *__restrict__ order, uint32_t *__restrict__ queues,
    const uint2 *__restrict__ ranges, const uint32_t *__restrict__ ids,
    const uint8_t *__restrict__ records, RenderArgs ra, uint2 *__restrict__ pixstate,
    unsigned long long *__restrict__ evalcount, u32x4 *__restrict__ zero_acc, uint32_t zero_n4)
{
    constexpr int NT = TILE * TILE;
    constexpr int CH = rec_stride(K) / 16;
    static_assert(BATCH <= NT, "one id per thread");
    static_assert(BATCH <= 64, "one ballot bit per batch entry");
    __shared__ uint4 lds[BATCH * CH];
    __shared__ uint32_t s_ids[2][BATCH];
    __shared__ uint32_t s_item;
    __shared__ unsigned long long s_ev[EVAL_FIELDS];
    const int lane = threadIdx.x & 63, wbit = threadIdx.x >> 6;
    if (threadIdx.x < EVAL_FIELDS) s_ev[threadIdx.x] = 0ull;
    constexpr int NL = pipe_regs<K, NT, BATCH>();
    u32x4 pre[NL];
    uint32_t idr = 0;
    const ViewDesc *views = reinterpret_cast<const ViewDesc *>(frame + 1);
    const int nviews = (int)frame->nviews;
    const uint32_t total_tiles = frame->total_tiles;
    int q = blockIdx.x % NUM_QUEUES, tried = 0;
    uint32_t cnext = 0, cend = 0;
    // work counters: pairs tested / pairs past the max-line test (the hull
    // sizes and wavefront evaluations of the same pairs are counted by the
    // backward walk, where they cost less)
    uint32_t nevals = 0, nfull = 0;
    // the backward's accumulators (zero_n4 16-byte words, or none) are cleared
    // here, one slice per tile item, by stores that overlap the compositing
    const uint32_t zper = total_tiles ? (zero_n4 + total_tiles - 1) / total_tiles : 0u;
    for (;;) {
        const uint32_t item = next_item<FWD_CHUNK>(queues, total_tiles, q, tried, cnext, cend, &s_item);
        if (item == 0xFFFFFFFFu) break;
        if (zper) {
            const uint32_t z0 = min(item * zper, zero_n4), z1 = min(z0 + zper, zero_n4);
            for (uint32_t z = z0 + threadIdx.x; z < z1; z += NT) zero_acc[z] = u32x4{0u, 0u, 0u, 0u};
        }
        const int gt = order ? (int)order[item] : (int)item;
        const int v = find_view(views, nviews, gt);
        const ViewDesc &vd = views[v];
        const int lt = gt - vd.tile_off;
        const int tx = lt % vd.tiles_x, ty = lt / vd.tiles_x;
        const int W = vd.cam.W, H = vd.cam.H;
        int pdx, pdy;
        tile_pixel<TILE>(pdx, pdy);
        const int u = tx * TILE + pdx, y = ty * TILE + pdy;
        const int su = tx * TILE + (wbit % (TILE / 8)) * 8, sv = ty * TILE + (wbit / (TILE / 8)) * 8; // wave's square
        const bool inside = u < W && y < H;
        const float pxf = (float)u + 0.5f, pyf = (float)y + 0.5f;
        const uint2 rg = ranges[gt];
        const int start = (int)rg.x, end = (int)rg.y;

        float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, Tlast = 1.0f;
        int nend = 0;
        bool done = !inside;
        const int nb = (end - start + BATCH - 1) / BATCH;
        if (nb > 0) { // prologue: ids of batches 0 and 1, records of batch 0
            idr = pipe_load_id(ids, start, min(BATCH, end - start));
            if ((int)threadIdx.x < BATCH) s_ids[0][threadIdx.x] = idr;
            if (nb > 1) idr = pipe_load_id(ids, start + BATCH, min(BATCH, end - start - BATCH));
            __syncthreads();
            pipe_load_records<K, NT, NL>(pre, s_ids[0], records, min(BATCH, end - start));
        }
        for (int bi = 0; bi < nb; ++bi) {
            const int base = start + bi * BATCH;
            const int cnt = min(BATCH, end - base);
            __syncthreads();
            pipe_store_records<K, NT, NL>(pre, lds, cnt);
            if ((int)threadIdx.x < BATCH) s_ids[(bi + 1) & 1][threadIdx.x] = idr;
            __syncthreads();
            if (bi + 2 < nb) idr = pipe_load_id(ids, base + 2 * BATCH, min(BATCH, end - base - 2 * BATCH));
            if (bi + 1 < nb) pipe_load_records<K, NT, NL>(pre, s_ids[(bi + 1) & 1], records, min(BATCH, end - base - BATCH));
            // the wave's records of this batch (lane e tests entry e against
            // the wave's square), front to back in a wave-uniform walk
            uint64_t M = 0;
            if (!__all(done)) {
                const bool meets = lane < cnt && square_meets<K>(reinterpret_cast<const uint8_t *>(&lds[min(lane, BATCH - 1) * CH]), su, sv);
                M = __ballot(meets);
            }
            while (M) {
                const int e = __builtin_ctzll(M);
                M &= M - 1;
                const uint8_t *rec = reinterpret_cast<const uint8_t *>(&lds[e * CH]);
                PairEval<K> pe;
                bool tested, full;
                // all K line slots (slots past T hold null lines): a dispatch on
                // T costs the forward more than the null lines it saves
                const bool hit = eval_pair<K, K>(rec, !done, u, y, pxf, pyf, ra.eps_alpha, pe, tested, full);
                nevals += tested;
                nfull += full;
                if (hit) {
                    const RecHeader &h = *reinterpret_cast<const RecHeader *>(rec);
                    const float w = T * pe.alpha;
                    C0 = fmaf(w, h.rgb[0], C0);
                    C1 = fmaf(w, h.rgb[1], C1);
                    C2 = fmaf(w, h.rgb[2], C2);
                    Tlast = T;
                    T = T * pe.oma;
                    nend = base - start + e + 1;
                    done = T < ra.t_min;
                }
                if (__all(done)) break;
            }
            if (__syncthreads_and(done)) break;
        }
        if (inside) {
            const size_t pix = (size_t)y * W + u;
            float *o = vd.out_rgb + 3 * pix;
            o[0] = fmaf(T, ra.bg[0], C0);
            o[1] = fmaf(T, ra.bg[1], C1);
            o[2] = fmaf(T, ra.bg[2], C2);
            pixstate[vd.pix_off + pix] = make_uint2((uint32_t)nend, __float_as_uint(Tlast));
        }
    }
    if (evalcount) store_work_counts(evalcount, s_ev, nevals, nfull, 0u, 0u);
}

// Compact per-pair gradient values of a record with NL hull lines: a[NL]
// b[NL] c[NL] (base-2 line coefficients), sigma', opacity, rgb[3], and
// sum_j dL/dx2_j x2_j, padded with zeros to a multiple of 4 for the wave sums.
template <int NL> constexpr int bwd_values() { return 3 * NL + 6; }
template <int NL> constexpr int bwd_padded() { return (bwd_values<NL>() + 3) & ~3; }

// Slot of compact value qv of a record with T lines in the accumulator row
// a[K] b[K] c[K] sigma' opacity rgb[3] x2sum.
template <int K> __device__ __forceinline__ int acc_slot(int qv, int T)
{
    return qv < T ? qv : qv < 2 * T ? K + (qv - T) : qv < 3 * T ? 2 * K + (qv - 2 * T) : 3 * K + (qv - 3 * T);
}

// Backward of one record for the wavefront's pixels: recompute the pair (the
// forward's decisions, bit for bit), recover T_n, form the pixel's gradient
// values, sum them over the wavefront and add the four row sums into the
// record's LDS slot (compact layout, bwd_padded<K>() floats).
// A pixel's state in the back-to-front walk: dL/dC, the transmittance after
// its last contributor, the transmittance before the pair being walked (T_n,
// recovered by division), and the colour composited behind it.
struct BwdPixel {
    float g0, g1, g2, Tlast, Tcur, B0, B1, B2;
    bool first;
};

// A pixel's compact gradient values of one record (see bwd_values), stored
// into val (ADD: added to it), and the pixel's walk advanced past the record.
template <int K, int NL, bool ADD>
__device__ __forceinline__ void pixel_values(const RecHeader &h, const PairEval<K> &pe, bool contrib, BwdPixel &P,
                                             float pxf, float pyf, float *val)
{
    // branch-free: a lane that does not contribute takes Tn = 0, which zeroes
    // all of its values (every pe field is finite)
    const float Tn = contrib ? (P.first ? P.Tlast : P.Tcur * __builtin_amdgcn_rcpf(pe.oma)) : 0.0f;
    const float dLda = Tn * (P.g0 * (h.rgb[0] - P.B0) + P.g1 * (h.rgb[1] - P.B1) + P.g2 * (h.rgb[2] - P.B2));
    const float ta = Tn * pe.alpha;
    float v[bwd_values<NL>()];
    v[3 * NL + 2] = P.g0 * ta;
    v[3 * NL + 3] = P.g1 * ta;
    v[3 * NL + 4] = P.g2 * ta;
    v[3 * NL + 1] = dLda * pe.I;
    const float dLdz = -dLda * h.opacity * pe.I * pe.omI; // I = Sigmoid(-z), z = sigma' phi
    v[3 * NL] = dLdz * pe.phi2 * (float)LN2;
    const float dLdphi2 = dLdz * h.sigma_p * (float)LN2;
    const float gs = dLdphi2 * pe.inv_sum; // dL/dx2_j = gs e_j (softmax weights)
    const float dxf = pxf - h.ox, dyf = pyf - h.oy;
    float gdl = 0.0f;
#pragma unroll
    for (int j = 0; j < NL; ++j) {
        const float gx = gs * pe.e[j];
        v[j] = gx * dxf;
        v[NL + j] = gx * dyf;
        v[2 * NL + j] = gx;
        gdl = fmaf(gx, pe.x2[j], gdl);
    }
    v[3 * NL + 5] = gdl;
#pragma unroll
    for (int qv = 0; qv < bwd_values<NL>(); ++qv) val[qv] = ADD ? val[qv] + v[qv] : v[qv];
    if (contrib) {
        P.first = false;
        P.Tcur = Tn;
        P.B0 = fmaf(pe.alpha, h.rgb[0], pe.oma * P.B0);
        P.B1 = fmaf(pe.alpha, h.rgb[1], pe.oma * P.B1);
        P.B2 = fmaf(pe.alpha, h.rgb[2], pe.oma * P.B2);
    }
}

template <int K, int NL>
__device__ __forceinline__ void bwd_record(const uint8_t *rec, bool live, int u, int y, float pxf, float pyf,
                                           float eps, BwdPixel &P, float *slot, bool &full)
{
    constexpr int NP = bwd_padded<NL>();
    constexpr int Q = NP / 4;
    PairEval<K> pe;
    bool tested;
    const bool contrib = eval_pair<K, NL>(rec, live, u, y, pxf, pyf, eps, pe, tested, full);
    if (__ballot(contrib) == 0ull) return; // wave-uniform
    const RecHeader &h = *reinterpret_cast<const RecHeader *>(rec);
    float val[NP];
    pixel_values<K, NL, false>(h, pe, contrib, P, pxf, pyf, val);
#pragma unroll
    for (int qv = bwd_values<NL>(); qv < NP; ++qv) val[qv] = 0.0f;
    // whole-wave sums even when few lanes contribute: lane-by-lane LDS atomics
    // serialise badly when a record covers the square
    wave_to_rows<NP>(val);
    const float total = row_reduce<Q>(val);
    const int li = threadIdx.x & 15;
    if ((rr_first_lanes(Q) >> li) & 1u) { // one lane per (row, value) adds the wave's sum
        const int qv = (int)((rr_map(Q) >> (4 * li)) & 15u);
        atomicAdd(slot + ((threadIdx.x & 63) >> 4) * Q + qv, total);
    }
}

template <int K, int TILE, int BATCH>
__global__ __launch_bounds__(TILE *TILE) void render_bwd_kernel(
    const FrameHeader *__restrict__ frame, const uint32_t *__restrict__ order, uint32_t *__restrict__ queues,
    const uint2 *__restrict__ ranges, const uint32_t *__restrict__ ids,
    const uint8_t *__restrict__ records, RenderArgs ra, const uint2 *__restrict__ pixstate,
    float *__restrict__ acc, unsigned long long *__restrict__ evalcount)
{
    constexpr int NT = TILE * TILE;
    constexpr int CH = rec_stride(K) / 16;
    constexpr int AS = acc_stride(K);
    constexpr int NP = bwd_padded<K>(); // LDS slot per batch entry (compact values of the largest hull)
    static_assert(BATCH <= NT, "one id per thread");
    static_assert(BATCH <= 64, "one ballot bit per batch entry");
    __shared__ uint4 lds[BATCH * CH];
    __shared__ uint32_t s_ids[BATCH];
    // per entry sums of the block's waves, flushed after each batch
    __shared__ float s_acc[BATCH * NP];
    __shared__ int s_maxn;
    __shared__ uint32_t s_item;
    __shared__ unsigned long long s_ev[EVAL_FIELDS];
    for (int c = threadIdx.x; c < BATCH * NP; c += NT) s_acc[c] = 0.0f;
    if (threadIdx.x < EVAL_FIELDS) s_ev[threadIdx.x] = 0ull;
    const ViewDesc *views = reinterpret_cast<const ViewDesc *>(frame + 1);
    const int nviews = (int)frame->nviews;
    const uint32_t total_tiles = frame->total_tiles;
    const int lane = threadIdx.x & 63, wbit = threadIdx.x >> 6;
    int q = blockIdx.x % NUM_QUEUES, tried = 0;
    uint32_t cnext = 0, cend = 0;
    uint32_t nfull = 0, nsumT = 0, nwave = 0;
    for (;;) {
        const uint32_t item = next_item<1>(queues, total_tiles, q, tried, cnext, cend, &s_item);
        if (item == 0xFFFFFFFFu) break;
        const int gt = order ? (int)order[item] : (int)item;
        const int v = find_view(views, nviews, gt);
        const ViewDesc &vd = views[v];
        const int lt = gt - vd.tile_off;
        const int tx = lt % vd.tiles_x, ty = lt / vd.tiles_x;
        const int W = vd.cam.W, H = vd.cam.H;
        int pdx, pdy;
        tile_pixel<TILE>(pdx, pdy);
        const int u = tx * TILE + pdx, y = ty * TILE + pdy;
        const int su = tx * TILE + (wbit % (TILE / 8)) * 8, sv = ty * TILE + (wbit / (TILE / 8)) * 8; // wave's square
        const bool inside = u < W && y < H;
        const float pxf = (float)u + 0.5f, pyf = (float)y + 0.5f;
        const int start = (int)ranges[gt].x;

        BwdPixel P{0.f, 0.f, 0.f, 1.f, 1.f, ra.bg[0], ra.bg[1], ra.bg[2], true};
        int nend = 0;
        if (inside) {
            const size_t pix = (size_t)y * W + u;
            const float *g = vd.dl_drgb + 3 * pix;
            P.g0 = g[0];
            P.g1 = g[1];
            P.g2 = g[2];
            const uint2 ps = pixstate[vd.pix_off + pix];
            nend = (int)ps.x;
            P.Tlast = __uint_as_float(ps.y);
            P.Tcur = P.Tlast;
        }
        if (threadIdx.x == 0) s_maxn = 0;
        __syncthreads();
        if (nend > 0) atomicMax(&s_maxn, nend);
        __syncthreads();
        const int maxn = s_maxn;
        int wmaxn = nend; // the wave's last contributor
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) wmaxn = max(wmaxn, __shfl_xor(wmaxn, o, 64));

        // batches walk the list back to front (the walk is VALU-bound: plain loads,
        // no prefetch registers)
        for (int hi = maxn; hi > 0; hi -= BATCH) {
            const int lo = max(hi - BATCH, 0);
            const int cnt = hi - lo;
            __syncthreads();
            if ((int)threadIdx.x < cnt) s_ids[threadIdx.x] = ids[start + lo + threadIdx.x];
            __syncthreads();
            load_records_direct<K, NT>(lds, s_ids, records, cnt);
            __syncthreads();
            // the wave's records of this batch before its last contributor, back to front
            const uint8_t *mine = reinterpret_cast<const uint8_t *>(&lds[min(lane, BATCH - 1) * CH]);
            const bool meets = lane < min(cnt, wmaxn - lo) && square_meets<K>(mine, su, sv);
            const int myT = reinterpret_cast<const RecHeader *>(mine)->T; // lane e: hull size of entry e
            uint64_t M = __ballot(meets);
            while (M) {
                const int e = 63 - __builtin_clzll(M);
                M &= ~(1ull << e);
                const uint8_t *rec = reinterpret_cast<const uint8_t *>(&lds[e * CH]);
                const int Tr = __builtin_amdgcn_readlane(myT, e);
                const bool live = lo + e < nend;
                bool full = false;
                CS_DISPATCH_NL(K, Tr, bwd_record<K, NLL>(rec, live, u, y, pxf, pyf, ra.eps_alpha, P, &s_acc[e * NP], full));
                nfull += full;
                nsumT += full ? (uint32_t)Tr : 0u;
                nwave += __any(full) ? 1u : 0u;
            }
            // one global atomic per (entry, value) for the whole workgroup; the
            // compact values of entry e go to the slots of its hull size
            __syncthreads();
            for (int c = threadIdx.x; c < cnt * NP; c += NT) {
                const int e = c / NP, qv = c - e * NP;
                float *src = &s_acc[c];
                const float a = *src;
                if (a != 0.0f) {
                    const int T = reinterpret_cast<const RecHeader *>(&lds[e * CH])->T;
                    unsafeAtomicAdd(&acc[(size_t)s_ids[e] * AS + acc_slot<K>(qv, T)], a);
                    *src = 0.0f;
                }
            }
        }
    }
    if (evalcount) store_work_counts(evalcount, s_ev, 0u, nfull, nsumT, nwave);
}

// ------------------------------------------------------------- launchers ---


#define CS_DISPATCH_K(K, ...)                                                                                      \
    switch (K) {                                                                                                   \
    case 3: { constexpr int KK = 3; __VA_ARGS__; } break;                                                          \
    case 4: { constexpr int KK = 4; __VA_ARGS__; } break;                                                          \
    case 5: { constexpr int KK = 5; __VA_ARGS__; } break;                                                          \
    case 6: { constexpr int KK = 6; __VA_ARGS__; } break;                                                          \
    case 7: { constexpr int KK = 7; __VA_ARGS__; } break;                                                          \
    case 8: { constexpr int KK = 8; __VA_ARGS__; } break;                                                          \
    default: break;                                                                                                \
    }

#define CS_DISPATCH_TILE(TILEV, ...)                                                                               \
    switch (TILEV) {                                                                                               \
    case 8: { constexpr int TT = 8, BF = 32, BBW = 32; __VA_ARGS__; } break;                                       \
    case 16: { constexpr int TT = 16, BF = 64, BBW = 64; __VA_ARGS__; } break;                                     \
    case 32: { constexpr int TT = 32, BF = 64, BBW = 64; __VA_ARGS__; } break;                                     \
    default: break;                                                                                                \
    }

namespace {
// Resident workgroups of a kernel on the whole device, cached per kernel.
template <class F> int persistent_grid(F kernel, int threads)
{
    static std::mutex mu;
    static std::unordered_map<const void *, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    const void *key = reinterpret_cast<const void *>(kernel);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int dev = 0, cus = 0, per = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0);
    const int g = std::max(1, cus) * std::max(1, per);
    cache[key] = g;
    return g;
}
} // namespace

// max_items bounds the grid (a persistent grid larger than the work only idles).
// Returns the grid size (the number of evalcount slots written).
int launch_render_fwd(hipStream_t st, int K, int tile, const FrameHeader *frame, const uint32_t *order,
                      uint32_t max_items, uint32_t *queues, const uint2 *ranges, const uint32_t *ids,
                      const uint8_t *records, const RenderArgs &ra, uint2 *pixstate, unsigned long long *evalcount,
                      float *zero_acc, size_t zero_floats)
{
    // the accumulator rows are whole 16-byte words (acc_stride is a multiple of 4)
    u32x4 *z4 = reinterpret_cast<u32x4 *>(zero_acc);
    const uint32_t n4 = zero_acc ? (uint32_t)(zero_floats / 4) : 0u;
    if (max_items == 0) return 0;
    int used = 0;
    CS_DISPATCH_K(K, CS_DISPATCH_TILE(tile, {
        auto kern = render_fwd_kernel<KK, TT, BF>;
        const int grid = std::min({persistent_grid(kern, TT * TT), (int)max_items, EVAL_SLOTS});
        hipLaunchKernelGGL(kern, dim3(grid), dim3(TT * TT), 0, st, frame, order, queues, ranges, ids, records, ra,
                           pixstate, evalcount, z4, n4);
        used = grid;
    }));
    return used;
}

// Returns the grid size (the number of evalcount slots written).
int launch_render_bwd(hipStream_t st, int K, int tile, const FrameHeader *frame, const uint32_t *order,
                      uint32_t max_items, uint32_t *queues, const uint2 *ranges, const uint32_t *ids,
                      const uint8_t *records, const RenderArgs &ra, const uint2 *pixstate, float *acc,
                      unsigned long long *evalcount)
{
    if (max_items == 0) return 0;
    int used = 0;
    CS_DISPATCH_K(K, CS_DISPATCH_TILE(tile, {
        auto kern = render_bwd_kernel<KK, TT, BBW>;
        const int grid = std::min({persistent_grid(kern, TT * TT), (int)max_items, EVAL_SLOTS});
        hipLaunchKernelGGL(kern, dim3(grid), dim3(TT * TT), 0, st, frame, order, queues, ranges, ids, records, ra,
                           pixstate, acc, evalcount);
        used = grid;
    }));
    return used;
}

// ------------------------------------------------------------ L1 loss ----

// block_sum (nullable): each block stores its sum of |rgb - target| in its
// own slot (same-address atomics from every block would serialise)
__global__ __launch_bounds__(256) void l1_grad_kernel(const float *__restrict__ rgb, const float *__restrict__ target,
                                                      size_t n, float scale, float *__restrict__ grad,
                                                      float *__restrict__ block_sum)
{
    __shared__ float s_w[4];
    float part = 0.0f;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float d = rgb[i] - target[i];
        grad[i] = d > 0.0f ? scale : (d < 0.0f ? -scale : 0.0f);
        part += fabsf(d);
    }
    if (block_sum) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
        if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = part;
        __syncthreads();
        if (threadIdx.x == 0) block_sum[blockIdx.x] = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
    }
}

// *loss += scale * (sum of the nb block sums): one workgroup
__global__ __launch_bounds__(1024) void sum_slots_kernel(const float *__restrict__ slots, int nb, float scale,
                                                         float *__restrict__ loss)
{
    __shared__ float s_w[16];
    float t = 0.0f;
    for (int b = threadIdx.x; b < nb; b += 1024) t += slots[b];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        float u = 0.0f;
        for (int w = 0; w < 16; ++w) u += s_w[w];
        *loss += u * scale;
    }
}

// Returns hipSuccess, or the error of the scratch allocation (loss only).
hipError_t launch_l1_grad(hipStream_t st, const float *rgb, const float *target, size_t n, float *grad, float *loss)
{
    if (n == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 2048);
    float *slots = nullptr;
    if (loss) {
        const hipError_t e = hipMallocAsync((void **)&slots, blocks * sizeof(float), st);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(l1_grad_kernel, dim3((unsigned)blocks), dim3(256), 0, st, rgb, target, n, 1.0f / (float)n,
                       grad, slots);
    if (loss) {
        hipLaunchKernelGGL(sum_slots_kernel, dim3(1), dim3(1024), 0, st, slots, (int)blocks, 1.0f / (float)n, loss);
        (void)hipFreeAsync(slots, st);
    }
    return hipSuccess;
}

} // namespace cs
