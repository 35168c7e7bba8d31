// Adaptive density control of the convex set (gfx950): the split / prune step
// between optimisation steps (paper Sec. 3.3, "Adaptive convex shape
// refinement"; Supp. Initialization & Hyperparameters) as on-device stream
// compaction and expansion.
//
//   classify : one thread per convex -> prune / keep / split (float32
//              decisions in a fixed order), per-block keep and split counts
//   scan     : one workgroup, exclusive scans of the block counts and totals
//   scatter  : block-local ranks from wave ballots; the block's kept
//              convexes are copied to their run of output rows, its split
//              ones' K children to their run after all kept convexes
//
// A child of convex i centred at its point k is the convex scaled by
// child_scale about p_k: points p_k + s (p_j - c), c the point mean; delta is
// kept, sigma and opacity are scaled, the SH coefficients are copied.
#include <algorithm>

#include "common.hpp"
#include "convexsplat.h"
#include "runtime.hpp"

namespace cs {

namespace {

constexpr int DN_BLOCK = 256;
constexpr int DN_SCAN_THREADS = 1024;
enum : uint8_t { DN_PRUNE = 0, DN_KEEP = 1, DN_SPLIT = 2 };

// Point mean and squared radius of a convex in float32: sums in point order,
// one division by K, squared distances as (dx dx + dy dy) + dz dz.
__device__ __forceinline__ void centre_radius(const float *p, int K, float &cx, float &cy, float &cz, float &r2)
{
    cx = p[0];
    cy = p[1];
    cz = p[2];
    for (int k = 1; k < K; ++k) {
        cx = cx + p[3 * k];
        cy = cy + p[3 * k + 1];
        cz = cz + p[3 * k + 2];
    }
    const float fk = (float)K;
    cx = cx / fk;
    cy = cy / fk;
    cz = cz / fk;
    r2 = 0.0f;
    for (int k = 0; k < K; ++k) {
        const float dx = p[3 * k] - cx, dy = p[3 * k + 1] - cy, dz = p[3 * k + 2] - cz;
        r2 = fmaxf(r2, (dx * dx + dy * dy) + dz * dz);
    }
}

__device__ __forceinline__ uint8_t decide(const float *p, int K, float opacity, float acc, float den,
                                          const cs_densify_params &dp)
{
    float cx, cy, cz, r2;
    centre_radius(p, K, cx, cy, cz, r2);
    if (opacity < dp.opacity_min || r2 > dp.size_max * dp.size_max) return DN_PRUNE;
    if (den > 0.0f && acc / den > dp.split_threshold) return DN_SPLIT;
    return DN_KEEP;
}

__global__ __launch_bounds__(DN_BLOCK) void densify_classify_kernel(int n, int K, const float *__restrict__ points,
                                                                    const float *__restrict__ opacity,
                                                                    const float *__restrict__ accum,
                                                                    const float *__restrict__ denom,
                                                                    cs_densify_params dp, uint8_t *__restrict__ code,
                                                                    uint32_t *__restrict__ blk)
{
    __shared__ uint32_t s_cnt[2];
    if (threadIdx.x < 2) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const int i = blockIdx.x * DN_BLOCK + threadIdx.x;
    uint8_t c = DN_PRUNE;
    if (i < n) {
        c = decide(points + (size_t)i * 3 * K, K, opacity[i], accum[i], denom[i], dp);
        code[i] = c;
    }
    const uint32_t nk = (uint32_t)__popcll(__ballot(i < n && c == DN_KEEP));
    const uint32_t ns = (uint32_t)__popcll(__ballot(i < n && c == DN_SPLIT));
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&s_cnt[0], nk);
        atomicAdd(&s_cnt[1], ns);
    }
    __syncthreads();
    if (threadIdx.x < 2) blk[2 * blockIdx.x + threadIdx.x] = s_cnt[threadIdx.x];
}

// Exclusive scans of the per-block keep and split counts (in place) and the
// totals (keep, split) in tot[0..1].
__global__ __launch_bounds__(DN_SCAN_THREADS) void densify_scan_kernel(int nb, uint32_t *__restrict__ blk,
                                                                      uint32_t *__restrict__ tot)
{
    __shared__ uint32_t s_part[2][DN_SCAN_THREADS];
    const int t = threadIdx.x;
    const int per = (nb + DN_SCAN_THREADS - 1) / DN_SCAN_THREADS;
    const int b0 = min(nb, t * per), b1 = min(nb, b0 + per);
    uint32_t sk = 0, ss = 0;
    for (int b = b0; b < b1; ++b) {
        sk += blk[2 * b];
        ss += blk[2 * b + 1];
    }
    s_part[0][t] = sk;
    s_part[1][t] = ss;
    __syncthreads();
    // Hillis-Steele inclusive scan over the thread partials
    for (int o = 1; o < DN_SCAN_THREADS; o <<= 1) {
        const uint32_t ak = t >= o ? s_part[0][t - o] : 0u, as = t >= o ? s_part[1][t - o] : 0u;
        __syncthreads();
        s_part[0][t] += ak;
        s_part[1][t] += as;
        __syncthreads();
    }
    uint32_t rk = s_part[0][t] - sk, rs = s_part[1][t] - ss;
    for (int b = b0; b < b1; ++b) {
        const uint32_t ck = blk[2 * b], cs = blk[2 * b + 1];
        blk[2 * b] = rk;
        blk[2 * b + 1] = rs;
        rk += ck;
        rs += cs;
    }
    if (t == DN_SCAN_THREADS - 1) {
        tot[0] = s_part[0][t];
        tot[1] = s_part[1][t];
    }
}

// for j in [threadIdx.x, total) in steps of DN_BLOCK: store(j, load(j)), with
// U loads of a thread issued before their stores (a plain copy loop waits for
// each load in turn: the stores might alias the next loads).
template <int U, typename L, typename S> __device__ __forceinline__ void batched_for(int total, L load, S store)
{
    for (int j0 = threadIdx.x; j0 < total; j0 += U * DN_BLOCK) {
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = load(min(j0 + u * DN_BLOCK, total - 1)); // unconditional loads
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = j0 + u * DN_BLOCK;
            if (j < total) store(j, v[u]);
        }
    }
}

// The block's kept convexes go to one contiguous run of output rows and its
// children to another, so the rows are copied cooperatively (consecutive
// threads, consecutive floats) from LDS lists of the block's kept and split
// convexes.
__global__ __launch_bounds__(DN_BLOCK) void densify_scatter_kernel(
    int n, int K, int nsh, const float *__restrict__ points, const float *__restrict__ delta,
    const float *__restrict__ sigma, const float *__restrict__ opacity, const float *__restrict__ sh,
    const uint8_t *__restrict__ code, const uint32_t *__restrict__ blk, const uint32_t *__restrict__ tot,
    cs_densify_params dp, cs_scene_out out)
{
    __shared__ uint32_t s_wk[DN_BLOCK / 64], s_ws[DN_BLOCK / 64];
    __shared__ uint32_t s_keep[DN_BLOCK], s_split[DN_BLOCK]; // input index by block-local rank
    __shared__ float s_c[3 * DN_BLOCK];                       // point mean of each split convex
    const int i = blockIdx.x * DN_BLOCK + threadIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint8_t c = i < n ? code[i] : DN_PRUNE;
    const uint64_t mk = __ballot(c == DN_KEEP), ms = __ballot(c == DN_SPLIT);
    if (lane == 0) {
        s_wk[w] = (uint32_t)__popcll(mk);
        s_ws[w] = (uint32_t)__popcll(ms);
    }
    __syncthreads();
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t lk = (uint32_t)__popcll(mk & below), ls = (uint32_t)__popcll(ms & below);
    uint32_t nk = 0, ns = 0;
    for (int v = 0; v < DN_BLOCK / 64; ++v) {
        if (v < w) {
            lk += s_wk[v];
            ls += s_ws[v];
        }
        nk += s_wk[v];
        ns += s_ws[v];
    }
    const int PK = 3 * K;
    if (c == DN_KEEP) s_keep[lk] = (uint32_t)i;
    if (c == DN_SPLIT) {
        s_split[ls] = (uint32_t)i;
        float cx, cy, cz, r2;
        centre_radius(points + (size_t)i * PK, K, cx, cy, cz, r2);
        s_c[3 * ls] = cx;
        s_c[3 * ls + 1] = cy;
        s_c[3 * ls + 2] = cz;
    }
    __syncthreads();
    const size_t kbase = blk[2 * blockIdx.x], sbase = (size_t)tot[0] + (size_t)K * blk[2 * blockIdx.x + 1];
    // kept rows
    batched_for<8>((int)nk * PK, [&](int j) {
        const int r = j / PK, e = j - r * PK;
        return points[(size_t)s_keep[r] * PK + e];
    }, [&](int j, float x) {
        const int r = j / PK, e = j - r * PK;
        out.points[(kbase + r) * PK + e] = x;
    });
    batched_for<8>((int)nk * nsh, [&](int j) {
        const int r = j / nsh, e = j - r * nsh;
        return sh[(size_t)s_keep[r] * nsh + e];
    }, [&](int j, float x) {
        const int r = j / nsh, e = j - r * nsh;
        out.sh[(kbase + r) * nsh + e] = x;
    });
    for (int r = threadIdx.x; r < (int)nk; r += DN_BLOCK) {
        const uint32_t src = s_keep[r];
        out.delta[kbase + r] = delta[src];
        out.sigma[kbase + r] = sigma[src];
        out.opacity[kbase + r] = opacity[src];
        out.src[kbase + r] = (int32_t)src;
    }
    // children: row q = t K + k is child k of the block's t-th split convex,
    // the convex scaled by child_scale about its point k
    const float s = dp.child_scale;
    batched_for<8>((int)ns * K * PK, [&](int j) {
        const int q = j / PK, e = j - q * PK;
        const int t = q / K, k = q - t * K, d = e % 3;
        const float *p = points + (size_t)s_split[t] * PK;
        return p[3 * k + d] + s * (p[e] - s_c[3 * t + d]);
    }, [&](int j, float x) { out.points[sbase * PK + j] = x; });
    batched_for<8>((int)ns * K * nsh, [&](int j) {
        const int q = j / nsh, e = j - q * nsh;
        return sh[(size_t)s_split[q / K] * nsh + e];
    }, [&](int j, float x) { out.sh[sbase * nsh + j] = x; });
    for (int q = threadIdx.x; q < (int)ns * K; q += DN_BLOCK) {
        const uint32_t src = s_split[q / K];
        out.delta[sbase + q] = delta[src];
        out.sigma[sbase + q] = sigma[src] * dp.child_sigma_scale;
        out.opacity[sbase + q] = opacity[src] * dp.child_opacity_scale;
        out.src[sbase + q] = (int32_t)src;
    }
}

// accum[i] += |g[i]| and denom[i] += views where instance v n + i reached a tile
__global__ __launch_bounds__(DN_BLOCK) void densify_accumulate_kernel(int n, int nviews, const uint4 *__restrict__ bins,
                                                                     const float *__restrict__ g,
                                                                     float *__restrict__ accum,
                                                                     float *__restrict__ denom)
{
    const int i = blockIdx.x * DN_BLOCK + threadIdx.x;
    if (i >= n) return;
    int seen = 0;
    for (int v = 0; v < nviews; ++v) seen += bin_count(bins[(size_t)v * n + i]) > 0u;
    if (seen) {
        accum[i] += fabsf(g[i]);
        denom[i] += (float)seen;
    }
}

} // namespace

} // namespace cs

using namespace cs;

extern "C" {

int cs_densify_accumulate(cs_ctx *ctx, const cs_fwd_state *state, const float *g_sigma, float *accum, float *denom,
                          void *hip_stream)
{
    if (!ctx) return fail(CS_EINVAL, "ctx is NULL");
    if (!state || !state->frame) return fail(CS_EINVAL, "state is NULL");
    const Frame &F = *state->frame;
    if (F.n > 0 && (!g_sigma || !accum || !denom)) return fail(CS_EINVAL, "array pointer is NULL");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(CS_EHIP, "hipSetDevice failed");
    if (F.n <= 0) return CS_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(densify_accumulate_kernel, dim3((F.n + DN_BLOCK - 1) / DN_BLOCK), dim3(DN_BLOCK), 0, st, F.n,
                       F.V, F.bins, g_sigma, accum, denom);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? CS_OK : fail(CS_EHIP, "densify accumulate launch: %s", hipGetErrorString(e));
}

int cs_densify(cs_ctx *ctx, const cs_scene *sc, const float *accum, const float *denom,
               const cs_densify_params *dp, int64_t capacity, const cs_scene_out *out, int64_t *n_out,
               void *hip_stream)
{
    if (!ctx) return fail(CS_EINVAL, "ctx is NULL");
    int r = check_scene(sc);
    if (r) return r;
    if (sc->dtype != CS_DTYPE_F32) return fail(CS_EINVAL, "cs_densify takes a float32 scene");
    if (!dp || !out || !n_out) return fail(CS_EINVAL, "params, out or n_out is NULL");
    if (sc->n > 0 && (!accum || !denom)) return fail(CS_EINVAL, "accum or denom is NULL");
    if (capacity < 0) return fail(CS_EINVAL, "capacity < 0");
    if ((int64_t)sc->n * sc->k > (1ll << 28)) return fail(CS_EINVAL, "scene too large to split");
    *n_out = 0;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(CS_EHIP, "hipSetDevice failed");
    const int n = sc->n, K = sc->k, nsh = 3 * (sc->sh_degree + 1) * (sc->sh_degree + 1);
    if (n == 0) return CS_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    const int nb = (n + DN_BLOCK - 1) / DN_BLOCK;
    // scratch: codes [n] u8, block counts [2 nb] u32, totals [2] u32
    const size_t code_bytes = ((size_t)n + 255) & ~(size_t)255;
    void *scratch = nullptr;
    hipError_t e = hipMallocAsync(&scratch, code_bytes + (2 * (size_t)nb + 2) * 4, st);
    if (e != hipSuccess) return fail(CS_ENOMEM, "densify scratch: %s", hipGetErrorString(e));
    uint8_t *code = reinterpret_cast<uint8_t *>(scratch);
    uint32_t *blk = reinterpret_cast<uint32_t *>(code + code_bytes), *tot = blk + 2 * (size_t)nb;
    const float *points = static_cast<const float *>(sc->points);
    hipLaunchKernelGGL(densify_classify_kernel, dim3(nb), dim3(DN_BLOCK), 0, st, n, K, points,
                       static_cast<const float *>(sc->opacity), accum, denom, *dp, code, blk);
    hipLaunchKernelGGL(densify_scan_kernel, dim3(1), dim3(DN_SCAN_THREADS), 0, st, nb, blk, tot);
    uint32_t *hw = ctx->ring.h_word + 8;
    e = hipMemcpyAsync(hw, tot, 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipFreeAsync(scratch, st);
        return fail(CS_EHIP, "densify count read-back: %s", hipGetErrorString(e));
    }
    const int64_t total = (int64_t)hw[0] + (int64_t)K * hw[1];
    *n_out = total;
    if (total > capacity) {
        (void)hipFreeAsync(scratch, st);
        return fail(CS_EOVERFLOW, "densify: %lld convexes do not fit capacity %lld", (long long)total,
                    (long long)capacity);
    }
    if (total > 0 && (!out->points || !out->delta || !out->sigma || !out->opacity || !out->sh || !out->src)) {
        (void)hipFreeAsync(scratch, st);
        return fail(CS_EINVAL, "output array pointer is NULL");
    }
    hipLaunchKernelGGL(densify_scatter_kernel, dim3(nb), dim3(DN_BLOCK), 0, st, n, K, nsh, points,
                       static_cast<const float *>(sc->delta), static_cast<const float *>(sc->sigma),
                       static_cast<const float *>(sc->opacity), static_cast<const float *>(sc->sh), code, blk, tot,
                       *dp, *out);
    e = hipGetLastError();
    (void)hipFreeAsync(scratch, st);
    return e == hipSuccess ? CS_OK : fail(CS_EHIP, "densify launch: %s", hipGetErrorString(e));
}

} // extern "C"
