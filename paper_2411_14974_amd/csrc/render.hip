// Per-tile compositing, forward and backward (gfx950).
//
// One 256-thread workgroup per 16x16 tile, one pixel per thread.  The tile's
// depth-ordered convex list is streamed through LDS in batches of records;
// every thread walks the batch front to back and evaluates, for its pixel,
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
// decisions), recovering T_n = T_{n+1} / (1 - alpha_n), and reduces the per-pair
// gradients over the wavefront before one atomic add per convex value.
#include <algorithm>
#include <utility>

#include "common.hpp"

namespace cs {

namespace {

constexpr int TILE = 16;
constexpr int BLOCK = 256;

template <int K> struct PairEval {
    float I, omI, alpha, oma, phi2, inv_sum;
    float e[K];  // 2^(x2_j - max)
    float x2[K]; // x2_j rounded to float
};

// The one evaluation of a (pixel, convex) pair shared by both passes.
// Returns false when the pair is skipped (alpha < eps_alpha).
template <int K>
__device__ __forceinline__ bool eval_pair(const uint8_t *rec, float pxf, float pyf, float eps, PairEval<K> &pe)
{
    const RecHeader &h = *reinterpret_cast<const RecHeader *>(rec);
    const double *ln = reinterpret_cast<const double *>(rec + 64);
    const int T = h.T;
    pe.inv_sum = 0.0f;
    const double dx = (double)(pxf - h.ox), dy = (double)(pyf - h.oy);
    double x[K];
    double m = -INFINITY;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j < T) {
            x[j] = fma(ln[3 * j], dx, fma(ln[3 * j + 1], dy, ln[3 * j + 2]));
            m = fmax(m, x[j]);
        } else {
            x[j] = -INFINITY;
        }
    }
    // LogSumExp >= its largest term: past thr2 alpha < eps for certain
    if (!(m <= (double)h.thr2)) return false;
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const float e = (j < T) ? __builtin_amdgcn_exp2f((float)(x[j] - m)) : 0.0f;
        pe.e[j] = e;
        pe.x2[j] = (j < T) ? (float)x[j] : 0.0f;
        s += e;
    }
    pe.inv_sum = __builtin_amdgcn_rcpf(s);
    const float phi2 = (float)m + __builtin_amdgcn_logf(s);
    const float z = h.sigma_p * phi2; // I = 1 / (1 + 2^z)
    const float ez = __builtin_amdgcn_exp2f(-fabsf(z));
    const float r = __builtin_amdgcn_rcpf(1.0f + ez);
    pe.I = z > 0.0f ? ez * r : r;
    pe.omI = z > 0.0f ? r : ez * r;
    pe.alpha = h.opacity * pe.I;
    if (pe.alpha < eps) return false;
    pe.oma = (1.0f - h.opacity) + h.opacity * pe.omI;
    pe.phi2 = phi2;
    return true;
}

// Tiles are dealt to workgroups so that each of the 8 XCDs (which receive
// workgroups round-robin) owns a contiguous band of tiles: neighbouring tiles
// share convex records, and they then share an L2.
__device__ __forceinline__ int xcd_tile(int ntiles)
{
    const int per_xcd = (ntiles + 7) / 8;
    return (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
}

__device__ __forceinline__ float wave_sum(float x)
{
    x += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, true));  // quad_perm 1,0,3,2
    x += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x4E, 0xF, 0xF, true));  // quad_perm 2,3,0,1
    x += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x141, 0xF, 0xF, true)); // row_half_mirror
    x += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x140, 0xF, 0xF, true)); // row_mirror
    const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 0));
    const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 16));
    const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 32));
    const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 48));
    return (a + b) + (c + d);
}

template <int K, int BATCH>
__device__ __forceinline__ void load_batch(uint4 *lds, const uint32_t *__restrict__ ids,
                                           const uint8_t *__restrict__ records, int base, int cnt)
{
    constexpr int CH = rec_stride(K) / 16;
    for (int c = threadIdx.x; c < cnt * CH; c += BLOCK) {
        const int e = c / CH, part = c - e * CH;
        const uint32_t id = ids[base + e];
        lds[c] = reinterpret_cast<const uint4 *>(records + (size_t)id * rec_stride(K))[part];
    }
}

} // namespace

template <int K, int BATCH>
__global__ __launch_bounds__(BLOCK) void render_fwd_kernel(const uint2 *__restrict__ ranges,
                                                          const uint32_t *__restrict__ ids,
                                                          const uint8_t *__restrict__ records, RenderArgs ra, int W,
                                                          int H, float *__restrict__ out_rgb,
                                                          uint2 *__restrict__ pixstate,
                                                          unsigned long long *__restrict__ evalcount)
{
    constexpr int CH = rec_stride(K) / 16;
    __shared__ uint4 lds[BATCH * CH];
    const int ntiles = ra.tiles_x * ra.tiles_y;
    const int tile = xcd_tile(ntiles);
    if (tile >= ntiles) return;
    const int tx = tile % ra.tiles_x, ty = tile / ra.tiles_x;
    const int u = tx * TILE + (threadIdx.x & (TILE - 1)), v = ty * TILE + (threadIdx.x / TILE);
    const bool inside = u < W && v < H;
    const float pxf = (float)u + 0.5f, pyf = (float)v + 0.5f;
    const uint2 rg = ranges[tile];
    const int start = (int)rg.x, end = (int)rg.y;

    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, Tlast = 1.0f;
    int nend = 0;
    uint32_t nevals = 0, nfull = 0; // pairs evaluated / pairs past the max-line test
    bool done = !inside;
    for (int base = start; base < end; base += BATCH) {
        const int cnt = min(BATCH, end - base);
        __syncthreads();
        load_batch<K, BATCH>(lds, ids, records, base, cnt);
        __syncthreads();
        if (!done) {
            for (int e = 0; e < cnt; ++e) {
                const uint8_t *rec = reinterpret_cast<const uint8_t *>(&lds[e * CH]);
                PairEval<K> pe;
                ++nevals;
                const bool hit = eval_pair<K>(rec, pxf, pyf, ra.eps_alpha, pe);
                if (evalcount) nfull += pe.inv_sum > 0.0f;
                if (!hit) continue;
                const RecHeader &h = *reinterpret_cast<const RecHeader *>(rec);
                const float w = T * pe.alpha;
                C0 = fmaf(w, h.rgb[0], C0);
                C1 = fmaf(w, h.rgb[1], C1);
                C2 = fmaf(w, h.rgb[2], C2);
                Tlast = T;
                T = T * pe.oma;
                nend = base - start + e + 1;
                if (T < ra.t_min) { done = true; break; }
            }
        }
        if (__syncthreads_and(done)) break;
    }
    if (inside) {
        const size_t pix = (size_t)v * W + u;
        out_rgb[3 * pix + 0] = fmaf(T, ra.bg[0], C0);
        out_rgb[3 * pix + 1] = fmaf(T, ra.bg[1], C1);
        out_rgb[3 * pix + 2] = fmaf(T, ra.bg[2], C2);
        pixstate[pix] = make_uint2((uint32_t)nend, __float_as_uint(Tlast));
    }
    if (evalcount) {
        unsigned long long c = nevals, f = nfull;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            c += __shfl_xor(c, o, 64);
            f += __shfl_xor(f, o, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(evalcount, c);
            atomicAdd(evalcount + 1, f);
        }
    }
}

template <int K, int BATCH>
__global__ __launch_bounds__(BLOCK) void render_bwd_kernel(const uint2 *__restrict__ ranges,
                                                          const uint32_t *__restrict__ ids,
                                                          const uint8_t *__restrict__ records, RenderArgs ra, int W,
                                                          int H, const float *__restrict__ dl_drgb,
                                                          const uint2 *__restrict__ pixstate, float *__restrict__ acc)
{
    constexpr int CH = rec_stride(K) / 16;
    constexpr int NV = acc_values(K); // a[K] b[K] c[K] sigma' o rgb[3] x2-weighted sum
    constexpr int AS = acc_stride(K);
    static_assert(NV <= 64, "one lane per reduced value");
    __shared__ uint4 lds[BATCH * CH];
    __shared__ uint32_t s_ids[BATCH];
    __shared__ int s_maxn;
    const int ntiles = ra.tiles_x * ra.tiles_y;
    const int tile = xcd_tile(ntiles);
    if (tile >= ntiles) return;
    const int tx = tile % ra.tiles_x, ty = tile / ra.tiles_x;
    const int u = tx * TILE + (threadIdx.x & (TILE - 1)), v = ty * TILE + (threadIdx.x / TILE);
    const bool inside = u < W && v < H;
    const float pxf = (float)u + 0.5f, pyf = (float)v + 0.5f;
    const int lane = threadIdx.x & 63;
    const uint2 rg = ranges[tile];
    const int start = (int)rg.x;

    float g0 = 0.f, g1 = 0.f, g2 = 0.f, Tlast = 1.f;
    int nend = 0;
    if (inside) {
        const size_t pix = (size_t)v * W + u;
        g0 = dl_drgb[3 * pix + 0];
        g1 = dl_drgb[3 * pix + 1];
        g2 = dl_drgb[3 * pix + 2];
        const uint2 ps = pixstate[pix];
        nend = (int)ps.x;
        Tlast = __uint_as_float(ps.y);
    }
    if (threadIdx.x == 0) s_maxn = 0;
    __syncthreads();
    if (nend > 0) atomicMax(&s_maxn, nend);
    __syncthreads();
    const int maxn = s_maxn;

    float B0 = ra.bg[0], B1 = ra.bg[1], B2 = ra.bg[2];
    float Tcur = Tlast;
    bool first = true;
    for (int hi = maxn; hi > 0; hi -= BATCH) {
        const int lo = max(hi - BATCH, 0);
        const int cnt = hi - lo;
        __syncthreads();
        load_batch<K, BATCH>(lds, ids, records, start + lo, cnt);
        for (int c = threadIdx.x; c < cnt; c += BLOCK) s_ids[c] = ids[start + lo + c];
        __syncthreads();
        for (int e = cnt - 1; e >= 0; --e) {
            const int pos = lo + e;
            if (!__any(pos < nend)) continue; // wave-uniform
            const uint8_t *rec = reinterpret_cast<const uint8_t *>(&lds[e * CH]);
            const RecHeader &h = *reinterpret_cast<const RecHeader *>(rec);
            PairEval<K> pe;
            const bool contrib = (pos < nend) && eval_pair<K>(rec, pxf, pyf, ra.eps_alpha, pe);
            if (__ballot(contrib) == 0ull) continue; // wave-uniform
            float val[NV];
#pragma unroll
            for (int q = 0; q < NV; ++q) val[q] = 0.0f;
            if (contrib) {
                const float Tn = first ? Tlast : Tcur / pe.oma;
                first = false;
                Tcur = Tn;
                const float dLda = Tn * (g0 * (h.rgb[0] - B0) + g1 * (h.rgb[1] - B1) + g2 * (h.rgb[2] - B2));
                const float ta = Tn * pe.alpha;
                val[3 * K + 2] = g0 * ta;
                val[3 * K + 3] = g1 * ta;
                val[3 * K + 4] = g2 * ta;
                val[3 * K + 1] = dLda * pe.I;
                const float dLdz = -dLda * h.opacity * pe.I * pe.omI; // I = Sigmoid(-z), z = sigma' phi
                val[3 * K] = dLdz * pe.phi2 * (float)LN2;
                const float dLdphi2 = dLdz * h.sigma_p * (float)LN2;
                const float dxf = pxf - h.ox, dyf = pyf - h.oy;
                float gdl = 0.0f;
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    const float gx = dLdphi2 * pe.e[j] * pe.inv_sum;
                    val[j] = gx * dxf;
                    val[K + j] = gx * dyf;
                    val[2 * K + j] = gx;
                    gdl = fmaf(gx, pe.x2[j], gdl);
                }
                val[3 * K + 5] = gdl;
                B0 = fmaf(pe.alpha, h.rgb[0], pe.oma * B0);
                B1 = fmaf(pe.alpha, h.rgb[1], pe.oma * B1);
                B2 = fmaf(pe.alpha, h.rgb[2], pe.oma * B2);
            }
            const int T = h.T;
            float mine = 0.0f;
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                const int j = q < 3 * K ? q % K : 0;
                if (j < T) { // uniform
                    const float s = wave_sum(val[q]);
                    if (lane == q) mine = s;
                }
            }
            const int jl = lane < 3 * K ? lane % K : 0;
            if (lane < NV && jl < T && mine != 0.0f)
                unsafeAtomicAdd(&acc[(size_t)s_ids[e] * AS + lane], mine);
        }
    }
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

constexpr int FWD_BATCH = 64;
constexpr int BWD_BATCH = 64;

int render_grid(int ntiles) { return ((ntiles + 7) / 8) * 8; }

void launch_render_fwd(hipStream_t st, int K, int ntiles, const uint2 *ranges, const uint32_t *ids,
                       const uint8_t *records, const RenderArgs &ra, int W, int H, float *out_rgb, uint2 *pixstate,
                       unsigned long long *evalcount)
{
    if (ntiles <= 0) return;
    dim3 grid(render_grid(ntiles)), block(BLOCK);
    CS_DISPATCH_K(K, hipLaunchKernelGGL((render_fwd_kernel<KK, FWD_BATCH>), grid, block, 0, st, ranges, ids, records,
                                        ra, W, H, out_rgb, pixstate, evalcount));
}

void launch_render_bwd(hipStream_t st, int K, int ntiles, const uint2 *ranges, const uint32_t *ids,
                       const uint8_t *records, const RenderArgs &ra, int W, int H, const float *dl_drgb,
                       const uint2 *pixstate, float *acc)
{
    if (ntiles <= 0) return;
    dim3 grid(render_grid(ntiles)), block(BLOCK);
    CS_DISPATCH_K(K, hipLaunchKernelGGL((render_bwd_kernel<KK, BWD_BATCH>), grid, block, 0, st, ranges, ids, records,
                                        ra, W, H, dl_drgb, pixstate, acc));
}

// ------------------------------------------------------------ L1 loss ----

__global__ void l1_grad_kernel(const float *__restrict__ rgb, const float *__restrict__ target, size_t n, float scale,
                               float *__restrict__ grad, float *__restrict__ loss)
{
    float part = 0.0f;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float d = rgb[i] - target[i];
        grad[i] = d > 0.0f ? scale : (d < 0.0f ? -scale : 0.0f);
        part += fabsf(d);
    }
    if (loss) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
        if ((threadIdx.x & 63) == 0) atomicAdd(loss, part * scale);
    }
}

void launch_l1_grad(hipStream_t st, const float *rgb, const float *target, size_t n, float *grad, float *loss)
{
    if (n == 0) return;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(l1_grad_kernel, dim3((unsigned)blocks), dim3(256), 0, st, rgb, target, n, 1.0f / (float)n,
                       grad, loss);
}

} // namespace cs
