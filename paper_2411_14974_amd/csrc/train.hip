// Training-step kernels around the rasterizer (gfx950), paper Sec. 3.3
// "Initialization and losses":
//
// * the photometric loss L = (1 - lambda) L1 + lambda (1 - SSIM) and its
//   gradient with respect to the rendered image, in two tiled passes: the
//   first blurs x, y, x^2, y^2 and xy with the 11x11 Gaussian window
//   (separably, through LDS, zero padding), forms the SSIM map and its
//   partial derivatives with respect to the blurred moments; the second blurs
//   those partials (the window is symmetric: the same blur is its adjoint)
//   and combines them with x and y into dL/dx;
// * the fused Adam step on the raw parameters with their activations
//   (sigmoid opacity, exponential delta and sigma): one launch per parameter
//   array, one element per thread and iteration, read raw, m, v and
//   dL/d(activated) (16 B), write raw, m, v and the new activated value (16 B).
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "convexsplat.h"
#include "runtime.hpp"

namespace cs {

namespace {

// ------------------------------------------------------- L1 + D-SSIM ----

constexpr int SS_TILE = 16;                 // output pixels per side of a workgroup
constexpr int SS_R = 5;                     // window radius (11 taps)
constexpr int SS_IN = SS_TILE + 2 * SS_R;   // input rows / columns with the halo
constexpr float SS_C1 = 0.01f * 0.01f;      // SSIM constants for values in [0, 1]
constexpr float SS_C2 = 0.03f * 0.03f;

struct SsimArgs {
    int W, H;
    float lambda;
    float inv_n;      // 1 / (3 W H): the means run over pixels and channels
    float g[2 * SS_R + 1]; // normalised Gaussian window, sigma 1.5
};

// Pass 1: per pixel and channel the SSIM value S and its partial derivatives
// with respect to the blurred moments mu_x, E[x^2] and E[xy] (mu_y and E[y^2]
// do not depend on the rendered image); the loss terms are summed into *loss.
__global__ __launch_bounds__(SS_TILE * SS_TILE) void ssim_moments_kernel(const float *__restrict__ x,
                                                                         const float *__restrict__ y, SsimArgs a,
                                                                         float *__restrict__ part,
                                                                         float *__restrict__ block_loss)
{
    constexpr int NM = 15; // per channel: x, y, x^2, y^2, xy
    __shared__ float s_in[SS_IN * SS_IN * 6];
    __shared__ float s_h[SS_IN * SS_TILE * NM];
    const int tx0 = blockIdx.x * SS_TILE - SS_R, ty0 = blockIdx.y * SS_TILE - SS_R;
    {
        // the halo tile: every load of a thread issued before its LDS stores
        constexpr int NIN = SS_IN * SS_IN, PER = (NIN + SS_TILE * SS_TILE - 1) / (SS_TILE * SS_TILE);
        float xv[PER][3], yv[PER][3];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int j = threadIdx.x + k * SS_TILE * SS_TILE;
            const int r = j / SS_IN, c = j - r * SS_IN, u = tx0 + c, v = ty0 + r;
            const bool in = j < NIN && u >= 0 && u < a.W && v >= 0 && v < a.H;
            const size_t p = in ? 3 * ((size_t)v * a.W + u) : 0; // unconditional loads, zeroed after
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const float xl = x[p + ch], yl = y[p + ch];
                xv[k][ch] = in ? xl : 0.0f;
                yv[k][ch] = in ? yl : 0.0f;
            }
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int j = threadIdx.x + k * SS_TILE * SS_TILE;
            if (j < NIN)
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    s_in[j * 6 + ch] = xv[k][ch];
                    s_in[j * 6 + 3 + ch] = yv[k][ch];
                }
        }
    }
    __syncthreads();
    // horizontal pass: rows of the halo, the tile's columns
    for (int j = threadIdx.x; j < SS_IN * SS_TILE; j += SS_TILE * SS_TILE) {
        const int r = j / SS_TILE, c = j - r * SS_TILE;
        float acc[NM];
#pragma unroll
        for (int q = 0; q < NM; ++q) acc[q] = 0.0f;
#pragma unroll
        for (int t = 0; t <= 2 * SS_R; ++t) {
            const float *e = &s_in[(r * SS_IN + c + t) * 6];
            const float w = a.g[t];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const float xv = e[ch], yv = e[3 + ch];
                acc[5 * ch] = fmaf(w, xv, acc[5 * ch]);
                acc[5 * ch + 1] = fmaf(w, yv, acc[5 * ch + 1]);
                acc[5 * ch + 2] = fmaf(w, xv * xv, acc[5 * ch + 2]);
                acc[5 * ch + 3] = fmaf(w, yv * yv, acc[5 * ch + 3]);
                acc[5 * ch + 4] = fmaf(w, xv * yv, acc[5 * ch + 4]);
            }
        }
#pragma unroll
        for (int q = 0; q < NM; ++q) s_h[j * NM + q] = acc[q];
    }
    __syncthreads();
    const int cx = threadIdx.x % SS_TILE, cy = threadIdx.x / SS_TILE;
    const int u = blockIdx.x * SS_TILE + cx, v = blockIdx.y * SS_TILE + cy;
    float contrib = 0.0f;
    if (u < a.W && v < a.H) {
        float m[NM];
#pragma unroll
        for (int q = 0; q < NM; ++q) m[q] = 0.0f;
#pragma unroll
        for (int t = 0; t <= 2 * SS_R; ++t) {
            const float *e = &s_h[((cy + t) * SS_TILE + cx) * NM];
            const float w = a.g[t];
#pragma unroll
            for (int q = 0; q < NM; ++q) m[q] = fmaf(w, e[q], m[q]);
        }
        const size_t p = 3 * ((size_t)v * a.W + u);
        const float *xin = &s_in[((cy + SS_R) * SS_IN + cx + SS_R) * 6];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float mx = m[5 * ch], my = m[5 * ch + 1];
            const float sxx = m[5 * ch + 2] - mx * mx, syy = m[5 * ch + 3] - my * my, sxy = m[5 * ch + 4] - mx * my;
            const float A1 = 2.0f * mx * my + SS_C1, A2 = 2.0f * sxy + SS_C2;
            const float B1 = mx * mx + my * my + SS_C1, B2 = sxx + syy + SS_C2;
            const float S = (A1 * A2) / (B1 * B2);
            // dS/dmu_x, dS/dE[x^2], dS/dE[xy]
            part[3 * p + 3 * ch] = S * (2.0f * my / A1 - 2.0f * my / A2 - 2.0f * mx / B1 + 2.0f * mx / B2);
            part[3 * p + 3 * ch + 1] = -S / B2;
            part[3 * p + 3 * ch + 2] = 2.0f * S / A2;
            contrib += (1.0f - a.lambda) * fabsf(xin[ch] - xin[3 + ch]) - a.lambda * S;
        }
    }
    // the block's loss terms into its own slot (same-address atomics from
    // every block would serialise); a last pass adds the slots
    __shared__ float s_w[SS_TILE * SS_TILE / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) contrib += __shfl_xor(contrib, o, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = contrib;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int w = 0; w < SS_TILE * SS_TILE / 64; ++w) t += s_w[w];
        block_loss[blockIdx.y * gridDim.x + blockIdx.x] = t;
    }
}

// loss += lambda + inv_n * (sum of the blocks' terms): one workgroup.
__global__ __launch_bounds__(1024) void ssim_loss_sum_kernel(const float *__restrict__ block_loss, int nb, SsimArgs a,
                                                             float *__restrict__ loss)
{
    __shared__ float s_w[16];
    float t = 0.0f;
    for (int b = threadIdx.x; b < nb; b += 1024) t += block_loss[b];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        float u = 0.0f;
        for (int w = 0; w < 16; ++w) u += s_w[w];
        *loss += a.lambda + u * a.inv_n;
    }
}

// Pass 2: dL/dx = (1 - lambda) sign(x - y) / n - lambda / n (G*d_mu + 2 x G*d_xx + y G*d_xy).
__global__ __launch_bounds__(SS_TILE * SS_TILE) void ssim_grad_kernel(const float *__restrict__ x,
                                                                      const float *__restrict__ y, SsimArgs a,
                                                                      const float *__restrict__ part,
                                                                      float *__restrict__ grad)
{
    constexpr int NP = 9;
    __shared__ float s_in[SS_IN * SS_IN * NP];
    __shared__ float s_h[SS_IN * SS_TILE * NP];
    const int tx0 = blockIdx.x * SS_TILE - SS_R, ty0 = blockIdx.y * SS_TILE - SS_R;
    {
        // the halo tile of the partials: every load of a thread issued before its LDS stores
        constexpr int NE = SS_IN * SS_IN * NP, PER = (NE + SS_TILE * SS_TILE - 1) / (SS_TILE * SS_TILE);
        float pv[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int j = threadIdx.x + k * SS_TILE * SS_TILE;
            const int pix = j / NP, q = j - pix * NP;
            const int r = pix / SS_IN, c = pix - r * SS_IN, u = tx0 + c, v = ty0 + r;
            const bool in = j < NE && u >= 0 && u < a.W && v >= 0 && v < a.H;
            const float l = part[in ? NP * ((size_t)v * a.W + u) + q : 0]; // unconditional load, zeroed after
            pv[k] = in ? l : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int j = threadIdx.x + k * SS_TILE * SS_TILE;
            if (j < NE) s_in[j] = pv[k];
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < SS_IN * SS_TILE; j += SS_TILE * SS_TILE) {
        const int r = j / SS_TILE, c = j - r * SS_TILE;
        float acc[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) acc[q] = 0.0f;
#pragma unroll
        for (int t = 0; t <= 2 * SS_R; ++t) {
            const float *e = &s_in[(r * SS_IN + c + t) * NP];
            const float w = a.g[t];
#pragma unroll
            for (int q = 0; q < NP; ++q) acc[q] = fmaf(w, e[q], acc[q]);
        }
#pragma unroll
        for (int q = 0; q < NP; ++q) s_h[j * NP + q] = acc[q];
    }
    __syncthreads();
    const int cx = threadIdx.x % SS_TILE, cy = threadIdx.x / SS_TILE;
    const int u = blockIdx.x * SS_TILE + cx, v = blockIdx.y * SS_TILE + cy;
    if (u >= a.W || v >= a.H) return;
    float b[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) b[q] = 0.0f;
#pragma unroll
    for (int t = 0; t <= 2 * SS_R; ++t) {
        const float *e = &s_h[((cy + t) * SS_TILE + cx) * NP];
        const float w = a.g[t];
#pragma unroll
        for (int q = 0; q < NP; ++q) b[q] = fmaf(w, e[q], b[q]);
    }
    const size_t p = 3 * ((size_t)v * a.W + u);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const float xv = x[p + ch], yv = y[p + ch], d = xv - yv;
        const float sg = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
        const float ds = b[3 * ch] + 2.0f * xv * b[3 * ch + 1] + yv * b[3 * ch + 2];
        grad[p + ch] = a.inv_n * ((1.0f - a.lambda) * sg - a.lambda * ds);
    }
}

enum : int { ACT_ID = 0, ACT_EXP = 1, ACT_SIGMOID = 2 };

template <int ACT> __device__ __forceinline__ float activate(float r)
{
    if constexpr (ACT == ACT_EXP) return expf(r);
    else if constexpr (ACT == ACT_SIGMOID) return 1.0f / (1.0f + expf(-r));
    else return r;
}

struct AdamArgs {
    float beta1, beta2, omb1, omb2, eps; // betas and 1 - betas (formed in double)
    float step_size;  // lr / (1 - beta1^t) of the first rate
    float step_size2; // the same for the second rate (SH coefficients past the first)
    float bc2_sqrt;   // sqrt(1 - beta2^t)
};

// Elements e with row > 0 and e % row >= first take the second rate.
// One parameter element: the activation's derivative at the current raw
// value, the moment updates and the step on the raw value.
template <int ACT>
__device__ __forceinline__ void adam_element(size_t e, size_t n, float r, float gact, float m0, float v0, int row,
                                             int first, const AdamArgs &a, float &rn, float &mm, float &vv)
{
    float da = 1.0f; // d activated / d raw at the current raw value
    if constexpr (ACT == ACT_EXP) da = expf(r);
    else if constexpr (ACT == ACT_SIGMOID) {
        const float s = 1.0f / (1.0f + expf(-r));
        da = s * (1.0f - s);
    }
    const float g = gact * da;
    mm = m0 + a.omb1 * (g - m0);
    vv = a.beta2 * v0 + a.omb2 * (g * g);
    const float denom = sqrtf(vv) / a.bc2_sqrt + a.eps;
    // position in the row (32-bit arithmetic when the index fits: a 64-bit
    // remainder is a long software sequence)
    const uint32_t col = row <= 0 ? 0u : (n >> 32) == 0 ? (uint32_t)e % (uint32_t)row : (uint32_t)(e % (size_t)row);
    const float ss = (row > 0 && (int)col >= first) ? a.step_size2 : a.step_size;
    rn = r - ss * (mm / denom);
}

template <int ACT>
__global__ __launch_bounds__(256) void adam_kernel(size_t n, const float *__restrict__ g_act, float *__restrict__ raw,
                                                   float *__restrict__ m, float *__restrict__ v,
                                                   float *__restrict__ act_out, int row, int first, AdamArgs a)
{
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        float rn, mm, vv;
        adam_element<ACT>(e, n, raw[e], g_act[e], m[e], v[e], row, first, a, rn, mm, vv);
        raw[e] = rn;
        m[e] = mm;
        v[e] = vv;
        if (act_out) act_out[e] = activate<ACT>(rn);
    }
}

// The same update, four elements per thread in 16-byte accesses (every array
// 16-byte aligned and n a multiple of 4); the arithmetic per element is the
// scalar kernel's, so the results are identical.
template <int ACT>
__global__ __launch_bounds__(256) void adam4_kernel(size_t n, const float4 *__restrict__ g_act, float4 *__restrict__ raw,
                                                    float4 *__restrict__ m, float4 *__restrict__ v,
                                                    float4 *__restrict__ act_out, int row, int first, AdamArgs a)
{
    const size_t n4 = n / 4;
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n4; q += (size_t)gridDim.x * blockDim.x) {
        const float4 r4 = raw[q], g4 = g_act[q], m4 = m[q], v4 = v[q];
        const float rr[4] = {r4.x, r4.y, r4.z, r4.w}, gg[4] = {g4.x, g4.y, g4.z, g4.w};
        const float mi[4] = {m4.x, m4.y, m4.z, m4.w}, vi[4] = {v4.x, v4.y, v4.z, v4.w};
        float rn[4], mm[4], vv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) adam_element<ACT>(4 * q + j, n, rr[j], gg[j], mi[j], vi[j], row, first, a, rn[j], mm[j], vv[j]);
        raw[q] = make_float4(rn[0], rn[1], rn[2], rn[3]);
        m[q] = make_float4(mm[0], mm[1], mm[2], mm[3]);
        v[q] = make_float4(vv[0], vv[1], vv[2], vv[3]);
        if (act_out)
            act_out[q] = make_float4(activate<ACT>(rn[0]), activate<ACT>(rn[1]), activate<ACT>(rn[2]),
                                     activate<ACT>(rn[3]));
    }
}

template <int ACT>
void launch_adam(hipStream_t st, size_t n, const float *g, float *raw, float *m, float *v, float *act, int row,
                 int first, const AdamArgs &a)
{
    if (n == 0) return;
    auto al = [](const void *p) { return ((uintptr_t)p & 15u) == 0; };
    if (n % 4 == 0 && al(g) && al(raw) && al(m) && al(v) && (!act || al(act))) {
        const size_t blocks = std::min<size_t>((n / 4 + 255) / 256, 8192);
        hipLaunchKernelGGL(adam4_kernel<ACT>, dim3((unsigned)blocks), dim3(256), 0, st, n, (const float4 *)g,
                           (float4 *)raw, (float4 *)m, (float4 *)v, (float4 *)act, row, first, a);
        return;
    }
    const size_t blocks = std::min<size_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(adam_kernel<ACT>, dim3((unsigned)blocks), dim3(256), 0, st, n, g, raw, m, v, act, row, first,
                       a);
}

bool set_complete(const cs_param_set *p)
{
    return p && p->points && p->delta && p->sigma && p->opacity && p->sh;
}

} // namespace

} // namespace cs

using namespace cs;

extern "C" {

int cs_adam_step(cs_ctx *ctx, int32_t n, int32_t k, int32_t sh_degree, const cs_grads *grad, const cs_param_set *raw,
                 const cs_param_set *m, const cs_param_set *v, const cs_param_set *activated,
                 const cs_adam_params *prm, void *hip_stream)
{
    if (!ctx) return fail(CS_EINVAL, "ctx is NULL");
    if (n < 0 || k < 3 || k > CS_MAX_K || sh_degree < 0 || sh_degree > CS_MAX_SH_DEGREE)
        return fail(CS_EINVAL, "bad n, k or sh_degree");
    if (!prm) return fail(CS_EINVAL, "params is NULL");
    if (prm->step < 1) return fail(CS_EINVAL, "adam step %d < 1", prm->step);
    if (!(prm->beta1 >= 0.0 && prm->beta1 < 1.0 && prm->beta2 >= 0.0 && prm->beta2 < 1.0))
        return fail(CS_EINVAL, "betas outside [0, 1)");
    if (n == 0) return CS_OK;
    if (!grad || !grad->points || !grad->delta || !grad->sigma || !grad->opacity || !grad->sh || !set_complete(raw) ||
        !set_complete(m) || !set_complete(v) || (activated && !set_complete(activated)))
        return fail(CS_EINVAL, "array pointer is NULL");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(CS_EHIP, "hipSetDevice failed");
    hipStream_t st = (hipStream_t)hip_stream;
    const double bc1 = 1.0 - std::pow(prm->beta1, (double)prm->step);
    const double bc2 = 1.0 - std::pow(prm->beta2, (double)prm->step);
    auto args = [&](float lr, float lr2) {
        AdamArgs a;
        a.beta1 = (float)prm->beta1;
        a.beta2 = (float)prm->beta2;
        a.omb1 = (float)(1.0 - prm->beta1);
        a.omb2 = (float)(1.0 - prm->beta2);
        a.eps = prm->eps;
        a.step_size = (float)(lr / bc1);
        a.step_size2 = (float)(lr2 / bc1);
        a.bc2_sqrt = (float)std::sqrt(bc2);
        return a;
    };
    const size_t N = (size_t)n;
    const int nsh = 3 * (sh_degree + 1) * (sh_degree + 1);
    auto act = [&](float *cs_param_set::*f) { return activated ? activated->*f : nullptr; };
    launch_adam<ACT_ID>(st, N * 3 * k, grad->points, raw->points, m->points, v->points, act(&cs_param_set::points), 0,
                        0, args(prm->lr_points, prm->lr_points));
    launch_adam<ACT_EXP>(st, N, grad->delta, raw->delta, m->delta, v->delta, act(&cs_param_set::delta), 0, 0,
                         args(prm->lr_delta, prm->lr_delta));
    launch_adam<ACT_EXP>(st, N, grad->sigma, raw->sigma, m->sigma, v->sigma, act(&cs_param_set::sigma), 0, 0,
                         args(prm->lr_sigma, prm->lr_sigma));
    launch_adam<ACT_SIGMOID>(st, N, grad->opacity, raw->opacity, m->opacity, v->opacity,
                             act(&cs_param_set::opacity), 0, 0, args(prm->lr_opacity, prm->lr_opacity));
    launch_adam<ACT_ID>(st, N * nsh, grad->sh, raw->sh, m->sh, v->sh, act(&cs_param_set::sh), nsh, 3,
                        args(prm->lr_sh_dc, prm->lr_sh_rest));
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? CS_OK : fail(CS_EHIP, "adam launch: %s", hipGetErrorString(e));
}

int cs_ssim_loss_grad(cs_ctx *ctx, const float *rgb, const float *target, int32_t width, int32_t height, float lambda,
                      float *dl_drgb, float *loss, void *hip_stream)
{
    if (!ctx || !rgb || !target || !dl_drgb || !loss) return fail(CS_EINVAL, "NULL argument");
    if (width <= 0 || height <= 0 || width > 16384 || height > 16384) return fail(CS_EINVAL, "bad image size");
    if (!(lambda >= 0.0f && lambda <= 1.0f)) return fail(CS_EINVAL, "lambda outside [0, 1]");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(CS_EHIP, "hipSetDevice failed");
    hipStream_t st = (hipStream_t)hip_stream;
    SsimArgs a;
    a.W = width;
    a.H = height;
    a.lambda = lambda;
    a.inv_n = (float)(1.0 / (3.0 * (double)width * (double)height));
    double gs[2 * SS_R + 1], tot = 0.0;
    for (int t = -SS_R; t <= SS_R; ++t) tot += gs[t + SS_R] = std::exp(-(double)(t * t) / (2.0 * 1.5 * 1.5));
    for (int t = 0; t <= 2 * SS_R; ++t) a.g[t] = (float)(gs[t] / tot);
    const dim3 grid((width + SS_TILE - 1) / SS_TILE, (height + SS_TILE - 1) / SS_TILE), block(SS_TILE * SS_TILE);
    const int nb = (int)(grid.x * grid.y);
    float *part = nullptr;
    const size_t part_floats = (size_t)width * height * 9;
    hipError_t e = hipMallocAsync((void **)&part, (part_floats + nb) * sizeof(float), st);
    if (e != hipSuccess) return fail(CS_ENOMEM, "ssim scratch: %s", hipGetErrorString(e));
    float *block_loss = part + part_floats;
    hipLaunchKernelGGL(ssim_moments_kernel, grid, block, 0, st, rgb, target, a, part, block_loss);
    hipLaunchKernelGGL(ssim_loss_sum_kernel, dim3(1), dim3(1024), 0, st, block_loss, nb, a, loss);
    hipLaunchKernelGGL(ssim_grad_kernel, grid, block, 0, st, rgb, target, a, part, dl_drgb);
    e = hipGetLastError();
    (void)hipFreeAsync(part, st);
    return e == hipSuccess ? CS_OK : fail(CS_EHIP, "ssim launch: %s", hipGetErrorString(e));
}

} // extern "C"
