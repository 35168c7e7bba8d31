// Initial convex set from a point cloud (gfx950), paper Sec. 3.3
// "Initialization and losses" and Supp. Initialization & Hyperparameters: one
// convex per cloud point, its K points spread uniformly over a sphere round
// the cloud point (Fibonacci sphere), the sphere's radius a multiple of the
// mean distance to the point's three nearest neighbours in the cloud.
//
// The three nearest neighbours are found exactly by brute force: a workgroup
// holds 256 query points, candidate points stream through LDS in tiles of 256,
// every thread keeps its three smallest squared distances (O(N^2), one-time:
// about 10^10 pair distances for 10^5 points).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "convexsplat.h"
#include "runtime.hpp"
#include "sh.hpp"

namespace cs {

namespace {

constexpr int KN_BLOCK = 256;

struct InitArgs {
    int n, K, nsh;
    float radius_scale, radius_min;
    float delta0, sigma0, opacity0;
    float dir[3 * CS_MAX_K]; // unit Fibonacci-sphere directions
};

__global__ __launch_bounds__(KN_BLOCK) void knn3_mean_kernel(int n, const float *__restrict__ xyz,
                                                             float *__restrict__ mean_dist)
{
    __shared__ float s_p[3 * KN_BLOCK];
    const int i = blockIdx.x * KN_BLOCK + threadIdx.x;
    const float qx = i < n ? xyz[3 * i] : 0.0f, qy = i < n ? xyz[3 * i + 1] : 0.0f, qz = i < n ? xyz[3 * i + 2] : 0.0f;
    float d0 = INFINITY, d1 = INFINITY, d2 = INFINITY; // ascending
    for (int base = 0; base < n; base += KN_BLOCK) {
        const int cnt = min(KN_BLOCK, n - base);
        __syncthreads();
        for (int j = threadIdx.x; j < 3 * cnt; j += KN_BLOCK) s_p[j] = xyz[3 * (size_t)base + j];
        __syncthreads();
        for (int c = 0; c < cnt; ++c) {
            const float dx = s_p[3 * c] - qx, dy = s_p[3 * c + 1] - qy, dz = s_p[3 * c + 2] - qz;
            const float d = (dx * dx + dy * dy) + dz * dz;
            const bool self = base + c == i;
            if (!self && d < d2) {
                if (d < d1) {
                    d2 = d1;
                    if (d < d0) { d1 = d0; d0 = d; }
                    else d1 = d;
                } else {
                    d2 = d;
                }
            }
        }
    }
    if (i >= n) return;
    // fewer than three other points: the mean of those there are
    float sum = 0.0f;
    int m = 0;
    if (d0 < INFINITY) { sum += sqrtf(d0); ++m; }
    if (d1 < INFINITY) { sum += sqrtf(d1); ++m; }
    if (d2 < INFINITY) { sum += sqrtf(d2); ++m; }
    mean_dist[i] = m ? sum / (float)m : 0.0f;
}

__global__ __launch_bounds__(KN_BLOCK) void init_convex_kernel(const float *__restrict__ xyz,
                                                               const float *__restrict__ rgb,
                                                               const float *__restrict__ mean_dist, InitArgs a,
                                                               cs_param_set out)
{
    const int i = blockIdx.x * KN_BLOCK + threadIdx.x;
    if (i >= a.n) return;
    const float r = a.radius_scale * fmaxf(mean_dist[i], a.radius_min);
    const float cx = xyz[3 * i], cy = xyz[3 * i + 1], cz = xyz[3 * i + 2];
    float *p = out.points + (size_t)i * 3 * a.K;
    for (int k = 0; k < a.K; ++k) {
        p[3 * k] = cx + r * a.dir[3 * k];
        p[3 * k + 1] = cy + r * a.dir[3 * k + 1];
        p[3 * k + 2] = cz + r * a.dir[3 * k + 2];
    }
    out.delta[i] = a.delta0;
    out.sigma[i] = a.sigma0;
    out.opacity[i] = a.opacity0;
    // colour = 0.5 + Y00 f_dc (the renderer's convention): f_dc = (rgb - 0.5) / Y00, higher orders 0
    float *f = out.sh + (size_t)i * a.nsh;
    for (int c = 0; c < 3; ++c) f[c] = rgb ? (rgb[3 * i + c] - 0.5f) / SH_C0 : 0.0f;
    for (int j = 3; j < a.nsh; ++j) f[j] = 0.0f;
}

} // namespace

} // namespace cs

using namespace cs;

extern "C" {

int cs_init_from_points(cs_ctx *ctx, int32_t n, const float *xyz, const float *rgb, int32_t k, int32_t sh_degree,
                        const cs_init_params *prm, const cs_param_set *out, void *hip_stream)
{
    if (!ctx) return fail(CS_EINVAL, "ctx is NULL");
    if (n < 0 || k < 3 || k > CS_MAX_K || sh_degree < 0 || sh_degree > CS_MAX_SH_DEGREE)
        return fail(CS_EINVAL, "bad n, k or sh_degree");
    if (!prm) return fail(CS_EINVAL, "params is NULL");
    if (n == 0) return CS_OK;
    if (!xyz || !out || !out->points || !out->delta || !out->sigma || !out->opacity || !out->sh)
        return fail(CS_EINVAL, "array pointer is NULL");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(CS_EHIP, "hipSetDevice failed");
    hipStream_t st = (hipStream_t)hip_stream;
    InitArgs a;
    a.n = n;
    a.K = k;
    a.nsh = 3 * (sh_degree + 1) * (sh_degree + 1);
    a.radius_scale = prm->radius_scale;
    a.radius_min = prm->radius_min;
    a.delta0 = prm->delta0;
    a.sigma0 = prm->sigma0;
    a.opacity0 = prm->opacity0;
    // Fibonacci sphere: heights 1 - (2j + 1) / K, azimuth steps of the golden angle
    const double golden = M_PI * (3.0 - std::sqrt(5.0));
    for (int j = 0; j < k; ++j) {
        const double yv = 1.0 - (2.0 * j + 1.0) / k, rxy = std::sqrt(1.0 - yv * yv), phi = golden * j;
        a.dir[3 * j] = (float)(std::cos(phi) * rxy);
        a.dir[3 * j + 1] = (float)yv;
        a.dir[3 * j + 2] = (float)(std::sin(phi) * rxy);
    }
    float *md = nullptr;
    hipError_t e = hipMallocAsync((void **)&md, (size_t)n * sizeof(float), st);
    if (e != hipSuccess) return fail(CS_ENOMEM, "init scratch: %s", hipGetErrorString(e));
    const dim3 grid((n + KN_BLOCK - 1) / KN_BLOCK), block(KN_BLOCK);
    hipLaunchKernelGGL(knn3_mean_kernel, grid, block, 0, st, n, xyz, md);
    hipLaunchKernelGGL(init_convex_kernel, grid, block, 0, st, xyz, rgb, md, a, *out);
    e = hipGetLastError();
    (void)hipFreeAsync(md, st);
    return e == hipSuccess ? CS_OK : fail(CS_EHIP, "init launch: %s", hipGetErrorString(e));
}

} // extern "C"
