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
    int32_t pad[6];
};
static_assert(sizeof(RecHeader) == 64, "record header is 64 bytes");

__host__ __device__ constexpr int rec_stride(int K) { return (64 + 24 * K + 15) & ~15; }
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
    int32_t tile, tiles_x, tiles_y;
};

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
