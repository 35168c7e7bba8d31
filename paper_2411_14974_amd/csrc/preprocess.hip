// Per-convex preprocess, forward and backward (gfx950).
//
// Forward, one thread per convex (paper Sec. 3.2): camera transform and
// pinhole projection (Eq. projection with the homogeneous divide), the 2D
// convex hull of the projected points, the hull's edge lines as signed
// distances (Sec. 3.1 Eq. signed_distance), the distance scaling of delta and
// sigma (Supp. B), the SH colour, the float32 depth key used for the
// front-to-back order, and the rectangle of tiles outside of which the
// convex's alpha stays below eps_alpha.
//
// The hull is built by gift wrapping (at most K steps of K orientation tests
// for K <= 8 points held in registers), which yields the same extreme points in
// the same cyclic order as the paper's Graham scan.
#include <algorithm>

#include "common.hpp"
#include "sh.hpp"

namespace cs {

namespace {

__device__ __forceinline__ double orient(double ax, double ay, double bx, double by, double cx, double cy)
{
    return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
}

// Inclusive pixel range [lo, hi] whose centres (u + 0.5) fall in [a, b], clamped to [0, n).
__device__ __forceinline__ void pixel_span(double a, double b, int n, int &lo, int &hi)
{
    double l = ceil(a - 0.5), h = floor(b - 0.5);
    l = fmax(l, 0.0);
    h = fmin(h, (double)(n - 1));
    if (!(l <= h)) { lo = 1; hi = 0; return; }
    lo = (int)l;
    hi = (int)h;
}

} // namespace

template <int K>
__global__ __launch_bounds__(256) void preprocess_fwd_kernel(
    int n, int deg, const float *__restrict__ points, const float *__restrict__ delta,
    const float *__restrict__ sigma, const float *__restrict__ opacity, const float *__restrict__ sh,
    const FrameHeader *__restrict__ frame, RenderArgs ra, uint8_t *__restrict__ records, uint32_t *__restrict__ keys,
    uint32_t *__restrict__ ids, uint2 *__restrict__ rects, uint32_t *__restrict__ counts,
    uint32_t *__restrict__ hullpk, DebugConvex *__restrict__ dbg)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // one (view, convex) instance per thread; all outputs are indexed by the instance
    const CamArgs cam = reinterpret_cast<const ViewDesc *>(frame + 1)[blockIdx.y].cam;
    const size_t inst = (size_t)blockIdx.y * n + i;
    ids[inst] = (uint32_t)inst;

    const float *p = points + (size_t)i * K * 3;
    float px[K], py[K], pz[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        px[k] = p[3 * k];
        py[k] = p[3 * k + 1];
        pz[k] = p[3 * k + 2];
    }

    // float32 depth key: each Z_k as an fma chain, summed in point order
    float zsum = 0.0f;
    bool near = false;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        float z = fmaf(cam.R[6], px[k], fmaf(cam.R[7], py[k], fmaf(cam.R[8], pz[k], cam.t[2])));
        near |= (z <= cam.znear);
        zsum = (k == 0) ? z : zsum + z;
    }

    int status = ST_VISIBLE;
    uint32_t key = __float_as_uint(zsum);
    uint32_t packed = 0;
    int T = 0;
    int tx0 = 1, tx1 = 0, ty0 = 1, ty1 = 0;
    double dd = 0.0, dp = 0.0, sp = 0.0;
    float rgb[3] = {0.f, 0.f, 0.f};
    int clampmask = 0;
    double lineA[K], lineB[K], lineC[K]; // debug copy (unscaled, absolute pixel frame)

    if (near) {
        status = ST_NEAR;
    } else {
        // camera space and projection, FP64
        double X[K], Y[K], Z[K], qx[K], qy[K];
        const double r0 = cam.R[0], r1 = cam.R[1], r2 = cam.R[2], r3 = cam.R[3], r4 = cam.R[4], r5 = cam.R[5];
        const double r6 = cam.R[6], r7 = cam.R[7], r8 = cam.R[8];
        double zs = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double x = px[k], y = py[k], z = pz[k];
            X[k] = r0 * x + r1 * y + r2 * z + (double)cam.t[0];
            Y[k] = r3 * x + r4 * y + r5 * z + (double)cam.t[1];
            Z[k] = r6 * x + r7 * y + r8 * z + (double)cam.t[2];
            qx[k] = (double)cam.fx * X[k] / Z[k] + (double)cam.cx;
            qy[k] = (double)cam.fy * Y[k] / Z[k] + (double)cam.cy;
            zs += Z[k];
        }
        dd = zs / K;
        dp = dd * (double)delta[i];
        sp = dd * (double)sigma[i];
        const double o = (double)opacity[i];

        // start at the point with the smallest (y, x)
        int start = 0;
        double sx = qx[0], sy = qy[0];
#pragma unroll
        for (int k = 1; k < K; ++k)
            if (qy[k] < sy || (qy[k] == sy && qx[k] < sx)) { start = k; sx = qx[k]; sy = qy[k]; }

        const double ox = rint(sx), oy = rint(sy);
        const double s2 = dp * LOG2E;
        uint8_t *rec = records + inst * rec_stride(K);
        double *lines = reinterpret_cast<double *>(rec + 64);

        // cut-off radius: outside { L_j <= r for all j } alpha < eps_alpha
        const double eps = (double)ra.eps_alpha;
        const bool faint = !(o > eps);
        const double r = faint ? 0.0 : log(o / eps - 1.0) / (sp * dp);
        double bx0 = 1e300, by0 = 1e300, bx1 = -1e300, by1 = -1e300;
        bool unbounded = false;

        int cur = start;
        double cxp = sx, cyp = sy;
        double firstA = 0, firstB = 0, firstC = 0, prevA = 0, prevB = 0, prevC = 0;
        bool closed = false;
        for (int step = 0; step < K; ++step) {
            packed |= (uint32_t)cur << (3 * T);
            ++T;
            // gift wrapping: the next vertex leaves no point to its right
            int nxt = -1;
            double nxp = 0.0, nyp = 0.0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (k == cur) continue;
                if (nxt < 0) { nxt = k; nxp = qx[k]; nyp = qy[k]; continue; }
                const double ot = orient(cxp, cyp, nxp, nyp, qx[k], qy[k]);
                bool take = ot < 0.0;
                if (ot == 0.0) {
                    const double dk = (qx[k] - cxp) * (qx[k] - cxp) + (qy[k] - cyp) * (qy[k] - cyp);
                    const double dn = (nxp - cxp) * (nxp - cxp) + (nyp - cyp) * (nyp - cyp);
                    take = dk > dn;
                }
                if (take) { nxt = k; nxp = qx[k]; nyp = qy[k]; }
            }
            // edge cur -> nxt: outward unit normal (e_y, -e_x)/|e|
            const double ex = nxp - cxp, ey = nyp - cyp;
            const double len = sqrt(ex * ex + ey * ey);
            const double A = ey / len, B = -ex / len;
            const double Cabs = -(A * cxp + B * cyp);
            const double Crel = -(A * (cxp - ox) + B * (cyp - oy));
            const int j = T - 1;
            lines[3 * j + 0] = s2 * A;
            lines[3 * j + 1] = s2 * B;
            lines[3 * j + 2] = s2 * Crel;
#pragma unroll
            for (int jj = 0; jj < K; ++jj)
                if (jj == j) { lineA[jj] = A; lineB[jj] = B; lineC[jj] = Cabs; }
            // corner of the pushed-out polygon at vertex cur (needs the incoming line)
            if (j == 0) {
                firstA = A; firstB = B; firstC = Cabs;
            } else {
                const double den = 1.0 + prevA * A + prevB * B;
                if (den < 1e-6) unbounded = true;
                const double mx = cxp + r * (prevA + A) / den, my = cyp + r * (prevB + B) / den;
                bx0 = fmin(bx0, fmin(mx, cxp)); bx1 = fmax(bx1, fmax(mx, cxp));
                by0 = fmin(by0, fmin(my, cyp)); by1 = fmax(by1, fmax(my, cyp));
            }
            prevA = A; prevB = B; prevC = Cabs;
            if (nxt == start) { closed = true; break; }
            cur = nxt; cxp = nxp; cyp = nyp;
        }
        (void)prevC; (void)firstC;
        if (closed && T >= 3) {
            const double den = 1.0 + prevA * firstA + prevB * firstB;
            if (den < 1e-6) unbounded = true;
            const double mx = sx + r * (prevA + firstA) / den, my = sy + r * (prevB + firstB) / den;
            bx0 = fmin(bx0, fmin(mx, sx)); bx1 = fmax(bx1, fmax(mx, sx));
            by0 = fmin(by0, fmin(my, sy)); by1 = fmax(by1, fmax(my, sy));
        }

        if (!closed || T < 3) {
            status = ST_HULL;
        } else {
            // colour from SH at the direction camera -> point centroid
            double cxw = 0, cyw = 0, czw = 0;
#pragma unroll
            for (int k = 0; k < K; ++k) { cxw += px[k]; cyw += py[k]; czw += pz[k]; }
            const double vx = cxw / K - cam.campos[0], vy = cyw / K - cam.campos[1], vz = czw / K - cam.campos[2];
            const double inv = 1.0 / sqrt(vx * vx + vy * vy + vz * vz);
            float Yb[16];
            sh_eval(deg, (float)(vx * inv), (float)(vy * inv), (float)(vz * inv), Yb);
            const int nc = (deg + 1) * (deg + 1);
            const float *f = sh + (size_t)i * nc * 3;
            float raw[3] = {0.5f, 0.5f, 0.5f};
            for (int c = 0; c < nc; ++c) {
                raw[0] = fmaf(Yb[c], f[3 * c + 0], raw[0]);
                raw[1] = fmaf(Yb[c], f[3 * c + 1], raw[1]);
                raw[2] = fmaf(Yb[c], f[3 * c + 2], raw[2]);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (raw[c] > 0.0f) rgb[c] = raw[c];
                else { rgb[c] = 0.0f; clampmask |= 1 << c; }
            }

            RecHeader h;
            h.ox = (float)ox;
            h.oy = (float)oy;
            h.sigma_p = (float)sp;
            // skip when max_j x2_j > log2(o/eps - 1) / sigma'  (LogSumExp >= its max)
            h.thr2 = faint ? -INFINITY : (float)(log2(o / eps - 1.0) / sp);
            h.opacity = (float)o;
            h.rgb[0] = rgb[0]; h.rgb[1] = rgb[1]; h.rgb[2] = rgb[2];
            h.T = T;
            h.id = (int32_t)inst;
#pragma unroll
            for (int q = 0; q < 6; ++q) h.pad[q] = 0;
            const uint4 *hs = reinterpret_cast<const uint4 *>(&h);
            uint4 *hd = reinterpret_cast<uint4 *>(rec);
#pragma unroll
            for (int q = 0; q < 4; ++q) hd[q] = hs[q];

            if (faint) {
                status = ST_FAINT;
            } else {
                if (r <= 0.0) { // region inside the hull: its vertex box bounds it
                    bx0 = by0 = 1e300; bx1 = by1 = -1e300;
                    for (int j = 0; j < T; ++j) {
                        const int v = (packed >> (3 * j)) & 7;
#pragma unroll
                        for (int k = 0; k < K; ++k)
                            if (k == v) {
                                bx0 = fmin(bx0, qx[k]); bx1 = fmax(bx1, qx[k]);
                                by0 = fmin(by0, qy[k]); by1 = fmax(by1, qy[k]);
                            }
                    }
                }
                if (unbounded) { bx0 = by0 = -1e300; bx1 = by1 = 1e300; }
                const double mg = 1e-3;
                int u0, u1, v0, v1;
                pixel_span(bx0 - mg, bx1 + mg, cam.W, u0, u1);
                pixel_span(by0 - mg, by1 + mg, cam.H, v0, v1);
                if (u0 <= u1 && v0 <= v1) {
                    tx0 = u0 / ra.tile; tx1 = u1 / ra.tile;
                    ty0 = v0 / ra.tile; ty1 = v1 / ra.tile;
                }
            }
        }
    }

    const bool has_tiles = status == ST_VISIBLE && tx0 <= tx1 && ty0 <= ty1;
    keys[inst] = status == ST_VISIBLE ? key : KEY_CULLED;
    counts[inst] = has_tiles ? (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1)) : 0u;
    rects[inst] = has_tiles ? make_uint2((uint32_t)tx0 | ((uint32_t)ty0 << 16), (uint32_t)tx1 | ((uint32_t)ty1 << 16))
                         : make_uint2(1u, 0u);
    hullpk[inst] = (status == ST_VISIBLE || status == ST_FAINT) ? (packed | ((uint32_t)T << 28)) : 0u;

    if (dbg) {
        DebugConvex &o = dbg[inst];
        o.status = status;
        o.T = (status == ST_NEAR) ? 0 : T;
        for (int j = 0; j < MAXK; ++j) {
            o.hull[j] = (j < T && status != ST_NEAR) ? (int32_t)((packed >> (3 * j)) & 7) : -1;
            o.A[j] = o.B[j] = o.C[j] = 0.0;
        }
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (j < T && status != ST_NEAR) { o.A[j] = lineA[j]; o.B[j] = lineB[j]; o.C[j] = lineC[j]; }
        o.depth_key = key;
        o.clampmask = clampmask;
        o.d = dd;
        o.delta_p = dp;
        o.sigma_p = sp;
        o.rgb[0] = rgb[0]; o.rgb[1] = rgb[1]; o.rgb[2] = rgb[2];
        o.tile_rect[0] = has_tiles ? tx0 : 1;
        o.tile_rect[1] = has_tiles ? ty0 : 1;
        o.tile_rect[2] = has_tiles ? tx1 : 0;
        o.tile_rect[3] = has_tiles ? ty1 : 0;
    }
}

// Backward, one thread per convex, summed over the views of the frame: chain
// each instance's accumulators of the compositing backward (base-2 line
// coefficients, sigma', opacity, colour, x2-weighted sum) through lines -> hull
// vertices -> projection -> points, delta' and sigma' -> (delta, sigma, d),
// d -> every point, colour -> SH and view direction.  The geometry is
// recomputed from the points and the stored hull indices, bit-identically to
// the forward pass.
template <int K>
__device__ __forceinline__ void view_backward(int deg, const float *px, const float *py, const float *pz, double dl,
                                              double sg, const float *f, const CamArgs &cam, uint32_t hp,
                                              const float *__restrict__ A, float *gp, float &gdelta, float &gsigma,
                                              float &gopac, float *gsh)
{
    const int T = (int)(hp >> 28);
    const int nc = (deg + 1) * (deg + 1);
    double X[K], Y[K], Z[K], qx[K], qy[K];
    const double r0 = cam.R[0], r1 = cam.R[1], r2 = cam.R[2], r3 = cam.R[3], r4 = cam.R[4], r5 = cam.R[5];
    const double r6 = cam.R[6], r7 = cam.R[7], r8 = cam.R[8];
    double zs = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double x = px[k], y = py[k], z = pz[k];
        X[k] = r0 * x + r1 * y + r2 * z + (double)cam.t[0];
        Y[k] = r3 * x + r4 * y + r5 * z + (double)cam.t[1];
        Z[k] = r6 * x + r7 * y + r8 * z + (double)cam.t[2];
        qx[k] = (double)cam.fx * X[k] / Z[k] + (double)cam.cx;
        qy[k] = (double)cam.fy * Y[k] / Z[k] + (double)cam.cy;
        zs += Z[k];
    }
    const double dd = zs / K;
    const double dp = dd * dl;
    const double s2 = dp * LOG2E;

    // hull vertices in order
    double vx[K], vy[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int v = (hp >> (3 * j)) & 7;
        vx[j] = 0.0;
        vy[j] = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (k == v) { vx[j] = qx[k]; vy[j] = qy[k]; }
    }
    // origin used by the forward pass: the start vertex rounded
    const double ox = rint(vx[0]), oy = rint(vy[0]);

    double gvx[K], gvy[K];
#pragma unroll
    for (int j = 0; j < K; ++j) { gvx[j] = 0.0; gvy[j] = 0.0; }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j >= T) continue;
        // edge j: vertex j -> vertex j+1 (mod T)
        double bxv = vx[0], byv = vy[0];
#pragma unroll
        for (int jj = 1; jj < K; ++jj)
            if (jj == j + 1 && jj < T) { bxv = vx[jj]; byv = vy[jj]; }
        const double ex = bxv - vx[j], ey = byv - vy[j];
        const double len = sqrt(ex * ex + ey * ey);
        const double tx = ex / len, ty = ey / len;
        const double nA = ty, nB = -tx;
        const double ax = vx[j] - ox, ay = vy[j] - oy;
        // stored (a, b, c) = s2 * (A, B, C'), C' = -(A ax + B ay)
        const double gA = s2 * (double)A[j], gB = s2 * (double)A[K + j], gC = s2 * (double)A[2 * K + j];
        const double gAt = gA - gC * ax, gBt = gB - gC * ay;
        gvx[j] -= gC * nA;
        gvy[j] -= gC * nB;
        // n = (e_y, -e_x)/|e|  =>  dL/de = -((g_n . t)/|e|) n
        const double sdot = (gAt * tx + gBt * ty) / len;
        const double gex = -sdot * nA, gey = -sdot * nB;
        gvx[j] -= gex;
        gvy[j] -= gey;
#pragma unroll
        for (int jj = 0; jj < K; ++jj)
            if (jj == ((j + 1 == T) ? 0 : j + 1)) { gvx[jj] += gex; gvy[jj] += gey; }
    }
    // x2_j = delta' log2(e) L_j  =>  dx2_j / ddelta' = x2_j / delta'
    const double gdp = (double)A[3 * K + 5] / dp;
    const double gsp = (double)A[3 * K];
    gdelta += (float)(dd * gdp);
    gsigma += (float)(dd * gsp);
    gopac += A[3 * K + 1];
    const double gd = dl * gdp + sg * gsp;

    // hull vertices -> projected points
    double gqx[K], gqy[K];
#pragma unroll
    for (int k = 0; k < K; ++k) { gqx[k] = 0.0; gqy[k] = 0.0; }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j >= T) continue;
        const int v = (hp >> (3 * j)) & 7;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (k == v) { gqx[k] += gvx[j]; gqy[k] += gvy[j]; }
    }

    // colour -> SH coefficients and the view direction
    double cxw = 0, cyw = 0, czw = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) { cxw += px[k]; cyw += py[k]; czw += pz[k]; }
    const double wx = cxw / K - cam.campos[0], wy = cyw / K - cam.campos[1], wz = czw / K - cam.campos[2];
    const double dist = sqrt(wx * wx + wy * wy + wz * wz);
    const float dx = (float)(wx / dist), dy = (float)(wy / dist), dz = (float)(wz / dist);
    float Yb[16];
    sh_eval(deg, dx, dy, dz, Yb);
    float raw[3] = {0.5f, 0.5f, 0.5f};
    for (int c = 0; c < nc; ++c) {
        raw[0] = fmaf(Yb[c], f[3 * c + 0], raw[0]);
        raw[1] = fmaf(Yb[c], f[3 * c + 1], raw[1]);
        raw[2] = fmaf(Yb[c], f[3 * c + 2], raw[2]);
    }
    float graw[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) graw[c] = raw[c] > 0.0f ? A[3 * K + 2 + c] : 0.0f;
    float wsum[16];
    for (int c = 0; c < nc; ++c) {
        gsh[3 * c + 0] += graw[0] * Yb[c];
        gsh[3 * c + 1] += graw[1] * Yb[c];
        gsh[3 * c + 2] += graw[2] * Yb[c];
        wsum[c] = graw[0] * f[3 * c + 0] + graw[1] * f[3 * c + 1] + graw[2] * f[3 * c + 2];
    }
    float gdx = 0.f, gdy = 0.f, gdz = 0.f;
    sh_grad_dot(deg, dx, dy, dz, wsum, gdx, gdy, gdz);
    // unit direction -> centre:  (I - dir dir^T) / |centre - campos|
    const double dot = (double)dx * gdx + (double)dy * gdy + (double)dz * gdz;
    const double gcx = ((double)gdx - dx * dot) / dist / K;
    const double gcy = ((double)gdy - dy * dot) / dist / K;
    const double gcz = ((double)gdz - dz * dot) / dist / K;

    // projection and depth -> camera space -> world (R^T)
    const double fx = cam.fx, fy = cam.fy;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double iz = 1.0 / Z[k];
        const double gX = gqx[k] * fx * iz, gY = gqy[k] * fy * iz;
        const double gZ = -(gqx[k] * fx * X[k] + gqy[k] * fy * Y[k]) * iz * iz + gd / K;
        gp[3 * k + 0] += (float)(r0 * gX + r3 * gY + r6 * gZ + gcx);
        gp[3 * k + 1] += (float)(r1 * gX + r4 * gY + r7 * gZ + gcy);
        gp[3 * k + 2] += (float)(r2 * gX + r5 * gY + r8 * gZ + gcz);
    }
}

template <int K>
__global__ __launch_bounds__(256) void preprocess_bwd_kernel(
    int n, int nviews, int deg, const float *__restrict__ points, const float *__restrict__ delta,
    const float *__restrict__ sigma, const float *__restrict__ sh, const FrameHeader *__restrict__ frame,
    const uint32_t *__restrict__ hullpk, const float *__restrict__ acc, float *__restrict__ g_points,
    float *__restrict__ g_delta, float *__restrict__ g_sigma, float *__restrict__ g_opacity,
    float *__restrict__ g_sh)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int nc = (deg + 1) * (deg + 1);
    float gp[3 * K], gsh[48];
#pragma unroll
    for (int k = 0; k < 3 * K; ++k) gp[k] = 0.0f;
#pragma unroll
    for (int c = 0; c < 48; ++c) gsh[c] = 0.0f;
    float gdelta = 0.0f, gsigma = 0.0f, gopac = 0.0f;

    const float *p = points + (size_t)i * K * 3;
    float px[K], py[K], pz[K];
#pragma unroll
    for (int k = 0; k < K; ++k) { px[k] = p[3 * k]; py[k] = p[3 * k + 1]; pz[k] = p[3 * k + 2]; }
    const double dl = (double)delta[i], sg = (double)sigma[i];
    const float *f = sh + (size_t)i * nc * 3;
    const ViewDesc *views = reinterpret_cast<const ViewDesc *>(frame + 1);
    for (int v = 0; v < nviews; ++v) {
        const size_t inst = (size_t)v * n + i;
        const uint32_t hp = hullpk[inst];
        if ((int)(hp >> 28) < 3) continue; // dropped in this view: no gradient
        view_backward<K>(deg, px, py, pz, dl, sg, f, views[v].cam, hp, acc + inst * acc_stride(K), gp, gdelta,
                         gsigma, gopac, gsh);
    }
    float *gpo = g_points + (size_t)i * K * 3;
#pragma unroll
    for (int k = 0; k < 3 * K; ++k) gpo[k] = gp[k];
    float *gso = g_sh + (size_t)i * nc * 3;
    for (int c = 0; c < 3 * nc; ++c) gso[c] = gsh[c];
    g_delta[i] = gdelta;
    g_sigma[i] = gsigma;
    g_opacity[i] = gopac;
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

void launch_preprocess_fwd(hipStream_t st, int n, int nviews, int K, int deg, const float *points,
                           const float *delta, const float *sigma, const float *opacity, const float *sh,
                           const FrameHeader *views, const RenderArgs &ra, uint8_t *records, uint32_t *keys,
                           uint32_t *ids, uint2 *rects, uint32_t *counts, uint32_t *hullpk, DebugConvex *dbg)
{
    if (n <= 0 || nviews <= 0) return;
    dim3 grid((n + 255) / 256, nviews), block(256);
    CS_DISPATCH_K(K, hipLaunchKernelGGL(preprocess_fwd_kernel<KK>, grid, block, 0, st, n, deg, points, delta, sigma,
                                        opacity, sh, views, ra, records, keys, ids, rects, counts, hullpk, dbg));
}

void launch_preprocess_bwd(hipStream_t st, int n, int nviews, int K, int deg, const float *points,
                           const float *delta, const float *sigma, const float *sh, const FrameHeader *views,
                           const uint32_t *hullpk, const float *acc, float *g_points, float *g_delta,
                           float *g_sigma, float *g_opacity, float *g_sh)
{
    if (n <= 0) return;
    dim3 grid((n + 255) / 256), block(256);
    CS_DISPATCH_K(K, hipLaunchKernelGGL(preprocess_bwd_kernel<KK>, grid, block, 0, st, n, nviews, deg, points, delta,
                                        sigma, sh, views, hullpk, acc, g_points, g_delta, g_sigma, g_opacity, g_sh));
}

} // namespace cs
