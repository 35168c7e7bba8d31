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
#include "convexsplat.h"
#include "sh.hpp"

namespace cs {

namespace {

__device__ __forceinline__ double orient(double ax, double ay, double bx, double by, double cx, double cy)
{
    return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
}

// Storage formats of the scene parameters: float32, or the 16-bit formats of
// the light model (IEEE half, bfloat16).  Every load converts to float32
// (exactly), and all arithmetic after it is the float32 path's.
struct Half { uint16_t b; };
struct BHalf { uint16_t b; };
__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(Half v) { return (float)__builtin_bit_cast(_Float16, v.b); }
__device__ __forceinline__ float to_f32(BHalf v) { return __uint_as_float((uint32_t)v.b << 16); }
template <typename P> __device__ __forceinline__ float ld(const P *p, size_t i) { return to_f32(p[i]); }
// Values 4q .. 4q+3 of a row: one 16-byte load for float32, one 8-byte load
// for the 16-bit formats (little-endian: element 4q is the low half of x).
template <typename P> __device__ __forceinline__ float4 ld4(const P *p, int q)
{
    if constexpr (sizeof(P) == 4) {
        return reinterpret_cast<const float4 *>(p)[q];
    } else {
        const uint2 w = reinterpret_cast<const uint2 *>(p)[q];
        return make_float4(to_f32(P{(uint16_t)(w.x & 0xFFFFu)}), to_f32(P{(uint16_t)(w.x >> 16)}),
                           to_f32(P{(uint16_t)(w.y & 0xFFFFu)}), to_f32(P{(uint16_t)(w.y >> 16)}));
    }
}

// 1/x and 1/sqrt(x) in FP64: the hardware estimate and two Newton steps (each
// doubles the correct bits), to within an ulp or two of the rounded result for
// the finite, nonzero, normal arguments they get here (depths beyond the near
// plane, squared edge lengths of distinct hull vertices, polygon-corner
// denominators, nonzero line slopes); the correctly rounded division is an
// eleven-instruction sequence.
__device__ __forceinline__ double rcp64(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}
__device__ __forceinline__ double rsq64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    double t = fma(-h * y, y, 0.5); // y <- y (1.5 - x y^2 / 2)
    y = fma(y, t, y);
    t = fma(-h * y, y, 0.5);
    return fma(y, t, y);
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

// Block-cooperative copy of `rows` contiguous global rows of W values into
// LDS rows of stride S.  U loads per thread are issued before the first LDS
// store: a plain loop would wait for each load in turn.
template <int NT, int U, typename P>
__device__ __forceinline__ void stage_rows(float *lds, const P *g, int rows, int W, int S)
{
    const int total = rows * W;
    const int drow = NT / W, dcol = NT - drow * W;
    int row = (int)threadIdx.x / W, col = (int)threadIdx.x - row * W;
    for (int j0 = threadIdx.x; j0 < total; j0 += U * NT) {
        float v[U];
        // unconditional loads (a clamped index): a guarded load compiles to a
        // branch and a wait of its own
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = ld(g, min(j0 + u * NT, total - 1));
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (j0 + u * NT < total) lds[row * S + col] = v[u];
            row += drow;
            col += dcol;
            if (col >= W) { col -= W; ++row; }
        }
    }
}

} // namespace

constexpr int PF_BLOCK = 128;

// DBG: also fill the per-instance debug record (a separate instantiation, so
// that the debug copies of the lines cost no registers in the plain one).
template <int K, bool DBG, typename P>
__global__ __launch_bounds__(PF_BLOCK) void preprocess_fwd_kernel(
    int n, int deg, const P *__restrict__ points, const P *__restrict__ delta,
    const P *__restrict__ sigma, const P *__restrict__ opacity, const P *__restrict__ sh,
    const FrameHeader *__restrict__ frame, RenderArgs ra, uint8_t *__restrict__ records, uint32_t *__restrict__ keys,
    uint32_t *__restrict__ ids, uint4 *__restrict__ bins, uint32_t *__restrict__ hullpk,
    DebugConvex *__restrict__ dbg, ZeroSpans zero)
{
    zero_share(zero); // the frame's counters and the depth sort's temporaries, when asked
    // The block's points arrive through LDS (coalesced loads; odd row stride);
    // once they are in registers the same LDS holds the block's records, which
    // leave in coalesced 16-byte stores (one contiguous run per block).
    constexpr int PS = 3 * K + 1;
    constexpr int RC = rec_stride(K) / 16;
    constexpr int BUF = (PF_BLOCK * RC > (PF_BLOCK * PS + 3) / 4) ? PF_BLOCK * RC : (PF_BLOCK * PS + 3) / 4;
    __shared__ uint4 s_buf[BUF];
    float *s_pts = reinterpret_cast<float *>(s_buf);
    const int base = blockIdx.x * PF_BLOCK;
    const int cnt = min(PF_BLOCK, n - base);
    stage_rows<PF_BLOCK, 3 * K>(s_pts, points + (size_t)base * 3 * K, cnt, 3 * K, PS);
    __syncthreads();
    // one (view, convex) instance per thread; all outputs are indexed by the
    // instance (threads past n compute on the last convex, whose row they read,
    // and store nothing)
    const bool active = base + (int)threadIdx.x < n;
    const int i = active ? base + (int)threadIdx.x : n - 1;
    const int srow = active ? (int)threadIdx.x : cnt - 1;
    const CamArgs cam = reinterpret_cast<const ViewDesc *>(frame + 1)[blockIdx.y].cam;
    const size_t inst = (size_t)blockIdx.y * n + i;
    if (active) ids[inst] = (uint32_t)inst;

    float px[K], py[K], pz[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        px[k] = s_pts[srow * PS + 3 * k];
        py[k] = s_pts[srow * PS + 3 * k + 1];
        pz[k] = s_pts[srow * PS + 3 * k + 2];
    }
    __syncthreads(); // the LDS now takes the records
    // point centroid (for the SH view direction), taken now so the points can retire early
    double cxw = 0, cyw = 0, czw = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) { cxw += px[k]; cyw += py[k]; czw += pz[k]; }

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
    uint64_t tmask = 0;  // kept tiles of the rectangle (binning record encoding)
    double dd = 0.0, dp = 0.0, sp = 0.0;
    float rgb[3] = {0.f, 0.f, 0.f};
    int clampmask = 0;
    double lineA[DBG ? K : 1], lineB[DBG ? K : 1], lineC[DBG ? K : 1]; // debug copy (unscaled, absolute pixel frame)

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
            // the projection with true divisions: the hull's orientation tests
            // and the edge normals read it bit for bit, and a one-ulp change of
            // a point moves the normal of a short edge by far more than an ulp
            qx[k] = (double)cam.fx * X[k] / Z[k] + (double)cam.cx;
            qy[k] = (double)cam.fy * Y[k] / Z[k] + (double)cam.cy;
            zs += Z[k];
        }
        dd = zs / K;
        dp = dd * (double)ld(delta, i);
        sp = dd * (double)ld(sigma, i);
        const double o = (double)ld(opacity, i);

        // start at the point with the smallest (y, x)
        int start = 0;
        double sx = qx[0], sy = qy[0];
#pragma unroll
        for (int k = 1; k < K; ++k)
            if (qy[k] < sy || (qy[k] == sy && qx[k] < sx)) { start = k; sx = qx[k]; sy = qy[k]; }

        const double ox = rint(sx), oy = rint(sy);
        const double s2 = dp * LOG2E;
        uint8_t *rec = reinterpret_cast<uint8_t *>(s_buf) + threadIdx.x * rec_stride(K);
        // the lines leave as aligned pairs of doubles (16-byte stores): line j
        // occupies doubles 3j..3j+2 after the header; an odd line's first value
        // waits in `carry` for the even line's last one
        double2 *lines2 = reinterpret_cast<double2 *>(rec + REC_HEADER);
        double carry = 0.0;

        // cut-off radius: outside { L_j <= r for all j } alpha < eps_alpha.  The
        // logarithm in float32 (the radius is a sub-pixel length bounded with a
        // 1e-3 pixel margin; the skip threshold below is stored as a float)
        const double eps = (double)ra.eps_alpha;
        const bool faint = !(o > eps);
        const float lg2 = faint ? 0.0f : __log2f((float)(o / eps - 1.0));
        const double r = faint ? 0.0 : (double)lg2 * LN2 * rcp64(sp * dp);
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
            const double il = rsq64(ex * ex + ey * ey);
            const double A = ey * il, B = -ex * il;
            const double Cabs = -(A * cxp + B * cyp);
            const double Crel = -(A * (cxp - ox) + B * (cyp - oy));
            const int j = T - 1;
            if ((j & 1) == 0) {
                lines2[(3 * j) >> 1] = make_double2(s2 * A, s2 * B);
                carry = s2 * Crel;
            } else {
                lines2[(3 * j - 1) >> 1] = make_double2(carry, s2 * A);
                lines2[(3 * j + 1) >> 1] = make_double2(s2 * B, s2 * Crel);
            }
            if constexpr (DBG) {
#pragma unroll
                for (int jj = 0; jj < K; ++jj)
                    if (jj == j) { lineA[jj] = A; lineB[jj] = B; lineC[jj] = Cabs; }
            }
            // corner of the pushed-out polygon at vertex cur (needs the incoming line)
            if (j == 0) {
                firstA = A; firstB = B; firstC = Cabs;
            } else {
                const double den = 1.0 + prevA * A + prevB * B;
                if (den < 1e-6) unbounded = true; // (then the box is unbounded, whatever rd is)
                const double rd = r * rcp64(den);
                const double mx = cxp + rd * (prevA + A), my = cyp + rd * (prevB + B);
                bx0 = fmin(bx0, fmin(mx, cxp)); bx1 = fmax(bx1, fmax(mx, cxp));
                by0 = fmin(by0, fmin(my, cyp)); by1 = fmax(by1, fmax(my, cyp));
            }
            prevA = A; prevB = B; prevC = Cabs;
            if (nxt == start) { closed = true; break; }
            cur = nxt; cxp = nxp; cyp = nyp;
        }
        (void)prevC; (void)firstC;
        // null lines in the slots past T (same pairing of doubles)
        for (int j = T; j < K; ++j) {
            if ((j & 1) == 0) {
                lines2[(3 * j) >> 1] = make_double2(0.0, 0.0);
                carry = NULL_LINE_C;
            } else {
                lines2[(3 * j - 1) >> 1] = make_double2(carry, 0.0);
                lines2[(3 * j + 1) >> 1] = make_double2(0.0, NULL_LINE_C);
            }
        }
        if (K & 1) lines2[(3 * K - 1) >> 1] = make_double2(carry, 0.0); // the last line's c
        if (closed && T >= 3) {
            const double den = 1.0 + prevA * firstA + prevB * firstB;
            if (den < 1e-6) unbounded = true;
            const double rd = r * rcp64(den);
            const double mx = sx + rd * (prevA + firstA), my = sy + rd * (prevB + firstB);
            bx0 = fmin(bx0, fmin(mx, sx)); bx1 = fmax(bx1, fmax(mx, sx));
            by0 = fmin(by0, fmin(my, sy)); by1 = fmax(by1, fmax(my, sy));
        }

        if (!closed || T < 3) {
            status = ST_HULL;
        } else {
            // colour from SH at the direction camera -> point centroid
            const double vx = cxw / K - cam.campos[0], vy = cyw / K - cam.campos[1], vz = czw / K - cam.campos[2];
            const double inv = 1.0 / sqrt(vx * vx + vy * vy + vz * vz);
            float Yb[16];
            sh_eval(deg, (float)(vx * inv), (float)(vy * inv), (float)(vz * inv), Yb);
            const int nc = (deg + 1) * (deg + 1);
            const P *f = sh + (size_t)i * nc * 3;
            float raw[3] = {0.5f, 0.5f, 0.5f};
            if (deg == 3) { // 48-value rows: 4 values per load, same summation order
#pragma unroll
                for (int q = 0; q < 12; ++q) {
                    const float4 w = ld4(f, q);
                    const float wv[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int e = 4 * q + t; // coefficient e / 3, channel e % 3
                        raw[e % 3] = fmaf(Yb[e / 3], wv[t], raw[e % 3]);
                    }
                }
            } else {
                for (int c = 0; c < nc; ++c) {
                    raw[0] = fmaf(Yb[c], ld(f, 3 * c + 0), raw[0]);
                    raw[1] = fmaf(Yb[c], ld(f, 3 * c + 1), raw[1]);
                    raw[2] = fmaf(Yb[c], ld(f, 3 * c + 2), raw[2]);
                }
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
            h.thr2 = faint ? -INFINITY : (float)((double)lg2 * rcp64(sp));
            h.opacity = (float)o;
            h.rgb[0] = rgb[0]; h.rgb[1] = rgb[1]; h.rgb[2] = rgb[2];
            h.T = T;
            h.id = (int32_t)inst;
            h.box_u = 1u; // empty until the cut-off rectangle is known
            h.box_v = 1u;

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
                    h.box_u = (uint32_t)u0 | ((uint32_t)u1 << 16);
                    h.box_v = (uint32_t)v0 | ((uint32_t)v1 << 16);
                    // Drop the tiles where one line keeps x2 above the skip
                    // threshold over every pixel centre of the tile's part of the
                    // box: there the compositing skips the convex at every pixel
                    // (max_j x2_j > thr2), so the pair is not emitted.  The minimum
                    // of a line over the rectangle is at a corner; the margin covers
                    // the rounding of both evaluations.
                    // A small rectangle one tile wide or high keeps every tile:
                    // the polygon is connected and its bounding box spans the
                    // strip.  A rectangle of more than 64 tiles is culled the
                    // same way per band of rows, in blocks of columns.
                    const int tw = tx1 - tx0 + 1, th = ty1 - ty0 + 1;
                    const bool big = tw * th > 64;
                    tmask = (tw * th < 64) ? ((1ull << (tw * th)) - 1ull) : ~0ull;
                    if (big || (tw >= 2 && th >= 2)) {
                        // the lines as stored, into registers once (slots past T unused)
                        const double *ln = reinterpret_cast<const double *>(rec + REC_HEADER);
                        double la[K], lb[K], lc[K];
#pragma unroll
                        for (int j = 0; j < K; ++j) {
                            la[j] = ln[3 * j];
                            lb[j] = ln[3 * j + 1];
                            lc[j] = ln[3 * j + 2];
                        }
                        const double lim = (double)h.thr2 + 1e-3;
                        // per line: la x + lb y + lc <= lim on the kept part; over a
                        // tile row (pixel-centre rows c0..c1) the line keeps the
                        // columns with x <= hi_j (la > 0) or x >= lo_j (la < 0), so
                        // each row keeps one interval of tiles (cost per row, not per tile)
                        double inv[K];
#pragma unroll
                        for (int j = 0; j < K; ++j) inv[j] = la[j] != 0.0 ? rcp64(la[j]) : 0.0;
                        // small: one tile row per step; big: one band of bh rows
                        const int bh = big ? big_bh(th) : 1, bw = big ? big_bw(tw) : 1;
                        uint64_t m = big ? BIG_EMPTY : 0ull;
                        for (int ty = ty0, r = 0; ty <= ty1; ty += bh, ++r) {
                            const int tyb = min(ty + bh - 1, ty1);
                            const double c0 = (double)max(ty * ra.tile, v0) + 0.5 - oy;
                            const double c1 = (double)min(tyb * ra.tile + ra.tile - 1, v1) + 0.5 - oy;
                            double xlo = -INFINITY, xhi = INFINITY; // kept pixel centres, origin-relative
                            bool none = false;
#pragma unroll
                            for (int j = 0; j < K; ++j) { // null lines never drop a tile
                                const double rest = lim - (lc[j] + fmin(lb[j] * c0, lb[j] * c1));
                                const double b = rest * inv[j];
                                if (la[j] > 0.0) xhi = fmin(xhi, b);
                                else if (la[j] < 0.0) xlo = fmax(xlo, b);
                                else none = none || rest < 0.0;
                            }
                            // first and last pixel columns of the box with a centre in [xlo, xhi]
                            const double ulo = fmax(ceil(xlo + ox - 0.5), (double)u0);
                            const double uhi = fmin(floor(xhi + ox - 0.5), (double)u1);
                            if (none || !(ulo <= uhi)) continue;
                            const int kx0 = (int)ulo / ra.tile - tx0, kx1 = (int)uhi / ra.tile - tx0;
                            if (big) {
                                m = (m & ~(BIG_FIELD << (2 * BIG_BITS * r))) | big_field(kx0 / bw, kx1 / bw, r);
                            } else {
                                const int nk = kx1 - kx0 + 1;
                                m |= ((nk == 64) ? ~0ull : ((1ull << nk) - 1ull)) << ((ty - ty0) * tw + kx0);
                            }
                        }
                        tmask = m;
                    }
                }
            }
            const uint4 *hs = reinterpret_cast<const uint4 *>(&h);
            uint4 *hd = reinterpret_cast<uint4 *>(rec);
#pragma unroll
            for (int q = 0; q < REC_HEADER / 16; ++q) hd[q] = hs[q];
        }
    }

    const bool has_tiles = status == ST_VISIBLE && tx0 <= tx1 && ty0 <= ty1;
    if (active) {
        keys[inst] = status == ST_VISIBLE ? key : KEY_CULLED;
        bins[inst] = has_tiles ? make_bin(tx0, ty0, tx1, ty1, tmask) : make_bin(1, 0, 0, 0, 0);
        // hull indices (3 bits each, bits 0-23), the clamped colour channels
        // (bits 24-26: the backward pass's colour gradient is zero there), T
        hullpk[inst] = (status == ST_VISIBLE || status == ST_FAINT)
                           ? (packed | ((uint32_t)clampmask << 24) | ((uint32_t)T << 28))
                           : 0u;
    }
    // the block's records (culled convexes' slots hold whatever the LDS held:
    // nothing reads a culled convex's record)
    __syncthreads();
    {
        uint4 *dst = reinterpret_cast<uint4 *>(records + ((size_t)blockIdx.y * n + base) * rec_stride(K));
        for (int c = threadIdx.x; c < cnt * RC; c += PF_BLOCK) dst[c] = s_buf[c];
    }

    if constexpr (DBG) {
        if (!active) return;
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
// recomputed from the points (camera transform in FP64, the rest in FP32 with
// pixel coordinates relative to the record's origin, the frame in which the
// forward pass stored its lines); gradients need relative, not absolute,
// accuracy.  The colour clamp max(0, raw) is the forward pass's own decision,
// carried in the packed hull word.

// Unit view direction (camera centre -> point centroid) and its SH basis
// values, with the forward pass's arithmetic.
template <int K>
__device__ __forceinline__ void view_dir(int deg, const float *P, const CamArgs &cam, float &dx, float &dy, float &dz,
                                         double &inv, float *Yb)
{
    double cxw = 0, cyw = 0, czw = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) { cxw += P[3 * k]; cyw += P[3 * k + 1]; czw += P[3 * k + 2]; }
    const double wx = cxw / K - cam.campos[0], wy = cyw / K - cam.campos[1], wz = czw / K - cam.campos[2];
    inv = 1.0 / sqrt(wx * wx + wy * wy + wz * wz);
    dx = (float)(wx * inv);
    dy = (float)(wy * inv);
    dz = (float)(wz * inv);
    sh_eval(deg, dx, dy, dz, Yb);
}

// An instance's accumulator row, in 16-byte loads.
template <int K> __device__ __forceinline__ void load_acc_row(const float *__restrict__ Ag, float *A)
{
#pragma unroll
    for (int q = 0; q < acc_stride(K) / 4; ++q) {
        const float4 w = reinterpret_cast<const float4 *>(Ag)[q];
        A[4 * q] = w.x; A[4 * q + 1] = w.y; A[4 * q + 2] = w.z; A[4 * q + 3] = w.w;
    }
}

// Everything after the SH coefficients: wsum_c = sum_t dL/draw_t f_ct gives
// the direction's gradient; then the hull lines, projection and depth.
// ADD: G accumulates (several views); otherwise G is assigned, after the
// last read of P (G may be P's own row).
template <int K, bool ADD>
__device__ __forceinline__ void geometry_backward(int deg, const float *P, float dl, float sg, const CamArgs &cam,
                                                  uint32_t hp, const float *A, const float *wsum,
                                                  float dx, float dy, float dz, double inv, float *G, float &gdelta,
                                                  float &gsigma, float &gopac)
{
    const int T = (int)(hp >> 28);
    float gdx = 0.f, gdy = 0.f, gdz = 0.f;
    sh_grad_dot(deg, dx, dy, dz, wsum, gdx, gdy, gdz);
    // unit direction -> centre:  (I - dir dir^T) / |centre - campos|, then / K per point
    const float dot = dx * gdx + dy * gdy + dz * gdz;
    const float sc = (float)inv / K;
    const float gcx = (gdx - dx * dot) * sc, gcy = (gdy - dy * dot) * sc, gcz = (gdz - dz * dot) * sc;

    const double r0 = cam.R[0], r1 = cam.R[1], r2 = cam.R[2], r3 = cam.R[3], r4 = cam.R[4], r5 = cam.R[5];
    const double r6 = cam.R[6], r7 = cam.R[7], r8 = cam.R[8];
    // the lines' origin: the hull's start vertex (first hull index) rounded to
    // whole pixels, with the forward pass's own projection arithmetic (so the
    // same integers)
    double ox, oy;
    {
        const int s0 = (int)(hp & 7u);
        const double x = P[3 * s0], y = P[3 * s0 + 1], z = P[3 * s0 + 2];
        const double X = r0 * x + r1 * y + r2 * z + (double)cam.t[0];
        const double Y = r3 * x + r4 * y + r5 * z + (double)cam.t[1];
        const double Z = r6 * x + r7 * y + r8 * z + (double)cam.t[2];
        ox = rint((double)cam.fx * X / Z + (double)cam.cx);
        oy = rint((double)cam.fy * Y / Z + (double)cam.cy);
    }
    // per point: projected position relative to the origin, 1/Z, X/Z, Y/Z
    float qx[K], qy[K], iz[K], xz[K], yz[K];
    double zs = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double x = P[3 * k], y = P[3 * k + 1], z = P[3 * k + 2];
        const double X = r0 * x + r1 * y + r2 * z + (double)cam.t[0];
        const double Y = r3 * x + r4 * y + r5 * z + (double)cam.t[1];
        const double Z = r6 * x + r7 * y + r8 * z + (double)cam.t[2];
        const double izd = 1.0 / Z;
        qx[k] = (float)((double)cam.fx * X * izd + (double)cam.cx - ox);
        qy[k] = (float)((double)cam.fy * Y * izd + (double)cam.cy - oy);
        iz[k] = (float)izd;
        xz[k] = (float)(X * izd);
        yz[k] = (float)(Y * izd);
        zs += Z;
    }
    const float dd = (float)(zs / K);
    const float dp = dd * dl;
    const float s2 = dp * (float)LOG2E;

    // hull vertices in order (relative to the origin)
    float vx[K], vy[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int v = (hp >> (3 * j)) & 7;
        vx[j] = 0.0f;
        vy[j] = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (k == v) { vx[j] = qx[k]; vy[j] = qy[k]; }
    }
    float gvx[K], gvy[K];
#pragma unroll
    for (int j = 0; j < K; ++j) { gvx[j] = 0.0f; gvy[j] = 0.0f; }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j >= T) continue;
        // edge j: vertex j -> vertex j+1 (mod T)
        float bxv = vx[0], byv = vy[0];
#pragma unroll
        for (int jj = 1; jj < K; ++jj)
            if (jj == j + 1 && jj < T) { bxv = vx[jj]; byv = vy[jj]; }
        const float ex = bxv - vx[j], ey = byv - vy[j];
        const float il = 1.0f / sqrtf(ex * ex + ey * ey);
        const float tx = ex * il, ty = ey * il;
        const float nA = ty, nB = -tx;
        // stored (a, b, c) = s2 * (A, B, C'), C' = -(A vx + B vy) in the origin's frame
        const float gA = s2 * A[j], gB = s2 * A[K + j], gC = s2 * A[2 * K + j];
        const float gAt = gA - gC * vx[j], gBt = gB - gC * vy[j];
        gvx[j] -= gC * nA;
        gvy[j] -= gC * nB;
        // n = (e_y, -e_x)/|e|  =>  dL/de = -((g_n . t)/|e|) n
        const float sdot = (gAt * tx + gBt * ty) * il;
        const float gex = -sdot * nA, gey = -sdot * nB;
        gvx[j] -= gex;
        gvy[j] -= gey;
#pragma unroll
        for (int jj = 0; jj < K; ++jj)
            if (jj == ((j + 1 == T) ? 0 : j + 1)) { gvx[jj] += gex; gvy[jj] += gey; }
    }
    // x2_j = delta' log2(e) L_j  =>  dx2_j / ddelta' = x2_j / delta'
    const float gdp = A[3 * K + 5] / dp;
    const float gsp = A[3 * K];
    gdelta += dd * gdp;
    gsigma += dd * gsp;
    gopac += A[3 * K + 1];
    const float gd = dl * gdp + sg * gsp;

    // hull vertices -> projected points
    float gqx[K], gqy[K];
#pragma unroll
    for (int k = 0; k < K; ++k) { gqx[k] = 0.0f; gqy[k] = 0.0f; }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j >= T) continue;
        const int v = (hp >> (3 * j)) & 7;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (k == v) { gqx[k] += gvx[j]; gqy[k] += gvy[j]; }
    }

    // projection and depth -> camera space -> world (R^T)
    const float fx = cam.fx, fy = cam.fy;
    const float R0 = cam.R[0], R1 = cam.R[1], R2 = cam.R[2], R3 = cam.R[3], R4 = cam.R[4], R5 = cam.R[5];
    const float R6 = cam.R[6], R7 = cam.R[7], R8 = cam.R[8];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const float gX = gqx[k] * fx * iz[k], gY = gqy[k] * fy * iz[k];
        const float gZ = -(gX * xz[k] + gY * yz[k]) + gd / K;
        const float o0 = R0 * gX + R3 * gY + R6 * gZ + gcx;
        const float o1 = R1 * gX + R4 * gY + R7 * gZ + gcy;
        const float o2 = R2 * gX + R5 * gY + R8 * gZ + gcz;
        G[3 * k + 0] = ADD ? G[3 * k + 0] + o0 : o0;
        G[3 * k + 1] = ADD ? G[3 * k + 1] + o1 : o1;
        G[3 * k + 2] = ADD ? G[3 * k + 2] + o2 : o2;
    }
}


// One view of a convex whose SH gradient row (in LDS) sums several views.
// D3 (degree 3): the convex's 48 coefficients arrive in registers (read once
// for all views); otherwise the thread reads its own coefficient row.
// A: the instance's accumulator row (in registers).
template <int K, bool D3, typename SP>
__device__ __forceinline__ void view_backward_rows(int deg, const float *P, float dl, float sg, const SP *f,
                                                   const float *fr, const CamArgs &cam, uint32_t hp, const float *A,
                                                   float *G, float &gdelta, float &gsigma, float &gopac, float *gsh)
{
    float dx, dy, dz, Yb[16];
    double inv;
    view_dir<K>(deg, P, cam, dx, dy, dz, inv, Yb);
    float gr[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) gr[c] = ((hp >> (24 + c)) & 1u) ? 0.0f : A[3 * K + 2 + c];
    float wsum[16];
    if constexpr (D3) {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            wsum[c] = gr[0] * fr[3 * c] + gr[1] * fr[3 * c + 1] + gr[2] * fr[3 * c + 2];
#pragma unroll
            for (int t = 0; t < 3; ++t) gsh[3 * c + t] += gr[t] * Yb[c];
        }
    } else {
        const int nc = (deg + 1) * (deg + 1);
        for (int c = 0; c < nc; ++c) {
            const float f0 = ld(f, 3 * c + 0), f1 = ld(f, 3 * c + 1), f2 = ld(f, 3 * c + 2);
            wsum[c] = gr[0] * f0 + gr[1] * f1 + gr[2] * f2;
            gsh[3 * c + 0] += gr[0] * Yb[c];
            gsh[3 * c + 1] += gr[1] * Yb[c];
            gsh[3 * c + 2] += gr[2] * Yb[c];
        }
    }
    geometry_backward<K, true>(deg, P, dl, sg, cam, hp, A, wsum, dx, dy, dz, inv, G, gdelta, gsigma, gopac);
}

// The views of one convex (several views): the next view's packed hull word
// and accumulator row are loaded while the current view is worked on.
template <int K, bool D3, typename SP>
__device__ __forceinline__ void views_backward(int n, int i, int nviews, int deg, const float *P, float dl, float sg,
                                               const SP *f, const float *fr, const ViewDesc *views,
                                               const uint32_t *__restrict__ hullpk, const float *__restrict__ acc,
                                               float *G, float &gdelta, float &gsigma, float &gopac, float *gsh)
{
    uint32_t hp = hullpk[i];
    float A[acc_stride(K)];
    load_acc_row<K>(acc + (size_t)i * acc_stride(K), A);
    for (int v = 0; v < nviews; ++v) {
        const int vn = min(v + 1, nviews - 1); // the last view reloads itself (unused)
        const size_t instn = (size_t)vn * n + i;
        const uint32_t hpn = hullpk[instn];
        float An[acc_stride(K)];
        load_acc_row<K>(acc + instn * acc_stride(K), An);
        if ((int)(hp >> 28) >= 3) // else dropped in this view: no gradient
            view_backward_rows<K, D3>(deg, P, dl, sg, f, fr, views[v].cam, hp, A, G, gdelta, gsigma, gopac, gsh);
        hp = hpn;
#pragma unroll
        for (int q = 0; q < acc_stride(K); ++q) A[q] = An[q];
    }
}

constexpr int PB_BLOCK = 128;
constexpr int PB_SH_STRIDE = 49; // odd LDS row stride: per-thread rows conflict-free
// Block-cooperative, coalesced copy of LDS rows of stride S into a
// contiguous global run of `rows` rows of W floats.
template <int W, int S> __device__ __forceinline__ void rows_from_lds(float *g, const float *lds, int rows)
{
    for (int j = threadIdx.x; j < rows * W; j += PB_BLOCK) g[j] = lds[(j / W) * S + j % W];
}
// One thread per convex, 128 convexes per workgroup.  Points arrive and their
// gradients leave through LDS as coalesced rows (the point gradients are
// summed over the views in LDS).
// One view (MV false): the SH work runs block-cooperatively on (convex,
// coefficient) items, so the coefficient rows are read and their gradient
// rows written as contiguous runs: each thread puts its direction's basis
// values and its colour gradient in LDS, the items read the three channels
// of one coefficient, store their gradients and leave wsum_c in place of the
// basis value, and each thread finishes its convex's geometry.
// Several views (MV true): each thread adds its views into its LDS gradient
// row, which leaves as coalesced rows at the end.
template <int K, typename P, bool MV>
__global__ __launch_bounds__(PB_BLOCK) __attribute__((amdgpu_waves_per_eu(MV || K > 6 ? 1 : 4))) void preprocess_bwd_kernel(
    int n, int nviews, int deg, const P *__restrict__ points, const P *__restrict__ delta,
    const P *__restrict__ sigma, const P *__restrict__ sh, const FrameHeader *__restrict__ frame,
    const uint32_t *__restrict__ hullpk, const float *__restrict__ acc,
    float *__restrict__ g_points, float *__restrict__ g_delta, float *__restrict__ g_sigma,
    float *__restrict__ g_opacity, float *__restrict__ g_sh)
{
    constexpr int PS = 3 * K + 1;
    constexpr int YS = 17; // odd LDS row stride of the basis values / wsum
    __shared__ float s_pts[PB_BLOCK * PS];
    // point gradients: summed over the views apart (MV); with one view each
    // thread overwrites its own point row once it has read it
    __shared__ float s_gpv[MV ? PB_BLOCK * PS : 1];
    float *s_gp = MV ? s_gpv : s_pts;
    __shared__ float s_gsh[MV ? PB_BLOCK * PB_SH_STRIDE : PB_BLOCK * YS];
    __shared__ float s_gr[MV ? 1 : PB_BLOCK * 3];
    const int base = blockIdx.x * PB_BLOCK;
    const int cnt = min(PB_BLOCK, n - base);
    const int tid = threadIdx.x;
    const int nc = (deg + 1) * (deg + 1);
    stage_rows<PB_BLOCK, 3 * K>(s_pts, points + (size_t)base * 3 * K, cnt, 3 * K, PS);
    if constexpr (MV) {
#pragma unroll
        for (int k = 0; k < 3 * K; ++k) s_gp[tid * PS + k] = 0.0f;
        for (int j = tid; j < PB_BLOCK * PB_SH_STRIDE; j += PB_BLOCK) s_gsh[j] = 0.0f;
    }
    __syncthreads();

    const int i = base + tid;
    const ViewDesc *views = reinterpret_cast<const ViewDesc *>(frame + 1);
    if constexpr (MV) {
        if (tid < cnt) {
            float gdelta = 0.0f, gsigma = 0.0f, gopac = 0.0f;
            const float dl = ld(delta, i), sg = ld(sigma, i);
            const P *f = sh + (size_t)i * 3 * nc;
            if (deg == 3) {
                float fr[48];
#pragma unroll
                for (int q = 0; q < 12; ++q) {
                    const float4 w = ld4(f, q);
                    fr[4 * q] = w.x; fr[4 * q + 1] = w.y; fr[4 * q + 2] = w.z; fr[4 * q + 3] = w.w;
                }
                views_backward<K, true>(n, i, nviews, deg, &s_pts[tid * PS], dl, sg, f, fr, views, hullpk, acc,
                                        &s_gp[tid * PS], gdelta, gsigma, gopac, &s_gsh[tid * PB_SH_STRIDE]);
            } else {
                views_backward<K, false>(n, i, nviews, deg, &s_pts[tid * PS], dl, sg, f, nullptr, views, hullpk,
                                         acc, &s_gp[tid * PS], gdelta, gsigma, gopac, &s_gsh[tid * PB_SH_STRIDE]);
            }
            g_delta[i] = gdelta;
            g_sigma[i] = gsigma;
            g_opacity[i] = gopac;
        }
        __syncthreads();
        float *g = g_sh + (size_t)base * 3 * nc;
        for (int j = tid; j < cnt * 3 * nc; j += PB_BLOCK) g[j] = s_gsh[(j / (3 * nc)) * PB_SH_STRIDE + j % (3 * nc)];
    } else {
        const CamArgs &cam = views[0].cam;
        const uint32_t hp = tid < cnt ? hullpk[i] : 0u;
        const bool live = (int)(hp >> 28) >= 3; // dropped (or past n): no gradient
        const float *Ag = acc + (size_t)i * acc_stride(K);
        float dx = 0.f, dy = 0.f, dz = 0.f, Yb[16];
        double inv = 0.0;
        // the accumulator row, read once and held until the geometry step (a
        // second read after the SH phase would find it evicted)
        float A[acc_stride(K)];
        if (live) {
            load_acc_row<K>(Ag, A);
            view_dir<K>(deg, &s_pts[tid * PS], cam, dx, dy, dz, inv, Yb);
            for (int c = 0; c < nc; ++c) s_gsh[tid * YS + c] = Yb[c];
#pragma unroll
            for (int c = 0; c < 3; ++c) s_gr[tid * 3 + c] = ((hp >> (24 + c)) & 1u) ? 0.0f : A[3 * K + 2 + c];
        } else {
            for (int c = 0; c < nc; ++c) s_gsh[tid * YS + c] = 0.0f;
#pragma unroll
            for (int c = 0; c < 3; ++c) s_gr[tid * 3 + c] = 0.0f;
        }
        __syncthreads();
        {
            // U items per thread in flight (their loads issued together)
            constexpr int U = 4;
            const P *f = sh + (size_t)base * 3 * nc;
            float *g = g_sh + (size_t)base * 3 * nc;
            const int total = cnt * nc;
            const int drow = PB_BLOCK / nc, dc = PB_BLOCK - drow * nc;
            int row = tid / nc, c = tid - row * nc;
            for (int j0 = tid; j0 < total; j0 += U * PB_BLOCK) {
                float fv[U][3];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    // 16-bit loads unconditional (a clamped index): guarded, they
                    // compile to a branch and a wait each; float32 loads are
                    // predicated and issue back to back either way
                    const int j = j0 + u * PB_BLOCK, jc = min(j, total - 1);
#pragma unroll
                    for (int t = 0; t < 3; ++t)
                        fv[u][t] = sizeof(P) == 4 ? (j < total ? ld(f, 3 * j + t) : 0.0f) : ld(f, 3 * jc + t);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int j = j0 + u * PB_BLOCK;
                    if (j < total) {
                        const float gr0 = s_gr[row * 3], gr1 = s_gr[row * 3 + 1], gr2 = s_gr[row * 3 + 2];
                        const float y = s_gsh[row * YS + c];
                        g[3 * j] = gr0 * y;
                        g[3 * j + 1] = gr1 * y;
                        g[3 * j + 2] = gr2 * y;
                        s_gsh[row * YS + c] = gr0 * fv[u][0] + gr1 * fv[u][1] + gr2 * fv[u][2];
                    }
                    row += drow;
                    c += dc;
                    if (c >= nc) { c -= nc; ++row; }
                }
            }
        }
        __syncthreads();
        if (tid < cnt) {
            float gdelta = 0.0f, gsigma = 0.0f, gopac = 0.0f;
            if (live) {
                float wsum[16];
                for (int c = 0; c < nc; ++c) wsum[c] = s_gsh[tid * YS + c];
                geometry_backward<K, false>(deg, &s_pts[tid * PS], ld(delta, i), ld(sigma, i), cam, hp, A, wsum,
                                            dx, dy, dz, inv, &s_pts[tid * PS], gdelta, gsigma, gopac);
            } else {
#pragma unroll
                for (int k = 0; k < 3 * K; ++k) s_pts[tid * PS + k] = 0.0f;
            }
            g_delta[i] = gdelta;
            g_sigma[i] = gsigma;
            g_opacity[i] = gopac;
        }
    }
    __syncthreads();
    rows_from_lds<3 * K, PS>(g_points + (size_t)base * 3 * K, s_gp, cnt);
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

#define CS_DISPATCH_P(DT, ...)                                                                                     \
    switch (DT) {                                                                                                  \
    case CS_DTYPE_F32: { using PP = float; __VA_ARGS__; } break;                                                   \
    case CS_DTYPE_F16: { using PP = Half; __VA_ARGS__; } break;                                                    \
    case CS_DTYPE_BF16: { using PP = BHalf; __VA_ARGS__; } break;                                                  \
    default: break;                                                                                                \
    }

void launch_preprocess_fwd(hipStream_t st, int n, int nviews, int K, int deg, int dtype, const void *points,
                           const void *delta, const void *sigma, const void *opacity, const void *sh,
                           const FrameHeader *views, const RenderArgs &ra, uint8_t *records, uint32_t *keys,
                           uint32_t *ids, uint4 *bins, uint32_t *hullpk, DebugConvex *dbg, const ZeroSpans &zero)
{
    if (n <= 0 || nviews <= 0) return;
    dim3 grid((n + PF_BLOCK - 1) / PF_BLOCK, nviews), block(PF_BLOCK);
    if (dbg)
        CS_DISPATCH_P(dtype, CS_DISPATCH_K(K, hipLaunchKernelGGL((preprocess_fwd_kernel<KK, true, PP>), grid, block, 0, st, n,
                                                             deg, (const PP *)points, (const PP *)delta,
                                                             (const PP *)sigma, (const PP *)opacity, (const PP *)sh,
                                                             views, ra, records, keys, ids, bins, hullpk, dbg, zero)))
    else
        CS_DISPATCH_P(dtype, CS_DISPATCH_K(K, hipLaunchKernelGGL((preprocess_fwd_kernel<KK, false, PP>), grid, block, 0, st,
                                                             n, deg, (const PP *)points, (const PP *)delta,
                                                             (const PP *)sigma, (const PP *)opacity, (const PP *)sh,
                                                             views, ra, records, keys, ids, bins, hullpk, dbg, zero)))
}

void launch_preprocess_bwd(hipStream_t st, int n, int nviews, int K, int deg, int dtype, const void *points,
                           const void *delta, const void *sigma, const void *sh, const FrameHeader *views,
                           const uint32_t *hullpk, const float *acc, float *g_points, float *g_delta,
                           float *g_sigma, float *g_opacity, float *g_sh)
{
    if (n <= 0) return;
    dim3 grid((n + PB_BLOCK - 1) / PB_BLOCK), block(PB_BLOCK);
    if (nviews > 1)
        CS_DISPATCH_P(dtype, CS_DISPATCH_K(K, hipLaunchKernelGGL((preprocess_bwd_kernel<KK, PP, true>), grid, block, 0,
                                                             st, n, nviews, deg, (const PP *)points,
                                                             (const PP *)delta, (const PP *)sigma, (const PP *)sh,
                                                             views, hullpk, acc, g_points, g_delta, g_sigma,
                                                             g_opacity, g_sh)))
    else
        CS_DISPATCH_P(dtype, CS_DISPATCH_K(K, hipLaunchKernelGGL((preprocess_bwd_kernel<KK, PP, false>), grid, block, 0,
                                                             st, n, nviews, deg, (const PP *)points,
                                                             (const PP *)delta, (const PP *)sigma, (const PP *)sh,
                                                             views, hullpk, acc, g_points, g_delta, g_sigma,
                                                             g_opacity, g_sh)))
}

} // namespace cs
