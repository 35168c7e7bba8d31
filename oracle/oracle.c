/*
 * FP64 CPU oracle of the smooth-convex rasterizer (3D Convex Splatting,
 * Held et al., CVPR 2025).  TEST INFRASTRUCTURE ONLY: only tests, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code
 * with the HIP library.
 *
 * The definitions followed, by section / equation of the paper:
 *   Sec. 3.1 Eq. signed_distance   L_j(p) = n_j . p + d_j, outward unit normal
 *   Sec. 3.1 Eq. smoothness        phi = log sum_j exp(delta L_j)
 *   Sec. 3.1 Eq. sharpness         I = Sigmoid(-sigma phi)
 *   Sec. 3.2 Eq. projection        q_k = K (R p_k + t)
 *   Sec. 3.2 "2D convex hull"      the hull of the projected points
 *   Sec. 3.2 "2D indicator" + Supp. B (Eq. smoothness_supp / sharpness_supp)
 *                                  delta and sigma scaled by the distance d
 *   Sec. 3.2 compositing equation  C = sum_n c_n o_n I_n prod_{i<n} (1 - o_i I_i),
 *                                  convexes ordered by increasing distance
 *   Sec. 3.2 / Sec. 4              colour c_n from degree-3 spherical harmonics
 *   Sec. 3.3                       optimised parameters: points, delta, sigma,
 *                                  opacity, SH -> the backward pass below
 *
 * Readings where the paper is silent, ambiguous or garbled (each applied once):
 *   R1  Eq. projection leaves the homogeneous divide implicit: q = (fx X/Z + cx,
 *       fy Y/Z + cy), in pixel units.  Pixel (u, v) is sampled at (u+.5, v+.5).
 *   R2  L_j are signed distances with unit normals, in pixels.
 *   R3  d ("distance" of Supp. B) = camera-space depth of the point centroid,
 *       d = (1/K) sum_k Z_k, and it carries gradient to every point.
 *   R4  "increasing distance to their centres": ascending pinned float32 key
 *       key = (((Z0 + Z1) + Z2) + ...), Z_k = fmaf(R20, x, fmaf(R21, y,
 *       fmaf(R22, z, t_z))) in float32 from the float32 inputs; ties by index.
 *   R5  a convex with any float32 Z_k <= znear is dropped (not in the paper).
 *   R6  strict hull: collinear boundary points are not vertices (the scan of
 *       Sec. 3.2 keeps them only when the cross product is exactly zero, which
 *       generic inputs never produce); fewer than 3 vertices drops the convex.
 *   R7  hull order: positive orientation, orient(a,b,c) = (b-a) x (c-a) > 0 for
 *       every other point c, starting at the vertex with smallest (y, x).
 *   R8  colour c = max(0, 0.5 + sum_lm Y_lm(dir) f_lm) per channel, real
 *       orthonormal SH (Condon-Shortley phase kept in the complex SH),
 *       dir = unit(centre - camera position), centre = mean of the K points;
 *       the clamp passes gradient only where 0.5 + sum > 0.
 *   R9  background colour bg is added with the final transmittance.
 *   R10 "matched" mode: a pair with alpha < eps_alpha is skipped, and the walk
 *       stops after the convex that brings T below t_min.  "exact" mode keeps
 *       every pair down to alpha >= 1e-15 and never stops early.
 *   R11 1 - alpha is evaluated as (1 - o) + o (1 - I), with 1 - I from the
 *       sign-split logistic, so an opaque convex keeps full relative accuracy.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

#define PI 3.14159265358979323846
#define EXACT_ALPHA 1e-15
#define NACC (3 * ORC_MAXK + 6) /* per-convex: nx[8] ny[8] off[8] dp sp o rgb[3] */

/* ------------------------------------------------------------------ SH ---- */

static double fact(int n) { double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }
static double choose(int n, int k) { return fact(n) / (fact(k) * fact(n - k)); }

/* m-th derivative of the Legendre polynomial P_l at z, from the explicit sum
 * P_l(z) = 2^-l sum_k (-1)^k C(l,k) C(2l-2k, l) z^(l-2k). */
static double legendre_deriv(int l, int m, double z)
{
    double s = 0.0;
    for (int k = 0; 2 * k <= l; ++k) {
        int p = l - 2 * k;
        if (p < m) continue;
        double c = ((k & 1) ? -1.0 : 1.0) * choose(l, k) * choose(2 * l - 2 * k, l) / pow(2.0, l);
        s += c * (fact(p) / fact(p - m)) * pow(z, p - m);
    }
    return s;
}

/* Sum of the absolute values of the monomials of legendre_deriv at z. */
static double legendre_deriv_magnitude(int l, int m, double z)
{
    double s = 0.0;
    for (int k = 0; 2 * k <= l; ++k) {
        int p = l - 2 * k;
        if (p < m) continue;
        s += choose(l, k) * choose(2 * l - 2 * k, l) / pow(2.0, l) * (fact(p) / fact(p - m)) * pow(fabs(z), p - m);
    }
    return s;
}

/* (x + i y)^m */
static void cpow_xy(double x, double y, int m, double *re, double *im)
{
    double r = 1.0, i = 0.0;
    for (int k = 0; k < m; ++k) { double nr = r * x - i * y; i = r * y + i * x; r = nr; }
    *re = r; *im = i;
}

/* Complex SH with the Condon-Shortley phase on the unit sphere:
 *   Y_l^m = N_lm (-1)^m P_l^(m)(z) (x + i y)^m,  m >= 0,
 * real basis: m > 0 -> sqrt2 Re Y_l^m, m = 0 -> Y_l^0, m < 0 -> sqrt2 Im Y_l^|m|.
 * dY is the gradient of that polynomial in (x, y, z). */
void orc_sh_basis(int deg, const double *dir, double *Y, double *dY)
{
    double x = dir[0], y = dir[1], z = dir[2];
    int idx = 0;
    for (int l = 0; l <= deg; ++l) {
        for (int m = -l; m <= l; ++m, ++idx) {
            int am = m < 0 ? -m : m;
            double N = sqrt((2.0 * l + 1.0) / (4.0 * PI) * fact(l - am) / fact(l + am));
            double P = legendre_deriv(l, am, z);
            double dP = legendre_deriv(l, am + 1, z);
            double re, im, re1 = 0, im1 = 0;
            cpow_xy(x, y, am, &re, &im);
            if (am >= 1) cpow_xy(x, y, am - 1, &re1, &im1);
            double sg = (am & 1) ? -1.0 : 1.0;
            double g[3];
            if (m == 0) {
                Y[idx] = N * P;
                g[0] = 0; g[1] = 0; g[2] = N * dP;
            } else if (m > 0) {
                double f = sqrt(2.0) * N * sg;
                Y[idx] = f * P * re;
                g[0] = f * P * am * re1; g[1] = -f * P * am * im1; g[2] = f * dP * re;
            } else {
                double f = sqrt(2.0) * N * sg;
                Y[idx] = f * P * im;
                g[0] = f * P * am * im1; g[1] = f * P * am * re1; g[2] = f * dP * im;
            }
            if (dY) { dY[3 * idx] = g[0]; dY[3 * idx + 1] = g[1]; dY[3 * idx + 2] = g[2]; }
        }
    }
}

/* Per basis function of orc_sh_basis, a bound on the sum of the absolute
 * values of the monomials of its polynomial in (x, y, z) (exact for each of
 * the two factors, the Legendre part and Re / Im (x + i y)^m): the scale of its rounding error
 * near a nodal line, where the value itself cancels to zero.  Exact for the
 * single-monomial functions of degree <= 1. */
static void sh_basis_magnitude(int deg, const double *dir, double *Ym)
{
    double ax = fabs(dir[0]), ay = fabs(dir[1]), z = dir[2];
    int idx = 0;
    for (int l = 0; l <= deg; ++l)
        for (int m = -l; m <= l; ++m, ++idx) {
            int am = m < 0 ? -m : m;
            double N = sqrt((2.0 * l + 1.0) / (4.0 * PI) * fact(l - am) / fact(l + am));
            double f = m == 0 ? N : sqrt(2.0) * N;
            /* |monomials| of Re (x + i y)^m: even powers of y; of Im: odd ones */
            double pp = pow(ax + ay, am), pm = pow(ax - ay, am);
            double xy = m >= 0 ? 0.5 * (pp + pm) : 0.5 * (pp - pm);
            Ym[idx] = f * legendre_deriv_magnitude(l, am, z) * xy;
        }
}

/* ----------------------------------------------------------- preprocess --- */

static double orient(const double *a, const double *b, const double *c)
{
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]);
}

/* Pinned float32 depth key (R4); also the float32 depths used by the near cull. */
static uint32_t depth_key(const double *p, int k, const double *cam, float *z32)
{
    float r20 = (float)cam[12], r21 = (float)cam[13], r22 = (float)cam[14], tz = (float)cam[17];
    float sum = 0.0f;
    for (int i = 0; i < k; ++i) {
        float x = (float)p[3 * i], y = (float)p[3 * i + 1], z = (float)p[3 * i + 2];
        float zi = fmaf(r20, x, fmaf(r21, y, fmaf(r22, z, tz)));
        z32[i] = zi;
        sum = (i == 0) ? zi : sum + zi;
    }
    uint32_t bits;
    memcpy(&bits, &sum, 4);
    return bits;
}

static void preprocess_one(const orc_scene *s, const double *cam, double rect_alpha, int n, orc_convex *c)
{
    memset(c, 0, sizeof(*c));
    const int K = s->k;
    const double *p = s->points + (size_t)n * K * 3;
    const double *R = cam + 6, *t = cam + 15;
    const double fx = cam[2], fy = cam[3], cx = cam[4], cy = cam[5], znear = cam[18];

    float z32[ORC_MAXK];
    c->key = depth_key(p, K, cam, z32);
    for (int k = 0; k < K; ++k)
        if (z32[k] <= (float)znear) { c->status = ORC_CULL_NEAR; return; }

    /* Eq. projection (R1) */
    for (int k = 0; k < K; ++k) {
        for (int r = 0; r < 3; ++r)
            c->X[k][r] = R[3 * r] * p[3 * k] + R[3 * r + 1] * p[3 * k + 1] + R[3 * r + 2] * p[3 * k + 2] + t[r];
        c->q[k][0] = fx * c->X[k][0] / c->X[k][2] + cx;
        c->q[k][1] = fy * c->X[k][1] / c->X[k][2] + cy;
    }

    /* near-collinear triples make the hull ill-posed: flag them */
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j)
            for (int k = 0; k < K; ++k) {
                if (i == j || j == k || i == k) continue;
                double la = hypot(c->q[j][0] - c->q[i][0], c->q[j][1] - c->q[i][1]);
                double lb = hypot(c->q[k][0] - c->q[i][0], c->q[k][1] - c->q[i][1]);
                double o = orient(c->q[i], c->q[j], c->q[k]);
                if (!(fabs(o) >= 1e-9 * la * lb) || la == 0.0 || lb == 0.0) c->status |= ORC_DEGENERATE;
            }

    /* brute-force hull (R6, R7): i -> j is an edge iff every other point lies
     * strictly left of it */
    int nxt[ORC_MAXK];
    for (int i = 0; i < K; ++i) {
        nxt[i] = -1;
        for (int j = 0; j < K; ++j) {
            if (j == i) continue;
            int ok = 1;
            for (int k = 0; k < K && ok; ++k)
                if (k != i && k != j && !(orient(c->q[i], c->q[j], c->q[k]) > 0.0)) ok = 0;
            if (ok) { if (nxt[i] >= 0) c->status |= ORC_DEGENERATE; nxt[i] = j; }
        }
    }
    int start = -1, nverts = 0;
    for (int i = 0; i < K; ++i) {
        if (nxt[i] < 0) continue;
        ++nverts;
        if (start < 0 || c->q[i][1] < c->q[start][1] ||
            (c->q[i][1] == c->q[start][1] && c->q[i][0] < c->q[start][0]))
            start = i;
    }
    int T = 0;
    if (start >= 0) {
        int v = start;
        do {
            if (T >= K || v < 0) { T = 0; break; }
            c->hull[T++] = v;
            v = nxt[v];
        } while (v != start);
    }
    if (T != nverts) { c->status |= ORC_DEGENERATE; T = T < nverts ? T : nverts; }
    c->T = T;
    if (T < 3) { c->status = (c->status & ORC_DEGENERATE) | ORC_CULL_HULL; return; }

    /* Eq. signed_distance in 2D: outward unit normal of each hull edge (R2) */
    for (int j = 0; j < T; ++j) {
        const double *a = c->q[c->hull[j]], *b = c->q[c->hull[(j + 1) % T]];
        double ex = b[0] - a[0], ey = b[1] - a[1], l = hypot(ex, ey);
        c->nx[j] = ey / l;
        c->ny[j] = -ex / l;
        c->off[j] = -(c->nx[j] * a[0] + c->ny[j] * a[1]);
    }

    /* Supp. B: distance scaling (R3) */
    double zs = 0.0;
    for (int k = 0; k < K; ++k) zs += c->X[k][2];
    c->d = zs / K;
    c->dp = c->d * s->delta[n];
    c->sp = c->d * s->sigma[n];

    /* colour (R8) */
    double ctr[3] = {0, 0, 0}, campos[3];
    for (int k = 0; k < K; ++k) for (int r = 0; r < 3; ++r) ctr[r] += p[3 * k + r];
    for (int r = 0; r < 3; ++r) ctr[r] /= K;
    for (int r = 0; r < 3; ++r) campos[r] = -(R[r] * t[0] + R[3 + r] * t[1] + R[6 + r] * t[2]);
    double v[3] = {ctr[0] - campos[0], ctr[1] - campos[1], ctr[2] - campos[2]};
    c->camdist = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int r = 0; r < 3; ++r) c->dir[r] = v[r] / c->camdist;
    double Y[16];
    orc_sh_basis(s->deg, c->dir, Y, NULL);
    const int nc = (s->deg + 1) * (s->deg + 1);
    const double *sh = s->sh + (size_t)n * nc * 3;
    for (int ch = 0; ch < 3; ++ch) {
        double raw = 0.5;
        for (int i = 0; i < nc; ++i) raw += Y[i] * sh[3 * i + ch];
        if (raw > 0.0) c->rgb[ch] = raw;
        else { c->rgb[ch] = 0.0; c->clampmask |= 1 << ch; }
    }

    /* Region where alpha can reach rect_alpha.  phi >= delta' max_j L_j (LSE is
     * at least its largest term), and alpha >= a needs sigma' phi <= ln(o/a - 1),
     * so every L_j <= r = ln(o/a - 1) / (sigma' delta'): the hull pushed out by
     * r, whose corners are the intersections of neighbouring shifted lines. */
    double o = s->opacity[n];
    if (!(o > rect_alpha)) {
        c->rect[0] = 1; c->rect[1] = 1; c->rect[2] = 0; c->rect[3] = 0;
        return;
    }
    double r = log(o / rect_alpha - 1.0) / (c->sp * c->dp);
    double xmin = INFINITY, ymin = INFINITY, xmax = -INFINITY, ymax = -INFINITY;
    if (r <= 0.0) {
        for (int j = 0; j < T; ++j) {
            const double *a = c->q[c->hull[j]];
            xmin = fmin(xmin, a[0]); xmax = fmax(xmax, a[0]);
            ymin = fmin(ymin, a[1]); ymax = fmax(ymax, a[1]);
        }
    } else {
        for (int j = 0; j < T; ++j) {
            int i = (j + T - 1) % T;
            double det = c->nx[i] * c->ny[j] - c->ny[i] * c->nx[j];
            if (fabs(det) < 1e-12) { xmin = ymin = -1e30; xmax = ymax = 1e30; break; }
            double bi = r - c->off[i], bj = r - c->off[j];
            double px = (bi * c->ny[j] - bj * c->ny[i]) / det;
            double py = (c->nx[i] * bj - c->nx[j] * bi) / det;
            xmin = fmin(xmin, px); xmax = fmax(xmax, px);
            ymin = fmin(ymin, py); ymax = fmax(ymax, py);
        }
    }
    double mg = 1e-6;
    c->rect[0] = xmin - mg - 1e-12 * fabs(xmin);
    c->rect[1] = ymin - mg - 1e-12 * fabs(ymin);
    c->rect[2] = xmax + mg + 1e-12 * fabs(xmax);
    c->rect[3] = ymax + mg + 1e-12 * fabs(ymax);
}

int orc_preprocess(const orc_scene *s, const double *cam, double rect_alpha, orc_convex *out)
{
    if (!s || !cam || !out || s->k < 3 || s->k > ORC_MAXK || s->deg < 0 || s->deg > 3) return -1;
#pragma omp parallel for schedule(static)
    for (int n = 0; n < s->n; ++n) preprocess_one(s, cam, rect_alpha, n, &out[n]);
    return 0;
}

/* ----------------------------------------------------------------- order --- */

static const orc_convex *g_sort_cv;
static int cmp_order(const void *a, const void *b)
{
    int32_t i = *(const int32_t *)a, j = *(const int32_t *)b;
    uint32_t ki = g_sort_cv[i].key, kj = g_sort_cv[j].key;
    if (ki != kj) return ki < kj ? -1 : 1;
    return i < j ? -1 : (i > j);
}

int orc_order(int n, const orc_convex *cv, int32_t *order)
{
    int m = 0;
    for (int i = 0; i < n; ++i)
        if ((cv[i].status & 0xff) == ORC_VISIBLE) order[m++] = i;
    g_sort_cv = cv; /* qsort has no context argument; the oracle orders serially */
    qsort(order, m, sizeof(int32_t), cmp_order);
    return m;
}

/* ------------------------------------------------------------ per pixel --- */

typedef struct {
    double L[ORC_MAXK], x[ORC_MAXK], w[ORC_MAXK];
    double phi, xmax, lsum, I, omI, alpha, oma; /* phi = xmax + lsum */
} pair_eval;

/* Eqs. smoothness/sharpness with distance scaling (Supp. B) at pixel point q */
static void eval_pair(const orc_convex *c, double o, double qx, double qy, pair_eval *e)
{
    double m = -INFINITY;
    for (int j = 0; j < c->T; ++j) {
        e->L[j] = c->nx[j] * qx + c->ny[j] * qy + c->off[j];
        e->x[j] = c->dp * e->L[j];
        if (e->x[j] > m) m = e->x[j];
    }
    double sum = 0.0;
    for (int j = 0; j < c->T; ++j) { e->w[j] = exp(e->x[j] - m); sum += e->w[j]; }
    for (int j = 0; j < c->T; ++j) e->w[j] /= sum;
    e->xmax = m;
    e->lsum = log(sum);
    e->phi = m + e->lsum;
    double z = c->sp * e->phi; /* I = Sigmoid(-z) */
    if (z >= 0.0) { double ez = exp(-z); e->I = ez / (1.0 + ez); e->omI = 1.0 / (1.0 + ez); }
    else          { double ez = exp(z);  e->I = 1.0 / (1.0 + ez); e->omI = ez / (1.0 + ez); }
    e->alpha = o * e->I;
    e->oma = (1.0 - o) + o * e->omI; /* R11 */
}

/* A listed pair of a pixel: CON_IN when it is a term of the compositing sum;
 * CON_AMB when its skip or stop decision lies within the relative band tau of
 * the threshold, so that an evaluation in another precision may take it the
 * other way. */
#define CON_IN 1
#define CON_AMB 2
typedef struct {
    int32_t idx, flags;
    double T;
} contrib;

typedef struct {
    const orc_scene *s;
    const orc_convex *cv;
    const int32_t *order;
    int nvis;
    double eps, tmin, bg[3], tau;
    int matched;
} frame;

static void list_push(contrib **list, int *cap, int n, int idx, int flags, double T)
{
    if (n == *cap) { *cap = *cap ? 2 * *cap : 64; *list = realloc(*list, (size_t)*cap * sizeof(contrib)); }
    (*list)[n].idx = idx;
    (*list)[n].flags = flags;
    (*list)[n].T = T;
}

/* Compositing equation for one pixel; optionally lists the contributors.
 * With f->tau > 0 (matched mode) the list also holds the pairs whose decision
 * is ambiguous at relative precision tau: alpha within tau of eps (taken or
 * not), and, once T comes within tau of t_min, every later pair until T is
 * below t_min (1 - tau) for certain.  Those past the walk's own end are listed
 * without CON_IN and change neither C nor the returned T. */
static int pixel_forward(const frame *f, double qx, double qy, double *C, double *Tout,
                         contrib **list, int *cap)
{
    const double thr = f->matched ? f->eps : EXACT_ALPHA;
    const double tau = f->matched ? f->tau : 0.0;
    double T = 1.0, Tend = 1.0;
    C[0] = C[1] = C[2] = 0.0;
    int nl = 0, stopped = 0, tail = 0;
    pair_eval e;
    for (int a = 0; a < f->nvis; ++a) {
        int idx = f->order[a];
        const orc_convex *c = &f->cv[idx];
        if (qx < c->rect[0] || qx > c->rect[2] || qy < c->rect[1] || qy > c->rect[3]) continue;
        eval_pair(c, f->s->opacity[idx], qx, qy, &e);
        int taken = e.alpha >= thr;
        int amb = tau > 0.0 && ((e.alpha >= thr * (1.0 - tau) && e.alpha < thr * (1.0 + tau)) ||
                                (tail && e.alpha >= thr * (1.0 - tau)));
        int in = taken && !stopped;
        if (!in && !amb) continue;
        if (in)
            for (int ch = 0; ch < 3; ++ch) C[ch] += T * e.alpha * c->rgb[ch];
        if (list) list_push(list, cap, nl, idx, (in ? CON_IN : 0) | (amb ? CON_AMB : 0), T);
        ++nl;
        if (!taken) continue; /* an ambiguous skip leaves T as it is */
        T *= e.oma;
        if (!stopped && f->matched && T < f->tmin) { stopped = 1; Tend = T; }
        if (tau > 0.0) tail = T < f->tmin * (1.0 + tau) && T >= f->tmin * (1.0 - tau);
        if (stopped && !tail) break;
    }
    if (!stopped) Tend = T;
    for (int ch = 0; ch < 3; ++ch) C[ch] += Tend * f->bg[ch];
    *Tout = Tend;
    return nl;
}

static int setup_frame(const orc_scene *s, const double *cam, const double *par, double tau, frame *f,
                       orc_convex **cv, int32_t **order)
{
    if (!s || !cam || !par || s->k < 3 || s->k > ORC_MAXK || s->deg < 0 || s->deg > 3) return -1;
    f->s = s;
    f->eps = par[0];
    f->tmin = par[1];
    f->bg[0] = par[2]; f->bg[1] = par[3]; f->bg[2] = par[4];
    f->matched = par[5] != 0.0;
    f->tau = tau;
    *cv = (orc_convex *)malloc((size_t)(s->n > 0 ? s->n : 1) * sizeof(orc_convex));
    *order = (int32_t *)malloc((size_t)(s->n > 0 ? s->n : 1) * sizeof(int32_t));
    orc_preprocess(s, cam, f->matched ? f->eps * (1.0 - tau) : EXACT_ALPHA, *cv);
    f->cv = *cv;
    f->nvis = orc_order(s->n, *cv, *order);
    f->order = *order;
    return 0;
}

int orc_render(const orc_scene *s, const double *cam, const double *par, int npix, const int32_t *pix,
               double *out_rgb, double *out_T, int32_t *out_n)
{
    frame f;
    orc_convex *cv;
    int32_t *order;
    if (setup_frame(s, cam, par, 0.0, &f, &cv, &order)) return -1;
    const int W = (int)cam[0];
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < npix; ++i) {
        int u = pix ? pix[2 * i] : i % W, v = pix ? pix[2 * i + 1] : i / W;
        double T;
        int nc = pixel_forward(&f, u + 0.5, v + 0.5, &out_rgb[3 * i], &T, NULL, NULL);
        if (out_T) out_T[i] = T;
        if (out_n) out_n[i] = nc;
    }
    free(cv);
    free(order);
    return 0;
}

/* ----------------------------------------------------------- backward ----- */

static void atomic_add(double *p, double v)
{
#pragma omp atomic
    *p += v;
}

/* One term of a gradient sum: the term itself, or its absolute value when the
 * magnitude of the sum is wanted instead (see orc_backward_magnitude). */
#define TERM(x) (mag ? fabs(x) : (x))

static void alpha_terms(const orc_convex *c, const pair_eval *e, double o, double qx, double qy, double dLda,
                        double *A, int mag);

/* Per-pixel products of one (pixel, convex) pair, added into the convex's
 * accumulator row A (nx[8] ny[8] v[8] dp sp o rgb[3]).  The line
 * L_j(q) = n_j . (q - v_j) of Eq. signed_distance is differentiated in that
 * form: dL_j/dn_j = q - v_j, dL_j/dv_j = -n_j. */
static void pair_terms(const orc_convex *c, const pair_eval *e, double o, double qx, double qy, const double *g,
                       double T, const double *B, double *A, int mag)
{
    /* dC/dalpha_n = T_n (c_n - B_n) */
    double dLda = 0.0;
    for (int ch = 0; ch < 3; ++ch)
        dLda += mag ? fabs(g[ch]) * T * (fabs(c->rgb[ch]) + fabs(B[ch])) : g[ch] * T * (c->rgb[ch] - B[ch]);
    for (int ch = 0; ch < 3; ++ch) atomic_add(&A[3 * ORC_MAXK + 3 + ch], TERM(g[ch] * T * e->alpha));
    alpha_terms(c, e, o, qx, qy, dLda, A, mag);
}

/* The same products, but only those that pass through dL/dalpha (everything
 * but the colour), for a given dL/dalpha. */
static void alpha_terms(const orc_convex *c, const pair_eval *e, double o, double qx, double qy, double dLda,
                        double *A, int mag)
{
    atomic_add(&A[3 * ORC_MAXK + 2], TERM(dLda * e->I));
    double dLdI = dLda * o;
    double s_ = e->I * e->omI;
    double dLdphi = dLdI * (-c->sp * s_);
    /* dphi/dsigma' term; its magnitude counts phi = max + log-sum as |max| + |log-sum| */
    atomic_add(&A[3 * ORC_MAXK + 1], mag ? fabs(dLdI * s_) * (fabs(e->xmax) + fabs(e->lsum)) : dLdI * (-e->phi * s_));
    double gdp = 0.0;
    for (int j = 0; j < c->T; ++j) {
        const double *vj = c->q[c->hull[j]];
        double gx = dLdphi * e->w[j];
        atomic_add(&A[j], TERM(gx * c->dp * (qx - vj[0])));
        atomic_add(&A[ORC_MAXK + j], TERM(gx * c->dp * (qy - vj[1])));
        atomic_add(&A[2 * ORC_MAXK + j], TERM(gx * c->dp));
        gdp += TERM(gx * e->L[j]);
    }
    atomic_add(&A[3 * ORC_MAXK], gdp);
}

/* Chain rule of one convex from its accumulator row to the optimised
 * parameters (points, delta, sigma, opacity, SH). */
static void convex_chain(const orc_scene *s, const double *cam, int n, const orc_convex *c, const double *A,
                         double *gp, double *g_delta, double *g_sigma, double *g_opacity, double *gsh, int mag)
{
    const int K = s->k, nc = (s->deg + 1) * (s->deg + 1);
    const double *R = cam + 6;
    const double fx = cam[2], fy = cam[3];
    double gdp = A[3 * ORC_MAXK], gsp = A[3 * ORC_MAXK + 1];
    *g_opacity = A[3 * ORC_MAXK + 2];
    *g_delta = c->d * gdp;
    *g_sigma = c->d * gsp;
    double gd = s->delta[n] * gdp + s->sigma[n] * gsp;

    /* lines -> hull vertices:  n_j = (e_y, -e_x)/|e|,  e = v_{j+1} - v_j */
    double gq[ORC_MAXK][2];
    memset(gq, 0, sizeof(gq));
    for (int j = 0; j < c->T; ++j) {
        int ia = c->hull[j], ib = c->hull[(j + 1) % c->T];
        const double *a = c->q[ia], *b = c->q[ib];
        double ex = b[0] - a[0], ey = b[1] - a[1], l = hypot(ex, ey);
        double tx = ex / l, ty = ey / l;
        double gv = A[2 * ORC_MAXK + j]; /* dL/dv_j = -gv n_j */
        double gnx = A[j], gny = A[ORC_MAXK + j];
        gq[ia][0] += TERM(-gv * c->nx[j]);
        gq[ia][1] += TERM(-gv * c->ny[j]);
        /* d n / d e = -(n t^T)/|e| */
        double sdot = (TERM(gnx * tx) + TERM(gny * ty)) / l;
        double gex = TERM(-sdot * c->nx[j]), gey = TERM(-sdot * c->ny[j]);
        gq[ib][0] += gex; gq[ib][1] += gey;
        gq[ia][0] += TERM(-gex); gq[ia][1] += TERM(-gey);
    }
    /* projection and depth -> camera space -> world */
    for (int k = 0; k < K; ++k) {
        double X = c->X[k][0], Y = c->X[k][1], Z = c->X[k][2];
        double gX = gq[k][0] * fx / Z, gY = gq[k][1] * fy / Z;
        double gZ = (TERM(-gq[k][0] * fx * X) + TERM(-gq[k][1] * fy * Y)) / (Z * Z) + gd / K;
        for (int r = 0; r < 3; ++r) gp[3 * k + r] = TERM(R[r] * gX) + TERM(R[3 + r] * gY) + TERM(R[6 + r] * gZ);
    }
    /* colour -> SH coefficients and view direction -> centre -> points */
    double Y[16], dY[48], graw[3], gdir[3] = {0, 0, 0};
    orc_sh_basis(s->deg, c->dir, Y, dY);
    if (mag) sh_basis_magnitude(s->deg, c->dir, Y);
    const double *sh = s->sh + (size_t)n * nc * 3;
    for (int ch = 0; ch < 3; ++ch) graw[ch] = (c->clampmask >> ch & 1) ? 0.0 : A[3 * ORC_MAXK + 3 + ch];
    for (int i = 0; i < nc; ++i)
        for (int ch = 0; ch < 3; ++ch) {
            gsh[3 * i + ch] = TERM(graw[ch] * Y[i]);
            for (int r = 0; r < 3; ++r) gdir[r] += TERM(graw[ch] * sh[3 * i + ch] * dY[3 * i + r]);
        }
    double dd = TERM(c->dir[0] * gdir[0]) + TERM(c->dir[1] * gdir[1]) + TERM(c->dir[2] * gdir[2]);
    for (int r = 0; r < 3; ++r) {
        double gc = (gdir[r] + TERM(-c->dir[r] * dd)) / c->camdist;
        for (int k = 0; k < K; ++k) gp[3 * k + r] += gc / K;
    }
}

typedef struct {
    double *points, *delta, *sigma, *opacity, *sh;
} grad_out;

/* Gradient of L = sum_pixels dl . C (mag = 0); or (mag = 1), for every output
 * element, the sum of the absolute values of all the products that the chain
 * rule adds into it, and, in amb when given, that sum over the products of the
 * pairs listed as ambiguous at relative precision tau. */
static int backward_impl(const orc_scene *s, const double *cam, const double *par, int npix, const int32_t *pix,
                         const double *dl_drgb, grad_out out, grad_out amb, double tau, int mag)
{
    frame f;
    orc_convex *cv;
    int32_t *order;
    if (setup_frame(s, cam, par, mag ? tau : 0.0, &f, &cv, &order)) return -1;
    const int N = s->n, K = s->k, W = (int)cam[0];
    const int nc = (s->deg + 1) * (s->deg + 1);
    const int want_amb = mag && amb.points;
    double *acc = (double *)calloc((size_t)(N > 0 ? N : 1) * NACC, sizeof(double));
    double *acc_amb = want_amb ? (double *)calloc((size_t)(N > 0 ? N : 1) * NACC, sizeof(double)) : NULL;

    /* per pixel: reverse walk over the contributors of the compositing equation */
#pragma omp parallel
    {
        contrib *list = NULL;
        int cap = 0;
        pair_eval e;
#pragma omp for schedule(dynamic, 16)
        for (int i = 0; i < npix; ++i) {
            const double *g = &dl_drgb[3 * i];
            if (g[0] == 0.0 && g[1] == 0.0 && g[2] == 0.0) continue;
            int u = pix ? pix[2 * i] : i % W, v = pix ? pix[2 * i + 1] : i / W;
            double qx = u + 0.5, qy = v + 0.5, C[3], Tf;
            int nl = pixel_forward(&f, qx, qy, C, &Tf, &list, &cap);
            double B[3] = {f.bg[0], f.bg[1], f.bg[2]}; /* colour seen behind the current convex */
            /* sum over the ambiguous pairs behind the current one of
             * T_m alpha_m (|c_m| + |B_m| + |bg|): taking them or not moves the
             * colour behind the current pair by at most this over T_{n+1} */
            double X[3] = {0.0, 0.0, 0.0};
            for (int a = nl - 1; a >= 0; --a) {
                int idx = list[a].idx, fl = list[a].flags;
                double T = list[a].T, o = s->opacity[idx];
                const orc_convex *c = &cv[idx];
                eval_pair(c, o, qx, qy, &e);
                if (fl & CON_IN) pair_terms(c, &e, o, qx, qy, g, T, B, &acc[(size_t)idx * NACC], mag);
                if (want_amb) {
                    double *Aa = &acc_amb[(size_t)idx * NACC];
                    if (fl & CON_AMB) pair_terms(c, &e, o, qx, qy, g, T, B, Aa, 1);
                    if ((fl & CON_IN) && (X[0] > 0.0 || X[1] > 0.0 || X[2] > 0.0)) {
                        double dLda = 0.0; /* |g| T_n |dB_n|, dB_n = X / (T_n (1 - alpha_n)) */
                        for (int ch = 0; ch < 3; ++ch) dLda += fabs(g[ch]) * X[ch] / e.oma;
                        alpha_terms(c, &e, o, qx, qy, dLda, Aa, 1);
                    }
                    if (fl & CON_AMB)
                        for (int ch = 0; ch < 3; ++ch)
                            X[ch] += T * e.alpha * (fabs(c->rgb[ch]) + fabs(B[ch]) + fabs(f.bg[ch]));
                }
                if (fl & CON_IN)
                    for (int ch = 0; ch < 3; ++ch) B[ch] = e.alpha * c->rgb[ch] + e.oma * B[ch];
            }
        }
        free(list);
    }

    /* per convex: chain rule to the optimised parameters */
#pragma omp parallel for schedule(static)
    for (int n = 0; n < N; ++n) {
        for (int w = 0; w < 1 + want_amb; ++w) {
            grad_out o = w ? amb : out;
            double *gp = o.points + (size_t)n * K * 3, *gsh = o.sh + (size_t)n * nc * 3;
            memset(gp, 0, sizeof(double) * K * 3);
            memset(gsh, 0, sizeof(double) * nc * 3);
            o.delta[n] = o.sigma[n] = o.opacity[n] = 0.0;
            const orc_convex *c = &cv[n];
            if ((c->status & 0xff) != ORC_VISIBLE) continue;
            const double *A = &(w ? acc_amb : acc)[(size_t)n * NACC];
            convex_chain(s, cam, n, c, A, gp, &o.delta[n], &o.sigma[n], &o.opacity[n], gsh, mag);
        }
    }
    free(acc);
    free(acc_amb);
    free(cv);
    free(order);
    return 0;
}
#undef TERM

int orc_backward(const orc_scene *s, const double *cam, const double *par, int npix, const int32_t *pix,
                 const double *dl_drgb, double *g_points, double *g_delta, double *g_sigma, double *g_opacity,
                 double *g_sh)
{
    grad_out out = {g_points, g_delta, g_sigma, g_opacity, g_sh}, none = {0};
    return backward_impl(s, cam, par, npix, pix, dl_drgb, out, none, 0.0, 0);
}

int orc_backward_magnitude(const orc_scene *s, const double *cam, const double *par, int npix, const int32_t *pix,
                           const double *dl_drgb, double tau, double *m_points, double *m_delta, double *m_sigma,
                           double *m_opacity, double *m_sh, double *a_points, double *a_delta, double *a_sigma,
                           double *a_opacity, double *a_sh)
{
    grad_out m = {m_points, m_delta, m_sigma, m_opacity, m_sh}, a = {a_points, a_delta, a_sigma, a_opacity, a_sh};
    if (!m_points || !m_delta || !m_sigma || !m_opacity || !m_sh) return -1;
    if (a_points && (!a_delta || !a_sigma || !a_opacity || !a_sh)) return -1;
    if (!(tau >= 0.0 && tau < 1.0)) return -1;
    return backward_impl(s, cam, par, npix, pix, dl_drgb, m, a, tau, 1);
}

/* ------------------------------------------------------ tile candidates --- */

int orc_tile_candidates(const orc_scene *s, const double *cam, double eps_alpha, int tile, int tx, int ty,
                        int32_t *ids, int cap)
{
    if (!s || !cam || tile <= 0) return -1;
    const int W = (int)cam[0], H = (int)cam[1], N = s->n;
    orc_convex *cv = (orc_convex *)malloc((size_t)(N > 0 ? N : 1) * sizeof(orc_convex));
    orc_preprocess(s, cam, eps_alpha, cv);
    int count = 0;
    pair_eval e;
    for (int n = 0; n < N; ++n) {
        const orc_convex *c = &cv[n];
        if ((c->status & 0xff) != ORC_VISIBLE) continue;
        int hit = 0;
        for (int v = ty * tile; v < (ty + 1) * tile && v < H && !hit; ++v)
            for (int u = tx * tile; u < (tx + 1) * tile && u < W && !hit; ++u) {
                double qx = u + 0.5, qy = v + 0.5;
                if (qx < c->rect[0] || qx > c->rect[2] || qy < c->rect[1] || qy > c->rect[3]) continue;
                eval_pair(c, s->opacity[n], qx, qy, &e);
                if (e.alpha >= eps_alpha) hit = 1;
            }
        if (hit) { if (count < cap) ids[count] = n; ++count; }
    }
    free(cv);
    return count;
}
