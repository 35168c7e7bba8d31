/*
 * FP64 CPU oracle for the differentiable smooth-convex rasterizer of
 * "3D Convex Splatting" (Held et al., CVPR 2025).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code; it exists so that tests and the benchmark's CPU baseline can
 * check the HIP path against a plain, slow evaluation of the paper's
 * definitions.  It shares no code, header, table or constant with the HIP
 * library.
 *
 * What it computes (paper section / equation):
 *   - pinhole projection of every point of a convex    (Sec. 3.2, Eq. projection)
 *   - 2D convex hull of the projected points            (Sec. 3.2, "2D convex hull
 *     computation"); brute force over directed pairs, not Graham scan: the
 *     result (the set and cyclic order of extreme points) is the same object
 *   - hull edge lines as signed distances               (Sec. 3.1, Eq. signed_distance)
 *   - smooth SDF phi = log sum exp(d*delta*L_t)         (Supp. B, Eq. smoothness_supp)
 *   - indicator I = Sigmoid(-d*sigma*phi)               (Supp. B, Eq. sharpness_supp)
 *   - front-to-back alpha compositing                   (Sec. 3.2, compositing equation)
 *   - view-dependent colour from real SH, degree <= 3   (Sec. 3.2 and Sec. 4 impl. details)
 *   - the analytic gradient of all of the above w.r.t. points, delta, sigma,
 *     opacity and SH coefficients                       (Sec. 3.3, optimised parameters)
 *
 * Readings of points the paper leaves open are listed in the header of
 * oracle.c; each one is applied in exactly one place there.
 */
#ifndef CONVEX_ORACLE_H
#define CONVEX_ORACLE_H
#include <stdint.h>

#define ORC_MAXK 8

typedef struct {
    int32_t n, k, deg, pad;
    const double *points;   /* [n][k][3] world space */
    const double *delta;    /* [n] smoothness, > 0 (activated) */
    const double *sigma;    /* [n] sharpness,  > 0 (activated) */
    const double *opacity;  /* [n] in [0,1]   (activated) */
    const double *sh;       /* [n][(deg+1)^2][3] */
} orc_scene;

/* camera: 19 doubles {W, H, fx, fy, cx, cy, R[9] row-major world->camera, t[3], znear} */
#define ORC_CAM_LEN 19

/* params: {eps_alpha, t_min, bg_r, bg_g, bg_b, mode}; mode 0 = exact, 1 = matched */
#define ORC_PAR_LEN 6

/* status bits of a convex */
#define ORC_VISIBLE     0
#define ORC_CULL_NEAR   1
#define ORC_CULL_HULL   2
#define ORC_DEGENERATE  256   /* or-ed flag: some point triple is nearly collinear */

typedef struct {
    int32_t status;            /* ORC_* */
    int32_t T;                 /* hull size */
    int32_t hull[ORC_MAXK];    /* point indices, positive orientation, from min (y, x) */
    uint32_t key;              /* bits of the pinned float32 depth key */
    int32_t clampmask;         /* bit c set when colour channel c was clamped at 0 */
    double X[ORC_MAXK][3];     /* camera-space points */
    double q[ORC_MAXK][2];     /* projected points, pixel units */
    double nx[ORC_MAXK], ny[ORC_MAXK], off[ORC_MAXK]; /* L_j(q) = nx*qx + ny*qy + off */
    double d, dp, sp;          /* depth d, delta' = d*delta, sigma' = d*sigma */
    double rgb[3];             /* clamped colour */
    double dir[3];             /* unit view direction used for the colour */
    double camdist;            /* |centre - camera position| */
    double rect[4];            /* xmin, ymin, xmax, ymax: outside it alpha < rect threshold */
} orc_convex;

/* Per-convex quantities; rect_alpha is the alpha threshold the rect bounds. */
int orc_preprocess(const orc_scene *s, const double *cam, double rect_alpha, orc_convex *out);

/* Visible convexes sorted by (key, index); returns how many. */
int orc_order(int n, const orc_convex *cv, int32_t *order);

/* Colour of pixels. pix = NULL renders the whole image in row-major order
 * (npix must then be W*H); otherwise pix holds npix (u, v) pairs.
 * out_T: transmittance after the last convex; out_n: number of contributors. */
int orc_render(const orc_scene *s, const double *cam, const double *par,
               int npix, const int32_t *pix,
               double *out_rgb, double *out_T, int32_t *out_n);

/* Gradient of L = sum_pixels dl_drgb . C with respect to every parameter.
 * Gradient arrays have the shapes of the scene arrays and are overwritten. */
int orc_backward(const orc_scene *s, const double *cam, const double *par,
                 int npix, const int32_t *pix, const double *dl_drgb,
                 double *g_points, double *g_delta, double *g_sigma,
                 double *g_opacity, double *g_sh);

/* Conditioning of orc_backward, for a parity check of an evaluation in
 * another precision or summation order (test use):
 *   m_*: per output element, the sum of the absolute values of all the
 *        products the chain rule adds into it (colour differences c - B
 *        counted as |c| + |B|).  Rounding moves a sum by a small multiple of
 *        the unit roundoff times this magnitude; a gradient that cancels (|g|
 *        much smaller than m) has no better relative accuracy than that.
 *   a_*: (optional, NULL to skip) the same sums over the pairs whose matched-
 *        mode decision is within the relative band tau of its threshold:
 *        alpha within tau of eps_alpha, or after T came within tau of t_min.
 *        Another precision may keep or drop exactly those pairs.
 * Returns -1 on bad arguments (tau outside [0, 1), a NULL m_* array). */
int orc_backward_magnitude(const orc_scene *s, const double *cam, const double *par,
                           int npix, const int32_t *pix, const double *dl_drgb, double tau,
                           double *m_points, double *m_delta, double *m_sigma,
                           double *m_opacity, double *m_sh,
                           double *a_points, double *a_delta, double *a_sigma,
                           double *a_opacity, double *a_sh);

/* Ids of the convexes whose alpha reaches eps_alpha at some pixel of a tile;
 * returns the count (ids are written up to cap). */
int orc_tile_candidates(const orc_scene *s, const double *cam, double eps_alpha,
                        int tile, int tx, int ty, int32_t *ids, int cap);

/* Real spherical harmonic basis (and its gradient in R^3 of the polynomial
 * extension) at unit direction dir, degree <= 3: 16 values, (l, m) order. */
void orc_sh_basis(int deg, const double *dir, double *Y, double *dY /* [16][3] or NULL */);

#endif
