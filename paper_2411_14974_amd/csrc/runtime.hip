// C-ABI runtime of the convex rasterizer: argument checks, stream-ordered
// buffer management, and the launch sequence of the forward and backward
// passes.  Every compute step runs in the HIP kernels of this library.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "convexsplat.h"
#include "common.hpp"

namespace cs {
void launch_preprocess_fwd(hipStream_t, int, int, int, const float *, const float *, const float *, const float *,
                           const float *, const CamArgs &, const RenderArgs &, uint8_t *, uint32_t *, uint32_t *,
                           uint2 *, uint32_t *, uint32_t *, DebugConvex *);
void launch_preprocess_bwd(hipStream_t, int, int, int, const float *, const float *, const float *, const float *,
                           const CamArgs &, const uint32_t *, const float *, float *, float *, float *, float *,
                           float *);
void radix_sort(hipStream_t, uint32_t **, uint32_t **, uint32_t **, uint32_t **, uint32_t, const uint32_t *, int, int,
                uint32_t *, uint32_t *);
int radix_blocks(uint32_t);
size_t radix_hist_words(int);
size_t scan_temp_words(uint32_t);
void scan_exclusive(hipStream_t, const uint32_t *, uint32_t *, uint32_t, uint32_t *, uint32_t *);
void launch_fill_u32(hipStream_t, uint32_t *, size_t, uint32_t);
void launch_gather_counts(hipStream_t, uint32_t, const uint32_t *, const uint32_t *, uint32_t *);
void launch_emit_pairs(hipStream_t, uint32_t, const uint32_t *, const uint32_t *, const uint2 *, int, uint32_t,
                       uint32_t *, uint32_t *);
void launch_tile_ranges(hipStream_t, const uint32_t *, uint32_t, const uint32_t *, uint32_t, uint2 *);
void launch_render_fwd(hipStream_t, int, int, const uint2 *, const uint32_t *, const uint8_t *, const RenderArgs &,
                       int, int, float *, uint2 *, unsigned long long *);
void launch_render_bwd(hipStream_t, int, int, const uint2 *, const uint32_t *, const uint8_t *, const RenderArgs &,
                       int, int, const float *, const uint2 *, float *);
void launch_l1_grad(hipStream_t, const float *, const float *, size_t, float *, float *);
} // namespace cs

using namespace cs;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define CS_HIP(expr)                                                                                               \
    do {                                                                                                           \
        hipError_t e_ = (expr);                                                                                    \
        if (e_ != hipSuccess) return fail(CS_EHIP, "%s: %s", #expr, hipGetErrorString(e_));                        \
    } while (0)

#define CS_TRY(expr)                                                                                               \
    do {                                                                                                           \
        int r_ = (expr);                                                                                           \
        if (r_ != CS_OK) return r_;                                                                                \
    } while (0)

int ilog2_ceil(uint32_t v)
{
    int b = 0;
    while ((1u << b) < v) ++b;
    return b;
}

// Stream-ordered allocations of one call; freed (stream-ordered) on scope exit
// unless released to a longer-lived owner.
struct Scratch {
    hipStream_t st;
    void *ptrs[32];
    int n = 0;
    explicit Scratch(hipStream_t s) : st(s) {}
    ~Scratch()
    {
        for (int i = 0; i < n; ++i)
            if (ptrs[i]) (void)hipFreeAsync(ptrs[i], st);
    }
    template <class T> int get(T **out, size_t count)
    {
        void *p = nullptr;
        const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
        hipError_t e = hipMallocAsync(&p, bytes, st);
        if (e != hipSuccess) return fail(CS_ENOMEM, "device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
        ptrs[n++] = p;
        *out = static_cast<T *>(p);
        return CS_OK;
    }
    // hand one allocation over to a longer-lived owner
    void keep(const void *p)
    {
        for (int i = 0; i < n; ++i)
            if (ptrs[i] == p) ptrs[i] = nullptr;
    }
};

} // namespace

struct cs_ctx {
    int device = 0;
    size_t budget = 0;
    uint32_t *h_word = nullptr; // pinned host word for the pair-count read-back
    // stage timing
    struct Pending { int stage; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> spare;
    double stage_ms[CS_NUM_STAGES] = {};
    int64_t stage_count[CS_NUM_STAGES] = {};
};

struct cs_fwd_state {
    int n = 0, K = 0, deg = 0, W = 0, H = 0, tiles_x = 0, tiles_y = 0;
    uint32_t npairs = 0;
    hipStream_t stream = nullptr;
    uint8_t *records = nullptr;
    uint32_t *hullpk = nullptr;
    uint32_t *pair_ids = nullptr;
    uint2 *ranges = nullptr;
    uint2 *pixstate = nullptr;
    unsigned long long *evalcount = nullptr;
};

namespace {

// Records hipEvents around the stages of one call when CS_FLAG_TIMING is set.
struct StageTimer {
    cs_ctx *ctx;
    hipStream_t st;
    bool on;
    hipEvent_t a = nullptr;
    StageTimer(cs_ctx *c, hipStream_t s, const cs_params *p) : ctx(c), st(s), on(p && (p->flags & CS_FLAG_TIMING)) {}
    hipEvent_t take()
    {
        if (!ctx->spare.empty()) {
            hipEvent_t e = ctx->spare.back();
            ctx->spare.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
    void begin()
    {
        if (!on) return;
        a = take();
        (void)hipEventRecord(a, st);
    }
    void end(int stage)
    {
        if (!on || !a) return;
        hipEvent_t b = take();
        (void)hipEventRecord(b, st);
        ctx->pending.push_back({stage, a, b});
        a = nullptr;
    }
};

int check_scene(const cs_scene *s)
{
    if (!s) return fail(CS_EINVAL, "scene is NULL");
    if (s->n < 0) return fail(CS_EINVAL, "scene.n = %d < 0", s->n);
    if (s->k < 3 || s->k > CS_MAX_K) return fail(CS_EINVAL, "scene.k = %d outside [3, %d]", s->k, CS_MAX_K);
    if (s->sh_degree < 0 || s->sh_degree > CS_MAX_SH_DEGREE)
        return fail(CS_EINVAL, "scene.sh_degree = %d outside [0, 3]", s->sh_degree);
    if (s->n > 0 && (!s->points || !s->delta || !s->sigma || !s->opacity || !s->sh))
        return fail(CS_EINVAL, "scene array pointer is NULL");
    if ((int64_t)s->n * s->k > (1ll << 30)) return fail(CS_EINVAL, "scene too large");
    return CS_OK;
}

int check_camera(const cs_camera *c)
{
    if (!c) return fail(CS_EINVAL, "camera is NULL");
    if (c->width <= 0 || c->height <= 0 || c->width > 16384 || c->height > 16384)
        return fail(CS_EINVAL, "image size %dx%d outside [1, 16384]", c->width, c->height);
    if (!(c->fx > 0.0f) || !(c->fy > 0.0f)) return fail(CS_EINVAL, "focal lengths must be positive");
    if (!(c->znear > 0.0f)) return fail(CS_EINVAL, "znear must be positive");
    return CS_OK;
}

int make_args(const cs_camera *c, const cs_params *p, CamArgs &ca, RenderArgs &ra)
{
    ca.W = c->width;
    ca.H = c->height;
    ca.fx = c->fx; ca.fy = c->fy; ca.cx = c->cx; ca.cy = c->cy;
    for (int i = 0; i < 9; ++i) ca.R[i] = c->R[i];
    for (int i = 0; i < 3; ++i) ca.t[i] = c->t[i];
    ca.znear = c->znear;
    for (int r = 0; r < 3; ++r)
        ca.campos[r] = -((double)c->R[r] * c->t[0] + (double)c->R[3 + r] * c->t[1] + (double)c->R[6 + r] * c->t[2]);
    ra.eps_alpha = p ? p->eps_alpha : 1e-6f;
    ra.t_min = p ? p->t_min : 1e-5f;
    for (int i = 0; i < 3; ++i) ra.bg[i] = p ? p->background[i] : 0.0f;
    int tile = p ? p->tile : 0;
    if (tile == 0) tile = 16;
    if (tile != 16) return fail(CS_EINVAL, "tile size %d unsupported (16)", tile);
    if (!(ra.eps_alpha > 0.0f) || !(ra.eps_alpha < 1.0f)) return fail(CS_EINVAL, "eps_alpha must be in (0, 1)");
    if (!(ra.t_min >= 0.0f) || !(ra.t_min < 1.0f)) return fail(CS_EINVAL, "t_min must be in [0, 1)");
    ra.tile = tile;
    ra.tiles_x = (c->width + tile - 1) / tile;
    ra.tiles_y = (c->height + tile - 1) / tile;
    return CS_OK;
}

} // namespace

extern "C" {

int cs_version(void) { return 100; }

const char *cs_last_error(void) { return g_err.c_str(); }

int cs_create(int device, size_t hbm_budget_bytes, cs_ctx **out)
{
    if (!out) return fail(CS_EINVAL, "out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return fail(CS_ENODEV, "HIP device %d not available (%d devices)", device, count);
    hipDeviceProp_t prop;
    CS_HIP(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(CS_ENODEV, "device %d is %s; this library is built for gfx950", device, prop.gcnArchName);
    CS_HIP(hipSetDevice(device));
    hipMemPool_t pool;
    CS_HIP(hipDeviceGetDefaultMemPool(&pool, device));
    uint64_t threshold = UINT64_MAX; // keep freed blocks cached for the next call
    CS_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &threshold));
    cs_ctx *c = new cs_ctx;
    c->device = device;
    c->budget = hbm_budget_bytes;
    if (hipHostMalloc((void **)&c->h_word, 16, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return fail(CS_ENOMEM, "pinned host allocation failed");
    }
    *out = c;
    return CS_OK;
}

int cs_destroy(cs_ctx *ctx)
{
    if (!ctx) return CS_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->h_word) (void)hipHostFree(ctx->h_word);
    for (auto &p : ctx->pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto e : ctx->spare) (void)hipEventDestroy(e);
    delete ctx;
    return CS_OK;
}

int cs_state_release(cs_ctx *ctx, cs_fwd_state *s)
{
    if (!s) return CS_OK;
    if (ctx) (void)hipSetDevice(ctx->device);
    void *ptrs[] = {s->records, s->hullpk, s->pair_ids, s->ranges, s->pixstate, s->evalcount};
    for (void *p : ptrs)
        if (p) (void)hipFreeAsync(p, s->stream);
    delete s;
    return CS_OK;
}

int cs_render_forward(cs_ctx *ctx, const cs_scene *sc, const cs_camera *cam, const cs_params *prm, float *out_rgb,
                      cs_fwd_state **state_out, void *hip_stream)
{
    if (state_out) *state_out = nullptr;
    if (!ctx) return fail(CS_EINVAL, "ctx is NULL");
    CS_TRY(check_scene(sc));
    CS_TRY(check_camera(cam));
    if (!out_rgb) return fail(CS_EINVAL, "out_rgb is NULL");
    CamArgs ca;
    RenderArgs ra;
    CS_TRY(make_args(cam, prm, ca, ra));
    CS_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    const int n = sc->n, K = sc->k;
    const int ntiles = ra.tiles_x * ra.tiles_y;
    const uint32_t un = (uint32_t)n;

    Scratch S(st);
    uint8_t *records;
    uint32_t *keys, *ids, *keys_alt, *ids_alt, *counts, *hullpk, *counts_sorted, *offsets, *hist, *scan_tmp, *total;
    uint2 *rects, *ranges, *pixstate;
    unsigned long long *evalcount;
    const int nb_depth = radix_blocks(un);
    CS_TRY(S.get(&records, (size_t)n * rec_stride(K)));
    CS_TRY(S.get(&keys, n));
    CS_TRY(S.get(&ids, n));
    CS_TRY(S.get(&keys_alt, n));
    CS_TRY(S.get(&ids_alt, n));
    CS_TRY(S.get(&counts, n));
    CS_TRY(S.get(&hullpk, n));
    CS_TRY(S.get(&counts_sorted, n));
    CS_TRY(S.get(&offsets, n));
    CS_TRY(S.get(&rects, n));
    CS_TRY(S.get(&total, 4));
    CS_TRY(S.get(&ranges, ntiles));
    CS_TRY(S.get(&pixstate, (size_t)cam->width * cam->height));
    CS_TRY(S.get(&evalcount, 1));

    StageTimer tm(ctx, st, prm);
    launch_fill_u32(st, reinterpret_cast<uint32_t *>(evalcount), 4, 0u);
    tm.begin();
    launch_preprocess_fwd(st, n, K, sc->sh_degree, sc->points, sc->delta, sc->sigma, sc->opacity, sc->sh, ca, ra,
                          records, keys, ids, rects, counts, hullpk, nullptr);
    tm.end(CS_STAGE_PREPROCESS);

    // depth order of the convexes (stable, ties by index)
    uint32_t M = 0;
    if (n > 0) {
        const size_t hw = radix_hist_words(nb_depth);
        CS_TRY(S.get(&hist, hw));
        CS_TRY(S.get(&scan_tmp, scan_temp_words((uint32_t)std::max<size_t>(hw, un)) + 16));
        tm.begin();
        radix_sort(st, &keys, &ids, &keys_alt, &ids_alt, un, nullptr, nb_depth, 32, hist, scan_tmp);
        tm.end(CS_STAGE_DEPTH_SORT);
        tm.begin();
        launch_gather_counts(st, un, ids, counts, counts_sorted);
        scan_exclusive(st, counts_sorted, offsets, un, total, scan_tmp);
        tm.end(CS_STAGE_BIN_SCAN);
        CS_HIP(hipMemcpyAsync(ctx->h_word, total, 4, hipMemcpyDeviceToHost, st));
        CS_HIP(hipStreamSynchronize(st));
        M = *ctx->h_word;
    }

    uint32_t *pt, *pi, *pt_alt, *pi_alt;
    CS_TRY(S.get(&pt, M));
    CS_TRY(S.get(&pi, M));
    CS_TRY(S.get(&pt_alt, M));
    CS_TRY(S.get(&pi_alt, M));
    launch_fill_u32(st, reinterpret_cast<uint32_t *>(ranges), 2 * (size_t)ntiles, 0u);
    if (M > 0) {
        tm.begin();
        launch_emit_pairs(st, un, ids, offsets, rects, ra.tiles_x, M, pt, pi);
        tm.end(CS_STAGE_EMIT);
        const int nb_pairs = radix_blocks(M);
        uint32_t *hist2, *scan2;
        const size_t hw2 = radix_hist_words(nb_pairs);
        CS_TRY(S.get(&hist2, hw2));
        CS_TRY(S.get(&scan2, scan_temp_words((uint32_t)hw2) + 16));
        tm.begin();
        radix_sort(st, &pt, &pi, &pt_alt, &pi_alt, M, nullptr, nb_pairs, std::max(1, ilog2_ceil((uint32_t)ntiles)),
                   hist2, scan2);
        tm.end(CS_STAGE_TILE_SORT);
        tm.begin();
        launch_tile_ranges(st, pt, M, nullptr, M, ranges);
        tm.end(CS_STAGE_RANGES);
    }
    tm.begin();
    launch_render_fwd(st, K, ntiles, ranges, pi, records, ra, cam->width, cam->height, out_rgb, pixstate, evalcount);
    tm.end(CS_STAGE_RENDER_FWD);
    CS_HIP(hipGetLastError());

    if (state_out) {
        cs_fwd_state *s = new cs_fwd_state;
        s->n = n; s->K = K; s->deg = sc->sh_degree; s->W = cam->width; s->H = cam->height;
        s->tiles_x = ra.tiles_x; s->tiles_y = ra.tiles_y;
        s->npairs = M;
        s->stream = st;
        s->records = records; s->hullpk = hullpk; s->pair_ids = pi; s->ranges = ranges; s->pixstate = pixstate;
        s->evalcount = evalcount;
        for (const void *p : {(const void *)records, (const void *)hullpk, (const void *)pi, (const void *)ranges,
                              (const void *)pixstate, (const void *)evalcount})
            S.keep(p);
        *state_out = s;
    }
    return CS_OK;
}

int cs_render_backward(cs_ctx *ctx, const cs_scene *sc, const cs_camera *cam, const cs_params *prm,
                       const cs_fwd_state *state, const float *dl_drgb, cs_grads *g, void *hip_stream)
{
    if (!ctx) return fail(CS_EINVAL, "ctx is NULL");
    if (!state) return fail(CS_EINVAL, "state is NULL");
    CS_TRY(check_scene(sc));
    CS_TRY(check_camera(cam));
    if (!dl_drgb || !g) return fail(CS_EINVAL, "dl_drgb or grads is NULL");
    if (sc->n > 0 && (!g->points || !g->delta || !g->sigma || !g->opacity || !g->sh))
        return fail(CS_EINVAL, "gradient array pointer is NULL");
    if (sc->n != state->n || sc->k != state->K || sc->sh_degree != state->deg || cam->width != state->W ||
        cam->height != state->H)
        return fail(CS_EINVAL, "scene or camera differs from the forward call");
    CamArgs ca;
    RenderArgs ra;
    CS_TRY(make_args(cam, prm, ca, ra));
    CS_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    const int n = sc->n, K = sc->k;
    Scratch S(st);
    float *acc;
    CS_TRY(S.get(&acc, (size_t)n * acc_stride(K)));
    launch_fill_u32(st, reinterpret_cast<uint32_t *>(acc), (size_t)n * acc_stride(K), 0u);
    StageTimer tm(ctx, st, prm);
    tm.begin();
    launch_render_bwd(st, K, ra.tiles_x * ra.tiles_y, state->ranges, state->pair_ids, state->records, ra, cam->width,
                      cam->height, dl_drgb, state->pixstate, acc);
    tm.end(CS_STAGE_RENDER_BWD);
    tm.begin();
    launch_preprocess_bwd(st, n, K, sc->sh_degree, sc->points, sc->delta, sc->sigma, sc->sh, ca, state->hullpk, acc,
                          g->points, g->delta, g->sigma, g->opacity, g->sh);
    tm.end(CS_STAGE_PREPROCESS_BWD);
    CS_HIP(hipGetLastError());
    return CS_OK;
}

int cs_state_stats(cs_ctx *ctx, const cs_fwd_state *s, int64_t *n_pairs, int64_t *n_evaluated, int64_t *n_full)
{
    if (!ctx || !s) return fail(CS_EINVAL, "ctx or state is NULL");
    CS_HIP(hipSetDevice(ctx->device));
    unsigned long long ev[2] = {0, 0};
    CS_HIP(hipMemcpyAsync(ev, s->evalcount, sizeof(ev), hipMemcpyDeviceToHost, s->stream));
    CS_HIP(hipStreamSynchronize(s->stream));
    if (n_pairs) *n_pairs = s->npairs;
    if (n_evaluated) *n_evaluated = (int64_t)ev[0];
    if (n_full) *n_full = (int64_t)ev[1];
    return CS_OK;
}

int cs_timing_read(cs_ctx *ctx, double *ms, int64_t *count, int reset)
{
    if (!ctx) return fail(CS_EINVAL, "ctx is NULL");
    CS_HIP(hipSetDevice(ctx->device));
    for (auto &p : ctx->pending) {
        CS_HIP(hipEventSynchronize(p.b));
        float e = 0.0f;
        CS_HIP(hipEventElapsedTime(&e, p.a, p.b));
        ctx->stage_ms[p.stage] += e;
        ctx->stage_count[p.stage] += 1;
        ctx->spare.push_back(p.a);
        ctx->spare.push_back(p.b);
    }
    ctx->pending.clear();
    for (int i = 0; i < CS_NUM_STAGES; ++i) {
        if (ms) ms[i] = ctx->stage_ms[i];
        if (count) count[i] = ctx->stage_count[i];
        if (reset) { ctx->stage_ms[i] = 0.0; ctx->stage_count[i] = 0; }
    }
    return CS_OK;
}

int cs_debug_preprocess(cs_ctx *ctx, const cs_scene *sc, const cs_camera *cam, const cs_params *prm,
                        cs_debug_convex *out, void *hip_stream)
{
    static_assert(sizeof(cs_debug_convex) == sizeof(DebugConvex), "debug record layout");
    if (!ctx || !out) return fail(CS_EINVAL, "ctx or out is NULL");
    CS_TRY(check_scene(sc));
    CS_TRY(check_camera(cam));
    CamArgs ca;
    RenderArgs ra;
    CS_TRY(make_args(cam, prm, ca, ra));
    CS_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    const int n = sc->n, K = sc->k;
    if (n == 0) return CS_OK;
    Scratch S(st);
    uint8_t *records;
    uint32_t *keys, *ids, *counts, *hullpk;
    uint2 *rects;
    DebugConvex *dbg;
    CS_TRY(S.get(&records, (size_t)n * rec_stride(K)));
    CS_TRY(S.get(&keys, n));
    CS_TRY(S.get(&ids, n));
    CS_TRY(S.get(&counts, n));
    CS_TRY(S.get(&hullpk, n));
    CS_TRY(S.get(&rects, n));
    CS_TRY(S.get(&dbg, n));
    launch_preprocess_fwd(st, n, K, sc->sh_degree, sc->points, sc->delta, sc->sigma, sc->opacity, sc->sh, ca, ra,
                          records, keys, ids, rects, counts, hullpk, dbg);
    CS_HIP(hipGetLastError());
    CS_HIP(hipMemcpyAsync(out, dbg, sizeof(DebugConvex) * (size_t)n, hipMemcpyDeviceToHost, st));
    CS_HIP(hipStreamSynchronize(st));
    return CS_OK;
}

int cs_debug_tile_lists(cs_ctx *ctx, const cs_fwd_state *s, int32_t *ranges, int64_t ranges_len, int32_t *ids,
                        int64_t ids_len)
{
    if (!ctx || !s || !ranges || (!ids && s->npairs)) return fail(CS_EINVAL, "NULL argument");
    const int64_t nt = (int64_t)s->tiles_x * s->tiles_y;
    if (ranges_len < 2 * nt || ids_len < (int64_t)s->npairs)
        return fail(CS_EOVERFLOW, "host buffers too small (%lld ranges, %lld ids needed)", (long long)(2 * nt),
                    (long long)s->npairs);
    CS_HIP(hipSetDevice(ctx->device));
    CS_HIP(hipMemcpyAsync(ranges, s->ranges, sizeof(uint2) * nt, hipMemcpyDeviceToHost, s->stream));
    if (s->npairs)
        CS_HIP(hipMemcpyAsync(ids, s->pair_ids, sizeof(uint32_t) * s->npairs, hipMemcpyDeviceToHost, s->stream));
    CS_HIP(hipStreamSynchronize(s->stream));
    return CS_OK;
}

int cs_l1_loss_grad(cs_ctx *ctx, const float *rgb, const float *target, int32_t width, int32_t height,
                    float *dl_drgb, float *loss, void *hip_stream)
{
    if (!ctx || !rgb || !target || !dl_drgb) return fail(CS_EINVAL, "NULL argument");
    if (width <= 0 || height <= 0) return fail(CS_EINVAL, "bad image size");
    CS_HIP(hipSetDevice(ctx->device));
    launch_l1_grad((hipStream_t)hip_stream, rgb, target, (size_t)width * height * 3, dl_drgb, loss);
    CS_HIP(hipGetLastError());
    return CS_OK;
}

} // extern "C"
