// C-ABI runtime of the convex rasterizer: argument checks, frame buffers,
// the launch sequence of the forward and backward passes (eager, or captured
// into a hipGraph and replayed), the autotuner and the stage timers.  Every
// compute step runs in the HIP kernels of this library.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <atomic>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "convexsplat.h"
#include "common.hpp"
#include "runtime.hpp"

namespace cs {
void launch_preprocess_fwd(hipStream_t, int, int, int, int, int, const void *, const void *, const void *,
                           const void *, const void *, const FrameHeader *, const RenderArgs &, uint8_t *,
                           uint32_t *, uint32_t *, uint4 *, uint32_t *, DebugConvex *, const ZeroSpans &);
void launch_preprocess_bwd(hipStream_t, int, int, int, int, int, const void *, const void *, const void *,
                           const void *, const FrameHeader *, const uint32_t *, const float *,
                           float *, float *, float *, float *, float *);
void radix_sort(hipStream_t, uint32_t **, uint32_t **, uint32_t **, uint32_t **, uint32_t, const uint32_t *, uint32_t, int,
                uint32_t *, int, uint32_t *, bool);
size_t radix_sort_words(uint32_t, bool, uint32_t, int, int);
size_t sort_temp_words(uint32_t, int, int);
size_t scan_status_words(uint32_t);
void launch_gather_scan(hipStream_t, uint32_t, const uint32_t *, const uint4 *, uint4 *, uint32_t *, uint32_t *,
                        uint32_t *, unsigned long long *, uint32_t, uint32_t, uint32_t *, uint32_t);
void launch_fill_u32(hipStream_t, uint32_t *, size_t, uint32_t);
void launch_emit_pairs(hipStream_t, uint32_t, uint32_t, const uint32_t *, const uint32_t *, const uint32_t *,
                       const uint4 *, const FrameHeader *, uint32_t, uint32_t *, uint32_t *, uint32_t *, uint32_t);
void launch_prepare_tail(hipStream_t, uint32_t *, uint32_t, uint32_t *, size_t);
void launch_zero_ranges(hipStream_t, uint32_t *, size_t, uint32_t *, size_t, uint32_t *, size_t);
void launch_tile_length_keys(hipStream_t, uint32_t, const uint2 *, uint32_t *, uint32_t *);
void launch_tile_ranges(hipStream_t, const uint32_t *, uint32_t, const uint32_t *, uint32_t, uint2 *, uint32_t);
int launch_render_fwd(hipStream_t, int, int, const FrameHeader *, const uint32_t *, uint32_t, uint32_t *,
                       const uint2 *, const uint32_t *, const uint8_t *, const RenderArgs &, uint2 *,
                       unsigned long long *, float *, size_t);
int launch_render_bwd(hipStream_t, int, int, const FrameHeader *, const uint32_t *, uint32_t, uint32_t *,
                      const uint2 *, const uint32_t *, const uint8_t *, const RenderArgs &, const uint2 *, float *,
                      unsigned long long *);
hipError_t launch_l1_grad(hipStream_t, const float *, const float *, size_t, float *, float *);
} // namespace cs

using namespace cs;

// --------------------------------------------------------------- errors ----

namespace cs {
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
} // namespace cs

namespace {

int ilog2_ceil(uint64_t v)
{
    int b = 0;
    while ((1ull << b) < v) ++b;
    return b;
}

} // namespace

// -------------------------------------------------------- frame buffers ----

// Device memory of the allocation-free forward entry point: one copy per
// device that loads the library, held until the process ends.  In host code
// the name only stands for the symbol: cs_create looks up each device's
// address of it (cs_ctx::scratch), and only that address reaches kernels.
static __device__ __align__(256) uint8_t scratch[CS_NOALLOC_SCRATCH_BYTES];

namespace cs {

int Frame::alloc(void **p, size_t bytes)
{
    if (fixed) return fail(CS_ENOMEM, "internal: allocation in an allocation-free frame");
    bytes = std::max<size_t>(bytes, 256);
    hipError_t e = hipMallocAsync(p, bytes, st);
    if (e != hipSuccess) return fail(CS_ENOMEM, "device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    allocs.push_back(*p);
    bytes_held += bytes;
    return CS_OK;
}

void Frame::release_buffer(void *p)
{
    for (auto &a : allocs)
        if (a == p) {
            (void)hipFreeAsync(a, st);
            a = nullptr;
        }
}

void Frame::drop_graphs()
{
    if (gfwd) (void)hipGraphExecDestroy(gfwd);
    if (gbwd) (void)hipGraphExecDestroy(gbwd);
    if (gbwd_nz) (void)hipGraphExecDestroy(gbwd_nz);
    gfwd = gbwd = gbwd_nz = nullptr;
    gfwd_zero = false;
}

Frame::~Frame()
{
    drop_graphs();
    for (void *p : allocs)
        if (p) (void)hipFreeAsync(p, st);
    if (counters_ev) (void)hipEventSynchronize(counters_ev), (void)hipEventDestroy(counters_ev);
    if (h_counters) (void)hipHostFree(h_counters);
    if (ready) (void)hipEventDestroy(ready);
}

static constexpr size_t VIEW_TABLE_BYTES = sizeof(FrameHeader) + sizeof(ViewDesc) * MAX_VIEWS;

int HostRing::init()
{
    for (auto &s : slot) {
        if (hipHostMalloc(&s.host, VIEW_TABLE_BYTES, hipHostMallocDefault) != hipSuccess)
            return fail(CS_ENOMEM, "pinned staging allocation failed");
        if (hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) != hipSuccess)
            return fail(CS_EHIP, "event creation failed");
    }
    if (hipHostMalloc((void **)&h_word, 64, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
        return fail(CS_ENOMEM, "pinned allocation failed");
    // pinned memory comes back with whatever it held (often an earlier ring's
    // tagged count): zero it, so that no tag is found before a kernel writes it
    std::memset(h_word, 0, 64);
    if (hipHostGetDevicePointer((void **)&d_word, h_word, 0) != hipSuccess)
        return fail(CS_EHIP, "pinned word has no device address");
    return CS_OK;
}

HostRing::~HostRing()
{
    for (auto &s : slot) {
        if (s.ev) (void)hipEventSynchronize(s.ev), (void)hipEventDestroy(s.ev);
        if (s.host) (void)hipHostFree(s.host);
    }
    if (h_word) (void)hipHostFree(h_word);
}

int Frame::init_async_readback()
{
    if (h_counters) return CS_OK;
    if (hipHostMalloc((void **)&h_counters, CNT_WORDS * 4, hipHostMallocDefault) != hipSuccess)
        return fail(CS_ENOMEM, "pinned counter allocation failed");
    std::memset(h_counters, 0, CNT_WORDS * 4);
    if (hipEventCreateWithFlags(&counters_ev, hipEventDisableTiming) != hipSuccess)
        return fail(CS_EHIP, "event creation failed");
    return CS_OK;
}

// Instance-, tile- and pixel-level buffers (pairs come later).
// Capacities are rounded up to one of four steps per octave (at most 25 %
// spare), so that cached frames serve whole size classes of later requests.
static size_t capacity_class(size_t x)
{
    if (x <= 1024) return 1024;
    int lg = 0;
    while ((x >> (lg + 1)) != 0) ++lg;
    const size_t q = (size_t)1 << (lg - 2);
    return (x + q - 1) / q * q;
}

int Frame::init(int n_, int K_, int deg_, int V_, size_t tiles, size_t pix, hipStream_t s, HostRing *r,
                size_t min_inst)
{
    n = n_; K = K_; deg = deg_; V = V_; st = s; ring = r;
    ninst = (size_t)n * V;
    cap_inst = capacity_class(std::max(ninst, min_inst));
    cap_tiles = capacity_class(std::max<size_t>(tiles, 1));
    cap_pix = capacity_class(std::max<size_t>(pix, 1));
    const uint32_t ui = (uint32_t)cap_inst;
#define CS_A(ptr, bytes) do { int r_ = alloc((void **)&(ptr), (bytes)); if (r_) return r_; } while (0)
    CS_A(d_frame, VIEW_TABLE_BYTES);
    CS_A(d_frame_b, VIEW_TABLE_BYTES);
    table_sent[0].clear();
    table_sent[1].clear();
    CS_A(records, cap_inst * rec_stride(K));
    CS_A(keys, cap_inst * 4);
    CS_A(ids, cap_inst * 4);
    CS_A(keys_alt, cap_inst * 4);
    CS_A(ids_alt, cap_inst * 4);
    CS_A(counts_sorted, cap_inst * 4);
    CS_A(offsets, cap_inst * 4);
    CS_A(hullpk, cap_inst * 4);
    CS_A(bins, cap_inst * 16);
    CS_A(bins_sorted, cap_inst * 16);
    CS_A(ranges, cap_tiles * 8);
    CS_A(ord_k, cap_tiles * 4);
    CS_A(ord_v, cap_tiles * 4);
    CS_A(ord_k_alt, cap_tiles * 4);
    CS_A(ord_v_alt, cap_tiles * 4);
    CS_A(pixstate, cap_pix * 8);
    counter_words = CNT_STATUS + scan_status_words((uint32_t)cap_inst);
    CS_A(counters, counter_words * 4);
    CS_A(evalcount, (size_t)2 * EVAL_SLOTS * EVAL_FIELDS * 8);
#undef CS_A
    return CS_OK;
}

int Frame::ensure_pairs(size_t m)
{
    if (m <= cap_pairs && pt) return CS_OK;
    if (fixed)
        return fail(CS_ENOMEM, "%zu (tile, convex) pairs exceed the %zu that fit the allocation-free scratch", m,
                    cap_pairs);
    for (void *p : {(void *)pt, (void *)pi, (void *)pt_alt, (void *)pi_alt, (void *)hist})
        if (p) release_buffer(p);
    cap_pairs = std::max<size_t>(m, 1);
    // sort temporaries: the largest of the depth, tile and tile-order sorts
    // (tile keys sorted in digits of 4 to 8 bits: sized for the most passes)
    const int tile_bits = std::max(1, ilog2_ceil(cap_tiles));
    const size_t hw = std::max({sort_temp_words((uint32_t)cap_inst, 32, 8),
                                sort_temp_words((uint32_t)cap_pairs, tile_bits, 4),
                                sort_temp_words((uint32_t)cap_tiles, 16, 8)});
#define CS_A(ptr, bytes) do { int r_ = alloc((void **)&(ptr), (bytes)); if (r_) return r_; } while (0)
    CS_A(pt, cap_pairs * 4);
    CS_A(pi, cap_pairs * 4);
    CS_A(pt_alt, cap_pairs * 4);
    CS_A(pi_alt, cap_pairs * 4);
    CS_A(hist, hw * 4);
#undef CS_A
    return CS_OK;
}

int Frame::ensure_acc()
{
    if (acc) return CS_OK;
    if (fixed) return fail(CS_EINVAL, "internal: backward on an allocation-free frame");
    return alloc((void **)&acc, cap_inst * acc_stride(K) * 4);
}

// One-view frame whose buffers are carved, 256-byte aligned, from `bytes` of
// device memory at `base` instead of allocated: the instance, tile and pixel
// buffers at their exact sizes, and the pair buffers (with the sort
// temporaries sized for them) as large as the rest allows.  CS_ENOMEM when the
// fixed part leaves no room for pairs.
int Frame::bind(uint8_t *base, size_t bytes, int n_, int K_, int deg_, size_t tiles, size_t pix, hipStream_t s)
{
    fixed = true;
    n = n_; K = K_; deg = deg_; V = 1; st = s;
    ninst = (size_t)n;
    cap_inst = std::max<size_t>(ninst, 1);
    cap_tiles = std::max<size_t>(tiles, 1);
    cap_pix = std::max<size_t>(pix, 1);
    counter_words = CNT_STATUS + scan_status_words((uint32_t)cap_inst);
    size_t off = 0;
    auto carve = [&](size_t b) {
        off = (off + 255) & ~(size_t)255;
        uint8_t *p = base + off;
        off += std::max<size_t>(b, 256);
        return (void *)p;
    };
    d_frame = (FrameHeader *)carve(VIEW_TABLE_BYTES);
    d_frame_b = (FrameHeader *)carve(VIEW_TABLE_BYTES);
    table_sent[0].clear();
    table_sent[1].clear();
    records = (uint8_t *)carve(cap_inst * rec_stride(K));
    keys = (uint32_t *)carve(cap_inst * 4);
    ids = (uint32_t *)carve(cap_inst * 4);
    keys_alt = (uint32_t *)carve(cap_inst * 4);
    ids_alt = (uint32_t *)carve(cap_inst * 4);
    counts_sorted = (uint32_t *)carve(cap_inst * 4);
    offsets = (uint32_t *)carve(cap_inst * 4);
    hullpk = (uint32_t *)carve(cap_inst * 4);
    bins = (uint4 *)carve(cap_inst * 16);
    bins_sorted = (uint4 *)carve(cap_inst * 16);
    ranges = (uint2 *)carve(cap_tiles * 8);
    ord_k = (uint32_t *)carve(cap_tiles * 4);
    ord_v = (uint32_t *)carve(cap_tiles * 4);
    ord_k_alt = (uint32_t *)carve(cap_tiles * 4);
    ord_v_alt = (uint32_t *)carve(cap_tiles * 4);
    pixstate = (uint2 *)carve(cap_pix * 8);
    counters = (uint32_t *)carve(counter_words * 4);
    evalcount = (unsigned long long *)carve((size_t)2 * EVAL_SLOTS * EVAL_FIELDS * 8);
    acc = nullptr;
    // pairs: four arrays of cap_pairs words, then the sort temporaries
    const int tile_bits = std::max(1, ilog2_ceil(cap_tiles));
    auto need = [&](size_t m) {
        const size_t hw = std::max({sort_temp_words((uint32_t)cap_inst, 32, 8),
                                    sort_temp_words((uint32_t)std::max<size_t>(m, 1), tile_bits, 4),
                                    sort_temp_words((uint32_t)cap_tiles, 16, 8)});
        return 4 * (((m * 4 + 255) & ~(size_t)255) + 256) + hw * 4 + 512;
    };
    const size_t fixed_bytes = (off + 255) & ~(size_t)255;
    if (fixed_bytes + need(1) > bytes)
        return fail(CS_ENOMEM, "%d convexes and %zu pixels need %zu MiB of the allocation-free scratch's %zu MiB before any pair",
                    n, pix, (fixed_bytes + need(1)) >> 20, bytes >> 20);
    size_t lo = 1, hi = std::min<size_t>((bytes - fixed_bytes) / 16, 0xFFFFFFFFu);
    while (lo < hi) { // largest pair capacity that fits
        const size_t mid = lo + (hi - lo + 1) / 2;
        if (fixed_bytes + need(mid) <= bytes) lo = mid;
        else hi = mid - 1;
    }
    cap_pairs = lo;
    pt = (uint32_t *)carve(cap_pairs * 4);
    pi = (uint32_t *)carve(cap_pairs * 4);
    pt_alt = (uint32_t *)carve(cap_pairs * 4);
    pi_alt = (uint32_t *)carve(cap_pairs * 4);
    const size_t hw = std::max({sort_temp_words((uint32_t)cap_inst, 32, 8), sort_temp_words((uint32_t)cap_pairs, tile_bits, 4),
                                sort_temp_words((uint32_t)cap_tiles, 16, 8)});
    hist = (uint32_t *)carve(hw * 4);
    if (off > bytes) return fail(CS_ENOMEM, "internal: allocation-free scratch layout overflows");
    return CS_OK;
}

// Upload the view table through the context's ring of pinned staging buffers.
int Frame::upload_views(const FrameHeader &hdr, const ViewDesc *views, int table)
{
    const size_t bytes = sizeof(FrameHeader) + sizeof(ViewDesc) * hdr.nviews;
    std::vector<char> &sent = table_sent[table];
    if (table_stream[table] == st && sent.size() == bytes && std::memcmp(sent.data(), &hdr, sizeof(hdr)) == 0 &&
        std::memcmp(sent.data() + sizeof(FrameHeader), views, bytes - sizeof(FrameHeader)) == 0)
        return CS_OK; // the table on the device is this one (its upload is ordered before this stream's work)
    HostRing::Slot &sg = ring->slot[ring->next];
    ring->next = (ring->next + 1) % (int)(sizeof(ring->slot) / sizeof(ring->slot[0]));
    if (sg.used) {
        hipError_t e = hipEventSynchronize(sg.ev);
        if (e != hipSuccess) return fail(CS_EHIP, "staging wait: %s", hipGetErrorString(e));
    }
    std::memcpy(sg.host, &hdr, sizeof(hdr));
    std::memcpy((char *)sg.host + sizeof(FrameHeader), views, sizeof(ViewDesc) * hdr.nviews);
    hipError_t e = hipMemcpyAsync(table ? d_frame_b : d_frame, sg.host, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        sent.clear();
        return fail(CS_EHIP, "view table upload: %s", hipGetErrorString(e));
    }
    (void)hipEventRecord(sg.ev, st);
    sg.used = true;
    sent.assign((const char *)sg.host, (const char *)sg.host + bytes);
    table_stream[table] = st;
    return CS_OK;
}

int check_scene(const cs_scene *s)
{
    if (!s) return fail(CS_EINVAL, "scene is NULL");
    if (s->n < 0) return fail(CS_EINVAL, "scene.n = %d < 0", s->n);
    if (s->k < 3 || s->k > CS_MAX_K) return fail(CS_EINVAL, "scene.k = %d outside [3, %d]", s->k, CS_MAX_K);
    if (s->sh_degree < 0 || s->sh_degree > CS_MAX_SH_DEGREE)
        return fail(CS_EINVAL, "scene.sh_degree = %d outside [0, 3]", s->sh_degree);
    if (s->n > 0 && (!s->points || !s->delta || !s->sigma || !s->opacity || !s->sh))
        return fail(CS_EINVAL, "scene array pointer is NULL");
    if (s->dtype != CS_DTYPE_F32 && s->dtype != CS_DTYPE_F16 && s->dtype != CS_DTYPE_BF16)
        return fail(CS_EINVAL, "scene.dtype = %d is not a CS_DTYPE_*", s->dtype);
    if ((int64_t)s->n * s->k > (1ll << 30)) return fail(CS_EINVAL, "scene too large");
    return CS_OK;
}

} // namespace cs

// ------------------------------------------------------------- context -----

namespace {

// Records hipEvents around the stages of one call when CS_FLAG_TIMING is set.
struct StageTimer {
    cs_ctx *ctx;
    hipStream_t st;
    bool on;
    hipEvent_t a = nullptr;
    StageTimer(cs_ctx *c, hipStream_t s, bool enabled) : ctx(c), st(s), on(enabled) {}
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


int check_camera(const cs_camera *c)
{
    if (!c) return fail(CS_EINVAL, "camera is NULL");
    if (c->width <= 0 || c->height <= 0 || c->width > 16384 || c->height > 16384)
        return fail(CS_EINVAL, "image size %dx%d outside [1, 16384]", c->width, c->height);
    if (!(c->fx > 0.0f) || !(c->fy > 0.0f)) return fail(CS_EINVAL, "focal lengths must be positive");
    if (!(c->znear > 0.0f)) return fail(CS_EINVAL, "znear must be positive");
    return CS_OK;
}

CamArgs cam_args(const cs_camera *c)
{
    CamArgs ca;
    ca.W = c->width;
    ca.H = c->height;
    ca.fx = c->fx; ca.fy = c->fy; ca.cx = c->cx; ca.cy = c->cy;
    for (int i = 0; i < 9; ++i) ca.R[i] = c->R[i];
    for (int i = 0; i < 3; ++i) ca.t[i] = c->t[i];
    ca.znear = c->znear;
    for (int r = 0; r < 3; ++r)
        ca.campos[r] = -((double)c->R[r] * c->t[0] + (double)c->R[3 + r] * c->t[1] + (double)c->R[6 + r] * c->t[2]);
    return ca;
}

struct Knobs {
    int tile = 16, longest = 0, digits = 8;
};

int render_args(const cs_params *p, RenderArgs &ra, Knobs &kn)
{
    ra.eps_alpha = p ? p->eps_alpha : 1e-6f;
    ra.t_min = p ? p->t_min : 1e-5f;
    for (int i = 0; i < 3; ++i) ra.bg[i] = p ? p->background[i] : 0.0f;
    const int flags = p ? p->flags : 0;
    kn.tile = p ? p->tile : 0;
    if (kn.tile == 0) kn.tile = 16;
    if (kn.tile != 8 && kn.tile != 16 && kn.tile != 32) return fail(CS_EINVAL, "tile size %d unsupported (8, 16, 32)", kn.tile);
    kn.longest = (flags & CS_FLAG_LONGEST_FIRST) ? 1 : 0;
    kn.digits = (flags >> 8) & 15;
    if (kn.digits == 0) kn.digits = 8;
    if (kn.digits < 4 || kn.digits > 8) return fail(CS_EINVAL, "pair-sort digit width %d outside [4, 8]", kn.digits);
    if (!(ra.eps_alpha > 0.0f) || !(ra.eps_alpha < 1.0f)) return fail(CS_EINVAL, "eps_alpha must be in (0, 1)");
    if (!(ra.t_min >= 0.0f) || !(ra.t_min < 1.0f)) return fail(CS_EINVAL, "t_min must be in [0, 1)");
    ra.tile = kn.tile;
    return CS_OK;
}

// Host view table of a call: tile and pixel offsets of every view.
struct ViewPlan {
    FrameHeader hdr{};
    std::vector<ViewDesc> views;
};

int plan_views(int nviews, const cs_camera *cams, int tile, float *const *out, const float *const *dl, ViewPlan &vp)
{
    if (nviews < 1 || nviews > MAX_VIEWS) return fail(CS_EINVAL, "n_views = %d outside [1, %d]", nviews, MAX_VIEWS);
    if (!cams) return fail(CS_EINVAL, "cameras are NULL");
    vp.views.resize(nviews);
    int64_t toff = 0, poff = 0;
    for (int v = 0; v < nviews; ++v) {
        int r = check_camera(&cams[v]);
        if (r) return r;
        ViewDesc &d = vp.views[v];
        std::memset(&d, 0, sizeof(d));
        d.cam = cam_args(&cams[v]);
        d.tiles_x = (cams[v].width + tile - 1) / tile;
        d.tiles_y = (cams[v].height + tile - 1) / tile;
        d.tile_off = (int32_t)toff;
        d.pix_off = poff;
        d.out_rgb = out ? out[v] : nullptr;
        d.dl_drgb = dl ? dl[v] : nullptr;
        toff += (int64_t)d.tiles_x * d.tiles_y;
        poff += (int64_t)cams[v].width * cams[v].height;
    }
    if (toff >= (1ll << 30)) return fail(CS_EINVAL, "too many tiles in one call");
    vp.hdr.nviews = (uint32_t)nviews;
    vp.hdr.total_tiles = (uint32_t)toff;
    vp.hdr.total_pix = poff;
    return CS_OK;
}

// --------------------------------------------------------- launch sequence --

// Tags of the pair counts: unique in the process (never 0), so that a word
// that still holds another call's or another ring's count never matches.
static uint32_t next_count_tag()
{
    static std::atomic<uint32_t> last{0};
    uint32_t t;
    do t = last.fetch_add(1, std::memory_order_relaxed) + 1;
    while (t == 0);
    return t;
}

// Waits for the pair count tagged `tag` in the pinned word (polling: a
// blocking wait wakes up late and the GPU idles).  The stream is queried now
// and then, so that a stream that finished or failed without writing it ends
// the wait with an error.
static int wait_pair_count(const HostRing &ring, uint32_t tag, hipStream_t st, uint32_t *count)
{
    const unsigned long long *w = reinterpret_cast<const unsigned long long *>(ring.h_word);
    for (uint64_t spin = 1;; ++spin) {
        const unsigned long long v = __atomic_load_n(w, __ATOMIC_ACQUIRE);
        if ((uint32_t)(v >> 32) == tag) {
            *count = (uint32_t)v;
            return CS_OK;
        }
        if ((spin & 4095) == 0) {
            const hipError_t q = hipStreamQuery(st);
            if (q == hipErrorNotReady) continue;
            const unsigned long long v2 = __atomic_load_n(w, __ATOMIC_ACQUIRE);
            if (q == hipSuccess && (uint32_t)(v2 >> 32) == tag) {
                *count = (uint32_t)v2;
                return CS_OK;
            }
            return fail(CS_EHIP, "pair count read-back: %s", q == hipSuccess ? "the count was not written"
                                                                          : hipGetErrorString(q));
        }
    }
}

// Forward pass on frame F.  device_count: the pair count stays on the device
// (fixed capacities, graph capture); otherwise it is read back to size the
// pair buffers exactly (plus `margin`).
int enqueue_forward(cs_ctx *ctx, Frame &F, const cs_scene *sc, const RenderArgs &ra, const Knobs &kn,
                    bool device_count, double margin, StageTimer &tm)
{
    hipStream_t st = F.st;
    const int n = sc->n;
    const uint32_t ninst = (uint32_t)F.ninst;
    F.tile = kn.tile;
    F.longest = kn.longest;
    F.digits = kn.digits;
    // The clearing of the frame's counters, the sort temporaries and the tile
    // ranges rides on the kernels before their users (preprocess, pair scan,
    // emission) instead of launches of their own, when those kernels run.
    const bool fused = ninst > 0 && n > 0;
    // A frame that already holds pair buffers (a reused one) runs the tail at
    // once on the device-side count; the host reads the count back while the
    // GPU works and, in the rare case that it did not fit, grows the buffers
    // and runs the tail again before returning.  A new frame waits for the
    // count to size its buffers.
    const bool speculative = !device_count && ninst > 0 && F.pt != nullptr;
    if (fused && !F.pt) { // first sizing: the sort temporaries come with the pair buffers
        int r = F.ensure_pairs(1);
        if (r) return r;
    }
    ZeroSpans zpre{{nullptr, nullptr}, {0u, 0u}};
    if (fused)
        zpre = ZeroSpans{{F.counters, F.hist},
                         {(uint32_t)F.counter_words, (uint32_t)radix_sort_words(ninst, false, ninst, 32, 8)}};
    else
        launch_zero_ranges(st, F.counters, F.counter_words, nullptr, 0, nullptr, 0);
    tm.begin();
    launch_preprocess_fwd(st, n, F.V, F.K, F.deg, sc->dtype, sc->points, sc->delta, sc->sigma, sc->opacity, sc->sh, F.d_frame,
                          ra, F.records, F.keys, F.ids, F.bins, F.hullpk, nullptr, zpre);
    tm.end(CS_STAGE_PREPROCESS);

    uint32_t *keys = F.keys, *ids = F.ids, *keys_alt = F.keys_alt, *ids_alt = F.ids_alt;
    // A frame that holds backward accumulators (from an earlier backward) has
    // them cleared by the compositing kernel, which leaves HBM mostly idle, so
    // that the backward that follows skips its clearing pass (under graph
    // capture too: the batched backward keeps a graph with and one without
    // its clearing pass and replays the one that matches).
    const bool zero_acc = F.acc != nullptr;
    F.acc_zeroed = false;
    // Everything after the pair count: emission, tile sort, ranges, tile order,
    // compositing.  m_dev: the device-side pair count clamped to the buffers, or
    // NULL when the count (M_host) is known here.
    // scan_prepared: the pair scan has set the clamped count and the overflow
    // flag for the current buffers and cleared the tile ranges.
    bool scan_prepared = false;
    auto tail = [&](uint32_t M_host, const uint32_t *m_dev) {
        if (!scan_prepared)
            launch_prepare_tail(st, F.counters, (uint32_t)F.cap_pairs, reinterpret_cast<uint32_t *>(F.ranges),
                                2 * F.cap_tiles);
        scan_prepared = false;
        uint32_t *pt = F.pt, *pi = F.pi, *pt_alt = F.pt_alt, *pi_alt = F.pi_alt;
        if (ninst > 0) {
            const int tile_bits = std::max(1, ilog2_ceil(F.cap_tiles));
            // the emission clears the tile sort's temporaries
            const size_t tw = radix_sort_words(M_host, m_dev != nullptr, (uint32_t)F.cap_pairs, tile_bits, kn.digits);
            tm.begin();
            launch_emit_pairs(st, ninst, (uint32_t)n, ids, F.offsets, F.counts_sorted, F.bins_sorted, F.d_frame,
                              (uint32_t)F.cap_pairs, pt, pi, F.hist, (uint32_t)tw);
            tm.end(CS_STAGE_EMIT);
            tm.begin();
            radix_sort(st, &pt, &pi, &pt_alt, &pi_alt, M_host, m_dev, (uint32_t)F.cap_pairs, tile_bits, F.hist,
                       kn.digits, F.counters + CNT_SORT_ERR, true);
            tm.end(CS_STAGE_TILE_SORT);
            tm.begin();
            launch_tile_ranges(st, pt, M_host, m_dev, m_dev ? (uint32_t)F.cap_pairs : M_host, F.ranges,
                               (uint32_t)F.cap_tiles);
            tm.end(CS_STAGE_RANGES);
        }
        F.sorted_ids = pi;
        F.order = nullptr;
        if (kn.longest) {
            uint32_t *ok = F.ord_k, *ov = F.ord_v, *ok2 = F.ord_k_alt, *ov2 = F.ord_v_alt;
            tm.begin();
            launch_tile_length_keys(st, (uint32_t)F.cap_tiles, F.ranges, ok, ov);
            radix_sort(st, &ok, &ov, &ok2, &ov2, (uint32_t)F.cap_tiles, nullptr, (uint32_t)F.cap_tiles, 16, F.hist,
                       8, F.counters + CNT_SORT_ERR, false);
            tm.end(CS_STAGE_ORDER);
            F.order = ov;
        }
        tm.begin();
        F.eval_slots = launch_render_fwd(st, F.K, kn.tile, F.d_frame, F.order, (uint32_t)F.cap_tiles, F.counters + CNT_QUEUE, F.ranges,
                          F.sorted_ids, F.records, ra, F.pixstate, F.evalcount, zero_acc ? F.acc : nullptr,
                          zero_acc ? F.ninst * acc_stride(F.K) : 0);
        tm.end(CS_STAGE_RENDER_FWD);
    };

    uint32_t M = 0;
    const uint32_t tag = next_count_tag();
    if (ninst > 0) {
        if (!F.pt) { // first sizing: the sort temporaries come with the pair buffers
            int r = F.ensure_pairs(1);
            if (r) return r;
        }
        tm.begin();
        radix_sort(st, &keys, &ids, &keys_alt, &ids_alt, ninst, nullptr, ninst, 32, F.hist, 8, F.counters + CNT_SORT_ERR,
                   fused);
        tm.end(CS_STAGE_DEPTH_SORT);
        tm.begin();
        // the count also goes straight to pinned host memory (no copy in the
        // stream); with the pair buffers' size known (a reused frame, graph
        // capture) the scan also prepares the pair pass
        scan_prepared = device_count || speculative;
        launch_gather_scan(st, ninst, ids, F.bins, F.bins_sorted, F.counts_sorted, F.offsets, F.counters,
                           device_count ? nullptr : reinterpret_cast<unsigned long long *>(F.ring->d_word), tag,
                           scan_prepared ? (uint32_t)F.cap_pairs : 0u, reinterpret_cast<uint32_t *>(F.ranges),
                           (uint32_t)(2 * F.cap_tiles));
        tm.end(CS_STAGE_BIN_SCAN);
        if (!device_count) {
            if (!speculative) { // a new frame waits for its count here
                int r = wait_pair_count(*F.ring, tag, st, &M);
                if (r) return r;
                r = F.ensure_pairs((size_t)std::ceil(M * margin));
                if (r) return r;
                F.npairs = M;
            }
        }
    }
    if (!F.pt) {
        int r = F.ensure_pairs(1);
        if (r) return r;
    }
    tail(M, (device_count || speculative) ? F.counters + CNT_PAIRS_EFF : nullptr);
    if (speculative) {
        int r = wait_pair_count(*F.ring, tag, st, &M);
        if (r) return r;
        F.npairs = M;
        if (M > F.cap_pairs) { // did not fit: grow, reset the tile queues and counts, run the tail again
            int r = F.ensure_pairs((size_t)std::ceil(M * margin));
            if (r) return r;
            launch_zero_ranges(st, F.counters + CNT_QUEUE, QUEUE_WORDS, nullptr, 0,
                               nullptr, 0);
            tail(M, nullptr);
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CS_EHIP, "kernel launch: %s", hipGetErrorString(e));
    F.acc_zeroed = zero_acc && F.eval_slots > 0; // the compositing kernel ran (and cleared them)
    return CS_OK;
}

// clear: clear the accumulators first (false when the forward compositing
// kernel has cleared them since their last use).
int enqueue_backward(Frame &F, const cs_scene *sc, const cs_grads *g, const RenderArgs &ra, StageTimer &tm,
                     bool clear)
{
    hipStream_t st = F.st;
    int r = F.ensure_acc();
    if (r) return r;
    // without clear the forward that just ran has cleared the accumulators and,
    // with its counters, the backward's work queues
    if (clear)
        launch_zero_ranges(st, reinterpret_cast<uint32_t *>(F.acc), F.ninst * acc_stride(F.K), F.counters + CNT_QUEUE_B,
                           QUEUE_WORDS, nullptr, 0);
    F.acc_zeroed = false; // a second backward of the same forward clears them again
    tm.begin();
    F.eval_slots_bwd = launch_render_bwd(st, F.K, F.tile, F.d_frame_b, F.order, (uint32_t)F.cap_tiles, F.counters + CNT_QUEUE_B,
                                         F.ranges, F.sorted_ids, F.records, ra, F.pixstate, F.acc,
                                         F.evalcount + (size_t)EVAL_SLOTS * EVAL_FIELDS);
    tm.end(CS_STAGE_RENDER_BWD);
    tm.begin();
    launch_preprocess_bwd(st, sc->n, F.V, F.K, F.deg, sc->dtype, sc->points, sc->delta, sc->sigma, sc->sh, F.d_frame_b,
                          F.hullpk, F.acc, g->points, g->delta, g->sigma, g->opacity, g->sh);
    tm.end(CS_STAGE_PREPROCESS_BWD);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CS_EHIP, "kernel launch: %s", hipGetErrorString(e));
    return CS_OK;
}

// Capture the work `enqueue` issues on frame F into an executable graph.
template <class Fn> int capture_graph(cs_ctx *ctx, Frame &F, hipGraphExec_t *exec, Fn enqueue)
{
    if (!ctx->capture_stream) {
        hipError_t e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return fail(CS_EHIP, "capture stream: %s", hipGetErrorString(e));
    }
    hipStream_t caller = F.st;
    F.st = ctx->capture_stream;
    hipError_t e = hipStreamBeginCapture(F.st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        F.st = caller;
        return fail(CS_EHIP, "begin capture: %s", hipGetErrorString(e));
    }
    int r = enqueue();
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(F.st, &g);
    F.st = caller;
    if (r) {
        if (g) (void)hipGraphDestroy(g);
        return r;
    }
    if (e != hipSuccess) return fail(CS_EHIP, "graph capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(CS_EHIP, "graph instantiate: %s", hipGetErrorString(e));
    return CS_OK;
}

uint64_t mix(uint64_t h, uint64_t v) { return (h ^ (v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2))); }

uint64_t scene_key(const cs_scene *sc, int V, const Knobs &kn, const RenderArgs &ra)
{
    uint64_t h = 1469598103934665603ull;
    for (uint64_t v : {(uint64_t)sc->n, (uint64_t)sc->k, (uint64_t)sc->sh_degree, (uint64_t)sc->dtype, (uint64_t)V,
                       (uint64_t)(uintptr_t)sc->points, (uint64_t)(uintptr_t)sc->delta, (uint64_t)(uintptr_t)sc->sigma,
                       (uint64_t)(uintptr_t)sc->opacity, (uint64_t)(uintptr_t)sc->sh, (uint64_t)kn.tile,
                       (uint64_t)kn.longest, (uint64_t)kn.digits})
        h = mix(h, v);
    uint32_t bits[5];
    std::memcpy(bits, &ra, sizeof(float) * 5);
    for (uint32_t b : bits) h = mix(h, b);
    return h;
}

// An eager frame for (n, K, deg, V) with at least the given instance, tile and
// pixel capacity: a cached one when available (ordered after its last use),
// else new.  A cached frame serves any scene size and view count that fit its
// buffers (up to 4x larger, so that a small request does not hold a large
// frame); the one that fits most tightly is taken.
int acquire_frame(cs_ctx *ctx, int n, int K, int deg, int V, size_t tiles, size_t pix, hipStream_t st, Frame **out)
{
    const size_t inst = (size_t)n * V;
    // the classes a new frame would take: a cached one qualifies from there up to 4x
    const size_t ci = capacity_class(inst), ct = capacity_class(std::max<size_t>(tiles, 1));
    const size_t cp = capacity_class(std::max<size_t>(pix, 1));
    int best = -1;
    for (size_t i = 0; i < ctx->free_frames.size(); ++i) {
        const Frame *F = ctx->free_frames[i];
        if (F->K == K && F->deg == deg && F->cap_inst >= ci && F->cap_inst <= 4 * ci && F->cap_tiles >= ct &&
            F->cap_tiles <= 4 * ct && F->cap_pix >= cp &&
            (best < 0 || F->cap_inst < ctx->free_frames[best]->cap_inst))
            best = (int)i;
    }
    if (best >= 0) {
        Frame *F = ctx->free_frames[best];
        ctx->free_frames.erase(ctx->free_frames.begin() + best);
        if (F->ready) (void)hipStreamWaitEvent(st, F->ready, 0);
        F->st = st;
        F->n = n;
        F->V = V;
        F->ninst = inst;
        *out = F;
        return CS_OK;
    }
    Frame *F = new Frame;
    int r = F->init(n, K, deg, V, tiles, pix, st, &ctx->ring);
    if (r) {
        delete F;
        return r;
    }
    *out = F;
    return CS_OK;
}

void release_frame(cs_ctx *ctx, Frame *F)
{
    if (!F) return;
    if (!F->ready && hipEventCreateWithFlags(&F->ready, hipEventDisableTiming) != hipSuccess) {
        delete F;
        return;
    }
    (void)hipEventRecord(F->ready, F->st);
    // the cache must not outlive the caller's stream: later users order on the event
    F->st = nullptr;
    ctx->free_frames.push_back(F);
    while (ctx->free_frames.size() > 4) {
        Frame *old = ctx->free_frames.front();
        if (old->ready) (void)hipEventSynchronize(old->ready); // its last stream may not order with the null stream
        delete old;
        ctx->free_frames.erase(ctx->free_frames.begin());
    }
}

int check_grads(const cs_scene *sc, const cs_grads *g)
{
    if (!g) return fail(CS_EINVAL, "grads is NULL");
    if (sc->n > 0 && (!g->points || !g->delta || !g->sigma || !g->opacity || !g->sh))
        return fail(CS_EINVAL, "gradient array pointer is NULL");
    return CS_OK;
}

} // namespace

#define CS_TRY(expr)                                                                                               \
    do {                                                                                                           \
        int r_ = (expr);                                                                                           \
        if (r_ != CS_OK) return r_;                                                                                \
    } while (0)
#define CS_HIP(expr)                                                                                               \
    do {                                                                                                           \
        hipError_t e_ = (expr);                                                                                    \
        if (e_ != hipSuccess) return fail(CS_EHIP, "%s: %s", #expr, hipGetErrorString(e_));                        \
    } while (0)

// ---------------------------------------------------------- entry points ---

extern "C" {

int cs_version(void) { return 300; }

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
    int r = c->ring.init();
    if (!r) { // this device's copy of the allocation-free scratch, and the frame carved from it
        void *sp = nullptr;
        const hipError_t e = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
        if (e != hipSuccess) r = fail(CS_EHIP, "scratch symbol address: %s", hipGetErrorString(e));
        c->scratch = (uint8_t *)sp;
    }
    if (!r) {
        c->noalloc = new Frame;
        c->noalloc->ring = &c->ring;
    }
    if (r) {
        delete c->noalloc;
        delete c;
        return r;
    }
    *out = c;
    return CS_OK;
}

int cs_destroy(cs_ctx *ctx)
{
    if (!ctx) return CS_OK;
    if (ctx->server) cs_serve_stop(ctx);
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    // everything has completed: free on the null stream, whatever became of the callers' streams
    if (ctx->batch) ctx->batch->st = nullptr;
    delete ctx->batch;
    for (Frame *F : ctx->free_frames) {
        F->st = nullptr;
        delete F;
    }
    ctx->free_frames.clear();
    if (ctx->noalloc) ctx->noalloc->st = nullptr;
    delete ctx->noalloc; // owns no memory: its buffers lie in the static scratch
    (void)hipDeviceSynchronize();
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    for (auto &p : ctx->pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto e : ctx->spare) (void)hipEventDestroy(e);
    delete ctx;
    return CS_OK;
}

int cs_state_release(cs_ctx *ctx, cs_fwd_state *s)
{
    if (!s) return CS_OK;
    if (ctx) (void)hipSetDevice(ctx->device);
    if (s->owned) {
        if (ctx) release_frame(ctx, s->frame);
        else delete s->frame;
    }
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
    RenderArgs ra;
    Knobs kn;
    CS_TRY(render_args(prm, ra, kn));
    CS_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    ViewPlan vp;
    CS_TRY(plan_views(1, cam, kn.tile, &out_rgb, nullptr, vp));
    Frame *F = nullptr;
    CS_TRY(acquire_frame(ctx, sc->n, sc->k, sc->sh_degree, 1, vp.hdr.total_tiles, (size_t)vp.hdr.total_pix, st, &F));
    int r = F->upload_views(vp.hdr, vp.views.data());
    StageTimer tm(ctx, st, prm && (prm->flags & CS_FLAG_TIMING));
    if (!r) r = enqueue_forward(ctx, *F, sc, ra, kn, false, 1.3, tm);
    if (r) {
        delete F;
        return r;
    }
    if (state_out) {
        cs_fwd_state *s = new cs_fwd_state;
        s->frame = F;
        s->owned = true;
        s->nviews = 1;
        *state_out = s;
    } else {
        release_frame(ctx, F);
    }
    return CS_OK;
}

int cs_render_forward_noalloc(cs_ctx *ctx, const cs_scene *sc, const cs_camera *cam, const cs_params *prm,
                              float *out_rgb, void *hip_stream)
{
    if (!ctx) return fail(CS_EINVAL, "ctx is NULL");
    CS_TRY(check_scene(sc));
    CS_TRY(check_camera(cam));
    if (!out_rgb) return fail(CS_EINVAL, "out_rgb is NULL");
    RenderArgs ra;
    Knobs kn;
    CS_TRY(render_args(prm, ra, kn));
    if (!ctx->noalloc || !ctx->scratch) return fail(CS_EINVAL, "context has no allocation-free scratch");
    CS_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    ViewPlan vp;
    CS_TRY(plan_views(1, cam, kn.tile, &out_rgb, nullptr, vp));
    Frame &F = *ctx->noalloc;
    CS_TRY(F.bind(ctx->scratch, CS_NOALLOC_SCRATCH_BYTES, sc->n, sc->k, sc->sh_degree, vp.hdr.total_tiles,
                  (size_t)vp.hdr.total_pix, st));
    CS_TRY(F.upload_views(vp.hdr, vp.views.data()));
    StageTimer tm(ctx, st, false); // stage timing would create events: never here
    // pair buffers are bound at the scratch's capacity, so the tail runs on the
    // device-side count at once and a count beyond it comes back as CS_ENOMEM
    return enqueue_forward(ctx, F, sc, ra, kn, false, 1.0, tm);
}

int cs_render_backward(cs_ctx *ctx, const cs_scene *sc, const cs_camera *cam, const cs_params *prm,
                       const cs_fwd_state *state, const float *dl_drgb, cs_grads *g, void *hip_stream)
{
    if (!ctx) return fail(CS_EINVAL, "ctx is NULL");
    if (!state) return fail(CS_EINVAL, "state is NULL");
    CS_TRY(check_scene(sc));
    CS_TRY(check_camera(cam));
    if (!dl_drgb) return fail(CS_EINVAL, "dl_drgb is NULL");
    CS_TRY(check_grads(sc, g));
    return cs_render_backward_batch(ctx, sc, 1, cam, prm, state, &dl_drgb, g, hip_stream);
}

int cs_render_forward_batch(cs_ctx *ctx, const cs_scene *sc, int32_t n_views, const cs_camera *cams,
                            const cs_params *prm, float *const *out_rgb, cs_fwd_state **state_out, void *hip_stream)
{
    if (state_out) *state_out = nullptr;
    if (!ctx) return fail(CS_EINVAL, "ctx is NULL");
    CS_TRY(check_scene(sc));
    if (n_views < 1 || n_views > MAX_VIEWS) return fail(CS_EINVAL, "n_views = %d outside [1, %d]", n_views, MAX_VIEWS);
    if (!cams) return fail(CS_EINVAL, "cameras are NULL");
    for (int v = 0; v < n_views; ++v) CS_TRY(check_camera(&cams[v]));
    if (!out_rgb) return fail(CS_EINVAL, "out_rgb is NULL");
    for (int v = 0; v < n_views && v < MAX_VIEWS; ++v)
        if (!out_rgb[v]) return fail(CS_EINVAL, "out_rgb[%d] is NULL", v);
    RenderArgs ra;
    Knobs kn;
    CS_TRY(render_args(prm, ra, kn));
    const int flags = prm ? prm->flags : 0;
    CS_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    if ((flags & CS_FLAG_AUTOTUNE) && (!prm || prm->tile == 0)) {
        cs_tuning t;
        CS_TRY(cs_autotune(ctx, sc, n_views, cams, prm, &t, hip_stream));
        kn.tile = t.tile;
        kn.longest = t.longest_first;
        kn.digits = t.digit_bits;
        ra.tile = kn.tile;
    }
    ViewPlan vp;
    CS_TRY(plan_views(n_views, cams, kn.tile, out_rgb, nullptr, vp));
    StageTimer tm(ctx, st, (flags & CS_FLAG_TIMING) != 0);

    if (!(flags & CS_FLAG_GRAPH)) { // eager: buffers owned by the state (cached by the context after it)
        Frame *F = nullptr;
        CS_TRY(acquire_frame(ctx, sc->n, sc->k, sc->sh_degree, n_views, vp.hdr.total_tiles,
                             (size_t)vp.hdr.total_pix, st, &F));
        int r = F->upload_views(vp.hdr, vp.views.data());
        if (!r) r = enqueue_forward(ctx, *F, sc, ra, kn, false, 1.3, tm);
        if (r) { delete F; return r; }
        if (state_out) {
            cs_fwd_state *s = new cs_fwd_state;
            s->frame = F;
            s->nviews = n_views;
            *state_out = s;
        } else {
            release_frame(ctx, F);
        }
        return CS_OK;
    }

    // graph mode: the context's frame, captured once and replayed
    const uint64_t key = scene_key(sc, n_views, kn, ra);
    Frame *F = ctx->batch;
    const bool fits = F && ctx->batch_key == key && F->st == st && vp.hdr.total_tiles <= F->cap_tiles &&
                      (size_t)vp.hdr.total_pix <= F->cap_pix;
    if (!fits) {
        if (F) {
            (void)hipStreamSynchronize(F->st);
            delete F;
        }
        ctx->batch = nullptr;
        F = new Frame;
        int r = F->init(sc->n, sc->k, sc->sh_degree, n_views, vp.hdr.total_tiles, (size_t)vp.hdr.total_pix, st, &ctx->ring);
        if (!r) r = F->upload_views(vp.hdr, vp.views.data());
        if (!r) r = F->init_async_readback();
        // first frame: eager, pair buffers sized from its count plus 30 %
        if (!r) r = enqueue_forward(ctx, *F, sc, ra, kn, false, 1.3, tm);
        if (r) { delete F; return r; }
        ctx->batch = F;
        ctx->batch_key = key;
    } else {
        CS_TRY(F->upload_views(vp.hdr, vp.views.data()));
        if (F->gfwd && F->acc && !F->gfwd_zero) { // accumulators appeared: capture again with their clearing
            (void)hipGraphExecDestroy(F->gfwd);
            F->gfwd = nullptr;
        }
        if (!F->gfwd) {
            StageTimer off(ctx, st, false);
            CS_TRY(capture_graph(ctx, *F, &F->gfwd, [&] { return enqueue_forward(ctx, *F, sc, ra, kn, true, 1.0, off); }));
            F->gfwd_zero = F->acc != nullptr;
        }
        tm.begin();
        CS_HIP(hipGraphLaunch(F->gfwd, st));
        F->acc_zeroed = F->gfwd_zero;
        tm.end(CS_STAGE_GRAPH_FWD);
    }
    F->epoch++;
    CS_HIP(hipMemcpyAsync(F->h_counters, F->counters, CNT_WORDS * 4, hipMemcpyDeviceToHost, st));
    CS_HIP(hipEventRecord(F->counters_ev, st));
    if (state_out) {
        cs_fwd_state *s = new cs_fwd_state;
        s->frame = F;
        s->owned = false;
        s->nviews = n_views;
        s->epoch = F->epoch;
        *state_out = s;
    }
    return CS_OK;
}

int cs_batch_check(cs_ctx *ctx, const cs_fwd_state *s)
{
    if (!ctx || !s || !s->frame) return fail(CS_EINVAL, "ctx or state is NULL");
    Frame *F = s->frame;
    if (!s->owned && (ctx->batch != F || F->epoch != s->epoch))
        return fail(CS_EINVAL, "batch state was replaced by a later batched forward");
    CS_HIP(hipSetDevice(ctx->device));
    if (s->owned) {
        uint32_t err = 0;
        CS_HIP(hipMemcpyAsync(&err, F->counters + CNT_SORT_ERR, 4, hipMemcpyDeviceToHost, F->st));
        CS_HIP(hipStreamSynchronize(F->st));
        if (err) return fail(CS_EHIP, "radix sort: a look-back wait exceeded its bound");
        return CS_OK;
    }
    CS_HIP(hipEventSynchronize(F->counters_ev));
    if (F->h_counters[CNT_SORT_ERR]) return fail(CS_EHIP, "radix sort: a look-back wait exceeded its bound");
    if (F->h_counters[CNT_OVERFLOW]) {
        const size_t m = F->h_counters[CNT_PAIRS];
        CS_HIP(hipStreamSynchronize(F->st));
        F->drop_graphs();
        int r = F->ensure_pairs((size_t)std::ceil(m * 1.3));
        if (r) return r;
        return fail(CS_EOVERFLOW, "frame needed %zu (convex, tile) pairs; buffers grown, render it again", m);
    }
    return CS_OK;
}

int cs_render_backward_batch(cs_ctx *ctx, const cs_scene *sc, int32_t n_views, const cs_camera *cams,
                             const cs_params *prm, const cs_fwd_state *state, const float *const *dl_drgb,
                             cs_grads *g, void *hip_stream)
{
    if (!ctx) return fail(CS_EINVAL, "ctx is NULL");
    if (!state || !state->frame) return fail(CS_EINVAL, "state is NULL");
    CS_TRY(check_scene(sc));
    CS_TRY(check_grads(sc, g));
    if (!dl_drgb) return fail(CS_EINVAL, "dl_drgb is NULL");
    Frame *F = state->frame;
    if (n_views != state->nviews || sc->n != F->n || sc->k != F->K || sc->sh_degree != F->deg)
        return fail(CS_EINVAL, "scene or views differ from the forward call");
    for (int v = 0; v < n_views; ++v)
        if (!dl_drgb[v]) return fail(CS_EINVAL, "dl_drgb[%d] is NULL", v);
    RenderArgs ra;
    Knobs kn;
    CS_TRY(render_args(prm, ra, kn));
    ra.tile = F->tile;
    CS_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    if (!state->owned) CS_TRY(cs_batch_check(ctx, state));
    ViewPlan vp;
    CS_TRY(plan_views(n_views, cams, F->tile, nullptr, dl_drgb, vp));
    if (vp.hdr.total_tiles > F->cap_tiles || (size_t)vp.hdr.total_pix > F->cap_pix)
        return fail(CS_EINVAL, "cameras differ from the forward call");
    F->st = st;
    CS_TRY(F->upload_views(vp.hdr, vp.views.data(), 1));
    const bool timing = prm && (prm->flags & CS_FLAG_TIMING);
    if (state->owned || !(prm && (prm->flags & CS_FLAG_GRAPH))) {
        StageTimer tm(ctx, st, timing);
        return enqueue_backward(*F, sc, g, ra, tm, !F->acc_zeroed);
    }
    uint64_t key = 1469598103934665603ull;
    for (uint64_t v : {(uint64_t)(uintptr_t)g->points, (uint64_t)(uintptr_t)g->delta, (uint64_t)(uintptr_t)g->sigma,
                       (uint64_t)(uintptr_t)g->opacity, (uint64_t)(uintptr_t)g->sh})
        key = mix(key, v);
    if (F->kbwd != key) { // other gradient buffers: both backward graphs are stale
        if (F->gbwd) { (void)hipGraphExecDestroy(F->gbwd); F->gbwd = nullptr; }
        if (F->gbwd_nz) { (void)hipGraphExecDestroy(F->gbwd_nz); F->gbwd_nz = nullptr; }
        F->kbwd = key;
    }
    // the graph without the clearing pass when the forward has cleared the accumulators
    const bool cleared = F->acc_zeroed;
    hipGraphExec_t &gx = cleared ? F->gbwd_nz : F->gbwd;
    if (!gx) {
        CS_TRY(F->ensure_acc());
        StageTimer off(ctx, st, false);
        CS_TRY(capture_graph(ctx, *F, &gx, [&] { return enqueue_backward(*F, sc, g, ra, off, !cleared); }));
    }
    StageTimer tm(ctx, st, timing);
    tm.begin();
    CS_HIP(hipGraphLaunch(gx, st));
    F->acc_zeroed = false; // the graph's backward has used them
    tm.end(CS_STAGE_GRAPH_BWD);
    return CS_OK;
}

int cs_autotune(cs_ctx *ctx, const cs_scene *sc, int32_t n_views, const cs_camera *cams, const cs_params *prm,
                cs_tuning *out, void *hip_stream)
{
    if (!ctx || !out) return fail(CS_EINVAL, "ctx or out is NULL");
    CS_TRY(check_scene(sc));
    RenderArgs ra;
    Knobs kn;
    cs_params base = prm ? *prm : cs_params{1e-6f, 1e-5f, {0.f, 0.f, 0.f}, 16, 0};
    base.tile = 16;
    base.flags &= ~(CS_FLAG_AUTOTUNE | CS_FLAG_GRAPH | CS_FLAG_TIMING);
    CS_TRY(render_args(&base, ra, kn));
    CS_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    ViewPlan vp0;
    CS_TRY(plan_views(n_views, cams, 16, nullptr, nullptr, vp0));
    const auto tkey = std::make_tuple(sc->k, sc->sh_degree, (int)n_views, ilog2_ceil(std::max(1, sc->n)),
                                      ilog2_ceil((uint64_t)std::max<int64_t>(1, vp0.hdr.total_pix)));
    auto it = ctx->tune.find(tkey);
    if (it != ctx->tune.end()) {
        *out = it->second;
        return CS_OK;
    }
    // scratch images, upstream gradient and parameter gradients
    const size_t npix = (size_t)vp0.hdr.total_pix;
    const int nc = (sc->sh_degree + 1) * (sc->sh_degree + 1);
    float *img = nullptr, *gbuf = nullptr;
    CS_HIP(hipMallocAsync((void **)&img, npix * 3 * 4 * 2, st));
    CS_HIP(hipMallocAsync((void **)&gbuf, (size_t)std::max(1, sc->n) * (3 * sc->k + 3 + 3 * nc) * 4, st));
    launch_fill_u32(st, reinterpret_cast<uint32_t *>(img), npix * 6, 0x358637bdu); // 1e-6f everywhere
    std::vector<float *> outs(n_views), dls(n_views);
    {
        size_t off = 0;
        for (int v = 0; v < n_views; ++v) {
            outs[v] = img + off;
            dls[v] = img + npix * 3 + off;
            off += (size_t)cams[v].width * cams[v].height * 3;
        }
    }
    cs_grads gr{gbuf, gbuf + (size_t)sc->n * 3 * sc->k, gbuf + (size_t)sc->n * (3 * sc->k + 1),
                gbuf + (size_t)sc->n * (3 * sc->k + 2), gbuf + (size_t)sc->n * (3 * sc->k + 3)};
    hipEvent_t e0, e1;
    CS_HIP(hipEventCreate(&e0));
    CS_HIP(hipEventCreate(&e1));
    cs_tuning best{16, 0, 8, 1e30f, 0.0f};
    int status = CS_OK;
    for (int tile : {8, 16, 32})
        for (int longest : {0, 1})
            for (int digits : {6, 8}) {
                cs_params p = base;
                p.tile = tile;
                p.flags = (base.flags & ~0xF0E) | (longest ? CS_FLAG_LONGEST_FIRST : 0) | CS_FLAG_DIGITS(digits);
                float ms = 0.0f;
                for (int rep = 0; rep < 3 && status == CS_OK; ++rep) {
                    cs_fwd_state *s = nullptr;
                    (void)hipEventRecord(e0, st);
                    status = cs_render_forward_batch(ctx, sc, n_views, cams, &p, outs.data(), &s, hip_stream);
                    if (status == CS_OK)
                        status = cs_render_backward_batch(ctx, sc, n_views, cams, &p, s, dls.data(), &gr, hip_stream);
                    (void)hipEventRecord(e1, st);
                    (void)hipEventSynchronize(e1);
                    cs_state_release(ctx, s);
                    if (rep > 0) {
                        float t = 0.0f;
                        (void)hipEventElapsedTime(&t, e0, e1);
                        ms += t / 2.0f;
                    }
                }
                if (status != CS_OK) break;
                if (tile == 16 && !longest && digits == 8) best.ms_default = ms;
                if (ms < best.ms) {
                    best.tile = tile;
                    best.longest_first = longest;
                    best.digit_bits = digits;
                    best.ms = ms;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFreeAsync(img, st);
    (void)hipFreeAsync(gbuf, st);
    if (status != CS_OK) return status;
    ctx->tune[tkey] = best;
    *out = best;
    return CS_OK;
}

namespace {
// Sums of the work counters of a frame's last forward and backward passes.
int read_work_counters(Frame *F, cs_work_counters *w)
{
    std::vector<unsigned long long> ev(2 * (size_t)EVAL_SLOTS * EVAL_FIELDS, 0ull);
    uint32_t cnt[CNT_WORDS];
    if (F->eval_slots > 0)
        CS_HIP(hipMemcpyAsync(ev.data(), F->evalcount, (size_t)EVAL_FIELDS * 8 * F->eval_slots,
                              hipMemcpyDeviceToHost, F->st));
    if (F->eval_slots_bwd > 0)
        CS_HIP(hipMemcpyAsync(ev.data() + (size_t)EVAL_SLOTS * EVAL_FIELDS, F->evalcount + (size_t)EVAL_SLOTS * EVAL_FIELDS,
                              (size_t)EVAL_FIELDS * 8 * F->eval_slots_bwd, hipMemcpyDeviceToHost, F->st));
    CS_HIP(hipMemcpyAsync(cnt, F->counters, sizeof(cnt), hipMemcpyDeviceToHost, F->st));
    CS_HIP(hipStreamSynchronize(F->st));
    if (cnt[CNT_SORT_ERR]) return fail(CS_EHIP, "radix sort: a look-back wait exceeded its bound");
    std::memset(w, 0, sizeof(*w));
    w->pairs = cnt[CNT_PAIRS];
    for (int g = 0; g < F->eval_slots; ++g) {
        const unsigned long long *e = &ev[(size_t)EVAL_FIELDS * g];
        w->tested += (int64_t)e[EV_TESTED];
        w->full += (int64_t)e[EV_FULL];
    }
    for (int g = 0; g < F->eval_slots_bwd; ++g) {
        const unsigned long long *e = &ev[(size_t)EVAL_SLOTS * EVAL_FIELDS + (size_t)EVAL_FIELDS * g];
        w->full_bwd += (int64_t)e[EV_FULL];
        w->sum_T_full += (int64_t)e[EV_SUM_T];
        w->wave_evals += (int64_t)e[EV_WAVES];
    }
    return CS_OK;
}
} // namespace

int cs_state_stats(cs_ctx *ctx, const cs_fwd_state *s, int64_t *n_pairs, int64_t *n_evaluated, int64_t *n_full)
{
    if (!ctx || !s || !s->frame) return fail(CS_EINVAL, "ctx or state is NULL");
    CS_HIP(hipSetDevice(ctx->device));
    cs_work_counters w;
    CS_TRY(read_work_counters(s->frame, &w));
    if (n_pairs) *n_pairs = w.pairs;
    if (n_evaluated) *n_evaluated = w.tested;
    if (n_full) *n_full = w.full;
    return CS_OK;
}

int cs_state_counters(cs_ctx *ctx, const cs_fwd_state *s, cs_work_counters *out)
{
    if (!ctx || !s || !s->frame || !out) return fail(CS_EINVAL, "ctx, state or out is NULL");
    CS_HIP(hipSetDevice(ctx->device));
    return read_work_counters(s->frame, out);
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
    RenderArgs ra;
    Knobs kn;
    CS_TRY(render_args(prm, ra, kn));
    CS_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    if (sc->n == 0) return CS_OK;
    ViewPlan vp;
    CS_TRY(plan_views(1, cam, kn.tile, nullptr, nullptr, vp));
    Frame F;
    CS_TRY(F.init(sc->n, sc->k, sc->sh_degree, 1, vp.hdr.total_tiles, 1, st, &ctx->ring));
    CS_TRY(F.upload_views(vp.hdr, vp.views.data()));
    DebugConvex *dbg = nullptr;
    CS_TRY(F.alloc((void **)&dbg, sizeof(DebugConvex) * (size_t)sc->n));
    launch_preprocess_fwd(st, sc->n, 1, sc->k, sc->sh_degree, sc->dtype, sc->points, sc->delta, sc->sigma, sc->opacity, sc->sh,
                          F.d_frame, ra, F.records, F.keys, F.ids, F.bins, F.hullpk, dbg,
                          ZeroSpans{{nullptr, nullptr}, {0u, 0u}});
    CS_HIP(hipGetLastError());
    CS_HIP(hipMemcpyAsync(out, dbg, sizeof(DebugConvex) * (size_t)sc->n, hipMemcpyDeviceToHost, st));
    CS_HIP(hipStreamSynchronize(st));
    return CS_OK;
}

int cs_debug_tile_lists(cs_ctx *ctx, const cs_fwd_state *s, int32_t *ranges, int64_t ranges_len, int32_t *ids,
                        int64_t ids_len)
{
    if (!ctx || !s || !s->frame || !ranges) return fail(CS_EINVAL, "NULL argument");
    Frame *F = s->frame;
    CS_HIP(hipSetDevice(ctx->device));
    uint32_t cnt[CNT_WORDS];
    CS_HIP(hipMemcpyAsync(cnt, F->counters, sizeof(cnt), hipMemcpyDeviceToHost, F->st));
    CS_HIP(hipStreamSynchronize(F->st));
    const int64_t npairs = cnt[CNT_PAIRS_EFF];
    FrameHeader hdr;
    CS_HIP(hipMemcpy(&hdr, F->d_frame, sizeof(hdr), hipMemcpyDeviceToHost));
    const int64_t nt = hdr.total_tiles;
    if (ranges_len < 2 * nt || ids_len < npairs || (!ids && npairs))
        return fail(CS_EOVERFLOW, "host buffers too small (%lld ranges, %lld ids needed)", (long long)(2 * nt),
                    (long long)npairs);
    CS_HIP(hipMemcpyAsync(ranges, F->ranges, sizeof(uint2) * nt, hipMemcpyDeviceToHost, F->st));
    if (npairs)
        CS_HIP(hipMemcpyAsync(ids, F->sorted_ids, sizeof(uint32_t) * npairs, hipMemcpyDeviceToHost, F->st));
    CS_HIP(hipStreamSynchronize(F->st));
    return CS_OK;
}

int cs_l1_loss_grad(cs_ctx *ctx, const float *rgb, const float *target, int32_t width, int32_t height,
                    float *dl_drgb, float *loss, void *hip_stream)
{
    if (!ctx || !rgb || !target || !dl_drgb) return fail(CS_EINVAL, "NULL argument");
    if (width <= 0 || height <= 0) return fail(CS_EINVAL, "bad image size");
    CS_HIP(hipSetDevice(ctx->device));
    const hipError_t e = launch_l1_grad((hipStream_t)hip_stream, rgb, target, (size_t)width * height * 3, dl_drgb, loss);
    if (e != hipSuccess) return fail(CS_ENOMEM, "l1 loss scratch: %s", hipGetErrorString(e));
    CS_HIP(hipGetLastError());
    return CS_OK;
}

} // extern "C"

namespace cs {

int forward_batch_on(cs_ctx *ctx, Frame **Fp, const cs_scene *sc, int n_views, const cs_camera *cams,
                     const cs_params *prm, float *const *out_rgb, hipStream_t st, bool *created)
{
    *created = false;
    if (!ctx || !Fp) return fail(CS_EINVAL, "ctx or frame slot is NULL");
    CS_TRY(check_scene(sc));
    if (n_views < 1 || n_views > MAX_VIEWS) return fail(CS_EINVAL, "n_views = %d outside [1, %d]", n_views, MAX_VIEWS);
    if (!cams || !out_rgb) return fail(CS_EINVAL, "cameras or outputs are NULL");
    RenderArgs ra;
    Knobs kn;
    CS_TRY(render_args(prm, ra, kn));
    CS_HIP(hipSetDevice(ctx->device));
    ViewPlan vp;
    CS_TRY(plan_views(n_views, cams, kn.tile, out_rgb, nullptr, vp));
    const size_t inst = (size_t)sc->n * n_views, tiles = vp.hdr.total_tiles, pix = (size_t)vp.hdr.total_pix;
    Frame *F = *Fp;
    if (F && F->K == sc->k && F->deg == sc->sh_degree && F->cap_inst >= inst && F->cap_tiles >= tiles &&
        F->cap_pix >= pix) {
        F->st = st;
        F->n = sc->n;
        F->V = n_views;
        F->ninst = inst;
    } else { // re-create, at least as large as the frame it replaces
        size_t min_inst = 0, min_tiles = tiles, min_pix = pix;
        if (F) {
            if (F->K == sc->k && F->deg == sc->sh_degree) {
                min_inst = F->cap_inst;
                min_tiles = std::max(min_tiles, F->cap_tiles);
                min_pix = std::max(min_pix, F->cap_pix);
            }
            F->st = nullptr; // idle: its buffers go back on the null stream
            delete F;
            *Fp = nullptr;
        }
        F = new Frame;
        int r = F->init(sc->n, sc->k, sc->sh_degree, n_views, min_tiles, min_pix, st, &ctx->ring, min_inst);
        if (r) {
            delete F;
            return r;
        }
        *Fp = F;
        *created = true;
    }
    F->ring = &ctx->ring;
    CS_TRY(F->upload_views(vp.hdr, vp.views.data()));
    StageTimer tm(ctx, st, false);
    return enqueue_forward(ctx, *F, sc, ra, kn, false, 1.3, tm);
}

} // namespace cs
