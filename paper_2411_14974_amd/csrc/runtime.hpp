// Runtime-side structures of the convex rasterizer (host code only).
#pragma once
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "convexsplat.h"
#include "common.hpp"

namespace cs {

int fail(int code, const char *fmt, ...);
// CS_OK, or CS_EINVAL (with the message set) for a malformed scene description
int check_scene(const cs_scene *s);

// Pinned staging buffers for view-table uploads, shared by the frames of one
// context; a slot is reused only after its previous copy has completed.
struct HostRing {
    struct Slot {
        void *host = nullptr;
        hipEvent_t ev = nullptr;
        bool used = false;
    } slot[8];
    int next = 0;
    uint32_t *h_word = nullptr; // coherent pinned words for read-backs (kernels write them directly)
    uint32_t *d_word = nullptr; // the device's address of h_word
    int init();
    ~HostRing();
};

// Device buffers of one forward pass over V views of an N-convex scene, plus
// what its backward pass needs.  Instance i of view v is v * N + i.
struct Frame {
    int n = 0, K = 0, deg = 0, V = 0;
    int tile = 16, longest = 0, digits = 8;
    size_t cap_inst = 0, cap_pairs = 0, cap_tiles = 0, cap_pix = 0;
    size_t ninst = 0; // instances of the current use (n V <= cap_inst)
    uint32_t npairs = 0;
    hipStream_t st = nullptr;
    std::vector<void *> allocs;
    size_t bytes_held = 0;

    FrameHeader *d_frame = nullptr;   // header + ViewDesc[MAX_VIEWS]: the forward's view table
    FrameHeader *d_frame_b = nullptr; // the backward's (its views carry dL/dC instead of the output)
    // the bytes last uploaded to each table and the stream of that upload: an
    // identical table on the same stream is not sent again
    std::vector<char> table_sent[2];
    hipStream_t table_stream[2] = {nullptr, nullptr};
    uint8_t *records = nullptr;
    uint32_t *keys = nullptr, *ids = nullptr, *keys_alt = nullptr, *ids_alt = nullptr;
    uint32_t *counts_sorted = nullptr, *offsets = nullptr, *hullpk = nullptr;
    uint4 *bins = nullptr, *bins_sorted = nullptr; // binning records by instance / in depth order
    uint32_t *hist = nullptr; // radix sort temporaries (histograms, tile counters, look-back status)
    uint32_t *pt = nullptr, *pi = nullptr, *pt_alt = nullptr, *pi_alt = nullptr;
    uint2 *ranges = nullptr;
    uint32_t *ord_k = nullptr, *ord_v = nullptr, *ord_k_alt = nullptr, *ord_v_alt = nullptr;
    uint2 *pixstate = nullptr;
    float *acc = nullptr;
    bool acc_zeroed = false; // acc was cleared by the last forward compositing launch
    uint32_t *counters = nullptr; // CNT_WORDS counters, then the pair-offset scan's look-back status
    size_t counter_words = 0;
    // work counters of the last passes' workgroups: EVAL_SLOTS slots of
    // EVAL_FIELDS words for the forward, then as many for the backward
    unsigned long long *evalcount = nullptr;
    int eval_slots = 0, eval_slots_bwd = 0; // slots that the launches wrote
    uint32_t *h_counters = nullptr; // pinned read-back of the counters
    hipEvent_t counters_ev = nullptr;

    // results of the last forward pass (point into the buffers above)
    uint32_t *sorted_ids = nullptr;
    uint32_t *order = nullptr;

    // captured graphs (batched path): the forward (gfwd_zero: it clears the
    // backward's accumulators), the backward with and without its clearing pass
    hipGraphExec_t gfwd = nullptr, gbwd = nullptr, gbwd_nz = nullptr;
    bool gfwd_zero = false;
    uint64_t kbwd = 0;
    void drop_graphs();
    uint64_t epoch = 0;

    HostRing *ring = nullptr;
    hipEvent_t ready = nullptr; // recorded when the frame is handed back to the context's cache

    bool fixed = false; // buffers carved from caller memory (bind): nothing is allocated or freed

    // min_inst: a floor for the instance capacity (a frame re-created larger)
    int init(int n, int K, int deg, int V, size_t tiles, size_t pix, hipStream_t st, HostRing *ring,
             size_t min_inst = 0);
    int bind(uint8_t *base, size_t bytes, int n, int K, int deg, size_t tiles, size_t pix, hipStream_t st);
    int init_async_readback();
    int alloc(void **p, size_t bytes);
    void release_buffer(void *p);
    int ensure_pairs(size_t m);
    int ensure_acc();
    int upload_views(const FrameHeader &hdr, const ViewDesc *views, int table = 0);
    ~Frame();
};

struct Server;

// Batched eager forward of n_views views on a frame owned by the caller (the
// serving loop).  *F (nullable) is used when the batch fits its capacities,
// else replaced by a new frame at least as large as it (*created set); its
// pair buffers grow inside the pass.  The frame is idle again once the
// stream's work completes.
int forward_batch_on(cs_ctx *ctx, Frame **F, const cs_scene *sc, int n_views, const cs_camera *cams,
                     const cs_params *prm, float *const *out_rgb, hipStream_t st, bool *created);

} // namespace cs

struct cs_ctx {
    int device = 0;
    size_t budget = 0;
    cs::HostRing ring;
    // stage timing
    struct Pending { int stage; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> spare;
    double stage_ms[CS_NUM_STAGES] = {};
    int64_t stage_count[CS_NUM_STAGES] = {};
    // batched graph frame and tuning cache
    hipStream_t capture_stream = nullptr; // graphs are captured here (the null stream cannot be) and launched on the caller's
    cs::Frame *batch = nullptr;
    uint64_t batch_key = 0;
    std::map<std::tuple<int, int, int, int, int>, cs_tuning> tune;
    // request loop (serve.hip)
    cs::Server *server = nullptr;
    // frames of finished eager calls, reused by later ones
    std::vector<cs::Frame *> free_frames;
    // allocation-free forward: this device's address of the library's static
    // scratch array, and the frame whose buffers are carved from it per call
    uint8_t *scratch = nullptr;
    cs::Frame *noalloc = nullptr;
};

struct cs_fwd_state {
    cs::Frame *frame = nullptr;
    bool owned = true; // plain states own their frame; batch-graph states borrow the context's
    int nviews = 1;
    uint64_t epoch = 0;
};

