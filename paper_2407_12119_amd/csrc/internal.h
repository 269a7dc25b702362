// internal.h -- shared declarations of the HIP implementation (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "velognn.h"

namespace velo {

// Error bits latched on the device.
constexpr unsigned kErrInput = 1u;     // invalid hits (offsets, planes, order, non-finite)
constexpr unsigned kErrCapacity = 2u;  // more edges than the edge arrays hold

constexpr int kPlaneSlots = VELO_N_PLANES + 1;   // plane_off entries per event


typedef float f32x4 __attribute__((ext_vector_type(4)));

// Offsets (in floats) of every tensor of the parameter blob.
struct Lin { int64_t w, b; int out, in; };
struct ParamLayout {
    int H = 0, iters = 0;
    Lin emb[3];
    Lin nenc[2], eenc[2];
    Lin node[16][2], edge[16][2];
    Lin cls[2];
    int64_t total = 0;
};
bool make_param_layout(int H, int iters, ParamLayout *L);

struct Workspace {
    float *emb = nullptr;        // [max_hits x 4]
    int *hit_event = nullptr;    // [max_hits]
    int *plane_off = nullptr;    // [max_events x 27]
    int *deg = nullptr;          // [max_hits]
    int *row_ptr = nullptr;      // [max_hits + 1]
    int *nbr = nullptr;          // [max_hits x k_max] staging of selected neighbours
    int *src_g = nullptr;        // [max_edges] batch-global source hit
    int *dst_g = nullptr;        // [max_edges] batch-global destination hit
    int *in_ptr = nullptr;       // [max_hits + 1]
    int *in_list = nullptr;      // [max_edges]
    int *scan_tmp = nullptr;     // block sums of the scans
    int64_t scan_tmp_len = 0;
    void *h[2] = {nullptr, nullptr};    // [max_hits x H] hit encodings (ping-pong), fp32 or bf16
    float *m = nullptr;          // [max_hits x 2H] messages, float32 in every precision
    float *ab = nullptr;         // [max_hits x 2H] per-hit first-layer products of an edge MLP
    void *e = nullptr;           // [max_edges x H] edge encodings (updated in place), fp32 or bf16
    int *n_edges = nullptr;      // [1] internal edge count
    unsigned *flags = nullptr;   // [1] latched device errors
    int *grab = nullptr;         // [8 x 32] per-XCD work counters of the dynamic source-hit walk
                                 // (one 128-byte line each)
    int *eoff_tmp = nullptr;     // [max_events + 1]
    float *scales = nullptr;     // [4 x n_slots] fp8 per-tensor scales
    float *amax = nullptr;       // [2 x n_slots] calibration maxima of the MLP inputs
    float *tmp_logit = nullptr;  // [max_edges] logits of the calibration pass (fp8 contexts)
    float *i8_scales = nullptr;  // [4] INT8 embedding scales {s_x2, s_w2, s_x3, s_w3}
    float *i8_amax = nullptr;    // [2] INT8 calibration maxima of the embedding's layer inputs
    // training (allocated when the config asks for it)
    void *ck_h = nullptr;        // [(n+1) x max_hits x H] hit encodings h^0..h^n
    void *ck_e = nullptr;        // [(n+1) x max_edges x H] edge encodings e^0..e^n
    float *ck_m = nullptr;       // [n x max_hits x 2H] messages of every step
    float *ck_ab = nullptr;      // [(n+1) x max_hits x 2H] per-hit first-layer products (slot k: edge
                                 // network k, slot n: edge encoder)
    float *g_sd = nullptr;       // [max_hits x 2H] per-hit sums of dL/d(hidden) over out- and in-edges
    float *g_e[2] = {nullptr, nullptr};   // [max_edges x H] dL/de (ping-pong)
    float *g_h[2] = {nullptr, nullptr};   // [max_hits x H] dL/dh (ping-pong)
    float *g_da = nullptr, *g_r = nullptr;   // [max(E,N) x H] hidden gradient / activation
    float *g_m = nullptr;        // [max_hits x 2H] dL/dm
    float *g_part = nullptr;     // [n_chunks x part_len] weight-gradient partial sums
    float *g_red = nullptr;      // [32 x part_len] group sums of the partials
    float *g_loss = nullptr;     // [n_chunks] loss partial sums
    // embedding training (allocated with training)
    float *t_u = nullptr;        // [max_hits x 4] normalised inputs u0 u1 u2 0
    float *t_a1 = nullptr, *t_a2 = nullptr;     // [max_hits x 128] hidden activations
    float *t_dz1 = nullptr, *t_dz2 = nullptr;   // [max_hits x 128] their gradients (pre-ReLU)
    float *t_dz3 = nullptr;      // [max_hits x 4] dL/d(embedding)
    int *t_nbr = nullptr;        // [max_hits x VELO_EMB_TRAIN_KMAX] bounded neighbour lists
    int *t_deg = nullptr;        // [max_hits]
    unsigned long long *t_acc = nullptr;   // [max_hits x 8] fixed-point gradient sums (genuine, fake)
    unsigned long long *t_stat = nullptr;  // [4] fixed-point loss sums and pair counts
    float *t_part = nullptr;     // [chunks x embedding parameters] weight-gradient partials
};

// The triplet stage's workspace (allocated by velo_set_triplet_params).
struct TripletWs {
    int64_t cap = 0;             // triplets each list holds
    float *params = nullptr;     // both triplet classifiers, float32
    int *cnt_art = nullptr, *cnt_elb = nullptr;     // [max_hits] per common hit
    int *art_ptr = nullptr, *elb_ptr = nullptr;     // [max_hits + 1] exclusive scans
    int *art_g = nullptr, *elb_g = nullptr;         // [2 cap] batch-global edge ids
    int *n_int = nullptr;        // [4] internal counts: articulations, elbows (clamped), tracks
    int *par = nullptr;          // [max_edges] union-find parents over edges, then segment roots
    int *first = nullptr, *second = nullptr;        // [max_edges] uses of an edge in articulations
    unsigned char *dup = nullptr, *touched = nullptr;   // [max_edges]
    int *single = nullptr;       // [max_edges] 1: a segment root making a track of its own
    int *single_ptr = nullptr;   // [max_edges + 1]
    int *shared = nullptr;       // [cap] 1: a shared articulation
    int *shared_ptr = nullptr;   // [cap + 1]
    int *scan_tmp = nullptr;     // scan_tmp_ints(max(max_hits, max_edges, cap))
};

}  // namespace velo

struct StageEvents {
    int stage;
    hipEvent_t start, stop;
};

struct velo_ctx {
    velo_config cfg;
    int device = 0;
    int n_cu = 0;
    size_t lds_max = 0;
    velo::ParamLayout layout;
    float *params = nullptr;     // float32 copy of the blob
    bool params_set = false;
    bool train_ready = false;    // a velo_train_forward has filled the checkpoints
    bool calibrated = false;     // fp8 activation scales are set
    bool emb_int8 = false;       // the embedding runs on INT8 operands (scales in ws.i8_scales)
    // triplet stage: with parameters set, the GNN keeps the final edge states
    // (the classifier is not fused into the last edge network)
    bool tri_set = false;
    float tri_cut = 0.f;         // keep a triplet iff logit >= tri_cut
    velo::TripletWs tri;
    uint64_t ws_epoch = 0;       // counts calls that use the workspace
    uint64_t tri_epoch = 0;      // epoch of the last GNN pass whose final edge states are kept
    velo::Workspace ws;
    std::string last_error;
    // launch parameters per stage, chosen by velo_autotune (0 = built-in default)
    int tune_per_cu[VELO_N_STAGES] = {};
    int tune_xcd[VELO_N_STAGES] = {};   // 1: XCD-blocked work mapping
    int tune_knn_run = 0;                // neighbour search: query hits per wavefront task (0 = 16)
    int tune_mlp_block[VELO_N_STAGES] = {};   // MLP stages: threads per workgroup (0 = 512)
    // per-stage timing
    bool timing = false;
    std::vector<StageEvents> ev_pool;     // created on first enable
    size_t ev_used = 0;
    int64_t ev_dropped = 0;               // stage launches not timed: the pool was full
    double stage_ms[VELO_N_STAGES] = {};
    int64_t stage_launches[VELO_N_STAGES] = {};
};

namespace velo {

// ---- launchers (graph.hip) ----
void launch_prepare(velo_ctx *c, const velo_hits *h, hipStream_t s);
// the same with explicit working memory: plane_off [n_events x 27], hit_event [n_hits], flags [1]
void launch_prepare_raw(const velo_hits *h, int max_event_hits, int *plane_off, int *hit_event, unsigned *flags,
                        hipStream_t s);
void launch_knn(velo_ctx *c, const velo_hits *h, const float *emb, hipStream_t s);
void launch_knn_loop(velo_ctx *c, const velo_hits *h, const float *emb, hipStream_t s);
void launch_knn_into(velo_ctx *c, const velo_hits *h, const float *emb, int kmax, float d2max, int *nbr, int *deg,
                     hipStream_t s);
void launch_scan(velo_ctx *c, const int *in, int *out, int64_t n, hipStream_t s);
// exclusive scan of n ints into out[0..n] (out[n] = total) with a temporary of scan_tmp_ints(n) ints
void launch_scan_with(const int *in, int *out, int64_t n, int *tmp, hipStream_t s);
int64_t scan_tmp_ints(int64_t n);
void launch_compact(velo_ctx *c, const velo_hits *h, velo_outputs *g, hipStream_t s);
void launch_globalise(velo_ctx *c, const velo_hits *h, const velo_outputs *g, hipStream_t s);
// the same with explicit working memory; src_g/dst_g may be null (validation and the clamped
// edge count n_internal only)
void launch_globalise_raw(const velo_hits *h, const velo_outputs *g, int64_t cap, int *src_g, int *dst_g,
                          int *n_internal, unsigned *flags, hipStream_t s);
// row_ptr of a given graph (edges grouped by source, checked by launch_globalise)
void launch_row_ptr(velo_ctx *c, const velo_hits *h, const velo_outputs *g, hipStream_t s);
void launch_fill(int *p, int v, int64_t n, hipStream_t s);
void launch_in_lists_plane(velo_ctx *c, const velo_hits *h, hipStream_t s);

// ---- launchers (gnn.hip) ----
size_t state_bytes(int precision);              // bytes per stored encoding element
bool gnn_supported(int hidden, int precision);  // compiled (hidden, precision) pairs
void launch_embed(velo_ctx *c, const velo_hits *h, float *emb, bool calib, hipStream_t s);
// float32 embedding recording the largest input of its second and third layers into ws.i8_amax
void launch_embed_int8_amax(velo_ctx *c, const velo_hits *h, float *emb, hipStream_t s);
void launch_components_sweep(velo_ctx *c, const velo_hits *h, const velo_outputs *g, hipStream_t s);
void launch_focal(velo_ctx *c, const float *logit, const uint8_t *y, float alpha, float gamma, int64_t n,
                  float *loss, float *dlogit, hipStream_t s);
void launch_embed_train(velo_ctx *c, const velo_hits *h, const float *params, float *emb, float *sv,
                        float *sa1, float *sa2, hipStream_t s);
int64_t emb_train_chunks(int64_t n_hits);
void launch_embed_train_grad(velo_ctx *c, const velo_hits *h, const velo_embed_truth *truth, const float *params,
                             int k_train, float d2_train, float margin, float w_genuine, float *dparams,
                             float *loss, int64_t *counts, float *emb, hipStream_t s);
// GNN forward over the graph in the workspace (src_g, dst_g, row_ptr, in lists)
void launch_gnn(velo_ctx *c, const velo_hits *h, float *logit, const float *params, bool train, bool calib,
                hipStream_t s);

// fp8 scale table: one slot of four floats {s_x1, s_w1, s_x2, s_w2} per MLP
// (inputs and weights of its two matrix layers) and two calibration maxima.
constexpr int kSlotEmbed = 0;     // embedding layers 2 and 3
constexpr int kSlotNodeEnc = 1;   // node encoder layer 2 (x2, w2)
constexpr int kSlotEdgeEnc = 2;
inline int slot_node(int k) { return 3 + 2 * k; }
inline int slot_edge(int k) { return 4 + 2 * k; }
inline int slot_cls(int iters) { return 3 + 2 * iters; }   // classifier layer 1 (x1, w1)
inline int n_slots(int iters) { return 4 + 2 * iters; }
void launch_weight_scales(velo_ctx *c, hipStream_t s);
void launch_act_scales(velo_ctx *c, hipStream_t s);

// ---- launchers (train.hip) ----
bool train_supported(int hidden, int precision);
size_t train_part_floats(int H);
size_t train_red_floats(int H);
void launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
                 int step, hipStream_t s);
void launch_bce(velo_ctx *c, const float *logit, const uint8_t *y, float pos_weight, int64_t n, float *loss,
                float *dlogit, hipStream_t s);
void launch_gnn_backward(velo_ctx *c, const velo_hits *h, const float *params, const float *dlogit, float *dparams,
                         hipStream_t s);

// ---- launchers (triplets.hip) ----
bool triplet_supported(int hidden);
void launch_triplets(velo_ctx *c, const velo_hits *h, const velo_outputs *g, const velo_triplet_outputs *t,
                     hipStream_t s);

// ---- launchers (wcc.hip) ----
void launch_components(velo_ctx *c, const velo_hits *h, const velo_outputs *g, hipStream_t s);
void launch_components_raw(const velo_hits *h, const velo_outputs *g, int64_t cap, float thr, int max_event_hits,
                           size_t lds_max, const int *n_internal, unsigned *flags, hipStream_t s);

// Records events around the launches of one stage while timing is enabled.
struct StageTimer {
    velo_ctx *c;
    hipStream_t s;
    StageEvents *ev = nullptr;
    StageTimer(velo_ctx *ctx, int stage, hipStream_t stream) : c(ctx), s(stream) {
        if (!c->timing) return;
        if (c->ev_used < c->ev_pool.size()) {
            ev = &c->ev_pool[c->ev_used++];
            ev->stage = stage;
            (void)hipEventRecord(ev->start, s);   // a failed record fails velo_read_timing
        } else {
            c->ev_dropped++;         // reported by velo_read_timing
        }
    }
    ~StageTimer() {
        if (ev) (void)hipEventRecord(ev->stop, s);
    }
};

// Grid size for persistent kernels: `per_cu` blocks on every compute unit.
inline int persistent_grid(const velo_ctx *c, int per_cu) { return c->n_cu * per_cu; }

// Blocks per CU for a stage: the tuned value if set (capped by what fits),
// else `dflt`.
inline int stage_per_cu(const velo_ctx *c, int stage, int dflt, int cap = 1 << 30) {
    const int t = c->tune_per_cu[stage];
    int v = t > 0 ? t : dflt;
    if (v > cap) v = cap;
    return v < 1 ? 1 : v;
}

// Work mapping of persistent kernels over `units` work items.  Interleaved:
// wave w takes units w, w + W, ...  XCD-blocked: workgroups are dispatched
// round-robin over the XCDs, so block b runs on XCD b % kXcds; each XCD gets
// a contiguous slice of the units (consecutive edges and hits belong to the
// same events), keeping an event's states in one XCD's L2.
constexpr int kXcds = 8;
struct WaveRange {
    int64_t first, step, end;
};
__device__ inline WaveRange wave_range(int64_t units, bool xcd) {
    const int wpb = blockDim.x >> 6, wib = threadIdx.x >> 6;
    if (!xcd || (gridDim.x % kXcds) != 0) {
        const int64_t w = (int64_t)blockIdx.x * wpb + wib;
        return {w, (int64_t)gridDim.x * wpb, units};
    }
    const int x = blockIdx.x % kXcds;
    const int64_t bx = blockIdx.x / kXcds, nbx = gridDim.x / kXcds;
    const int64_t per = (units + kXcds - 1) / kXcds;
    const int64_t lo = per * x, hi = min(units, lo + per);
    return {lo + bx * wpb + wib, nbx * wpb, hi};
}

// A value the caller knows to be the same in every lane, moved to scalar
// registers (lane 0's copy).
__device__ inline int64_t uniform64(int64_t v) {
    const uint64_t u = (uint64_t)v;
    return (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(u >> 32)) << 32) |
                     (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u));
}

// Read-only view of device memory through the constant address space: reads
// at wave-uniform addresses become scalar loads.  For buffers that no kernel
// running at the same time writes.
template <typename T>
using const_as = const __attribute__((address_space(4))) T;

}  // namespace velo
