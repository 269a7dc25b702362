/*
 * velognn.h -- C ABI of the MI355X (gfx950) VELO GNN track-finding library.
 *
 * The library runs the data-parallel inference path of the GNN track finder of
 * "Graph Neural Network-Based Track Finding in the LHCb Vertex Detector"
 * (arXiv 2407.12119) over a batch of independent events:
 *
 *   hits (x, y, z, plane) of many events
 *     -> hit embedding MLP                     (Sec. 5.1)
 *     -> rough graph: hits on plane p joined to hits on p+1, p+2 within a
 *        squared embedding distance, at most k_max per hit   (Sec. 5.1, 7.2)
 *     -> interaction-network GNN edge logits   (Sec. 5.2)
 *     -> edge cut and connected components     (Sec. 5, 7.3)
 *   -> per-hit track labels and per-edge scores.
 *
 * Conventions shared by every call:
 *   - All array pointers are DEVICE pointers unless the name says otherwise;
 *     the caller owns every input and output buffer.  The library owns the
 *     context, its workspace and its converted copy of the parameters.
 *   - `stream` is a hipStream_t passed as void*.  Every call is asynchronous
 *     on that stream and allocates nothing; velo_create/velo_destroy allocate
 *     and free.  A context is not thread-safe: one context per host thread.
 *   - Hits are grouped by event: event b owns hits
 *     [event_offsets[b], event_offsets[b+1]).  Within an event the hits are
 *     sorted by plane (non-decreasing); plane lies in [0, VELO_N_PLANES).
 *   - Every index in an output is EVENT-LOCAL (0 .. hits of that event - 1),
 *     so an event gives identical outputs alone or inside a batch.
 *   - Errors found on the host are returned at once.  Errors found on the
 *     device (invalid input, capacity overflow) are latched in the context
 *     and returned by velo_check(), which synchronises the stream; while an
 *     error is latched the device stages of later calls do no work.
 *   - No call aborts the process and no C++ exception crosses this ABI.
 */
#ifndef VELOGNN_H
#define VELOGNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VELO_N_PLANES 26      /* VELO planes (Sec. 2) */
#define VELO_EMB_HIDDEN 128   /* embedding MLP width: 3 -> 128 -> 128 -> 4 */
#define VELO_EMB_DIM 4        /* embedding dimension n_dim (Sec. 5.1) */

typedef enum {
    VELO_OK = 0,
    VELO_ERR_INVALID_ARG = 1,   /* bad host argument (null pointer, size, config) */
    VELO_ERR_CAPACITY = 2,      /* more hits/edges/events than the context holds */
    VELO_ERR_OOM = 3,           /* device allocation failed in velo_create */
    VELO_ERR_DEVICE = 4,        /* a HIP runtime call failed */
    VELO_ERR_UNSUPPORTED = 5,   /* configuration not compiled in (e.g. hidden width) */
    VELO_ERR_INPUT = 6,         /* device-side validation of the hits failed */
    VELO_ERR_NOT_CALIBRATED = 7 /* fp8 context used before velo_calibrate */
} velo_status;

typedef enum {
    VELO_FP32 = 0,   /* MLP operands and state in float32 */
    VELO_BF16 = 1,   /* MLP operands bfloat16, float32 accumulation */
    VELO_FP8 = 2,    /* MLP operands OCP FP8 E4M3 with static per-tensor scales,
                        float32 accumulation; encodings stored bf16 */
    VELO_BF16X2 = 3  /* bf16 MLP weights; activations that are not stored encodings
                        (hidden layers, message sums, the classifier's input)
                        enter as two bf16 operands v = hi + lo, lo = bf16(v - hi),
                        two bf16 MFMA products; float32 accumulation; encodings
                        stored bf16 */
} velo_precision;

/* Network and capacity configuration, fixed for the life of a context. */
typedef struct {
    int32_t gnn_hidden;      /* H = n_h = n_e (Sec. 5.2); 32, 64 or 128 */
    int32_t gnn_iters;       /* message-passing steps n (Sec. 5.2); 0..16 */
    float d2_max;            /* edge iff squared distance < d2_max (Sec. 5.1) */
    int32_t k_max;           /* most edges per hit (Sec. 5.1); 1..64 */
    float edge_logit_min;    /* keep an edge iff logit >= this (0 == score 0.5) */
    int32_t precision;       /* velo_precision */
    int64_t max_hits;        /* capacity: hits per call */
    int64_t max_edges;       /* capacity: edges per call (< 2^31) */
    int32_t max_events;      /* capacity: events per call */
    int32_t max_event_hits;  /* capacity: hits of one event; (max_event_hits + 1024) ints
                                must fit one workgroup's LDS (160 KB on MI355X) */
    int32_t training;        /* 1: also allocate the training workspace (fp32 only) */
} velo_config;

/* A batch of hits.  n_events and n_hits are HOST values; n_hits must equal
 * event_offsets[n_events] (checked on the device). */
typedef struct {
    int32_t n_events;
    int64_t n_hits;
    const int32_t *event_offsets;   /* [n_events + 1], event_offsets[0] == 0 */
    const float *x, *y, *z;         /* [n_hits], mm */
    const int32_t *plane;           /* [n_hits] */
} velo_hits;

/* Per-edge and per-hit results.  Any pointer a call does not write may be
 * NULL.  n_edges receives the total edge count even when it exceeds
 * edge_capacity (then the edge arrays hold only the first edge_capacity
 * edges and velo_check returns VELO_ERR_CAPACITY). */
typedef struct {
    int32_t *labels;          /* [n_hits] track label: smallest event-local hit index of the component */
    int32_t *edge_offsets;    /* [n_events + 1] edges of event b: [edge_offsets[b], edge_offsets[b+1]) */
    int32_t *edge_src;        /* [edge_capacity] event-local source hit (lower plane) */
    int32_t *edge_dst;        /* [edge_capacity] event-local destination hit */
    float *edge_logit;        /* [edge_capacity] classifier logit; score = sigmoid(logit) */
    int64_t edge_capacity;
    int32_t *n_edges;         /* [1] total edges of the batch */
} velo_outputs;

/* Results of the triplet stage (velo_triplets).  Edge indices are
 * event-local: positions within the event's slice of the graph's edge
 * arrays.  Every pointer must be valid for the sizes given. */
typedef struct {
    int32_t *art;              /* [capacity x 2] articulations (a, b): a = A->C, b = C->B */
    int32_t *art_offsets;      /* [n_events + 1] */
    float *art_logit;          /* [capacity] articulation classifier logit */
    int32_t *elb;              /* [capacity x 2] elbows (a, b), a < b: left C->A, C->B; right A->C, B->C */
    int8_t *elb_type;          /* [capacity] 1 = left elbow, 2 = right elbow */
    int32_t *elb_offsets;      /* [n_events + 1] */
    float *elb_logit;          /* [capacity] elbow classifier logit */
    int64_t capacity;          /* pairs each of the two lists holds (<= the context's max_triplets) */
    int32_t *n_triplets;       /* [2] totals: articulations, elbows (required sizes on overflow) */
    int32_t *edge_seg;         /* [the graph's edge_capacity] segment of each kept edge (its smallest
                                  event-local edge index), -1 for edges below the cut */
    int32_t *tracks;           /* [track_capacity x 2] segments of each track; the second is -1 for a
                                  track of one segment */
    int32_t *track_offsets;    /* [n_events + 1] */
    int64_t track_capacity;
    int32_t *n_tracks;         /* [1] total tracks (required size on overflow) */
} velo_triplet_outputs;

typedef struct velo_ctx velo_ctx;

/* Number of float32 entries of the parameter blob for hidden width H and n
 * steps.  Blob layout (every Linear row-major [out x in], then its bias):
 *   norm[12] = emb_mu[3], emb_sigma[3] (over r, phi, z; Sec. 5.1 footnote),
 *              gnn_mu[3], gnn_sigma[3] (over x, y, z; Sec. 5.2)
 *   embedding [128x3] [128x128] [4x128]
 *   node encoder [Hx3] [HxH]; edge encoder [Hx2H] [HxH]
 *   for each step k: node net [Hx3H] [HxH], edge net [Hx3H] [HxH]
 *   edge classifier [HxH] [1xH]
 * Every MLP has a ReLU between its layers and none after the last.
 * Returns -1 for an unsupported shape. */
int64_t velo_param_count(int32_t gnn_hidden, int32_t gnn_iters);

/* Create a context: validates `cfg`, allocates the workspace for its
 * capacities and a parameter buffer.  *out is NULL on failure. */
velo_status velo_create(const velo_config *cfg, velo_ctx **out);

/* Free everything the context owns (waits for its work).  NULL is a no-op. */
void velo_destroy(velo_ctx *ctx);

/* Copy the float32 parameter blob (device pointer, n entries, layout above)
 * into the context and convert it for the context's precision.  Must be
 * called before any compute call; may be called again (e.g. after an
 * optimiser step) and is ordered with later work on the same stream. */
velo_status velo_set_params(velo_ctx *ctx, const float *params, int64_t n, void *stream);

/* fp8 contexts: derive the static per-tensor activation scales from a
 * calibration batch (the paper calibrates its INT8 embedding on 5,000 events,
 * Sec. 7.4).  Runs the path with bf16 operands on `hits`, records the largest
 * |value| entering every MLP layer and sets s_x = max / 448 (the largest E4M3
 * value); weight scales s_w = max |W| / 448 are set by velo_set_params, which
 * also invalidates earlier activation scales.  Compute calls on an fp8
 * context return VELO_ERR_NOT_CALIBRATED until this has been called. */
velo_status velo_calibrate(velo_ctx *ctx, const velo_hits *hits, void *stream);

/* Number of float32 entries of the triplet classifiers' parameters for
 * hidden width H (Sec. 5.3: separate classifiers for articulations and
 * elbows): for the articulation classifier, then the elbow classifier, a
 * Linear [H x 2H] + bias [H], ReLU, a Linear [1 x H] + bias [1], applied to
 * the concatenated final edge encodings [e_a || e_b].  -1: unsupported H. */
int64_t velo_triplet_param_count(int32_t gnn_hidden);

/* Enable the triplet stage (Sec. 5.3-5.4) on a context: copies the triplet
 * classifiers' parameters (device, n floats as velo_triplet_param_count
 * gives), keeps a triplet iff its logit >= triplet_logit_min, and sizes the
 * stage's workspace for max_triplets articulations and as many elbows.
 * From then on velo_gnn and velo_infer keep the final edge encodings for
 * velo_triplets (the edge classifier then runs as its own kernel).
 * n == 0 with params NULL disables the stage and frees its workspace. */
velo_status velo_set_triplet_params(velo_ctx *ctx, const float *params, int64_t n, float triplet_logit_min,
                                    int64_t max_triplets, void *stream);

/* The triplet stage on the graph of the directly preceding velo_gnn or
 * velo_infer call on this context (same hits and graph; any other call in
 * between that takes hits is refused with VELO_ERR_INVALID_ARG):
 *  1. triplets (Sec. 5.3) of the edges kept by the edge cut (logit >=
 *     edge_logit_min): for every common hit C, articulations (every kept
 *     in-edge with every kept out-edge), then left elbows (pairs of kept
 *     out-edges), then right elbows (pairs of kept in-edges); edges in
 *     ascending index order, hits in index order;
 *  2. the two triplet classifiers on [e_a || e_b] of the final edge
 *     encodings (bf16 operands in bf16 and fp8 contexts);
 *  3. tracks (Sec. 5.4): kept elbows join their edges and mark the edge
 *     spanning more planes a duplicate; kept articulations without a
 *     duplicate edge join theirs, except shared ones (whose first edge starts
 *     or whose second edge ends another such articulation); the joined edge
 *     sets are the segments; each shared articulation is a track of its two
 *     segments, every other segment a track of its own (per event: the
 *     one-segment tracks by label, then the shared articulations in order).
 * On overflow of a triplet list the totals are written and nothing else;
 * on overflow of the tracks everything but the tracks and their offsets.
 * Either way velo_check returns VELO_ERR_CAPACITY. */
velo_status velo_triplets(velo_ctx *ctx, const velo_hits *hits, const velo_outputs *graph,
                          velo_triplet_outputs *out, void *stream);

/* INT8 embedding (Sec. 7.4: the embedding network quantised to INT8 with
 * calibration, which adds a few percent of extra edges).  With scales set,
 * velo_embed and velo_infer run the embedding's second and third layers
 * (the two 128-wide-input ones) on INT8 operands, whatever the context's
 * precision: an operand v enters as q = clamp(rint(fl32(v * fl32(1/s))),
 * -127, 127) (ties to even) under its tensor's scale s, the integer products
 * are summed exactly and each layer's sum is descaled by s_x * s_w in
 * float32 before the bias.  The first layer (three inputs) stays float32.
 * scales_host = {s_x2, s_w2, s_x3, s_w3}, all positive and finite (the
 * inputs and weights of the second and third layers); NULL turns INT8 off.
 * velo_set_params turns it off too (the scales belong to the weights). */
velo_status velo_set_embed_int8(velo_ctx *ctx, const float *scales_host);

/* Calibrate and enable the INT8 embedding on a calibration batch: runs the
 * float32 embedding on `hits`, takes the largest value entering the second
 * and third layers (after their ReLU) and the largest |W| of those layers'
 * weights, sets s = max / 127 (float32; 1 for an all-zero tensor), writes the
 * four scales to scales_host (may be NULL) and enables them as
 * velo_set_embed_int8 does.  Synchronises the stream. */
velo_status velo_calibrate_embed_int8(velo_ctx *ctx, const velo_hits *hits, float *scales_host, void *stream);

/* Whole path: embedding, rough graph, GNN, edge cut, components.  Writes
 * labels, edge_offsets, edge_src, edge_dst, edge_logit and n_edges. */
velo_status velo_infer(velo_ctx *ctx, const velo_hits *hits, velo_outputs *out, void *stream);

/* Stage: embedding of every hit, emb[i * VELO_EMB_DIM + c], float32 (Sec. 5.1). */
velo_status velo_embed(velo_ctx *ctx, const velo_hits *hits, float *emb, void *stream);

/* Stage: rough graph from a given embedding (float32 [n_hits x 4]).  Writes
 * edge_offsets, edge_src, edge_dst, n_edges.  Within an event edges are
 * sorted by source hit, then destination hit.  The squared distance is
 * evaluated in float32 as d = a_c - b_c, s = d_0*d_0, s = fma(d_c, d_c, s)
 * for c = 1..3; among more than k_max candidates the k_max smallest under
 * (s, destination index) are kept (Sec. 5.1, 7.2). */
velo_status velo_build_graph(velo_ctx *ctx, const velo_hits *hits, const float *emb,
                             velo_outputs *graph, void *stream);

/* Comparison variant of velo_build_graph with the paper's neighbour search
 * (Sec. 7.2): one thread per hit loops over its candidates in index order
 * and keeps at most k_max of them, replacing the list's largest (d2, j)
 * entry when a closer candidate comes.  Same result as velo_build_graph
 * (the k_max smallest under (d2, j)); slower, since it does not spread a
 * hit's candidates over lanes.  Same arguments and errors. */
velo_status velo_build_graph_loop(velo_ctx *ctx, const velo_hits *hits, const float *emb, velo_outputs *graph,
                                  void *stream);

/* Stage: GNN edge logits (Sec. 5.2) for a given graph: reads
 * graph->edge_offsets, edge_src, edge_dst and n_edges (edges grouped by event
 * and sorted by source within an event, as velo_build_graph writes them)
 * and writes graph->edge_logit.  A graph not grouped by source, or with an
 * index outside its event, is rejected with VELO_ERR_INPUT (reported by the
 * next synchronising call). */
velo_status velo_gnn(velo_ctx *ctx, const velo_hits *hits, velo_outputs *graph, void *stream);

/* Stage: connected components of the edges with logit >= edge_logit_min
 * (Sec. 7.3), taken as undirected; reads the graph and logits of `graph` and
 * writes graph->labels. */
velo_status velo_components(velo_ctx *ctx, const velo_hits *hits, velo_outputs *graph, void *stream);

/* Comparison variant of velo_components: the paper's two plane sweeps
 * (Sec. 7.3) instead of exact components.  Labels start as the event-local
 * index; forward over planes 1 .. 25 each hit takes the smallest of its
 * label and those of the hits joined to it by kept edges from planes p-1 and
 * p-2, then backward over planes 24 .. 0 the smallest of its label and those
 * of the hits its kept edges reach on planes p+1 and p+2.  Edges that do not
 * go one or two planes forward take no part.  The result can leave one
 * component with several labels (a hit joined to two hits of an earlier
 * plane passes on only the smaller label), which is why velo_components is
 * exact instead.  Same arguments and errors as velo_components. */
velo_status velo_components_sweep(velo_ctx *ctx, const velo_hits *hits, velo_outputs *graph, void *stream);

/* velo_components without a context and without any device allocation, for
 * callers that cannot allocate memory (code under stream capture, serving
 * loops, harnesses that forbid hipMalloc).  Same validation and labels as
 * velo_components with a context whose edge cut is edge_logit_min and whose
 * max_event_hits is the argument; edge_capacity alone bounds the edges read.
 * Its working memory is a fixed device array inside the library, one per
 * GPU, held until the process ends (about 6 MB): batches of at most
 * VELO_NOALLOC_MAX_HITS hits and VELO_NOALLOC_MAX_EVENTS events, and
 * max_event_hits at most the workgroup LDS in ints (40,960 on MI355X); larger
 * ones are refused with VELO_ERR_CAPACITY before any launch.  Every call on
 * a GPU shares that array, so calls that overlap on one GPU (other streams,
 * other threads) race.  The call waits for `stream` and returns the device
 * validation result: VELO_ERR_INPUT (invalid hits or edges), VELO_ERR_CAPACITY
 * (n_edges above edge_capacity; labels then unwritten) or VELO_OK. */
#define VELO_NOALLOC_MAX_HITS (1 << 20)
#define VELO_NOALLOC_MAX_EVENTS (1 << 14)
velo_status velo_components_noalloc(const velo_hits *hits, const velo_outputs *graph, float edge_logit_min,
                                    int32_t max_event_hits, void *stream);

/* Stages of the path, for per-stage device timing. */
typedef enum {
    VELO_STAGE_PREPARE = 0,    /* validation and plane bucketing */
    VELO_STAGE_EMBED = 1,      /* embedding MLP (Sec. 5.1) */
    VELO_STAGE_KNN = 2,        /* neighbour search with top-k (Sec. 5.1, 7.2) */
    VELO_STAGE_COMPACT = 3,    /* degree scan and CSR compaction */
    VELO_STAGE_LISTS = 4,      /* incoming lists (and row pointers of a given graph) */
    VELO_STAGE_NODE_ENC = 5,   /* node encoder (Sec. 5.2) */
    VELO_STAGE_EDGE_ENC = 6,   /* edge encoder (Sec. 5.2) */
    VELO_STAGE_MESSAGES = 7,   /* scatter_add message sums, one launch per step */
    VELO_STAGE_NODE_NET = 8,   /* node network, one launch per step */
    VELO_STAGE_EDGE_NET = 9,   /* edge network, one launch per step except the last */
    VELO_STAGE_EDGE_CLS = 10,  /* last step's edge network fused with the edge classifier */
    VELO_STAGE_COMPONENTS = 11,/* edge cut and connected components (Sec. 7.3) */
    VELO_STAGE_BCE = 12,       /* training: weighted BCE and dL/dz */
    VELO_STAGE_BWD_MLP = 13,   /* training: recompute and back-propagate every MLP (dX, with the
                                  message sums' dual) */
    VELO_STAGE_BWD_DW = 14,    /* training: split-K weight gradients and their reduction */
    VELO_STAGE_BWD_GRAPH = 15, /* training: per-hit sums of dL/d(hidden) of the edge MLPs */
    VELO_STAGE_ADAM = 16,      /* training: Adam update */
    VELO_STAGE_HIT_PROJ = 17,  /* fp32 inference: per-hit first-layer products of the edge MLPs */
    VELO_STAGE_EMB_LOSS = 18,  /* embedding training: training pairs and the hinge loss (Sec. 5.1) */
    VELO_STAGE_EMB_BWD = 19,   /* embedding training: back-propagation and weight gradients */
    VELO_STAGE_TRIPLETS = 20,  /* triplet stage: triplets, their classifiers, track building */
    VELO_N_STAGES = 21
} velo_stage;

/* Enable (1) or disable (0) per-stage timing: while enabled every call
 * records a pair of HIP events around each stage launch on its stream.
 * Not for use under stream capture. */
velo_status velo_set_timing(velo_ctx *ctx, int32_t enable);

/* Synchronise the recorded events and return, per stage, the summed device
 * milliseconds (ms[VELO_N_STAGES]) and the number of timed launches
 * (launches[VELO_N_STAGES]) since the previous read; resets the sums.
 * The context holds 8192 event pairs between reads: launches beyond that are
 * not timed, and the read then still fills both arrays (timed launches only)
 * but returns VELO_ERR_CAPACITY, with the number of untimed launches in
 * velo_last_error. */
velo_status velo_read_timing(velo_ctx *ctx, double *ms_host, int64_t *launches_host);

/* ---- graph capture ---- */

typedef struct velo_graph velo_graph;

/* Capture one velo_infer call on `stream` into a HIP graph and instantiate
 * it.  The graph keeps the device pointers of `hits` and `out` (and
 * n_events/n_hits): to run it on new data, write the new hits into the same
 * buffers (same event and hit counts) and call velo_graph_launch.  Timing
 * must be off, and `stream` must not be the legacy default stream (NULL).
 * The context must stay alive while the graph is used. */
velo_status velo_graph_capture(velo_ctx *ctx, const velo_hits *hits, velo_outputs *out, void *stream,
                               velo_graph **graph);

/* Launch a captured graph on `stream` (asynchronous). */
velo_status velo_graph_launch(velo_graph *graph, void *stream);

/* Free a captured graph.  NULL is a no-op. */
void velo_graph_destroy(velo_graph *graph);

/* ---- training form (fp32 contexts created with training = 1) ---- */

/* Forward pass of the GNN for training: like velo_gnn on the given graph
 * (edges grouped by event and by source within it, event-local indices,
 * n_edges; other orders are rejected with VELO_ERR_INPUT), but with the
 * caller's float32 parameter blob `params` (device, velo_param_count entries)
 * and keeping the step-boundary hit/edge encodings, the messages and the
 * per-hit first-layer products of the edge MLPs in the context for
 * velo_train_backward.  Writes graph->edge_logit. */
velo_status velo_train_forward(velo_ctx *ctx, const velo_hits *hits, velo_outputs *graph, const float *params,
                               void *stream);

/* Weighted binary cross-entropy on n logits (training loss):
 *   loss = (1/n) sum_q w_q [softplus(z_q) - y_q z_q], w = pos_weight if y = 1 else 1,
 *   dlogit_q = w_q (sigmoid(z_q) - y_q) / n.
 * logit, y (uint8 0/1), dlogit: [n] device; loss: [1] device. */
velo_status velo_bce(velo_ctx *ctx, const float *logit, const uint8_t *y, float pos_weight, int64_t n,
                     float *loss, float *dlogit, void *stream);

/* Sigmoid focal loss on n logits, the classifier loss the paper trains with
 * (Sec. 5.2; the form of Lin et al.): p_t = sigmoid(z) if y = 1 else
 * 1 - sigmoid(z), a_t = alpha if y = 1 else 1 - alpha (alpha < 0: a_t = 1),
 *   loss = (1/n) sum_q a_t (1 - p_t)^gamma [softplus(z_q) - y_q z_q],
 *   dlogit_q = a_t (1 - p_t)^gamma [(sigmoid(z_q) - y_q) - gamma (2 y_q - 1) p_t ce_q] / n.
 * alpha <= 1, gamma >= 0 (gamma = 0 and alpha < 0 give the plain
 * cross-entropy).  logit, y (uint8 0/1), dlogit: [n] device; loss: [1] device. */
velo_status velo_focal(velo_ctx *ctx, const float *logit, const uint8_t *y, float alpha, float gamma, int64_t n,
                       float *loss, float *dlogit, void *stream);

/* Reverse-mode pass of the last velo_train_forward: given dL/dlogit (device,
 * one per edge of that graph) writes dL/dparams (device, blob-shaped; the
 * normalisation and embedding entries are zero, graph building being not
 * differentiable).  Hidden activations are recomputed from the kept
 * step-boundary states; no floating-point atomics, so it is deterministic. */
velo_status velo_train_backward(velo_ctx *ctx, const velo_hits *hits, const float *params, const float *dlogit,
                                float *dparams, void *stream);

/* One Adam step with bias correction on n float32 parameters (all device):
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps); step >= 1. */
velo_status velo_adam_step(velo_ctx *ctx, float *params, const float *grad, float *m, float *v, int64_t n, float lr,
                           float b1, float b2, float eps, int32_t step, void *stream);

/* Embedding training (Sec. 5.1, the two loss equations).  Truth of the
 * training events, all device arrays over the hits of the batch:
 *   pid    particle of each hit (>= 0; events are given without noise hits,
 *          which the paper removes from the training events),
 *   query  1 for a query hit (the caller's choice; the paper takes hits of
 *          reconstructible particles, not electrons),
 *   rnd    one uniform 32-bit draw per hit, which picks the query's random
 *          partner: candidate number floor(rnd * C / 2^32) of the C hits on
 *          planes p+1 and p+2, in index order. */
typedef struct {
    const int32_t *pid;
    const uint8_t *query;
    const uint32_t *rnd;
} velo_embed_truth;

#define VELO_EMB_TRAIN_KMAX 64   /* largest k_train accepted */

/* Loss and gradient of one embedding training step (Sec. 5.1).  Runs the
 * embedding with the caller's float32 parameter blob `params` (device), then
 * builds the training pairs of every query q: the hard negatives (the members
 * of another particle in q's bounded neighbour list, k_train nearest with
 * d2 < d2_train, ties by index, as the graph stage builds it), every genuine
 * pair (a candidate of q's particle on planes p+1, p+2) and one random pair;
 * the three lists are concatenated.  The loss is pooled over the batch:
 *   L = w_genuine * (1/N_g) sum_genuine d2 + (1/N_f) sum_fake max(0, margin - d2),
 * with d2 and the hinge decision in float32.  Writes dL/dparams for the
 * embedding entries of the blob-shaped dparams (device; every other entry
 * is left as it is), loss[3] = {L, genuine term, fake term} (device float)
 * and counts[2] = {N_g, N_f} (device int64); emb (device [N x 4], optional)
 * receives the embedding the pairs were built on.  Per-hit gradient sums are
 * accumulated in 64-bit fixed point (2^-32; a single pair's term is clamped
 * to +-1e6), so the result does not depend on the order of the pairs and is
 * bitwise reproducible.  Needs a context
 * created with training = 1 whose parameters have been set once (as every
 * call on hits does); 1 <= k_train <= VELO_EMB_TRAIN_KMAX. */
velo_status velo_embed_train_grad(velo_ctx *ctx, const velo_hits *hits, const velo_embed_truth *truth,
                                  const float *params, int32_t k_train, float d2_train, float margin,
                                  float w_genuine, float *dparams, float *loss, int64_t *counts, float *emb,
                                  void *stream);

/* Choose launch parameters and tile shapes by measurement: runs velo_infer
 * on (hits, out) under each of eight candidate configurations, times every
 * stage with HIP events and keeps, per stage, the fastest candidate for later
 * calls on this context.  Candidate k sets, for every tunable stage at once:
 *   k                          0    1    2    3    4    5    6    7
 *   MLP blocks per CU (0: by occupancy)
 *                              0    0    1    2    0    1    0    2
 *   MLP workgroup (threads)  512  512  512  512  256  256 1024 1024
 *   k-NN / message blocks per CU
 *                             16   16    4    8   32   32    8   16
 *   k-NN query hits per wavefront task
 *                             16   16    8   32    8   32   32    8
 *   XCD-blocked work mapping   0    1    1    1    1    0    0    1
 * A 1024-thread workgroup applies to the H = 128 edge encoder and edge
 * networks with 2-byte states (16 wavefronts share the LDS weights, one
 * 16-edge chunk each, and take their source hits from a work counter per
 * XCD, so those launches ignore the XCD-mapping row); elsewhere it means
 * 512.  Every candidate gives bitwise the same results.  The tunable stages are the
 * neighbour search, the edge encoder, the messages, the node and edge
 * networks and the classifier-fused edge network.
 * choice_host (optional, VELO_N_STAGES entries) receives the candidate index
 * picked per stage (0 for stages that are not tuned).  Synchronises the
 * stream. */
velo_status velo_autotune(velo_ctx *ctx, const velo_hits *hits, velo_outputs *out, void *stream,
                          int32_t *choice_host);

/* Apply given candidates of velo_autotune's table without measuring: choice_host
 * holds VELO_N_STAGES candidate indices (0..7; entries of stages that are not
 * tuned are ignored), for example a previous velo_autotune's output; NULL
 * restores the built-in launch parameters (candidate 0).  Launch parameters
 * and tile shapes change only which wavefront processes which work unit:
 * results are bitwise those of candidate 0. */
velo_status velo_set_tuning(velo_ctx *ctx, const int32_t *choice_host);

/* Synchronise `stream` and return (and clear) the error latched on the
 * device by earlier calls: VELO_OK, VELO_ERR_INPUT or VELO_ERR_CAPACITY. */
velo_status velo_check(velo_ctx *ctx, void *stream);

/* Static description of a status code: a velo_status value; any other
 * value gives "unknown status". */
const char *velo_status_str(int status);

/* Detail of the last host-side error of the context ("" if none). */
const char *velo_last_error(const velo_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* VELOGNN_H */
