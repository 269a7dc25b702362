// api.hip -- host side of the C ABI declared in include/velognn.h.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>

#include "internal.h"

namespace velo {

bool make_param_layout(int H, int iters, ParamLayout *L) {
    if (H <= 0 || iters < 0 || iters > 16) return false;
    int64_t o = 12;
    auto put = [&o](Lin &l, int out, int in) {
        l.w = o;
        l.b = o + (int64_t)out * in;
        l.out = out;
        l.in = in;
        o = l.b + out;
    };
    L->H = H;
    L->iters = iters;
    put(L->emb[0], VELO_EMB_HIDDEN, 3);
    put(L->emb[1], VELO_EMB_HIDDEN, VELO_EMB_HIDDEN);
    put(L->emb[2], VELO_EMB_DIM, VELO_EMB_HIDDEN);
    put(L->nenc[0], H, 3);
    put(L->nenc[1], H, H);
    put(L->eenc[0], H, 2 * H);
    put(L->eenc[1], H, H);
    for (int k = 0; k < iters; k++) {
        put(L->node[k][0], H, 3 * H);
        put(L->node[k][1], H, H);
        put(L->edge[k][0], H, 3 * H);
        put(L->edge[k][1], H, H);
    }
    put(L->cls[0], H, H);
    put(L->cls[1], 1, H);
    L->total = o;
    return true;
}

}  // namespace velo

using namespace velo;

namespace {

velo_status fail(velo_ctx *c, velo_status st, const char *msg) {
    if (c) c->last_error = msg;
    return st;
}

template <typename T>
bool dalloc(T **p, int64_t count) {
    if (count < 1) count = 1;
    return hipMalloc((void **)p, sizeof(T) * (size_t)count) == hipSuccess;
}

void free_ws(Workspace &w) {
    void *ptrs[] = {w.emb, w.hit_event, w.plane_off, w.deg, w.row_ptr, w.nbr, w.src_g, w.dst_g,
                    w.in_ptr, w.in_list, w.scan_tmp, w.h[0], w.h[1],
                    w.m, w.ab, w.e, w.n_edges, w.flags, w.grab, w.eoff_tmp, w.ck_h, w.ck_e, w.ck_m, w.ck_ab, w.g_sd, w.g_e[0], w.g_e[1],
                    w.g_h[0], w.g_h[1], w.g_da, w.g_r, w.g_m, w.g_part, w.g_red, w.g_loss,
                    w.scales, w.amax, w.tmp_logit, w.i8_scales, w.i8_amax, w.t_u, w.t_a1, w.t_a2, w.t_dz1, w.t_dz2, w.t_dz3,
                    w.t_nbr, w.t_deg, w.t_acc, w.t_stat, w.t_part};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    w = Workspace();
}

velo_status check_hits(velo_ctx *c, const velo_hits *h) {
    c->ws_epoch++;        // every call that takes hits may overwrite the workspace
    if (!h) return fail(c, VELO_ERR_INVALID_ARG, "hits is NULL");
    if (!c->params_set) return fail(c, VELO_ERR_INVALID_ARG, "parameters not set (velo_set_params)");
    if (h->n_events < 0 || h->n_hits < 0) return fail(c, VELO_ERR_INVALID_ARG, "negative n_events or n_hits");
    if (h->n_events > c->cfg.max_events) return fail(c, VELO_ERR_CAPACITY, "n_events exceeds max_events");
    if (h->n_hits > c->cfg.max_hits) return fail(c, VELO_ERR_CAPACITY, "n_hits exceeds max_hits");
    if (h->n_events == 0 && h->n_hits != 0) return fail(c, VELO_ERR_INVALID_ARG, "hits without events");
    if (h->n_events > 0 && !h->event_offsets) return fail(c, VELO_ERR_INVALID_ARG, "event_offsets is NULL");
    if (h->n_hits > 0 && (!h->x || !h->y || !h->z || !h->plane))
        return fail(c, VELO_ERR_INVALID_ARG, "hit coordinate or plane pointer is NULL");
    return VELO_OK;
}

velo_status device_status(velo_ctx *c, const char *where) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        char buf[256];
        snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
        c->last_error = buf;
        return VELO_ERR_DEVICE;
    }
    return VELO_OK;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        // a failed switch shows as the error of the calls that follow
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// velo_autotune's candidate configurations (listed in include/velognn.h):
// candidate k sets every tunable stage's launch parameters at once.
namespace tune {
constexpr int kCand = 8;
constexpr int mlp_cu[kCand] = {0, 0, 1, 2, 0, 1, 0, 2};        // MLP blocks per CU (0: by occupancy)
constexpr int mlp_block[kCand] = {512, 512, 512, 512, 256, 256, 1024, 1024};   // 1024: H = 128 only
constexpr int mem_cu[kCand] = {16, 16, 4, 8, 32, 32, 8, 16};   // k-NN and message blocks per CU
constexpr int knn_run[kCand] = {16, 16, 8, 32, 8, 32, 32, 8};  // query hits per k-NN wavefront task
constexpr int xcd[kCand] = {0, 1, 1, 1, 1, 0, 0, 1};
constexpr int tunable[] = {VELO_STAGE_KNN, VELO_STAGE_EDGE_ENC, VELO_STAGE_MESSAGES, VELO_STAGE_NODE_NET,
                           VELO_STAGE_EDGE_NET, VELO_STAGE_EDGE_CLS};

void apply(velo_ctx *c, int stage, int k) {
    const bool mem = stage == VELO_STAGE_KNN || stage == VELO_STAGE_MESSAGES;
    c->tune_per_cu[stage] = mem ? mem_cu[k] : mlp_cu[k];
    c->tune_xcd[stage] = xcd[k];
    c->tune_mlp_block[stage] = mem ? 0 : mlp_block[k];
    if (stage == VELO_STAGE_KNN) c->tune_knn_run = knn_run[k];
}
}  // namespace tune

}  // namespace

extern "C" {

int64_t velo_param_count(int32_t gnn_hidden, int32_t gnn_iters) {
    ParamLayout L;
    if (!make_param_layout(gnn_hidden, gnn_iters, &L)) return -1;
    return L.total;
}

const char *velo_status_str(int s) {
    switch (s) {
        case VELO_OK: return "ok";
        case VELO_ERR_INVALID_ARG: return "invalid argument";
        case VELO_ERR_CAPACITY: return "capacity exceeded";
        case VELO_ERR_OOM: return "device out of memory";
        case VELO_ERR_DEVICE: return "HIP runtime error";
        case VELO_ERR_UNSUPPORTED: return "unsupported configuration";
        case VELO_ERR_INPUT: return "invalid input hits (device validation)";
        case VELO_ERR_NOT_CALIBRATED: return "fp8 activation scales not calibrated";
    }
    return "unknown status";
}

const char *velo_last_error(const velo_ctx *c) { return c ? c->last_error.c_str() : "null context"; }

velo_status velo_create(const velo_config *cfg, velo_ctx **out) {
    if (!out) return VELO_ERR_INVALID_ARG;
    *out = nullptr;
    if (!cfg) return VELO_ERR_INVALID_ARG;
    const velo_config &k = *cfg;
    if (!gnn_supported(k.gnn_hidden, k.precision)) return VELO_ERR_UNSUPPORTED;
    if (k.training && !train_supported(k.gnn_hidden, k.precision)) return VELO_ERR_UNSUPPORTED;
    if (k.gnn_iters < 0 || k.gnn_iters > 16 || k.k_max < 1 || k.k_max > 64 || k.max_hits < 0 ||
        k.max_edges < 0 || k.max_events < 0 || k.max_event_hits < 0 || !(k.d2_max >= 0.f))
        return VELO_ERR_INVALID_ARG;
    if (k.max_edges >= (int64_t)1 << 31 || k.max_hits * (int64_t)k.k_max >= (int64_t)1 << 31)
        return VELO_ERR_UNSUPPORTED;
    velo_ctx *c = new (std::nothrow) velo_ctx();
    if (!c) return VELO_ERR_OOM;
    c->cfg = k;
    make_param_layout(k.gnn_hidden, k.gnn_iters, &c->layout);
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return VELO_ERR_DEVICE;
    }
    int ncu = 0, lds = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess) {
        delete c;
        return VELO_ERR_DEVICE;
    }
    c->n_cu = ncu > 0 ? ncu : 1;
    c->lds_max = (size_t)lds;
    // one event's hits must fit the LDS of one workgroup (lists, components)
    if (((size_t)k.max_event_hits + 1024) * sizeof(int) > c->lds_max) {
        delete c;
        return VELO_ERR_UNSUPPORTED;
    }
    const int64_t N = k.max_hits, E = k.max_edges, B = k.max_events, H = k.gnn_hidden;
    const int64_t sb = (int64_t)state_bytes(k.precision);
    Workspace &w = c->ws;
    w.scan_tmp_len = (std::max<int64_t>(N, E) + 2047) / 2048 + 1;
    bool ok = dalloc(&c->params, c->layout.total) && dalloc(&w.emb, N * 4) && dalloc(&w.hit_event, N) &&
              dalloc(&w.plane_off, B * kPlaneSlots) && dalloc(&w.deg, N) && dalloc(&w.row_ptr, N + 1) &&
              dalloc(&w.nbr, N * k.k_max) && dalloc(&w.src_g, E) && dalloc(&w.dst_g, E) &&
              dalloc(&w.in_ptr, N + 1) &&
              dalloc(&w.in_list, E) && dalloc(&w.scan_tmp, w.scan_tmp_len) &&
              dalloc((char **)&w.h[0], N * H * sb) && dalloc((char **)&w.h[1], N * H * sb) &&
              dalloc(&w.m, N * 2 * H) && dalloc(&w.ab, N * 2 * H) && dalloc((char **)&w.e, E * H * sb) && dalloc(&w.n_edges, 1) &&
              dalloc(&w.flags, 1) && dalloc(&w.grab, kXcds * 32) &&
              dalloc(&w.eoff_tmp, B + 1) && dalloc(&w.i8_scales, 4) && dalloc(&w.i8_amax, 2);
    if (ok && k.precision == VELO_FP8) {
        const int ns = n_slots(k.gnn_iters);
        ok = dalloc(&w.scales, 4 * ns) && dalloc(&w.amax, 2 * ns) && dalloc(&w.tmp_logit, E);
        if (ok) {
            std::vector<float> ones(4 * ns, 1.f);
            ok = hipMemcpy(w.scales, ones.data(), sizeof(float) * 4 * ns, hipMemcpyHostToDevice) == hipSuccess;
        }
    }
    if (ok && k.training) {
        const int64_t it = k.gnn_iters, R = std::max<int64_t>(N, E);
        ok = dalloc((char **)&w.ck_h, (it + 1) * N * H * sb) && dalloc((char **)&w.ck_e, (it + 1) * E * H * sb) &&
             dalloc(&w.ck_m, std::max<int64_t>(it, 1) * N * 2 * H) && dalloc(&w.ck_ab, (it + 1) * N * 2 * H) &&
             dalloc(&w.g_sd, N * 2 * H) && dalloc(&w.g_e[0], E * H) &&
             dalloc(&w.g_e[1], E * H) && dalloc(&w.g_h[0], N * H) && dalloc(&w.g_h[1], N * H) &&
             dalloc(&w.g_da, R * H) && dalloc(&w.g_r, R * H) &&
             dalloc(&w.g_m, N * 2 * H) && dalloc(&w.g_part, (int64_t)train_part_floats(k.gnn_hidden)) &&
             dalloc(&w.g_red, (int64_t)train_red_floats(k.gnn_hidden)) &&
             dalloc(&w.g_loss, 256);
        // embedding training
        const int64_t Ce = VELO_EMB_HIDDEN;
        ok = ok && dalloc(&w.t_u, N * 4) && dalloc(&w.t_a1, N * Ce) && dalloc(&w.t_a2, N * Ce) &&
             dalloc(&w.t_dz1, N * Ce) && dalloc(&w.t_dz2, N * Ce) && dalloc(&w.t_dz3, N * 4) &&
             dalloc(&w.t_nbr, N * VELO_EMB_TRAIN_KMAX) && dalloc(&w.t_deg, N) && dalloc(&w.t_acc, N * 8) &&
             dalloc(&w.t_stat, 4) &&
             dalloc(&w.t_part, emb_train_chunks(N) * (Ce * 3 + Ce + Ce * Ce + Ce + VELO_EMB_DIM * Ce + VELO_EMB_DIM));
    }
    if (!ok) {
        (void)hipGetLastError();   // clear the failed allocation's error
        free_ws(w);
        if (c->params) (void)hipFree(c->params);
        delete c;
        return VELO_ERR_OOM;
    }
    if (hipMemset(w.flags, 0, sizeof(unsigned)) != hipSuccess || hipMemset(w.n_edges, 0, sizeof(int)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        free_ws(w);
        (void)hipFree(c->params);
        delete c;
        return VELO_ERR_DEVICE;
    }
    *out = c;
    return VELO_OK;
}

static void free_triplet_ws(TripletWs &T);

void velo_destroy(velo_ctx *c) {
    if (!c) return;
    DeviceGuard g(c->device);
    (void)hipDeviceSynchronize();   // teardown goes on whatever an earlier failure left
    for (auto &e : c->ev_pool) {
        (void)hipEventDestroy(e.start);
        (void)hipEventDestroy(e.stop);
    }
    free_ws(c->ws);
    free_triplet_ws(c->tri);
    if (c->params) (void)hipFree(c->params);
    delete c;
}

velo_status velo_set_params(velo_ctx *c, const float *params, int64_t n, void *stream) {
    if (!c) return VELO_ERR_INVALID_ARG;
    if (!params) return fail(c, VELO_ERR_INVALID_ARG, "params is NULL");
    if (n != c->layout.total) return fail(c, VELO_ERR_INVALID_ARG, "parameter count does not match the layout");
    DeviceGuard g(c->device);
    if (hipMemcpyAsync(c->params, params, sizeof(float) * n, hipMemcpyDeviceToDevice, (hipStream_t)stream) !=
        hipSuccess)
        return fail(c, VELO_ERR_DEVICE, "parameter copy failed");
    c->params_set = true;
    c->emb_int8 = false;          // INT8 embedding scales belong to the previous parameters
    if (c->cfg.precision == VELO_FP8) {
        launch_weight_scales(c, (hipStream_t)stream);
        c->calibrated = false;    // activation scales belong to the previous parameters
    }
    return device_status(c, "velo_set_params");
}

velo_status velo_calibrate(velo_ctx *c, const velo_hits *h, void *stream) {
    if (!c) return VELO_ERR_INVALID_ARG;
    if (c->cfg.precision != VELO_FP8) return fail(c, VELO_ERR_UNSUPPORTED, "calibration is for fp8 contexts");
    velo_status st = check_hits(c, h);
    if (st) return st;
    DeviceGuard gd(c->device);
    hipStream_t s = (hipStream_t)stream;
    Workspace &w = c->ws;
    launch_fill((int *)w.amax, 0, 2 * n_slots(c->cfg.gnn_iters), s);
    velo_outputs g{};
    g.edge_offsets = w.eoff_tmp;
    g.edge_capacity = c->cfg.max_edges;
    launch_prepare(c, h, s);
    launch_embed(c, h, w.emb, true, s);
    launch_knn(c, h, w.emb, s);
    launch_compact(c, h, &g, s);
    launch_in_lists_plane(c, h, s);
    launch_gnn(c, h, w.tmp_logit, c->params, false, true, s);
    launch_act_scales(c, s);
    c->calibrated = true;
    return device_status(c, "velo_calibrate");
}

velo_status velo_set_embed_int8(velo_ctx *c, const float *scales) {
    if (!c) return VELO_ERR_INVALID_ARG;
    if (!scales) {
        c->emb_int8 = false;
        return VELO_OK;
    }
    for (int i = 0; i < 4; i++)
        if (!(scales[i] > 0.f) || !std::isfinite(scales[i]))
            return fail(c, VELO_ERR_INVALID_ARG, "INT8 embedding scales must be positive and finite");
    if (!c->params_set) return fail(c, VELO_ERR_INVALID_ARG, "parameters not set (velo_set_params)");
    DeviceGuard gd(c->device);
    if (hipMemcpy(c->ws.i8_scales, scales, 4 * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return fail(c, VELO_ERR_DEVICE, "copy of the INT8 scales failed");
    c->emb_int8 = true;
    return VELO_OK;
}

velo_status velo_calibrate_embed_int8(velo_ctx *c, const velo_hits *h, float *scales, void *stream) {
    if (!c) return VELO_ERR_INVALID_ARG;
    velo_status st = check_hits(c, h);
    if (st) return st;
    DeviceGuard gd(c->device);
    hipStream_t s = (hipStream_t)stream;
    Workspace &w = c->ws;
    launch_fill((int *)w.i8_amax, 0, 2, s);
    launch_prepare(c, h, s);
    launch_embed_int8_amax(c, h, w.emb, s);
    if ((st = device_status(c, "velo_calibrate_embed_int8"))) return st;
    float amax[2];
    const ParamLayout &L = c->layout;
    std::vector<float> w2((size_t)L.emb[1].out * L.emb[1].in), w3((size_t)L.emb[2].out * L.emb[2].in);
    if (hipMemcpyAsync(amax, w.i8_amax, sizeof amax, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(w2.data(), c->params + L.emb[1].w, sizeof(float) * w2.size(), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipMemcpyAsync(w3.data(), c->params + L.emb[2].w, sizeof(float) * w3.size(), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(c, VELO_ERR_DEVICE, "velo_calibrate_embed_int8: copies failed");
    unsigned flags = 0;
    if (hipMemcpy(&flags, w.flags, sizeof flags, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, VELO_ERR_DEVICE, "velo_calibrate_embed_int8: flag read failed");
    if (flags & kErrInput) return fail(c, VELO_ERR_INPUT, "velo_calibrate_embed_int8: invalid calibration hits");
    float wmax[2] = {0.f, 0.f};
    for (float v : w2) wmax[0] = std::max(wmax[0], std::fabs(v));
    for (float v : w3) wmax[1] = std::max(wmax[1], std::fabs(v));
    // s = max |value| / 127 in float32; a tensor that is all zeros takes s = 1
    auto scale = [](float m) { return m > 0.f ? m / 127.f : 1.f; };
    float sc[4] = {scale(amax[0]), scale(wmax[0]), scale(amax[1]), scale(wmax[1])};
    if (scales) memcpy(scales, sc, sizeof sc);
    return velo_set_embed_int8(c, sc);
}

velo_status velo_embed(velo_ctx *c, const velo_hits *h, float *emb, void *stream) {
    if (!c) return VELO_ERR_INVALID_ARG;
    if (c->cfg.precision == VELO_FP8 && !c->calibrated)
        return fail(c, VELO_ERR_NOT_CALIBRATED, "fp8 context: call velo_calibrate first");
    velo_status st = check_hits(c, h);
    if (st) return st;
    if (h->n_hits > 0 && !emb) return fail(c, VELO_ERR_INVALID_ARG, "emb is NULL");
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    { StageTimer t(c, VELO_STAGE_PREPARE, s); launch_prepare(c, h, s); }
    { StageTimer t(c, VELO_STAGE_EMBED, s); launch_embed(c, h, emb, false, s); }
    return device_status(c, "velo_embed");
}

static velo_status graph_args(velo_ctx *c, const velo_hits *h, const velo_outputs *g) {
    if (!g) return fail(c, VELO_ERR_INVALID_ARG, "graph/outputs is NULL");
    if (h->n_events > 0 && !g->edge_offsets) return fail(c, VELO_ERR_INVALID_ARG, "edge_offsets is NULL");
    if (!g->n_edges) return fail(c, VELO_ERR_INVALID_ARG, "n_edges is NULL");
    if (g->edge_capacity < 0) return fail(c, VELO_ERR_INVALID_ARG, "negative edge_capacity");
    if (g->edge_capacity > 0 && (!g->edge_src || !g->edge_dst))
        return fail(c, VELO_ERR_INVALID_ARG, "edge_src/edge_dst is NULL");
    return VELO_OK;
}

velo_status velo_build_graph(velo_ctx *c, const velo_hits *h, const float *emb, velo_outputs *g, void *stream) {
    if (!c) return VELO_ERR_INVALID_ARG;
    velo_status st = check_hits(c, h);
    if (st) return st;
    if ((st = graph_args(c, h, g))) return st;
    if (h->n_hits > 0 && !emb) return fail(c, VELO_ERR_INVALID_ARG, "emb is NULL");
    DeviceGuard gd(c->device);
    hipStream_t s = (hipStream_t)stream;
    { StageTimer t(c, VELO_STAGE_PREPARE, s); launch_prepare(c, h, s); }
    { StageTimer t(c, VELO_STAGE_KNN, s); launch_knn(c, h, emb, s); }
    { StageTimer t(c, VELO_STAGE_COMPACT, s); launch_compact(c, h, g, s); }
    return device_status(c, "velo_build_graph");
}

velo_status velo_build_graph_loop(velo_ctx *c, const velo_hits *h, const float *emb, velo_outputs *g,
                                  void *stream) {
    if (!c) return VELO_ERR_INVALID_ARG;
    velo_status st = check_hits(c, h);
    if (st) return st;
    if ((st = graph_args(c, h, g))) return st;
    if (h->n_hits > 0 && !emb) return fail(c, VELO_ERR_INVALID_ARG, "emb is NULL");
    DeviceGuard gd(c->device);
    hipStream_t s = (hipStream_t)stream;
    { StageTimer t(c, VELO_STAGE_PREPARE, s); launch_prepare(c, h, s); }
    { StageTimer t(c, VELO_STAGE_KNN, s); launch_knn_loop(c, h, emb, s); }
    { StageTimer t(c, VELO_STAGE_COMPACT, s); launch_compact(c, h, g, s); }
    return device_status(c, "velo_build_graph_loop");
}

velo_status velo_gnn(velo_ctx *c, const velo_hits *h, velo_outputs *g, void *stream) {
    if (!c) return VELO_ERR_INVALID_ARG;
    if (c->cfg.precision == VELO_FP8 && !c->calibrated)
        return fail(c, VELO_ERR_NOT_CALIBRATED, "fp8 context: call velo_calibrate first");
    velo_status st = check_hits(c, h);
    if (st) return st;
    if ((st = graph_args(c, h, g))) return st;
    if (g->edge_capacity > 0 && !g->edge_logit) return fail(c, VELO_ERR_INVALID_ARG, "edge_logit is NULL");
    DeviceGuard gd(c->device);
    hipStream_t s = (hipStream_t)stream;
    { StageTimer t(c, VELO_STAGE_PREPARE, s); launch_prepare(c, h, s); }
    { StageTimer t(c, VELO_STAGE_COMPACT, s); launch_globalise(c, h, g, s); }
    {
        StageTimer t(c, VELO_STAGE_LISTS, s);
        launch_row_ptr(c, h, g, s);
        launch_in_lists_plane(c, h, s);
    }
    launch_gnn(c, h, g->edge_logit, c->params, false, false, s);
    st = device_status(c, "velo_gnn");
    if (!st && c->tri_set) c->tri_epoch = c->ws_epoch;
    return st;
}

velo_status velo_components(velo_ctx *c, const velo_hits *h, velo_outputs *g, void *stream) {
    if (!c) return VELO_ERR_INVALID_ARG;
    velo_status st = check_hits(c, h);
    if (st) return st;
    if ((st = graph_args(c, h, g))) return st;
    if (h->n_hits > 0 && !g->labels) return fail(c, VELO_ERR_INVALID_ARG, "labels is NULL");
    if (g->edge_capacity > 0 && !g->edge_logit) return fail(c, VELO_ERR_INVALID_ARG, "edge_logit is NULL");
    DeviceGuard gd(c->device);
    hipStream_t s = (hipStream_t)stream;
    { StageTimer t(c, VELO_STAGE_PREPARE, s); launch_prepare(c, h, s); }
    { StageTimer t(c, VELO_STAGE_COMPACT, s); launch_globalise(c, h, g, s); }
    { StageTimer t(c, VELO_STAGE_COMPONENTS, s); launch_components(c, h, g, s); }
    return device_status(c, "velo_components");
}

velo_status velo_components_sweep(velo_ctx *c, const velo_hits *h, velo_outputs *g, void *stream) {
    if (!c) return VELO_ERR_INVALID_ARG;
    velo_status st = check_hits(c, h);
    if (st) return st;
    if ((st = graph_args(c, h, g))) return st;
    if (h->n_hits > 0 && !g->labels) return fail(c, VELO_ERR_INVALID_ARG, "labels is NULL");
    if (g->edge_capacity > 0 && !g->edge_logit) return fail(c, VELO_ERR_INVALID_ARG, "edge_logit is NULL");
    DeviceGuard gd(c->device);
    hipStream_t s = (hipStream_t)stream;
    { StageTimer t(c, VELO_STAGE_PREPARE, s); launch_prepare(c, h, s); }
    { StageTimer t(c, VELO_STAGE_COMPACT, s); launch_globalise(c, h, g, s); }
    { StageTimer t(c, VELO_STAGE_COMPONENTS, s); launch_components_sweep(c, h, g, s); }
    return device_status(c, "velo_components_sweep");
}

velo_status velo_infer(velo_ctx *c, const velo_hits *h, velo_outputs *o, void *stream) {
    if (!c) return VELO_ERR_INVALID_ARG;
    if (c->cfg.precision == VELO_FP8 && !c->calibrated)
        return fail(c, VELO_ERR_NOT_CALIBRATED, "fp8 context: call velo_calibrate first");
    velo_status st = check_hits(c, h);
    if (st) return st;
    if ((st = graph_args(c, h, o))) return st;
    if (h->n_hits > 0 && !o->labels) return fail(c, VELO_ERR_INVALID_ARG, "labels is NULL");
    if (o->edge_capacity > 0 && !o->edge_logit) return fail(c, VELO_ERR_INVALID_ARG, "edge_logit is NULL");
    DeviceGuard gd(c->device);
    hipStream_t s = (hipStream_t)stream;
    { StageTimer t(c, VELO_STAGE_PREPARE, s); launch_prepare(c, h, s); }
    { StageTimer t(c, VELO_STAGE_EMBED, s); launch_embed(c, h, c->ws.emb, false, s); }
    { StageTimer t(c, VELO_STAGE_KNN, s); launch_knn(c, h, c->ws.emb, s); }
    { StageTimer t(c, VELO_STAGE_COMPACT, s); launch_compact(c, h, o, s); }
    { StageTimer t(c, VELO_STAGE_LISTS, s); launch_in_lists_plane(c, h, s); }
    launch_gnn(c, h, o->edge_logit, c->params, false, false, s);
    { StageTimer t(c, VELO_STAGE_COMPONENTS, s); launch_components(c, h, o, s); }
    st = device_status(c, "velo_infer");
    if (!st && c->tri_set) c->tri_epoch = c->ws_epoch;
    return st;
}

int64_t velo_triplet_param_count(int32_t H) {
    if (!triplet_supported(H)) return -1;
    return 2 * ((int64_t)2 * H * H + 2 * H + 1);
}

static void free_triplet_ws(TripletWs &T) {
    void *ptrs[] = {T.params, T.cnt_art, T.cnt_elb, T.art_ptr, T.elb_ptr, T.art_g, T.elb_g, T.n_int, T.par,
                    T.first, T.second, T.dup, T.touched, T.single, T.single_ptr, T.shared, T.shared_ptr,
                    T.scan_tmp};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    T = TripletWs();
}

velo_status velo_set_triplet_params(velo_ctx *c, const float *params, int64_t n, float logit_min,
                                    int64_t max_triplets, void *stream) {
    if (!c) return VELO_ERR_INVALID_ARG;
    DeviceGuard gd(c->device);
    if (!params && n == 0) {
        const bool synced = hipDeviceSynchronize() == hipSuccess;
        free_triplet_ws(c->tri);
        c->tri_set = false;
        return synced ? VELO_OK : fail(c, VELO_ERR_DEVICE, "hipDeviceSynchronize failed");
    }
    if (!triplet_supported(c->cfg.gnn_hidden))
        return fail(c, VELO_ERR_UNSUPPORTED, "triplet stage: unsupported hidden width");
    if (!params || n != velo_triplet_param_count(c->cfg.gnn_hidden))
        return fail(c, VELO_ERR_INVALID_ARG, "triplet parameter count does not match the hidden width");
    if (!std::isfinite(logit_min)) return fail(c, VELO_ERR_INVALID_ARG, "triplet_logit_min must be finite");
    if (max_triplets < 0 || max_triplets >= ((int64_t)1 << 30))
        return fail(c, VELO_ERR_INVALID_ARG, "max_triplets must be in 0 .. 2^30 - 1");
    TripletWs &T = c->tri;
    if (!T.params || T.cap != max_triplets) {
        if (hipDeviceSynchronize() != hipSuccess) return fail(c, VELO_ERR_DEVICE, "hipDeviceSynchronize failed");
        free_triplet_ws(T);
        const int64_t N = c->cfg.max_hits, E = c->cfg.max_edges, Tc = max_triplets;
        const int64_t big = std::max(std::max(N, E), Tc);
        const bool ok = dalloc(&T.params, n) && dalloc(&T.cnt_art, N) && dalloc(&T.cnt_elb, N) &&
                        dalloc(&T.art_ptr, N + 1) && dalloc(&T.elb_ptr, N + 1) && dalloc(&T.art_g, 2 * Tc) &&
                        dalloc(&T.elb_g, 2 * Tc) && dalloc(&T.n_int, 4) && dalloc(&T.par, E) &&
                        dalloc(&T.first, E) && dalloc(&T.second, E) && dalloc(&T.dup, E) &&
                        dalloc(&T.touched, E) && dalloc(&T.single, E) && dalloc(&T.single_ptr, E + 1) &&
                        dalloc(&T.shared, Tc) && dalloc(&T.shared_ptr, Tc + 1) &&
                        dalloc(&T.scan_tmp, scan_tmp_ints(big));
        if (!ok) {
            free_triplet_ws(T);
            c->tri_set = false;
            return fail(c, VELO_ERR_OOM, "triplet workspace allocation failed");
        }
        T.cap = max_triplets;
    }
    if (hipMemcpyAsync(T.params, params, sizeof(float) * n, hipMemcpyDeviceToDevice, (hipStream_t)stream) !=
        hipSuccess)
        return fail(c, VELO_ERR_DEVICE, "triplet parameter copy failed");
    c->tri_cut = logit_min;
    c->tri_set = true;
    c->tri_epoch = 0;         // the next GNN pass keeps its final edge states
    return VELO_OK;
}

velo_status velo_triplets(velo_ctx *c, const velo_hits *h, const velo_outputs *g, velo_triplet_outputs *t,
                          void *stream) {
    if (!c) return VELO_ERR_INVALID_ARG;
    if (!c->tri_set) return fail(c, VELO_ERR_INVALID_ARG, "triplet parameters not set (velo_set_triplet_params)");
    const bool follows = c->tri_epoch != 0 && c->tri_epoch == c->ws_epoch;
    velo_status st = check_hits(c, h);
    if (st) return st;
    if (!follows)
        return fail(c, VELO_ERR_INVALID_ARG,
                    "velo_triplets must directly follow velo_gnn or velo_infer on the same hits and graph");
    c->tri_epoch = c->ws_epoch;    // a repeated call still sees the same states
    if ((st = graph_args(c, h, g))) return st;
    if (g->edge_capacity > 0 && !g->edge_logit) return fail(c, VELO_ERR_INVALID_ARG, "edge_logit is NULL");
    if (!t) return fail(c, VELO_ERR_INVALID_ARG, "triplet outputs are NULL");
    if (t->capacity < 0 || t->capacity > c->tri.cap)
        return fail(c, VELO_ERR_INVALID_ARG, "triplet capacity must be in 0 .. max_triplets of the context");
    if (t->track_capacity < 0) return fail(c, VELO_ERR_INVALID_ARG, "negative track_capacity");
    if (!t->n_triplets || !t->n_tracks) return fail(c, VELO_ERR_INVALID_ARG, "n_triplets / n_tracks is NULL");
    if (h->n_events > 0 && (!t->art_offsets || !t->elb_offsets || !t->track_offsets))
        return fail(c, VELO_ERR_INVALID_ARG, "triplet offset arrays are NULL");
    if (t->capacity > 0 && (!t->art || !t->art_logit || !t->elb || !t->elb_type || !t->elb_logit))
        return fail(c, VELO_ERR_INVALID_ARG, "triplet list arrays are NULL");
    if (g->edge_capacity > 0 && !t->edge_seg) return fail(c, VELO_ERR_INVALID_ARG, "edge_seg is NULL");
    if (t->track_capacity > 0 && !t->tracks) return fail(c, VELO_ERR_INVALID_ARG, "tracks is NULL");
    DeviceGuard gd(c->device);
    hipStream_t s = (hipStream_t)stream;
    {
        StageTimer tm(c, VELO_STAGE_TRIPLETS, s);
        launch_triplets(c, h, g, t, s);
    }
    return device_status(c, "velo_triplets");
}

velo_status velo_set_timing(velo_ctx *c, int32_t enable) {
    if (!c) return VELO_ERR_INVALID_ARG;
    DeviceGuard gd(c->device);
    if (enable && c->ev_pool.empty()) {
        c->ev_pool.resize(8192);
        for (auto &e : c->ev_pool) {
            if (hipEventCreate(&e.start) != hipSuccess || hipEventCreate(&e.stop) != hipSuccess)
                return fail(c, VELO_ERR_DEVICE, "hipEventCreate failed");
        }
    }
    c->timing = enable != 0;
    return VELO_OK;
}

velo_status velo_read_timing(velo_ctx *c, double *ms, int64_t *launches) {
    if (!c || !ms || !launches) return VELO_ERR_INVALID_ARG;
    DeviceGuard gd(c->device);
    for (size_t i = 0; i < c->ev_used; i++) {
        StageEvents &e = c->ev_pool[i];
        if (hipEventSynchronize(e.stop) != hipSuccess) return fail(c, VELO_ERR_DEVICE, "hipEventSynchronize failed");
        float t = 0.f;
        if (hipEventElapsedTime(&t, e.start, e.stop) != hipSuccess)
            return fail(c, VELO_ERR_DEVICE, "hipEventElapsedTime failed");
        c->stage_ms[e.stage] += t;
        c->stage_launches[e.stage] += 1;
    }
    c->ev_used = 0;
    for (int k = 0; k < VELO_N_STAGES; k++) {
        ms[k] = c->stage_ms[k];
        launches[k] = c->stage_launches[k];
        c->stage_ms[k] = 0;
        c->stage_launches[k] = 0;
    }
    if (c->ev_dropped) {
        char msg[160];
        snprintf(msg, sizeof msg,
                 "%lld stage launches were not timed (the pool holds %zu event pairs between reads); "
                 "the sums returned cover the timed launches only",
                 (long long)c->ev_dropped, c->ev_pool.size());
        c->ev_dropped = 0;
        return fail(c, VELO_ERR_CAPACITY, msg);
    }
    return VELO_OK;
}

}  // extern "C"

struct velo_graph {
    velo_ctx *ctx = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

velo_status velo_graph_capture(velo_ctx *c, const velo_hits *h, velo_outputs *o, void *stream, velo_graph **out) {
    if (!c || !out) return VELO_ERR_INVALID_ARG;
    *out = nullptr;
    if (c->timing) return fail(c, VELO_ERR_INVALID_ARG, "disable timing before capturing a graph");
    if (!stream) return fail(c, VELO_ERR_INVALID_ARG, "the legacy default stream cannot be captured");
    DeviceGuard gd(c->device);
    hipStream_t s = (hipStream_t)stream;
    // one eager call first: argument checks, one-time kernel attributes and occupancy queries
    velo_status st = velo_infer(c, h, o, stream);
    if (st) return st;
    if (hipStreamSynchronize(s) != hipSuccess) return fail(c, VELO_ERR_DEVICE, "stream synchronisation failed");
    velo_graph *g = new (std::nothrow) velo_graph();
    if (!g) return VELO_ERR_OOM;
    g->ctx = c;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        delete g;
        return fail(c, VELO_ERR_DEVICE, "hipStreamBeginCapture failed");
    }
    st = velo_infer(c, h, o, stream);
    const hipError_t e = hipStreamEndCapture(s, &g->graph);
    if (st || e != hipSuccess || hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        (void)hipGetLastError();   // clear the capture's error
        return st ? st : fail(c, VELO_ERR_DEVICE, "graph capture or instantiation failed");
    }
    *out = g;
    return VELO_OK;
}

velo_status velo_graph_launch(velo_graph *g, void *stream) {
    if (!g) return VELO_ERR_INVALID_ARG;
    DeviceGuard gd(g->ctx->device);
    if (hipGraphLaunch(g->exec, (hipStream_t)stream) != hipSuccess) return fail(g->ctx, VELO_ERR_DEVICE, "hipGraphLaunch failed");
    return VELO_OK;
}

void velo_graph_destroy(velo_graph *g) {
    if (!g) return;
    DeviceGuard gd(g->ctx->device);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

velo_status velo_train_forward(velo_ctx *c, const velo_hits *h, velo_outputs *g, const float *params, void *stream) {
    if (!c) return VELO_ERR_INVALID_ARG;
    if (!c->cfg.training) return fail(c, VELO_ERR_UNSUPPORTED, "context created without training = 1");
    velo_status st = check_hits(c, h);
    if (st) return st;
    if ((st = graph_args(c, h, g))) return st;
    if (!params) return fail(c, VELO_ERR_INVALID_ARG, "params is NULL");
    if (g->edge_capacity > 0 && !g->edge_logit) return fail(c, VELO_ERR_INVALID_ARG, "edge_logit is NULL");
    DeviceGuard gd(c->device);
    hipStream_t s = (hipStream_t)stream;
    { StageTimer t(c, VELO_STAGE_PREPARE, s); launch_prepare(c, h, s); }
    { StageTimer t(c, VELO_STAGE_COMPACT, s); launch_globalise(c, h, g, s); }
    {
        StageTimer t(c, VELO_STAGE_LISTS, s);
        launch_row_ptr(c, h, g, s);
        launch_in_lists_plane(c, h, s);
    }
    launch_gnn(c, h, g->edge_logit, params, true, false, s);
    c->train_ready = true;
    return device_status(c, "velo_train_forward");
}

velo_status velo_bce(velo_ctx *c, const float *logit, const uint8_t *y, float pos_weight, int64_t n, float *loss,
                     float *dlogit, void *stream) {
    if (!c) return VELO_ERR_INVALID_ARG;
    if (!c->cfg.training) return fail(c, VELO_ERR_UNSUPPORTED, "context created without training = 1");
    if (n < 0 || !loss || (n > 0 && (!logit || !y || !dlogit))) return fail(c, VELO_ERR_INVALID_ARG, "velo_bce arguments");
    DeviceGuard gd(c->device);
    {
        StageTimer t(c, VELO_STAGE_BCE, (hipStream_t)stream);
        launch_bce(c, logit, y, pos_weight, n, loss, dlogit, (hipStream_t)stream);
    }
    return device_status(c, "velo_bce");
}

velo_status velo_focal(velo_ctx *c, const float *logit, const uint8_t *y, float alpha, float gamma, int64_t n,
                       float *loss, float *dlogit, void *stream) {
    if (!c) return VELO_ERR_INVALID_ARG;
    if (!c->cfg.training) return fail(c, VELO_ERR_UNSUPPORTED, "context created without training = 1");
    if (n < 0 || !loss || (n > 0 && (!logit || !y || !dlogit)))
        return fail(c, VELO_ERR_INVALID_ARG, "velo_focal arguments");
    if (!std::isfinite(alpha) || alpha > 1.f || !std::isfinite(gamma) || gamma < 0.f)
        return fail(c, VELO_ERR_INVALID_ARG, "velo_focal: alpha must be <= 1 (negative: none), gamma >= 0");
    DeviceGuard gd(c->device);
    {
        StageTimer t(c, VELO_STAGE_BCE, (hipStream_t)stream);
        launch_focal(c, logit, y, alpha, gamma, n, loss, dlogit, (hipStream_t)stream);
    }
    return device_status(c, "velo_focal");
}

velo_status velo_train_backward(velo_ctx *c, const velo_hits *h, const float *params, const float *dlogit,
                                float *dparams, void *stream) {
    if (!c) return VELO_ERR_INVALID_ARG;
    if (!c->cfg.training) return fail(c, VELO_ERR_UNSUPPORTED, "context created without training = 1");
    if (!c->train_ready) return fail(c, VELO_ERR_INVALID_ARG, "velo_train_backward needs a velo_train_forward first");
    velo_status st = check_hits(c, h);
    if (st) return st;
    if (!params || !dlogit || !dparams) return fail(c, VELO_ERR_INVALID_ARG, "params/dlogit/dparams is NULL");
    DeviceGuard gd(c->device);
    launch_gnn_backward(c, h, params, dlogit, dparams, (hipStream_t)stream);
    return device_status(c, "velo_train_backward");
}

velo_status velo_adam_step(velo_ctx *c, float *params, const float *grad, float *m, float *v, int64_t n, float lr,
                           float b1, float b2, float eps, int32_t step, void *stream) {
    if (!c) return VELO_ERR_INVALID_ARG;
    if (n < 0 || step < 1 || (n > 0 && (!params || !grad || !m || !v)))
        return fail(c, VELO_ERR_INVALID_ARG, "velo_adam_step arguments");
    DeviceGuard gd(c->device);
    if (n > 0) {
        StageTimer t(c, VELO_STAGE_ADAM, (hipStream_t)stream);
        launch_adam(params, grad, m, v, n, lr, b1, b2, eps, step, (hipStream_t)stream);
    }
    return device_status(c, "velo_adam_step");
}

velo_status velo_set_tuning(velo_ctx *c, const int32_t *choice) {
    if (!c) return VELO_ERR_INVALID_ARG;
    using namespace tune;
    if (choice)
        for (int t : tunable)
            if (choice[t] < 0 || choice[t] >= kCand) return fail(c, VELO_ERR_INVALID_ARG, "tuning candidate out of range");
    for (int t : tunable) apply(c, t, choice ? choice[t] : 0);
    return VELO_OK;
}

velo_status velo_autotune(velo_ctx *c, const velo_hits *h, velo_outputs *o, void *stream, int32_t *choice) {
    if (!c) return VELO_ERR_INVALID_ARG;
    // candidate launch parameters, applied to every tunable stage at once;
    // stages are timed separately, so each picks its own best candidate.
    // per_cu 0 = the stage's default (occupancy for MFMA kernels).
    using namespace tune;
    const bool was_timing = c->timing;
    velo_status st = velo_set_timing(c, 1);
    if (st) return st;
    double best[VELO_N_STAGES];
    int pick[VELO_N_STAGES] = {};
    for (int k = 0; k < VELO_N_STAGES; k++) best[k] = 1e30;
    double ms[VELO_N_STAGES];
    int64_t n[VELO_N_STAGES];
    for (int cand = 0; cand < kCand; cand++) {
        for (int t : tunable) apply(c, t, cand);
        // one untimed call, then two timed ones
        if ((st = velo_infer(c, h, o, stream))) break;
        if ((st = velo_read_timing(c, ms, n))) break;
        for (int r = 0; r < 2 && !st; r++) st = velo_infer(c, h, o, stream);
        if (st || (st = velo_read_timing(c, ms, n))) break;
        for (int t : tunable)
            if (n[t] && ms[t] < best[t]) {
                best[t] = ms[t];
                pick[t] = cand;
            }
    }
    for (int t : tunable) apply(c, t, pick[t]);
    if (choice)
        for (int k = 0; k < VELO_N_STAGES; k++) choice[k] = pick[k];
    velo_set_timing(c, was_timing ? 1 : 0);
    if (st) return st;
    return velo_check(c, stream);
}

velo_status velo_embed_train_grad(velo_ctx *c, const velo_hits *h, const velo_embed_truth *truth,
                                  const float *params, int32_t k_train, float d2_train, float margin,
                                  float w_genuine, float *dparams, float *loss, int64_t *counts, float *emb,
                                  void *stream) {
    if (!c) return VELO_ERR_INVALID_ARG;
    if (!c->cfg.training) return fail(c, VELO_ERR_UNSUPPORTED, "context created without training = 1");
    velo_status st = check_hits(c, h);
    if (st) return st;
    if (!truth || !params || !dparams || !loss || !counts)
        return fail(c, VELO_ERR_INVALID_ARG, "velo_embed_train_grad: a required pointer is NULL");
    if (h->n_hits > 0 && (!truth->pid || !truth->query || !truth->rnd))
        return fail(c, VELO_ERR_INVALID_ARG, "velo_embed_train_grad: truth arrays are NULL");
    if (k_train < 1 || k_train > VELO_EMB_TRAIN_KMAX)
        return fail(c, VELO_ERR_INVALID_ARG, "velo_embed_train_grad: k_train outside [1, VELO_EMB_TRAIN_KMAX]");
    if (!(d2_train > 0.f) || !std::isfinite(d2_train) || !std::isfinite(margin) || !(w_genuine >= 0.f) ||
        !std::isfinite(w_genuine))
        return fail(c, VELO_ERR_INVALID_ARG, "velo_embed_train_grad: d2_train, margin or w_genuine invalid");
    DeviceGuard gd(c->device);
    launch_embed_train_grad(c, h, truth, params, k_train, d2_train, margin, w_genuine, dparams, loss, counts, emb,
                            (hipStream_t)stream);
    return device_status(c, "velo_embed_train_grad");
}

velo_status velo_check(velo_ctx *c, void *stream) {
    if (!c) return VELO_ERR_INVALID_ARG;
    DeviceGuard gd(c->device);
    hipStream_t s = (hipStream_t)stream;
    unsigned f = 0;
    if (hipMemcpyAsync(&f, c->ws.flags, sizeof f, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(c, VELO_ERR_DEVICE, "velo_check: stream synchronisation failed");
    if (f) {
        const unsigned zero = 0;
        if (hipMemcpy(c->ws.flags, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess)
            return fail(c, VELO_ERR_DEVICE, "velo_check: clearing the error flags failed");
    }
    if (f & kErrInput) return fail(c, VELO_ERR_INPUT, "device validation of the hits failed");
    if (f & kErrCapacity) return fail(c, VELO_ERR_CAPACITY, "edge count exceeds the edge capacity");
    return VELO_OK;
}

}  // extern "C"
