// wcc.hip -- connected components of the purified hit graph (paper Sec. 5
// overview and Sec. 7.3): edges with logit >= edge_logit_min, taken as
// undirected, define the components; each hit's label is the smallest
// event-local hit index of its component.
//
// One workgroup per event keeps the event's parent array in LDS.  Kept edges
// are hooked concurrently with a lock-free union-find: the larger of the two
// roots is linked under the smaller with an LDS compare-and-swap, retried
// until the two hits share a root.  Every parent pointer only ever points to
// a smaller index, so each root is its component's minimum and the labels do
// not depend on the order in which edges are processed.  (The paper's plane
// sweep is replaced because it is not exact on every graph.)
#include <mutex>

#include "internal.h"

namespace velo {

namespace {

__device__ inline int find_root(volatile int *par, int x) {
    int p = par[x];
    while (p != x) {
        const int gp = par[p];
        if (gp != p) par[x] = gp;   // path halving; gp is an ancestor of x
        x = p;
        p = gp;
    }
    return x;
}

__device__ inline void unite(int *par, int u, int v) {
    volatile int *vp = par;
    while (true) {
        u = find_root(vp, u);
        v = find_root(vp, v);
        if (u == v) return;
        if (u > v) {
            const int t = u; u = v; v = t;
        }
        // link root v under the smaller root u
        const int old = atomicCAS(&par[v], v, u);
        if (old == v) return;
        v = old;
    }
}

__global__ __launch_bounds__(1024) void k_wcc(int B, const int *__restrict__ off, const int *__restrict__ eoff,
                                              const int *__restrict__ n_edges, int64_t cap,
                                              const int *__restrict__ esrc, const int *__restrict__ edst,
                                              const float *__restrict__ logit, float thr,
                                              int *__restrict__ labels, int max_ev,
                                              unsigned *__restrict__ flags) {
    extern __shared__ int par[];
    if (*flags) return;
    const int b = blockIdx.x;
    const int s = off[b], n = off[b + 1] - s;
    if (n > max_ev) return;     // rejected by validation
    const int E = min((int64_t)*n_edges, cap);
    const int e0 = min(eoff[b], E), e1 = min(eoff[b + 1], E);
    for (int l = threadIdx.x; l < n; l += blockDim.x) par[l] = l;
    __syncthreads();
    bool err = false;
    // each thread takes 4 edges at a time, reading all of them before the
    // first union (the reads of an edge do not wait on the previous unions)
    constexpr int U = 4;
    for (int q0 = e0 + threadIdx.x; q0 < e1; q0 += U * blockDim.x) {
        bool keep[U];
        int su[U], sv[U];
#pragma unroll
        for (int j = 0; j < U; j++) {
            const int q = q0 + j * blockDim.x;
            const bool in = q < e1;
            keep[j] = in && logit[in ? q : e0] >= thr;
            su[j] = in ? esrc[q] : 0;
            sv[j] = in ? edst[q] : 0;
        }
#pragma unroll
        for (int j = 0; j < U; j++) {
            if (!keep[j]) continue;
            const int u = su[j], v = sv[j];
            if (u < 0 || u >= n || v < 0 || v >= n) {
                err = true;
                continue;
            }
            unite(par, u, v);
        }
    }
    if (err) atomicOr(flags, kErrInput);
    __syncthreads();
    for (int l = threadIdx.x; l < n; l += blockDim.x) labels[s + l] = find_root(par, l);
}

// The two plane sweeps of Sec. 7.3, kept as a comparison variant (not exact
// on every graph; see the file comment).  One workgroup per event, labels in
// LDS, starting as the event-local index.  Forward, planes 1 .. 25: each hit
// on plane p takes the smallest of its label and the labels of the hits
// joined to it by kept edges from planes p-1 and p-2; backward, planes 24 .. 0:
// the smallest of its label and those of the hits its kept edges reach on
// planes p+1 and p+2.  Edges are grouped by source and sources are sorted by
// plane, so the edges leaving plane q are one range, found by binary search;
// a plane step reads only labels of other planes, so it is an LDS atomicMin
// per edge whose result does not depend on the order.
__global__ __launch_bounds__(1024) void k_wcc_sweep(int B, const int *__restrict__ off, const int *__restrict__ eoff,
                                                    const int *__restrict__ n_edges, int64_t cap,
                                                    const int *__restrict__ esrc, const int *__restrict__ edst,
                                                    const float *__restrict__ logit, float thr,
                                                    const int *__restrict__ plane, const int *__restrict__ plane_off,
                                                    int *__restrict__ labels, int max_ev,
                                                    unsigned *__restrict__ flags) {
    extern __shared__ int lab[];
    __shared__ int epl[kPlaneSlots];   // first edge of each source plane (and the end)
    if (*flags) return;
    const int b = blockIdx.x;
    const int s = off[b], n = off[b + 1] - s;
    if (n > max_ev) return;     // rejected by validation
    const int E = min((int64_t)*n_edges, cap);
    const int e0 = min(eoff[b], E), e1 = min(eoff[b + 1], E);
    const int *po = plane_off + (int64_t)b * kPlaneSlots;
    for (int l = threadIdx.x; l < n; l += blockDim.x) lab[l] = l;
    if (threadIdx.x < kPlaneSlots) {
        const int first = po[threadIdx.x];    // first event-local hit on this plane or later
        int lo = e0, hi = e1;                 // first edge whose source is at or after it
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (esrc[mid] < first) lo = mid + 1;
            else hi = mid;
        }
        epl[threadIdx.x] = lo;
    }
    __syncthreads();
    bool err = false;
    auto ok = [&](int u, int v) {
        if (u < 0 || u >= n || v < 0 || v >= n) {
            err = true;
            return false;
        }
        return true;
    };
    for (int p = 1; p < VELO_N_PLANES; p++) {
        for (int q = epl[max(p - 2, 0)] + threadIdx.x; q < epl[p]; q += blockDim.x) {
            const int u = esrc[q], v = edst[q];
            if (!(logit[q] >= thr) || !ok(u, v)) continue;
            const int pu = plane[s + u], pv = plane[s + v];
            if (pv == p && (pv - pu == 1 || pv - pu == 2)) atomicMin(&lab[v], lab[u]);
        }
        __syncthreads();
    }
    for (int p = VELO_N_PLANES - 2; p >= 0; p--) {
        for (int q = epl[p] + threadIdx.x; q < epl[p + 1]; q += blockDim.x) {
            const int u = esrc[q], v = edst[q];
            if (!(logit[q] >= thr) || !ok(u, v)) continue;
            const int pu = plane[s + u], pv = plane[s + v];
            if (pu == p && (pv - pu == 1 || pv - pu == 2)) atomicMin(&lab[u], lab[v]);
        }
        __syncthreads();
    }
    if (err) atomicOr(flags, kErrInput);
    for (int l = threadIdx.x; l < n; l += blockDim.x) labels[s + l] = lab[l];
}

}  // namespace

void launch_components_sweep(velo_ctx *c, const velo_hits *h, const velo_outputs *g, hipStream_t s) {
    if (h->n_events <= 0) return;
    const int64_t cap = g->edge_capacity < c->cfg.max_edges ? g->edge_capacity : c->cfg.max_edges;
    const size_t lds = sizeof(int) * (size_t)(c->cfg.max_event_hits > 0 ? c->cfg.max_event_hits : 1);
    static bool attr = false;
    if (!attr) {
        // the kernel's static LDS (the plane ranges) comes out of the same budget
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_wcc_sweep),
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(c->lds_max - sizeof(int) * kPlaneSlots));   // a failure is the launch's error
        attr = true;
    }
    k_wcc_sweep<<<h->n_events, 1024, lds, s>>>(h->n_events, h->event_offsets, g->edge_offsets, c->ws.n_edges, cap,
                                               g->edge_src, g->edge_dst, g->edge_logit, c->cfg.edge_logit_min,
                                               h->plane, c->ws.plane_off, g->labels, c->cfg.max_event_hits,
                                               c->ws.flags);
}

void launch_components_raw(const velo_hits *h, const velo_outputs *g, int64_t cap, float thr, int max_event_hits,
                           size_t lds_max, const int *n_internal, unsigned *flags, hipStream_t s) {
    if (h->n_events <= 0) return;
    const size_t lds = sizeof(int) * (size_t)(max_event_hits > 0 ? max_event_hits : 1);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_wcc), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds_max);
        attr = true;
    }
    k_wcc<<<h->n_events, 1024, lds, s>>>(h->n_events, h->event_offsets, g->edge_offsets, n_internal, cap,
                                         g->edge_src, g->edge_dst, g->edge_logit, thr, g->labels, max_event_hits,
                                         flags);
}

void launch_components(velo_ctx *c, const velo_hits *h, const velo_outputs *g, hipStream_t s) {
    const int64_t cap = g->edge_capacity < c->cfg.max_edges ? g->edge_capacity : c->cfg.max_edges;
    launch_components_raw(h, g, cap, c->cfg.edge_logit_min, c->cfg.max_event_hits, c->lds_max, c->ws.n_edges,
                          c->ws.flags, s);
}

}  // namespace velo

// ------------------------------------------------------------------------
// velo_components_noalloc: the components stage without a context, for
// callers that cannot allocate device memory.  Its working memory (the
// error word, the clamped edge count, and the validation kernel's plane
// offsets and hit-to-event map) is the fixed array `scratch` below: every
// GPU the library runs on holds its own copy for the life of the process,
// and every call on that GPU shares it.
// ------------------------------------------------------------------------
namespace {

constexpr int64_t kNaHead = 64;                                  // [0] error bits, [1] clamped edge count
constexpr int64_t kNaPlaneOff = kNaHead;                         // [VELO_NOALLOC_MAX_EVENTS x 27]
constexpr int64_t kNaHitEvent = kNaPlaneOff + (int64_t)VELO_NOALLOC_MAX_EVENTS * velo::kPlaneSlots;
constexpr int64_t kNaInts = kNaHitEvent + (int64_t)VELO_NOALLOC_MAX_HITS;   // [VELO_NOALLOC_MAX_HITS]

}  // namespace

// Host code must not pass this name to a kernel: it is a host-side stand-in.
// Kernels get the device address that hipGetSymbolAddress returns.
static __device__ __align__(256) int scratch[kNaInts];

namespace {

constexpr int kNaMaxDevices = 64;
std::mutex na_mu;
int *na_ptr[kNaMaxDevices] = {};
size_t na_lds[kNaMaxDevices] = {};

// The device address of `scratch` on device `dev` (the current device),
// looked up once per device.
int *noalloc_scratch(int dev, size_t *lds_max) {
    std::lock_guard<std::mutex> lock(na_mu);
    if (dev < 0 || dev >= kNaMaxDevices) return nullptr;
    if (!na_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return nullptr;
        na_lds[dev] = (size_t)lds;
        na_ptr[dev] = static_cast<int *>(p);
    }
    *lds_max = na_lds[dev];
    return na_ptr[dev];
}

}  // namespace

extern "C" velo_status velo_components_noalloc(const velo_hits *h, const velo_outputs *g, float edge_logit_min,
                                               int32_t max_event_hits, void *stream) {
    using namespace velo;
    if (!h || !g) return VELO_ERR_INVALID_ARG;
    if (h->n_events < 0 || h->n_hits < 0 || max_event_hits < 0 || g->edge_capacity < 0)
        return VELO_ERR_INVALID_ARG;
    if (h->n_events == 0 && h->n_hits != 0) return VELO_ERR_INVALID_ARG;
    if (h->n_events > 0 && (!h->event_offsets || !g->edge_offsets)) return VELO_ERR_INVALID_ARG;
    if (h->n_hits > 0 && (!h->x || !h->y || !h->z || !h->plane || !g->labels)) return VELO_ERR_INVALID_ARG;
    if (!g->n_edges) return VELO_ERR_INVALID_ARG;
    if (g->edge_capacity > 0 && (!g->edge_src || !g->edge_dst || !g->edge_logit)) return VELO_ERR_INVALID_ARG;
    if (g->edge_capacity >= (int64_t)1 << 31) return VELO_ERR_UNSUPPORTED;
    // the sizes the fixed working memory holds
    if (h->n_events > VELO_NOALLOC_MAX_EVENTS || h->n_hits > VELO_NOALLOC_MAX_HITS) return VELO_ERR_CAPACITY;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return VELO_ERR_DEVICE;
    size_t lds_max = 0;
    int *scr = noalloc_scratch(dev, &lds_max);
    if (!scr) return VELO_ERR_DEVICE;
    // one event's hits are one workgroup's LDS parent array
    if ((size_t)max_event_hits * sizeof(int) > lds_max) return VELO_ERR_CAPACITY;
    hipStream_t s = (hipStream_t)stream;
    unsigned *flags = reinterpret_cast<unsigned *>(scr);
    int *n_internal = scr + 1;
    launch_fill(scr, 0, 2, s);       // the previous call's error bits and count
    launch_prepare_raw(h, max_event_hits, scr + kNaPlaneOff, scr + kNaHitEvent, flags, s);
    launch_globalise_raw(h, g, g->edge_capacity, nullptr, nullptr, n_internal, flags, s);
    launch_components_raw(h, g, g->edge_capacity, edge_logit_min, max_event_hits, lds_max, n_internal, flags, s);
    if (hipGetLastError() != hipSuccess) return VELO_ERR_DEVICE;
    unsigned f = 0;
    if (hipMemcpyAsync(&f, flags, sizeof f, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return VELO_ERR_DEVICE;
    if (f & kErrInput) return VELO_ERR_INPUT;
    if (f & kErrCapacity) return VELO_ERR_CAPACITY;
    return VELO_OK;
}
