// triplets.hip -- the triplet stage: triplet building and classification
// (paper Sec. 5.3) and track building from the purified edge graph (Sec. 5.4),
// batched over events, on the graph and final edge encodings of the GNN pass
// that ran just before on the same context.
//
// Layout.  Edges are batch-global positions of the graph's arrays, grouped by
// source hit (row_ptr) and, through the incoming lists (in_ptr, in_list, edge
// ids ascending), by destination hit.  An edge is kept when its logit passes
// the edge cut.
//   1. k_tri_count   per common hit C: kept in-edges kin, kept out-edges kout;
//                    kin*kout articulations, C(kout,2) + C(kin,2) elbows.
//      scans         per-hit offsets of both lists (hits in index order keep
//                    the events contiguous).
//   2. k_tri_emit    per C, in the order the ABI states; the pairs are written
//                    event-local (output) and batch-global (workspace).
//   3. k_tri_cls     one classifier per list: hidden = relu(b1 + W1 [e_a; e_b])
//                    on MFMA, 16 triplets per wavefront unit, logit = w2 . hidden
//                    + b2 on the vector ALU.
//   4. track building (per edge / per triplet kernels over the whole batch):
//      union-find over edges in global memory with min-index hooking (every
//      parent is smaller than its child, so each root is its set's smallest
//      edge and the result does not depend on the order of the unions).
#include "mfma.h"

namespace velo {

namespace {

using namespace mfma;

constexpr int kTriBlock = 256;

inline int tri_grid(int64_t n, int block = kTriBlock, int cap = 16384) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

#define GRID_STRIDE(i, n) \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

__device__ inline bool edge_kept(const float *logit, int q, float cut) { return logit[q] >= cut; }

// ------------------------------------------------------------------------
// 1. counts per common hit
// ------------------------------------------------------------------------
__global__ void k_tri_count(int64_t N, const int *__restrict__ row_ptr, const int *__restrict__ in_ptr,
                            const int *__restrict__ in_list, const float *__restrict__ logit, float cut,
                            int *__restrict__ cnt_art, int *__restrict__ cnt_elb, const unsigned *__restrict__ flags) {
    if (*flags) return;
    GRID_STRIDE(i, N) {
        int kin = 0, kout = 0;
        for (int p = in_ptr[i]; p < in_ptr[i + 1]; p++) kin += edge_kept(logit, in_list[p], cut);
        for (int q = row_ptr[i]; q < row_ptr[i + 1]; q++) kout += edge_kept(logit, q, cut);
        cnt_art[i] = kin * kout;
        cnt_elb[i] = kout * (kout - 1) / 2 + kin * (kin - 1) / 2;
    }
}

// totals -> caller (required sizes) and clamped internal counts; overflow
// of either list stops the stage (kErrCapacity)
__global__ void k_tri_totals(int64_t N, const int *__restrict__ art_ptr, const int *__restrict__ elb_ptr,
                             int64_t cap, int *__restrict__ n_out, int *__restrict__ n_int,
                             unsigned *__restrict__ flags) {
    if (*flags) return;
    const int na = art_ptr[N], ne = elb_ptr[N];
    n_out[0] = na;
    n_out[1] = ne;
    n_int[0] = (int)min((int64_t)na, cap);
    n_int[1] = (int)min((int64_t)ne, cap);
    if (na < 0 || ne < 0 || na > cap || ne > cap) atomicOr(flags, kErrCapacity);
}

__global__ void k_tri_event_offsets(int B, const int *__restrict__ ev_off, const int *__restrict__ art_ptr,
                                    const int *__restrict__ elb_ptr, int *__restrict__ art_off,
                                    int *__restrict__ elb_off, const unsigned *__restrict__ flags) {
    if (*flags) return;
    GRID_STRIDE(b, (int64_t)B + 1) {
        art_off[b] = art_ptr[ev_off[b]];
        elb_off[b] = elb_ptr[ev_off[b]];
    }
}

// ------------------------------------------------------------------------
// 2. the triplets of each common hit, in the stated order
// ------------------------------------------------------------------------
__global__ void k_tri_emit(int64_t N, const int *__restrict__ hit_event, const int *__restrict__ eoff,
                           const int *__restrict__ row_ptr, const int *__restrict__ in_ptr,
                           const int *__restrict__ in_list, const float *__restrict__ logit, float cut,
                           const int *__restrict__ art_ptr, const int *__restrict__ elb_ptr,
                           int *__restrict__ art, int *__restrict__ art_g, int *__restrict__ elb,
                           int8_t *__restrict__ elb_type, int *__restrict__ elb_g, const unsigned *__restrict__ flags) {
    if (*flags) return;
    GRID_STRIDE(i, N) {
        const int e0 = eoff[hit_event[i]];
        const int r0 = row_ptr[i], r1 = row_ptr[i + 1], p0 = in_ptr[i], p1 = in_ptr[i + 1];
        int ta = art_ptr[i], te = elb_ptr[i];
        // articulations: kept in-edge a = A -> C, kept out-edge b = C -> B
        for (int p = p0; p < p1; p++) {
            const int a = in_list[p];
            if (!edge_kept(logit, a, cut)) continue;
            for (int q = r0; q < r1; q++) {
                if (!edge_kept(logit, q, cut)) continue;
                art[2 * ta] = a - e0;
                art[2 * ta + 1] = q - e0;
                art_g[2 * ta] = a;
                art_g[2 * ta + 1] = q;
                ta++;
            }
        }
        // left elbows: two kept out-edges of C
        for (int q = r0; q < r1; q++) {
            if (!edge_kept(logit, q, cut)) continue;
            for (int q2 = q + 1; q2 < r1; q2++) {
                if (!edge_kept(logit, q2, cut)) continue;
                elb[2 * te] = q - e0;
                elb[2 * te + 1] = q2 - e0;
                elb_g[2 * te] = q;
                elb_g[2 * te + 1] = q2;
                elb_type[te] = 1;
                te++;
            }
        }
        // right elbows: two kept in-edges of C
        for (int p = p0; p < p1; p++) {
            const int a = in_list[p];
            if (!edge_kept(logit, a, cut)) continue;
            for (int p2 = p + 1; p2 < p1; p2++) {
                const int a2 = in_list[p2];
                if (!edge_kept(logit, a2, cut)) continue;
                elb[2 * te] = a - e0;
                elb[2 * te + 1] = a2 - e0;
                elb_g[2 * te] = a;
                elb_g[2 * te + 1] = a2;
                elb_type[te] = 2;
                te++;
            }
        }
    }
}

// ------------------------------------------------------------------------
// 3. triplet classifier: logit = w2 . relu(b1 + W1 [e_a; e_b]) + b2
// ------------------------------------------------------------------------
template <class P, int H>
__global__ __launch_bounds__(512) void k_tri_cls(const int *__restrict__ n_dev, const int *__restrict__ pairs,
                                                 const typename P::state_t *__restrict__ e,
                                                 const float *__restrict__ Pw, float *__restrict__ logit,
                                                 const unsigned *__restrict__ flags) {
    using W = typename P::wfrag_t;
    constexpr int MO = H / 16, KB = H / P::KBLK;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    W *sW1 = (W *)lds_raw;
    float *sB = (float *)(lds_raw + frag_bytes<P>(H, 2 * H));   // b1 [H], w2 [H]
    stage<P>(sW1, Pw, H, 2 * H, MO);
    for (int t = threadIdx.x; t < H; t += blockDim.x) {
        sB[t] = Pw[2 * H * H + t];
        sB[H + t] = Pw[2 * H * H + H + t];
    }
    __syncthreads();
    if (*flags) return;
    const float b2 = Pw[2 * H * H + 2 * H];
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    const int64_t T = *n_dev;
    const int64_t units = (T + 15) >> 4;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t u = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); u < units; u += waves) {
        const int64_t t = u * 16 + n;
        const int64_t tc = t < T ? t : T - 1;
        const int64_t a = pairs[2 * tc], b = pairs[2 * tc + 1];
        typename P::frag_t X[2 * KB];
#pragma unroll
        for (int kb = 0; kb < KB; kb++) {
            X[kb] = P::load(e + a * H, kb, g, 1.f);
            X[KB + kb] = P::load(e + b * H, kb, g, 1.f);
        }
        f32x4 hid[MO];
        load_bias<MO>(sB, hid, g);
        gemm<P, MO, 2 * KB, 0, 2 * KB, true>(sW1, X, hid, lane);   // both inputs are stored encodings
        f32x4 w2[MO];
        load_bias<MO>(sB + H, w2, g);
        float part = 0.f;
#pragma unroll
        for (int mo = 0; mo < MO; mo++)
#pragma unroll
            for (int i = 0; i < 4; i++) part += w2[mo][i] * fmaxf(hid[mo][i], 0.f);
        part += __shfl_xor(part, 16);
        part += __shfl_xor(part, 32);
        if (g == 0 && t < T) logit[t] = part + b2;
    }
}

// ------------------------------------------------------------------------
// 4. track building
// ------------------------------------------------------------------------
__device__ inline int uf_root(const int *par, int x) {
    for (;;) {
        const int p = __hip_atomic_load(par + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (p == x) return x;
        x = p;
    }
}

// join the sets of a and b: the larger root is hooked under the smaller one
__device__ inline void uf_join(int *par, int a, int b) {
    for (;;) {
        a = uf_root(par, a);
        b = uf_root(par, b);
        if (a == b) return;
        if (a > b) {
            const int t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(par + b, b, a) == b) return;
    }
}

__global__ void k_tb_init(const int *__restrict__ n_edges, int64_t cap, int *__restrict__ par,
                          int *__restrict__ first, int *__restrict__ second, unsigned char *__restrict__ dup,
                          unsigned char *__restrict__ touched, const unsigned *__restrict__ flags) {
    if (*flags) return;
    const int64_t E = min((int64_t)*n_edges, cap);
    GRID_STRIDE(q, E) {
        par[q] = (int)q;
        first[q] = 0;
        second[q] = 0;
        dup[q] = 0;
        touched[q] = 0;
    }
}

// step 1 of Sec. 5.4: kept elbows join their edges; of two edges spanning a
// different number of planes, the longer duplicates the path through the
// third hit
__global__ void k_tb_elbows(const int *__restrict__ n_int, const int *__restrict__ elb_g,
                            const float *__restrict__ elb_logit, float tcut, const int *__restrict__ src_g,
                            const int *__restrict__ dst_g, const int *__restrict__ plane, int *__restrict__ par,
                            unsigned char *__restrict__ dup, const unsigned *__restrict__ flags) {
    if (*flags) return;
    GRID_STRIDE(t, (int64_t)n_int[1]) {
        if (!(elb_logit[t] >= tcut)) continue;
        const int a = elb_g[2 * t], b = elb_g[2 * t + 1];
        const int ga = plane[dst_g[a]] - plane[src_g[a]], gb = plane[dst_g[b]] - plane[src_g[b]];
        if (ga > gb) dup[a] = 1;
        else if (gb > ga) dup[b] = 1;
        uf_join(par, a, b);
    }
}

__device__ inline bool art_live(const float *art_logit, float tcut, const unsigned char *dup, int t, int a, int b) {
    return art_logit[t] >= tcut && !dup[a] && !dup[b];
}

// step 2: how often each edge is the first / second edge of a kept
// articulation without duplicates
__global__ void k_tb_art_count(const int *__restrict__ n_int, const int *__restrict__ art_g,
                               const float *__restrict__ art_logit, float tcut, const unsigned char *__restrict__ dup,
                               int *__restrict__ first, int *__restrict__ second, const unsigned *__restrict__ flags) {
    if (*flags) return;
    GRID_STRIDE(t, (int64_t)n_int[0]) {
        const int a = art_g[2 * t], b = art_g[2 * t + 1];
        if (!art_live(art_logit, tcut, dup, (int)t, a, b)) continue;
        atomicAdd(first + a, 1);
        atomicAdd(second + b, 1);
    }
}

// shared articulations (tracks part or join there) are kept apart; the
// others join their two edges
__global__ void k_tb_art_join(const int *__restrict__ n_int, const int *__restrict__ art_g,
                              const float *__restrict__ art_logit, float tcut, const unsigned char *__restrict__ dup,
                              const int *__restrict__ first, const int *__restrict__ second, int *__restrict__ par,
                              int *__restrict__ shared, const unsigned *__restrict__ flags) {
    if (*flags) return;
    GRID_STRIDE(t, (int64_t)n_int[0]) {
        const int a = art_g[2 * t], b = art_g[2 * t + 1];
        int sh = 0;
        if (art_live(art_logit, tcut, dup, (int)t, a, b)) {
            if (first[a] > 1 || second[b] > 1) sh = 1;
            else uf_join(par, a, b);
        }
        shared[t] = sh;
    }
}

// segments: every parent now final; compress each edge to its root and
// write the event-local segment of every kept edge
__global__ void k_tb_label(const int *__restrict__ n_edges, int64_t cap, const int *__restrict__ src_g,
                           const int *__restrict__ hit_event, const int *__restrict__ eoff,
                           const float *__restrict__ logit, float cut, int *__restrict__ par,
                           int *__restrict__ edge_seg, const unsigned *__restrict__ flags) {
    if (*flags) return;
    const int64_t E = min((int64_t)*n_edges, cap);
    GRID_STRIDE(q, E) {
        const int r = uf_root(par, (int)q);
        par[q] = r;
        edge_seg[q] = edge_kept(logit, (int)q, cut) ? r - eoff[hit_event[src_g[q]]] : -1;
    }
}

// step 3: the segments of shared articulations become parts of their tracks
__global__ void k_tb_touch(const int *__restrict__ n_int, const int *__restrict__ art_g,
                           const int *__restrict__ shared, const int *__restrict__ par,
                           unsigned char *__restrict__ touched, const unsigned *__restrict__ flags) {
    if (*flags) return;
    GRID_STRIDE(t, (int64_t)n_int[0]) {
        if (!shared[t]) continue;
        touched[par[art_g[2 * t]]] = 1;
        touched[par[art_g[2 * t + 1]]] = 1;
    }
}

__global__ void k_tb_single(const int *__restrict__ n_edges, int64_t cap, const float *__restrict__ logit, float cut,
                            const int *__restrict__ par, const unsigned char *__restrict__ touched,
                            int *__restrict__ single, const unsigned *__restrict__ flags) {
    if (*flags) return;
    const int64_t E = min((int64_t)*n_edges, cap);
    GRID_STRIDE(q, E) single[q] = edge_kept(logit, (int)q, cut) && par[q] == q && !touched[q];
}

// per event: tracks before it (one-segment tracks of earlier events and their
// shared articulations); the total, its check against the capacity
__global__ void k_tb_offsets(int B, const int *__restrict__ eoff, const int *__restrict__ art_off,
                             const int *__restrict__ single_ptr, const int *__restrict__ shared_ptr,
                             int64_t track_cap, int *__restrict__ track_off, int *__restrict__ n_tracks,
                             int *__restrict__ n_int, unsigned *__restrict__ flags) {
    if (*flags) return;
    GRID_STRIDE(b, (int64_t)B + 1) {
        const int v = single_ptr[eoff[b]] + shared_ptr[art_off[b]];
        track_off[b] = v;
        if (b == B) {
            *n_tracks = v;
            n_int[2] = v;
            if (v < 0 || v > track_cap) atomicOr(flags, kErrCapacity);
        }
    }
}

__global__ void k_tb_emit_single(const int *__restrict__ n_edges, int64_t cap, const int *__restrict__ src_g,
                                 const int *__restrict__ hit_event, const int *__restrict__ eoff,
                                 const int *__restrict__ art_off, const int *__restrict__ single,
                                 const int *__restrict__ single_ptr, const int *__restrict__ shared_ptr,
                                 int *__restrict__ tracks, const unsigned *__restrict__ flags) {
    if (*flags) return;
    const int64_t E = min((int64_t)*n_edges, cap);
    GRID_STRIDE(q, E) {
        if (!single[q]) continue;
        const int b = hit_event[src_g[q]];
        // the event's tracks start after every earlier event's; its
        // one-segment tracks come first, in edge order
        const int pos = single_ptr[q] + shared_ptr[art_off[b]];
        tracks[2 * pos] = (int)q - eoff[b];
        tracks[2 * pos + 1] = -1;
    }
}

__global__ void k_tb_emit_shared(const int *__restrict__ n_int, const int *__restrict__ art_g,
                                 const int *__restrict__ src_g, const int *__restrict__ hit_event,
                                 const int *__restrict__ eoff, const int *__restrict__ par,
                                 const int *__restrict__ shared, const int *__restrict__ single_ptr,
                                 const int *__restrict__ shared_ptr, int *__restrict__ tracks,
                                 const unsigned *__restrict__ flags) {
    if (*flags) return;
    GRID_STRIDE(t, (int64_t)n_int[0]) {
        if (!shared[t]) continue;
        const int a = art_g[2 * t], b = art_g[2 * t + 1];
        const int ev = hit_event[src_g[b]];      // b leaves the common hit
        // after all one-segment tracks of events up to this one and the
        // shared articulations before t
        const int pos = single_ptr[eoff[ev + 1]] + shared_ptr[t];
        tracks[2 * pos] = par[a] - eoff[ev];
        tracks[2 * pos + 1] = par[b] - eoff[ev];
    }
}

template <class P, int H>
void run_tri_cls(velo_ctx *c, const int *n_dev, const int *pairs, const float *Pw, float *logit, hipStream_t s) {
    const size_t lds = frag_bytes<P>(H, 2 * H) + sizeof(float) * 2 * H;
    int per_cu = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(&k_tri_cls<P, H>),
                                                       512, lds);   // 0 on failure: one block per CU
    if (per_cu < 1) per_cu = 1;
    k_tri_cls<P, H><<<persistent_grid(c, per_cu), 512, lds, s>>>(n_dev, pairs,
                                                                 (const typename P::state_t *)c->ws.e, Pw, logit,
                                                                 c->ws.flags);
}

template <class P>
void tri_cls(velo_ctx *c, const int *n_dev, const int *pairs, const float *Pw, float *logit, hipStream_t s) {
    switch (c->cfg.gnn_hidden) {
        case 32: run_tri_cls<P, 32>(c, n_dev, pairs, Pw, logit, s); break;
        case 64: run_tri_cls<P, 64>(c, n_dev, pairs, Pw, logit, s); break;
        case 128: run_tri_cls<P, 128>(c, n_dev, pairs, Pw, logit, s); break;
    }
}

}  // namespace

bool triplet_supported(int hidden) { return hidden == 32 || hidden == 64 || hidden == 128; }

void launch_triplets(velo_ctx *c, const velo_hits *h, const velo_outputs *g, const velo_triplet_outputs *t,
                     hipStream_t s) {
    Workspace &w = c->ws;
    TripletWs &T = c->tri;
    const int64_t N = h->n_hits;
    const int B = h->n_events;
    const float cut = c->cfg.edge_logit_min, tcut = c->tri_cut;
    const int64_t ecap = g->edge_capacity < c->cfg.max_edges ? g->edge_capacity : c->cfg.max_edges;
    const int H = c->cfg.gnn_hidden;
    const float *P_art = T.params, *P_elb = T.params + (2 * H * H + 2 * H + 1);
    // 1. counts and offsets
    if (N > 0)
        k_tri_count<<<tri_grid(N), kTriBlock, 0, s>>>(N, w.row_ptr, w.in_ptr, w.in_list, g->edge_logit, cut,
                                                      T.cnt_art, T.cnt_elb, w.flags);
    launch_scan_with(T.cnt_art, T.art_ptr, N, T.scan_tmp, s);
    launch_scan_with(T.cnt_elb, T.elb_ptr, N, T.scan_tmp, s);
    k_tri_totals<<<1, 1, 0, s>>>(N, T.art_ptr, T.elb_ptr, t->capacity, t->n_triplets, T.n_int, w.flags);
    if (B > 0)
        k_tri_event_offsets<<<tri_grid(B + 1), kTriBlock, 0, s>>>(B, h->event_offsets, T.art_ptr, T.elb_ptr,
                                                                  t->art_offsets, t->elb_offsets, w.flags);
    // 2. the lists
    if (N > 0)
        k_tri_emit<<<tri_grid(N), kTriBlock, 0, s>>>(N, w.hit_event, g->edge_offsets, w.row_ptr, w.in_ptr, w.in_list,
                                                     g->edge_logit, cut, T.art_ptr, T.elb_ptr, t->art, T.art_g, t->elb,
                                                     t->elb_type, T.elb_g, w.flags);
    // 3. classifiers (bf16 operands on 2-byte states)
    if (c->cfg.precision == VELO_FP32) {
        tri_cls<F32>(c, T.n_int, T.art_g, P_art, t->art_logit, s);
        tri_cls<F32>(c, T.n_int + 1, T.elb_g, P_elb, t->elb_logit, s);
    } else if (c->cfg.precision == VELO_BF16X2) {
        tri_cls<BF16X2>(c, T.n_int, T.art_g, P_art, t->art_logit, s);
        tri_cls<BF16X2>(c, T.n_int + 1, T.elb_g, P_elb, t->elb_logit, s);
    } else {
        tri_cls<BF16>(c, T.n_int, T.art_g, P_art, t->art_logit, s);
        tri_cls<BF16>(c, T.n_int + 1, T.elb_g, P_elb, t->elb_logit, s);
    }
    // 4. tracks
    const int eg = tri_grid(ecap), tg = tri_grid(t->capacity);
    k_tb_init<<<eg, kTriBlock, 0, s>>>(w.n_edges, ecap, T.par, T.first, T.second, T.dup, T.touched, w.flags);
    k_tb_elbows<<<tg, kTriBlock, 0, s>>>(T.n_int, T.elb_g, t->elb_logit, tcut, w.src_g, w.dst_g, h->plane, T.par,
                                         T.dup, w.flags);
    k_tb_art_count<<<tg, kTriBlock, 0, s>>>(T.n_int, T.art_g, t->art_logit, tcut, T.dup, T.first, T.second,
                                            w.flags);
    k_tb_art_join<<<tg, kTriBlock, 0, s>>>(T.n_int, T.art_g, t->art_logit, tcut, T.dup, T.first, T.second, T.par,
                                           T.shared, w.flags);
    k_tb_label<<<eg, kTriBlock, 0, s>>>(w.n_edges, ecap, w.src_g, w.hit_event, g->edge_offsets, g->edge_logit, cut,
                                        T.par, t->edge_seg, w.flags);
    k_tb_touch<<<tg, kTriBlock, 0, s>>>(T.n_int, T.art_g, T.shared, T.par, T.touched, w.flags);
    k_tb_single<<<eg, kTriBlock, 0, s>>>(w.n_edges, ecap, g->edge_logit, cut, T.par, T.touched, T.single, w.flags);
    launch_scan_with(T.single, T.single_ptr, ecap, T.scan_tmp, s);
    launch_scan_with(T.shared, T.shared_ptr, t->capacity, T.scan_tmp, s);
    if (B > 0) {
        k_tb_offsets<<<tri_grid(B + 1), kTriBlock, 0, s>>>(B, g->edge_offsets, t->art_offsets, T.single_ptr,
                                                           T.shared_ptr, t->track_capacity, t->track_offsets,
                                                           t->n_tracks, T.n_int, w.flags);
        k_tb_emit_single<<<eg, kTriBlock, 0, s>>>(w.n_edges, ecap, w.src_g, w.hit_event, g->edge_offsets,
                                                  t->art_offsets, T.single, T.single_ptr, T.shared_ptr, t->tracks,
                                                  w.flags);
        k_tb_emit_shared<<<tg, kTriBlock, 0, s>>>(T.n_int, T.art_g, w.src_g, w.hit_event, g->edge_offsets, T.par,
                                                  T.shared, T.single_ptr, T.shared_ptr, t->tracks, w.flags);
    }
}

}  // namespace velo
