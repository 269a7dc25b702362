// embtrain.hip -- one training step of the hit embedding (paper Sec. 5.1,
// the two loss equations).
//
// Step: the embedding MLP runs with the caller's parameters and keeps its
// inputs and hidden activations; the bounded neighbour search (k_train,
// d2_train) gives the hard-negative candidates; one wavefront per query hit
// builds its pairs (hard negatives: the members of another particle in its
// neighbour list; genuine: every candidate of its particle on planes p+1,
// p+2; one random candidate) and adds each pair's gradient with respect to
// the two embeddings, 2 (e_q - e_j) with the pair's sign, to both hits.
// Those per-hit sums and the loss sums are kept in 64-bit fixed point, so the
// scatter of a pair to its second hit is an integer atomic whose result does
// not depend on the order of the pairs.  Then, per 16 hits on MFMA, the
// gradient goes back through layer 3 (W3^T dE, on the vector ALU: K = 4) and
// layer 2 (W2^T, a 128 x 128 contraction), and the weight gradients are
// summed over the hits in fixed-size chunks and then over the chunks, both in
// a fixed order.
#include "mfma.h"

namespace velo {

namespace {

using namespace mfma;

constexpr int kCe = VELO_EMB_HIDDEN;   // hidden width 128
constexpr int kD = VELO_EMB_DIM;       // embedding dimension 4
// embedding parameters in blob order: W1 [Ce x 3], b1, W2 [Ce x Ce], b2, W3 [D x Ce], b3
constexpr int kOffB1 = kCe * 3, kOffW2 = kOffB1 + kCe, kOffB2 = kOffW2 + kCe * kCe, kOffW3 = kOffB2 + kCe,
              kOffB3 = kOffW3 + kD * kCe, kEmbParams = kOffB3 + kD;
constexpr int kDwChunk = 256;   // hits per weight-gradient partial
constexpr int kDwSub = 16;      // hits staged in LDS at a time
constexpr double kGradFix = 4294967296.0;   // 2^32: scale of the per-hit gradient sums
constexpr double kLossFix = 16777216.0;     // 2^24: scale of the loss sums
constexpr float kFixClamp = 1.0e6f;         // contributions are clamped to +-1e6 (far beyond any step)

static_assert(kCe == 128 && kD == 4, "the embedding training kernels are written for 3 -> 128 -> 128 -> 4");

__device__ inline unsigned long long to_fix(float v, double scale) {
    v = fminf(fmaxf(v, -kFixClamp), kFixClamp);
    return (unsigned long long)__double2ll_rn((double)v * scale);
}
__device__ inline double from_fix(unsigned long long v, double scale) { return (double)(long long)v / scale; }

// float32 squared distance, evaluated as s = d0*d0, then s = fma(d_c, d_c, s)
// (the order the neighbour search decides in)
__device__ inline float sqdist(f32x4 a, f32x4 b) {
    float d = a[0] - b[0];
    float s = d * d;
    d = a[1] - b[1];
    s = __builtin_fmaf(d, d, s);
    d = a[2] - b[2];
    s = __builtin_fmaf(d, d, s);
    d = a[3] - b[3];
    s = __builtin_fmaf(d, d, s);
    return s;
}

// Training pairs of every query hit and their contributions.  A workgroup
// takes the queries of one (event, plane p), one wavefront per query: every
// pair's second hit lies in the shared candidate window (planes p+1, p+2),
// so the second hits' sums are gathered in LDS (64-bit integer adds) and
// flushed with one global atomic per entry; windows larger than kPairLds
// hits add to global memory directly.  acc[j * 8 + c]: fixed-point sum of
// the genuine (c < 4) and fake (c >= 4) pairs' gradients with respect to
// e_j; stat: {sum of genuine d2, sum of active fake hinges (both 2^-24 fixed
// point), N_g, N_f}.
constexpr int kPairBlock = 256;
constexpr int kPairLds = 512;    // window hits whose sums fit in LDS (32 KB)

__global__ __launch_bounds__(kPairBlock) void k_emb_pairs(int B, const int *__restrict__ off,
                                                          const int *__restrict__ plane_off,
                                                          const f32x4 *__restrict__ emb, const int *__restrict__ pid,
                                                          const uint8_t *__restrict__ query,
                                                          const unsigned *__restrict__ rnd, const int *__restrict__ nbr,
                                                          const int *__restrict__ deg, int kmax, float margin,
                                                          unsigned long long *__restrict__ acc,
                                                          unsigned long long *__restrict__ stat,
                                                          const unsigned *__restrict__ flags) {
    __shared__ unsigned long long win[kPairLds * 8];
    if (*flags & kErrInput) return;
    const int b = blockIdx.x / VELO_N_PLANES, p = blockIdx.x % VELO_N_PLANES;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t s = off[b];
    const int *po = plane_off + (int64_t)b * kPlaneSlots;
    const int q0 = po[p], q1 = po[p + 1];
    if (q0 >= q1) return;                                   // uniform over the workgroup
    const int c0 = po[min(p + 1, VELO_N_PLANES)];
    const int C = max(po[min(p + 3, VELO_N_PLANES)] - c0, 0);
    const int64_t base = s + c0;
    const bool in_lds = C <= kPairLds;
    if (in_lds)
        for (int k = threadIdx.x; k < C * 8; k += kPairBlock) win[k] = 0;
    __syncthreads();
    unsigned long long sg = 0, sf = 0, ng = 0, nf = 0;   // this lane's share
    for (int lq = q0 + w; lq < q1; lq += kPairBlock / 64) {
        const int64_t i = s + lq;
        if (!query[i]) continue;                            // uniform over the wavefront
        const f32x4 q = emb[i];
        const int pq = pid[i];
        // this lane's share of the query's own sums (genuine qg, fake qf; two
        // arrays, so that every index is a constant and they stay in
        // registers), added up over the wavefront before one atomic per entry
        unsigned long long qg[kD] = {0, 0, 0, 0}, qf[kD] = {0, 0, 0, 0};
        auto same = [&](int64_t j) { return pq >= 0 && pid[j] == pq; };
        // one pair (i, j), handled by the calling lane
        // (the genuine and fake sums are updated by selected values, not
        // through a selected pointer, so that they stay in registers)
        auto pair = [&](int64_t j) {
            const f32x4 e = emb[j];
            const float d2 = sqdist(q, e);
            const bool gen = same(j);
            ng += gen;
            nf += !gen;
            if (!gen && !(d2 < margin)) return;
            sg += gen ? to_fix(d2, kLossFix) : 0ull;
            sf += gen ? 0ull : to_fix(margin - d2, kLossFix);
            const float sign = gen ? 1.f : -1.f;
            unsigned long long *aj = in_lds ? win + (j - base) * 8 : acc + j * 8;
            aj += gen ? 0 : 4;
#pragma unroll
            for (int c = 0; c < kD; c++) {
                const float v = sign * 2.f * (q[c] - e[c]);
                const unsigned long long f = to_fix(v, kGradFix);
                qg[c] += gen ? f : 0ull;
                qf[c] += gen ? 0ull : f;
                atomicAdd(aj + c, to_fix(-v, kGradFix));
            }
        };
        // hard negatives: the other particles' members of the neighbour list
        const int dg = deg[i];
        for (int t = lane; t < dg; t += 64) {
            const int64_t j = s + nbr[i * kmax + t];
            if (!same(j)) pair(j);
        }
        // genuine pairs: the candidates of the query's particle
        for (int c = lane; c < C; c += 64)
            if (same(base + c)) pair(base + c);
        // the random pair
        if (C > 0 && lane == 0) pair(base + (int64_t)(((unsigned long long)rnd[i] * (unsigned)C) >> 32));
#pragma unroll
        for (int c = 0; c < kD; c++)
            for (int o = 32; o > 0; o >>= 1) {
                qg[c] += (unsigned long long)__shfl_xor((long long)qg[c], o);
                qf[c] += (unsigned long long)__shfl_xor((long long)qf[c], o);
            }
        if (lane < 8) {
            unsigned long long v = qg[0];
#pragma unroll
            for (int c = 1; c < 2 * kD; c++) v = lane == c ? (c < kD ? qg[c] : qf[c - kD]) : v;
            if (v) atomicAdd(acc + i * 8 + lane, v);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        sg += (unsigned long long)__shfl_xor((long long)sg, o);
        sf += (unsigned long long)__shfl_xor((long long)sf, o);
        ng += (unsigned long long)__shfl_xor((long long)ng, o);
        nf += (unsigned long long)__shfl_xor((long long)nf, o);
    }
    if (lane == 0) {
        if (sg) atomicAdd(stat + 0, sg);
        if (sf) atomicAdd(stat + 1, sf);
        if (ng) atomicAdd(stat + 2, ng);
        if (nf) atomicAdd(stat + 3, nf);
    }
    if (in_lds) {
        __syncthreads();
        for (int k = threadIdx.x; k < C * 8; k += kPairBlock)
            if (win[k]) atomicAdd(acc + base * 8 + k, win[k]);
    }
}

// Back-propagation per hit, 16 hits per wavefront unit in the transposed MFMA
// form: dE = (w / N_g) G_g + (1 / N_f) G_f, dz2 = [a2 > 0] (W3^T dE),
// dz1 = [a1 > 0] (W2^T dz2).  Writes dz3 = dE, dz2, dz1 per hit.
__global__ __launch_bounds__(512) void k_emb_bwd(int64_t n_hits, const float *__restrict__ P_, int64_t o_w2,
                                                 int64_t o_w3, const unsigned long long *__restrict__ acc,
                                                 const unsigned long long *__restrict__ stat, float w_genuine,
                                                 const float *__restrict__ a1, const float *__restrict__ a2,
                                                 float *__restrict__ dz1, float *__restrict__ dz2,
                                                 float *__restrict__ dz3, const unsigned *__restrict__ flags) {
    constexpr int MO = kCe / 16, KB = kCe / F32::KBLK;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    f32x4 *sW2T = (f32x4 *)lds_raw;
    float *sW3 = (float *)(lds_raw + frag_bytes<F32>(kCe, kCe));
    stage<F32, true>(sW2T, P_ + o_w2, kCe, kCe, MO);
    for (int t = threadIdx.x; t < kD * kCe; t += blockDim.x) sW3[t] = P_[o_w3 + t];
    __syncthreads();
    if (*flags & kErrInput) return;
    const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
    const double ngd = (double)(long long)stat[2], nfd = (double)(long long)stat[3];
    const double cg = ngd > 0 ? (double)w_genuine / ngd : 0.0, cf = nfd > 0 ? 1.0 / nfd : 0.0;
    const int64_t units = (n_hits + 15) >> 4;
    for (int64_t u = wave_id(); u < units; u += n_waves()) {
        const int64_t i = u * 16 + n;
        const int64_t ic = i < n_hits ? i : n_hits - 1;
        float dE[kD];
#pragma unroll
        for (int c = 0; c < kD; c++)
            dE[c] = (float)(cg * from_fix(acc[ic * 8 + c], kGradFix) + cf * from_fix(acc[ic * 8 + 4 + c], kGradFix));
        if (g == 0 && i < n_hits) *(f32x4 *)(dz3 + i * 4) = f32x4{dE[0], dE[1], dE[2], dE[3]};
        f32x4 x2[MO];
#pragma unroll
        for (int mo = 0; mo < MO; mo++) {
            const f32x4 r2 = *(const f32x4 *)(a2 + ic * kCe + 16 * mo + 4 * g);
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int ch = 16 * mo + 4 * g + j;
                float s = 0.f;
#pragma unroll
                for (int c = 0; c < kD; c++) s = __builtin_fmaf(sW3[c * kCe + ch], dE[c], s);
                x2[mo][j] = r2[j] > 0.f ? s : 0.f;
            }
        }
        if (i < n_hits) F32::store_all<MO>(dz2 + i * kCe, g, x2);
        f32x4 y1[MO];
        zero<MO>(y1);
        gemm<F32, MO, KB>(sW2T, x2, y1, lane);
#pragma unroll
        for (int mo = 0; mo < MO; mo++) {
            const f32x4 r1 = *(const f32x4 *)(a1 + ic * kCe + 16 * mo + 4 * g);
#pragma unroll
            for (int j = 0; j < 4; j++) y1[mo][j] = r1[j] > 0.f ? y1[mo][j] : 0.f;
        }
        if (i < n_hits) F32::store_all<MO>(dz1 + i * kCe, g, y1);
    }
}

// Weight-gradient partial sums of one chunk of kDwChunk hits (block per
// chunk), every sum over the chunk's hits in index order:
//   dW1 = sum dz1 u^T, db1 = sum dz1, dW2 = sum dz2 a1^T, db2 = sum dz2,
//   dW3 = sum dE a2^T, db3 = sum dE.
// Thread t owns dW2 rows t/2, columns 64 (t % 2) .. +63; threads below 128
// also own row t of dW3^T and db2[t], the others row t - 128 of dW1 and db1.
__global__ __launch_bounds__(256) void k_emb_dw(int64_t n_hits, const float *__restrict__ sv,
                                                const float *__restrict__ a1, const float *__restrict__ a2,
                                                const float *__restrict__ dz1, const float *__restrict__ dz2,
                                                const float *__restrict__ dz3, float *__restrict__ part) {
    __shared__ __align__(16) float sA1[kDwSub][kCe], sA2[kDwSub][kCe], sZ1[kDwSub][kCe], sZ2[kDwSub][kCe];
    __shared__ __align__(16) float sZ3[kDwSub][4], sU[kDwSub][4];
    const int t = threadIdx.x;
    const int o = t >> 1, k0 = (t & 1) * 64;
    const int64_t h0 = (int64_t)blockIdx.x * kDwChunk, h1 = min(h0 + kDwChunk, n_hits);
    float w2[64];
#pragma unroll
    for (int q = 0; q < 64; q++) w2[q] = 0.f;
    float ex[4] = {0.f, 0.f, 0.f, 0.f}, eb = 0.f, b3 = 0.f;
    for (int64_t hs = h0; hs < h1; hs += kDwSub) {
        const int ns = (int)min((int64_t)kDwSub, h1 - hs);
        __syncthreads();   // the previous rows are consumed
        for (int f = t; f < kDwSub * kCe / 4; f += blockDim.x) {
            const int r = f / (kCe / 4), c4 = (f % (kCe / 4)) * 4;
            const bool in = r < ns;
            const int64_t row = (hs + r) * kCe + c4;
            const f32x4 z = f32x4{0.f, 0.f, 0.f, 0.f};
            *(f32x4 *)&sA1[r][c4] = in ? *(const f32x4 *)(a1 + row) : z;
            *(f32x4 *)&sA2[r][c4] = in ? *(const f32x4 *)(a2 + row) : z;
            *(f32x4 *)&sZ1[r][c4] = in ? *(const f32x4 *)(dz1 + row) : z;
            *(f32x4 *)&sZ2[r][c4] = in ? *(const f32x4 *)(dz2 + row) : z;
        }
        if (t < kDwSub) {
            const bool in = t < ns;
            const f32x4 z = f32x4{0.f, 0.f, 0.f, 0.f};
            *(f32x4 *)&sZ3[t][0] = in ? *(const f32x4 *)(dz3 + (hs + t) * 4) : z;
            *(f32x4 *)&sU[t][0] = in ? *(const f32x4 *)(sv + (hs + t) * 4) : z;
        }
        __syncthreads();
        for (int r = 0; r < kDwSub; r++) {
            const float z2 = sZ2[r][o];
#pragma unroll
            for (int q = 0; q < 64; q += 4) {
                const f32x4 a = *(const f32x4 *)&sA1[r][k0 + q];
#pragma unroll
                for (int j = 0; j < 4; j++) w2[q + j] = __builtin_fmaf(z2, a[j], w2[q + j]);
            }
            if (t < kCe) {
                const float a2v = sA2[r][t];
#pragma unroll
                for (int c = 0; c < kD; c++) ex[c] = __builtin_fmaf(sZ3[r][c], a2v, ex[c]);
                eb += sZ2[r][t];
            } else {
                const float z1 = sZ1[r][t - kCe];
#pragma unroll
                for (int c = 0; c < 3; c++) ex[c] = __builtin_fmaf(z1, sU[r][c], ex[c]);
                eb += z1;
            }
            if (t < kD) b3 += sZ3[r][t];
        }
    }
    float *out = part + (int64_t)blockIdx.x * kEmbParams;
#pragma unroll
    for (int q = 0; q < 64; q++) out[kOffW2 + o * kCe + k0 + q] = w2[q];
    if (t < kCe) {
#pragma unroll
        for (int c = 0; c < kD; c++) out[kOffW3 + c * kCe + t] = ex[c];
        out[kOffB2 + t] = eb;
    } else {
        const int k = t - kCe;
#pragma unroll
        for (int c = 0; c < 3; c++) out[k * 3 + c] = ex[c];
        out[kOffB1 + k] = eb;
    }
    if (t < kD) out[kOffB3 + t] = b3;
}

// dparams[o_emb + q] = sum over the chunks, in order, of part[chunk][q]
__global__ __launch_bounds__(256) void k_emb_dw_reduce(int64_t chunks, const float *__restrict__ part,
                                                       float *__restrict__ dparams, int64_t o_emb) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < kEmbParams; q += gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int64_t ch = 0; ch < chunks; ch++) s += part[ch * kEmbParams + q];
        dparams[o_emb + q] = s;
    }
}

// loss = {w S_g / N_g + S_f / N_f, S_g / N_g, S_f / N_f}; counts = {N_g, N_f}
__global__ void k_emb_loss(const unsigned long long *__restrict__ stat, float w_genuine, float *__restrict__ loss,
                           int64_t *__restrict__ counts) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double Sg = from_fix(stat[0], kLossFix), Sf = from_fix(stat[1], kLossFix);
    const long long ng = (long long)stat[2], nf = (long long)stat[3];
    const double lg = ng > 0 ? Sg / (double)ng : 0.0, lf = nf > 0 ? Sf / (double)nf : 0.0;
    loss[0] = (float)((double)w_genuine * lg + lf);
    loss[1] = (float)lg;
    loss[2] = (float)lf;
    counts[0] = ng;
    counts[1] = nf;
}

inline int blocks_per_cu_dyn(const void *kernel, int block, size_t lds) {
    (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   // a failure is the launch's error
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, block, lds) != hipSuccess || n < 1) n = 1;
    return n;
}

}  // namespace

int64_t emb_train_chunks(int64_t n_hits) { return (n_hits + kDwChunk - 1) / kDwChunk; }

void launch_embed_train_grad(velo_ctx *c, const velo_hits *h, const velo_embed_truth *truth, const float *params,
                             int k_train, float d2_train, float margin, float w_genuine, float *dparams,
                             float *loss, int64_t *counts, float *emb, hipStream_t s) {
    Workspace &w = c->ws;
    const ParamLayout &L = c->layout;
    const int64_t N = h->n_hits;
    float *e = emb ? emb : w.emb;
    { StageTimer t(c, VELO_STAGE_PREPARE, s); launch_prepare(c, h, s); }
    { StageTimer t(c, VELO_STAGE_EMBED, s); launch_embed_train(c, h, params, e, w.t_u, w.t_a1, w.t_a2, s); }
    { StageTimer t(c, VELO_STAGE_KNN, s); launch_knn_into(c, h, e, k_train, d2_train, w.t_nbr, w.t_deg, s); }
    {
        StageTimer t(c, VELO_STAGE_EMB_LOSS, s);
        launch_fill((int *)w.t_acc, 0, N * 16, s);
        launch_fill((int *)w.t_stat, 0, 8, s);
        if (N > 0)
            k_emb_pairs<<<h->n_events * VELO_N_PLANES, kPairBlock, 0, s>>>(
                h->n_events, h->event_offsets, w.plane_off, (const f32x4 *)e, truth->pid, truth->query,
                truth->rnd, w.t_nbr, w.t_deg, k_train, margin, w.t_acc, w.t_stat, w.flags);
        k_emb_loss<<<1, 64, 0, s>>>(w.t_stat, w_genuine, loss, counts);
    }
    {
        StageTimer t(c, VELO_STAGE_EMB_BWD, s);
        const int64_t chunks = emb_train_chunks(N);
        if (N > 0) {
            constexpr size_t lds = frag_bytes<F32>(kCe, kCe) + sizeof(float) * kD * kCe;
            static const int per_cu = blocks_per_cu_dyn(reinterpret_cast<const void *>(&k_emb_bwd), 512, lds);
            k_emb_bwd<<<persistent_grid(c, per_cu), 512, lds, s>>>(N, params, L.emb[1].w, L.emb[2].w, w.t_acc,
                                                                  w.t_stat, w_genuine, w.t_a1, w.t_a2, w.t_dz1,
                                                                  w.t_dz2, w.t_dz3, w.flags);
            k_emb_dw<<<(int)chunks, 256, 0, s>>>(N, w.t_u, w.t_a1, w.t_a2, w.t_dz1, w.t_dz2, w.t_dz3, w.t_part);
        }
        k_emb_dw_reduce<<<(kEmbParams + 255) / 256, 256, 0, s>>>(chunks, w.t_part, dparams, L.emb[0].w);
    }
}

}  // namespace velo
