// gnn.hip -- embedding MLP and interaction-network GNN on MFMA (gfx950).
//
// Every MLP of the path (paper Sec. 5.1 embedding; Sec. 5.2 node/edge
// encoders, node/edge networks, edge classifier) is a dense contraction and
// runs on v_mfma_f32_16x16x4f32 in the "transposed" form
//     OUT^T (channels x items) = W (channels x K) * X^T (K x items)
// with 16 items (hits or edges) per wavefront unit.  Lane l = 16 g + n owns
// item n and, of every 16-wide block of channels or inputs, the four values
// 16 kb + 4 g + (0..3).  With that ownership
//   * a lane loads its item's inputs as float4 (B operand, 4 k-steps),
//   * the weight fragment of a k-step is a float4 of a weight row (A operand),
//   * the 16x16 accumulator of an output block holds exactly the values the
//     next layer needs as its B operand, so two-layer MLPs chain in registers
//     and the residual input is already in the lane that adds it.
// Weights are staged once per block in LDS with a padded row stride.
//
// Messages (the scatter_add of the message equation, Sec. 5.2) are sums in a
// fixed order over per-hit incidence lists, in float32.
#include "internal.h"

namespace velo {

namespace {

__device__ inline f32x4 mfma(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ inline f32x4 zero4() { return f32x4{0.f, 0.f, 0.f, 0.f}; }

// Copy a row-major [rows x cols] matrix into LDS with row stride `stride`,
// zero-filling rows [rows, rows_pad).
__device__ inline void stage(float *dst, const float *__restrict__ W, int rows, int cols, int stride,
                             int rows_pad) {
    const int total = rows_pad * cols;
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
        const int r = t / cols, c = t - r * cols;
        dst[r * stride + c] = r < rows ? W[t] : 0.f;
    }
}

// acc[mo] += W[16 mo + r, 16 kb + 4 g + i] * X[kb][i]   over kb < KB, i < 4
template <int MO, int KB>
__device__ inline void gemm(const float *sW, int stride, const f32x4 *X, f32x4 *acc, int r, int g) {
#pragma unroll
    for (int kb = 0; kb < KB; kb++) {
        // keep one k-block of weight fragments live at a time
        __builtin_amdgcn_sched_barrier(0);
        f32x4 a[MO];
#pragma unroll
        for (int mo = 0; mo < MO; mo++)
            a[mo] = *(const f32x4 *)(sW + (16 * mo + r) * stride + 16 * kb + 4 * g);
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int mo = 0; mo < MO; mo++) acc[mo] = mfma(a[mo][i], X[kb][i], acc[mo]);
    }
}

// Per-lane copy of bias values b[16 mo + 4 g + i].
template <int MO>
__device__ inline void load_bias(const float *__restrict__ b, f32x4 *rb, int g) {
#pragma unroll
    for (int mo = 0; mo < MO; mo++) rb[mo] = *(const f32x4 *)(b + 16 * mo + 4 * g);
}

template <int MO>
__device__ inline void bias_relu(f32x4 *acc, const f32x4 *rb) {
#pragma unroll
    for (int mo = 0; mo < MO; mo++)
#pragma unroll
        for (int i = 0; i < 4; i++) acc[mo][i] = fmaxf(acc[mo][i] + rb[mo][i], 0.f);
}

__device__ inline int wave_id() { return (blockIdx.x * blockDim.x + threadIdx.x) >> 6; }
__device__ inline int n_waves() { return (gridDim.x * blockDim.x) >> 6; }

// ------------------------------------------------------------------------
// embedding MLP 3 -> 128 -> 128 -> 4 on normalised (r, phi, z)  (Sec. 5.1)
// ------------------------------------------------------------------------
constexpr int kCe = VELO_EMB_HIDDEN;
constexpr int kSe = kCe + 4;    // LDS row stride

__global__ __launch_bounds__(512) void k_embed(int64_t n_hits, const float *__restrict__ x,
                                               const float *__restrict__ y, const float *__restrict__ z,
                                               const float *__restrict__ P, int64_t o_w1, int64_t o_w2,
                                               int64_t o_w3, float *__restrict__ emb,
                                               const unsigned *__restrict__ flags) {
    extern __shared__ float lds[];
    float *sW2 = lds;                       // [128 x kSe]
    float *sW3 = sW2 + kCe * kSe;           // [16 x kSe], rows >= 4 zero
    float *sW1 = sW3 + 16 * kSe;            // [128 x 3] + b1[128]
    stage(sW2, P + o_w2, kCe, kCe, kSe, kCe);
    stage(sW3, P + o_w3, VELO_EMB_DIM, kCe, kSe, 16);
    for (int t = threadIdx.x; t < kCe * 4; t += blockDim.x) sW1[t] = P[o_w1 + t];   // W1 then b1
    __syncthreads();
    if (*flags & kErrInput) return;

    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    const float *b2 = P + o_w2 + kCe * kCe, *b3 = P + o_w3 + VELO_EMB_DIM * kCe;
    const float mu0 = P[0], mu1 = P[1], mu2 = P[2], sg0 = P[3], sg1 = P[4], sg2 = P[5];
    f32x4 rb2[8];
    load_bias<8>(b2, rb2, g);
    const int64_t units = (n_hits + 15) >> 4;
    for (int64_t u = wave_id(); u < units; u += n_waves()) {
        const int64_t i = u * 16 + n;
        const int64_t ic = i < n_hits ? i : n_hits - 1;
        const float X = x[ic], Y = y[ic], Z = z[ic];
        const float u0 = (sqrtf(X * X + Y * Y) - mu0) / sg0;
        const float u1 = (atan2f(Y, X) - mu1) / sg1;
        const float u2 = (Z - mu2) / sg2;
        f32x4 h1[8];
#pragma unroll
        for (int mo = 0; mo < 8; mo++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int c = 16 * mo + 4 * g + q;
                const float v = sW1[c * 3 + 0] * u0 + sW1[c * 3 + 1] * u1 + sW1[c * 3 + 2] * u2 + sW1[kCe * 3 + c];
                h1[mo][q] = fmaxf(v, 0.f);
            }
        f32x4 h2[8];
#pragma unroll
        for (int mo = 0; mo < 8; mo++) h2[mo] = zero4();
        gemm<8, 8>(sW2, kSe, h1, h2, n, g);
        bias_relu<8>(h2, rb2);
        f32x4 o[1] = {zero4()};
        gemm<1, 8>(sW3, kSe, h2, o, n, g);
        if (g == 0 && i < n_hits) {
            f32x4 r;
#pragma unroll
            for (int q = 0; q < 4; q++) r[q] = o[0][q] + b3[q];
            *(f32x4 *)(emb + i * 4) = r;
        }
    }
}

// ------------------------------------------------------------------------
// node encoder 3 -> H -> H on normalised (x, y, z)  (Sec. 5.2)
// ------------------------------------------------------------------------
template <int H>
__global__ __launch_bounds__(512) void k_node_enc(int64_t n_hits, const float *__restrict__ x,
                                                  const float *__restrict__ y, const float *__restrict__ z,
                                                  const float *__restrict__ P, int64_t o_w1, int64_t o_w2,
                                                  float *__restrict__ h, const unsigned *__restrict__ flags) {
    constexpr int MO = H / 16, S = H + 4;
    extern __shared__ float lds[];
    float *sW2 = lds;
    float *sW1 = sW2 + H * S;     // [H x 3] then b1[H]
    stage(sW2, P + o_w2, H, H, S, H);
    for (int t = threadIdx.x; t < H * 4; t += blockDim.x) sW1[t] = P[o_w1 + t];
    __syncthreads();
    if (*flags) return;
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    const float mu0 = P[6], mu1 = P[7], mu2 = P[8], sg0 = P[9], sg1 = P[10], sg2 = P[11];
    f32x4 rb2[MO];
    load_bias<MO>(P + o_w2 + H * H, rb2, g);
    const int64_t units = (n_hits + 15) >> 4;
    for (int64_t u = wave_id(); u < units; u += n_waves()) {
        const int64_t i = u * 16 + n;
        const int64_t ic = i < n_hits ? i : n_hits - 1;
        const float u0 = (x[ic] - mu0) / sg0, u1 = (y[ic] - mu1) / sg1, u2 = (z[ic] - mu2) / sg2;
        f32x4 h1[MO];
#pragma unroll
        for (int mo = 0; mo < MO; mo++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int c = 16 * mo + 4 * g + q;
                h1[mo][q] = fmaxf(sW1[c * 3] * u0 + sW1[c * 3 + 1] * u1 + sW1[c * 3 + 2] * u2 + sW1[H * 3 + c], 0.f);
            }
        f32x4 o[MO];
#pragma unroll
        for (int mo = 0; mo < MO; mo++) o[mo] = zero4();
        gemm<MO, MO>(sW2, S, h1, o, n, g);
        if (i < n_hits) {
#pragma unroll
            for (int mo = 0; mo < MO; mo++) {
                f32x4 r = o[mo] + rb2[mo];
                *(f32x4 *)(h + i * H + 16 * mo + 4 * g) = r;
            }
        }
    }
}

// ------------------------------------------------------------------------
// generic two-layer MLP over gathered segments
//   NODE:     X = [h_in[i], m[i, 0:H], m[i, H:2H]],  h_out[i] = h_in[i] + MLP(X)
//   EDGE:     X = [e[q], h[src q], h[dst q]],        e[q] = e[q] + MLP(X) (in place)
//   EDGE_ENC: X = [h[src q], h[dst q]],              e[q] = MLP(X)
// With CLS the edge classifier H -> H -> 1 runs on the result (Sec. 5.2) and
// writes the logit.
// ------------------------------------------------------------------------
enum Mode { NODE = 0, EDGE = 1, EDGE_ENC = 2, CLS_ONLY = 3 };

struct MlpArgs {
    const int *n_dev;      // device item count (edges) or null
    int64_t n_host;        // host item count (hits) or cap for edges
    const int *src_g, *dst_g;
    const float *a;        // NODE: h_in; EDGE: e (in/out); EDGE_ENC: h0; CLS_ONLY: e
    const float *b;        // NODE: m; EDGE: h (updated)
    float *out;            // NODE: h_out; EDGE/EDGE_ENC: e
    const float *P;
    int64_t o_w1, o_w2;    // this MLP's layers
    int64_t o_c1, o_c2;    // classifier layers (CLS)
    float *logit;
    const unsigned *flags;
};

template <int H, int MO>
__device__ inline void classify(const float *sC1, int S, const float *__restrict__ P, int64_t o_c1,
                                int64_t o_c2, const f32x4 *ev, int n, int g, bool ok, int64_t q,
                                float *__restrict__ logit) {
    f32x4 hc[MO];
#pragma unroll
    for (int mo = 0; mo < MO; mo++) hc[mo] = zero4();
    gemm<MO, MO>(sC1, S, ev, hc, n, g);
    f32x4 rb[MO], w2[MO];
    load_bias<MO>(P + o_c1 + H * H, rb, g);
    load_bias<MO>(P + o_c2, w2, g);
    float part = 0.f;
#pragma unroll
    for (int mo = 0; mo < MO; mo++)
#pragma unroll
        for (int i = 0; i < 4; i++) part += w2[mo][i] * fmaxf(hc[mo][i] + rb[mo][i], 0.f);
    part += __shfl_xor(part, 16);
    part += __shfl_xor(part, 32);
    if (g == 0 && ok) logit[q] = part + P[o_c2 + H];
}

template <int H, int MODE, bool CLS>
__global__ __launch_bounds__(512) void k_mlp(MlpArgs A) {
    constexpr int MO = H / 16;
    constexpr int NSEG = MODE == EDGE_ENC ? 2 : (MODE == CLS_ONLY ? 0 : 3);
    constexpr int K1 = NSEG * H, S1 = K1 + 4, S = H + 4;
    extern __shared__ float lds[];
    float *sW1 = lds;                          // [H x S1]
    float *sW2 = sW1 + (NSEG ? H * S1 : 0);    // [H x S]
    float *sC1 = sW2 + (NSEG ? H * S : 0);     // [H x S] classifier layer 1
    if (NSEG) {
        stage(sW1, A.P + A.o_w1, H, K1, S1, H);
        stage(sW2, A.P + A.o_w2, H, H, S, H);
    }
    if (CLS) stage(sC1, A.P + A.o_c1, H, H, S, H);
    __syncthreads();
    if (*A.flags) return;

    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    int64_t N = A.n_host;
    if (A.n_dev) N = min((int64_t)*A.n_dev, A.n_host);
    f32x4 rb1[MO], rb2[MO];
    if (NSEG) {
        load_bias<MO>(A.P + A.o_w1 + (int64_t)H * K1, rb1, g);
        load_bias<MO>(A.P + A.o_w2 + (int64_t)H * H, rb2, g);
    }
    const int64_t units = (N + 15) >> 4;
    for (int64_t u = wave_id(); u < units; u += n_waves()) {
        const int64_t q = u * 16 + n;
        const bool ok = q < N;
        const int64_t qc = ok ? q : N - 1;
        f32x4 X[NSEG > 0 ? NSEG * MO : MO];
        if (MODE == NODE) {
#pragma unroll
            for (int kb = 0; kb < MO; kb++) {
                X[kb] = *(const f32x4 *)(A.a + qc * H + 16 * kb + 4 * g);
                X[MO + kb] = *(const f32x4 *)(A.b + qc * 2 * H + 16 * kb + 4 * g);
                X[2 * MO + kb] = *(const f32x4 *)(A.b + qc * 2 * H + H + 16 * kb + 4 * g);
            }
        } else if (MODE == EDGE) {
            const int64_t s = A.src_g[qc], d = A.dst_g[qc];
#pragma unroll
            for (int kb = 0; kb < MO; kb++) {
                X[kb] = *(const f32x4 *)(A.a + qc * H + 16 * kb + 4 * g);
                X[MO + kb] = *(const f32x4 *)(A.b + s * H + 16 * kb + 4 * g);
                X[2 * MO + kb] = *(const f32x4 *)(A.b + d * H + 16 * kb + 4 * g);
            }
        } else if (MODE == EDGE_ENC) {
            const int64_t s = A.src_g[qc], d = A.dst_g[qc];
#pragma unroll
            for (int kb = 0; kb < MO; kb++) {
                X[kb] = *(const f32x4 *)(A.a + s * H + 16 * kb + 4 * g);
                X[MO + kb] = *(const f32x4 *)(A.a + d * H + 16 * kb + 4 * g);
            }
        } else {
#pragma unroll
            for (int kb = 0; kb < MO; kb++) X[kb] = *(const f32x4 *)(A.a + qc * H + 16 * kb + 4 * g);
        }
        f32x4 o[MO];
        if (NSEG) {
            f32x4 hid[MO];
#pragma unroll
            for (int mo = 0; mo < MO; mo++) hid[mo] = zero4();
            gemm<MO, NSEG * MO>(sW1, S1, X, hid, n, g);
            bias_relu<MO>(hid, rb1);
#pragma unroll
            for (int mo = 0; mo < MO; mo++) o[mo] = zero4();
            gemm<MO, MO>(sW2, S, hid, o, n, g);
#pragma unroll
            for (int mo = 0; mo < MO; mo++) {
                o[mo] += rb2[mo];
                if (MODE != EDGE_ENC) o[mo] += X[mo];     // residual (Sec. 5.2)
            }
            if (ok && !(CLS && MODE == EDGE)) {
#pragma unroll
                for (int mo = 0; mo < MO; mo++) *(f32x4 *)(A.out + q * H + 16 * mo + 4 * g) = o[mo];
            }
        } else {
#pragma unroll
            for (int mo = 0; mo < MO; mo++) o[mo] = X[mo];
        }
        if (CLS) classify<H, MO>(sC1, S, A.P, A.o_c1, A.o_c2, o, n, g, ok, q, A.logit);
    }
}

// ------------------------------------------------------------------------
// messages m_i = [sum_{i->j} e_ij, sum_{j->i} e_ji]  (Sec. 5.2, scatter_add)
// H/4 lanes per hit, float4 per lane; fixed summation order (edge id order)
// ------------------------------------------------------------------------
template <int H>
__global__ __launch_bounds__(256) void k_messages(int64_t n_hits, const int *__restrict__ out_ptr,
                                                  const int *__restrict__ out_list,
                                                  const int *__restrict__ in_ptr,
                                                  const int *__restrict__ in_list,
                                                  const float *__restrict__ e, float *__restrict__ m,
                                                  const unsigned *__restrict__ flags) {
    if (*flags) return;
    constexpr int LPN = H / 4, NPW = 64 / LPN;
    const int lane = threadIdx.x & 63, sub = lane / LPN, c = 4 * (lane % LPN);
    for (int64_t base = (int64_t)wave_id() * NPW; base < n_hits; base += (int64_t)n_waves() * NPW) {
        const int64_t i = base + sub;
        if (i >= n_hits) continue;
        f32x4 so = zero4(), si = zero4();
        const int a0 = out_ptr[i], a1 = out_ptr[i + 1];
        if (out_list) {
            for (int a = a0; a < a1; a++) so += *(const f32x4 *)(e + (int64_t)out_list[a] * H + c);
        } else {
            int a = a0;
            for (; a + 4 <= a1; a += 4) {
                const f32x4 v0 = *(const f32x4 *)(e + (int64_t)a * H + c);
                const f32x4 v1 = *(const f32x4 *)(e + (int64_t)(a + 1) * H + c);
                const f32x4 v2 = *(const f32x4 *)(e + (int64_t)(a + 2) * H + c);
                const f32x4 v3 = *(const f32x4 *)(e + (int64_t)(a + 3) * H + c);
                so += v0; so += v1; so += v2; so += v3;
            }
            for (; a < a1; a++) so += *(const f32x4 *)(e + (int64_t)a * H + c);
        }
        const int b0 = in_ptr[i], b1 = in_ptr[i + 1];
        int b = b0;
        for (; b + 4 <= b1; b += 4) {
            const int q0 = in_list[b], q1 = in_list[b + 1], q2 = in_list[b + 2], q3 = in_list[b + 3];
            const f32x4 v0 = *(const f32x4 *)(e + (int64_t)q0 * H + c);
            const f32x4 v1 = *(const f32x4 *)(e + (int64_t)q1 * H + c);
            const f32x4 v2 = *(const f32x4 *)(e + (int64_t)q2 * H + c);
            const f32x4 v3 = *(const f32x4 *)(e + (int64_t)q3 * H + c);
            si += v0; si += v1; si += v2; si += v3;
        }
        for (; b < b1; b++) si += *(const f32x4 *)(e + (int64_t)in_list[b] * H + c);
        *(f32x4 *)(m + i * 2 * H + c) = so;
        *(f32x4 *)(m + i * 2 * H + H + c) = si;
    }
}

constexpr int kMlpBlock = 512;

template <int H, int MODE, bool CLS>
void run_mlp(velo_ctx *c, const MlpArgs &a, hipStream_t s) {
    constexpr int NSEG = MODE == EDGE_ENC ? 2 : (MODE == CLS_ONLY ? 0 : 3);
    const size_t lds = sizeof(float) * ((NSEG ? H * (NSEG * H + 4) + H * (H + 4) : 0) + (CLS ? H * (H + 4) : 0));
    static bool attr = false;
    if (!attr) {
        hipFuncSetAttribute(reinterpret_cast<const void *>(&k_mlp<H, MODE, CLS>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        attr = true;
    }
    k_mlp<H, MODE, CLS><<<persistent_grid(c, 1), kMlpBlock, lds, s>>>(a);
}

template <int H>
void gnn_h(velo_ctx *c, const velo_hits *hits, bool out_identity, float *logit, hipStream_t s) {
    Workspace &w = c->ws;
    const ParamLayout &L = c->layout;
    const float *P = c->params;
    const int64_t N = hits->n_hits, Ecap = c->cfg.max_edges;
    if (N > 0) {
        const size_t lds = sizeof(float) * (H * (H + 4) + H * 4);
        StageTimer t(c, VELO_STAGE_NODE_ENC, s);
        k_node_enc<H><<<persistent_grid(c, 1), kMlpBlock, lds, s>>>(N, hits->x, hits->y, hits->z, P,
                                                                   L.nenc[0].w, L.nenc[1].w, w.h[0], w.flags);
    }
    MlpArgs a{};
    a.n_dev = w.n_edges; a.n_host = Ecap; a.src_g = w.src_g; a.dst_g = w.dst_g;
    a.P = P; a.flags = w.flags; a.logit = logit;
    a.o_c1 = L.cls[0].w; a.o_c2 = L.cls[1].w;
    a.a = w.h[0]; a.out = w.e; a.o_w1 = L.eenc[0].w; a.o_w2 = L.eenc[1].w;
    const int iters = c->cfg.gnn_iters;
    if (iters == 0) {
        StageTimer t(c, VELO_STAGE_EDGE_CLS, s);
        run_mlp<H, EDGE_ENC, true>(c, a, s);
        return;
    }
    {
        StageTimer t(c, VELO_STAGE_EDGE_ENC, s);
        run_mlp<H, EDGE_ENC, false>(c, a, s);
    }
    int cur = 0;
    const int *optr = out_identity ? w.row_ptr : w.out_ptr;
    const int *olist = out_identity ? nullptr : w.out_list;
    for (int k = 0; k < iters; k++) {
        if (N > 0) {
            StageTimer t(c, VELO_STAGE_MESSAGES, s);
            k_messages<H><<<persistent_grid(c, 16), 256, 0, s>>>(N, optr, olist, w.in_ptr, w.in_list, w.e,
                                                               w.m, w.flags);
        }
        MlpArgs nd{};
        nd.n_dev = nullptr; nd.n_host = N; nd.a = w.h[cur]; nd.b = w.m; nd.out = w.h[cur ^ 1];
        nd.P = P; nd.o_w1 = L.node[k][0].w; nd.o_w2 = L.node[k][1].w; nd.flags = w.flags;
        if (N > 0) {
            StageTimer t(c, VELO_STAGE_NODE_NET, s);
            run_mlp<H, NODE, false>(c, nd, s);
        }
        cur ^= 1;
        MlpArgs ed = a;
        ed.a = w.e; ed.b = w.h[cur]; ed.out = w.e; ed.o_w1 = L.edge[k][0].w; ed.o_w2 = L.edge[k][1].w;
        StageTimer t(c, k == iters - 1 ? VELO_STAGE_EDGE_CLS : VELO_STAGE_EDGE_NET, s);
        if (k == iters - 1)
            run_mlp<H, EDGE, true>(c, ed, s);
        else
            run_mlp<H, EDGE, false>(c, ed, s);
    }
}

}  // namespace

void launch_embed(velo_ctx *c, const velo_hits *h, float *emb, hipStream_t s) {
    if (h->n_hits <= 0) return;
    const size_t lds = sizeof(float) * (kCe * kSe + 16 * kSe + kCe * 4);
    static bool attr = false;
    if (!attr) {
        hipFuncSetAttribute(reinterpret_cast<const void *>(&k_embed), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
        attr = true;
    }
    const ParamLayout &L = c->layout;
    k_embed<<<persistent_grid(c, 1), kMlpBlock, lds, s>>>(h->n_hits, h->x, h->y, h->z, c->params,
                                                          L.emb[0].w, L.emb[1].w, L.emb[2].w, emb,
                                                          c->ws.flags);
}

void launch_gnn(velo_ctx *c, const velo_hits *h, bool out_identity, float *logit, hipStream_t s) {
    switch (c->cfg.gnn_hidden) {
        case 32: gnn_h<32>(c, h, out_identity, logit, s); break;
        case 64: gnn_h<64>(c, h, out_identity, logit, s); break;
        default: break;   // rejected by velo_create
    }
}

}  // namespace velo
