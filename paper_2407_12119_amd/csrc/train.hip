// train.hip -- the training form of the GNN: weighted binary cross-entropy on
// the edge logits and the reverse-mode pass through the classifier, the n
// message-passing steps and the encoders (paper Sec. 5.2 defines the
// forward; the paper trains with a sigmoid focal loss, here weighted BCE).
//
// Memory: the forward pass keeps only the step-boundary states h^k, e^k and
// the messages m^k; every MLP's hidden activation is recomputed from them in
// the backward kernel (one recompute per MLP, no stored activations).
//
// The edge MLPs' first layers are factorised as in the forward pass:
// W1 [e, h_s, h_d] = W1_e e + AB[s][0:H] + AB[d][H:2H] with the per-hit
// products AB of every step kept by the forward pass.
// Per step k, in reverse:
//   k_bwd<EDGE_AB> recompute a = b1 + AB_s + AB_d + W1_e e^k exactly as the
//                 forward kernel does, r = relu(a); da = (W2^T dout) * [a > 0];
//                 dL/de^k = dout + W1_e^T da (residual).
//   k_gather_pair per hit: S = sum of da over out-edges, D = over in-edges
//                 (the dual of the gathers, in a fixed order).
//   k_hit_dual    dL/dh^{k+1} += W1_s^T S + W1_d^T D.
//   k_bwd<NODE>   the same for the node network; dL/dh^k, dL/dm^k.
//   The dual of step k's message sums, dL/de^k += dL/dm_out[src] +
//   dL/dm_in[dst], is added where dL/de^k is read: in the backward kernel of
//   edge network k-1 (or of the edge encoder), which writes the sum back.
//   k_dw_lds      weight and bias gradients, dW = G^T Y summed over rows, on
//                 MFMA with the row dimension as K, split over chunks of rows;
//                 k_chunk_groups and k_dw_reduce add the chunk partials in a
//                 fixed order (groups of chunks, then the groups).
// No floating-point atomics: gradients are bitwise reproducible.
#include "mfma.h"

namespace velo {

namespace {

using namespace mfma;
using P = F32;

// B_EDGE / B_EDGE_ENC: the concatenated first layer (weight gradients);
// B_EDGE_AB / B_ENC_AB: the factorised one (recompute and input gradients)
enum BMode { B_EDGE = 0, B_NODE = 1, B_EDGE_ENC = 2, B_NODE_ENC = 3, B_CLS = 4, B_EDGE_AB = 5, B_ENC_AB = 6 };

constexpr int kBwdBlock = 256;
constexpr int kChunks = 1024;       // row chunks of the weight-gradient reduction
constexpr int kRedGroups = 32;      // the chunk partials are summed in 32 groups of 32, then the groups

struct BwdArgs {
    const int *n_dev;       // device row count (edges) or null
    int64_t n_host;         // host row count (hits) or the edge capacity
    const int *src_g, *dst_g;
    const float *a;         // EDGE: e^k; NODE: h^k; EDGE_ENC: h^0; CLS: e^n
    const float *b;         // EDGE: h^{k+1}; NODE: m^k
    const float *dout;      // dL/d(output) rows [rows x H]; CLS: dL/dlogit [rows]
    float *dres;            // EDGE, NODE: dout + dX(seg 0); CLS: dL/de^n
    float *dx1;             // NODE: dL/dm [rows x 2H]
    float *da, *r;          // hidden gradient and activation [rows x H]
    const float *x, *y, *z; // hit coordinates (NODE_ENC)
    const float *ab;        // EDGE_AB, ENC_AB: per-hit first-layer products [N x 2H]
    const float *dm;        // EDGE_AB, ENC_AB: dL/dm of the step this edge state fed, or null
    float *dout_w;          // with dm: where dout + the message duals are written (dout's rows)
    const float *P;
    int64_t o_w1, o_w2;
    const unsigned *flags;
};

// first-layer input segments multiplied per row, and stored in the weight
template <int MODE>
constexpr int bseg() {
    return MODE == B_EDGE || MODE == B_NODE ? 3 : (MODE == B_EDGE_ENC ? 2 : (MODE == B_ENC_AB ? 0 : 1));
}
template <int MODE>
constexpr int bkseg() { return MODE == B_EDGE_AB ? 3 : (MODE == B_ENC_AB ? 2 : bseg<MODE>()); }

__device__ inline int64_t row_count(const BwdArgs &A) {
    return A.n_dev ? min((int64_t)*A.n_dev, A.n_host) : A.n_host;
}

// ------------------------------------------------------------------------
// recompute + backward of one two-layer MLP over 16-row units
// ------------------------------------------------------------------------
template <int H, int MODE>
__global__ __launch_bounds__(kBwdBlock) void k_bwd(BwdArgs A) {
    constexpr int MO = H / 16, NSEG = bseg<MODE>(), K1 = NSEG * H, K1F = bkseg<MODE>() * H;
    constexpr bool CLS = MODE == B_CLS, AB = MODE == B_EDGE_AB || MODE == B_ENC_AB;
    static_assert(MODE != B_EDGE && MODE != B_EDGE_ENC, "the edge MLPs are recomputed in factorised form");
    extern __shared__ __align__(16) unsigned char lds_raw[];
    f32x4 *sW1 = (f32x4 *)lds_raw;                                  // W1 [H x K1] (its first K1 columns)
    f32x4 *sW2T = sW1 + frag_bytes<P>(H, K1) / sizeof(f32x4);       // W2^T [H x H] (not CLS)
    f32x4 *sW1T = sW2T + (CLS ? 0 : frag_bytes<P>(H, H) / sizeof(f32x4));   // W1^T [K1 x H]
    if (NSEG) stage<P>(sW1, A.P + A.o_w1, H, K1, MO, 1.f, K1F);
    if (!CLS) stage<P, true>(sW2T, A.P + A.o_w2, H, H, MO);
    if (NSEG) stage<P, true>(sW1T, A.P + A.o_w1, K1, H, K1 / 16, 1.f, K1F);
    __syncthreads();
    if (*A.flags) return;
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    const int64_t N = row_count(A);
    f32x4 rb1[MO], w2[MO];
    load_bias<MO>(A.P + A.o_w1 + (int64_t)H * K1F, rb1, g);
    if (CLS) load_bias<MO>(A.P + A.o_w2, w2, g);     // classifier output weights (1 x H)
    const int64_t units = (N + 15) >> 4;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t u = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; u < units; u += nw) {
        const int64_t q = u * 16 + n;
        const bool ok = q < N;
        const int64_t qc = ok ? q : N - 1;
        f32x4 X[NSEG ? NSEG * MO : 1];
        f32x4 G[AB ? 2 * MO : 1];
        if (AB) {
            const int64_t s = A.src_g[qc], d = A.dst_g[qc];
#pragma unroll
            for (int mo = 0; mo < MO; mo++) {
                G[mo] = *(const f32x4 *)(A.ab + s * 2 * H + 16 * mo + 4 * g);
                G[MO + mo] = *(const f32x4 *)(A.ab + d * 2 * H + H + 16 * mo + 4 * g);
            }
            if (MODE == B_EDGE_AB) {
#pragma unroll
                for (int kb = 0; kb < MO; kb++) X[kb] = P::load(A.a + qc * H, kb, g);
            }
        } else if (MODE == B_NODE) {
#pragma unroll
            for (int kb = 0; kb < MO; kb++) {
                X[kb] = P::load(A.a + qc * H, kb, g);
                X[MO + kb] = P::load(A.b + qc * 2 * H, kb, g);
                X[2 * MO + kb] = P::load(A.b + qc * 2 * H + H, kb, g);
            }
        } else {   // B_CLS
#pragma unroll
            for (int kb = 0; kb < MO; kb++) X[kb] = P::load(A.a + qc * H, kb, g);
        }
        // recompute the hidden layer exactly as the forward kernel does
        // (accumulators seeded with the bias), so the ReLU masks agree
        f32x4 r[MO];
#pragma unroll
        for (int mo = 0; mo < MO; mo++) r[mo] = rb1[mo];
        if (AB) {
#pragma unroll
            for (int mo = 0; mo < MO; mo++) {
                r[mo] += G[mo];
                r[mo] += G[MO + mo];
            }
        }
        if constexpr (NSEG > 0) gemm<P, MO, NSEG * MO>(sW1, X, r, lane);
        relu<MO>(r);
        // dL/d(hidden) = W2^T dout, masked by the ReLU
        f32x4 da[MO];
        if (CLS) {
            const float dz = ok ? A.dout[q] : 0.f;
#pragma unroll
            for (int mo = 0; mo < MO; mo++)
#pragma unroll
                for (int i = 0; i < 4; i++) da[mo][i] = r[mo][i] > 0.f ? w2[mo][i] * dz : 0.f;
        } else {
            f32x4 dO[MO];
#pragma unroll
            for (int kb = 0; kb < MO; kb++) dO[kb] = ok ? P::load(A.dout + q * H, kb, g) : zero4();
            if (A.dm) {
                // the dual of the message sums of this edge state (it fed step
                // k+1's messages): dL/de += dL/dm_out[src] + dL/dm_in[dst];
                // the completed gradient is written back for the weight pass
                const int64_t s = A.src_g[qc], d = A.dst_g[qc];
#pragma unroll
                for (int kb = 0; kb < MO; kb++) {
                    dO[kb] += P::load(A.dm + s * 2 * H, kb, g);
                    dO[kb] += P::load(A.dm + d * 2 * H + H, kb, g);
                }
                if (ok) P::store_all<MO>(A.dout_w + q * H, g, dO);
            }
            zero<MO>(da);
            gemm<P, MO, MO>(sW2T, dO, da, lane);
#pragma unroll
            for (int mo = 0; mo < MO; mo++)
#pragma unroll
                for (int i = 0; i < 4; i++) da[mo][i] = r[mo][i] > 0.f ? da[mo][i] : 0.f;
            // dX = W1^T da over the multiplied segments, then the outputs (the
            // hit segments of the edge MLPs are handled per hit from da)
            if constexpr (NSEG > 0) {
                f32x4 dX[NSEG * MO];
                zero<NSEG * MO>(dX);
                gemm<P, NSEG * MO, MO>(sW1T, da, dX, lane);
                if (ok) {
                    // residual path: the output gradient reaches segment 0 unchanged
#pragma unroll
                    for (int mo = 0; mo < MO; mo++) dX[mo] += dO[mo];
                    P::store_all<MO>(A.dres + q * H, g, dX);
                    if (MODE == B_NODE) {
                        P::store_all<MO>(A.dx1 + q * 2 * H, g, dX + MO);
                        P::store_all<MO>(A.dx1 + q * 2 * H + H, g, dX + 2 * MO);
                    }
                }
            }
        }
        if (CLS) {
            f32x4 dX[MO];
            zero<MO>(dX);
            gemm<P, MO, MO>(sW1T, da, dX, lane);
            if (ok) P::store_all<MO>(A.dres + q * H, g, dX);
        }
        if (ok) {
            P::store_all<MO>(A.da + q * H, g, da);
            P::store_all<MO>(A.r + q * H, g, r);
        }
    }
}

// Node encoder backward: recompute the hidden layer on the VALU (K = 3) and
// write dL/d(hidden) and the activation for the weight gradients.
template <int H>
__global__ __launch_bounds__(kBwdBlock) void k_bwd_node_enc(BwdArgs A) {
    constexpr int MO = H / 16;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    f32x4 *sW2T = (f32x4 *)lds_raw;
    float *sW1 = (float *)(lds_raw + frag_bytes<P>(H, H));
    stage<P, true>(sW2T, A.P + A.o_w2, H, H, MO);
    for (int t = threadIdx.x; t < H * 4; t += blockDim.x) sW1[t] = A.P[A.o_w1 + t];
    __syncthreads();
    if (*A.flags) return;
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    const int64_t N = A.n_host;
    const float *Pn = A.P;
    const float mu0 = Pn[6], mu1 = Pn[7], mu2 = Pn[8], sg0 = Pn[9], sg1 = Pn[10], sg2 = Pn[11];
    const int64_t units = (N + 15) >> 4;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t u = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; u < units; u += nw) {
        const int64_t q = u * 16 + n;
        const bool ok = q < N;
        const int64_t qc = ok ? q : N - 1;
        const float u0 = (A.x[qc] - mu0) / sg0, u1 = (A.y[qc] - mu1) / sg1, u2 = (A.z[qc] - mu2) / sg2;
        f32x4 r[MO];
#pragma unroll
        for (int mo = 0; mo < MO; mo++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int c = 16 * mo + 4 * g + i;
                r[mo][i] = fmaxf(sW1[c * 3] * u0 + sW1[c * 3 + 1] * u1 + sW1[c * 3 + 2] * u2 + sW1[H * 3 + c], 0.f);
            }
        f32x4 dO[MO], da[MO];
#pragma unroll
        for (int kb = 0; kb < MO; kb++) dO[kb] = ok ? P::load(A.dout + q * H, kb, g) : zero4();
        zero<MO>(da);
        gemm<P, MO, MO>(sW2T, dO, da, lane);
#pragma unroll
        for (int mo = 0; mo < MO; mo++)
#pragma unroll
            for (int i = 0; i < 4; i++) da[mo][i] = r[mo][i] > 0.f ? da[mo][i] : 0.f;
        if (ok) {
            P::store_all<MO>(A.da + q * H, g, da);
            P::store_all<MO>(A.r + q * H, g, r);
        }
    }
}

// ------------------------------------------------------------------------
// weight gradients of one MLP:
//   dW1 = sum_rows da (x) X,  db1 = sum da,  dW2 = sum dout (x) r,  db2 = sum dout
// written as one blob-shaped partial [dW1 | db1 | dW2 | db2] per row chunk.
// MFMA 16x16x4 with the row dimension as K: lane l supplies G[row][16 m + l%16]
// and Y[row][16 nb + l%16] for row = base + l/16.  Wave w of the block owns the
// output rows 16 w .. 16 w + 15.
// ------------------------------------------------------------------------
template <int H, int MODE>
__global__ __launch_bounds__(kBwdBlock) void k_dw(BwdArgs A, float *__restrict__ part) {
    static_assert(MODE == B_NODE_ENC, "the other MLPs use k_dw_lds");
    constexpr int MO = H / 16;
    constexpr int K1 = 3;
    constexpr int M2 = H;
    constexpr int PL = H * K1 + H + M2 * H + M2;
    if (*A.flags) return;
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
    const int64_t N = row_count(A);
    const int64_t per = (((N + kChunks - 1) / kChunks) + 3) & ~(int64_t)3;
    const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(r0 + per, N);
    float *out = part + (int64_t)blockIdx.x * PL;
    const bool active = w < MO;                        // waves beyond the output rows idle
    const int m = active ? w : 0;
    f32x4 acc1 = zero4(), acc2[MO];
    zero<MO>(acc2);
    float sb1 = 0.f, sb2 = 0.f;
    const float *Pn = A.P;
    for (int64_t base = r0; active && base < r1; base += 4) {
        const int64_t row = base + g;
        const bool ok = row < r1;
        const int64_t rc = ok ? row : (r1 > 0 ? r1 - 1 : 0);
        const float ga = ok ? A.da[rc * H + 16 * m + n] : 0.f;
        sb1 += ga;
        // layer-1 inputs of this row: the normalised coordinates
        float v = 0.f;
        if (n == 0) v = (A.x[rc] - Pn[6]) / Pn[9];
        if (n == 1) v = (A.y[rc] - Pn[7]) / Pn[10];
        if (n == 2) v = (A.z[rc] - Pn[8]) / Pn[11];
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ga, v, acc1, 0, 0, 0);
        const float gd = ok ? A.dout[rc * H + 16 * m + n] : 0.f;
        sb2 += gd;
#pragma unroll
        for (int nb = 0; nb < MO; nb++) {
            const float y = ok ? A.r[rc * H + 16 * nb + n] : 0.f;
            acc2[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(gd, y, acc2[nb], 0, 0, 0);
        }
    }
    if (!active) return;
    // reduce the bias sums over the 4 row groups of the wave
    sb1 += __shfl_xor(sb1, 16);
    sb1 += __shfl_xor(sb1, 32);
    sb2 += __shfl_xor(sb2, 16);
    sb2 += __shfl_xor(sb2, 32);
#pragma unroll
    for (int i = 0; i < 4; i++)
        if (n < K1) out[(16 * m + 4 * g + i) * K1 + n] = acc1[i];
    if (g == 0) out[H * K1 + 16 * m + n] = sb1;
    float *o2 = out + H * K1 + H;
#pragma unroll
    for (int nb = 0; nb < MO; nb++)
#pragma unroll
        for (int i = 0; i < 4; i++) o2[(16 * m + 4 * g + i) * H + 16 * nb + n] = acc2[nb][i];
    if (g == 0) o2[M2 * H + 16 * m + n] = sb2;
}

// The same weight gradients with the rows staged in LDS: a tile of kDwRows
// rows of the layer-1 inputs Y, of da, of r and of dout is loaded with
// 16-byte loads by the whole block (the next tile's loads are in flight
// while the current tile is multiplied), then each wave runs its 16 output
// rows of dW1 and dW2 as MFMA 16x16x4 over the tile with operands read from
// LDS.  Rows are padded by 16 floats so the 4 rows read by one MFMA operand
// fall in different LDS banks.  Not used for the node encoder (K1 = 3).
constexpr int kDwRows = 16;

template <int H, int MODE>
__global__ __launch_bounds__(kBwdBlock) void k_dw_lds(BwdArgs A, float *__restrict__ part) {
    constexpr int MO = H / 16;
    constexpr int K1 = bseg<MODE>() * H;   // the factorised edge MLPs: the e segment only (or none)
    constexpr int NB1 = K1 / 16;
    constexpr bool CLS = MODE == B_CLS;
    constexpr int M2 = CLS ? 1 : H;
    constexpr int PL = H * K1 + H + M2 * H + M2;
    constexpr int SY = K1 + 16, SH = H + 16;            // padded LDS row strides (floats)
    constexpr int CY = K1 / 4, CH = H / 4;               // float4 chunks per row
    __shared__ __align__(16) float sY[kDwRows * SY];
    __shared__ __align__(16) float sG1[kDwRows * SH];
    __shared__ __align__(16) float sR[kDwRows * SH];
    __shared__ __align__(16) float sG2[kDwRows * (CLS ? 1 : SH)];
    if (*A.flags) return;
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
    const int64_t N = row_count(A);
    const int64_t per = (((N + kChunks - 1) / kChunks) + 3) & ~(int64_t)3;
    const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(r0 + per, N);
    float *out = part + (int64_t)blockIdx.x * PL;
    const bool active = w < MO;                        // waves beyond the output rows only load
    const int m = active ? w : 0;

    // tile loads: thread (rr, q) = (t / 16, t % 16) loads row rr's float4
    // chunks q, q + 16, ... of Y (CY chunks), da, r and dout (CH chunks each)
    static_assert(kBwdBlock == 16 * kDwRows, "one 16-thread group per tile row");
    constexpr int NY = (CY + 15) / 16, NHC = (CH + 15) / 16;
    const int rr = threadIdx.x >> 4, q = threadIdx.x & 15;
    f32x4 ny[NY ? NY : 1], ng1[NHC], nr[NHC], ng2[CLS ? 1 : NHC];
    float g2n = 0.f;
    auto fetch_tile = [&](int64_t t0) {
        const int64_t row = t0 + rr;
        const bool ok = row < r1;
        const int64_t rc = ok ? row : r0;
        const float *seg[3];
        if (MODE == B_EDGE) {
            seg[0] = A.a + rc * H;
            seg[1] = A.b + (int64_t)A.src_g[rc] * H;
            seg[2] = A.b + (int64_t)A.dst_g[rc] * H;
        } else if (MODE == B_EDGE_AB || MODE == B_ENC_AB) {
            seg[0] = seg[1] = seg[2] = A.a + rc * H;
        } else if (MODE == B_NODE) {
            seg[0] = A.a + rc * H;
            seg[1] = A.b + rc * 2 * H;
            seg[2] = A.b + rc * 2 * H + H;
        } else if (MODE == B_EDGE_ENC) {
            seg[0] = A.a + (int64_t)A.src_g[rc] * H;
            seg[1] = seg[2] = A.a + (int64_t)A.dst_g[rc] * H;
        } else {
            seg[0] = seg[1] = seg[2] = A.a + rc * H;
        }
#pragma unroll
        for (int y = 0; y < NY; y++) {
            const int j = q + 16 * y;
            ny[y] = zero4();
            if (ok && j < CY) {
                ny[y] = *(const f32x4 *)(seg[j / CH] + 4 * (j % CH));
            }
        }
#pragma unroll
        for (int y = 0; y < NHC; y++) {
            const int j = q + 16 * y;
            const bool v = ok && j < CH;
            ng1[y] = v ? *(const f32x4 *)(A.da + rc * H + 4 * j) : zero4();
            nr[y] = v ? *(const f32x4 *)(A.r + rc * H + 4 * j) : zero4();
            if (!CLS) ng2[y] = v ? *(const f32x4 *)(A.dout + rc * H + 4 * j) : zero4();
        }
        if (CLS) g2n = ok ? A.dout[rc] : 0.f;
    };
    f32x4 acc1[NB1 ? NB1 : 1], acc2[MO];
    zero<NB1 ? NB1 : 1>(acc1);
    zero<MO>(acc2);
    float sb1 = 0.f, sb2 = 0.f;
    if (r0 < r1) fetch_tile(r0);
    for (int64_t t0 = r0; t0 < r1; t0 += kDwRows) {
        __syncthreads();                               // the previous tile's reads are done
#pragma unroll
        for (int y = 0; y < NY; y++) {
            const int j = q + 16 * y;
            if (j < CY) *(f32x4 *)(sY + rr * SY + 4 * j) = ny[y];
        }
#pragma unroll
        for (int y = 0; y < NHC; y++) {
            const int j = q + 16 * y;
            if (j < CH) {
                *(f32x4 *)(sG1 + rr * SH + 4 * j) = ng1[y];
                *(f32x4 *)(sR + rr * SH + 4 * j) = nr[y];
                if (!CLS) *(f32x4 *)(sG2 + rr * SH + 4 * j) = ng2[y];
            }
        }
        if (CLS && q == 0) sG2[rr] = g2n;
        __syncthreads();
        if (t0 + kDwRows < r1) fetch_tile(t0 + kDwRows);
        if (!active) continue;
#pragma unroll 1
        for (int ks = 0; ks < kDwRows / 4; ks++) {
            const int kr = 4 * ks + g;
            const float ga = sG1[kr * SH + 16 * m + n];
            sb1 += ga;
#pragma unroll
            for (int nb = 0; nb < NB1; nb++)
                acc1[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga, sY[kr * SY + 16 * nb + n], acc1[nb], 0, 0, 0);
            float gd;
            if (CLS) gd = m == 0 && n == 0 ? sG2[kr] : 0.f;
            else gd = sG2[kr * SH + 16 * m + n];
            sb2 += gd;
            if (!CLS || m == 0) {
#pragma unroll
                for (int nb = 0; nb < MO; nb++)
                    acc2[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(gd, sR[kr * SH + 16 * nb + n], acc2[nb], 0, 0, 0);
            }
        }
    }
    if (!active) return;
    sb1 += __shfl_xor(sb1, 16);
    sb1 += __shfl_xor(sb1, 32);
    sb2 += __shfl_xor(sb2, 16);
    sb2 += __shfl_xor(sb2, 32);
#pragma unroll
    for (int nb = 0; nb < NB1; nb++)
#pragma unroll
        for (int i = 0; i < 4; i++) out[(16 * m + 4 * g + i) * K1 + 16 * nb + n] = acc1[nb][i];
    if (g == 0) out[H * K1 + 16 * m + n] = sb1;
    float *o2 = out + H * K1 + H;
    if (CLS) {
        if (m == 0) {
#pragma unroll
            for (int nb = 0; nb < MO; nb++)
                if (g == 0) o2[16 * nb + n] = acc2[nb][0];    // output row 0
            if (lane == 0) o2[H] = sb2;
        }
    } else {
#pragma unroll
        for (int nb = 0; nb < MO; nb++)
#pragma unroll
            for (int i = 0; i < 4; i++) o2[(16 * m + 4 * g + i) * H + 16 * nb + n] = acc2[nb][i];
        if (g == 0) o2[M2 * H + 16 * m + n] = sb2;
    }
}

// First reduction level: red[g][i] = sum of the partials of chunks
// g*G .. g*G+G-1 in chunk order (G = kChunks / kRedGroups), one group per
// blockIdx.y, so the kChunks-long sums run kRedGroups-wide in parallel.
__global__ void k_chunk_groups(const float *__restrict__ part, int PL, float *__restrict__ red,
                               const unsigned *__restrict__ flags) {
    if (*flags) return;
    constexpr int G = kChunks / kRedGroups;
    const int grp = blockIdx.y;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < PL; i += gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int c = grp * G; c < grp * G + G; c++) s += part[(int64_t)c * PL + i];
        red[(int64_t)grp * PL + i] = s;
    }
}

// Second level: the group sums in group order into the blob-shaped
// gradient.  The partial holds the first layer's [rows x K1] block, then
// the rest of the MLP's parameters; the first layer is stored with row
// stride ld >= K1 (the factorised edge MLPs fill its first K1 columns here,
// the rest per hit).
__global__ void k_dw_reduce(const float *__restrict__ red, int PL, int rows, int K1, int ld,
                            float *__restrict__ grad, const unsigned *__restrict__ flags) {
    if (*flags) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < PL; i += gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int g = 0; g < kRedGroups; g++) s += red[(int64_t)g * PL + i];
        const int first = rows * K1;
        grad[i < first ? (i / K1) * ld + i % K1 : rows * ld + (i - first)] = s;
    }
}

// Weight gradients of the hit segments of a factorised edge MLP, summed over
// hits instead of edges:  dW1[:, cs:cs+H] = sum_i S_i h_i^T,
// dW1[:, cd:cd+H] = sum_i D_i h_i^T  ([S_i, D_i] = sd[i]).  Chunks of hits
// as in k_dw_lds; partial [2 x H x H] per chunk.
template <int H>
__global__ __launch_bounds__(kBwdBlock) void k_dw_hits(int64_t n_hits, const float *__restrict__ h,
                                                       const float *__restrict__ sd, float *__restrict__ part,
                                                       const unsigned *__restrict__ flags) {
    constexpr int MO = H / 16, CH = H / 4, SH = H + 16;
    static_assert(kBwdBlock == 16 * kDwRows && CH <= 16 * 2, "tile loads");
    __shared__ __align__(16) float sY[kDwRows * SH];
    __shared__ __align__(16) float sS[kDwRows * SH];
    __shared__ __align__(16) float sD[kDwRows * SH];
    if (*flags) return;
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
    const int64_t per = (((n_hits + kChunks - 1) / kChunks) + 3) & ~(int64_t)3;
    const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(r0 + per, n_hits);
    float *out = part + (int64_t)blockIdx.x * 2 * H * H;
    const bool active = w < MO;
    const int m = active ? w : 0;
    constexpr int NHC = (CH + 15) / 16;
    const int rr = threadIdx.x >> 4, q = threadIdx.x & 15;
    f32x4 ny[NHC], ns[NHC], nd[NHC];
    auto fetch_tile = [&](int64_t t0) {
        const int64_t row = t0 + rr;
        const bool ok = row < r1;
        const int64_t rc = ok ? row : r0;
#pragma unroll
        for (int y = 0; y < NHC; y++) {
            const int j = q + 16 * y;
            const bool v = ok && j < CH;
            ny[y] = v ? *(const f32x4 *)(h + rc * H + 4 * j) : zero4();
            ns[y] = v ? *(const f32x4 *)(sd + rc * 2 * H + 4 * j) : zero4();
            nd[y] = v ? *(const f32x4 *)(sd + rc * 2 * H + H + 4 * j) : zero4();
        }
    };
    f32x4 as[MO], ad[MO];
    zero<MO>(as);
    zero<MO>(ad);
    if (r0 < r1) fetch_tile(r0);
    for (int64_t t0 = r0; t0 < r1; t0 += kDwRows) {
        __syncthreads();
#pragma unroll
        for (int y = 0; y < NHC; y++) {
            const int j = q + 16 * y;
            if (j < CH) {
                *(f32x4 *)(sY + rr * SH + 4 * j) = ny[y];
                *(f32x4 *)(sS + rr * SH + 4 * j) = ns[y];
                *(f32x4 *)(sD + rr * SH + 4 * j) = nd[y];
            }
        }
        __syncthreads();
        if (t0 + kDwRows < r1) fetch_tile(t0 + kDwRows);
        if (!active) continue;
#pragma unroll 1
        for (int ks = 0; ks < kDwRows / 4; ks++) {
            const int kr = 4 * ks + g;
            const float gs = sS[kr * SH + 16 * m + n], gd = sD[kr * SH + 16 * m + n];
#pragma unroll
            for (int nb = 0; nb < MO; nb++) {
                const float y = sY[kr * SH + 16 * nb + n];
                as[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(gs, y, as[nb], 0, 0, 0);
                ad[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(gd, y, ad[nb], 0, 0, 0);
            }
        }
    }
    if (!active) return;
#pragma unroll
    for (int nb = 0; nb < MO; nb++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
            out[(16 * m + 4 * g + i) * H + 16 * nb + n] = as[nb][i];
            out[H * H + (16 * m + 4 * g + i) * H + 16 * nb + n] = ad[nb][i];
        }
}

// group sums of k_dw_hits partials (in group order) into the two column
// blocks of W1; red == null: zero (no hits)
__global__ void k_dw_hits_reduce(const float *__restrict__ red, int H, int ld, int cs, int cd,
                                 float *__restrict__ grad, const unsigned *__restrict__ flags) {
    if (*flags) return;
    const int PL = 2 * H * H;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < PL; i += gridDim.x * blockDim.x) {
        float s = 0.f;
        if (red)
            for (int g = 0; g < kRedGroups; g++) s += red[(int64_t)g * PL + i];
        const int b = i / (H * H), r = (i % (H * H)) / H, col = i % H;
        grad[r * ld + (b ? cd : cs) + col] = s;
    }
}

// ------------------------------------------------------------------------
// duals of the gathers and of the message sums
// ------------------------------------------------------------------------
// sd[l] = [sum_{l -> j} x[edge], sum_{i -> l} x[edge]]; H/4 lanes per hit.
// Rows are added in edge order; up to BATCH of them are requested before the
// first is added (incoming ids are read one per lane and passed round the
// hit's lane group).
template <int H>
__global__ __launch_bounds__(256) void k_gather_pair(int64_t n_hits, const int *__restrict__ out_ptr,
                                                     const int *__restrict__ in_ptr,
                                                     const int *__restrict__ in_list, const float *__restrict__ x,
                                                     float *__restrict__ sd, const unsigned *__restrict__ flags) {
    if (*flags) return;
    constexpr int LPN = H / 4, NPW = 64 / LPN, BATCH = LPN < 8 ? LPN : 8;
    const int lane = threadIdx.x & 63, sub = lane / LPN, l = lane % LPN, c = 4 * l, gbase = sub * LPN;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t base = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * NPW; base < n_hits; base += nw * NPW) {
        const int64_t i0 = base + sub;
        const bool live = i0 < n_hits;
        const int64_t i = live ? i0 : n_hits - 1;
        f32x4 so = zero4(), si = zero4();
        const int a1 = out_ptr[i + 1];
        for (int a = out_ptr[i]; a < a1; a += BATCH) {
            const int cnt = min(BATCH, a1 - a);
            f32x4 v[BATCH];
#pragma unroll
            for (int j = 0; j < BATCH; j++)
                if (j < cnt) v[j] = *(const f32x4 *)(x + (int64_t)(a + j) * H + c);
#pragma unroll
            for (int j = 0; j < BATCH; j++)
                if (j < cnt) so += v[j];
        }
        const int b1 = in_ptr[i + 1];
        for (int b = in_ptr[i]; b < b1; b += BATCH) {   // the group's lanes share the trip count
            const int cnt = min(BATCH, b1 - b);
            const int mine = l < cnt ? in_list[b + l] : 0;
            f32x4 v[BATCH];
#pragma unroll
            for (int j = 0; j < BATCH; j++) {
                const int q = __shfl(mine, gbase + j);
                if (j < cnt) v[j] = *(const f32x4 *)(x + (int64_t)q * H + c);
            }
#pragma unroll
            for (int j = 0; j < BATCH; j++)
                if (j < cnt) si += v[j];
        }
        if (live) {
            *(f32x4 *)(sd + i * 2 * H + c) = so;
            *(f32x4 *)(sd + i * 2 * H + H + c) = si;
        }
    }
}

// The hit segments' input gradients of a factorised edge MLP:
//   dh[i] += W1[:, cs:cs+H]^T S_i + W1[:, cd:cd+H]^T D_i,   [S_i, D_i] = sd[i]
// on MFMA, 16 hits per wavefront unit; W1 is row-major [H x k1f].
template <int H>
__global__ __launch_bounds__(kBwdBlock) void k_hit_dual(int64_t n_hits, const float *__restrict__ sd,
                                                        const float *__restrict__ P_, int64_t o_w1, int k1f, int cs,
                                                        int cd, float *__restrict__ dh,
                                                        const unsigned *__restrict__ flags) {
    constexpr int MO = H / 16;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    f32x4 *sTs = (f32x4 *)lds_raw;                              // W1_s^T [H x H]
    f32x4 *sTd = sTs + frag_bytes<P>(H, H) / sizeof(f32x4);     // W1_d^T [H x H]
    stage<P, true>(sTs, P_ + o_w1 + cs, H, H, MO, 1.f, k1f);
    stage<P, true>(sTd, P_ + o_w1 + cd, H, H, MO, 1.f, k1f);
    __syncthreads();
    if (*flags) return;
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    const int64_t units = (n_hits + 15) >> 4;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t u = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; u < units; u += nw) {
        const int64_t i = u * 16 + n;
        const bool ok = i < n_hits;
        const int64_t ic = ok ? i : n_hits - 1;
        f32x4 Xs[MO], Xd[MO], acc[MO];
#pragma unroll
        for (int kb = 0; kb < MO; kb++) {
            Xs[kb] = P::load(sd + ic * 2 * H, kb, g);
            Xd[kb] = P::load(sd + ic * 2 * H + H, kb, g);
            acc[kb] = *(const f32x4 *)(dh + ic * H + 16 * kb + 4 * g);
        }
        gemm<P, MO, MO>(sTs, Xs, acc, lane);
        gemm<P, MO, MO>(sTd, Xd, acc, lane);
        if (ok) P::store_all<MO>(dh + i * H, g, acc);
    }
}

__global__ void k_zero(float *__restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

// ------------------------------------------------------------------------
// weighted binary cross-entropy:  L = (1/E) sum w_y [softplus(z) - y z],
// w_1 = pos_weight, w_0 = 1;  dL/dz = w_y (sigmoid(z) - y) / E
// ------------------------------------------------------------------------
constexpr int kLossBlocks = 256;

__global__ __launch_bounds__(256) void k_bce(const float *__restrict__ z, const uint8_t *__restrict__ y, float pw,
                                             int64_t n, float *__restrict__ dz, float *__restrict__ part) {
    __shared__ float sh[256];
    float acc = 0.f;
    const float inv = n > 0 ? 1.f / (float)n : 0.f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float v = z[i];
        const bool pos = y[i] != 0;
        const float w = pos ? pw : 1.f;
        const float sp = v > 0.f ? v + log1pf(expf(-v)) : log1pf(expf(v));
        // sigmoid(t) without cancellation; sigmoid(z) - 1 = -sigmoid(-z)
        const float t = pos ? -v : v;
        const float sg = t >= 0.f ? 1.f / (1.f + expf(-t)) : expf(t) / (1.f + expf(t));
        acc += w * (sp - (pos ? v : 0.f));
        dz[i] = w * (pos ? -sg : sg) * inv;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if (threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Sigmoid focal loss (Sec. 5.2; the form of Lin et al.): with s = 2y - 1,
// p_t = sigmoid(s z), ce = softplus(z) - y z = -log p_t, a_t = alpha (y = 1)
// or 1 - alpha (alpha < 0: 1), the edge's term is a_t (1 - p_t)^gamma ce and
// dL/dz = a_t (1 - p_t)^gamma [(sigmoid(z) - y) - gamma s p_t ce] / n.
// Block partial sums of the terms go to part (summed by k_bce_total).
__global__ __launch_bounds__(256) void k_focal(const float *__restrict__ z, const uint8_t *__restrict__ y,
                                               float alpha, float gamma, int64_t n, float *__restrict__ dz,
                                               float *__restrict__ part) {
    __shared__ float sh[256];
    float acc = 0.f;
    const float inv = n > 0 ? 1.f / (float)n : 0.f;
    auto sigmoid = [](float t) { return t >= 0.f ? 1.f / (1.f + expf(-t)) : expf(t) / (1.f + expf(t)); };
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float v = z[i];
        const bool pos = y[i] != 0;
        const float s = pos ? 1.f : -1.f;
        const float at = alpha < 0.f ? 1.f : (pos ? alpha : 1.f - alpha);
        const float ce = (v > 0.f ? v + log1pf(expf(-v)) : log1pf(expf(v))) - (pos ? v : 0.f);
        const float pt = sigmoid(s * v), qt = sigmoid(-s * v);
        const float mod = gamma == 0.f ? 1.f : powf(qt, gamma);
        acc += at * mod * ce;
        dz[i] = at * mod * ((sigmoid(v) - (pos ? 1.f : 0.f)) - gamma * s * pt * ce) * inv;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if (threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_bce_total(const float *__restrict__ part, int64_t n, float *__restrict__ loss) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        float s = 0.f;
        for (int b = 0; b < kLossBlocks; b++) s += part[b];
        *loss = n > 0 ? s / (float)n : 0.f;
    }
}

inline int blocks_for(int64_t n, int block, int cap) {
    int64_t b = (n + block - 1) / block;
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

template <int H, int MODE>
void run_bwd(velo_ctx *c, const BwdArgs &a, hipStream_t s) {
    constexpr int NSEG = bseg<MODE>(), K1 = NSEG * H;
    constexpr bool CLS = MODE == B_CLS;
    constexpr size_t lds = frag_bytes<P>(H, K1) + (CLS ? 0 : frag_bytes<P>(H, H)) + frag_bytes<P>(K1, H);
    static const int per_cu = [] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_bwd<H, MODE>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   // a failure is the launch's error
        int n = 0;
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(&k_bwd<H, MODE>), kBwdBlock, lds);
        return n < 1 ? 1 : n;
    }();
    k_bwd<H, MODE><<<persistent_grid(c, per_cu), kBwdBlock, lds, s>>>(a);
}

template <int H, int MODE>
void run_dw(velo_ctx *c, const BwdArgs &a, float *grad_dst, hipStream_t s) {
    constexpr int K1 = MODE == B_NODE_ENC ? 3 : bseg<MODE>() * H;
    constexpr int LD = MODE == B_NODE_ENC ? 3 : bkseg<MODE>() * H;
    constexpr int M2 = MODE == B_CLS ? 1 : H;
    constexpr int PL = H * K1 + H + M2 * H + M2;
    if constexpr (MODE == B_NODE_ENC)
        k_dw<H, MODE><<<kChunks, kBwdBlock, 0, s>>>(a, c->ws.g_part);
    else
        k_dw_lds<H, MODE><<<kChunks, kBwdBlock, 0, s>>>(a, c->ws.g_part);
    k_chunk_groups<<<dim3(blocks_for(PL, 256, 1024), kRedGroups), 256, 0, s>>>(c->ws.g_part, PL, c->ws.g_red,
                                                                              c->ws.flags);
    k_dw_reduce<<<blocks_for(PL, 256, 1024), 256, 0, s>>>(c->ws.g_red, PL, H, K1, LD, grad_dst, c->ws.flags);
}

template <int H>
void backward_h(velo_ctx *c, const velo_hits *hits, const float *Pw, const float *dlogit, float *dparams,
                hipStream_t s) {
    Workspace &w = c->ws;
    const ParamLayout &L = c->layout;
    const int64_t N = hits->n_hits, Ecap = c->cfg.max_edges, Nmax = c->cfg.max_hits;
    const int n = c->cfg.gnn_iters;
    const float *ck_h = (const float *)w.ck_h, *ck_e = (const float *)w.ck_e;
    auto hk = [&](int k) { return ck_h + (int64_t)k * Nmax * H; };
    auto ek = [&](int k) { return ck_e + (int64_t)k * Ecap * H; };
    // parameters without gradient (normalisation, embedding) are zero
    k_zero<<<blocks_for(L.nenc[0].w, 256, 1024), 256, 0, s>>>(dparams, L.nenc[0].w);

    BwdArgs base{};
    base.src_g = w.src_g; base.dst_g = w.dst_g; base.P = Pw; base.flags = w.flags;
    base.da = w.g_da; base.r = w.g_r;
    // classifier: dL/de^n
    BwdArgs cl = base;
    cl.n_dev = w.n_edges; cl.n_host = Ecap; cl.a = ek(n); cl.dout = dlogit; cl.dres = w.g_e[0];
    cl.o_w1 = L.cls[0].w; cl.o_w2 = L.cls[1].w;
    { StageTimer t(c, VELO_STAGE_BWD_MLP, s); run_bwd<H, B_CLS>(c, cl, s); }
    { StageTimer t(c, VELO_STAGE_BWD_DW, s); run_dw<H, B_CLS>(c, cl, dparams + L.cls[0].w, s); }
    int ce = 0, ch = 0;
    if (N > 0) k_zero<<<blocks_for(N * H, 256, 4096), 256, 0, s>>>(w.g_h[0], N * H);
    // the hit segments of a factorised edge MLP: per-hit sums of da over out-
    // and in-edges, then dL/dh += W1_s^T S + W1_d^T D and the two column
    // blocks of dL/dW1 as sums over hits of S h^T and D h^T
    auto hit_duals = [&](int64_t o_w1, int k1f, int cs, int cd, float *dh, const float *h, float *grad) {
        if (N <= 0) {   // no hits, no edges: the hit blocks of dW1 are zero
            k_dw_hits_reduce<<<blocks_for(2 * H * H, 256, 64), 256, 0, s>>>(nullptr, H, k1f, cs, cd,
                                                                             grad + o_w1, w.flags);
            return;
        }
        {
            StageTimer t(c, VELO_STAGE_BWD_GRAPH, s);
            k_gather_pair<H><<<persistent_grid(c, 16), 256, 0, s>>>(N, w.row_ptr, w.in_ptr, w.in_list, w.g_da,
                                                                  w.g_sd, w.flags);
        }
        {
            StageTimer t(c, VELO_STAGE_BWD_MLP, s);
            constexpr size_t lds = 2 * frag_bytes<P>(H, H);
            static const int per_cu = [] {
                (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_hit_dual<H>),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                int m = 0;
                (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&m, reinterpret_cast<const void *>(&k_hit_dual<H>),
                                                             kBwdBlock, lds);
                return m < 1 ? 1 : m;
            }();
            k_hit_dual<H><<<persistent_grid(c, per_cu), kBwdBlock, lds, s>>>(N, w.g_sd, Pw, o_w1, k1f, cs, cd, dh,
                                                                            w.flags);
        }
        StageTimer t(c, VELO_STAGE_BWD_DW, s);
        k_dw_hits<H><<<kChunks, kBwdBlock, 0, s>>>(N, h, w.g_sd, w.g_part, w.flags);
        k_chunk_groups<<<dim3(blocks_for(2 * H * H, 256, 1024), kRedGroups), 256, 0, s>>>(w.g_part, 2 * H * H,
                                                                                         w.g_red, w.flags);
        k_dw_hits_reduce<<<blocks_for(2 * H * H, 256, 1024), 256, 0, s>>>(w.g_red, H, k1f, cs, cd, grad + o_w1,
                                                                          w.flags);
    };
    auto abk = [&](int slot) -> const float * { return w.ck_ab + (int64_t)slot * Nmax * 2 * H; };
    for (int k = n - 1; k >= 0; k--) {
        // edge network k
        BwdArgs ed = base;
        ed.n_dev = w.n_edges; ed.n_host = Ecap; ed.a = ek(k); ed.b = hk(k + 1);
        ed.dout = w.g_e[ce]; ed.dres = w.g_e[ce ^ 1]; ed.ab = abk(k);
        ed.dm = k < n - 1 ? w.g_m : nullptr; ed.dout_w = w.g_e[ce];   // dL/dm^{k+1} from node network k+1
        ed.o_w1 = L.edge[k][0].w; ed.o_w2 = L.edge[k][1].w;
        { StageTimer t(c, VELO_STAGE_BWD_MLP, s); run_bwd<H, B_EDGE_AB>(c, ed, s); }
        { StageTimer t(c, VELO_STAGE_BWD_DW, s); run_dw<H, B_EDGE_AB>(c, ed, dparams + L.edge[k][0].w, s); }
        hit_duals(L.edge[k][0].w, 3 * H, H, 2 * H, w.g_h[ch], hk(k + 1), dparams);
        ce ^= 1;
        // node network k
        BwdArgs nd = base;
        nd.n_dev = nullptr; nd.n_host = N; nd.a = hk(k); nd.b = w.ck_m + (int64_t)k * Nmax * 2 * H;
        nd.dout = w.g_h[ch]; nd.dres = w.g_h[ch ^ 1]; nd.dx1 = w.g_m;
        nd.o_w1 = L.node[k][0].w; nd.o_w2 = L.node[k][1].w;
        if (N > 0) {
            StageTimer t(c, VELO_STAGE_BWD_MLP, s);
            run_bwd<H, B_NODE>(c, nd, s);
        }
        { StageTimer t(c, VELO_STAGE_BWD_DW, s); run_dw<H, B_NODE>(c, nd, dparams + L.node[k][0].w, s); }
        ch ^= 1;
        // the message sums of step k: their dual is added by the next edge
        // MLP's backward kernel (edge network k-1, or the edge encoder)
    }
    // edge encoder
    BwdArgs ee = base;
    ee.n_dev = w.n_edges; ee.n_host = Ecap; ee.a = hk(0); ee.dout = w.g_e[ce]; ee.ab = abk(n);
    ee.dm = n > 0 ? w.g_m : nullptr; ee.dout_w = w.g_e[ce];   // dL/dm^0 from node network 0
    ee.o_w1 = L.eenc[0].w; ee.o_w2 = L.eenc[1].w;
    { StageTimer t(c, VELO_STAGE_BWD_MLP, s); run_bwd<H, B_ENC_AB>(c, ee, s); }
    { StageTimer t(c, VELO_STAGE_BWD_DW, s); run_dw<H, B_ENC_AB>(c, ee, dparams + L.eenc[0].w, s); }
    hit_duals(L.eenc[0].w, 2 * H, 0, H, w.g_h[ch], hk(0), dparams);
    // node encoder
    BwdArgs ne = base;
    ne.n_dev = nullptr; ne.n_host = N; ne.dout = w.g_h[ch]; ne.x = hits->x; ne.y = hits->y; ne.z = hits->z;
    ne.o_w1 = L.nenc[0].w; ne.o_w2 = L.nenc[1].w;
    if (N > 0) {
        StageTimer t(c, VELO_STAGE_BWD_MLP, s);
        constexpr size_t lds = frag_bytes<P>(H, H) + sizeof(float) * H * 4;
        k_bwd_node_enc<H><<<persistent_grid(c, 2), kBwdBlock, lds, s>>>(ne);
    }
    { StageTimer t(c, VELO_STAGE_BWD_DW, s); run_dw<H, B_NODE_ENC>(c, ne, dparams + L.nenc[0].w, s); }
}

// Adam with bias correction (one float32 parameter per thread).
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

}  // namespace

void launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
                 int step, hipStream_t s) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    k_adam<<<blocks_for(n, 256, 4096), 256, 0, s>>>(p, g, m, v, n, lr, b1, b2, eps, c1, c2);
}

bool train_supported(int hidden, int precision) { return precision == VELO_FP32 && (hidden == 32 || hidden == 64); }

size_t train_part_floats(int H) {
    // the largest blob-shaped partial: an edge or node network, [H x 3H | H | H x H | H]
    return (size_t)kChunks * (3 * H * H + H + H * H + H);
}

size_t train_red_floats(int H) { return (size_t)kRedGroups * (3 * H * H + H + H * H + H); }

void launch_bce(velo_ctx *c, const float *logit, const uint8_t *y, float pos_weight, int64_t n, float *loss,
                float *dlogit, hipStream_t s) {
    k_bce<<<kLossBlocks, 256, 0, s>>>(logit, y, pos_weight, n, dlogit, c->ws.g_loss);
    k_bce_total<<<1, 64, 0, s>>>(c->ws.g_loss, n, loss);
}

void launch_focal(velo_ctx *c, const float *logit, const uint8_t *y, float alpha, float gamma, int64_t n,
                  float *loss, float *dlogit, hipStream_t s) {
    k_focal<<<kLossBlocks, 256, 0, s>>>(logit, y, alpha, gamma, n, dlogit, c->ws.g_loss);
    k_bce_total<<<1, 64, 0, s>>>(c->ws.g_loss, n, loss);
}

void launch_gnn_backward(velo_ctx *c, const velo_hits *h, const float *params, const float *dlogit, float *dparams,
                         hipStream_t s) {
    if (c->cfg.gnn_hidden == 32) backward_h<32>(c, h, params, dlogit, dparams, s);
    if (c->cfg.gnn_hidden == 64) backward_h<64>(c, h, params, dlogit, dparams, s);
}

}  // namespace velo
