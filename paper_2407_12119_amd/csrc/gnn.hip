// gnn.hip -- embedding MLP and interaction-network GNN on MFMA (gfx950).
//
// Every MLP of the path (paper Sec. 5.1 embedding; Sec. 5.2 node/edge
// encoders, node/edge networks, edge classifier) is a dense contraction and
// runs on matrix cores in the "transposed" form
//     OUT^T (channels x items) = W (channels x K) * X^T (K x items)
// with 16 items (hits or edges) per wavefront unit.  Lane l = 16 g + n owns
// item n.  The 16x16 accumulator of an output block mo holds, in lane (n, g),
// channels 16 mo + 4 g + (0..3) of item n.  The K dimension is walked in
// blocks; within a block lane group g owns the inputs
//     fp32 (v_mfma_f32_16x16x4f32, 16-wide block):  16 kb + 4 g + (0..3)
//     bf16 (v_mfma_f32_16x16x32_bf16, 32-wide):     32 kb + 4 g + (0..3) and
//                                                   32 kb + 16 + 4 g + (0..3)
// so that, in both precisions,
//   * a lane loads its item's inputs with short vector loads (B operand),
//   * the accumulators of one layer are exactly the B operand of the next
//     layer (two-layer MLPs chain in registers), and the residual input of a
//     channel is already held by the lane that adds it,
//   * weights are staged once per block in LDS in fragment order, so the A
//     operand of every MFMA is one conflict-free 16-byte LDS read per lane.
// Matrix operands are fp32 or bf16; accumulation, biases, ReLU, residual
// adds and the classifier's last (H -> 1) layer are fp32.
//
// Messages (the scatter_add of the message equation, Sec. 5.2) are fp32 sums
// in a fixed order over per-hit incidence lists, in every precision.
#include "mfma.h"

namespace velo {

namespace {

using namespace mfma;

// ------------------------------------------------------------------------
// embedding MLP 3 -> 128 -> 128 -> 4 on normalised (r, phi, z)  (Sec. 5.1)
// ------------------------------------------------------------------------
constexpr int kCe = VELO_EMB_HIDDEN;

// sc: the embedding's scales {s_x2, s_w2, s_x3, s_w3} (fp8, else null);
// amax: its two layer inputs' calibration maxima (else null).  Training
// keeps, per hit, the normalised inputs (sv: u0 u1 u2 0) and both hidden
// activations after their ReLU (sa1, sa2: [n x 128] rows); null: not kept.
template <class P>
__global__ __launch_bounds__(512) void k_embed(int64_t n_hits, const float *__restrict__ x,
                                               const float *__restrict__ y, const float *__restrict__ z,
                                               const float *__restrict__ P_, int64_t o_w1, int64_t o_w2,
                                               int64_t o_w3, float *__restrict__ emb, const float *__restrict__ sc,
                                               float *__restrict__ amax, float *__restrict__ sv,
                                               float *__restrict__ sa1, float *__restrict__ sa2,
                                               const unsigned *__restrict__ flags) {
    using W = typename P::wfrag_t;
    constexpr int MO = kCe / 16, KB = kCe / P::KBLK;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    W *sW2 = (W *)lds_raw;
    W *sW3 = (W *)(lds_raw + frag_bytes<P>(kCe, kCe));
    float *sW1 = (float *)(lds_raw + frag_bytes<P>(kCe, kCe) + frag_bytes<P>(16, kCe));
    const MlpScales S = read_scales(sc);
    stage<P>(sW2, P_ + o_w2, kCe, kCe, MO, S.iw1);
    stage<P>(sW3, P_ + o_w3, VELO_EMB_DIM, kCe, 1, S.iw2);
    for (int t = threadIdx.x; t < kCe * 4; t += blockDim.x) sW1[t] = P_[o_w1 + t];   // W1 then b1
    __syncthreads();
    if (*flags & kErrInput) return;

    const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
    const float *b3 = P_ + o_w3 + VELO_EMB_DIM * kCe;
    const float mu0 = P_[0], mu1 = P_[1], mu2 = P_[2], sg0 = P_[3], sg1 = P_[4], sg2 = P_[5];
    f32x4 rb2[MO];
    load_bias<MO>(P_ + o_w2 + kCe * kCe, rb2, g);
    const int64_t units = (n_hits + 15) >> 4;
    for (int64_t u = wave_id(); u < units; u += n_waves()) {
        const int64_t i = u * 16 + n;
        const int64_t ic = i < n_hits ? i : n_hits - 1;
        const float X = x[ic], Y = y[ic], Z = z[ic];
        const float u0 = (sqrtf(X * X + Y * Y) - mu0) / sg0;
        const float u1 = (atan2f(Y, X) - mu1) / sg1;
        const float u2 = (Z - mu2) / sg2;
        f32x4 h1[MO];
        first_layer3<MO>(sW1, kCe, u0, u1, u2, g, h1);
        if (amax) record_amax(absmax4<MO>(h1), amax);
        if (sa1 && i < n_hits) {
            F32::store_all<MO>(sa1 + i * kCe, g, h1);
            if (g == 0) *(f32x4 *)(sv + i * 4) = f32x4{u0, u1, u2, 0.f};
        }
        typename P::frag_t x1[KB];
        P::template chain<MO>(h1, x1, S.ix1);
        f32x4 h2[MO];
        zero<MO>(h2);
        gemm<P, MO, KB>(sW2, x1, h2, lane);
        if (P::kScaled) rescale<MO>(h2, S.d1);
        bias_relu<MO>(h2, rb2);
        if (amax) record_amax(absmax4<MO>(h2), amax + 1);
        if (sa2 && i < n_hits) F32::store_all<MO>(sa2 + i * kCe, g, h2);
        typename P::frag_t x2[KB];
        P::template chain<MO>(h2, x2, S.ix2);
        f32x4 o[1];
        zero<1>(o);
        gemm<P, 1, KB>(sW3, x2, o, lane);
        if (P::kScaled) rescale<1>(o, S.d2);
        if (g == 0 && i < n_hits) {
            f32x4 r;
#pragma unroll
            for (int q = 0; q < 4; q++) r[q] = o[0][q] + b3[q];
            *(f32x4 *)(emb + i * 4) = r;
        }
    }
}

// ------------------------------------------------------------------------
// node encoder 3 -> H -> H on normalised (x, y, z)  (Sec. 5.2); the first
// layer runs on the vector ALU, the second on MFMA (scales sc[2], sc[3]).
// ------------------------------------------------------------------------
template <class P, int H>
__global__ __launch_bounds__(512) void k_node_enc(int64_t n_hits, const float *__restrict__ x,
                                                  const float *__restrict__ y, const float *__restrict__ z,
                                                  const float *__restrict__ P_, int64_t o_w1, int64_t o_w2,
                                                  typename P::state_t *__restrict__ h, const float *__restrict__ sc,
                                                  float *__restrict__ amax, const unsigned *__restrict__ flags) {
    using W = typename P::wfrag_t;
    constexpr int MO = H / 16, KB = H / P::KBLK;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    W *sW2 = (W *)lds_raw;
    float *sW1 = (float *)(lds_raw + frag_bytes<P>(H, H));
    const MlpScales S = read_scales(sc);
    stage<P>(sW2, P_ + o_w2, H, H, MO, S.iw2);
    for (int t = threadIdx.x; t < H * 4; t += blockDim.x) sW1[t] = P_[o_w1 + t];
    __syncthreads();
    if (*flags) return;
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    const float mu0 = P_[6], mu1 = P_[7], mu2 = P_[8], sg0 = P_[9], sg1 = P_[10], sg2 = P_[11];
    f32x4 rb2[MO];
    load_bias<MO>(P_ + o_w2 + H * H, rb2, g);
    const int64_t units = (n_hits + 15) >> 4;
    for (int64_t u = wave_id(); u < units; u += n_waves()) {
        const int64_t i = u * 16 + n;
        const int64_t ic = i < n_hits ? i : n_hits - 1;
        const float u0 = (x[ic] - mu0) / sg0, u1 = (y[ic] - mu1) / sg1, u2 = (z[ic] - mu2) / sg2;
        f32x4 h1[MO];
        first_layer3<MO>(sW1, H, u0, u1, u2, g, h1);
        if (amax) record_amax(absmax4<MO>(h1), amax + 1);
        typename P::frag_t x1[KB];
        P::template chain<MO>(h1, x1, S.ix2);
        f32x4 o[MO];
        zero<MO>(o);
        gemm<P, MO, KB>(sW2, x1, o, lane);
        if (P::kScaled) rescale<MO>(o, S.d2);
        if (i < n_hits) {
#pragma unroll
            for (int mo = 0; mo < MO; mo++) o[mo] += rb2[mo];
            P::template store_all<MO>(h + i * H, g, o);
        }
    }
}

// ------------------------------------------------------------------------
// per-hit first-layer products of an edge MLP (the AB modes below):
//   AB[i] = [W1[:, cs:cs+H] h_i, W1[:, cd:cd+H] h_i]
// with the MLP's operand precision and float32 accumulation; for fp8 the raw
// accumulators (the edge kernel descales them with its own products).  W1 is
// the row-major [H x k1f] first-layer weight of that MLP.
// ------------------------------------------------------------------------
template <class P, int H>
__global__ __launch_bounds__(512) void k_hit_proj(int64_t n_hits, const typename P::state_t *__restrict__ h,
                                                  const float *__restrict__ P_, int64_t o_w1, int k1f, int cs, int cd,
                                                  const float *__restrict__ sc, float *__restrict__ ab,
                                                  const unsigned *__restrict__ flags) {
    using W = typename P::wfrag_t;
    constexpr int MO = H / 16, KB = H / P::KBLK;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    W *sWs = (W *)lds_raw;
    W *sWd = (W *)(lds_raw + frag_bytes<P>(H, H));
    const MlpScales S = read_scales(sc);
    stage<P>(sWs, P_ + o_w1 + cs, H, H, MO, S.iw1, k1f);
    stage<P>(sWd, P_ + o_w1 + cd, H, H, MO, S.iw1, k1f);
    __syncthreads();
    if (*flags) return;
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    const int64_t units = (n_hits + 15) >> 4;
    for (int64_t u = wave_id(); u < units; u += n_waves()) {
        const int64_t i = u * 16 + n;
        const int64_t ic = i < n_hits ? i : n_hits - 1;
        typename P::frag_t X[KB];
#pragma unroll
        for (int kb = 0; kb < KB; kb++) X[kb] = P::load(h + ic * H, kb, g, S.ix1);
        f32x4 a[MO], b[MO];
        zero<MO>(a);
        zero<MO>(b);
        gemm<P, MO, KB>(sWs, X, a, lane);
        gemm<P, MO, KB>(sWd, X, b, lane);
        if (i < n_hits) {
#pragma unroll
            for (int mo = 0; mo < MO; mo++) {
                *(f32x4 *)(ab + i * 2 * H + 16 * mo + 4 * g) = a[mo];
                *(f32x4 *)(ab + i * 2 * H + H + 16 * mo + 4 * g) = b[mo];
            }
        }
    }
}

// ------------------------------------------------------------------------
// generic two-layer MLP over gathered segments
//   NODE:     X = [h_in[i], m[i, 0:H], m[i, H:2H]],  h_out[i] = h_in[i] + MLP(X)
//   EDGE:     X = [e[q], h[src q], h[dst q]],        e[q] = e[q] + MLP(X) (in place)
//   EDGE_ENC: X = [h[src q], h[dst q]],              e[q] = MLP(X)
//   CLS_ONLY: X = e[q]                               (classifier only)
// With CLS the edge classifier H -> H -> 1 runs on the result (Sec. 5.2) and
// writes the logit; the final edge state is then not stored.
// The first layer is linear in its concatenated input, so its products with
// the two hit segments can be formed once per hit (k_hit_proj: AB[i] =
// [W1_src h_i, W1_dst h_i], float32) instead of once per edge:
//   EDGE_AB:  X = [e[q]],   hidden = relu(b1 + W1_e e + AB[src][0:H] + AB[dst][H:2H])
//   ENC_AB:   no product,   hidden = relu(b1 + AB[src][0:H] + AB[dst][H:2H])
// the same sums as EDGE / EDGE_ENC in another order.
// ------------------------------------------------------------------------
enum Mode { NODE = 0, EDGE = 1, EDGE_ENC = 2, CLS_ONLY = 3, EDGE_AB = 4, ENC_AB = 5 };

struct MlpArgs {
    const int *n_dev;      // device item count (edges) or null
    int64_t n_host;        // host item count (hits) or the cap for edges
    const int *src_g, *dst_g;
    const void *a;         // NODE: h_in; EDGE: e (in/out); EDGE_ENC: h0; CLS_ONLY: e
    const void *b;         // NODE: m (float32); EDGE: h (updated)
    void *out;             // NODE: h_out; EDGE/EDGE_ENC: e
    const float *P;
    int64_t o_w1, o_w2;    // this MLP's layers
    int64_t o_c1, o_c2;    // classifier layers (CLS)
    float *logit;
    const float *sc, *sc_cls;      // fp8 scales of this MLP and of the classifier (else null)
    float *amax, *amax_cls;        // calibration maxima (else null)
    int xcd;                       // XCD-blocked work mapping
    // edge MLPs on 2-byte states: source rows (batch-global CSR over hits)
    // and where the outgoing message sums of the new edge states go (m rows
    // of 2H floats, first half; null: not wanted)
    const int *rows;
    int64_t n_rows;
    float *mout;
    const float *ab;               // EDGE_AB / ENC_AB: per-hit first-layer products [N x 2H]
    const unsigned *flags;
    // 16-wavefront source-hit walks: per-XCD work counters, zeroed before the
    // launch (null: the static mapping)
    int *grab;
};

// source hits a wavefront takes at a time from its XCD's work counter
constexpr int kGrab = 4;

constexpr int kMlpBlock = 512;

// input segments of the first layer's weight (in the parameter blob)
template <int MODE>
constexpr int kseg() { return (MODE == EDGE_ENC || MODE == ENC_AB) ? 2 : (MODE == CLS_ONLY ? 0 : 3); }
// segments multiplied per item (the AB modes take the hit segments from AB)
template <int MODE>
constexpr int nseg() { return MODE == EDGE_AB ? 1 : (MODE == ENC_AB ? 0 : kseg<MODE>()); }
template <int MODE>
constexpr bool has_ab() { return MODE == EDGE_AB || MODE == ENC_AB; }
// modes that update an edge state in place (residual from e)
template <int MODE>
constexpr bool edge_update() { return MODE == EDGE || MODE == EDGE_AB; }

// Edge MLPs that feed a message step (the edge encoder and every edge
// network but the one fused with the classifier) walk the edges source hit
// by source hit, 16 at a time, and also produce the outgoing message sums of
// the states they write: with 2-byte states, and with float32 states in the
// factorised (AB) form.  The concatenated float32 MLPs (training) are
// MFMA-bound: there the padding of each source's last chunk would cost more
// than the message kernel saves, so they keep 16-edge tiles.
template <class P, int MODE, bool CLS>
constexpr bool src_aligned() {
    return (sizeof(typename P::state_t) == 2 || has_ab<MODE>()) &&
           (MODE == EDGE || MODE == EDGE_ENC || MODE == EDGE_AB || MODE == ENC_AB) && !CLS;
}

// LDS: [W1 fragments (nseg H wide)] [W2] [classifier W1] [biases] [classifier biases] [carries]
template <class P, int H, int MODE>
constexpr size_t mlp_w_bytes() {
    return MODE == CLS_ONLY ? 0 : (nseg<MODE>() ? frag_bytes<P>(H, nseg<MODE>() * H) : 0) + frag_bytes<P>(H, H);
}

// WIDE: workgroups of 16 wavefronts (H = 128 source-walking edge MLPs):
// twice the wavefronts share one LDS copy of the weights, each holding one
// chunk at a time and half a K block of weight fragments, so that a lane
// needs at most 128 VGPRs and a SIMD runs four wavefronts instead of two.
template <class P, int H, int MODE, bool CLS>
constexpr bool wide_ok() {
    return H == 128 && sizeof(typename P::state_t) == 2 && src_aligned<P, MODE, CLS>();
}

template <class P, int H, int MODE, bool CLS, bool WIDE = false>
constexpr size_t mlp_lds() {
    return mlp_w_bytes<P, H, MODE>() + (MODE == CLS_ONLY ? 0 : sizeof(float) * 2 * H) +
           (CLS ? frag_bytes<P>(H, H) + sizeof(float) * 2 * H : 0) +
           (src_aligned<P, MODE, CLS>() ? sizeof(float) * H * ((WIDE ? 2 : 1) * kMlpBlock / 64) : 0);
}

// Row sums of V values per lane over the 16 lanes of each DPP row.  The
// partners n^8 (row rotate by 8), n^7 (half-row mirror), n^2 and n^1 (quad
// permutations) generate the whole row; at each step a lane keeps half of
// its values (the even or odd ones of each pair, by the bit of its row
// position n in which it differs from the partner: 8, 4, 2, 1) and adds the
// partner's copy of them, so the work halves at every step.  Afterwards v[t] (t < V / 16, or t = 0
// for V = 8) is the row total of value 16 t + r(n), r(n) = 8 b0 + 4 b1 + 2 b2
// + b3 with b_k bit k of n (for V = 8: value r(n) & 7, the last step a plain
// sum, so lanes n and n ^ 1 agree).  Fixed order, so deterministic.
template <int CTRL>
__device__ inline float dpp_move(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL, int BIT, int C>
__device__ inline void row_sums_step(float *v, int n) {
    if constexpr (C == 1) {
        v[0] += dpp_move<CTRL>(v[0]);
    } else {
        const bool hi = (n & BIT) != 0;
#pragma unroll
        for (int j = 0; j < C / 2; j++) {
            const float keep = hi ? v[2 * j + 1] : v[2 * j];
            const float send = hi ? v[2 * j] : v[2 * j + 1];
            v[j] = keep + dpp_move<CTRL>(send);
        }
    }
}
template <int V>
__device__ inline void row_sums(float *v, int n) {
    static_assert(V == 8 || V == 16 || V == 32, "4 MO values per lane");
    row_sums_step<0x128, 8, V>(v, n);
    row_sums_step<0x141, 4, V / 2>(v, n);
    row_sums_step<0x4E, 2, V / 4>(v, n);
    row_sums_step<0xB1, 1, (V / 8 > 1 ? V / 8 : 1)>(v, n);
}

// The first layer of an MLP: every input segment but the node network's two
// message sums is a stored encoding (bf16 already in 2-byte precisions, so a
// split operand's lo part is 0 there).
template <class P, int MO, int KB, int NSEG, int MODE, int AG = MO>
__device__ inline void gemm_first(const typename P::wfrag_t *sW1, const typename P::frag_t *X, f32x4 *acc,
                                  int lane) {
    if constexpr (MODE == NODE) {
        gemm<P, MO, NSEG * KB, 0, KB, true, AG>(sW1, X, acc, lane);
        gemm<P, MO, NSEG * KB, KB, NSEG * KB, false, AG>(sW1, X, acc, lane);
    } else {
        gemm<P, MO, NSEG * KB, 0, NSEG * KB, true, AG>(sW1, X, acc, lane);
    }
}

template <class P, int H>
// sCB: the classifier's hidden bias divided by its fp8 descale factor, then
// its output weights (2H floats in LDS); b_out: its output bias
__device__ inline void classify(const typename P::wfrag_t *sC1, const float *sCB, float b_out, const f32x4 *ev,
                                const MlpScales &S, float *amax, int lane, bool ok, int64_t q,
                                float *__restrict__ logit) {
    constexpr int MO = H / 16, KB = H / P::KBLK;
    const int g = lane >> 4;
    if (amax) record_amax(absmax4<MO>(ev), amax);
    typename P::frag_t xe[KB];
    P::template chain<MO>(ev, xe, S.ix1);
    f32x4 hc[MO];
    load_bias<MO>(sCB, hc, g);
    gemm<P, MO, KB>(sC1, xe, hc, lane);
    if (P::kScaled) rescale<MO>(hc, S.d1);
    f32x4 w2[MO];
    load_bias<MO>(sCB + H, w2, g);
    float part = 0.f;
#pragma unroll
    for (int mo = 0; mo < MO; mo++)
#pragma unroll
        for (int i = 0; i < 4; i++) part += w2[mo][i] * relu1(hc[mo][i]);
    part += __shfl_xor(part, 16);
    part += __shfl_xor(part, 32);
    if (g == 0 && ok) logit[q] = part + b_out;
}

// AMAX: the launch records its inputs' calibration maxima (A.amax,
// A.amax_cls); only then is that code compiled in.
template <class P, int H, int MODE, bool CLS, bool WIDE = false, bool AMAX = false>
__global__ __launch_bounds__(WIDE ? 1024 : 512) void k_mlp(MlpArgs A) {
    using S = typename P::state_t;
    using W = typename P::wfrag_t;
    constexpr int MO = H / 16, KB = H / P::KBLK, NSEG = nseg<MODE>();
    constexpr bool MLP = MODE != CLS_ONLY;
    constexpr int K1 = NSEG * H, K1F = kseg<MODE>() * H;   // multiplied / stored width of W1
    extern __shared__ __align__(16) unsigned char lds_raw[];
    W *sW1 = (W *)lds_raw;
    W *sW2 = (W *)(lds_raw + (NSEG ? frag_bytes<P>(H, K1) : 0));
    W *sC1 = (W *)(lds_raw + mlp_w_bytes<P, H, MODE>());
    // biases, pre-divided by the fp8 descale factor: they initialise the MFMA
    // accumulators (sB: this MLP's two layers; sCB: the classifier's hidden
    // layer, then its output weights)
    float *sB = (float *)(lds_raw + mlp_w_bytes<P, H, MODE>() + (CLS ? frag_bytes<P>(H, H) : 0));
    float *sCB = sB + (MLP ? 2 * H : 0);
    const MlpScales SC = read_scales(A.sc), SCc = read_scales(A.sc_cls);
    if (CLS)
        for (int t = threadIdx.x; t < H; t += blockDim.x) {
            sCB[t] = A.P[A.o_c1 + (int64_t)H * H + t] / SCc.d1;
            sCB[H + t] = A.P[A.o_c2 + t];
        }
    const float b_out = CLS ? A.P[A.o_c2 + H] : 0.f;
    if (MLP) {
        if (NSEG) stage<P>(sW1, A.P + A.o_w1, H, K1, MO, SC.iw1, K1F);
        stage<P>(sW2, A.P + A.o_w2, H, H, MO, SC.iw2);
        for (int t = threadIdx.x; t < H; t += blockDim.x) {
            sB[t] = A.P[A.o_w1 + (int64_t)H * K1F + t] / SC.d1;
            sB[H + t] = A.P[A.o_w2 + (int64_t)H * H + t] / SC.d2;
        }
    }
    if (CLS) stage<P>(sC1, A.P + A.o_c1, H, H, MO, SCc.iw1);
    __syncthreads();
    if (*A.flags) return;

    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    int64_t N = A.n_host;
    if (A.n_dev) N = min((int64_t)*A.n_dev, A.n_host);
    const S *sa = (const S *)A.a;
    const int64_t units = (N + 15) >> 4;
    constexpr int NX = NSEG > 0 ? NSEG * KB : KB;
    const float ix = SC.ix1;
    // gather the inputs of unit u into X
    // fp8 keeps the stored (bf16) state of segment 0 for the residual, so it
    // is not read twice
    constexpr bool RAW = P::kScaled && (MODE == NODE || edge_update<MODE>());
    using raw_t = BF16::frag_t;
    constexpr bool AB = has_ab<MODE>();
    // AB modes: the two per-hit first-layer products of an item (2 MO fragments)
    auto load_ab = [&](int64_t s, int64_t d, f32x4 *G) {
#pragma unroll
        for (int mo = 0; mo < MO; mo++) {
            G[mo] = *(const f32x4 *)(A.ab + s * 2 * H + 16 * mo + 4 * g);
            G[MO + mo] = *(const f32x4 *)(A.ab + d * 2 * H + H + 16 * mo + 4 * g);
        }
    };
    auto load_unit = [&](int64_t u, typename P::frag_t *X, raw_t *R, f32x4 *G) {
        const int64_t q = u * 16 + n;
        const int64_t qc = q < N ? q : N - 1;
        if constexpr (RAW) {
#pragma unroll
            for (int kb = 0; kb < KB; kb++) {
                R[kb] = BF16::load((const BF16::state_t *)sa + qc * H, kb, g);
                X[kb] = P::pack(R[kb], ix);
            }
        }
        if (MODE == NODE) {
            const float *m = (const float *)A.b + qc * 2 * H;
#pragma unroll
            for (int kb = 0; kb < KB; kb++) {
                if constexpr (!RAW) X[kb] = P::load(sa + qc * H, kb, g, ix);
                X[KB + kb] = P::load_f32(m, kb, g, ix);
                X[2 * KB + kb] = P::load_f32(m + H, kb, g, ix);
            }
        } else if (MODE == EDGE) {
            const S *hb = (const S *)A.b;
            const int64_t s = A.src_g[qc], d = A.dst_g[qc];
#pragma unroll
            for (int kb = 0; kb < KB; kb++) {
                if constexpr (!RAW) X[kb] = P::load(sa + qc * H, kb, g, ix);
                X[KB + kb] = P::load(hb + s * H, kb, g, ix);
                X[2 * KB + kb] = P::load(hb + d * H, kb, g, ix);
            }
        } else if (MODE == EDGE_ENC) {
            const int64_t s = A.src_g[qc], d = A.dst_g[qc];
#pragma unroll
            for (int kb = 0; kb < KB; kb++) {
                X[kb] = P::load(sa + s * H, kb, g, ix);
                X[KB + kb] = P::load(sa + d * H, kb, g, ix);
            }
        } else if (MODE == EDGE_AB) {
            const int64_t s = A.src_g[qc], d = A.dst_g[qc];
            if constexpr (!RAW) {
#pragma unroll
                for (int kb = 0; kb < KB; kb++) X[kb] = P::load(sa + qc * H, kb, g, ix);
            }
            load_ab(s, d, G);
        } else if (MODE == ENC_AB) {
            load_ab(A.src_g[qc], A.dst_g[qc], G);
        }
    };
    if constexpr (src_aligned<P, MODE, CLS>()) {
        // Work units are source hits (edges are grouped by source), walked in
        // chunks of 16 of their out-edges (two chunks in flight for the
        // 2-byte states and the factorised encoder, one otherwise).  After a
        // chunk's states are stored, their stored values are summed over the
        // chunk's edges per channel (row_sums: each lane ends with the totals
        // of H / 64 channels) and added up over the hit's chunks in order: the
        // outgoing message sum of the hit (Sec. 5.2), written by every lane
        // for its channels.  Partial sums of a hit with more than 16 edges
        // wait in this wave's LDS slot.
        float *carry = sB + 2 * H + (threadIdx.x >> 6) * H;
        // the walk is uniform over the wavefront: keep it in scalar registers
        const WaveRange wv = wave_range(A.n_rows, A.xcd != 0);
        const WaveRange wr{uniform64(wv.first), uniform64(wv.step), uniform64(wv.end)};
        struct Chunk {
            int64_t i, a0, c0, a1;   // source hit, its first edge, this chunk's first edge, its end
        };
        // the row pointers do not change during the kernel: read them through
        // the constant address space, so uniform reads become scalar loads
        // (which do not count against the vector-memory wait counter)
        const __attribute__((address_space(4))) int *rows4 = (const __attribute__((address_space(4))) int *)A.rows;
        auto from_hit = [&](int64_t i) -> Chunk {
            for (; i < wr.end; i += wr.step) {
                const int64_t a0 = rows4[i], a1 = min((int64_t)rows4[i + 1], N);
                if (a0 < a1) return Chunk{i, a0, a0, a1};
            }
            return Chunk{wr.end, 0, 0, 0};
        };
        auto next = [&](const Chunk &c) -> Chunk {
            if (c.i >= wr.end) return c;
            if (c.c0 + 16 < c.a1) return Chunk{c.i, c.a0, c.c0 + 16, c.a1};
            return from_hit(c.i + wr.step);
        };
        auto load_chunk = [&](const Chunk &c, typename P::frag_t *X, raw_t *R, f32x4 *G) {
            const int64_t q = c.c0 + n;
            const int64_t qc = q < c.a1 ? q : c.a1 - 1;
            const int64_t d = A.dst_g[qc];
            if constexpr (AB) {
                if constexpr (MODE == EDGE_AB) {
#pragma unroll
                    for (int kb = 0; kb < KB; kb++) {
                        if constexpr (RAW) {
                            R[kb] = BF16::load((const BF16::state_t *)sa + qc * H, kb, g);
                            X[kb] = P::pack(R[kb], ix);
                        } else {
                            X[kb] = P::load(sa + qc * H, kb, g, ix);
                        }
                    }
                }
                load_ab(c.i, d, G);
            } else if constexpr (MODE == EDGE) {
                const S *hb = (const S *)A.b;
#pragma unroll
                for (int kb = 0; kb < KB; kb++) {
                    if constexpr (RAW) {
                        R[kb] = BF16::load((const BF16::state_t *)sa + qc * H, kb, g);
                        X[kb] = P::pack(R[kb], ix);
                    } else {
                        X[kb] = P::load(sa + qc * H, kb, g, ix);
                    }
                    X[KB + kb] = P::load(hb + c.i * H, kb, g, ix);
                    X[2 * KB + kb] = P::load(hb + d * H, kb, g, ix);
                }
            } else {
#pragma unroll
                for (int kb = 0; kb < KB; kb++) {
                    X[kb] = P::load(sa + c.i * H, kb, g, ix);
                    X[KB + kb] = P::load(sa + d * H, kb, g, ix);
                }
            }
        };
        auto process = [&](const Chunk &cur, const typename P::frag_t *X, const raw_t *R, const f32x4 *G) {
            const int64_t q = cur.c0 + n;
            const bool ok = q < cur.a1;
            if (AMAX && !AB && A.amax) {   // calibration runs the unsplit modes
                float mx = 0.f;
#pragma unroll
                for (int k = 0; k < NX; k++) mx = fmaxf(mx, P::absmax(X[k]));
                record_amax(mx, A.amax);
            }
            f32x4 hid[MO], o[MO];
            load_bias<MO>(sB, hid, g);
            if constexpr (AB) {
#pragma unroll
                for (int mo = 0; mo < MO; mo++) {
                    hid[mo] += G[mo];
                    hid[mo] += G[MO + mo];
                }
            }
            constexpr int AG = WIDE ? MO / 2 : MO;   // weight fragments held at a time
            // The products run at raised wavefront priority: a wavefront with
            // its inputs in registers keeps the matrix cores until its chunk's
            // products are done, and the other wavefronts of the SIMD issue
            // their loads and epilogues in the gaps.  The wavefronts stay
            // staggered rather than reaching their loads together (measured:
            // -4% per float32 edge network launch; not in the 16-wavefront form)
            if constexpr (!WIDE) __builtin_amdgcn_s_setprio(1);
            if constexpr (NSEG > 0) gemm_first<P, MO, KB, NSEG, MODE, AG>(sW1, X, hid, lane);
            if (P::kScaled) rescale<MO>(hid, SC.d1);
            relu<MO>(hid);
            if (AMAX && A.amax) record_amax(absmax4<MO>(hid), A.amax + 1);
            typename P::frag_t xh[KB];
            P::template chain<MO>(hid, xh, SC.ix2);
            load_bias<MO>(sB + H, o, g);
            gemm<P, MO, KB, 0, KB, false, AG>(sW2, xh, o, lane);
            if constexpr (!WIDE) __builtin_amdgcn_s_setprio(0);
            if (P::kScaled) rescale<MO>(o, SC.d2);
            if constexpr (edge_update<MODE>()) {   // residual (Sec. 5.2), from the unquantised state
#pragma unroll
                for (int mo = 0; mo < MO; mo++)
#pragma unroll
                    for (int i = 0; i < 4; i++) {
                        if constexpr (RAW) o[mo][i] += BF16::seg0(R, mo, i);
                        else o[mo][i] += P::seg0(X, mo, i);
                    }
            }
            if (!A.mout) {
                if (ok) P::template store_all<MO>((S *)A.out + q * H, g, o);
            } else {
                // the states as stored, summed over the chunk's edges: lane n
                // of a row keeps the totals of values 16 t + r(n) (row_sums)
                P::template store_round<MO>((S *)A.out + q * H, g, o, ok);
                constexpr int V = 4 * MO, T = V >= 16 ? V / 16 : 1;
                float v[V];
#pragma unroll
                for (int mo = 0; mo < MO; mo++)
#pragma unroll
                    for (int i = 0; i < 4; i++) v[4 * mo + i] = o[mo][i];
                row_sums<V>(v, n);
                const int r = 8 * (n & 1) + 4 * ((n >> 1) & 1) + 2 * ((n >> 2) & 1) + ((n >> 3) & 1);
                if (V >= 16 || (n & 1) == 0) {
#pragma unroll
                    for (int t = 0; t < T; t++) {
                        const int k = V >= 16 ? 16 * t + r : (r & 7);
                        const int c = P::stored(k >> 2, g) + (k & 3);
                        float tot = v[t];
                        if (cur.c0 != cur.a0) tot += carry[c];
                        if (cur.c0 + 16 >= cur.a1)
                            A.mout[cur.i * 2 * H + c] = tot;
                        else
                            carry[c] = tot;
                    }
                }
            }
        };
        constexpr int NG = AB ? 2 * MO : 1;
        if constexpr (WIDE) {   // one chunk at a time: occupancy hides the loads
            static_assert(wide_ok<P, H, MODE, CLS>(), "WIDE is for the H = 128 2-byte edge MLPs");
            typename P::frag_t X[NX];
            raw_t R[RAW ? KB : 1];
            f32x4 G[NG];
            // Dynamic, XCD-blocked: workgroups are dispatched round-robin over
            // the XCDs, and the wavefronts of XCD x take its slice of source
            // hits kGrab at a time from its counter (A.grab, zeroed before the
            // launch).  They then stay within a window of about kGrab hits per
            // wavefront, so the destination rows they gather are shared in that
            // XCD's L2 (a static stride lets them drift apart by several
            // events).  With fewer workgroups than XCDs there are as many
            // slices as workgroups; a wavefront stops at the first grab past
            // its slice's end.
            const int nsl = min((int)gridDim.x, kXcds);
            const int x = blockIdx.x % nsl;
            const int64_t per = (A.n_rows + nsl - 1) / nsl;
            const int64_t lo = per * x, hi = min(A.n_rows, lo + per);
            int *ctr = A.grab + 32 * x;
            for (;;) {
                int v = 0;
                if (lane == 0) v = atomicAdd(ctr, kGrab);
                const int64_t s0 = lo + __builtin_amdgcn_readfirstlane(v);
                if (s0 >= hi) break;
                const int64_t s1 = min(s0 + kGrab, hi);
                for (int64_t i = s0; i < s1; i++) {
                    const int64_t a0 = rows4[i], a1 = min((int64_t)rows4[i + 1], N);
                    for (int64_t c0 = a0; c0 < a1; c0 += 16) {
                        const Chunk c{i, a0, c0, a1};
                        load_chunk(c, X, R, G);
                        process(c, X, R, G);
                    }
                }
            }
            return;
        }
        // float32 edge networks are MFMA-bound: no prefetch, fewer registers.
        // The factorised edge encoder (one matrix layer) prefetches like the
        // 2-byte precisions: its gathers of the per-hit products dominate.
        if constexpr (sizeof(S) == 4 && MODE != ENC_AB) {
            typename P::frag_t X[NX];
            raw_t R[RAW ? KB : 1];
            f32x4 G[NG];
            for (Chunk c = from_hit(wr.first); c.i < wr.end; c = next(c)) {
                load_chunk(c, X, R, G);
                process(c, X, R, G);
            }
            return;
        }
        // two input buffers in alternation (no register copies): the loads
        // of the next chunk are in flight while this one is computed
        typename P::frag_t XA[NX], XB[NX];
        raw_t RA[RAW ? KB : 1], RB[RAW ? KB : 1];
        f32x4 GA[NG], GB[NG];
        Chunk c0 = from_hit(wr.first);
        Chunk c1 = next(c0);
        if (c0.i < wr.end) load_chunk(c0, XA, RA, GA);
        while (c0.i < wr.end) {
            if (c1.i < wr.end) load_chunk(c1, XB, RB, GB);
            process(c0, XA, RA, GA);
            c0 = c1; c1 = next(c1);
            if (c0.i >= wr.end) break;
            if (c1.i < wr.end) load_chunk(c1, XA, RA, GA);
            process(c0, XB, RB, GB);
            c0 = c1; c1 = next(c1);
        }
        return;
    }
    // memory-bound precisions prefetch the next unit's inputs during the MFMAs,
    // except split operands at H = 128: one unit's inputs alone take about 80
    // registers there (the prefetch spilled and ran slower), and the weight
    // fragments are held half a K block at a time
    constexpr bool LEAN = P::kSplit && H == 128;
    constexpr bool PREFETCH = sizeof(S) < 4 && MLP && !LEAN;
    constexpr int AGU = LEAN ? MO / 2 : MO;
    constexpr int NG = AB ? 2 * MO : 1;
    // two units in flight: Xn holds unit u + step, Xm unit u + 2 step
    typename P::frag_t Xn[NX], Xm[NX];
    raw_t Rn[RAW ? KB : 1], Rm[RAW ? KB : 1];
    f32x4 Gn[NG], Gm[NG];
    const WaveRange wr = wave_range(units, A.xcd != 0);
    int64_t u = wr.first;
    if (PREFETCH && u < wr.end) load_unit(u, Xn, Rn, Gn);
    if (PREFETCH && u + wr.step < wr.end) load_unit(u + wr.step, Xm, Rm, Gm);
    for (; u < wr.end; u += wr.step) {
        const int64_t q = u * 16 + n;
        const bool ok = q < N;
        const int64_t qc = ok ? q : N - 1;
        typename P::frag_t X[NX];
        raw_t R[RAW ? KB : 1];
        f32x4 G[NG];
        if (PREFETCH) {
#pragma unroll
            for (int k = 0; k < NX; k++) {
                X[k] = Xn[k];
                Xn[k] = Xm[k];
            }
            if constexpr (RAW) {
#pragma unroll
                for (int k = 0; k < KB; k++) {
                    R[k] = Rn[k];
                    Rn[k] = Rm[k];
                }
            }
            if constexpr (AB) {
#pragma unroll
                for (int k = 0; k < NG; k++) {
                    G[k] = Gn[k];
                    Gn[k] = Gm[k];
                }
            }
            if (u + 2 * wr.step < wr.end) load_unit(u + 2 * wr.step, Xm, Rm, Gm);
        } else if (MLP) {
            load_unit(u, X, R, G);
        }
        f32x4 o[MO];
        if (MLP) {
            if (AMAX && !AB && A.amax) {   // calibration runs the unsplit modes
                float mx = 0.f;
#pragma unroll
                for (int k = 0; k < NX; k++) mx = fmaxf(mx, P::absmax(X[k]));
                record_amax(mx, A.amax);
            }
            f32x4 hid[MO];
            load_bias<MO>(sB, hid, g);
            if constexpr (AB) {
#pragma unroll
                for (int mo = 0; mo < MO; mo++) {
                    hid[mo] += G[mo];
                    hid[mo] += G[MO + mo];
                }
            }
            // raised priority over the products, as in the source walk (in the
            // classifier-fused edge network only: the node network ran slower)
            if constexpr (CLS) __builtin_amdgcn_s_setprio(1);
            if constexpr (NSEG > 0) gemm_first<P, MO, KB, NSEG, MODE, AGU>(sW1, X, hid, lane);
            if (P::kScaled) rescale<MO>(hid, SC.d1);
            relu<MO>(hid);
            if (AMAX && A.amax) record_amax(absmax4<MO>(hid), A.amax + 1);
            typename P::frag_t xh[KB];
            P::template chain<MO>(hid, xh, SC.ix2);
            load_bias<MO>(sB + H, o, g);
            gemm<P, MO, KB, 0, KB, false, AGU>(sW2, xh, o, lane);
            if (P::kScaled) rescale<MO>(o, SC.d2);
#pragma unroll
            for (int mo = 0; mo < MO; mo++) {
                if constexpr (MODE != EDGE_ENC && MODE != ENC_AB) {   // residual (Sec. 5.2), from the unquantised state
                    if constexpr (RAW) {
#pragma unroll
                        for (int i = 0; i < 4; i++) o[mo][i] += BF16::seg0(R, mo, i);
                    } else if constexpr (!P::kScaled) {
#pragma unroll
                        for (int i = 0; i < 4; i++) o[mo][i] += P::seg0(X, mo, i);
                    }
                }
            }
            if (ok && !(CLS && edge_update<MODE>())) P::template store_all<MO>((S *)A.out + q * H, g, o);
        } else {
#pragma unroll
            for (int mo = 0; mo < MO; mo++) o[mo] = P::load4(sa + qc * H + P::stored(mo, g));
        }
        if (CLS) classify<P, H>(sC1, sCB, b_out, o, SCc, AMAX ? A.amax_cls : nullptr, lane, ok, q, A.logit);
        if constexpr (CLS) __builtin_amdgcn_s_setprio(0);
    }
}

// ------------------------------------------------------------------------
// messages m_i = [sum_{i->j} e_ij, sum_{j->i} e_ji]  (Sec. 5.2, scatter_add)
// H/8 lanes per hit (8 channels each) for 2-byte states, H/4 (4 channels)
// for float32 ones; float32 sums in edge-id order.
// IN_ONLY: the outgoing sums of hits with out-edges were written by the
// edge MLP that produced e (it walks the edges source by source); only hits
// without out-edges get theirs (zero) here.
// Edges are taken in batches of up to 8: the group's lanes first read the
// batch's incoming edge ids (one each), the ids are passed round the group,
// and all of the batch's rows are requested before the first is added, so a
// hit waits for two memory round trips per batch rather than per edge.
// ------------------------------------------------------------------------
template <class P, int H, bool IN_ONLY>
__global__ __launch_bounds__(256) void k_messages(int64_t n_hits, const int *__restrict__ out_ptr,
                                                  const int *__restrict__ in_ptr,
                                                  const int *__restrict__ in_list,
                                                  const typename P::state_t *__restrict__ e,
                                                  float *__restrict__ m, int xcd, const unsigned *__restrict__ flags) {
    if (*flags) return;
    // a lane moves 16 bytes of a row: 8 channels of 2-byte states, 4 of
    // float32 ones; batches of up to 8 rows (one edge id per lane of the group)
    constexpr bool HALF = sizeof(typename P::state_t) == 2;
    constexpr int CPL = HALF ? 8 : 4, LPN = H / CPL, NPW = 64 / LPN, BATCH = LPN < 8 ? LPN : 8;
    const int lane = threadIdx.x & 63, sub = lane / LPN, l = lane % LPN, c = CPL * l, gbase = sub * LPN;
    // rows are kept as loaded (16 bytes) until they are added
    using raw_t = typename std::conditional<HALF, uint4, f32x4>::type;
    auto add = [](f32x4 *s, const raw_t &r) {
        if constexpr (HALF) {
            s[0] += f32x4{__uint_as_float(r.x << 16), __uint_as_float(r.x & 0xffff0000u),
                          __uint_as_float(r.y << 16), __uint_as_float(r.y & 0xffff0000u)};
            s[1] += f32x4{__uint_as_float(r.z << 16), __uint_as_float(r.z & 0xffff0000u),
                          __uint_as_float(r.w << 16), __uint_as_float(r.w & 0xffff0000u)};
        } else {
            s[0] += r;
        }
    };
    constexpr int NS = HALF ? 2 : 1;
    const WaveRange wr = wave_range((n_hits + NPW - 1) / NPW, xcd != 0);
    for (int64_t u = wr.first; u < wr.end; u += wr.step) {
        const int64_t i0 = u * NPW + sub;
        const bool live = i0 < n_hits;
        const int64_t i = live ? i0 : n_hits - 1;
        f32x4 so[NS], si[NS];
#pragma unroll
        for (int k = 0; k < NS; k++) so[k] = si[k] = zero4();
        const int a0 = out_ptr[i], a1 = IN_ONLY ? a0 : out_ptr[i + 1];
        for (int a = a0; !IN_ONLY && a < a1; a += BATCH) {
            const int cnt = min(BATCH, a1 - a);
            raw_t v[BATCH];
#pragma unroll
            for (int j = 0; j < BATCH; j++)
                if (j < cnt) v[j] = *(const raw_t *)(e + (int64_t)(a + j) * H + c);
#pragma unroll
            for (int j = 0; j < BATCH; j++)
                if (j < cnt) add(so, v[j]);
        }
        const int b0 = in_ptr[i], b1 = in_ptr[i + 1];
        for (int b = b0; b < b1; b += BATCH) {   // the group's lanes share the trip count
            const int cnt = min(BATCH, b1 - b);
            const int mine = l < cnt ? in_list[b + l] : 0;
            raw_t v[BATCH];
#pragma unroll
            for (int j = 0; j < BATCH; j++) {
                const int q = __shfl(mine, gbase + j);
                if (j < cnt) v[j] = *(const raw_t *)(e + (int64_t)q * H + c);
            }
#pragma unroll
            for (int j = 0; j < BATCH; j++)
                if (j < cnt) add(si, v[j]);
        }
        if (live) {
#pragma unroll
            for (int k = 0; k < NS; k++) {
                if (!IN_ONLY || a0 == out_ptr[i + 1]) *(f32x4 *)(m + i * 2 * H + c + 4 * k) = so[k];
                *(f32x4 *)(m + i * 2 * H + H + c + 4 * k) = si[k];
            }
        }
    }
}

// Blocks of `block` threads with `lds` bytes of LDS that fit on one compute
// unit together (at least 1); also lifts the dynamic-LDS launch limit.
inline int blocks_per_cu(const void *kernel, int block, size_t lds) {
    (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   // a failure is the launch's error
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, block, lds) != hipSuccess || n < 1) n = 1;
    return n;
}

template <class P, int H, int MODE, bool CLS>
void run_mlp(velo_ctx *c, int stage, MlpArgs a, hipStream_t s) {
    if (a.amax || a.amax_cls) {
        // calibration (bf16 kernels of an fp8 context): 8-wavefront workgroups
        if constexpr (std::is_same<P, BF16>::value) {
            constexpr size_t lds = mlp_lds<P, H, MODE, CLS>();
            const void *kernel = reinterpret_cast<const void *>(&k_mlp<P, H, MODE, CLS, false, true>);
            static const int occ = blocks_per_cu(kernel, kMlpBlock, lds);
            a.xcd = c->tune_xcd[stage];
            k_mlp<P, H, MODE, CLS, false, true><<<persistent_grid(c, stage_per_cu(c, stage, occ, occ)), kMlpBlock,
                                                  lds, s>>>(a);
            return;
        }
    }
    if constexpr (wide_ok<P, H, MODE, CLS>()) {
        if (c->tune_mlp_block[stage] == 2 * kMlpBlock) {
            constexpr size_t lds = mlp_lds<P, H, MODE, CLS, true>();
            const void *kernel = reinterpret_cast<const void *>(&k_mlp<P, H, MODE, CLS, true>);
            static const int occ = blocks_per_cu(kernel, 2 * kMlpBlock, lds);
            a.xcd = c->tune_xcd[stage];
            // the dynamic walk over per-XCD work counters, zeroed here
            a.grab = c->ws.grab;
            launch_fill(a.grab, 0, kXcds * 32, s);
            k_mlp<P, H, MODE, CLS, true><<<persistent_grid(c, stage_per_cu(c, stage, occ, occ)), 2 * kMlpBlock,
                                           lds, s>>>(a);
            return;
        }
    }
    constexpr size_t lds = mlp_lds<P, H, MODE, CLS>();
    // workgroup shape: 8 wavefronts sharing one staged copy of the weights,
    // or 4 (twice the copies, finer-grained residency); chosen by velo_autotune
    const void *kernel = reinterpret_cast<const void *>(&k_mlp<P, H, MODE, CLS>);
    static const int occ8 = blocks_per_cu(kernel, kMlpBlock, lds), occ4 = blocks_per_cu(kernel, kMlpBlock / 2, lds);
    const bool four = c->tune_mlp_block[stage] == kMlpBlock / 2;
    const int occ = four ? occ4 : occ8;
    a.xcd = c->tune_xcd[stage];
    k_mlp<P, H, MODE, CLS><<<persistent_grid(c, stage_per_cu(c, stage, occ, occ)), four ? kMlpBlock / 2 : kMlpBlock,
                             lds, s>>>(a);
}

// float32 MLPs are MFMA-bound: their edge MLPs take the hit segments'
// first-layer products from k_hit_proj (the AB modes), which removes two
// thirds of the edge encoder's and half of the edge network's per-edge
// matrix work.  The training form does the same and keeps the products of
// every step, so the backward pass recomputes the hidden layers with the
// same sums.  fp8 calibration keeps the concatenated form.
template <class P>
constexpr bool uses_ab() { return sizeof(typename P::state_t) == 4; }

template <class P, int H, int MODE, int MODE_AB, bool CLS>
void run_mlp_ab(velo_ctx *c, int stage, const MlpArgs &a, bool ab, hipStream_t s) {
    if constexpr (uses_ab<P>()) {
        if (ab) {
            run_mlp<P, H, MODE_AB, CLS>(c, stage, a, s);
            return;
        }
    }
    run_mlp<P, H, MODE, CLS>(c, stage, a, s);
}

// The GNN forward pass.  Inference updates the edge state in place and fuses
// the classifier into the last edge network; training (train = true) keeps
// every step's hit and edge encodings and messages as checkpoints for the
// backward pass (ck_h[k], ck_e[k], ck_m[k]) and reads the caller's parameters.
template <class P, int H>
void gnn_ph(velo_ctx *c, const velo_hits *hits, float *logit, const float *Pw, bool train,
            bool calib, hipStream_t s) {
    using S = typename P::state_t;
    Workspace &w = c->ws;
    const ParamLayout &L = c->layout;
    const int64_t N = hits->n_hits, Ecap = c->cfg.max_edges;
    const int64_t Nmax = c->cfg.max_hits;
    const int iters = c->cfg.gnn_iters;
    // per-MLP fp8 scales {s_x1, s_w1, s_x2, s_w2} and calibration maxima
    auto sc = [&](int slot) -> const float * { return P::kScaled ? w.scales + 4 * slot : nullptr; };
    auto am = [&](int slot) -> float * { return calib ? w.amax + 2 * slot : nullptr; };
    const int s_nenc = kSlotNodeEnc, s_eenc = kSlotEdgeEnc, s_cls = slot_cls(iters);
    auto hk = [&](int k) -> S * { return train ? (S *)w.ck_h + (int64_t)k * Nmax * H : (S *)w.h[k & 1]; };
    auto ek = [&](int k) -> S * { return train ? (S *)w.ck_e + (int64_t)k * Ecap * H : (S *)w.e; };
    auto mk = [&](int k) -> float * { return train ? w.ck_m + (int64_t)k * Nmax * 2 * H : w.m; };
    const bool ab = uses_ab<P>() && !calib;
    // where the per-hit products of edge MLP `slot` go (0..n-1: edge networks,
    // n: the edge encoder); training keeps every step's for the backward pass
    auto abk = [&](int slot) -> float * { return train ? w.ck_ab + (int64_t)slot * Nmax * 2 * H : w.ab; };
    auto hit_proj = [&](const S *h, int64_t o_w1, int k1f, int cs, int cd, const float *scp, float *dst) {
        if constexpr (uses_ab<P>()) {
            if (N <= 0) return;
            StageTimer t(c, VELO_STAGE_HIT_PROJ, s);
            constexpr size_t lds = 2 * frag_bytes<P>(H, H);
            static const int per_cu =
                blocks_per_cu(reinterpret_cast<const void *>(&k_hit_proj<P, H>), kMlpBlock, lds);
            k_hit_proj<P, H><<<persistent_grid(c, per_cu), kMlpBlock, lds, s>>>(N, h, Pw, o_w1, k1f, cs, cd, scp,
                                                                                dst, w.flags);
        }
    };
    // the classifier is fused into the last edge network when its weights fit in LDS too
    // (not when the triplet stage needs the final edge states)
    const bool fuse_cls = !train && !c->tri_set &&
                          (ab ? mlp_lds<P, H, EDGE_AB, true>() : mlp_lds<P, H, EDGE, true>()) <= c->lds_max;
    if (N > 0) {
        const size_t lds = frag_bytes<P>(H, H) + sizeof(float) * H * 4;
        static const int per_cu = blocks_per_cu(reinterpret_cast<const void *>(&k_node_enc<P, H>), kMlpBlock, lds);
        StageTimer t(c, VELO_STAGE_NODE_ENC, s);
        k_node_enc<P, H><<<persistent_grid(c, per_cu), kMlpBlock, lds, s>>>(
            N, hits->x, hits->y, hits->z, Pw, L.nenc[0].w, L.nenc[1].w, hk(0), sc(s_nenc), am(s_nenc), w.flags);
    }
    MlpArgs a{};
    a.n_dev = w.n_edges; a.n_host = Ecap; a.src_g = w.src_g; a.dst_g = w.dst_g;
    a.P = Pw; a.flags = w.flags; a.logit = logit;
    a.o_c1 = L.cls[0].w; a.o_c2 = L.cls[1].w;
    a.a = hk(0); a.out = ek(0); a.o_w1 = L.eenc[0].w; a.o_w2 = L.eenc[1].w;
    a.sc = sc(s_eenc); a.amax = am(s_eenc); a.sc_cls = sc(s_cls); a.amax_cls = am(s_cls);
    // 2-byte states: the edge encoder and every edge network but the last
    // also write the outgoing message sums of their output states
    static_assert(src_aligned<P, EDGE, false>() == src_aligned<P, EDGE_ENC, false>() &&
                      src_aligned<P, EDGE_AB, false>() == src_aligned<P, ENC_AB, false>(),
                  "both edge MLPs of a form write the outgoing sums or neither");
    const bool out_fused = ab ? src_aligned<P, EDGE_AB, false>() : src_aligned<P, EDGE, false>();
    a.rows = w.row_ptr; a.n_rows = N; a.mout = mk(0); a.ab = abk(iters);
    if (ab) hit_proj(hk(0), L.eenc[0].w, 2 * H, 0, H, sc(s_eenc), abk(iters));
    {
        StageTimer t(c, VELO_STAGE_EDGE_ENC, s);
        run_mlp_ab<P, H, EDGE_ENC, ENC_AB, false>(c, VELO_STAGE_EDGE_ENC, a, ab, s);
    }
    for (int k = 0; k < iters; k++) {
        if (N > 0) {
            StageTimer t(c, VELO_STAGE_MESSAGES, s);
            const int grid = persistent_grid(c, stage_per_cu(c, VELO_STAGE_MESSAGES, 16));
            if (out_fused)
                k_messages<P, H, true><<<grid, 256, 0, s>>>(N, w.row_ptr, w.in_ptr, w.in_list, ek(k), mk(k),
                                                             c->tune_xcd[VELO_STAGE_MESSAGES], w.flags);
            else
                k_messages<P, H, false><<<grid, 256, 0, s>>>(N, w.row_ptr, w.in_ptr, w.in_list, ek(k), mk(k),
                                                              c->tune_xcd[VELO_STAGE_MESSAGES], w.flags);
        }
        MlpArgs nd{};
        nd.n_dev = nullptr; nd.n_host = N; nd.a = hk(k); nd.b = mk(k); nd.out = hk(k + 1);
        nd.P = Pw; nd.o_w1 = L.node[k][0].w; nd.o_w2 = L.node[k][1].w; nd.flags = w.flags;
        nd.sc = sc(slot_node(k)); nd.amax = am(slot_node(k));
        if (N > 0) {
            StageTimer t(c, VELO_STAGE_NODE_NET, s);
            run_mlp<P, H, NODE, false>(c, VELO_STAGE_NODE_NET, nd, s);
        }
        MlpArgs ed = a;
        ed.a = ek(k); ed.b = hk(k + 1); ed.out = ek(k + 1); ed.o_w1 = L.edge[k][0].w; ed.o_w2 = L.edge[k][1].w;
        ed.sc = sc(slot_edge(k)); ed.amax = am(slot_edge(k));
        const bool last = k == iters - 1;
        ed.mout = last ? nullptr : mk(k + 1);
        ed.ab = abk(k);
        if (ab) hit_proj(hk(k + 1), L.edge[k][0].w, 3 * H, H, 2 * H, sc(slot_edge(k)), abk(k));
        StageTimer t(c, last && fuse_cls ? VELO_STAGE_EDGE_CLS : VELO_STAGE_EDGE_NET, s);
        if (last && fuse_cls)
            run_mlp_ab<P, H, EDGE, EDGE_AB, true>(c, VELO_STAGE_EDGE_CLS, ed, ab, s);
        else
            run_mlp_ab<P, H, EDGE, EDGE_AB, false>(c, VELO_STAGE_EDGE_NET, ed, ab, s);
    }
    if (iters == 0 || !fuse_cls) {
        MlpArgs cl = a;
        cl.a = ek(iters);
        StageTimer t(c, VELO_STAGE_EDGE_CLS, s);
        run_mlp<P, H, CLS_ONLY, true>(c, VELO_STAGE_EDGE_CLS, cl, s);
    }
}

template <class P>
void embed_p(velo_ctx *c, const velo_hits *h, float *emb, const float *sc, float *amax, hipStream_t s) {
    const size_t lds = frag_bytes<P>(kCe, kCe) + frag_bytes<P>(16, kCe) + sizeof(float) * kCe * 4;
    static const int per_cu = blocks_per_cu(reinterpret_cast<const void *>(&k_embed<P>), kMlpBlock, lds);
    const ParamLayout &L = c->layout;
    k_embed<P><<<persistent_grid(c, per_cu), kMlpBlock, lds, s>>>(h->n_hits, h->x, h->y, h->z, c->params, L.emb[0].w,
                                                             L.emb[1].w, L.emb[2].w, emb, sc, amax, nullptr,
                                                             nullptr, nullptr, c->ws.flags);
}

}  // namespace

namespace {

constexpr float kE4M3Max = 448.f;   // largest finite OCP E4M3 value
constexpr int kMaxWeightScales = 2 * (4 + 2 * 16);

struct WeightScaleDesc {
    int64_t off[kMaxWeightScales];
    int cnt[kMaxWeightScales];
    int dst[kMaxWeightScales];
    int n;
};

// s_w = max |W| / 448 for every fp8 weight matrix (one block per matrix)
__global__ __launch_bounds__(256) void k_weight_scales(const float *__restrict__ P, WeightScaleDesc d,
                                                       float *__restrict__ scales) {
    __shared__ float sh[256];
    const int j = blockIdx.x;
    if (j >= d.n) return;
    float m = 0.f;
    for (int i = threadIdx.x; i < d.cnt[j]; i += blockDim.x) m = fmaxf(m, fabsf(P[d.off[j] + i]));
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + k]);
        __syncthreads();
    }
    if (threadIdx.x == 0) scales[d.dst[j]] = sh[0] > 0.f ? sh[0] / kE4M3Max : 1.f;
}

// s_x = max |x| / 448 from the calibration maxima of every MLP input
__global__ void k_act_scales(const float *__restrict__ amax, float *__restrict__ scales, int n_slots) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n_slots) return;
    for (int j = 0; j < 2; j++) {
        const float a = amax[2 * m + j];
        scales[4 * m + 2 * j] = a > 0.f ? a / kE4M3Max : 1.f;
    }
}

}  // namespace

void launch_weight_scales(velo_ctx *c, hipStream_t s) {
    const ParamLayout &L = c->layout;
    WeightScaleDesc d{};
    auto add = [&](const Lin &l, int slot, int which) {
        d.off[d.n] = l.w;
        d.cnt[d.n] = l.out * l.in;
        d.dst[d.n] = 4 * slot + (which == 1 ? 1 : 3);
        d.n++;
    };
    add(L.emb[1], kSlotEmbed, 1);
    add(L.emb[2], kSlotEmbed, 2);
    add(L.nenc[1], kSlotNodeEnc, 2);
    add(L.eenc[0], kSlotEdgeEnc, 1);
    add(L.eenc[1], kSlotEdgeEnc, 2);
    for (int k = 0; k < c->cfg.gnn_iters; k++) {
        add(L.node[k][0], slot_node(k), 1);
        add(L.node[k][1], slot_node(k), 2);
        add(L.edge[k][0], slot_edge(k), 1);
        add(L.edge[k][1], slot_edge(k), 2);
    }
    add(L.cls[0], slot_cls(c->cfg.gnn_iters), 1);
    k_weight_scales<<<d.n, 256, 0, s>>>(c->params, d, c->ws.scales);
}

void launch_act_scales(velo_ctx *c, hipStream_t s) {
    const int n = n_slots(c->cfg.gnn_iters);
    k_act_scales<<<(n + 63) / 64, 64, 0, s>>>(c->ws.amax, c->ws.scales, n);
}

size_t state_bytes(int precision) { return precision == VELO_FP32 ? sizeof(float) : sizeof(uint16_t); }

bool gnn_supported(int hidden, int precision) {
    if (precision == VELO_FP32) return hidden == 32 || hidden == 64;
    if (precision == VELO_BF16 || precision == VELO_FP8) return hidden == 32 || hidden == 64 || hidden == 128;
    if (precision == VELO_BF16X2) return hidden == 32 || hidden == 64 || hidden == 128;
    return false;
}

// calib: run the bf16 kernels of an fp8 context and record every MLP input's
// largest |value| (the activation scales are derived from them).
void launch_embed_train(velo_ctx *c, const velo_hits *h, const float *params, float *emb, float *sv,
                        float *sa1, float *sa2, hipStream_t s) {
    if (h->n_hits <= 0) return;
    const size_t lds = frag_bytes<F32>(kCe, kCe) + frag_bytes<F32>(16, kCe) + sizeof(float) * kCe * 4;
    static const int per_cu = blocks_per_cu(reinterpret_cast<const void *>(&k_embed<F32>), kMlpBlock, lds);
    const ParamLayout &L = c->layout;
    k_embed<F32><<<persistent_grid(c, per_cu), kMlpBlock, lds, s>>>(h->n_hits, h->x, h->y, h->z, params, L.emb[0].w,
                                                                L.emb[1].w, L.emb[2].w, emb, nullptr, nullptr, sv,
                                                                sa1, sa2, c->ws.flags);
}

void launch_embed(velo_ctx *c, const velo_hits *h, float *emb, bool calib, hipStream_t s) {
    if (h->n_hits <= 0) return;
    const int p = c->cfg.precision;
    if (c->emb_int8 && !calib)
        embed_p<I8>(c, h, emb, c->ws.i8_scales, nullptr, s);
    else if (p == VELO_FP32 || p == VELO_BF16X2)   // bf16x2: bf16 weights would move pairs across the radius
        embed_p<F32>(c, h, emb, nullptr, nullptr, s);
    else if (p == VELO_BF16 || calib)
        embed_p<BF16>(c, h, emb, nullptr, calib ? c->ws.amax + 2 * kSlotEmbed : nullptr, s);
    else
        embed_p<FP8>(c, h, emb, c->ws.scales + 4 * kSlotEmbed, nullptr, s);
}

void launch_embed_int8_amax(velo_ctx *c, const velo_hits *h, float *emb, hipStream_t s) {
    if (h->n_hits <= 0) return;
    embed_p<F32>(c, h, emb, nullptr, c->ws.i8_amax, s);
}

void launch_gnn(velo_ctx *c, const velo_hits *h, float *logit, const float *params, bool train, bool calib,
                hipStream_t s) {
    const int H = c->cfg.gnn_hidden, p = c->cfg.precision;
    if (p == VELO_FP32) {
        if (H == 32) gnn_ph<F32, 32>(c, h, logit, params, train, false, s);
        if (H == 64) gnn_ph<F32, 64>(c, h, logit, params, train, false, s);
    } else if (p == VELO_BF16X2) {
        if (H == 32) gnn_ph<BF16X2, 32>(c, h, logit, params, train, false, s);
        if (H == 64) gnn_ph<BF16X2, 64>(c, h, logit, params, train, false, s);
        if (H == 128) gnn_ph<BF16X2, 128>(c, h, logit, params, train, false, s);
    } else if (p == VELO_BF16 || calib) {
        if (H == 32) gnn_ph<BF16, 32>(c, h, logit, params, train, calib, s);
        if (H == 64) gnn_ph<BF16, 64>(c, h, logit, params, train, calib, s);
        if (H == 128) gnn_ph<BF16, 128>(c, h, logit, params, train, calib, s);
    } else {
        if (H == 32) gnn_ph<FP8, 32>(c, h, logit, params, train, false, s);
        if (H == 64) gnn_ph<FP8, 64>(c, h, logit, params, train, false, s);
        if (H == 128) gnn_ph<FP8, 128>(c, h, logit, params, train, false, s);
    }
}

}  // namespace velo
