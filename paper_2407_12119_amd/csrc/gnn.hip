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
#include "internal.h"

namespace velo {

namespace {

typedef __bf16 bf16;
typedef bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ inline f32x4 zero4() { return f32x4{0.f, 0.f, 0.f, 0.f}; }

// ------------------------------------------------------------------------
// precision traits
// ------------------------------------------------------------------------
struct F32 {
    using state_t = float;       // hit/edge encodings in HBM
    using frag_t = f32x4;        // per-lane B operand of one K block
    using wfrag_t = f32x4;       // per-lane A operand of one (output block, K block)
    static constexpr int KBLK = 16;
    static constexpr int WJ = 4;
    __device__ static int col(int kb, int g, int j) { return 16 * kb + 4 * g + j; }
    __device__ static float wconv(float v) { return v; }
    __device__ static frag_t load(const float *row, int kb, int g) { return *(const f32x4 *)(row + 16 * kb + 4 * g); }
    __device__ static frag_t load_f32(const float *row, int kb, int g) { return load(row, kb, g); }
    template <int MO>
    __device__ static void mma(const wfrag_t *a, const frag_t &x, f32x4 *acc) {
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int mo = 0; mo < MO; mo++)
                acc[mo] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mo][i], x[i], acc[mo], 0, 0, 0);
    }
    // accumulators of MO output blocks -> B fragments of the next layer (MO*16/KBLK of them)
    template <int MO>
    __device__ static void chain(const f32x4 *h, frag_t *x) {
#pragma unroll
        for (int kb = 0; kb < MO; kb++) x[kb] = h[kb];
    }
    // value of input channel 16 mo + 4 g + i of segment 0
    __device__ static float seg0(const frag_t *x, int mo, int i) { return x[mo][i]; }
    // stored offset of logical channels 16 mo + 4 g + (0..3)
    __device__ static int stored(int mo, int g) { return 16 * mo + 4 * g; }
    template <int MO>
    __device__ static void store_all(float *row, int g, const f32x4 *o) {
#pragma unroll
        for (int mo = 0; mo < MO; mo++) *(f32x4 *)(row + 16 * mo + 4 * g) = o[mo];
    }
    __device__ static f32x4 load4(const float *p) { return *(const f32x4 *)p; }
};

struct BF16 {
    using state_t = bf16;
    using frag_t = bf16x8;
    using wfrag_t = bf16x8;
    static constexpr int KBLK = 32;
    static constexpr int WJ = 8;
    __device__ static int col(int kb, int g, int j) { return 32 * kb + (j < 4 ? 4 * g + j : 16 + 4 * g + j - 4); }
    __device__ static bf16 wconv(float v) { return (bf16)v; }
    __device__ static frag_t cat(bf16x4 lo, bf16x4 hi) {
        return frag_t{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    }
    __device__ static bf16x4 cvt(f32x4 v) { return bf16x4{(bf16)v[0], (bf16)v[1], (bf16)v[2], (bf16)v[3]}; }
    // Encodings are stored with each 32-channel block permuted so that the 8
    // channels a lane owns are contiguous: logical channel col(kb, g, j) sits
    // at 32 kb + 8 g + j.  Every internal state row (hit and edge encodings,
    // messages) uses this order; a lane moves its block with one 16-byte access.
    __device__ static frag_t load(const bf16 *row, int kb, int g) { return *(const bf16x8 *)(row + 32 * kb + 8 * g); }
    __device__ static frag_t load_f32(const float *row, int kb, int g) {
        return cat(cvt(*(const f32x4 *)(row + 32 * kb + 8 * g)), cvt(*(const f32x4 *)(row + 32 * kb + 8 * g + 4)));
    }
    __device__ static int stored(int mo, int g) { return 32 * (mo >> 1) + 8 * g + 4 * (mo & 1); }
    template <int MO>
    __device__ static void store_all(bf16 *row, int g, const f32x4 *o) {
#pragma unroll
        for (int kb = 0; kb < MO / 2; kb++) *(bf16x8 *)(row + 32 * kb + 8 * g) = cat(cvt(o[2 * kb]), cvt(o[2 * kb + 1]));
    }
    template <int MO>
    __device__ static void mma(const wfrag_t *a, const frag_t &x, f32x4 *acc) {
#pragma unroll
        for (int mo = 0; mo < MO; mo++) acc[mo] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mo], x, acc[mo], 0, 0, 0);
    }
    template <int MO>
    __device__ static void chain(const f32x4 *h, frag_t *x) {
#pragma unroll
        for (int kb = 0; kb < MO / 2; kb++) x[kb] = cat(cvt(h[2 * kb]), cvt(h[2 * kb + 1]));
    }
    __device__ static float seg0(const frag_t *x, int mo, int i) { return (float)x[mo >> 1][4 * (mo & 1) + i]; }
    __device__ static f32x4 load4(const bf16 *p) {
        const bf16x4 v = *(const bf16x4 *)p;
        return f32x4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
    }
};

// Stage a row-major [rows x K] float32 weight into LDS in fragment order:
// entry (mo, kb, lane) holds W[16 mo + (lane & 15)][col(kb, lane >> 4, j)],
// rows >= `rows` (padding up to 16*MO) are zero.
template <class P>
__device__ inline void stage(typename P::wfrag_t *dst, const float *__restrict__ W, int rows, int K, int MO) {
    const int KBn = K / P::KBLK;
    const int total = MO * KBn * 64;
    for (int f = threadIdx.x; f < total; f += blockDim.x) {
        const int lane = f & 63, mk = f >> 6, kb = mk % KBn, mo = mk / KBn;
        const int row = 16 * mo + (lane & 15), g = lane >> 4;
        typename P::wfrag_t v;
#pragma unroll
        for (int j = 0; j < P::WJ; j++) v[j] = P::wconv(row < rows ? W[(int64_t)row * K + P::col(kb, g, j)] : 0.f);
        dst[f] = v;
    }
}

template <class P>
constexpr size_t frag_bytes(int rows_pad, int K) {
    return (size_t)rows_pad * K * sizeof(typename P::wfrag_t) / P::WJ;
}

// acc[mo] += W[16 mo .., K] * X   (KB = K / KBLK blocks)
template <class P, int MO, int KB>
__device__ inline void gemm(const typename P::wfrag_t *sW, const typename P::frag_t *X, f32x4 *acc, int lane) {
#pragma unroll
    for (int kb = 0; kb < KB; kb++) {
        // keep one K block of weight fragments live at a time
        __builtin_amdgcn_sched_barrier(0);
        typename P::wfrag_t a[MO];
#pragma unroll
        for (int mo = 0; mo < MO; mo++) a[mo] = sW[(mo * KB + kb) * 64 + lane];
        P::template mma<MO>(a, X[kb], acc);
    }
}

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

template <int MO>
__device__ inline void zero(f32x4 *acc) {
#pragma unroll
    for (int mo = 0; mo < MO; mo++) acc[mo] = zero4();
}

__device__ inline int wave_id() { return (blockIdx.x * blockDim.x + threadIdx.x) >> 6; }
__device__ inline int n_waves() { return (gridDim.x * blockDim.x) >> 6; }

// First layer with three inputs (K = 3) on the vector ALU, written in the
// accumulator layout: h[mo][i] = relu(W[c] . u + b[c]), c = 16 mo + 4 g + i.
// sW holds W [C x 3] followed by b [C].
template <int MO>
__device__ inline void first_layer3(const float *sW, int C, float u0, float u1, float u2, int g, f32x4 *h) {
#pragma unroll
    for (int mo = 0; mo < MO; mo++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int c = 16 * mo + 4 * g + i;
            h[mo][i] = fmaxf(sW[c * 3] * u0 + sW[c * 3 + 1] * u1 + sW[c * 3 + 2] * u2 + sW[C * 3 + c], 0.f);
        }
}

// ------------------------------------------------------------------------
// embedding MLP 3 -> 128 -> 128 -> 4 on normalised (r, phi, z)  (Sec. 5.1)
// ------------------------------------------------------------------------
constexpr int kCe = VELO_EMB_HIDDEN;

template <class P>
__global__ __launch_bounds__(512) void k_embed(int64_t n_hits, const float *__restrict__ x,
                                               const float *__restrict__ y, const float *__restrict__ z,
                                               const float *__restrict__ P_, int64_t o_w1, int64_t o_w2,
                                               int64_t o_w3, float *__restrict__ emb,
                                               const unsigned *__restrict__ flags) {
    using W = typename P::wfrag_t;
    constexpr int MO = kCe / 16, KB = kCe / P::KBLK;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    W *sW2 = (W *)lds_raw;
    W *sW3 = (W *)(lds_raw + frag_bytes<P>(kCe, kCe));
    float *sW1 = (float *)(lds_raw + frag_bytes<P>(kCe, kCe) + frag_bytes<P>(16, kCe));
    stage<P>(sW2, P_ + o_w2, kCe, kCe, MO);
    stage<P>(sW3, P_ + o_w3, VELO_EMB_DIM, kCe, 1);
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
        typename P::frag_t x1[KB];
        P::template chain<MO>(h1, x1);
        f32x4 h2[MO];
        zero<MO>(h2);
        gemm<P, MO, KB>(sW2, x1, h2, lane);
        bias_relu<MO>(h2, rb2);
        typename P::frag_t x2[KB];
        P::template chain<MO>(h2, x2);
        f32x4 o[1];
        zero<1>(o);
        gemm<P, 1, KB>(sW3, x2, o, lane);
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
template <class P, int H>
__global__ __launch_bounds__(512) void k_node_enc(int64_t n_hits, const float *__restrict__ x,
                                                  const float *__restrict__ y, const float *__restrict__ z,
                                                  const float *__restrict__ P_, int64_t o_w1, int64_t o_w2,
                                                  typename P::state_t *__restrict__ h,
                                                  const unsigned *__restrict__ flags) {
    using W = typename P::wfrag_t;
    constexpr int MO = H / 16, KB = H / P::KBLK;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    W *sW2 = (W *)lds_raw;
    float *sW1 = (float *)(lds_raw + frag_bytes<P>(H, H));
    stage<P>(sW2, P_ + o_w2, H, H, MO);
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
        typename P::frag_t x1[KB];
        P::template chain<MO>(h1, x1);
        f32x4 o[MO];
        zero<MO>(o);
        gemm<P, MO, KB>(sW2, x1, o, lane);
        if (i < n_hits) {
#pragma unroll
            for (int mo = 0; mo < MO; mo++) o[mo] += rb2[mo];
            P::template store_all<MO>(h + i * H, g, o);
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
// ------------------------------------------------------------------------
enum Mode { NODE = 0, EDGE = 1, EDGE_ENC = 2, CLS_ONLY = 3 };

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
    const unsigned *flags;
};

template <int MODE>
constexpr int nseg() { return MODE == EDGE_ENC ? 2 : (MODE == CLS_ONLY ? 0 : 3); }

template <class P, int H, int MODE, bool CLS>
constexpr size_t mlp_lds() {
    return (nseg<MODE>() ? frag_bytes<P>(H, nseg<MODE>() * H) + frag_bytes<P>(H, H) : 0) +
           (CLS ? frag_bytes<P>(H, H) : 0);
}

template <class P, int H>
__device__ inline void classify(const typename P::wfrag_t *sC1, const float *__restrict__ Pw, int64_t o_c1,
                                int64_t o_c2, const f32x4 *ev, int lane, bool ok, int64_t q,
                                float *__restrict__ logit) {
    constexpr int MO = H / 16, KB = H / P::KBLK;
    const int g = lane >> 4;
    typename P::frag_t xe[KB];
    P::template chain<MO>(ev, xe);
    f32x4 hc[MO];
    zero<MO>(hc);
    gemm<P, MO, KB>(sC1, xe, hc, lane);
    f32x4 rb[MO], w2[MO];
    load_bias<MO>(Pw + o_c1 + H * H, rb, g);
    load_bias<MO>(Pw + o_c2, w2, g);
    float part = 0.f;
#pragma unroll
    for (int mo = 0; mo < MO; mo++)
#pragma unroll
        for (int i = 0; i < 4; i++) part += w2[mo][i] * fmaxf(hc[mo][i] + rb[mo][i], 0.f);
    part += __shfl_xor(part, 16);
    part += __shfl_xor(part, 32);
    if (g == 0 && ok) logit[q] = part + Pw[o_c2 + H];
}

template <class P, int H, int MODE, bool CLS>
__global__ __launch_bounds__(512) void k_mlp(MlpArgs A) {
    using S = typename P::state_t;
    using W = typename P::wfrag_t;
    constexpr int MO = H / 16, KB = H / P::KBLK, NSEG = nseg<MODE>();
    constexpr int K1 = NSEG * H;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    W *sW1 = (W *)lds_raw;
    W *sW2 = (W *)(lds_raw + (NSEG ? frag_bytes<P>(H, K1) : 0));
    W *sC1 = (W *)(lds_raw + (NSEG ? frag_bytes<P>(H, K1) + frag_bytes<P>(H, H) : 0));
    if (NSEG) {
        stage<P>(sW1, A.P + A.o_w1, H, K1, MO);
        stage<P>(sW2, A.P + A.o_w2, H, H, MO);
    }
    if (CLS) stage<P>(sC1, A.P + A.o_c1, H, H, MO);
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
    const S *sa = (const S *)A.a;
    const int64_t units = (N + 15) >> 4;
    constexpr int NX = NSEG > 0 ? NSEG * KB : KB;
    // gather the inputs of unit u into X
    auto load_unit = [&](int64_t u, typename P::frag_t *X) {
        const int64_t q = u * 16 + n;
        const int64_t qc = q < N ? q : N - 1;
        if (MODE == NODE) {
            const float *m = (const float *)A.b + qc * 2 * H;
#pragma unroll
            for (int kb = 0; kb < KB; kb++) {
                X[kb] = P::load(sa + qc * H, kb, g);
                X[KB + kb] = P::load_f32(m, kb, g);
                X[2 * KB + kb] = P::load_f32(m + H, kb, g);
            }
        } else if (MODE == EDGE) {
            const S *hb = (const S *)A.b;
            const int64_t s = A.src_g[qc], d = A.dst_g[qc];
#pragma unroll
            for (int kb = 0; kb < KB; kb++) {
                X[kb] = P::load(sa + qc * H, kb, g);
                X[KB + kb] = P::load(hb + s * H, kb, g);
                X[2 * KB + kb] = P::load(hb + d * H, kb, g);
            }
        } else if (MODE == EDGE_ENC) {
            const int64_t s = A.src_g[qc], d = A.dst_g[qc];
#pragma unroll
            for (int kb = 0; kb < KB; kb++) {
                X[kb] = P::load(sa + s * H, kb, g);
                X[KB + kb] = P::load(sa + d * H, kb, g);
            }
        }
    };
    // memory-bound precisions prefetch the next unit's inputs during the MFMAs
    constexpr bool PREFETCH = sizeof(S) < 4 && NSEG > 0;
    typename P::frag_t Xn[NX];
    int64_t u = wave_id();
    if (PREFETCH && u < units) load_unit(u, Xn);
    for (; u < units; u += n_waves()) {
        const int64_t q = u * 16 + n;
        const bool ok = q < N;
        const int64_t qc = ok ? q : N - 1;
        typename P::frag_t X[NX];
        if (PREFETCH) {
#pragma unroll
            for (int k = 0; k < NX; k++) X[k] = Xn[k];
            if (u + n_waves() < units) load_unit(u + n_waves(), Xn);
        } else if (NSEG > 0) {
            load_unit(u, X);
        }
        f32x4 o[MO];
        if (NSEG) {
            f32x4 hid[MO];
            zero<MO>(hid);
            gemm<P, MO, NSEG * KB>(sW1, X, hid, lane);
            bias_relu<MO>(hid, rb1);
            typename P::frag_t xh[KB];
            P::template chain<MO>(hid, xh);
            zero<MO>(o);
            gemm<P, MO, KB>(sW2, xh, o, lane);
#pragma unroll
            for (int mo = 0; mo < MO; mo++) {
                o[mo] += rb2[mo];
                if (MODE != EDGE_ENC)   // residual (Sec. 5.2)
#pragma unroll
                    for (int i = 0; i < 4; i++) o[mo][i] += P::seg0(X, mo, i);
            }
            if (ok && !(CLS && MODE == EDGE)) P::template store_all<MO>((S *)A.out + q * H, g, o);
        } else {
#pragma unroll
            for (int mo = 0; mo < MO; mo++) o[mo] = P::load4(sa + qc * H + P::stored(mo, g));
        }
        if (CLS) classify<P, H>(sC1, A.P, A.o_c1, A.o_c2, o, lane, ok, q, A.logit);
    }
}

// ------------------------------------------------------------------------
// messages m_i = [sum_{i->j} e_ij, sum_{j->i} e_ji]  (Sec. 5.2, scatter_add)
// H/4 lanes per hit, 4 channels per lane, float32 sums in edge-id order
// ------------------------------------------------------------------------
template <class P, int H>
__global__ __launch_bounds__(256) void k_messages(int64_t n_hits, const int *__restrict__ out_ptr,
                                                  const int *__restrict__ out_list,
                                                  const int *__restrict__ in_ptr,
                                                  const int *__restrict__ in_list,
                                                  const typename P::state_t *__restrict__ e,
                                                  float *__restrict__ m, const unsigned *__restrict__ flags) {
    if (*flags) return;
    constexpr int LPN = H / 4, NPW = 64 / LPN;
    const int lane = threadIdx.x & 63, sub = lane / LPN, c = 4 * (lane % LPN);
    for (int64_t base = (int64_t)wave_id() * NPW; base < n_hits; base += (int64_t)n_waves() * NPW) {
        const int64_t i = base + sub;
        if (i >= n_hits) continue;
        f32x4 so = zero4(), si = zero4();
        const int a0 = out_ptr[i], a1 = out_ptr[i + 1];
        if (out_list) {
            for (int a = a0; a < a1; a++) so += P::load4(e + (int64_t)out_list[a] * H + c);
        } else {
            int a = a0;
            for (; a + 4 <= a1; a += 4) {
                const f32x4 v0 = P::load4(e + (int64_t)a * H + c);
                const f32x4 v1 = P::load4(e + (int64_t)(a + 1) * H + c);
                const f32x4 v2 = P::load4(e + (int64_t)(a + 2) * H + c);
                const f32x4 v3 = P::load4(e + (int64_t)(a + 3) * H + c);
                so += v0; so += v1; so += v2; so += v3;
            }
            for (; a < a1; a++) so += P::load4(e + (int64_t)a * H + c);
        }
        const int b0 = in_ptr[i], b1 = in_ptr[i + 1];
        int b = b0;
        for (; b + 4 <= b1; b += 4) {
            const int q0 = in_list[b], q1 = in_list[b + 1], q2 = in_list[b + 2], q3 = in_list[b + 3];
            const f32x4 v0 = P::load4(e + (int64_t)q0 * H + c);
            const f32x4 v1 = P::load4(e + (int64_t)q1 * H + c);
            const f32x4 v2 = P::load4(e + (int64_t)q2 * H + c);
            const f32x4 v3 = P::load4(e + (int64_t)q3 * H + c);
            si += v0; si += v1; si += v2; si += v3;
        }
        for (; b < b1; b++) si += P::load4(e + (int64_t)in_list[b] * H + c);
        *(f32x4 *)(m + i * 2 * H + c) = so;
        *(f32x4 *)(m + i * 2 * H + H + c) = si;
    }
}

constexpr int kMlpBlock = 512;

// Blocks of `block` threads with `lds` bytes of LDS that fit on one compute
// unit together (at least 1); also lifts the dynamic-LDS launch limit.
inline int blocks_per_cu(const void *kernel, int block, size_t lds) {
    hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, block, lds) != hipSuccess || n < 1) n = 1;
    return n;
}

template <class P, int H, int MODE, bool CLS>
void run_mlp(velo_ctx *c, const MlpArgs &a, hipStream_t s) {
    constexpr size_t lds = mlp_lds<P, H, MODE, CLS>();
    static const int per_cu = blocks_per_cu(reinterpret_cast<const void *>(&k_mlp<P, H, MODE, CLS>), kMlpBlock, lds);
    k_mlp<P, H, MODE, CLS><<<persistent_grid(c, per_cu), kMlpBlock, lds, s>>>(a);
}

template <class P, int H>
void gnn_ph(velo_ctx *c, const velo_hits *hits, bool out_identity, float *logit, hipStream_t s) {
    using S = typename P::state_t;
    Workspace &w = c->ws;
    const ParamLayout &L = c->layout;
    const float *Pw = c->params;
    const int64_t N = hits->n_hits, Ecap = c->cfg.max_edges;
    S *h[2] = {(S *)w.h[0], (S *)w.h[1]};
    S *e = (S *)w.e;
    // the classifier is fused into the last edge network when its weights fit in LDS too
    const bool fuse_cls = mlp_lds<P, H, EDGE, true>() <= c->lds_max;
    if (N > 0) {
        const size_t lds = frag_bytes<P>(H, H) + sizeof(float) * H * 4;
        static const int per_cu = blocks_per_cu(reinterpret_cast<const void *>(&k_node_enc<P, H>), kMlpBlock, lds);
        StageTimer t(c, VELO_STAGE_NODE_ENC, s);
        k_node_enc<P, H><<<persistent_grid(c, per_cu), kMlpBlock, lds, s>>>(N, hits->x, hits->y, hits->z, Pw,
                                                                      L.nenc[0].w, L.nenc[1].w, h[0], w.flags);
    }
    MlpArgs a{};
    a.n_dev = w.n_edges; a.n_host = Ecap; a.src_g = w.src_g; a.dst_g = w.dst_g;
    a.P = Pw; a.flags = w.flags; a.logit = logit;
    a.o_c1 = L.cls[0].w; a.o_c2 = L.cls[1].w;
    a.a = h[0]; a.out = e; a.o_w1 = L.eenc[0].w; a.o_w2 = L.eenc[1].w;
    const int iters = c->cfg.gnn_iters;
    {
        StageTimer t(c, VELO_STAGE_EDGE_ENC, s);
        run_mlp<P, H, EDGE_ENC, false>(c, a, s);
    }
    int cur = 0;
    const int *optr = out_identity ? w.row_ptr : w.out_ptr;
    const int *olist = out_identity ? nullptr : w.out_list;
    for (int k = 0; k < iters; k++) {
        if (N > 0) {
            StageTimer t(c, VELO_STAGE_MESSAGES, s);
            k_messages<P, H><<<persistent_grid(c, 16), 256, 0, s>>>(N, optr, olist, w.in_ptr, w.in_list, e, w.m,
                                                                  w.flags);
        }
        MlpArgs nd{};
        nd.n_dev = nullptr; nd.n_host = N; nd.a = h[cur]; nd.b = w.m; nd.out = h[cur ^ 1];
        nd.P = Pw; nd.o_w1 = L.node[k][0].w; nd.o_w2 = L.node[k][1].w; nd.flags = w.flags;
        if (N > 0) {
            StageTimer t(c, VELO_STAGE_NODE_NET, s);
            run_mlp<P, H, NODE, false>(c, nd, s);
        }
        cur ^= 1;
        MlpArgs ed = a;
        ed.a = e; ed.b = h[cur]; ed.out = e; ed.o_w1 = L.edge[k][0].w; ed.o_w2 = L.edge[k][1].w;
        const bool last = k == iters - 1;
        StageTimer t(c, last && fuse_cls ? VELO_STAGE_EDGE_CLS : VELO_STAGE_EDGE_NET, s);
        if (last && fuse_cls)
            run_mlp<P, H, EDGE, true>(c, ed, s);
        else
            run_mlp<P, H, EDGE, false>(c, ed, s);
    }
    if (iters == 0 || !fuse_cls) {
        MlpArgs cl = a;
        cl.a = e;
        StageTimer t(c, VELO_STAGE_EDGE_CLS, s);
        run_mlp<P, H, CLS_ONLY, true>(c, cl, s);
    }
}

template <class P>
void embed_p(velo_ctx *c, const velo_hits *h, float *emb, hipStream_t s) {
    const size_t lds = frag_bytes<P>(kCe, kCe) + frag_bytes<P>(16, kCe) + sizeof(float) * kCe * 4;
    static const int per_cu = blocks_per_cu(reinterpret_cast<const void *>(&k_embed<P>), kMlpBlock, lds);
    const ParamLayout &L = c->layout;
    k_embed<P><<<persistent_grid(c, per_cu), kMlpBlock, lds, s>>>(h->n_hits, h->x, h->y, h->z, c->params, L.emb[0].w,
                                                             L.emb[1].w, L.emb[2].w, emb, c->ws.flags);
}

}  // namespace

size_t state_bytes(int precision) { return precision == VELO_FP32 ? sizeof(float) : sizeof(uint16_t); }

bool gnn_supported(int hidden, int precision) {
    if (precision == VELO_FP32) return hidden == 32 || hidden == 64;
    if (precision == VELO_BF16) return hidden == 32 || hidden == 64 || hidden == 128;
    return false;
}

void launch_embed(velo_ctx *c, const velo_hits *h, float *emb, hipStream_t s) {
    if (h->n_hits <= 0) return;
    if (c->cfg.precision == VELO_FP32)
        embed_p<F32>(c, h, emb, s);
    else
        embed_p<BF16>(c, h, emb, s);
}

void launch_gnn(velo_ctx *c, const velo_hits *h, bool out_identity, float *logit, hipStream_t s) {
    const int H = c->cfg.gnn_hidden;
    if (c->cfg.precision == VELO_FP32) {
        if (H == 32) gnn_ph<F32, 32>(c, h, out_identity, logit, s);
        if (H == 64) gnn_ph<F32, 64>(c, h, out_identity, logit, s);
    } else {
        if (H == 32) gnn_ph<BF16, 32>(c, h, out_identity, logit, s);
        if (H == 64) gnn_ph<BF16, 64>(c, h, out_identity, logit, s);
        if (H == 128) gnn_ph<BF16, 128>(c, h, out_identity, logit, s);
    }
}

}  // namespace velo
