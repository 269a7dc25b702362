// mfma.h -- device building blocks shared by the MFMA kernels (internal).
//
// See gnn.hip for the fragment layout.  Precision traits F32 and BF16 define
// how a lane loads, converts, multiplies and stores its fragments; stage()
// copies a weight matrix into LDS in fragment order; gemm() walks the K
// blocks of one layer.
#pragma once

#include "internal.h"

namespace velo {
namespace mfma {

typedef __bf16 bf16;
typedef bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ inline f32x4 zero4() { return f32x4{0.f, 0.f, 0.f, 0.f}; }

// ------------------------------------------------------------------------
// precision traits
// ------------------------------------------------------------------------
struct F32 {
    static constexpr bool kScaled = false;
    static constexpr bool kSplit = false;
    static constexpr bool kPrefetchW = true;   // matrix-core-bound: prefetch weight fragments
    using state_t = float;       // hit/edge encodings in HBM
    using frag_t = f32x4;        // per-lane B operand of one K block
    using wfrag_t = f32x4;       // per-lane A operand of one (output block, K block)
    static constexpr int KBLK = 16;
    static constexpr int WJ = 4;
    __device__ static int col(int kb, int g, int j) { return 16 * kb + 4 * g + j; }
    __device__ static float wconv(float v) { return v; }
    __device__ static frag_t load(const float *row, int kb, int g) { return *(const f32x4 *)(row + 16 * kb + 4 * g); }
    __device__ static frag_t load_f32(const float *row, int kb, int g) { return load(row, kb, g); }
    __device__ static frag_t load(const float *row, int kb, int g, float) { return load(row, kb, g); }
    __device__ static frag_t load_f32(const float *row, int kb, int g, float) { return load(row, kb, g); }
    template <int MO>
    __device__ static void chain(const f32x4 *h, frag_t *x, float) { chain<MO>(h, x); }
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
    // store_all where ok; o becomes the stored values (0 where not ok)
    template <int MO>
    __device__ static void store_round(float *row, int g, f32x4 *o, bool ok) {
        if (ok) store_all<MO>(row, g, o);
#pragma unroll
        for (int mo = 0; mo < MO; mo++)
#pragma unroll
            for (int i = 0; i < 4; i++) o[mo][i] = ok ? o[mo][i] : 0.f;
    }
    __device__ static f32x4 load4(const float *p) { return *(const f32x4 *)p; }
    __device__ static float absmax(const frag_t &f) {
        return fmaxf(fmaxf(fabsf(f[0]), fabsf(f[1])), fmaxf(fabsf(f[2]), fabsf(f[3])));
    }
};

struct BF16 {
    static constexpr bool kScaled = false;
    static constexpr bool kSplit = false;
    static constexpr bool kPrefetchW = false;
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
    __device__ static frag_t load(const bf16 *row, int kb, int g, float) { return load(row, kb, g); }
    __device__ static frag_t load_f32(const float *row, int kb, int g, float) { return load_f32(row, kb, g); }
    template <int MO>
    __device__ static void chain(const f32x4 *h, frag_t *x, float) { chain<MO>(h, x); }
    __device__ static int stored(int mo, int g) { return 32 * (mo >> 1) + 8 * g + 4 * (mo & 1); }
    template <int MO>
    __device__ static void store_all(bf16 *row, int g, const f32x4 *o) {
#pragma unroll
        for (int kb = 0; kb < MO / 2; kb++) *(bf16x8 *)(row + 32 * kb + 8 * g) = cat(cvt(o[2 * kb]), cvt(o[2 * kb + 1]));
    }
    // store_all where ok; o becomes the stored (rounded) values, 0 where not
    // ok: each value is rounded once, for the store and for the caller
    template <int MO>
    __device__ static void store_round(bf16 *row, int g, f32x4 *o, bool ok) {
#pragma unroll
        for (int kb = 0; kb < MO / 2; kb++) {
            const bf16x8 v = cat(cvt(o[2 * kb]), cvt(o[2 * kb + 1]));
            if (ok) *(bf16x8 *)(row + 32 * kb + 8 * g) = v;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                o[2 * kb][j] = ok ? (float)v[j] : 0.f;
                o[2 * kb + 1][j] = ok ? (float)v[4 + j] : 0.f;
            }
        }
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
    __device__ static float absmax(const frag_t &f) {
        float m = 0.f;
#pragma unroll
        for (int j = 0; j < 8; j++) m = fmaxf(m, fabsf((float)f[j]));
        return m;
    }
};

// BF16X2: bf16 weights; an activation that is not already a bf16 value
// (hidden layers, message sums, the final edge state entering the
// classifier) enters as two bf16 operands, v = hi + lo with hi = bf16(v) and
// lo = bf16(v - hi) (v - hi is exact in float32), and two MFMA products per
// block, W lo + W hi, so products keep the weight's bf16 rounding but not the
// activation's (about 2^-16 of it remains).  Operands read from stored
// encodings are bf16 already: gemm<..., true> gives them the single product
// W hi (their lo is 0).  Same fragment layout, weight fragments and stored
// (bf16, permuted) encodings as BF16.
struct bf16x8x2 {
    bf16x8 hi, lo;
};
struct BF16X2 {
    static constexpr bool kScaled = false;
    static constexpr bool kSplit = true;
    static constexpr bool kPrefetchW = false;
    using state_t = bf16;
    using frag_t = bf16x8x2;
    using wfrag_t = bf16x8;
    static constexpr int KBLK = 32;
    static constexpr int WJ = 8;
    __device__ static int col(int kb, int g, int j) { return BF16::col(kb, g, j); }
    __device__ static bf16x4 rest(f32x4 v, bf16x4 h) {
        return bf16x4{(bf16)(v[0] - (float)h[0]), (bf16)(v[1] - (float)h[1]), (bf16)(v[2] - (float)h[2]),
                      (bf16)(v[3] - (float)h[3])};
    }
    __device__ static frag_t split(f32x4 a, f32x4 b) {
        const bf16x4 ha = BF16::cvt(a), hb = BF16::cvt(b);
        return frag_t{BF16::cat(ha, hb), BF16::cat(rest(a, ha), rest(b, hb))};
    }
    __device__ static frag_t load(const bf16 *row, int kb, int g, float = 1.f) {
        return frag_t{BF16::load(row, kb, g), bf16x8{}};
    }
    __device__ static frag_t load_f32(const float *row, int kb, int g, float = 1.f) {
        return split(*(const f32x4 *)(row + 32 * kb + 8 * g), *(const f32x4 *)(row + 32 * kb + 8 * g + 4));
    }
    template <int MO>
    __device__ static void chain(const f32x4 *h, frag_t *x, float = 1.f) {
#pragma unroll
        for (int kb = 0; kb < MO / 2; kb++) x[kb] = split(h[2 * kb], h[2 * kb + 1]);
    }
    template <int MO>
    __device__ static void mma(const wfrag_t *a, const frag_t &x, f32x4 *acc) {
#pragma unroll
        for (int mo = 0; mo < MO; mo++) {
            acc[mo] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mo], x.lo, acc[mo], 0, 0, 0);
            acc[mo] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mo], x.hi, acc[mo], 0, 0, 0);
        }
    }
    // operands whose lo is 0 (read from stored encodings)
    template <int MO>
    __device__ static void mma_hi(const wfrag_t *a, const frag_t &x, f32x4 *acc) {
#pragma unroll
        for (int mo = 0; mo < MO; mo++) acc[mo] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mo], x.hi, acc[mo], 0, 0, 0);
    }
    __device__ static float seg0(const frag_t *x, int mo, int i) {
        const int j = 4 * (mo & 1) + i;
        return (float)x[mo >> 1].hi[j] + (float)x[mo >> 1].lo[j];
    }
    __device__ static int stored(int mo, int g) { return BF16::stored(mo, g); }
    template <int MO>
    __device__ static void store_all(bf16 *row, int g, const f32x4 *o) { BF16::store_all<MO>(row, g, o); }
    template <int MO>
    __device__ static void store_round(bf16 *row, int g, f32x4 *o, bool ok) { BF16::store_round<MO>(row, g, o, ok); }
    __device__ static f32x4 load4(const bf16 *p) { return BF16::load4(p); }
    __device__ static float absmax(const frag_t &f) { return BF16::absmax(f.hi); }
};

// FP8: OCP E4M3 matrix operands (v_mfma_f32_16x16x32_fp8_fp8, same fragment
// layout as bf16) with static per-tensor scales: an operand v is fed as
// e4m3(v / s) and every product is descaled by s_x * s_w after the MFMAs.
// Encodings stay stored in the permuted bf16 layout.
struct FP8 {
    static constexpr bool kScaled = true;
    static constexpr bool kSplit = false;
    static constexpr bool kPrefetchW = false;
    using state_t = bf16;
    using frag_t = long;         // 8 e4m3 values
    using wfrag_t = long;
    static constexpr int KBLK = 32;
    static constexpr int WJ = 8;
    __device__ static int col(int kb, int g, int j) { return BF16::col(kb, g, j); }
    __device__ static long pack8(f32x4 lo, f32x4 hi, float inv) {
        int a = 0, b = 0;
        a = __builtin_amdgcn_cvt_pk_fp8_f32(lo[0] * inv, lo[1] * inv, a, false);
        a = __builtin_amdgcn_cvt_pk_fp8_f32(lo[2] * inv, lo[3] * inv, a, true);
        b = __builtin_amdgcn_cvt_pk_fp8_f32(hi[0] * inv, hi[1] * inv, b, false);
        b = __builtin_amdgcn_cvt_pk_fp8_f32(hi[2] * inv, hi[3] * inv, b, true);
        return (long)(((unsigned long)(unsigned)b << 32) | (unsigned)a);
    }
    __device__ static f32x4 lo4(bf16x8 v) { return f32x4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]}; }
    __device__ static f32x4 hi4(bf16x8 v) { return f32x4{(float)v[4], (float)v[5], (float)v[6], (float)v[7]}; }
    __device__ static frag_t pack(bf16x8 v, float inv) { return pack8(lo4(v), hi4(v), inv); }
    __device__ static frag_t load(const bf16 *row, int kb, int g, float inv) {
        return pack(BF16::load(row, kb, g), inv);
    }
    __device__ static frag_t load_f32(const float *row, int kb, int g, float inv) {
        return pack8(*(const f32x4 *)(row + 32 * kb + 8 * g), *(const f32x4 *)(row + 32 * kb + 8 * g + 4), inv);
    }
    template <int MO>
    __device__ static void mma(const wfrag_t *a, const frag_t &x, f32x4 *acc) {
#pragma unroll
        for (int mo = 0; mo < MO; mo++)
            acc[mo] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a[mo], x, acc[mo], 0, 0, 0);
    }
    template <int MO>
    __device__ static void chain(const f32x4 *h, frag_t *x, float inv) {
#pragma unroll
        for (int kb = 0; kb < MO / 2; kb++) x[kb] = pack8(h[2 * kb], h[2 * kb + 1], inv);
    }
    __device__ static int stored(int mo, int g) { return BF16::stored(mo, g); }
    template <int MO>
    __device__ static void store_all(bf16 *row, int g, const f32x4 *o) { BF16::store_all<MO>(row, g, o); }
    template <int MO>
    __device__ static void store_round(bf16 *row, int g, f32x4 *o, bool ok) { BF16::store_round<MO>(row, g, o, ok); }
    __device__ static f32x4 load4(const bf16 *p) { return BF16::load4(p); }
    __device__ static float absmax(const frag_t &) { return 0.f; }
};

// I8: symmetric INT8 matrix operands (v_mfma_i32_16x16x64_i8) with static
// per-tensor scales, for the embedding MLP (Sec. 7.4 quantises the embedding
// to INT8).  An operand v is fed as the code q = clamp(rint(fl32(v * (1/s))),
// -127, 127) (ties to even); each 64-wide K block's integer sums (at most
// 64 * 127^2 in magnitude) are added to float32 accumulators, which stays
// exact while |sum| < 2^24 (K <= 1024), and the accumulators are descaled by
// s_x * s_w after the last block.  Lane group g owns channels
// 64 kb + 16 q + 4 g + (0..3), q = 0..3: the accumulators of output blocks
// 4 kb + q chain into the next layer's operand without moving.
typedef int i32x4 __attribute__((ext_vector_type(4)));
struct I8 {
    static constexpr bool kScaled = true;
    static constexpr bool kSplit = false;
    static constexpr bool kPrefetchW = false;
    using state_t = float;
    using frag_t = i32x4;        // 16 int8 codes
    using wfrag_t = i32x4;
    static constexpr int KBLK = 64;
    static constexpr int WJ = 16;
    __device__ static int col(int kb, int g, int j) { return 64 * kb + 16 * (j >> 2) + 4 * g + (j & 3); }
    __device__ static int code(float v, float inv) {
        const float t = __builtin_rintf(v * inv);
        return (int)fminf(fmaxf(t, -127.f), 127.f);
    }
    __device__ static int pack4(f32x4 v, float inv) {
        return (code(v[0], inv) & 0xff) | ((code(v[1], inv) & 0xff) << 8) | ((code(v[2], inv) & 0xff) << 16) |
               ((unsigned)code(v[3], inv) << 24);
    }
    template <int MO>
    __device__ static void mma(const wfrag_t *a, const frag_t &x, f32x4 *acc) {
#pragma unroll
        for (int mo = 0; mo < MO; mo++) {
            const i32x4 t = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[mo], x, i32x4{0, 0, 0, 0}, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; i++) acc[mo][i] += (float)t[i];
        }
    }
    template <int MO>
    __device__ static void chain(const f32x4 *h, frag_t *x, float inv) {
#pragma unroll
        for (int kb = 0; kb < MO / 4; kb++)
            x[kb] = i32x4{pack4(h[4 * kb], inv), pack4(h[4 * kb + 1], inv), pack4(h[4 * kb + 2], inv),
                          pack4(h[4 * kb + 3], inv)};
    }
};

// Weight staging converts every element with a scale: fp8 stores e4m3(w / s_w).
template <class P>
__device__ inline typename P::wfrag_t pack_weights(const float *w, float inv);

// Stage a row-major [rows x K] float32 weight into LDS in fragment order:
// entry (mo, kb, lane) holds W[16 mo + (lane & 15)][col(kb, lane >> 4, j)],
// rows >= `rows` (padding up to 16*MO) are zero.  With TRANS the staged
// matrix is W^T, read from a row-major W of shape [K x rows].
template <class P, bool TRANS = false>
__device__ inline void stage(typename P::wfrag_t *dst, const float *__restrict__ W, int rows, int K, int MO,
                             float inv_scale = 1.f, int ld = 0) {
    // row stride of W (a column block of a wider matrix has a larger one)
    if (ld == 0) ld = TRANS ? rows : K;
    const int KBn = K / P::KBLK;
    const int total = MO * KBn * 64;
    for (int f = threadIdx.x; f < total; f += blockDim.x) {
        const int lane = f & 63, mk = f >> 6, kb = mk % KBn, mo = mk / KBn;
        const int row = 16 * mo + (lane & 15), g = lane >> 4;
        float w[P::WJ];
#pragma unroll
        for (int j = 0; j < P::WJ; j++) {
            const int col = P::col(kb, g, j);
            w[j] = row < rows ? (TRANS ? W[(int64_t)col * ld + row] : W[(int64_t)row * ld + col]) : 0.f;
        }
        dst[f] = pack_weights<P>(w, inv_scale);
    }
}

template <>
__device__ inline f32x4 pack_weights<F32>(const float *w, float) {
    return f32x4{w[0], w[1], w[2], w[3]};
}
template <>
__device__ inline bf16x8 pack_weights<BF16>(const float *w, float) {
    return bf16x8{(bf16)w[0], (bf16)w[1], (bf16)w[2], (bf16)w[3], (bf16)w[4], (bf16)w[5], (bf16)w[6], (bf16)w[7]};
}
template <>
__device__ inline bf16x8 pack_weights<BF16X2>(const float *w, float inv) {
    return pack_weights<BF16>(w, inv);
}
template <>
__device__ inline long pack_weights<FP8>(const float *w, float inv) {
    return FP8::pack8(f32x4{w[0], w[1], w[2], w[3]}, f32x4{w[4], w[5], w[6], w[7]}, inv);
}

template <>
__device__ inline i32x4 pack_weights<I8>(const float *w, float inv) {
    return i32x4{I8::pack4(f32x4{w[0], w[1], w[2], w[3]}, inv), I8::pack4(f32x4{w[4], w[5], w[6], w[7]}, inv),
                 I8::pack4(f32x4{w[8], w[9], w[10], w[11]}, inv), I8::pack4(f32x4{w[12], w[13], w[14], w[15]}, inv)};
}

template <class P>
constexpr size_t frag_bytes(int rows_pad, int K) {
    return (size_t)rows_pad * K * sizeof(typename P::wfrag_t) / P::WJ;
}

// acc[mo] += W[16 mo .., K] * X   (KB = K / KBLK blocks; K blocks
// [KB0, KB1) of it).  STATE: the operands were read from stored encodings
// (for split traits their lo part is 0 and is not multiplied).  AG: weight
// fragments held at a time (MO: a whole K block; fewer: fewer registers);
// every accumulator takes the same products in the same order either way.
template <class P, int MO, int KB, int KB0 = 0, int KB1 = KB, bool STATE = false, int AG = MO>
__device__ inline void gemm(const typename P::wfrag_t *sW, const typename P::frag_t *X, f32x4 *acc, int lane) {
    static_assert(MO % AG == 0, "fragment groups divide the output blocks");
    if constexpr (P::kPrefetchW) {
        // matrix-core-bound traits: the next group's weight fragments are
        // read from LDS while this group's products run (two groups live)
        constexpr int NGM = MO / AG, NG = (KB1 - KB0) * NGM;
        typename P::wfrag_t a[2][AG];
#pragma unroll
        for (int mo = 0; mo < AG; mo++) a[0][mo] = sW[(mo * KB + KB0) * 64 + lane];
#pragma unroll
        for (int gi = 0; gi < NG; gi++) {
            const int kb = KB0 + gi / NGM, m0 = (gi % NGM) * AG;
            __builtin_amdgcn_sched_barrier(0);
            if (gi + 1 < NG) {
                const int kn = KB0 + (gi + 1) / NGM, mn = ((gi + 1) % NGM) * AG;
#pragma unroll
                for (int mo = 0; mo < AG; mo++) a[(gi + 1) & 1][mo] = sW[((mn + mo) * KB + kn) * 64 + lane];
            }
            if constexpr (STATE && P::kSplit)
                P::template mma_hi<AG>(a[gi & 1], X[kb], acc + m0);
            else
                P::template mma<AG>(a[gi & 1], X[kb], acc + m0);
        }
    } else {
#pragma unroll
        for (int kb = KB0; kb < KB1; kb++) {
#pragma unroll
            for (int m0 = 0; m0 < MO; m0 += AG) {
                // keep one group of weight fragments live at a time
                __builtin_amdgcn_sched_barrier(0);
                typename P::wfrag_t a[AG];
#pragma unroll
                for (int mo = 0; mo < AG; mo++) a[mo] = sW[((m0 + mo) * KB + kb) * 64 + lane];
                if constexpr (STATE && P::kSplit)
                    P::template mma_hi<AG>(a, X[kb], acc + m0);
                else
                    P::template mma<AG>(a, X[kb], acc + m0);
            }
        }
    }
}

template <int MO>
__device__ inline void load_bias(const float *__restrict__ b, f32x4 *rb, int g) {
#pragma unroll
    for (int mo = 0; mo < MO; mo++) rb[mo] = *(const f32x4 *)(b + 16 * mo + 4 * g);
}

// max(x, 0) as one integer max on the bit pattern: a float with its sign
// bit set is a negative int32 and becomes +0, any other keeps its value (a
// float max would first canonicalise a matrix-core result: two instructions)
__device__ inline float relu1(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

template <int MO>
__device__ inline void relu(f32x4 *acc) {
#pragma unroll
    for (int mo = 0; mo < MO; mo++)
#pragma unroll
        for (int i = 0; i < 4; i++) acc[mo][i] = relu1(acc[mo][i]);
}

template <int MO>
__device__ inline void bias_relu(f32x4 *acc, const f32x4 *rb) {
#pragma unroll
    for (int mo = 0; mo < MO; mo++)
#pragma unroll
        for (int i = 0; i < 4; i++) acc[mo][i] = relu1(acc[mo][i] + rb[mo][i]);
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


// Static per-tensor scales of one two-layer MLP (fp8): sc = {s_x1, s_w1,
// s_x2, s_w2} for the inputs and weights of its two layers.  Operands are fed
// as v / s and the accumulators rescaled by s_x * s_w.  Null: all ones.
struct MlpScales {
    float ix1 = 1.f, iw1 = 1.f, d1 = 1.f, ix2 = 1.f, iw2 = 1.f, d2 = 1.f;
};

__device__ inline MlpScales read_scales(const float *sc) {
    MlpScales r;
    if (sc) {
        r.ix1 = 1.f / sc[0];
        r.iw1 = 1.f / sc[1];
        r.d1 = sc[0] * sc[1];
        r.ix2 = 1.f / sc[2];
        r.iw2 = 1.f / sc[3];
        r.d2 = sc[2] * sc[3];
    }
    return r;
}

template <int MO>
__device__ inline void rescale(f32x4 *acc, float d) {
#pragma unroll
    for (int mo = 0; mo < MO; mo++) acc[mo] *= d;
}

template <int MO>
__device__ inline float absmax4(const f32x4 *v) {
    float m = 0.f;
#pragma unroll
    for (int mo = 0; mo < MO; mo++)
#pragma unroll
        for (int i = 0; i < 4; i++) m = fmaxf(m, fabsf(v[mo][i]));
    return m;
}

// Calibration: largest |value| seen by the wavefront, kept as float bits
// (non-negative floats order like unsigned integers, so the max is exact and
// independent of the order of the atomics).
__device__ inline void record_amax(float m, float *slot) {
    for (int d = 32; d >= 1; d >>= 1) m = fmaxf(m, __shfl_xor(m, d));
    if ((threadIdx.x & 63) == 0) atomicMax((unsigned *)slot, __float_as_uint(m));
}

}  // namespace mfma
}  // namespace velo
