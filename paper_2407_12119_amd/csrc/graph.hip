// graph.hip -- batch validation, plane bucketing and the rough hit graph.
//
// Rough graph (paper Sec. 5.1 and Sec. 7.2): a hit on plane p is joined to
// hits on planes p+1 and p+2 whose squared embedding distance is below
// d2_max, keeping at most k_max per hit.  Hits are sorted by plane inside each
// event, so the candidates of a hit on plane p are one contiguous index range.
//
// Work mapping: a 64-lane wavefront takes a run of consecutive query hits,
// one hit at a time.  The lanes hold the candidate range in chunks of 64 (up
// to kKeyChunks chunks of embeddings stay in registers while the queries
// share their event and plane), compute the float32 distance keys, and find
// the exact k_max smallest under (d2, index) by a search on the float bit
// pattern of d2 driven by wave ballots (no sorting, no scratch memory); the
// survivors are written in index order through ballot prefix counts.  This
// parallelises over the candidates of a hit as well as over hits.
#include "internal.h"

namespace velo {

namespace {

constexpr int kKeyChunks = 8;             // candidates cached in registers: 8 x 64
constexpr unsigned kInvalidKey = 0xffffffffu;

__device__ inline unsigned long long ballot(bool p) { return __ballot(p); }
__device__ inline int lanes_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// ------------------------------------------------------------------------
// validation and plane offsets: one block per event
// ------------------------------------------------------------------------
__global__ void k_prepare(int B, int64_t n_hits, const int *__restrict__ off,
                          const float *__restrict__ x, const float *__restrict__ y,
                          const float *__restrict__ z, const int *__restrict__ plane,
                          int max_event_hits, int *__restrict__ plane_off,
                          int *__restrict__ hit_event, unsigned *__restrict__ flags) {
    const int b = blockIdx.x;
    const int s = off[b], e = off[b + 1];
    bool bad = (b == 0 && s != 0) || (b == B - 1 && (int64_t)e != n_hits) || e < s ||
               s < 0 || (int64_t)e > n_hits || (e - s) > max_event_hits;
    int *po = plane_off + (int64_t)b * kPlaneSlots;
    if (bad) {
        if (threadIdx.x == 0) atomicOr(flags, kErrInput);
        for (int q = threadIdx.x; q < kPlaneSlots; q += blockDim.x) po[q] = 0;
        return;
    }
    const int n = e - s;
    if (n == 0) {
        for (int q = threadIdx.x; q < kPlaneSlots; q += blockDim.x) po[q] = 0;
        return;
    }
    bool err = false;
    for (int l = threadIdx.x; l < n; l += blockDim.x) {
        const int64_t i = (int64_t)s + l;
        const int p = plane[i];
        const int pp = l == 0 ? -1 : plane[i - 1];
        if (p < 0 || p >= VELO_N_PLANES || pp > p || !isfinite(x[i]) || !isfinite(y[i]) ||
            !isfinite(z[i]))
            err = true;
        hit_event[i] = b;
        const int lo = max(pp + 1, 0), hi = min(p, VELO_N_PLANES);
        for (int q = lo; q <= hi; q++) po[q] = l;
        if (l == n - 1)
            for (int q = max(p + 1, 0); q < kPlaneSlots; q++) po[q] = n;
    }
    if (err) atomicOr(flags, kErrInput);
}

// ------------------------------------------------------------------------
// neighbour search
// ------------------------------------------------------------------------

// Float32 squared distance with the evaluation order fixed by the ABI:
// s = d0*d0, then s = fma(d_c, d_c, s).
__device__ inline float dist2(f32x4 a, f32x4 b) {
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

__device__ inline unsigned cand_key(const f32x4 *__restrict__ emb, int64_t base, int C, int c,
                                    f32x4 q, float d2max) {
    if (c >= C) return kInvalidKey;
    const float s = dist2(q, emb[base + c]);
    return s < d2max ? __float_as_uint(s) : kInvalidKey;
}

// A wavefront task is a run of RUN consecutive query hits (8, 16 or 32;
// velo_autotune picks one): longer runs reuse the candidate embeddings held
// in registers over more queries, shorter ones balance uneven planes better.
constexpr int kKnnRunDefault = 16;
constexpr int kKnnBlock = 256;
constexpr int kHistBins = 256;   // key histogram of one query: four bins per lane

// Cross-lane steps on DPP (no LDS round trip).  All 64 lanes must be active.
template <int CTRL>
__device__ inline unsigned dpp_u32(unsigned v) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, true);
}
// smallest / largest value over the wavefront (every row of 16 lanes is
// reduced by a quad swap, a quad rotation, the half-row mirror and the row
// mirror, then the four rows through scalar registers)
__device__ inline unsigned wave_min_u32(unsigned v) {
    v = min(v, dpp_u32<0xB1>(v));    // quad_perm [1,0,3,2]
    v = min(v, dpp_u32<0x4E>(v));    // quad_perm [2,3,0,1]
    v = min(v, dpp_u32<0x141>(v));   // row_half_mirror
    v = min(v, dpp_u32<0x140>(v));   // row_mirror
    return min(min((unsigned)__builtin_amdgcn_readlane((int)v, 0), (unsigned)__builtin_amdgcn_readlane((int)v, 16)),
               min((unsigned)__builtin_amdgcn_readlane((int)v, 32), (unsigned)__builtin_amdgcn_readlane((int)v, 48)));
}
__device__ inline unsigned wave_max_u32(unsigned v) {
    v = max(v, dpp_u32<0xB1>(v));
    v = max(v, dpp_u32<0x4E>(v));
    v = max(v, dpp_u32<0x141>(v));
    v = max(v, dpp_u32<0x140>(v));
    return max(max((unsigned)__builtin_amdgcn_readlane((int)v, 0), (unsigned)__builtin_amdgcn_readlane((int)v, 16)),
               max((unsigned)__builtin_amdgcn_readlane((int)v, 32), (unsigned)__builtin_amdgcn_readlane((int)v, 48)));
}
// inclusive prefix sum over the lanes: row shifts by 1, 2, 4, 8 (lanes
// shifted in from outside the row read 0), then the totals of earlier rows
__device__ inline int wave_incl_scan(int v, int lane) {
    v += (int)dpp_u32<0x111>((unsigned)v);   // row_shr:1
    v += (int)dpp_u32<0x112>((unsigned)v);   // row_shr:2
    v += (int)dpp_u32<0x114>((unsigned)v);   // row_shr:4
    v += (int)dpp_u32<0x118>((unsigned)v);   // row_shr:8
    const int r0 = __builtin_amdgcn_readlane(v, 15), r1 = __builtin_amdgcn_readlane(v, 31),
              r2 = __builtin_amdgcn_readlane(v, 47);
    return v + (lane >= 16 ? r0 : 0) + (lane >= 32 ? r1 : 0) + (lane >= 48 ? r2 : 0);
}

// Orders one wavefront's LDS accesses (all lanes) before its next ones.
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <int RUN>
__global__ __launch_bounds__(kKnnBlock) void k_knn(int64_t n_hits, const int *__restrict__ off,
                                             const int *__restrict__ plane_off,
                                             const int *__restrict__ hit_event,
                                             const int *__restrict__ plane,
                                             const f32x4 *__restrict__ emb, float d2max, int kmax,
                                             int *__restrict__ nbr, int *__restrict__ deg, int xcd,
                                             const unsigned *__restrict__ flags) {
    __shared__ __align__(16) int hist_sh[kKnnBlock / 64][kHistBins];
    if (*flags & kErrInput) return;
    const int lane = threadIdx.x & 63;
    // per-hit bookkeeping is wave-uniform: scalar loads
    const_as<int> *hit_event4 = (const_as<int> *)hit_event;
    const_as<int> *plane4 = (const_as<int> *)plane;
    const_as<int> *off4 = (const_as<int> *)off;
    const_as<int> *plane_off4 = (const_as<int> *)plane_off;
    const_as<f32x4> *emb4 = (const_as<f32x4> *)emb;
    const int64_t n_runs = (n_hits + RUN - 1) / RUN;
    const WaveRange wv = wave_range(n_runs, xcd != 0);
    const WaveRange wr{uniform64(wv.first), uniform64(wv.step), uniform64(wv.end)};
    for (int64_t r = wr.first; r < wr.end; r += wr.step) {
        // Hits are sorted by (event, plane), so consecutive queries mostly share
        // their candidate range: its first kKeyChunks chunks of embeddings stay
        // in registers until the (event, plane) changes.
        int cb = -1, cp = -1;
        int c0 = 0, C = 0, nch = 0;
        int64_t base = 0;
        f32x4 cand[kKeyChunks];
        const int64_t i_end = min(r * RUN + RUN, n_hits);
        for (int64_t i = r * RUN; i < i_end; i++) {
            const int b = hit_event4[i], p = plane4[i];
            if (b != cb || p != cp) {
                cb = b;
                cp = p;
                const_as<int> *po = plane_off4 + (int64_t)b * kPlaneSlots;
                c0 = po[min(p + 1, VELO_N_PLANES)];
                C = max(po[min(p + 3, VELO_N_PLANES)] - c0, 0);
                base = (int64_t)off4[b] + c0;     // batch index of candidate 0
                nch = (C + 63) >> 6;
#pragma unroll
                for (int c = 0; c < kKeyChunks; c++)
                    if (c < nch) {
                        const int j = c * 64 + lane;
                        cand[c] = j < C ? emb[base + j] : f32x4{0.f, 0.f, 0.f, 0.f};
                    }
            }
            const f32x4 q = emb4[i];
            int *out = nbr + i * kmax;

            unsigned key[kKeyChunks];
            int m = 0;
            unsigned kmin = kInvalidKey, khi = 0;   // smallest and largest valid key (lane-local)
#pragma unroll
            for (int c = 0; c < kKeyChunks; c++) {
                key[c] = kInvalidKey;
                if (c < nch) {
                    if (c * 64 + lane < C) {
                        const float s = dist2(q, cand[c]);
                        if (s < d2max) key[c] = __float_as_uint(s);
                    }
                    const bool v = key[c] != kInvalidKey;
                    m += __popcll(ballot(v));
                    if (v) {
                        kmin = min(kmin, key[c]);
                        khi = max(khi, key[c]);
                    }
                }
            }
            for (int c = kKeyChunks; c < nch; c++) {
                const unsigned k = cand_key(emb, base, C, c * 64 + lane, q, d2max);
                const bool v = k != kInvalidKey;
                m += __popcll(ballot(v));
                if (v) {
                    kmin = min(kmin, k);
                    khi = max(khi, k);
                }
            }
            // number of keys below x over all chunks (uniform over the wavefront)
            auto count_below = [&](unsigned x) {
                int cnt = 0;
#pragma unroll
                for (int c = 0; c < kKeyChunks; c++)
                    if (c < nch) cnt += __popcll(ballot(key[c] < x));
                for (int c = kKeyChunks; c < nch; c++)
                    cnt += __popcll(ballot(cand_key(emb, base, C, c * 64 + lane, q, d2max) < x));
                return cnt;
            };

            // threshold T: the kmax-th smallest key (only needed when m > kmax).
            // Search on the key bit pattern (monotone in the non-negative float
            // d2) between the smallest and largest valid key of one histogram
            // bin (below), keeping
            // cnt(< lo) < kmax < cnt(< hi): probes alternate between linear
            // interpolation of the counts (few probes on smooth key sets) and
            // bisection (a bound on the worst case).  A probe with exactly kmax
            // keys below it ends the search: those keys are the kmax smallest and
            // none ties with a dropped one.  Otherwise the search ends with
            // hi = lo + 1: lo is the kmax-th smallest key, and kmax - cnt(< lo)
            // of the keys equal to it are taken, in index order.
            unsigned T = 0x7fffffffu;
            int need_ties = 0;
            if (m > kmax) {
                kmin = wave_min_u32(kmin);
                khi = wave_max_u32(khi);
                // First narrow [kmin, khi] to one of kHistBins equal key
                // intervals: a histogram of the keys in this wave's LDS
                // slice, a prefix sum over the bins, and the bin holding the
                // kmax-th smallest key.  The bin index is a monotone function
                // of the key, so the keys below the bin are exactly those
                // below its smallest key.
                int *hist = hist_sh[threadIdx.x >> 6];
                reinterpret_cast<int4 *>(hist)[lane] = int4{0, 0, 0, 0};
                wave_lds_sync();
                const float scale = (float)kHistBins / (float)(khi - kmin + 1u);
                auto bin = [&](unsigned k) { return min((int)((float)(k - kmin) * scale), kHistBins - 1); };
                int kbin[kKeyChunks];
#pragma unroll
                for (int c = 0; c < kKeyChunks; c++) {
                    kbin[c] = -1;
                    if (c < nch && key[c] != kInvalidKey) {
                        kbin[c] = bin(key[c]);
                        atomicAdd(&hist[kbin[c]], 1);
                    }
                }
                for (int c = kKeyChunks; c < nch; c++) {
                    const unsigned k = cand_key(emb, base, C, c * 64 + lane, q, d2max);
                    if (k != kInvalidKey) atomicAdd(&hist[bin(k)], 1);
                }
                wave_lds_sync();
                const int4 h4 = reinterpret_cast<const int4 *>(hist)[lane];
                const int hs[4] = {h4.x, h4.y, h4.z, h4.w};
                const int own = hs[0] + hs[1] + hs[2] + hs[3];
                const int incl = wave_incl_scan(own, lane);
                // the lane whose four bins hold the kmax-th key (exactly one)
                int bsel = 0, below = incl - own, upto = incl;
                const bool here = below < kmax && kmax <= incl;
                if (here) {
#pragma unroll
                    for (int j = 0; j < 4; j++)
                        if (below + hs[j] >= kmax) {
                            bsel = 4 * lane + j;
                            upto = below + hs[j];
                            break;
                        } else {
                            below += hs[j];
                        }
                }
                const int src = __builtin_ctzll(ballot(here));
                const int bstar = __builtin_amdgcn_readlane(bsel, src);
                int clo = __builtin_amdgcn_readlane(below, src), chi = __builtin_amdgcn_readlane(upto, src);
                // the bin's smallest and largest key
                unsigned blo = kInvalidKey, bhi = 0;
#pragma unroll
                for (int c = 0; c < kKeyChunks; c++)
                    if (c < nch && kbin[c] == bstar) {
                        blo = min(blo, key[c]);
                        bhi = max(bhi, key[c]);
                    }
                for (int c = kKeyChunks; c < nch; c++) {
                    const unsigned k = cand_key(emb, base, C, c * 64 + lane, q, d2max);
                    if (k != kInvalidKey && bin(k) == bstar) {
                        blo = min(blo, k);
                        bhi = max(bhi, k);
                    }
                }
                blo = wave_min_u32(blo);
                bhi = wave_max_u32(bhi);
                unsigned lo = blo, hi = bhi + 1;    // cnt(< lo) = clo < kmax <= chi = cnt(< hi)
                bool exact = false;
                if (chi == kmax) {
                    T = hi;
                    exact = true;
                }
                for (int it = 0; !exact && hi - lo > 1; it++) {
                    const unsigned span = hi - lo;
                    unsigned step = span / 2;
                    if ((it & 1) == 0) {
                        const float f = ((float)(kmax - clo) + 0.5f) / (float)(chi - clo);
                        step = (unsigned)(f * (float)span);
                        step = min(max(step, 1u), span - 1);
                    }
                    const unsigned mid = lo + step;
                    const int cnt = count_below(mid);
                    if (cnt == kmax) {
                        T = mid;
                        exact = true;
                        break;
                    }
                    if (cnt < kmax) {
                        lo = mid;
                        clo = cnt;
                    } else {
                        hi = mid;
                        chi = cnt;
                    }
                }
                if (!exact) {
                    T = lo;
                    need_ties = kmax - clo;
                }
            }
            // emit survivors in candidate (= destination index) order
            int written = 0, ties_seen = 0;
            auto emit = [&](unsigned k, int c) {
                // with m <= kmax, T lies above every valid key and below kInvalidKey
                bool sel = k < T;
                if (need_ties > 0) {                  // uniform over the wavefront
                    const unsigned long long tie = ballot(k == T);
                    sel = sel || (k == T && ties_seen + lanes_below(tie) < need_ties);
                    ties_seen += __popcll(tie);
                }
                const unsigned long long sm = ballot(sel);
                const int slot = written + lanes_below(sm);
                if (sel && slot < kmax) out[slot] = c0 + c * 64 + lane;   // the row never overflows
                written += __popcll(sm);
            };
#pragma unroll
            for (int c = 0; c < kKeyChunks; c++)
                if (c < nch) emit(key[c], c);
            for (int c = kKeyChunks; c < nch; c++) emit(cand_key(emb, base, C, c * 64 + lane, q, d2max), c);
            if (lane == 0) deg[i] = min(written, kmax);
        }
    }
}

// ------------------------------------------------------------------------
// The paper's neighbour search (Sec. 7.2), kept as a comparison variant: one
// thread per query hit loops over the candidates in index order and keeps a
// list of at most kmax (d2, j); when the list is full, its largest entry is
// found and replaced by a closer candidate.  With candidates in increasing j
// and the largest entry under (d2, j) evicted, the list ends as the kmax
// smallest under (d2, j): the same selection as k_knn.  Lists live in LDS
// (kLoopBlock threads x kmax entries); the survivors are written in index
// order.
// ------------------------------------------------------------------------
constexpr int kLoopBlock = 64;
constexpr int kLoopMaxK = 64;

__global__ __launch_bounds__(kLoopBlock) void k_knn_loop(int64_t n_hits, const int *__restrict__ off,
                                                         const int *__restrict__ plane_off,
                                                         const int *__restrict__ hit_event,
                                                         const int *__restrict__ plane,
                                                         const f32x4 *__restrict__ emb, float d2max, int kmax,
                                                         int *__restrict__ nbr, int *__restrict__ deg,
                                                         const unsigned *__restrict__ flags) {
    __shared__ float ld[kLoopBlock][kLoopMaxK];
    __shared__ int lj[kLoopBlock][kLoopMaxK];
    if (*flags & kErrInput) return;
    float *dl = ld[threadIdx.x];
    int *jl = lj[threadIdx.x];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_hits; i += (int64_t)gridDim.x * blockDim.x) {
        const int b = hit_event[i];
        const int64_t s = off[b];
        const int p = plane[i];
        const int *po = plane_off + (int64_t)b * kPlaneSlots;
        const int c0 = po[min(p + 1, VELO_N_PLANES)];
        const int C = max(po[min(p + 3, VELO_N_PLANES)] - c0, 0);
        const f32x4 q = emb[i];
        int cnt = 0;
        for (int c = 0; c < C; c++) {
            const float d = dist2(q, emb[s + c0 + c]);
            if (!(d < d2max)) continue;
            if (cnt < kmax) {
                dl[cnt] = d;
                jl[cnt] = c0 + c;
                cnt++;
                continue;
            }
            int m = 0;   // the largest entry under (d2, j)
            for (int a = 1; a < kmax; a++)
                if (dl[a] > dl[m] || (dl[a] == dl[m] && jl[a] > jl[m])) m = a;
            if (d < dl[m]) {
                dl[m] = d;
                jl[m] = c0 + c;
            }
        }
        // index order (insertion sort of the short list)
        for (int a = 1; a < cnt; a++) {
            const int v = jl[a];
            int z = a - 1;
            while (z >= 0 && jl[z] > v) {
                jl[z + 1] = jl[z];
                z--;
            }
            jl[z + 1] = v;
        }
        int *out = nbr + i * kmax;
        for (int a = 0; a < cnt; a++) out[a] = jl[a];
        deg[i] = cnt;
    }
}

// ------------------------------------------------------------------------
// exclusive scan of int32 counts: out[0..n] with out[n] = total
// ------------------------------------------------------------------------
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

__device__ inline int block_exclusive_scan(int v, int *sh, int *total) {
    // sh: kScanBlock ints
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int d = 1; d < kScanBlock; d <<= 1) {
        int add = t >= d ? sh[t - d] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    const int incl = sh[t];
    *total = sh[kScanBlock - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const int *__restrict__ in, int64_t n,
                                                            int *__restrict__ sums) {
    __shared__ int sh[kScanBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int v = 0;
    for (int j = 0; j < kScanItems; j++) {
        const int64_t i = base + (int64_t)j * kScanBlock + threadIdx.x;
        if (i < n) v += in[i];
    }
    int total;
    block_exclusive_scan(v, sh, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_sums(int *__restrict__ sums, int nb,
                                                          int *__restrict__ out_total) {
    __shared__ int sh[kScanBlock];
    int carry = 0;
    for (int base = 0; base < nb; base += kScanBlock) {
        const int i = base + threadIdx.x;
        const int v = i < nb ? sums[i] : 0;
        int total;
        const int ex = block_exclusive_scan(v, sh, &total);
        if (i < nb) sums[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) *out_total = carry;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const int *__restrict__ in, int64_t n,
                                                           const int *__restrict__ sums,
                                                           int *__restrict__ out) {
    __shared__ int sh[kScanBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int local = 0;
    for (int j = 0; j < kScanItems; j++) {
        const int64_t i = base + j;
        v[j] = i < n ? in[i] : 0;
        local += v[j];
    }
    int total;
    int run = block_exclusive_scan(local, sh, &total) + sums[blockIdx.x];
    for (int j = 0; j < kScanItems; j++) {
        const int64_t i = base + j;
        if (i < n) out[i] = run;
        run += v[j];
    }
}

__global__ void k_fill(int *__restrict__ p, int v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ------------------------------------------------------------------------
// CSR compaction of the staged neighbour lists
// ------------------------------------------------------------------------
__global__ void k_compact(int64_t n_hits, int kmax, const int *__restrict__ off,
                          const int *__restrict__ hit_event, const int *__restrict__ deg,
                          const int *__restrict__ row_ptr, const int *__restrict__ nbr,
                          int64_t cap, int *__restrict__ esrc, int *__restrict__ edst,
                          int *__restrict__ src_g, int *__restrict__ dst_g,
                          const unsigned *__restrict__ flags) {
    if (*flags & kErrInput) return;
    const int64_t slots = n_hits * kmax;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < slots;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / kmax;
        const int a = (int)(t - i * kmax);
        if (a >= deg[i]) continue;
        const int64_t e = (int64_t)row_ptr[i] + a;
        if (e >= cap) continue;
        const int s = off[hit_event[i]];
        const int j = nbr[t];
        if (esrc) esrc[e] = (int)(i - s);
        if (edst) edst[e] = j;
        src_g[e] = (int)i;
        dst_g[e] = s + j;
    }
}

__global__ void k_edge_offsets(int B, const int *__restrict__ off, const int *__restrict__ row_ptr,
                               int *__restrict__ eoff, const unsigned *__restrict__ flags) {
    if (*flags & kErrInput) return;
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b <= B; b += gridDim.x * blockDim.x)
        eoff[b] = row_ptr[off[b]];
}

// n_internal = min(total, cap) is what every later kernel iterates over;
// n_out (the caller's count, may be null) receives the full total.
__global__ void k_check_capacity(const int *__restrict__ total, int64_t cap, int *__restrict__ n_internal,
                                 int *__restrict__ n_out, unsigned *__restrict__ flags) {
    const int t = *total;
    const bool over = t < 0 || (int64_t)t > cap;
    if (n_out) *n_out = t;
    *n_internal = over ? (t < 0 ? 0 : (int)cap) : t;
    if (over) atomicOr(flags, t < 0 ? kErrInput : kErrCapacity);
}

// Caller-supplied edges (event-local) -> batch-global hit indices; one block per event.
__global__ void k_globalise(int B, const int *__restrict__ off, const int *__restrict__ eoff,
                            const int *__restrict__ n_edges, int64_t cap, const int *__restrict__ esrc,
                            const int *__restrict__ edst, const int *__restrict__ plane, int *__restrict__ src_g,
                            int *__restrict__ dst_g, unsigned *__restrict__ flags) {
    if (*flags) return;
    const int E = min((int64_t)*n_edges, cap);
    if (B == 0) {           // no events: there can be no edges
        if (E != 0 && threadIdx.x == 0) atomicOr(flags, kErrInput);
        return;
    }
    // block (b, y): event b, the y-th of gridDim.y interleaved slices of its edges
    const int b = blockIdx.x;
    const int s = off[b], n = off[b + 1] - s;
    const int e0 = eoff[b], e1 = eoff[b + 1];
    // every block checks its own window: a negative or inverted offset of any
    // event must not index the edge arrays
    if ((b == 0 && e0 != 0) || (b == B - 1 && e1 != E) || e0 < 0 || e1 < e0 || e1 > E) {
        if (threadIdx.x == 0 && blockIdx.y == 0) atomicOr(flags, kErrInput);
        return;
    }
    bool err = false;
    const int stride = blockDim.x * gridDim.y;
    for (int q = e0 + blockIdx.y * blockDim.x + threadIdx.x; q < e1; q += stride) {
        const int a = esrc[q], c = edst[q];
        // edges must come grouped by source (non-decreasing esrc) and join a
        // hit to one on the next or the second next plane (Sec. 5.1)
        const int dp = (a >= 0 && a < n && c >= 0 && c < n) ? plane[s + c] - plane[s + a] : 0;
        if (a < 0 || a >= n || c < 0 || c >= n || (q > e0 && esrc[q - 1] > a) || dp < 1 || dp > 2) {
            err = true;
            if (src_g) {
                src_g[q] = s;
                dst_g[q] = s;
            }
            continue;
        }
        if (src_g) {        // null: validation only
            src_g[q] = s + a;
            dst_g[q] = s + c;
        }
    }
    if (err) atomicOr(flags, kErrInput);
}

// ------------------------------------------------------------------------
// incidence lists (edges grouped by hit), one workgroup per event:
// counts with LDS atomics, a block scan, a fill through LDS cursors, then
// every list is put in edge-id order (rank sort in registers, one wavefront
// per hit) so that sums over a list always run in the same order.
// ------------------------------------------------------------------------
// row pointers of a given graph whose edges come grouped by source
// (validated by k_globalise): row_ptr[i] = first edge of hit i, by binary
// search within the hit's event
// ------------------------------------------------------------------------
__global__ void k_row_ptr(int64_t n_hits, const int *__restrict__ hit_event, const int *__restrict__ eoff,
                          const int *__restrict__ n_edges, int64_t cap, const int *__restrict__ src_g,
                          int *__restrict__ row_ptr, const unsigned *__restrict__ flags) {
    if (*flags) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_hits;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int b = hit_event[i];
        int lo = eoff[b], hi = eoff[b + 1];
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (src_g[mid] < i) lo = mid + 1;
            else hi = mid;
        }
        row_ptr[i] = lo;
        if (i == n_hits - 1) row_ptr[n_hits] = (int)min((int64_t)*n_edges, cap);
    }
}

// ------------------------------------------------------------------------
// incoming lists, one workgroup per (event, destination plane q).  The
// in-edges of hits on plane q all leave from the CSR rows of planes q-2 and
// q-1, one contiguous edge window [E0, E1); an edge in it points below the
// plane (q-2 -> q-1), into it, or above it (q-1 -> q+1).  Hence the first
// incoming slot of the plane is E0 plus the edges of the window that point
// below it, and in_ptr needs no global scan.  Each wavefront takes one
// contiguous quarter of the window and counts its edges per destination in
// LDS; a block scan over destinations (and over the quarters of each
// destination) turns the counts into per-quarter cursors.  Every wavefront
// then walks its quarter in edge order, 64 edges at a time: lanes with the
// same destination find each other with one ballot per bit of the
// destination offset, take consecutive slots in lane order, and the lowest of
// them advances the cursor.  So every list comes out in edge-id order (a
// stable counting sort) with no atomics on global memory and no sorting.
// Planes with more than kListMaxDst hits are handled in slices of that size.
// ------------------------------------------------------------------------
constexpr int kListBlock = 256;
constexpr int kListWaves = kListBlock / 64;
constexpr int kListMaxDst = 2048;    // destinations of one slice held in LDS

__global__ __launch_bounds__(kListBlock) void k_in_lists(int64_t n_hits, const int *__restrict__ off,
                                                         const int *__restrict__ plane_off,
                                                         const int *__restrict__ row_ptr,
                                                         const int *__restrict__ dst_g, int *__restrict__ in_ptr,
                                                         int *__restrict__ in_list, const unsigned *__restrict__ flags) {
    __shared__ int cnt[kListWaves][kListMaxDst];
    __shared__ int below_w[kListWaves];
    __shared__ int scan_sh[kListBlock];
    if (*flags) return;
    const int b = blockIdx.x / VELO_N_PLANES, q = blockIdx.x % VELO_N_PLANES;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int s = off[b];
    const int *po = plane_off + (int64_t)b * kPlaneSlots;
    const int d0 = po[q], D = po[q + 1] - d0;
    if (D <= 0) return;                                   // uniform over the block
    const int E0 = row_ptr[s + po[max(q - 2, 0)]], E1 = row_ptr[s + d0];
    const int quarter = (E1 - E0 + kListWaves - 1) / kListWaves;
    const int w0 = E0 + min(w * quarter, E1 - E0), w1 = E0 + min((w + 1) * quarter, E1 - E0);
    for (int c0 = 0; c0 < D; c0 += kListMaxDst) {
        const int Dc = min(D - c0, kListMaxDst);
        const int lo = s + d0 + c0, hi = lo + Dc;     // batch-global destinations of this slice
        __syncthreads();                              // the previous slice is done with cnt
        for (int i = t; i < Dc; i += kListBlock)
#pragma unroll
            for (int v = 0; v < kListWaves; v++) cnt[v][i] = 0;
        __syncthreads();
        int below = 0;
        for (int e0 = w0 + lane; e0 < w1; e0 += 4 * 64) {   // four loads in flight per lane
            int dd[4];
#pragma unroll
            for (int j = 0; j < 4; j++) dd[j] = e0 + 64 * j < w1 ? dst_g[e0 + 64 * j] : hi;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                if (dd[j] < lo) below++;
                else if (dd[j] < hi) atomicAdd(&cnt[w][dd[j] - lo], 1);
            }
        }
        for (int o = 32; o > 0; o >>= 1) below += __shfl_xor(below, o);
        if (lane == 0) below_w[w] = below;
        __syncthreads();
        int base = E0;
#pragma unroll
        for (int v = 0; v < kListWaves; v++) base += below_w[v];
        // thread t owns destinations [i0, i1) of the slice
        const int per = (Dc + kListBlock - 1) / kListBlock;
        const int i0 = min(t * per, Dc), i1 = min(i0 + per, Dc);
        int run = 0;
        for (int i = i0; i < i1; i++)
#pragma unroll
            for (int v = 0; v < kListWaves; v++) run += cnt[v][i];
        int total;
        int p = base + block_exclusive_scan(run, scan_sh, &total);
        for (int i = i0; i < i1; i++) {
            in_ptr[lo + i] = p;
#pragma unroll
            for (int v = 0; v < kListWaves; v++) {
                const int c = cnt[v][i];
                cnt[v][i] = p;                        // quarter v's cursor for this destination
                p += c;
            }
        }
        if ((int64_t)hi == n_hits && i0 < i1 && i1 == Dc) in_ptr[hi] = p;
        __syncthreads();
        const int nbits = Dc > 1 ? 32 - __clz(Dc - 1) : 0;
        int dn = w0 + lane < w1 ? dst_g[w0 + lane] : -1;   // the next chunk's destination, in flight
        for (int e0 = w0; e0 < w1; e0 += 64) {        // uniform over the wavefront
            const int e = e0 + lane;
            const int d = dn;
            dn = e + 64 < w1 ? dst_g[e + 64] : -1;
            const bool mine = d >= lo && d < hi;
            const int key = mine ? d - lo : 0;
            unsigned long long peers = ballot(mine);
            for (int k = 0; k < nbits; k++) {
                const bool bit = (key >> k) & 1;
                const unsigned long long m = ballot(mine && bit);
                peers &= bit ? m : ~m;
            }
            const int rank = lanes_below(peers);
            const int cur = mine ? cnt[w][key] : 0;
            if (mine) in_list[cur + rank] = e;
            if (mine && rank == 0) cnt[w][key] = cur + __popcll(peers);
        }
    }
}

inline int grid_for(int64_t n, int block, int cap_blocks = 65536) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap_blocks) g = cap_blocks;
    return (int)g;
}

}  // namespace

void launch_fill(int *p, int v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_fill<<<grid_for(n, 256, 4096), 256, 0, s>>>(p, v, n);
}

void launch_prepare_raw(const velo_hits *h, int max_event_hits, int *plane_off, int *hit_event, unsigned *flags,
                        hipStream_t s) {
    if (h->n_events <= 0) return;
    k_prepare<<<h->n_events, 256, 0, s>>>(h->n_events, h->n_hits, h->event_offsets, h->x, h->y, h->z,
                                          h->plane, max_event_hits, plane_off, hit_event, flags);
}

void launch_prepare(velo_ctx *c, const velo_hits *h, hipStream_t s) {
    launch_prepare_raw(h, c->cfg.max_event_hits, c->ws.plane_off, c->ws.hit_event, c->ws.flags, s);
}

void launch_scan_with(const int *in, int *out, int64_t n, int *tmp, hipStream_t s) {
    const int nb = (int)((n + kScanTile - 1) / kScanTile);
    if (nb > 0) k_scan_reduce<<<nb, kScanBlock, 0, s>>>(in, n, tmp);
    k_scan_sums<<<1, kScanBlock, 0, s>>>(tmp, nb, out + n);
    if (nb > 0) k_scan_apply<<<nb, kScanBlock, 0, s>>>(in, n, tmp, out);
}

int64_t scan_tmp_ints(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

void launch_scan(velo_ctx *c, const int *in, int *out, int64_t n, hipStream_t s) {
    launch_scan_with(in, out, n, c->ws.scan_tmp, s);
}

void launch_knn_into(velo_ctx *c, const velo_hits *h, const float *emb, int kmax, float d2max, int *nbr, int *deg,
                     hipStream_t s) {
    if (h->n_hits <= 0) return;
    const int blocks = persistent_grid(c, stage_per_cu(c, VELO_STAGE_KNN, 16));
    auto go = [&](auto kernel) {
        kernel<<<blocks, kKnnBlock, 0, s>>>(h->n_hits, h->event_offsets, c->ws.plane_off, c->ws.hit_event, h->plane,
                                            (const f32x4 *)emb, d2max, kmax, nbr, deg, c->tune_xcd[VELO_STAGE_KNN],
                                            c->ws.flags);
    };
    switch (c->tune_knn_run > 0 ? c->tune_knn_run : kKnnRunDefault) {
        case 8: go(k_knn<8>); break;
        case 32: go(k_knn<32>); break;
        default: go(k_knn<16>); break;
    }
}

void launch_knn_loop(velo_ctx *c, const velo_hits *h, const float *emb, hipStream_t s) {
    if (h->n_hits <= 0) return;
    k_knn_loop<<<grid_for(h->n_hits, kLoopBlock), kLoopBlock, 0, s>>>(
        h->n_hits, h->event_offsets, c->ws.plane_off, c->ws.hit_event, h->plane, (const f32x4 *)emb, c->cfg.d2_max,
        c->cfg.k_max, c->ws.nbr, c->ws.deg, c->ws.flags);
}

void launch_knn(velo_ctx *c, const velo_hits *h, const float *emb, hipStream_t s) {
    launch_knn_into(c, h, emb, c->cfg.k_max, c->cfg.d2_max, c->ws.nbr, c->ws.deg, s);
}

void launch_compact(velo_ctx *c, const velo_hits *h, velo_outputs *g, hipStream_t s) {
    Workspace &w = c->ws;
    const int64_t N = h->n_hits;
    // row_ptr = exclusive scan of the per-hit degrees; row_ptr[N] = edge total
    launch_scan(c, w.deg, w.row_ptr, N, s);
    const int64_t cap = g->edge_capacity < c->cfg.max_edges ? g->edge_capacity : c->cfg.max_edges;
    k_check_capacity<<<1, 1, 0, s>>>(w.row_ptr + N, cap, w.n_edges, g->n_edges, w.flags);
    if (N > 0) {
        const int64_t slots = N * c->cfg.k_max;
        k_compact<<<grid_for(slots, 256, persistent_grid(c, 32)), 256, 0, s>>>(
            N, c->cfg.k_max, h->event_offsets, w.hit_event, w.deg, w.row_ptr, w.nbr, cap,
            g->edge_src, g->edge_dst, w.src_g, w.dst_g, w.flags);
    }
    int *eoff = g->edge_offsets ? g->edge_offsets : w.eoff_tmp;
    k_edge_offsets<<<grid_for(h->n_events + 1, 256), 256, 0, s>>>(h->n_events, h->event_offsets,
                                                                  w.row_ptr, eoff, w.flags);
}

void launch_globalise_raw(const velo_hits *h, const velo_outputs *g, int64_t cap, int *src_g, int *dst_g,
                          int *n_internal, unsigned *flags, hipStream_t s) {
    k_check_capacity<<<1, 1, 0, s>>>(g->n_edges, cap, n_internal, nullptr, flags);
    const dim3 grid(h->n_events > 0 ? h->n_events : 1, h->n_events > 0 ? 16 : 1);
    k_globalise<<<grid, 256, 0, s>>>(h->n_events, h->event_offsets, g->edge_offsets, n_internal, cap, g->edge_src,
                                     g->edge_dst, h->plane, src_g, dst_g, flags);
}

void launch_globalise(velo_ctx *c, const velo_hits *h, const velo_outputs *g, hipStream_t s) {
    Workspace &w = c->ws;
    const int64_t cap = g->edge_capacity < c->cfg.max_edges ? g->edge_capacity : c->cfg.max_edges;
    launch_globalise_raw(h, g, cap, w.src_g, w.dst_g, w.n_edges, w.flags, s);
}

void launch_row_ptr(velo_ctx *c, const velo_hits *h, const velo_outputs *g, hipStream_t s) {
    Workspace &w = c->ws;
    if (h->n_hits <= 0 || h->n_events <= 0) return;
    const int *eoff = g->edge_offsets ? g->edge_offsets : w.eoff_tmp;
    const int64_t cap = g->edge_capacity < c->cfg.max_edges ? g->edge_capacity : c->cfg.max_edges;
    k_row_ptr<<<grid_for(h->n_hits, 256, 4096), 256, 0, s>>>(h->n_hits, w.hit_event, eoff, w.n_edges, cap, w.src_g,
                                                              w.row_ptr, w.flags);
}

}  // namespace velo

namespace velo {

void launch_in_lists_plane(velo_ctx *c, const velo_hits *h, hipStream_t s) {
    Workspace &w = c->ws;
    const int64_t N = h->n_hits;
    if (h->n_events <= 0 || N <= 0) {
        launch_scan(c, w.deg, w.in_ptr, 0, s);
        return;
    }
    k_in_lists<<<h->n_events * VELO_N_PLANES, kListBlock, 0, s>>>(N, h->event_offsets, w.plane_off, w.row_ptr,
                                                                  w.dst_g, w.in_ptr, w.in_list, w.flags);
}

}  // namespace velo
