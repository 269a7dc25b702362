/*
 * oracle.c -- plain, slow, CPU reference of the VELO GNN track-finding path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code, header, table or constant with the HIP
 * library.
 *
 * Everything is computed in float64 from float32 inputs promoted exactly,
 * except the one place where floating point decides an integer: the
 * neighbour-set decision is taken in float32 (the precision the paper's
 * implementation runs in), with the evaluation order fixed below, so that
 * both sides decide identically on identical embeddings.
 *
 * Stages (paper, Sec. 5):
 *   features      Sec. 5.1: normalised cylindrical (r, phi, z) for the embedding
 *   embedding     Sec. 5.1: hit -> e_h in R^{n_dim}, an MLP
 *   rough graph   Sec. 5.1, squared-distance equation: hits on plane p joined
 *                 to hits on p+1 and p+2 with d^2 < d2max, at most k_max per
 *                 node (Sec. 7.2 describes the per-node bounded list)
 *   GNN           Sec. 5.2: node/edge encoders, n message-passing steps with
 *                 the scatter_add message equation and residual node/edge
 *                 networks, distinct per step; edge classifier
 *   threshold     Sec. 5 (pipeline overview): edges scoring below the cut are
 *                 dropped
 *   components    Sec. 5 and Sec. 7.3: connected components of the purified
 *                 hit graph give the track labels (and, as a comparison
 *                 variant, the paper's two plane sweeps)
 *   loss/gradient weighted binary cross-entropy on the edge logits and its
 *                 exact gradient (training form), and the sigmoid focal loss
 *                 the paper trains with (Sec. 5.2)
 *   embedding     Sec. 5.1, the two loss equations: pairwise hinge
 *   training      embedding loss over genuine pairs, hard negatives from the
 *                 bounded neighbour list and one random pair per query, and
 *                 its exact gradient with respect to the embedding MLP
 *
 * Parameter blob (float32, every Linear row-major [out x in] then its bias):
 *   norm[12]: emb_mu[3] emb_sigma[3] gnn_mu[3] gnn_sigma[3]
 *   embedding: [Ce x 3], [Ce x Ce], [D x Ce]
 *   node encoder: [H x 3], [H x H];  edge encoder: [H x 2H], [H x H]
 *   per step k: node net [H x 3H], [H x H]; edge net [H x 3H], [H x H]
 *   classifier: [H x H], [1 x H]
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* parameter offsets                                                   */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t w, b;      /* offsets of weight and bias in the blob */
    int out, in;
} lin_t;

typedef struct {
    int H, iters, Ce, D;
    lin_t emb[3];
    lin_t nenc[2], eenc[2];
    lin_t node[64][2], edge[64][2];
    lin_t cls[2];
    int64_t total;
} layout_t;

static int64_t put(lin_t *l, int64_t off, int out, int in)
{
    l->w = off;
    l->b = off + (int64_t)out * in;
    l->out = out;
    l->in = in;
    return l->b + out;
}

static int make_layout(layout_t *L, int H, int iters, int Ce, int D)
{
    if (iters < 0 || iters > 64 || H <= 0 || Ce <= 0 || D <= 0)
        return -1;
    int64_t o = 12;
    L->H = H; L->iters = iters; L->Ce = Ce; L->D = D;
    o = put(&L->emb[0], o, Ce, 3);
    o = put(&L->emb[1], o, Ce, Ce);
    o = put(&L->emb[2], o, D, Ce);
    o = put(&L->nenc[0], o, H, 3);
    o = put(&L->nenc[1], o, H, H);
    o = put(&L->eenc[0], o, H, 2 * H);
    o = put(&L->eenc[1], o, H, H);
    for (int k = 0; k < iters; k++) {
        o = put(&L->node[k][0], o, H, 3 * H);
        o = put(&L->node[k][1], o, H, H);
        o = put(&L->edge[k][0], o, H, 3 * H);
        o = put(&L->edge[k][1], o, H, H);
    }
    o = put(&L->cls[0], o, H, H);
    o = put(&L->cls[1], o, 1, H);
    L->total = o;
    return 0;
}

int64_t oracle_param_count(int H, int iters, int Ce, int D)
{
    layout_t L;
    if (make_layout(&L, H, iters, Ce, D))
        return -1;
    return L.total;
}

/* y = W x + b for one Linear layer, float64, W row-major [out x in]. */
static void linear(const float *blob, const lin_t *l, const double *x, double *y)
{
    const float *W = blob + l->w, *b = blob + l->b;
    for (int o = 0; o < l->out; o++) {
        double s = (double)b[o];
        for (int i = 0; i < l->in; i++)
            s += (double)W[(int64_t)o * l->in + i] * x[i];
        y[o] = s;
    }
}

static void relu(double *v, int n)
{
    for (int i = 0; i < n; i++)
        if (!(v[i] > 0.0))
            v[i] = 0.0;
}

/* Two-layer MLP with a ReLU between: y = W1 relu(W0 x + b0) + b1.
 * `hid` (size l0->out) receives the pre-activation of the hidden layer. */
static void mlp2(const float *blob, const lin_t *l0, const lin_t *l1,
                 const double *x, double *hid, double *y)
{
    double a[1024];
    linear(blob, l0, x, hid);
    memcpy(a, hid, sizeof(double) * l0->out);
    relu(a, l0->out);
    linear(blob, l1, a, y);
}

/* ------------------------------------------------------------------ */
/* Sec. 5.1: features and embedding                                    */
/* ------------------------------------------------------------------ */

/* Normalised cylindrical coordinates (r, phi, z) of one hit, phi = atan2(y, x). */
static void embed_features(const float *norm, float x, float y, float z, double u[3])
{
    double X = x, Y = y, Z = z;
    double f[3] = { sqrt(X * X + Y * Y), atan2(Y, X), Z };
    for (int c = 0; c < 3; c++)
        u[c] = (f[c] - (double)norm[c]) / (double)norm[3 + c];
}

/* Embedding of every hit of one event: emb[i*D + c], float64. */
int oracle_embed(int64_t n, const float *x, const float *y, const float *z,
                 const float *blob, int Ce, int D, double *emb)
{
    layout_t L;
    if (make_layout(&L, 1, 0, Ce, D) || Ce > 1024)
        return -1;
    double u[3], h1[1024], h2[1024], pre[1024];
    for (int64_t i = 0; i < n; i++) {
        embed_features(blob, x[i], y[i], z[i], u);
        linear(blob, &L.emb[0], u, h1);
        relu(h1, Ce);
        linear(blob, &L.emb[1], h1, pre);
        memcpy(h2, pre, sizeof(double) * Ce);
        relu(h2, Ce);
        linear(blob, &L.emb[2], h2, emb + i * D);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Sec. 7.4: the embedding with INT8 matrix operands                   */
/* ------------------------------------------------------------------ */

/* Largest |value| entering the two matrix layers of the embedding that take
 * INT8 operands (the 128-wide hidden layers, after their ReLU), over the hits
 * of a calibration set, in float64 (the paper calibrates its INT8 embedding
 * on a set of events).  amax[0]: input of the second layer, amax[1]: input of
 * the third.  Accumulates into amax (the caller zeroes it once). */
int oracle_embed_amax(int64_t n, const float *x, const float *y, const float *z,
                      const float *blob, int Ce, int D, double *amax)
{
    layout_t L;
    if (make_layout(&L, 1, 0, Ce, D) || Ce > 1024)
        return -1;
    double u[3], h1[1024], h2[1024];
    for (int64_t i = 0; i < n; i++) {
        embed_features(blob, x[i], y[i], z[i], u);
        linear(blob, &L.emb[0], u, h1);
        relu(h1, Ce);
        linear(blob, &L.emb[1], h1, h2);
        relu(h2, Ce);
        for (int c = 0; c < Ce; c++) {
            if (h1[c] > amax[0]) amax[0] = h1[c];
            if (h2[c] > amax[1]) amax[1] = h2[c];
        }
    }
    return 0;
}

/* Symmetric INT8 code of v under the per-tensor scale whose reciprocal is
 * `inv` (float32): the decision is taken in float32, as on the device:
 * t = fl32(fl32(v) * inv), rounded to the nearest integer (ties to even),
 * clamped to [-127, 127]. */
static int32_t int8_code(double v, float inv)
{
    float t = (float)v * inv;
    t = rintf(t);
    if (t > 127.0f) t = 127.0f;
    if (t < -127.0f) t = -127.0f;
    return (int32_t)t;
}

/* One matrix layer on INT8 operands: y = s_x s_w (Q_W q_x) + b, with q_x
 * and Q_W the codes of the input and the weights, the integer products summed
 * exactly and the result descaled in float64. */
static void linear_int8(const float *blob, const lin_t *l, const double *x, float s_x, float s_w, double *y)
{
    const float *W = blob + l->w, *b = blob + l->b;
    const float ix = 1.0f / s_x, iw = 1.0f / s_w;
    int32_t qx[1024];
    for (int i = 0; i < l->in; i++)
        qx[i] = int8_code(x[i], ix);
    for (int o = 0; o < l->out; o++) {
        int64_t acc = 0;
        for (int i = 0; i < l->in; i++)
            acc += (int64_t)int8_code((double)W[(int64_t)o * l->in + i], iw) * qx[i];
        y[o] = (double)acc * (double)s_x * (double)s_w + (double)b[o];
    }
}

/* Embedding with INT8 operands in its two 128-wide-input layers (the first
 * layer, three inputs, stays in float64 like the rest of the oracle).
 * sc = {s_x2, s_w2, s_x3, s_w3}: the float32 scales of the inputs and weights
 * of the second and third layers (s = max |value| / 127). */
int oracle_embed_int8(int64_t n, const float *x, const float *y, const float *z,
                      const float *blob, int Ce, int D, const float *sc, double *emb)
{
    layout_t L;
    if (make_layout(&L, 1, 0, Ce, D) || Ce > 1024)
        return -1;
    if (!(sc[0] > 0.f) || !(sc[1] > 0.f) || !(sc[2] > 0.f) || !(sc[3] > 0.f))
        return -1;
    double u[3], h1[1024], h2[1024];
    for (int64_t i = 0; i < n; i++) {
        embed_features(blob, x[i], y[i], z[i], u);
        linear(blob, &L.emb[0], u, h1);
        relu(h1, Ce);
        linear_int8(blob, &L.emb[1], h1, sc[0], sc[1], h2);
        relu(h2, Ce);
        linear_int8(blob, &L.emb[2], h2, sc[2], sc[3], emb + i * D);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Sec. 5.1: rough graph                                               */
/* ------------------------------------------------------------------ */

/* Squared distance, decided in float32: d_c = a_c - b_c rounded to float32,
 * s = d_0*d_0 rounded, then s = fma(d_c, d_c, s) for c = 1..D-1. */
static float d2_f32(const float *a, const float *b, int D)
{
    float d = a[0] - b[0];
    float s = d * d;
    for (int c = 1; c < D; c++) {
        d = a[c] - b[c];
        s = fmaf(d, d, s);
    }
    return s;
}

typedef struct { float d2; int32_t j; } cand_t;

static int cand_less(const cand_t *a, const cand_t *b)
{
    return a->d2 < b->d2 || (a->d2 == b->d2 && a->j < b->j);
}

static int cmp_j(const void *a, const void *b)
{
    int32_t x = ((const cand_t *)a)->j, y = ((const cand_t *)b)->j;
    return (x > y) - (x < y);
}

/*
 * For every hit i of one event, with plane p, the candidates are the hits j
 * with plane(j) - p in {1, 2}; j is kept when d2(i, j) < d2max.  If more than
 * k_max are kept, the k_max smallest under the order (d2, j) remain (a
 * deterministic form of the bounded nearest-neighbour list).  Rows come out
 * sorted by j.  row_ptr has n+1 entries; col has room for `cap` entries.
 * Returns the edge count, or -(edge count) if it exceeds cap (nothing is
 * written past cap), or INT64_MIN on bad arguments.
 */
int64_t oracle_neighbours(int64_t n, const int32_t *plane, const float *emb, int D,
                          float d2max, int k_max, int32_t *row_ptr, int32_t *col, int64_t cap)
{
    if (n < 0 || D <= 0 || k_max <= 0)
        return INT64_MIN;
    cand_t *buf = (cand_t *)malloc(sizeof(cand_t) * (size_t)(n > 0 ? n : 1));
    if (!buf)
        return INT64_MIN;
    int64_t E = 0;
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; i++) {
        int m = 0;
        for (int64_t j = 0; j < n; j++) {
            int dp = plane[j] - plane[i];
            if (dp != 1 && dp != 2)
                continue;
            float d2 = d2_f32(emb + i * D, emb + j * D, D);
            if (d2 < d2max) {
                buf[m].d2 = d2;
                buf[m].j = (int32_t)j;
                m++;
            }
        }
        if (m > k_max) {
            /* selection: move the k_max smallest (d2, j) to the front */
            for (int a = 0; a < k_max; a++) {
                int best = a;
                for (int b = a + 1; b < m; b++)
                    if (cand_less(&buf[b], &buf[best]))
                        best = b;
                cand_t t = buf[a]; buf[a] = buf[best]; buf[best] = t;
            }
            m = k_max;
        }
        qsort(buf, (size_t)m, sizeof(cand_t), cmp_j);
        for (int a = 0; a < m; a++) {
            if (E + a < cap)
                col[E + a] = buf[a].j;
        }
        E += m;
        row_ptr[i + 1] = (int32_t)(E < cap ? E : cap);
    }
    free(buf);
    return E <= cap ? E : -E;
}

/* ------------------------------------------------------------------ */
/* Sec. 5.2: interaction-network GNN                                   */
/* ------------------------------------------------------------------ */

typedef struct {
    /* states per step: h[k] is n x H, e[k] is E x H, k = 0..iters */
    double **h, **e;
    /* hidden pre-activations: node/edge nets per step, encoders, classifier */
    double **hn, **he;
    double *hnenc, *heenc, *hcls;
    double *xhat;         /* n x 3 normalised Cartesian inputs */
    double *mo, *mi;      /* messages of every step: iters x n x H each */
} fwd_t;

static void fwd_free(fwd_t *F, int iters)
{
    if (F->h) for (int k = 0; k <= iters; k++) free(F->h[k]);
    if (F->e) for (int k = 0; k <= iters; k++) free(F->e[k]);
    if (F->hn) for (int k = 0; k < iters; k++) free(F->hn[k]);
    if (F->he) for (int k = 0; k < iters; k++) free(F->he[k]);
    free(F->h); free(F->e); free(F->hn); free(F->he);
    free(F->hnenc); free(F->heenc); free(F->hcls); free(F->xhat);
    free(F->mo); free(F->mi);
    memset(F, 0, sizeof(*F));
}

#define ALLOC(p, cnt) do { (p) = calloc((size_t)(cnt) > 0 ? (size_t)(cnt) : 1, sizeof(*(p))); if (!(p)) goto oom; } while (0)

/* Full forward pass of one event keeping every intermediate. */
static int gnn_forward_full(const layout_t *L, const float *blob, int64_t n,
                            const float *x, const float *y, const float *z,
                            int64_t E, const int32_t *src, const int32_t *dst,
                            fwd_t *F, double *logit)
{
    const int H = L->H, it = L->iters;
    const float *norm = blob;
    double *cat = NULL, *upd = NULL;
    memset(F, 0, sizeof(*F));
    ALLOC(F->h, it + 1); ALLOC(F->e, it + 1); ALLOC(F->hn, it > 0 ? it : 1); ALLOC(F->he, it > 0 ? it : 1);
    for (int k = 0; k <= it; k++) { ALLOC(F->h[k], n * H); ALLOC(F->e[k], E * H); }
    for (int k = 0; k < it; k++) { ALLOC(F->hn[k], n * H); ALLOC(F->he[k], E * H); }
    ALLOC(F->hnenc, n * H); ALLOC(F->heenc, E * H); ALLOC(F->hcls, E * H); ALLOC(F->xhat, n * 3);
    ALLOC(F->mo, (int64_t)it * n * H); ALLOC(F->mi, (int64_t)it * n * H);

    /* node encoder on normalised Cartesian coordinates */
    for (int64_t i = 0; i < n; i++) {
        double *xh = F->xhat + i * 3;
        xh[0] = ((double)x[i] - norm[6]) / (double)norm[9];
        xh[1] = ((double)y[i] - norm[7]) / (double)norm[10];
        xh[2] = ((double)z[i] - norm[8]) / (double)norm[11];
        mlp2(blob, &L->nenc[0], &L->nenc[1], xh, F->hnenc + i * H, F->h[0] + i * H);
    }
    /* edge encoder on [h0_src, h0_dst] */
    ALLOC(cat, 3 * H);
    for (int64_t q = 0; q < E; q++) {
        memcpy(cat, F->h[0] + (int64_t)src[q] * H, sizeof(double) * H);
        memcpy(cat + H, F->h[0] + (int64_t)dst[q] * H, sizeof(double) * H);
        mlp2(blob, &L->eenc[0], &L->eenc[1], cat, F->heenc + q * H, F->e[0] + q * H);
    }
    ALLOC(upd, H);
    for (int k = 0; k < it; k++) {
        double *mo = F->mo + (int64_t)k * n * H, *mi = F->mi + (int64_t)k * n * H;
        /* message: outgoing and incoming sums of e^k (scatter_add) */
        for (int64_t q = 0; q < E; q++)
            for (int c = 0; c < H; c++) {
                mo[(int64_t)src[q] * H + c] += F->e[k][q * H + c];
                mi[(int64_t)dst[q] * H + c] += F->e[k][q * H + c];
            }
        /* node network with residual: h^{k+1} = h^k + phi_k([h^k, m_out, m_in]) */
        for (int64_t i = 0; i < n; i++) {
            memcpy(cat, F->h[k] + i * H, sizeof(double) * H);
            memcpy(cat + H, mo + i * H, sizeof(double) * H);
            memcpy(cat + 2 * H, mi + i * H, sizeof(double) * H);
            mlp2(blob, &L->node[k][0], &L->node[k][1], cat, F->hn[k] + i * H, upd);
            for (int c = 0; c < H; c++)
                F->h[k + 1][i * H + c] = F->h[k][i * H + c] + upd[c];
        }
        /* edge network with residual, using the updated hit encodings */
        for (int64_t q = 0; q < E; q++) {
            memcpy(cat, F->e[k] + q * H, sizeof(double) * H);
            memcpy(cat + H, F->h[k + 1] + (int64_t)src[q] * H, sizeof(double) * H);
            memcpy(cat + 2 * H, F->h[k + 1] + (int64_t)dst[q] * H, sizeof(double) * H);
            mlp2(blob, &L->edge[k][0], &L->edge[k][1], cat, F->he[k] + q * H, upd);
            for (int c = 0; c < H; c++)
                F->e[k + 1][q * H + c] = F->e[k][q * H + c] + upd[c];
        }
    }
    /* edge classifier on e^n: a logit (score = sigmoid(logit)) */
    for (int64_t q = 0; q < E; q++)
        mlp2(blob, &L->cls[0], &L->cls[1], F->e[it] + q * H, F->hcls + q * H, logit + q);
    free(cat);
    free(upd);
    return 0;
oom:
    free(cat);
    free(upd);
    fwd_free(F, it);
    return -2;
}

int oracle_gnn_forward(int64_t n, const float *x, const float *y, const float *z,
                       int64_t E, const int32_t *src, const int32_t *dst,
                       const float *blob, int H, int iters, int Ce, int D, double *logit,
                       double *h_final, double *e_final)
{
    layout_t L;
    if (make_layout(&L, H, iters, Ce, D) || 3 * H > 1024)
        return -1;
    for (int64_t q = 0; q < E; q++)
        if (src[q] < 0 || src[q] >= n || dst[q] < 0 || dst[q] >= n)
            return -1;
    fwd_t F;
    int rc = gnn_forward_full(&L, blob, n, x, y, z, E, src, dst, &F, logit);
    if (rc)
        return rc;
    if (h_final) memcpy(h_final, F.h[iters], sizeof(double) * n * H);
    if (e_final) memcpy(e_final, F.e[iters], sizeof(double) * E * H);
    fwd_free(&F, iters);
    return 0;
}

/* ------------------------------------------------------------------ */
/* training form: weighted BCE and the exact gradient                  */
/* ------------------------------------------------------------------ */

/* L = (1/E) sum_q w_q [softplus(z_q) - y_q z_q], w = pos_weight if y = 1 else 1.
 * dL/dz_q = w_q (sigmoid(z_q) - y_q) / E.  Returns L (0 when E = 0). */
double oracle_bce(int64_t E, const double *z, const uint8_t *yv, double pos_weight, double *dz)
{
    double L = 0.0;
    for (int64_t q = 0; q < E; q++) {
        double w = yv[q] ? pos_weight : 1.0;
        double zz = z[q];
        double sp = zz > 0 ? zz + log1p(exp(-zz)) : log1p(exp(zz));
        double sig = zz >= 0 ? 1.0 / (1.0 + exp(-zz)) : exp(zz) / (1.0 + exp(zz));
        L += w * (sp - (yv[q] ? zz : 0.0));
        if (dz)
            dz[q] = w * (sig - (yv[q] ? 1.0 : 0.0)) / (double)E;
    }
    return E > 0 ? L / (double)E : 0.0;
}

/* Backward of y = W1 relu(W0 x + b0) + b1 given dy; accumulates dW/db into
 * g (blob-shaped, float64) and writes dx (size l0->in). `pre` is the saved
 * hidden pre-activation. */
static void mlp2_backward(const float *blob, const lin_t *l0, const lin_t *l1,
                          const double *x, const double *pre, const double *dy,
                          double *g, double *dx)
{
    const int Hh = l0->out, I = l0->in, O = l1->out;
    double da[1024];
    for (int o = 0; o < O; o++)
        g[l1->b + o] += dy[o];
    for (int h = 0; h < Hh; h++) {
        double a = pre[h] > 0.0 ? pre[h] : 0.0;
        double s = 0.0;
        for (int o = 0; o < O; o++) {
            g[l1->w + (int64_t)o * Hh + h] += dy[o] * a;
            s += (double)blob[l1->w + (int64_t)o * Hh + h] * dy[o];
        }
        da[h] = pre[h] > 0.0 ? s : 0.0;
    }
    for (int i = 0; i < I; i++)
        dx[i] = 0.0;
    for (int h = 0; h < Hh; h++) {
        g[l0->b + h] += da[h];
        for (int i = 0; i < I; i++) {
            g[l0->w + (int64_t)h * I + i] += da[h] * x[i];
            dx[i] += (double)blob[l0->w + (int64_t)h * I + i] * da[h];
        }
    }
}

/*
 * Gradient of sum_q dlogit[q] * logit[q] with respect to every GNN parameter
 * (node/edge encoders, node/edge networks, classifier), by reverse-mode
 * differentiation of the forward above.  grad is blob-shaped float64; the
 * normalisation and embedding entries stay zero (graph building is not
 * differentiable).  The forward is recomputed here.
 */
int oracle_gnn_backward(int64_t n, const float *x, const float *y, const float *z,
                        int64_t E, const int32_t *src, const int32_t *dst,
                        const float *blob, int H, int iters, int Ce, int D,
                        const double *dlogit, double *grad)
{
    layout_t L;
    if (make_layout(&L, H, iters, Ce, D) || 3 * H > 1024)
        return -1;
    for (int64_t q = 0; q < E; q++)
        if (src[q] < 0 || src[q] >= n || dst[q] < 0 || dst[q] >= n)
            return -1;
    memset(grad, 0, sizeof(double) * L.total);
    double *logit = NULL, *de = NULL, *dh = NULL, *dhn = NULL, *den = NULL, *cat = NULL, *dx = NULL;
    fwd_t F;
    memset(&F, 0, sizeof(F));
    ALLOC(logit, E);
    if (gnn_forward_full(&L, blob, n, x, y, z, E, src, dst, &F, logit)) {
        free(logit);
        return -2;
    }
    ALLOC(de, E * H); ALLOC(dh, n * H); ALLOC(dhn, n * H); ALLOC(den, E * H);
    ALLOC(cat, 3 * H); ALLOC(dx, 3 * H);

    /* classifier */
    for (int64_t q = 0; q < E; q++) {
        double dy = dlogit[q];
        mlp2_backward(blob, &L.cls[0], &L.cls[1], F.e[iters] + q * H, F.hcls + q * H, &dy, grad, dx);
        memcpy(de + q * H, dx, sizeof(double) * H);
    }
    /* de = dL/de^{k+1}, dh = dL/dh^{k+1} (contributions from step k+1 already in) */
    for (int k = iters - 1; k >= 0; k--) {
        double *mo = F.mo + (int64_t)k * n * H, *mi = F.mi + (int64_t)k * n * H;
        /* edge net k */
        for (int64_t q = 0; q < E; q++) {
            memcpy(cat, F.e[k] + q * H, sizeof(double) * H);
            memcpy(cat + H, F.h[k + 1] + (int64_t)src[q] * H, sizeof(double) * H);
            memcpy(cat + 2 * H, F.h[k + 1] + (int64_t)dst[q] * H, sizeof(double) * H);
            mlp2_backward(blob, &L.edge[k][0], &L.edge[k][1], cat, F.he[k] + q * H, de + q * H, grad, dx);
            for (int c = 0; c < H; c++) {
                den[q * H + c] = de[q * H + c] + dx[c];
                dh[(int64_t)src[q] * H + c] += dx[H + c];
                dh[(int64_t)dst[q] * H + c] += dx[2 * H + c];
            }
        }
        /* node net k */
        for (int64_t i = 0; i < n; i++) {
            memcpy(cat, F.h[k] + i * H, sizeof(double) * H);
            memcpy(cat + H, mo + i * H, sizeof(double) * H);
            memcpy(cat + 2 * H, mi + i * H, sizeof(double) * H);
            mlp2_backward(blob, &L.node[k][0], &L.node[k][1], cat, F.hn[k] + i * H, dh + i * H, grad, dx);
            for (int c = 0; c < H; c++) {
                dhn[i * H + c] = dh[i * H + c] + dx[c];
                mo[i * H + c] = dx[H + c];       /* reuse as dm_out */
                mi[i * H + c] = dx[2 * H + c];   /* reuse as dm_in */
            }
        }
        /* messages: the sums pass their gradient back to every summed edge */
        for (int64_t q = 0; q < E; q++)
            for (int c = 0; c < H; c++)
                den[q * H + c] += mo[(int64_t)src[q] * H + c] + mi[(int64_t)dst[q] * H + c];
        double *t = de; de = den; den = t;
        t = dh; dh = dhn; dhn = t;
    }
    /* edge encoder */
    for (int64_t q = 0; q < E; q++) {
        memcpy(cat, F.h[0] + (int64_t)src[q] * H, sizeof(double) * H);
        memcpy(cat + H, F.h[0] + (int64_t)dst[q] * H, sizeof(double) * H);
        mlp2_backward(blob, &L.eenc[0], &L.eenc[1], cat, F.heenc + q * H, de + q * H, grad, dx);
        for (int c = 0; c < H; c++) {
            dh[(int64_t)src[q] * H + c] += dx[c];
            dh[(int64_t)dst[q] * H + c] += dx[H + c];
        }
    }
    /* node encoder */
    for (int64_t i = 0; i < n; i++)
        mlp2_backward(blob, &L.nenc[0], &L.nenc[1], F.xhat + i * 3, F.hnenc + i * H, dh + i * H, grad, dx);

    fwd_free(&F, iters);
    free(logit); free(de); free(dh); free(dhn); free(den); free(cat); free(dx);
    return 0;
oom:
    fwd_free(&F, iters);
    free(logit); free(de); free(dh); free(dhn); free(den); free(cat); free(dx);
    return -2;
}

/* ------------------------------------------------------------------ */
/* Sec. 5.3: triplets of the purified hit graph                       */
/* ------------------------------------------------------------------ */

/*
 * The triplets of one event: pairs of kept edges that share a hit C.
 *   articulation  a = A -> C, b = C -> B   (the common hit in the middle)
 *   left elbow    a = C -> A, b = C -> B   (both leave C; a < b)
 *   right elbow   a = A -> C, b = B -> C   (both enter C; a < b)
 * Edges are event-local indices into src/dst (grouped by source); a and b
 * are edge indices.  Order: articulations by C, then a, then b; elbows by C,
 * the left ones of a hit before its right ones, then a, then b (edge
 * indices ascending).  art[2t], art[2t+1] = (a, b); elb likewise with
 * elb_type[t] = 1 (left) or 2 (right).  Returns 0, or -1 when a list would
 * exceed `cap` pairs (the counts still give the required sizes).
 */
int oracle_triplets(int64_t n, int64_t E, const int32_t *src, const int32_t *dst, const uint8_t *keep,
                    int64_t cap, int32_t *art, int64_t *n_art, int32_t *elb, int8_t *elb_type, int64_t *n_elb)
{
    int64_t *in_off = calloc((size_t)n + 1, sizeof(int64_t)), *out_off = calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *in_e = malloc(sizeof(int32_t) * (size_t)(E > 0 ? E : 1)), *out_e = malloc(sizeof(int32_t) * (size_t)(E > 0 ? E : 1));
    int64_t *fill = calloc((size_t)n + 1, sizeof(int64_t));
    if (!in_off || !out_off || !in_e || !out_e || !fill) {
        free(in_off); free(out_off); free(in_e); free(out_e); free(fill);
        return -2;
    }
    for (int64_t q = 0; q < E; q++)
        if (keep[q]) {
            if (src[q] < 0 || src[q] >= n || dst[q] < 0 || dst[q] >= n) {
                free(in_off); free(out_off); free(in_e); free(out_e); free(fill);
                return -3;
            }
            in_off[dst[q] + 1]++;
            out_off[src[q] + 1]++;
        }
    for (int64_t i = 0; i < n; i++) {
        in_off[i + 1] += in_off[i];
        out_off[i + 1] += out_off[i];
    }
    for (int64_t q = 0; q < E; q++)          /* edge indices ascending within every list */
        if (keep[q]) in_e[in_off[dst[q]] + fill[dst[q]]++] = (int32_t)q;
    memset(fill, 0, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t q = 0; q < E; q++)
        if (keep[q]) out_e[out_off[src[q]] + fill[src[q]]++] = (int32_t)q;
    int64_t na = 0, ne = 0;
    for (int64_t c = 0; c < n; c++)
        for (int64_t i = in_off[c]; i < in_off[c + 1]; i++)
            for (int64_t j = out_off[c]; j < out_off[c + 1]; j++) {
                if (na < cap) { art[2 * na] = in_e[i]; art[2 * na + 1] = out_e[j]; }
                na++;
            }
    for (int64_t c = 0; c < n; c++) {
        for (int64_t i = out_off[c]; i < out_off[c + 1]; i++)
            for (int64_t j = i + 1; j < out_off[c + 1]; j++) {
                if (ne < cap) { elb[2 * ne] = out_e[i]; elb[2 * ne + 1] = out_e[j]; elb_type[ne] = 1; }
                ne++;
            }
        for (int64_t i = in_off[c]; i < in_off[c + 1]; i++)
            for (int64_t j = i + 1; j < in_off[c + 1]; j++) {
                if (ne < cap) { elb[2 * ne] = in_e[i]; elb[2 * ne + 1] = in_e[j]; elb_type[ne] = 2; }
                ne++;
            }
    }
    *n_art = na;
    *n_elb = ne;
    free(in_off); free(out_off); free(in_e); free(out_e); free(fill);
    return na > cap || ne > cap ? -1 : 0;
}

/* Offsets of the two triplet classifiers in their parameter blob (Sec. 5.3:
 * separate classifiers for articulations and elbows): for each, a Linear
 * [H x 2H] + [H], ReLU, a Linear [1 x H] + [1]; articulations first. */
static void triplet_layout(int H, int which, lin_t *l0, lin_t *l1)
{
    int64_t o = (int64_t)which * ((int64_t)H * 2 * H + H + H + 1);
    put(l0, o, H, 2 * H);
    put(l1, l0->b + H, 1, H);
}

int64_t oracle_triplet_param_count(int H)
{
    return 2 * ((int64_t)H * 2 * H + H + H + 1);
}

/* Triplet logits z_t = MLP_which([e_a || e_b]) of T pairs (a, b) of edge
 * indices, with e the final edge encodings [E x H] (Sec. 5.3; score =
 * sigmoid(z), kept iff z >= the cut). */
int oracle_triplet_logits(int64_t T, const int32_t *pairs, int64_t E, const double *e, int H,
                          const float *tblob, int which, double *z)
{
    if (H < 1 || 2 * H > 1024 || (which != 0 && which != 1))
        return -1;
    lin_t l0, l1;
    triplet_layout(H, which, &l0, &l1);
    double cat[1024], hid[1024];
    for (int64_t t = 0; t < T; t++) {
        const int32_t a = pairs[2 * t], b = pairs[2 * t + 1];
        if (a < 0 || a >= E || b < 0 || b >= E)
            return -1;
        memcpy(cat, e + (int64_t)a * H, sizeof(double) * H);
        memcpy(cat + H, e + (int64_t)b * H, sizeof(double) * H);
        mlp2(tblob, &l0, &l1, cat, hid, z + t);
    }
    return 0;
}

/*
 * Tracks from the purified edge graph (Sec. 5.4), one event.  Inputs: the
 * kept edges, the triplet lists of oracle_triplets and each triplet's keep
 * decision.  The four steps:
 *  1. Kept elbows join their two edges.  When the two edges span different
 *     numbers of planes, the longer one (a hit skipped) duplicates the path
 *     through the third hit and takes no part in articulations.
 *  2. Among the kept articulations without a duplicate edge, one is shared
 *     when its first edge is the first edge of another of them, or its second
 *     edge the second edge of another (tracks parting or joining there).
 *     Every other one joins its two edges.  The joined sets of edges are the
 *     segments (exact union-find; a segment's label is its smallest edge index).
 *  3. Every shared articulation makes a track of its two edges' segments (a
 *     segment shared by several tracks is copied into each), and every
 *     segment that no shared articulation touches is a track of its own.
 *  4. (oracle_track_hits) a track's hits are the ends of its edges.
 * edge_seg[q]: segment of kept edge q, -1 for others.  tracks[2k], [2k+1]:
 * the track's segments, the second -1 for a single segment; single-segment
 * tracks come first, by segment label, then the shared articulations' tracks
 * in articulation order.  Returns 0, or -1 when more than `cap` tracks.
 */
static int32_t uf_find(int32_t *par, int32_t x)
{
    while (par[x] != x) {
        par[x] = par[par[x]];
        x = par[x];
    }
    return x;
}

static void uf_union(int32_t *par, int32_t u, int32_t v)
{
    u = uf_find(par, u);
    v = uf_find(par, v);
    if (u == v) return;
    if (u < v) par[v] = u;
    else par[u] = v;
}

int oracle_build_tracks(int64_t n, int64_t E, const int32_t *src, const int32_t *dst, const int32_t *plane,
                        const uint8_t *keep, int64_t n_art, const int32_t *art, const uint8_t *art_keep,
                        int64_t n_elb, const int32_t *elb, const uint8_t *elb_keep, int32_t *edge_seg,
                        int32_t *tracks, int64_t cap, int64_t *n_tracks)
{
    int32_t *par = malloc(sizeof(int32_t) * (size_t)(E > 0 ? E : 1));
    uint8_t *dup = calloc((size_t)(E > 0 ? E : 1), 1), *touched = calloc((size_t)(E > 0 ? E : 1), 1);
    int32_t *first = calloc((size_t)(E > 0 ? E : 1), sizeof(int32_t)), *second = calloc((size_t)(E > 0 ? E : 1), sizeof(int32_t));
    uint8_t *shared = calloc((size_t)(n_art > 0 ? n_art : 1), 1);
    int rc = 0;
    if (!par || !dup || !touched || !first || !second || !shared) { rc = -2; goto done; }
    (void)n;
    for (int64_t q = 0; q < E; q++) par[q] = (int32_t)q;
    /* 1. elbows */
    for (int64_t t = 0; t < n_elb; t++) {
        if (!elb_keep[t]) continue;
        const int32_t a = elb[2 * t], b = elb[2 * t + 1];
        uf_union(par, a, b);
        const int ga = plane[dst[a]] - plane[src[a]], gb = plane[dst[b]] - plane[src[b]];
        if (ga > gb) dup[a] = 1;
        else if (gb > ga) dup[b] = 1;
    }
    /* 2. articulations: shared ones part or join tracks; the others join edges */
    for (int64_t t = 0; t < n_art; t++) {
        const int32_t a = art[2 * t], b = art[2 * t + 1];
        if (art_keep[t] && !dup[a] && !dup[b]) { first[a]++; second[b]++; }
    }
    for (int64_t t = 0; t < n_art; t++) {
        const int32_t a = art[2 * t], b = art[2 * t + 1];
        if (!art_keep[t] || dup[a] || dup[b]) continue;
        if (first[a] > 1 || second[b] > 1) shared[t] = 1;
        else uf_union(par, a, b);
    }
    for (int64_t q = 0; q < E; q++)
        edge_seg[q] = keep[q] ? uf_find(par, (int32_t)q) : -1;
    /* 3. tracks */
    for (int64_t t = 0; t < n_art; t++)
        if (shared[t]) {
            touched[edge_seg[art[2 * t]]] = 1;
            touched[edge_seg[art[2 * t + 1]]] = 1;
        }
    int64_t k = 0;
    for (int64_t q = 0; q < E; q++)
        if (keep[q] && edge_seg[q] == q && !touched[q]) {
            if (k < cap) { tracks[2 * k] = (int32_t)q; tracks[2 * k + 1] = -1; }
            k++;
        }
    for (int64_t t = 0; t < n_art; t++)
        if (shared[t]) {
            if (k < cap) { tracks[2 * k] = edge_seg[art[2 * t]]; tracks[2 * k + 1] = edge_seg[art[2 * t + 1]]; }
            k++;
        }
    *n_tracks = k;
    if (k > cap) rc = -1;
done:
    free(par); free(dup); free(touched); free(first); free(second); free(shared);
    return rc;
}

static int cmp_i32(const void *a, const void *b)
{
    const int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Step 4 of Sec. 5.4: the hits of every track, the ends of the edges of its
 * segments, ascending and without repeats.  hit_off [n_tracks + 1];
 * returns 0, or -1 when more than `cap` hits in all. */
int oracle_track_hits(int64_t E, const int32_t *src, const int32_t *dst, const int32_t *edge_seg,
                      int64_t n_tracks, const int32_t *tracks, int64_t *hit_off, int32_t *hits, int64_t cap)
{
    int32_t *tmp = malloc(sizeof(int32_t) * (size_t)(2 * E + 2));
    if (!tmp) return -2;
    int64_t o = 0;
    hit_off[0] = 0;
    for (int64_t k = 0; k < n_tracks; k++) {
        const int32_t s1 = tracks[2 * k], s2 = tracks[2 * k + 1];
        int64_t m = 0;
        for (int64_t q = 0; q < E; q++)
            if (edge_seg[q] >= 0 && (edge_seg[q] == s1 || edge_seg[q] == s2)) {
                tmp[m++] = src[q];
                tmp[m++] = dst[q];
            }
        qsort(tmp, (size_t)m, sizeof(int32_t), cmp_i32);
        for (int64_t i = 0; i < m; i++)
            if (i == 0 || tmp[i] != tmp[i - 1]) {
                if (o < cap) hits[o] = tmp[i];
                o++;
            }
        hit_off[k + 1] = o;
    }
    free(tmp);
    return o > cap ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* Sec. 5 / Sec. 7.3: connected components of the purified hit graph  */
/* ------------------------------------------------------------------ */

/*
 * Exact weakly connected components by breadth-first search over the kept
 * edges taken as undirected.  Hits are visited as BFS roots in increasing
 * index order, so each label is the smallest hit index of its component.
 * Hits without kept edges are their own component.
 */
int oracle_components(int64_t n, int64_t E, const int32_t *src, const int32_t *dst,
                      const uint8_t *keep, int32_t *labels)
{
    int64_t *deg = calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *adj_ptr = calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *adj = malloc(sizeof(int32_t) * (size_t)(2 * E + 1));
    int64_t *fill = calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *queue = malloc(sizeof(int32_t) * (size_t)(n + 1));
    int rc = 0;
    if (!deg || !adj_ptr || !adj || !fill || !queue) { rc = -2; goto done; }
    for (int64_t q = 0; q < E; q++) {
        if (src[q] < 0 || src[q] >= n || dst[q] < 0 || dst[q] >= n) { rc = -1; goto done; }
        if (keep[q]) { deg[src[q]]++; deg[dst[q]]++; }
    }
    for (int64_t i = 0; i < n; i++)
        adj_ptr[i + 1] = adj_ptr[i] + deg[i];
    for (int64_t q = 0; q < E; q++)
        if (keep[q]) {
            adj[adj_ptr[src[q]] + fill[src[q]]++] = dst[q];
            adj[adj_ptr[dst[q]] + fill[dst[q]]++] = src[q];
        }
    for (int64_t i = 0; i < n; i++)
        labels[i] = -1;
    for (int64_t r = 0; r < n; r++) {
        if (labels[r] >= 0)
            continue;
        int64_t head = 0, tail = 0;
        labels[r] = (int32_t)r;
        queue[tail++] = (int32_t)r;
        while (head < tail) {
            int32_t u = queue[head++];
            for (int64_t a = adj_ptr[u]; a < adj_ptr[u + 1]; a++) {
                int32_t v = adj[a];
                if (labels[v] < 0) {
                    labels[v] = (int32_t)r;
                    queue[tail++] = v;
                }
            }
        }
    }
done:
    free(deg); free(adj_ptr); free(adj); free(fill); free(queue);
    return rc;
}

/*
 * The two plane sweeps of Sec. 7.3, kept as a comparison variant (they are
 * not exact on every graph).  Labels start as the event-local index.
 * Forward, planes 1 .. N_PLANES-1 in order: each hit on plane p takes the
 * smallest of its label and the labels of the hits joined to it by kept
 * edges from planes p-1 and p-2.  Backward, planes N_PLANES-2 .. 0: each hit
 * on plane p takes the smallest of its label and the labels of the hits its
 * kept edges reach on planes p+1 and p+2.  Edges whose destination is not
 * one or two planes after their source take no part.
 */
int oracle_components_sweep(int64_t n, const int32_t *plane, int64_t E, const int32_t *src,
                            const int32_t *dst, const uint8_t *keep, int32_t *labels)
{
    const int n_planes = 26;
    for (int64_t q = 0; q < E; q++)
        if (src[q] < 0 || src[q] >= n || dst[q] < 0 || dst[q] >= n)
            return -1;
    for (int64_t i = 0; i < n; i++)
        labels[i] = (int32_t)i;
    for (int p = 1; p < n_planes; p++)
        for (int64_t q = 0; q < E; q++) {
            int gap = plane[dst[q]] - plane[src[q]];
            if (keep[q] && plane[dst[q]] == p && (gap == 1 || gap == 2) && labels[src[q]] < labels[dst[q]])
                labels[dst[q]] = labels[src[q]];
        }
    for (int p = n_planes - 2; p >= 0; p--)
        for (int64_t q = 0; q < E; q++) {
            int gap = plane[dst[q]] - plane[src[q]];
            if (keep[q] && plane[src[q]] == p && (gap == 1 || gap == 2) && labels[dst[q]] < labels[src[q]])
                labels[src[q]] = labels[dst[q]];
        }
    return 0;
}

/* ------------------------------------------------------------------ */
/* whole path over a batch of independent events                       */
/* ------------------------------------------------------------------ */

/*
 * Runs features -> embedding -> rough graph -> GNN -> threshold -> components
 * for every event of a batch (events are independent; OpenMP over events).
 * The float64 embedding is rounded to float32 before the neighbour decision.
 * Outputs: labels (event-local), per-event edge lists concatenated in event
 * order with edge_offsets[B+1] (event-local src/dst), logits in float64, and
 * the float64 embedding.  edge capacity must be k_max * total hits.
 */
int oracle_pipeline(int32_t B, const int32_t *event_offsets,
                    const float *x, const float *y, const float *z, const int32_t *plane,
                    const float *blob, int H, int iters, int Ce, int D,
                    float d2max, int k_max, double logit_min,
                    double *emb_out, int32_t *labels, int64_t *edge_offsets,
                    int32_t *esrc, int32_t *edst, double *elogit)
{
    int rc = 0;
    int64_t *cnt = calloc((size_t)B + 1, sizeof(int64_t));
    if (!cnt)
        return -2;
    /* pass 1: embedding and rough graph per event, edges in a per-event slot */
    #pragma omp parallel for schedule(dynamic, 1)
    for (int32_t b = 0; b < B; b++) {
        int64_t s = event_offsets[b], n = event_offsets[b + 1] - s;
        int64_t slot = s * k_max;
        float *e32 = malloc(sizeof(float) * (size_t)(n * D + 1));
        int32_t *rp = malloc(sizeof(int32_t) * (size_t)(n + 1));
        if (!e32 || !rp) { rc = -2; free(e32); free(rp); continue; }
        if (oracle_embed(n, x + s, y + s, z + s, blob, Ce, D, emb_out + s * D)) rc = -1;
        for (int64_t i = 0; i < n * D; i++)
            e32[i] = (float)emb_out[s * D + i];
        int64_t E = oracle_neighbours(n, plane + s, e32, D, d2max, k_max, rp, edst + slot, n * k_max);
        if (E < 0) { rc = -1; E = 0; }
        for (int64_t i = 0; i < n; i++)
            for (int64_t a = rp[i]; a < rp[i + 1]; a++)
                esrc[slot + a] = (int32_t)i;
        cnt[b + 1] = E;
        free(e32);
        free(rp);
    }
    if (rc) { free(cnt); return rc; }
    /* pass 2: GNN, threshold and components per event */
    #pragma omp parallel for schedule(dynamic, 1)
    for (int32_t b = 0; b < B; b++) {
        int64_t s = event_offsets[b], n = event_offsets[b + 1] - s;
        int64_t slot = s * k_max, E = cnt[b + 1];
        uint8_t *keep = malloc((size_t)E + 1);
        if (!keep) { rc = -2; continue; }
        if (oracle_gnn_forward(n, x + s, y + s, z + s, E, esrc + slot, edst + slot,
                               blob, H, iters, Ce, D, elogit + slot, NULL, NULL)) rc = -1;
        for (int64_t q = 0; q < E; q++)
            keep[q] = elogit[slot + q] >= logit_min;
        if (oracle_components(n, E, esrc + slot, edst + slot, keep, labels + s)) rc = -1;
        free(keep);
    }
    /* compact the per-event slots into one concatenated list */
    edge_offsets[0] = 0;
    for (int32_t b = 0; b < B; b++)
        edge_offsets[b + 1] = edge_offsets[b] + cnt[b + 1];
    for (int32_t b = 0; b < B; b++) {
        int64_t slot = (int64_t)event_offsets[b] * k_max, o = edge_offsets[b];
        if (o != slot) {
            memmove(esrc + o, esrc + slot, sizeof(int32_t) * (size_t)cnt[b + 1]);
            memmove(edst + o, edst + slot, sizeof(int32_t) * (size_t)cnt[b + 1]);
            memmove(elogit + o, elogit + slot, sizeof(double) * (size_t)cnt[b + 1]);
        }
    }
    free(cnt);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Sec. 5.2: sigmoid focal loss (the paper's classifier loss)          */
/* ------------------------------------------------------------------ */

/*
 * Sigmoid focal loss of Lin et al., which the paper trains the edge
 * classifier with: p = sigmoid(z), p_t = p if y = 1 else 1 - p, the
 * cross-entropy ce = softplus(z) - y z = -log p_t, a_t = alpha if y = 1 else
 * 1 - alpha (alpha < 0: a_t = 1), and
 *   L = (1/E) sum_q a_t (1 - p_t)^gamma ce.
 * With s = 2y - 1, p_t = sigmoid(s z), 1 - p_t = sigmoid(-s z) and
 * d p_t / dz = s p_t (1 - p_t), so
 *   dL/dz = a_t (1 - p_t)^gamma [ (p - y) - gamma s p_t ce ] / E.
 * Returns L (0 when E = 0); dz may be NULL.
 */
static double sigmoid64(double t)
{
    return t >= 0 ? 1.0 / (1.0 + exp(-t)) : exp(t) / (1.0 + exp(t));
}

double oracle_focal(int64_t E, const double *z, const uint8_t *yv, double alpha, double gamma, double *dz)
{
    double L = 0.0;
    for (int64_t q = 0; q < E; q++) {
        double y = yv[q] ? 1.0 : 0.0, s = 2.0 * y - 1.0, zz = z[q];
        double at = alpha < 0 ? 1.0 : (yv[q] ? alpha : 1.0 - alpha);
        double ce = (zz > 0 ? zz + log1p(exp(-zz)) : log1p(exp(zz))) - y * zz;
        double pt = sigmoid64(s * zz), qt = sigmoid64(-s * zz);
        double mod = gamma == 0.0 ? 1.0 : pow(qt, gamma);
        L += at * mod * ce;
        if (dz)
            dz[q] = at * mod * ((sigmoid64(zz) - y) - gamma * s * pt * ce) / (double)E;
    }
    return E > 0 ? L / (double)E : 0.0;
}

/* ------------------------------------------------------------------ */
/* Sec. 5.1: embedding training (the two loss equations)               */
/* ------------------------------------------------------------------ */

/*
 * One event of the embedding's training set and the raw sums of its loss.
 * The event is given without noise hits (the paper drops them).  Query
 * hits (query[i] = 1) are chosen by the caller; for each query q on plane p
 * the candidates are the hits on planes p+1 and p+2, in index order:
 *   hard negatives  the bounded neighbour list of q (k_train nearest under
 *                   (d2, j) with d2 < d2_train, on the float32 embedding
 *                   emb32), those of another particle: fake pairs;
 *   genuine pairs   every candidate of q's particle (pid >= 0);
 *   random pair     candidate number floor(rnd[q] * C / 2^32) of the C
 *                   candidates, genuine or fake by pid (none when C = 0).
 * The three lists are concatenated (a pair in two lists counts twice).
 * Sums, with d2 in float64 from the float64 embedding:
 *   sums[0] = sum over genuine pairs of d2,
 *   sums[1] = sum over fake pairs of max(0, margin - d2),
 * counts[0], counts[1] = numbers of genuine and fake pairs.  Whether a fake
 * pair's hinge is active is decided in float32 on emb32 (the precision the
 * network runs in), as the neighbour list is.  gg and gf (blob-shaped,
 * float64, accumulated into) receive the gradients of sums[0] and sums[1]
 * with respect to the embedding parameters (the normalisation constants are
 * not trained).  The step's loss, pooled over the events of a batch, is
 *   L = w_genuine * S_genuine / N_genuine + S_fake / N_fake.
 */
int oracle_embed_train(int64_t n, const float *x, const float *y, const float *z,
                       const int32_t *plane, const int32_t *pid, const uint8_t *query,
                       const uint32_t *rnd, const float *emb32, const float *blob, int Ce, int D,
                       int k_train, float d2_train, double margin,
                       double *sums, int64_t *counts, double *gg, double *gf)
{
    layout_t L;
    if (n < 0 || make_layout(&L, 1, 0, Ce, D) || Ce > 1024 || D > 16 || k_train <= 0)
        return -1;
    int64_t nn = n > 0 ? n : 1;
    double *u = malloc(sizeof(double) * (size_t)nn * 3);
    double *pre1 = malloc(sizeof(double) * (size_t)nn * Ce);
    double *pre2 = malloc(sizeof(double) * (size_t)nn * Ce);
    double *e = malloc(sizeof(double) * (size_t)nn * D);
    double *dEg = calloc((size_t)nn * D, sizeof(double));
    double *dEf = calloc((size_t)nn * D, sizeof(double));
    int32_t *rp = malloc(sizeof(int32_t) * (size_t)(nn + 1));
    int32_t *col = malloc(sizeof(int32_t) * (size_t)nn * k_train);
    int rc = 0;
    if (!u || !pre1 || !pre2 || !e || !dEg || !dEf || !rp || !col) {
        rc = -2;
        goto out;
    }
    /* forward, keeping the inputs and both hidden pre-activations */
    for (int64_t i = 0; i < n; i++) {
        double a[1024];
        embed_features(blob, x[i], y[i], z[i], u + i * 3);
        linear(blob, &L.emb[0], u + i * 3, pre1 + i * Ce);
        memcpy(a, pre1 + i * Ce, sizeof(double) * Ce);
        relu(a, Ce);
        linear(blob, &L.emb[1], a, pre2 + i * Ce);
        memcpy(a, pre2 + i * Ce, sizeof(double) * Ce);
        relu(a, Ce);
        linear(blob, &L.emb[2], a, e + i * D);
    }
    /* hard-negative candidates: the bounded neighbour list on emb32 */
    if (oracle_neighbours(n, plane, emb32, D, d2_train, k_train, rp, col, nn * k_train) < 0) {
        rc = -1;
        goto out;
    }
    sums[0] = sums[1] = 0.0;
    counts[0] = counts[1] = 0;
    for (int64_t q = 0; q < n; q++) {
        if (!query[q])
            continue;
        /* one pair (q, j): genuine adds d2, fake adds the active hinge */
        #define PAIR(J)                                                              \
        do {                                                                         \
            int64_t j_ = (J);                                                        \
            int gen_ = pid[q] >= 0 && pid[j_] == pid[q];                             \
            double d2_ = 0.0, df_[16];                                               \
            for (int c = 0; c < D; c++) {                                            \
                df_[c] = e[q * D + c] - e[j_ * D + c];                               \
                d2_ += df_[c] * df_[c];                                              \
            }                                                                        \
            if (gen_) {                                                              \
                counts[0]++;                                                         \
                sums[0] += d2_;                                                      \
                for (int c = 0; c < D; c++) {                                        \
                    dEg[q * D + c] += 2.0 * df_[c];                                  \
                    dEg[j_ * D + c] -= 2.0 * df_[c];                                 \
                }                                                                    \
            } else {                                                                 \
                counts[1]++;                                                         \
                if (d2_f32(emb32 + q * D, emb32 + j_ * D, D) < (float)margin) {      \
                    sums[1] += margin - d2_;                                         \
                    for (int c = 0; c < D; c++) {                                    \
                        dEf[q * D + c] -= 2.0 * df_[c];                              \
                        dEf[j_ * D + c] += 2.0 * df_[c];                             \
                    }                                                                \
                }                                                                    \
            }                                                                        \
        } while (0)
        /* hard negatives: the fake members of q's neighbour list */
        for (int32_t a = rp[q]; a < rp[q + 1]; a++)
            if (!(pid[q] >= 0 && pid[col[a]] == pid[q]))
                PAIR(col[a]);
        /* genuine pairs and the candidate count */
        int64_t C = 0;
        for (int64_t j = 0; j < n; j++) {
            int dp = plane[j] - plane[q];
            if (dp != 1 && dp != 2)
                continue;
            C++;
            if (pid[q] >= 0 && pid[j] == pid[q])
                PAIR(j);
        }
        /* the random pair: candidate number floor(rnd * C / 2^32), index order */
        if (C > 0) {
            int64_t r = (int64_t)(((uint64_t)rnd[q] * (uint64_t)C) >> 32), seen = 0;
            for (int64_t j = 0; j < n; j++) {
                int dp = plane[j] - plane[q];
                if (dp != 1 && dp != 2)
                    continue;
                if (seen++ == r) {
                    PAIR(j);
                    break;
                }
            }
        }
        #undef PAIR
    }
    /* backward of both sums through the three layers */
    for (int pass = 0; pass < 2; pass++) {
        const double *dE = pass ? dEf : dEg;
        double *g = pass ? gf : gg;
        for (int64_t i = 0; i < n; i++) {
            double a2[1024], dpre2[1024], dx[3];
            for (int h = 0; h < Ce; h++)
                a2[h] = pre2[i * Ce + h] > 0.0 ? pre2[i * Ce + h] : 0.0;
            for (int c = 0; c < D; c++) {
                g[L.emb[2].b + c] += dE[i * D + c];
                for (int h = 0; h < Ce; h++)
                    g[L.emb[2].w + (int64_t)c * Ce + h] += dE[i * D + c] * a2[h];
            }
            for (int h = 0; h < Ce; h++) {
                double s = 0.0;
                for (int c = 0; c < D; c++)
                    s += (double)blob[L.emb[2].w + (int64_t)c * Ce + h] * dE[i * D + c];
                dpre2[h] = pre2[i * Ce + h] > 0.0 ? s : 0.0;
            }
            /* layers 0 and 1: y = W1 relu(W0 u + b0) + b1 with y = pre2 */
            mlp2_backward(blob, &L.emb[0], &L.emb[1], u + i * 3, pre1 + i * Ce, dpre2, g, dx);
        }
    }
out:
    free(u); free(pre1); free(pre2); free(e); free(dEg); free(dEf); free(rp); free(col);
    return rc;
}

/* Threads of the OpenMP loops over events in oracle_pipeline (the benchmark
 * times the oracle single-threaded and on all host cores).  Returns the
 * thread count now in effect. */
int oracle_set_threads(int n)
{
    if (n > 0)
        omp_set_num_threads(n);
    return omp_get_max_threads();
}
