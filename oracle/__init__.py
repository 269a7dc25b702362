"""ctypes binding of the plain float64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg may use this package; the product path never does.

`build()` compiles oracle.c with gcc; `lib()` loads the shared object and fails
loudly if it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# ORACLE_LIB: another build of oracle.c to load (the sanitizer test builds one)
_SO = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib: Optional[C.CDLL] = None


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function", _SRC, "-o", _SO + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise RuntimeError(f"oracle not built: {_SO} missing (run __graft_entry__.build())")
        L = C.CDLL(_SO)
        i64, i32, f32, f64 = C.c_int64, C.c_int32, C.c_float, C.c_double
        p = C.c_void_p
        L.oracle_param_count.argtypes = [C.c_int] * 4
        L.oracle_param_count.restype = i64
        L.oracle_embed.argtypes = [i64, p, p, p, p, C.c_int, C.c_int, p]
        L.oracle_embed.restype = C.c_int
        L.oracle_neighbours.argtypes = [i64, p, p, C.c_int, f32, C.c_int, p, p, i64]
        L.oracle_neighbours.restype = i64
        L.oracle_gnn_forward.argtypes = [i64, p, p, p, i64, p, p, p, C.c_int, C.c_int, C.c_int, C.c_int, p, p, p]
        L.oracle_gnn_forward.restype = C.c_int
        L.oracle_gnn_backward.argtypes = [i64, p, p, p, i64, p, p, p, C.c_int, C.c_int, C.c_int, C.c_int, p, p]
        L.oracle_gnn_backward.restype = C.c_int
        L.oracle_bce.argtypes = [i64, p, p, f64, p]
        L.oracle_bce.restype = f64
        L.oracle_components.argtypes = [i64, i64, p, p, p, p]
        L.oracle_components.restype = C.c_int
        L.oracle_pipeline.argtypes = [i32, p, p, p, p, p, p, C.c_int, C.c_int, C.c_int, C.c_int,
                                      f32, C.c_int, f64, p, p, p, p, p, p]
        L.oracle_pipeline.restype = C.c_int
        L.oracle_embed_train.argtypes = [i64, p, p, p, p, p, p, p, p, p, C.c_int, C.c_int,
                                         C.c_int, f32, f64, p, p, p, p]
        L.oracle_embed_train.restype = C.c_int
        L.oracle_focal.argtypes = [i64, p, p, f64, f64, p]
        L.oracle_focal.restype = f64
        L.oracle_components_sweep.argtypes = [i64, p, i64, p, p, p, p]
        L.oracle_components_sweep.restype = C.c_int
        L.oracle_embed_amax.argtypes = [i64, p, p, p, p, C.c_int, C.c_int, p]
        L.oracle_embed_amax.restype = C.c_int
        L.oracle_embed_int8.argtypes = [i64, p, p, p, p, C.c_int, C.c_int, p, p]
        L.oracle_embed_int8.restype = C.c_int
        L.oracle_triplets.argtypes = [i64, i64, p, p, p, i64, p, p, p, p, p]
        L.oracle_triplets.restype = C.c_int
        L.oracle_triplet_param_count.argtypes = [C.c_int]
        L.oracle_triplet_param_count.restype = i64
        L.oracle_triplet_logits.argtypes = [i64, p, i64, p, C.c_int, p, C.c_int, p]
        L.oracle_triplet_logits.restype = C.c_int
        L.oracle_build_tracks.argtypes = [i64, i64, p, p, p, p, i64, p, p, i64, p, p, p, p, i64, p]
        L.oracle_build_tracks.restype = C.c_int
        L.oracle_track_hits.argtypes = [i64, p, p, p, i64, p, p, p, i64]
        L.oracle_track_hits.restype = C.c_int
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_set_threads.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def param_count(H: int, iters: int, Ce: int = 128, D: int = 4) -> int:
    return int(lib().oracle_param_count(H, iters, Ce, D))


def embed(x, y, z, blob, Ce: int = 128, D: int = 4) -> np.ndarray:
    """Float64 embedding [N x D] of one event's hits (Sec. 5.1)."""
    x, y, z, blob = _c(x, np.float32), _c(y, np.float32), _c(z, np.float32), _c(blob, np.float32)
    out = np.zeros((x.shape[0], D), np.float64)
    rc = lib().oracle_embed(x.shape[0], _ptr(x), _ptr(y), _ptr(z), _ptr(blob), Ce, D, _ptr(out))
    assert rc == 0, rc
    return out


def neighbours(plane, emb32, d2max: float, k_max: int):
    """Rough graph of one event (Sec. 5.1): (row_ptr [N+1], col [E]) with event-local j.

    `emb32` is the float32 embedding the decision is taken on.
    """
    plane, emb32 = _c(plane, np.int32), _c(emb32, np.float32)
    n = plane.shape[0]
    D = emb32.shape[1] if emb32.ndim == 2 else 1
    cap = max(1, n * k_max)
    rp = np.zeros(n + 1, np.int32)
    col = np.zeros(cap, np.int32)
    E = lib().oracle_neighbours(n, _ptr(plane), _ptr(emb32), D, float(np.float32(d2max)), k_max,
                                _ptr(rp), _ptr(col), cap)
    assert E >= 0, E
    return rp, col[:E].copy()


def csr_to_edges(row_ptr: np.ndarray, col: np.ndarray):
    src = np.repeat(np.arange(row_ptr.shape[0] - 1, dtype=np.int32), np.diff(row_ptr))
    return src, col.astype(np.int32)


def gnn_forward(x, y, z, src, dst, blob, H: int, iters: int, Ce: int = 128, D: int = 4,
                want_states: bool = False):
    """Float64 edge logits of one event (Sec. 5.2); optionally h^n and e^n too."""
    x, y, z = _c(x, np.float32), _c(y, np.float32), _c(z, np.float32)
    src, dst, blob = _c(src, np.int32), _c(dst, np.int32), _c(blob, np.float32)
    n, E = x.shape[0], src.shape[0]
    logit = np.zeros(E, np.float64)
    hf = np.zeros((n, H), np.float64) if want_states else None
    ef = np.zeros((E, H), np.float64) if want_states else None
    rc = lib().oracle_gnn_forward(n, _ptr(x), _ptr(y), _ptr(z), E, _ptr(src), _ptr(dst), _ptr(blob),
                                  H, iters, Ce, D, _ptr(logit), _ptr(hf), _ptr(ef))
    assert rc == 0, rc
    return (logit, hf, ef) if want_states else logit


def gnn_backward(x, y, z, src, dst, blob, H: int, iters: int, dlogit, Ce: int = 128, D: int = 4):
    """Float64 gradient (blob-shaped) of sum(dlogit * logit) w.r.t. the GNN parameters."""
    x, y, z = _c(x, np.float32), _c(y, np.float32), _c(z, np.float32)
    src, dst, blob = _c(src, np.int32), _c(dst, np.int32), _c(blob, np.float32)
    dlogit = _c(dlogit, np.float64)
    grad = np.zeros(blob.shape[0], np.float64)
    rc = lib().oracle_gnn_backward(x.shape[0], _ptr(x), _ptr(y), _ptr(z), src.shape[0], _ptr(src),
                                   _ptr(dst), _ptr(blob), H, iters, Ce, D, _ptr(dlogit), _ptr(grad))
    assert rc == 0, rc
    return grad


def bce(logit, y, pos_weight: float):
    """Weighted BCE loss and dL/dlogit (float64)."""
    logit, y = _c(logit, np.float64), _c(y, np.uint8)
    dz = np.zeros(logit.shape[0], np.float64)
    L = lib().oracle_bce(logit.shape[0], _ptr(logit), _ptr(y), float(pos_weight), _ptr(dz))
    return float(L), dz


def focal(logit, y, alpha: float = 0.25, gamma: float = 2.0):
    """Sigmoid focal loss (Sec. 5.2) and dL/dlogit (float64); alpha < 0: no class weight."""
    logit, y = _c(logit, np.float64), _c(y, np.uint8)
    dz = np.zeros(logit.shape[0], np.float64)
    L = lib().oracle_focal(logit.shape[0], _ptr(logit), _ptr(y), float(alpha), float(gamma), _ptr(dz))
    return float(L), dz


def components(n: int, src, dst, keep) -> np.ndarray:
    """Component labels (smallest hit index of each component) over kept edges."""
    src, dst, keep = _c(src, np.int32), _c(dst, np.int32), _c(keep, np.uint8)
    lab = np.zeros(n, np.int32)
    rc = lib().oracle_components(n, src.shape[0], _ptr(src), _ptr(dst), _ptr(keep), _ptr(lab))
    assert rc == 0, rc
    return lab


def components_sweep(plane, src, dst, keep) -> np.ndarray:
    """Labels of the two plane sweeps of Sec. 7.3 (a comparison variant; not exact)."""
    plane, src, dst, keep = _c(plane, np.int32), _c(src, np.int32), _c(dst, np.int32), _c(keep, np.uint8)
    lab = np.zeros(plane.shape[0], np.int32)
    rc = lib().oracle_components_sweep(plane.shape[0], _ptr(plane), src.shape[0], _ptr(src), _ptr(dst),
                                       _ptr(keep), _ptr(lab))
    assert rc == 0, rc
    return lab


def embed_amax(events, blob, Ce: int = 128, D: int = 4) -> np.ndarray:
    """Largest |input| of the embedding's second and third layers over the
    hits of `events` (float64), for INT8 calibration."""
    amax = np.zeros(2, np.float64)
    blob = _c(blob, np.float32)
    for ev in events:
        x, y, z = _c(ev.x, np.float32), _c(ev.y, np.float32), _c(ev.z, np.float32)
        rc = lib().oracle_embed_amax(x.shape[0], _ptr(x), _ptr(y), _ptr(z), _ptr(blob), Ce, D, _ptr(amax))
        assert rc == 0, rc
    return amax


def int8_scales(amax, blob, Ce: int = 128, D: int = 4) -> np.ndarray:
    """{s_x2, s_w2, s_x3, s_w3} as float32: s = fl32(max |value| / 127) for the
    two layer inputs (from `amax`) and the two weight matrices."""
    o2 = 12 + Ce * 3 + Ce
    w2 = np.asarray(blob[o2:o2 + Ce * Ce], np.float32)
    o3 = o2 + Ce * Ce + Ce
    w3 = np.asarray(blob[o3:o3 + D * Ce], np.float32)
    q = np.float32(127.0)
    sx = [np.float32(np.float32(a) / q) if a > 0 else np.float32(1.0) for a in amax]
    sw = [np.float32(np.abs(w).max() / q) if np.abs(w).max() > 0 else np.float32(1.0) for w in (w2, w3)]
    return np.array([sx[0], sw[0], sx[1], sw[1]], np.float32)


def embed_int8(x, y, z, blob, scales, Ce: int = 128, D: int = 4) -> np.ndarray:
    """Embedding with INT8 operands in its second and third layers under the
    per-tensor float32 scales {s_x2, s_w2, s_x3, s_w3} (Sec. 7.4)."""
    x, y, z = _c(x, np.float32), _c(y, np.float32), _c(z, np.float32)
    blob, sc = _c(blob, np.float32), _c(scales, np.float32)
    out = np.zeros((x.shape[0], D), np.float64)
    rc = lib().oracle_embed_int8(x.shape[0], _ptr(x), _ptr(y), _ptr(z), _ptr(blob), Ce, D, _ptr(sc), _ptr(out))
    assert rc == 0, rc
    return out


def triplets(n: int, src, dst, keep):
    """Triplets of one event's kept edges (Sec. 5.3): (art [Ta x 2], elb [Te x 2],
    elb_type [Te] with 1 = left, 2 = right elbow), pairs of edge indices."""
    src, dst = _c(src, np.int32), _c(dst, np.int32)
    keep = _c(keep, np.uint8)
    E = src.shape[0]
    cap = 1 << 10
    while True:
        art = np.zeros((cap, 2), np.int32)
        elb = np.zeros((cap, 2), np.int32)
        et = np.zeros(cap, np.int8)
        na, ne = C.c_int64(0), C.c_int64(0)
        rc = lib().oracle_triplets(n, E, _ptr(src), _ptr(dst), _ptr(keep), cap, _ptr(art), C.byref(na),
                                   _ptr(elb), _ptr(et), C.byref(ne))
        if rc == 0:
            return art[:na.value].copy(), elb[:ne.value].copy(), et[:ne.value].copy()
        assert rc == -1, rc
        cap = max(na.value, ne.value)


def triplet_param_count(H: int) -> int:
    return int(lib().oracle_triplet_param_count(H))


def triplet_logits(pairs, e, tblob, which: int) -> np.ndarray:
    """Logits of the articulation (which = 0) or elbow (1) classifier on the
    pairs of edge encodings [e_a || e_b]; e: [E x H] float64."""
    pairs = _c(np.asarray(pairs).reshape(-1, 2), np.int32)
    e = _c(e, np.float64)
    tblob = _c(tblob, np.float32)
    z = np.zeros(pairs.shape[0], np.float64)
    rc = lib().oracle_triplet_logits(pairs.shape[0], _ptr(pairs), e.shape[0], _ptr(e), e.shape[1], _ptr(tblob),
                                     which, _ptr(z))
    assert rc == 0, rc
    return z


def triplet_classifier_grad(pairs, e, tblob, which: int, dlogit) -> np.ndarray:
    """Gradient of sum_t dlogit_t * z_t with respect to the parameters of
    triplet classifier `which` (0: articulations, 1: elbows), where z_t =
    W1 relu(W0 [e_a || e_b] + b0) + b1 (Sec. 5.3) and e [E x H] are the final
    edge encodings, taken as fixed.  Returned over the classifier's slice of
    the blob, in its layout (W0 [H x 2H] row-major, b0 [H], W1 [H], b1).
    Written with numpy in float64 for training the classifiers; the forward
    pass it differentiates is oracle_triplet_logits (C)."""
    pairs = np.asarray(pairs, np.int64).reshape(-1, 2)
    e = np.asarray(e, np.float64)
    H = e.shape[1]
    n = 2 * H * H + 2 * H + 1
    p = np.asarray(tblob, np.float64)[which * n:(which + 1) * n]
    W0 = p[:2 * H * H].reshape(H, 2 * H)
    b0 = p[2 * H * H:2 * H * H + H]
    W1 = p[2 * H * H + H:2 * H * H + 2 * H]
    dz = np.asarray(dlogit, np.float64)
    X = np.concatenate([e[pairs[:, 0]], e[pairs[:, 1]]], axis=1)     # [T x 2H]
    A = X @ W0.T + b0                                                 # hidden pre-activations
    R = np.where(A > 0.0, A, 0.0)
    dA = np.outer(dz, W1) * (A > 0.0)
    g = np.empty(n)
    g[:2 * H * H] = (dA.T @ X).ravel()
    g[2 * H * H:2 * H * H + H] = dA.sum(axis=0)
    g[2 * H * H + H:2 * H * H + 2 * H] = R.T @ dz
    g[-1] = dz.sum()
    return g


def build_tracks(n: int, src, dst, plane, keep, art, art_keep, elb, elb_keep):
    """Tracks from the purified edge graph (Sec. 5.4): (edge_seg [E], tracks
    [T x 2] of segment labels, the second -1 for one-segment tracks)."""
    src, dst, plane = _c(src, np.int32), _c(dst, np.int32), _c(plane, np.int32)
    keep = _c(keep, np.uint8)
    art, elb = _c(np.asarray(art).reshape(-1, 2), np.int32), _c(np.asarray(elb).reshape(-1, 2), np.int32)
    ak, ek = _c(art_keep, np.uint8), _c(elb_keep, np.uint8)
    E = src.shape[0]
    seg = np.zeros(max(E, 1), np.int32)
    cap = max(E, 1) + art.shape[0]
    tr = np.zeros((cap, 2), np.int32)
    nt = C.c_int64(0)
    rc = lib().oracle_build_tracks(n, E, _ptr(src), _ptr(dst), _ptr(plane), _ptr(keep), art.shape[0], _ptr(art),
                                   _ptr(ak), elb.shape[0], _ptr(elb), _ptr(ek), _ptr(seg), _ptr(tr), cap,
                                   C.byref(nt))
    assert rc == 0, rc
    return seg[:E].copy(), tr[:nt.value].copy()


def track_hits(src, dst, edge_seg, tracks):
    """Hits of every track (Sec. 5.4, step 4): a list of ascending int32 arrays."""
    src, dst, seg = _c(src, np.int32), _c(dst, np.int32), _c(edge_seg, np.int32)
    tracks = _c(np.asarray(tracks).reshape(-1, 2), np.int32)
    T = tracks.shape[0]
    off = np.zeros(T + 1, np.int64)
    cap = max(1, 4 * src.shape[0])
    while True:
        hits = np.zeros(cap, np.int32)
        rc = lib().oracle_track_hits(src.shape[0], _ptr(src), _ptr(dst), _ptr(seg), T, _ptr(tracks), _ptr(off),
                                     _ptr(hits), cap)
        if rc == 0:
            return [hits[off[k]:off[k + 1]].copy() for k in range(T)]
        assert rc == -1, rc
        cap = int(off[-1])


def set_threads(n: int) -> int:
    """Threads of the oracle's loops over events (n <= 0: unchanged); returns
    the count in effect."""
    return int(lib().oracle_set_threads(int(n)))


def pipeline(batch, blob, H: int, iters: int, radius: float = 0.1, k_max: int = 32,
             logit_min: float = 0.0, Ce: int = 128, D: int = 4):
    """Whole path over a batch (events independent).  Returns a dict of numpy arrays."""
    off = _c(batch.event_offsets, np.int32)
    x, y, z = _c(batch.x, np.float32), _c(batch.y, np.float32), _c(batch.z, np.float32)
    plane, blob = _c(batch.plane, np.int32), _c(blob, np.float32)
    N = int(off[-1]) if off.shape[0] else 0
    B = off.shape[0] - 1
    cap = max(1, N * k_max)
    emb = np.zeros((N, D), np.float64)
    labels = np.zeros(N, np.int32)
    eoff = np.zeros(B + 1, np.int64)
    esrc = np.zeros(cap, np.int32)
    edst = np.zeros(cap, np.int32)
    elog = np.zeros(cap, np.float64)
    d2max = d2max_f32(radius)
    rc = lib().oracle_pipeline(B, _ptr(off), _ptr(x), _ptr(y), _ptr(z), _ptr(plane), _ptr(blob),
                               H, iters, Ce, D, d2max, k_max, float(logit_min),
                               _ptr(emb), _ptr(labels), _ptr(eoff), _ptr(esrc), _ptr(edst), _ptr(elog))
    assert rc == 0, rc
    E = int(eoff[-1])
    return {"emb": emb, "labels": labels, "edge_offsets": eoff, "src": esrc[:E].copy(),
            "dst": edst[:E].copy(), "logit": elog[:E].copy()}


def embed_train_sums(x, y, z, plane, pid, query, rnd, emb32, blob, k_train: int = 50,
                     d2_train: float = 1.5, margin: float = 1.0, Ce: int = 128, D: int = 4):
    """Raw sums of the embedding loss of one noise-free event (Sec. 5.1, the
    two loss equations) and their float64 gradients (blob-shaped): returns
    (S_genuine, S_fake, N_genuine, N_fake, grad S_genuine, grad S_fake)."""
    x, y, z = _c(x, np.float32), _c(y, np.float32), _c(z, np.float32)
    plane, pid = _c(plane, np.int32), _c(pid, np.int32)
    query, rnd = _c(query, np.uint8), _c(rnd, np.uint32)
    emb32, blob = _c(emb32, np.float32), _c(blob, np.float32)
    sums = np.zeros(2, np.float64)
    counts = np.zeros(2, np.int64)
    gg = np.zeros(blob.shape[0], np.float64)
    gf = np.zeros(blob.shape[0], np.float64)
    rc = lib().oracle_embed_train(x.shape[0], _ptr(x), _ptr(y), _ptr(z), _ptr(plane), _ptr(pid),
                                  _ptr(query), _ptr(rnd), _ptr(emb32), _ptr(blob), Ce, D, int(k_train),
                                  float(np.float32(d2_train)), float(margin), _ptr(sums), _ptr(counts),
                                  _ptr(gg), _ptr(gf))
    assert rc == 0, rc
    return float(sums[0]), float(sums[1]), int(counts[0]), int(counts[1]), gg, gf


def embed_train_loss(parts, w_genuine: float):
    """Pool per-event sums into the step's loss and gradient:
    L = w * S_g / N_g + S_f / N_f (a term with no pairs is zero)."""
    Sg = sum(p[0] for p in parts); Sf = sum(p[1] for p in parts)
    Ng = sum(p[2] for p in parts); Nf = sum(p[3] for p in parts)
    cg = w_genuine / Ng if Ng else 0.0
    cf = 1.0 / Nf if Nf else 0.0
    grad = sum(cg * p[4] + cf * p[5] for p in parts)
    return {"loss": cg * Sg + cf * Sf, "loss_genuine": Sg / Ng if Ng else 0.0,
            "loss_fake": Sf / Nf if Nf else 0.0, "n_genuine": Ng, "n_fake": Nf, "grad": grad}


def d2max_f32(radius: float) -> float:
    """The squared radius rounded once to float32: the value both sides compare against."""
    return float(np.float32(float(radius) * float(radius)))
