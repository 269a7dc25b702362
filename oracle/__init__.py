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
_SO = os.path.join(_HERE, "liboracle.so")
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
